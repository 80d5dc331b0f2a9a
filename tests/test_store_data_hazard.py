"""Survivor rows are stored with at most 8 bytes per lane and store.

The vector memory unit reads the data registers of a store of more than
8 bytes after the store issues; an instruction that writes them too soon
changes what the last lanes store.  This was measured on MI355X with a row
layout whose 16-byte stores were followed directly by such a write: the
lanes read last (lanes 12-15 of every 16-lane row) stored the new values,
and every parity test caught it.  The compiler does not reliably keep the
distance (a later build of the 256-state kernel placed such a write right
after a 16-byte row store), so the row stores are 8 bytes wide, which have
no such window.  This test disassembles the built code objects (the
library's own build) and checks that no 12- or 16-byte buffer store is
left; should one come back, every path after it -- fall-through, taken
branches and loop back-edges -- is searched for an instruction that writes
one of its data VGPRs (vector ALU results, vector-memory and LDS loads,
returning atomics) within MIN_DISTANCE instructions."""
import glob
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BUILD = os.path.join(ROOT, "paper_1608_00066_amd", "_build")
LLVM = "/opt/rocm/llvm/bin"
MIN_DISTANCE = 3  # a write of the store data must be at least this many instructions later


def _regs(tok):
    out = set()
    for m in re.finditer(r"v\[(\d+):(\d+)\]|\bv(\d+)\b", tok):
        if m.group(3):
            out.add(int(m.group(3)))
        else:
            out.update(range(int(m.group(1)), int(m.group(2)) + 1))
    return out


def _disassemble(obj, tmp):
    fat = os.path.join(tmp, "x.fatbin")
    co = os.path.join(tmp, "x.co")
    subprocess.run([os.path.join(LLVM, "llvm-objcopy"), "--dump-section=.hip_fatbin=" + fat, obj,
                    os.path.join(tmp, "x.o")], check=True, capture_output=True)
    subprocess.run([os.path.join(LLVM, "clang-offload-bundler"), "--type=o",
                    "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", "--input=" + fat,
                    "--output=" + co, "--unbundle"], check=True, capture_output=True)
    r = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", "--mcpu=gfx950", co],
                       check=True, capture_output=True, text=True)
    return r.stdout


_INSN = re.compile(r"^\s*([a-z_0-9]+)(?:\s+([^/]*?))?\s*//\s*([0-9A-Fa-f]+):")
_FUNC = re.compile(r"^([0-9a-f]+) <([^>]+)>:$")
_TARGET = re.compile(r"<([^>+]+)\+0x([0-9a-f]+)>\s*$")


def _parse(text):
    """Instructions of a disassembly: (mnemonic, operands, branch target
    index or None), in address order, and the index of each address."""
    funcs, insns, at = {}, [], {}
    raw = []
    for line in text.split("\n"):
        m = _FUNC.match(line.strip())
        if m:
            funcs[m.group(2)] = int(m.group(1), 16)
            continue
        m = _INSN.match(line)
        if not m:
            continue
        addr = int(m.group(3), 16)
        tgt = None
        if m.group(1).startswith(("s_branch", "s_cbranch")):
            t = _TARGET.search(line)
            if t:
                tgt = (t.group(1), int(t.group(2), 16))
        at[addr] = len(raw)
        raw.append((m.group(1), m.group(2) or "", tgt))
    for mn, ops, tgt in raw:
        ti = None
        if tgt and tgt[0] in funcs:
            ti = at.get(funcs[tgt[0]] + tgt[1])
        insns.append((mn, ops, ti))
    return insns


def _writes_vgprs(mn, ops):
    """VGPRs an instruction writes: the destination operand of vector ALU
    instructions and of loads (vector memory, LDS) and returning atomics."""
    if not ops:
        return set()
    returns = mn.startswith("v_") or "_load" in mn or mn.startswith("ds_read") or \
        mn.startswith("ds_bpermute") or mn.startswith("ds_permute") or \
        ("atomic" in mn and re.search(r"\b(glc|sc0)\b", ops) is not None)
    if not returns:
        return set()
    return _regs(ops.split(",")[0])


def _violations(text):
    """Every path of fewer than MIN_DISTANCE instructions after a 12- or
    16-byte buffer store (fall-through and branch targets, loop back-edges
    included) is searched for an instruction that writes one of the
    store's data VGPRs."""
    insns = _parse(text)
    bad, n_stores = [], 0
    for i, (mn, ops, _) in enumerate(insns):
        if mn not in ("buffer_store_dwordx4", "buffer_store_dwordx3"):
            continue
        n_stores += 1
        data = _regs(ops.split(",")[0])
        # depth-first over successors; seen[(index)] = fewest steps to reach it
        stack, seen = [(i, 0)], {}
        while stack:
            k, n = stack.pop()
            mk, _, tk = insns[k]
            succ = []
            if not mk.startswith(("s_branch", "s_endpgm", "s_setpc")):
                succ.append(k + 1)
            if tk is not None:
                succ.append(tk)
            for j in succ:
                if j >= len(insns):
                    continue
                nj = n + 1
                if nj >= MIN_DISTANCE or seen.get(j, MIN_DISTANCE + 1) <= nj:
                    continue
                seen[j] = nj
                mj, oj, _ = insns[j]
                if _writes_vgprs(mj, oj) & data:
                    bad.append((mn + " " + ops, mj + " " + oj, nj))
                    stack.clear()
                    break
                stack.append((j, nj))
            if bad and bad[-1][0] == mn + " " + ops:
                break
    return bad, n_stores


def test_row_store_data_registers_not_overwritten_at_once(tmp_path):
    objs = sorted(glob.glob(os.path.join(BUILD, "code_*.o")))
    if not objs:
        pytest.skip("the library is not built (python -m paper_1608_00066_amd.build)")
    for tool in ("llvm-objcopy", "clang-offload-bundler", "llvm-objdump"):
        if not shutil.which(os.path.join(LLVM, tool)):
            pytest.skip("ROCm LLVM tools not found")
    total = 0
    for obj in objs:
        bad, n = _violations(_disassemble(obj, str(tmp_path)))
        total += n
        assert not bad, "%s: a store's data VGPRs are overwritten %d instructions later: %s / %s" % (
            os.path.basename(obj), bad[0][2], bad[0][0], bad[0][1])
    assert total == 0, "%d buffer stores of more than 8 bytes in the decoder kernels" % total
