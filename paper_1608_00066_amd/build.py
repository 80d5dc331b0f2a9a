"""Build ``libpbvd.so`` (HIP kernels for gfx950 + the C ABI) in-tree.

Every translation unit is compiled with hipcc for gfx950 only; the per-code
kernel unit is compiled once per registered code so the builds run in
parallel.  Usage: ``python -m paper_1608_00066_amd.build`` or ``build()``.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libpbvd.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
# -packed-fp32-ops: keep hipcc from forming packed fp32 instructions
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", INCLUDE, "-I", CSRC]


def _registry_rows(macro: str, csrc: str = CSRC) -> int:
    """Rows X(...) of one list macro of the registry header."""
    with open(os.path.join(csrc, "pbvd_registry.hpp")) as f:
        text = f.read()
    body = text[text.index("#define " + macro):]
    rows = 0
    for line in body.split("\n")[1:]:
        if not re.match(r"^\s*X\(\d+,", line):
            break
        rows += 1
    return rows


def num_codes() -> int:
    return _registry_rows("PBVD_CODE_LIST(X)")


def num_pairs() -> int:
    return _registry_rows("PBVD_PAIR_LIST(X)")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(line for line in r.stdout.splitlines()
                    if "packed-fp32-ops" not in line)
    if r.returncode != 0:
        raise RuntimeError("command failed (%d): %s\n%s" % (r.returncode, " ".join(cmd), out))
    return out


def build(jobs: int | None = None, verbose: bool = False, csrc: str = CSRC,
          build_dir: str = BUILD_DIR, lib: str = LIB, defines=(), incremental: bool = False) -> str:
    """Compile every unit and link ``libpbvd.so``; returns its path.
    ``csrc``/``build_dir``/``lib``/``defines`` let a copy of the sources be
    built elsewhere with other tuning macros.  ``incremental`` keeps object
    files newer than every source and header (a full build otherwise)."""
    os.makedirs(build_dir, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    flags = [f if f.startswith("-") else "-D" + f for f in defines]
    flags += ["-I", csrc]
    units = []
    for i in range(num_codes()):
        units.append((os.path.join(csrc, "pbvd_code_inst.hip"),
                      os.path.join(build_dir, "code_%02d.o" % i), ["-DPBVD_CODE_IDX=%d" % i]))
    for i in range(num_pairs()):
        for kind in (0, 1):
            units.append((os.path.join(csrc, "pbvd_pair_inst.hip"),
                          os.path.join(build_dir, "pair_%02d_%d.o" % (i, kind)),
                          ["-DPBVD_PAIR_IDX=%d" % i, "-DPBVD_PAIR_KIND=%d" % kind]))
    for k in range(3, 10):
        units.append((os.path.join(csrc, "pbvd_wave_inst.hip"),
                      os.path.join(build_dir, "wave_k%d.o" % k), ["-DPBVD_WAVE_K=%d" % k]))
        units.append((os.path.join(csrc, "pbvd_group_inst.hip"),
                      os.path.join(build_dir, "group_k%d.o" % k), ["-DPBVD_GROUP_K=%d" % k]))
    for name in ("pbvd_capi", "pbvd_batch", "pbvd_server", "pbvd_aux"):
        units.append((os.path.join(csrc, name + ".hip"), os.path.join(build_dir, name + ".o"), []))

    def newest_dep(src):
        """Latest modification time of a source and the local headers it
        includes (directly or not)."""
        seen, stack, t = set(), [src], 0.0
        while stack:
            f = stack.pop()
            if f in seen or not os.path.exists(f):
                continue
            seen.add(f)
            t = max(t, os.path.getmtime(f))
            with open(f) as fh:
                for name in re.findall(r'^\s*#\s*include\s+"([^"]+)"', fh.read(), flags=re.M):
                    for d in (csrc, INCLUDE):
                        stack.append(os.path.join(d, name))
        return t

    def compile_unit(u):
        src, obj, extra = u
        if (incremental and not defines and os.path.exists(obj)
                and os.path.getmtime(obj) > newest_dep(src)):
            return obj
        _run([HIPCC, *COMMON[:-2], *flags, *extra, "-c", src, "-o", obj])
        if verbose:
            print("built", os.path.basename(obj), flush=True)
        return obj

    # longest units first: the pair kernels, then the per-code kernels
    order = {"pair": 0, "code": 1}
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_unit, sorted(
            units, key=lambda u: (order.get(os.path.basename(u[1]).split("_")[0], 2), u[1]))))
    tmp = lib + ".tmp%d" % os.getpid()
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *sorted(objs)])
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    path = build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv)
    print(path)
