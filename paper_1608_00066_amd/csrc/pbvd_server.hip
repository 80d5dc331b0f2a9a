// Request server (pbvd_server_* of include/pbvd.h): continuous batching of
// independent decode requests.
//
// Submitters hand in one frame each (host symbols, host output buffer).  A
// worker thread owns `max_inflight` batch slots.  Each slot has a fixed part
// of the device budget (inputs, outputs, work list, survivor rows), pinned
// staging buffers and its own stream.  Whenever a slot is free and requests
// wait, the worker admits as many as fit the slot (FIFO), uploads their
// symbols and work list with one copy, launches the batched decode kernels
// (one per code, cheapest first) each with its read-back, and returns to
// admitting; finished codes and slots are reaped by polling their events.
// So requests that arrive while other batches run are decoded concurrently
// with them, and a request's bits do not depend on what it was batched with:
// every frame is decoded exactly as pbvd_decode would decode it alone.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pbvd.h"
#include "pbvd_host.hpp"
#include "pbvd_registry.hpp"

using namespace pbvd_host;

namespace {

constexpr int kMaxInflight = 8;
constexpr int64_t kAlign = 256;
constexpr int64_t kIdleSpinNs = 2000000;  // worker polls 2 ms before it sleeps

int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    int64_t ticket = 0;
    int32_t code = 0;
    int64_t n_bits = 0;
    std::vector<uint8_t> syms;  // copy of the caller's symbols
    uint8_t *out = nullptr;     // caller's host buffer, ceil(n_bits/8) bytes
    int64_t submit_ns = 0, start_ns = 0, done_ns = 0;
    int32_t batch_frames = 0;
    int32_t status = PBVD_OK;
    bool done = false;
    // admission footprint: all PBs, and those of them that start their
    // traceback from the best state (the end of an unterminated frame)
    int64_t sym_bytes = 0, out_bytes = 0, n_pbs = 0, n_argmin_pbs = 0;
};

// PBs of a frame that start their traceback from the best state: on an
// unterminated frame, every PB whose forward range reaches the last stage T
// (bD + D + L >= T); with L >= D there are several.
int64_t argmin_pbs(const pbvd_code &c, int64_t n_bits) {
    if (c.terminated) return 0;
    const int64_t nb = ceil_div(n_bits, c.D);
    const int64_t T = n_bits;
    const int64_t lim = T - c.D - c.L;  // b*D >= lim
    const int64_t first = lim <= 0 ? 0 : ceil_div(lim, c.D);
    return first >= nb ? 0 : nb - first;
}

// Bytes a set of requests needs in one slot.  Tile count per code, an upper
// bound of what build_work_list makes: the other PBs fill whole waves, plus
// one partial tile at each change of the first traced stage (PBs b with
// b*D < L start at stage b*D, the others at L: at most ceil(L/D) changes),
// and every best-state-start PB is counted as a tile of its own (they share
// tiles only with PBs of the same length).
struct Footprint {
    int64_t sym = 0, out = 0, frames = 0;
    int64_t pbs[kMaxCodes] = {};
    int64_t argmin[kMaxCodes] = {};

    void add(const Request &r, const CodeSet &) {
        sym += r.sym_bytes;
        out += r.out_bytes;
        frames += 1;
        pbs[r.code] += r.n_pbs - r.n_argmin_pbs;
        argmin[r.code] += r.n_argmin_pbs;
    }
    // lb[] of the code set: 64 >> lb PBs per tile; the state-parallel
    // kernel (kWaveLb) takes one PB per wave and one descriptor per PB
    int64_t tiles(int ci, const CodeSet &cs) const {
        if (cs.lb[ci] == kWaveLb) return pbs[ci] + argmin[ci];
        const int64_t splits = pbs[ci] > 0 ? ceil_div((int64_t)cs.codes[ci].L, cs.codes[ci].D) : 0;
        return ceil_div(pbs[ci], pbvd::kWave >> cs.lb[ci]) + splits + argmin[ci];
    }
    int64_t lanes_bytes(const CodeSet &cs) const {
        int64_t t = 0;
        for (int ci = 0; ci < cs.n; ++ci)
            if (cs.lb[ci] != kWaveLb) t += tiles(ci, cs);
        return align_up(t * pbvd::kWave * (int64_t)sizeof(pbvd::LaneDesc));
    }
    int64_t heads_bytes(const CodeSet &cs) const {
        int64_t t = 0;
        for (int ci = 0; ci < cs.n; ++ci)
            if (cs.lb[ci] != kWaveLb) t += tiles(ci, cs);
        return align_up(t * (int64_t)sizeof(pbvd::TileHead));
    }
    int64_t descs_bytes(const CodeSet &cs) const {
        int64_t t = 0;
        for (int ci = 0; ci < cs.n; ++ci)
            if (cs.lb[ci] == kWaveLb) t += tiles(ci, cs);
        return align_up(t * (int64_t)sizeof(pbvd::LaneDesc));
    }
    int64_t sp_bytes(const CodeSet &cs) const {
        int64_t b = 0;
        for (int ci = 0; ci < cs.n; ++ci) {
            const int64_t per = cs.lb[ci] == kWaveLb ? wave_slot_dwords(cs.codes[ci])
                                                     : slot_dwords(cs.codes[ci], cs.lb[ci]);
            b += align_up(tiles(ci, cs) * per * 4);
        }
        return b;
    }
    int64_t in_bytes(const CodeSet &cs) const {
        return align_up(sym) + lanes_bytes(cs) + heads_bytes(cs) + descs_bytes(cs);
    }
    int64_t device_bytes(const CodeSet &cs) const { return in_bytes(cs) + align_up(out) + sp_bytes(cs); }
};

// One batch in flight on the slot's stream: upload, then per code (cheapest
// first) its kernels, its read-back and its completion event, so a code's
// requests finish without waiting for slower codes of the batch; the slot
// is free again once every code has finished.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done[kMaxCodes] = {};
    uint8_t *dev = nullptr;       // this slot's part of the device arena
    uint8_t *pin_in = nullptr;    // symbols + work list staging
    uint8_t *pin_out = nullptr;   // decoded bits staging
    std::vector<std::shared_ptr<Request>> reqs;  // grouped by code
    std::vector<int64_t> out_off;
    bool pending[kMaxCodes] = {};  // codes whose results are not back yet
    int n_pending = 0;
    bool busy = false;
};

}  // namespace

struct pbvd_server {
    CodeSet cs;
    pbvd_server_config cfg{};
    int device = 0;
    int64_t slot_bytes = 0, pin_in_bytes = 0, pin_out_bytes = 0;
    uint8_t *arena = nullptr;
    Slot slots[kMaxInflight];

    std::mutex mu;
    std::condition_variable cv_work;  // worker: new request or stop
    std::condition_variable cv_done;  // waiters: a request finished
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<int64_t, std::shared_ptr<Request>> live;
    int64_t next_ticket = 1;
    bool stop = false;
    std::atomic<int64_t> queued{0};
    std::thread worker;

    // counters (under mu)
    int64_t n_batches = 0, n_done = 0, peak_inflight = 0;
};

namespace {

// Launches one admitted batch on a slot; returns the first failure.
pbvd_status launch_slot(pbvd_server *sv, Slot &sl) {
    const CodeSet &cs = sv->cs;
    const int64_t n = (int64_t)sl.reqs.size();
    // group by code (first come first within a code): each code's outputs
    // are then one contiguous range to read back
    std::stable_sort(sl.reqs.begin(), sl.reqs.end(),
                     [](const std::shared_ptr<Request> &a, const std::shared_ptr<Request> &b) {
                         return a->code < b->code;
                     });
    int64_t out_lo[kMaxCodes], out_hi[kMaxCodes];
    for (int ci = 0; ci < kMaxCodes; ++ci) out_lo[ci] = out_hi[ci] = 0;
    std::vector<pbvd_frame> frames((size_t)n);
    sl.out_off.assign((size_t)n, 0);
    int64_t so = 0, oo = 0;
    for (int64_t i = 0; i < n; ++i) {
        const Request &r = *sl.reqs[(size_t)i];
        memcpy(sl.pin_in + so, r.syms.data(), (size_t)r.sym_bytes);
        frames[(size_t)i] = pbvd_frame{so, r.n_bits, oo, r.code, 0};
        sl.out_off[(size_t)i] = oo;
        if (i == 0 || sl.reqs[(size_t)i - 1]->code != r.code) out_lo[r.code] = oo;
        so += r.sym_bytes;
        oo += r.out_bytes;
        out_hi[r.code] = oo;
    }
    const int64_t sym_total = so, out_total = oo;
    WorkList wl;
    pbvd_status st = build_work_list(cs, frames.data(), n, sym_total, out_total, &wl);
    if (st != PBVD_OK) return st;
    // layout (device and pinned-in share the first four parts):
    // [symbols | lanes | heads | descs | outputs | survivors of code 0 | code 1 ...]
    const int64_t lanes_off = align_up(sym_total);
    const int64_t heads_off = lanes_off + align_up((int64_t)(wl.lanes.size() * sizeof(pbvd::LaneDesc)));
    const int64_t descs_off = heads_off + align_up((int64_t)(wl.heads.size() * sizeof(pbvd::TileHead)));
    const int64_t in_total = descs_off + align_up((int64_t)(wl.descs.size() * sizeof(pbvd::LaneDesc)));
    const int64_t out_dev = in_total;
    int64_t sp_off[kMaxCodes], end = out_dev + align_up(out_total);
    for (int ci = 0; ci < cs.n; ++ci) {
        sp_off[ci] = end;
        end += align_up(wl.groups[ci].n_tiles * wl.groups[ci].sp_wave_dwords * 4);
    }
    if (end > sv->slot_bytes || in_total > sv->pin_in_bytes || out_total > sv->pin_out_bytes)
        return fail(PBVD_ENOMEM, "batch exceeds its slot (%lld of %lld bytes)", (long long)end,
                    (long long)sv->slot_bytes);
    memcpy(sl.pin_in + lanes_off, wl.lanes.data(), wl.lanes.size() * sizeof(pbvd::LaneDesc));
    memcpy(sl.pin_in + heads_off, wl.heads.data(), wl.heads.size() * sizeof(pbvd::TileHead));
    memcpy(sl.pin_in + descs_off, wl.descs.data(), wl.descs.size() * sizeof(pbvd::LaneDesc));

    hipError_t e = hipMemcpyAsync(sl.dev, sl.pin_in, (size_t)in_total, hipMemcpyHostToDevice, sl.stream);
    if (e != hipSuccess) return fail_hip(e, "request upload");
    int active[kMaxCodes], n_active = 0;
    for (int ci = 0; ci < cs.n; ++ci)
        if (wl.groups[ci].n_tiles > 0) active[n_active++] = ci;
    const uint8_t *d_syms = sl.dev;
    const pbvd::LaneDesc *d_lanes = reinterpret_cast<const pbvd::LaneDesc *>(sl.dev + lanes_off);
    const pbvd::TileHead *d_heads = reinterpret_cast<const pbvd::TileHead *>(sl.dev + heads_off);
    const pbvd::LaneDesc *d_descs = reinterpret_cast<const pbvd::LaneDesc *>(sl.dev + descs_off);
    uint8_t *d_out = sl.dev + out_dev;
    // the codes run one after another on the slot's stream, cheapest first
    // (2^K R), each followed by its read-back and completion event: a code's
    // requests finish when its own kernel is done, and a slot's work stays on
    // one hardware queue, so batches in other slots are not queued behind it
    std::sort(active, active + n_active, [&cs](int x, int y) {
        const int64_t wx = (int64_t)cs.codes[x].R << cs.codes[x].K;
        const int64_t wy = (int64_t)cs.codes[y].R << cs.codes[y].K;
        return wx != wy ? wx < wy : x < y;
    });
    for (int k = 0; k < n_active; ++k) {
        const int ci = active[k];
        st = launch_group(cs, ci, wl.groups[ci], d_syms, sym_total, d_out, d_lanes, d_heads, d_descs,
                          reinterpret_cast<uint32_t *>(sl.dev + sp_off[ci]), wl.groups[ci].n_tiles, sl.stream);
        if (st != PBVD_OK) return st;
        e = hipMemcpyAsync(sl.pin_out + out_lo[ci], d_out + out_lo[ci], (size_t)(out_hi[ci] - out_lo[ci]),
                           hipMemcpyDeviceToHost, sl.stream);
        if (e != hipSuccess) return fail_hip(e, "result read-back");
        e = hipEventRecord(sl.done[ci], sl.stream);
        if (e != hipSuccess) return fail_hip(e, "completion event");
        sl.pending[ci] = true;
        sl.n_pending += 1;
    }
    return PBVD_OK;
}

// Takes requests from the queue front while they fit one slot (under mu).
void admit(pbvd_server *sv, Slot &sl) {
    Footprint fp;
    while (!sv->queue.empty() && fp.frames < sv->cfg.max_batch_frames) {
        Footprint next = fp;
        next.add(*sv->queue.front(), sv->cs);
        if (next.device_bytes(sv->cs) > sv->slot_bytes || next.in_bytes(sv->cs) > sv->pin_in_bytes ||
            next.out > sv->pin_out_bytes)
            break;
        fp = next;
        sl.reqs.push_back(sv->queue.front());
        sv->queue.pop_front();
    }
    sv->queued.store((int64_t)sv->queue.size());
}

// Hands the requests of code `ci` (all codes if ci < 0) back to their callers.
void finish(pbvd_server *sv, Slot &sl, int ci, pbvd_status st) {
    const int64_t t = now_ns();
    int64_t count = 0;
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
        Request &r = *sl.reqs[i];
        if (ci >= 0 && r.code != ci) continue;
        if (st == PBVD_OK) memcpy(r.out, sl.pin_out + sl.out_off[i], (size_t)r.out_bytes);
        ++count;
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (auto &r : sl.reqs) {
            if (ci >= 0 && r->code != ci) continue;
            r->status = st;
            r->done_ns = t;
            r->done = true;
        }
        sv->n_done += count;
    }
    sv->cv_done.notify_all();
    if (ci >= 0) {
        sl.pending[ci] = false;
        sl.n_pending -= 1;
    } else {
        for (int k = 0; k < kMaxCodes; ++k) sl.pending[k] = false;
        sl.n_pending = 0;
    }
    if (sl.n_pending == 0) {
        sl.reqs.clear();
        sl.busy = false;
    }
}

void worker_main(pbvd_server *sv) {
    (void)hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        // admit into every free slot
        for (int i = 0; i < sv->cfg.max_inflight && !sv->queue.empty(); ++i) {
            Slot &sl = sv->slots[i];
            if (sl.busy) continue;
            admit(sv, sl);
            if (sl.reqs.empty()) break;  // the head request waits for a slot to drain
            sl.busy = true;
            sv->n_batches += 1;
            int inflight = 0;
            for (int k = 0; k < sv->cfg.max_inflight; ++k) inflight += sv->slots[k].busy ? 1 : 0;
            sv->peak_inflight = std::max<int64_t>(sv->peak_inflight, inflight);
            const int64_t t = now_ns();
            for (auto &r : sl.reqs) {
                r->start_ns = t;
                r->batch_frames = (int32_t)sl.reqs.size();
            }
            lk.unlock();
            pbvd_status st;
            try {
                st = launch_slot(sv, sl);
            } catch (...) {
                st = fail(PBVD_ENOMEM, "host allocation failed while building a batch");
            }
            if (st != PBVD_OK) {
                (void)hipDeviceSynchronize();
                finish(sv, sl, -1, st);
            }
            lk.lock();
        }
        bool any_busy = false;
        for (int i = 0; i < sv->cfg.max_inflight; ++i) any_busy = any_busy || sv->slots[i].busy;
        if (!any_busy) {
            if (sv->stop && sv->queue.empty()) break;
            // idle: poll for a new request for a short while before sleeping,
            // since waking a sleeping thread costs tens of microseconds
            lk.unlock();
            const int64_t spin_end = now_ns() + kIdleSpinNs;
            while (sv->queued.load() == 0 && now_ns() < spin_end) std::this_thread::yield();
            lk.lock();
            sv->cv_work.wait(lk, [sv] { return sv->stop || !sv->queue.empty(); });
            continue;
        }
        // reap finished slots; go back to admitting as soon as a request
        // waits and a slot is free
        lk.unlock();
        for (;;) {
            bool reaped = false, any_free = false;
            for (int i = 0; i < sv->cfg.max_inflight; ++i) {
                Slot &sl = sv->slots[i];
                if (!sl.busy) {
                    any_free = true;
                    continue;
                }
                for (int ci = 0; ci < sv->cs.n && sl.busy; ++ci) {
                    if (!sl.pending[ci]) continue;
                    const hipError_t q = hipEventQuery(sl.done[ci]);
                    if (q == hipSuccess) {
                        finish(sv, sl, ci, PBVD_OK);
                        reaped = true;
                    } else if (q != hipErrorNotReady) {
                        (void)fail_hip(q, "batch execution");
                        (void)hipDeviceSynchronize();
                        finish(sv, sl, -1, PBVD_EHIP);
                        reaped = true;
                    }
                }
            }
            if (reaped || (any_free && sv->queued.load() > 0)) break;
            std::this_thread::yield();
        }
        lk.lock();
    }
}

void release(pbvd_server *sv) {
    DeviceGuard dg(sv->device);
    (void)hipDeviceSynchronize();
    for (Slot &sl : sv->slots) {
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        for (int i = 0; i < kMaxCodes; ++i)
            if (sl.done[i]) (void)hipEventDestroy(sl.done[i]);
        if (sl.pin_in) (void)hipHostFree(sl.pin_in);
        if (sl.pin_out) (void)hipHostFree(sl.pin_out);
    }
    if (sv->arena) (void)hipFree(sv->arena);
}

}  // namespace

extern "C" {

pbvd_status pbvd_server_create(const pbvd_code *codes, int32_t n_codes, const pbvd_server_config *cfg,
                               pbvd_server **out) {
    g_last_error[0] = 0;
    if (!codes || !cfg || !out) return fail(PBVD_EINVAL, "codes, cfg and out must not be NULL");
    if (cfg->max_inflight < 1 || cfg->max_inflight > kMaxInflight)
        return fail(PBVD_EINVAL, "max_inflight must be in [1, %d]", kMaxInflight);
    if (cfg->max_batch_frames < 1) return fail(PBVD_EINVAL, "max_batch_frames must be >= 1");
    if (cfg->max_queued < 1) return fail(PBVD_EINVAL, "max_queued must be >= 1");
    if (cfg->device_bytes < ((int64_t)cfg->max_inflight << 20))
        return fail(PBVD_EINVAL, "device_bytes must be at least 1 MiB per batch in flight");
    CodeSet cs;
    // latency first: codes that leave the mapping to the library decode on
    // the state-parallel kernel (a PB 64 lanes wide)
    pbvd_status st = make_code_set(codes, n_codes, &cs, kWaveLb);
    if (st != PBVD_OK) return st;
    for (int ci = 0; ci < cs.n; ++ci)
        if (cs.lb[ci] == kGroupLb)
            return fail(PBVD_ENOTSUP, "code %d: the server decodes on the register or the state-parallel mapping",
                        ci);
    pbvd_server *sv = new (std::nothrow) pbvd_server();
    if (!sv) return fail(PBVD_ENOMEM, "host allocation failed");
    sv->cs = cs;
    sv->cfg = *cfg;
    if (hipGetDevice(&sv->device) != hipSuccess) sv->device = 0;
    (void)hipGetLastError();
    sv->slot_bytes = cfg->device_bytes / cfg->max_inflight / kAlign * kAlign;
    // symbols and work list are a small part of a batch next to its survivor
    // rows (at least 2L+D rows of 2^(K-1) bits per PB against R bytes per stage)
    sv->pin_in_bytes = align_up(sv->slot_bytes / 4);
    sv->pin_out_bytes = align_up(sv->slot_bytes / 16);
    {
        DeviceGuard dg(sv->device);
        hipError_t e = dg.ok ? hipSuccess : hipErrorInvalidDevice;
        if (e == hipSuccess) e = hipMalloc(&sv->arena, (size_t)sv->slot_bytes * cfg->max_inflight);
        for (int i = 0; i < cfg->max_inflight && e == hipSuccess; ++i) {
            Slot &sl = sv->slots[i];
            sl.dev = sv->arena + (int64_t)i * sv->slot_bytes;
            e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
            for (int c = 0; c < cs.n && e == hipSuccess; ++c)
                e = hipEventCreateWithFlags(&sl.done[c], hipEventDisableTiming);
            if (e == hipSuccess) e = hipHostMalloc((void **)&sl.pin_in, (size_t)sv->pin_in_bytes, hipHostMallocDefault);
            if (e == hipSuccess) e = hipHostMalloc((void **)&sl.pin_out, (size_t)sv->pin_out_bytes, hipHostMallocDefault);
        }
        if (e != hipSuccess) {
            st = e == hipErrorOutOfMemory ? fail(PBVD_ENOMEM, "server buffers: %s", hipGetErrorString(e))
                                          : fail_hip(e, "server set-up");
            (void)hipGetLastError();
            release(sv);
            delete sv;
            return st;
        }
    }
    try {
        sv->worker = std::thread(worker_main, sv);
    } catch (...) {
        release(sv);
        delete sv;
        return fail(PBVD_ENOMEM, "cannot start the worker thread");
    }
    *out = sv;
    return PBVD_OK;
}

pbvd_status pbvd_server_submit(pbvd_server *sv, int32_t code, const void *syms, int64_t n_bits,
                               uint8_t *out_bits, int64_t *ticket) {
    g_last_error[0] = 0;
    if (!sv || !syms || !out_bits || !ticket) return fail(PBVD_EINVAL, "NULL argument");
    if (code < 0 || code >= sv->cs.n) return fail(PBVD_EINVAL, "bad code index %d", code);
    if (n_bits < 1) return fail(PBVD_EINVAL, "n_bits must be >= 1");
    const pbvd_code &c = sv->cs.codes[code];
    std::shared_ptr<Request> r;
    try {
        r = std::make_shared<Request>();
        r->code = code;
        r->n_bits = n_bits;
        r->sym_bytes = (n_bits + (c.terminated ? c.K - 1 : 0)) * c.R;
        r->out_bytes = ceil_div(n_bits, 8);
        r->n_pbs = ceil_div(n_bits, c.D);
        r->n_argmin_pbs = argmin_pbs(c, n_bits);
        Footprint alone;
        alone.add(*r, sv->cs);
        if (alone.device_bytes(sv->cs) > sv->slot_bytes || alone.in_bytes(sv->cs) > sv->pin_in_bytes ||
            alone.out > sv->pin_out_bytes)
            return fail(PBVD_EINVAL, "request of %lld bits needs %lld bytes, more than a batch slot (%lld)",
                        (long long)n_bits, (long long)alone.device_bytes(sv->cs), (long long)sv->slot_bytes);
        r->syms.assign((const uint8_t *)syms, (const uint8_t *)syms + r->sym_bytes);
        r->out = out_bits;
    } catch (...) {
        return fail(PBVD_ENOMEM, "host allocation failed");
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) return fail(PBVD_EINVAL, "server is shutting down");
        if ((int64_t)sv->queue.size() >= sv->cfg.max_queued)
            return fail(PBVD_EAGAIN, "queue full (%lld requests)", (long long)sv->queue.size());
        r->ticket = sv->next_ticket++;
        r->submit_ns = now_ns();
        try {
            sv->live.emplace(r->ticket, r);
            sv->queue.push_back(r);
        } catch (...) {
            sv->live.erase(r->ticket);
            return fail(PBVD_ENOMEM, "host allocation failed");
        }
        sv->queued.store((int64_t)sv->queue.size());
        *ticket = r->ticket;
    }
    sv->cv_work.notify_one();
    return PBVD_OK;
}

pbvd_status pbvd_server_wait(pbvd_server *sv, int64_t ticket, int64_t timeout_us, pbvd_request_info *info) {
    g_last_error[0] = 0;
    if (!sv) return fail(PBVD_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->live.find(ticket);
    if (it == sv->live.end()) return fail(PBVD_EINVAL, "unknown ticket %lld", (long long)ticket);
    std::shared_ptr<Request> r = it->second;
    auto ready = [&r] { return r->done; };
    if (timeout_us < 0) {
        sv->cv_done.wait(lk, ready);
    } else if (!sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return fail(PBVD_EAGAIN, "request %lld not finished", (long long)ticket);
    }
    if (info) {
        info->submit_ns = r->submit_ns;
        info->start_ns = r->start_ns;
        info->done_ns = r->done_ns;
        info->batch_frames = r->batch_frames;
        info->status = r->status;
    }
    sv->live.erase(ticket);
    if (r->status != PBVD_OK) return fail((pbvd_status)r->status, "the batch of request %lld failed", (long long)ticket);
    return PBVD_OK;
}

pbvd_status pbvd_server_counters(pbvd_server *sv, int64_t *batches, int64_t *requests_done,
                                 int64_t *peak_inflight) {
    if (!sv) return fail(PBVD_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (batches) *batches = sv->n_batches;
    if (requests_done) *requests_done = sv->n_done;
    if (peak_inflight) *peak_inflight = sv->peak_inflight;
    return PBVD_OK;
}

void pbvd_server_destroy(pbvd_server *sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    release(sv);
    delete sv;
}

}  // extern "C"
