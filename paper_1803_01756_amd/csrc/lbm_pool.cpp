// Slot pool: many independent channels stepped together (batched) and a
// request pool with admission by device footprint (served).  C-ABI in
// include/lbm.h (lbm_pool_*).
//
// Streams.  Chunks of steps run on the main stream, one batched launch per
// step over every active slot.  Slot start-up (zero fill, density upload,
// rest-equilibrium init) and result read-out (moments, device-to-host copy)
// run on an auxiliary stream, ordered against the main stream with events
// only, so a request can be admitted or read out while the batch runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "lbm.h"
#include "lbm_host.h"
#include "lbm_internal.h"

using lbmhost::fail;

namespace {

#define PCHK(expr)                                                                        \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(LBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

struct SlotState {
    bool used = false;
    lbm_params p;
    lbmhost::Layout L;
    lbmk::Grid g;
    lbmk::Phys k;
    char* mem = nullptr;
    size_t bytes = 0;        // footprint counted against the cap
    size_t block = 0;        // size of the device block holding it
    float* f[2] = {nullptr, nullptr};
    float* T[2] = {nullptr, nullptr};
    int cur_f = 0, cur_T = 0;
    int64_t n = 0;           // time level after the work enqueued so far
    int64_t steps_left = 0;  // steps still to enqueue
    bool ready_waited = false;
    bool reported = false;
    bool failed = false;     // retired early: its state became non-finite
    hipEvent_t ready = nullptr;  // start-up finished (aux stream)
    hipEvent_t done = nullptr;   // last enqueued chunk touching the slot finished (main)
    // the host copy of the counters after the slot's first chunk has landed:
    // from then on the mirrored counters are this slot's (an earlier copy may
    // still carry the counters of a released slot that had the same id)
    hipEvent_t counted = nullptr;
    bool counted_recorded = false;
};

// words per slot in the health-counter array: non-finite readings, clamps
constexpr int kSlotStat = 2;

// Buckets of fluid rows for the tuned launch shapes: up to 32, 64, 128, 256
// rows, and more.
constexpr int kRowBuckets = 5;
int row_bucket(int rows) {
    int b = 0;
    while (b < kRowBuckets - 1 && rows > (32 << b)) ++b;
    return b;
}

// Segments of about `target` rows, balanced over the slot's rows, with
// seg + 10 (the recomputed halo rows) a multiple of the six-row unroll.
int balanced_seg_rows(int rows, int target) {
    const int segs = std::max(1, (rows + target - 1) / target);
    int sr = (rows + segs - 1) / segs;
    sr = sr + (6 - (sr + 10) % 6) % 6;
    return std::min(sr, rows);
}

size_t slot_bytes(const lbmhost::Layout& L) {
    return 2 * lbmhost::align_up(9 * L.plane * 4) + 2 * lbmhost::align_up(L.plane * 4);
}

}  // namespace

struct lbm_pool {
    int dev = 0;
    size_t cap = 0, used = 0;
    hipStream_t main = nullptr, aux = nullptr;
    bool owns_main = false;
    std::vector<SlotState> slots;
    int seg_cap = 0;  // rows per wave in the batch (0: per-slot default)
    // tuned segment heights per bucket of fluid rows (lbm_pool_autotune;
    // 0: the default heuristic)
    int seg_target[kRowBuckets] = {};
    // table of the batched kernel: device copy and two pinned host stagings
    lbmk::Slot* table_dev = nullptr;
    lbmk::Slot* table_host[2] = {nullptr, nullptr};
    hipEvent_t table_free[2] = {nullptr, nullptr};
    int table_cap = 0, table_next = 0;
    // moment scratch on the aux stream: 7 doubles per node of the largest slot
    double* mom = nullptr;
    size_t mom_cells = 0;
    // health counters: kSlotStat words per slot id on the device (the step
    // adds to them), mirrored into pinned host memory after every chunk; the
    // last word of the array counts non-finite nodes of a read-out
    unsigned long long* stat_dev = nullptr;
    unsigned long long* stat_host = nullptr;
    int stat_cap = 0;
    // device blocks of released slots, reused by later admissions (freeing
    // device memory can stall the device while a batch runs)
    std::vector<std::pair<char*, size_t>> spare;
    int64_t steps_enqueued = 0;
    // completion events of the chunks enqueued and not yet waited for
    std::vector<hipEvent_t> chunk_events, spare_events;
};

namespace {

lbm_status ensure_table(lbm_pool* P, int n) {
    if (n <= P->table_cap) return LBM_OK;
    PCHK(hipStreamSynchronize(P->main));
    for (int b = 0; b < 2; ++b) {
        if (P->table_host[b]) PCHK(hipHostFree(P->table_host[b]));
        P->table_host[b] = nullptr;
    }
    if (P->table_dev) PCHK(hipFree(P->table_dev));
    P->table_dev = nullptr;
    const int cap = std::max(n, 2 * P->table_cap);
    PCHK(hipMalloc(reinterpret_cast<void**>(&P->table_dev), cap * sizeof(lbmk::Slot)));
    for (int b = 0; b < 2; ++b)
        PCHK(hipHostMalloc(reinterpret_cast<void**>(&P->table_host[b]), cap * sizeof(lbmk::Slot),
                           hipHostMallocDefault));
    P->table_cap = cap;
    return LBM_OK;
}

lbm_status ensure_mom(lbm_pool* P, size_t cells) {
    if (cells <= P->mom_cells) return LBM_OK;
    PCHK(hipStreamSynchronize(P->aux));
    if (P->mom) PCHK(hipFree(P->mom));
    P->mom = nullptr;
    PCHK(hipMalloc(reinterpret_cast<void**>(&P->mom), cells * 7 * sizeof(double)));
    P->mom_cells = cells;
    return LBM_OK;
}

// Room for the counters of slot ids 0..n-1 (plus the read-out word); a
// larger array is filled from the old one while no stream uses it.
lbm_status ensure_stat(lbm_pool* P, int n) {
    if (n <= P->stat_cap) return LBM_OK;
    PCHK(hipStreamSynchronize(P->main));
    PCHK(hipStreamSynchronize(P->aux));
    const int cap = std::max(n, std::max(64, 2 * P->stat_cap));
    const size_t words = (size_t)cap * kSlotStat + 1;
    unsigned long long *d = nullptr, *h = nullptr;
    PCHK(hipMalloc(reinterpret_cast<void**>(&d), words * sizeof(*d)));
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&h), words * sizeof(*h),
                                 hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemset(d, 0, words * sizeof(*d));
    if (e == hipSuccess && P->stat_dev)
        e = hipMemcpy(d, P->stat_dev, (size_t)P->stat_cap * kSlotStat * sizeof(*d),
                      hipMemcpyDeviceToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        if (h) (void)hipHostFree(h);
        return fail(LBM_EDEVICE, "health counters: %s", hipGetErrorString(e));
    }
    std::memset(h, 0, words * sizeof(*h));
    if (P->stat_host)
        std::memcpy(h, P->stat_host, (size_t)P->stat_cap * kSlotStat * sizeof(*h));
    if (P->stat_dev) (void)hipFree(P->stat_dev);
    if (P->stat_host) (void)hipHostFree(P->stat_host);
    P->stat_dev = d;
    P->stat_host = h;
    P->stat_cap = cap;
    return LBM_OK;
}

SlotState* get_slot(lbm_pool* P, int32_t id) {
    if (!P || id < 0 || id >= (int32_t)P->slots.size() || !P->slots[id].used) return nullptr;
    return &P->slots[id];
}

int seg_rows_for(const lbm_pool* P, const SlotState& s) {
    if (P->seg_cap > 0) return std::min(P->seg_cap, s.L.rows);
    const int t = P->seg_target[row_bucket(s.L.rows)];
    if (t > 0) return balanced_seg_rows(s.L.rows, t);
    // many channels share one launch, so each keeps segments of at least
    // 14 rows rather than aiming at a full round of waves by itself
    return lbmhost::default_seg_rows(s.p, s.L.rows, 14);
}

}  // namespace

extern "C" {

size_t lbm_pool_footprint(const lbm_params* pin) {
    if (!pin) return 0;
    lbm_params p = *pin;
    if (lbm_params_resolve(&p) != LBM_OK || lbmhost::validate(p) != LBM_OK) return 0;
    lbmhost::Layout L;
    lbmhost::make_layout(p, &L);
    return slot_bytes(L);
}

lbm_status lbm_pool_create(size_t cap_bytes, void* stream, lbm_pool** out) {
    if (!out) return fail(LBM_EINVAL, "null output handle");
    *out = nullptr;
    lbm_pool* P = new (std::nothrow) lbm_pool();
    if (!P) return fail(LBM_ENOMEM, "host allocation failed");
    P->cap = cap_bytes;
    hipError_t e = hipGetDevice(&P->dev);
    if (e == hipSuccess) {
        if (stream) {
            P->main = static_cast<hipStream_t>(stream);
        } else {
            e = hipStreamCreate(&P->main);
            P->owns_main = (e == hipSuccess);
        }
    }
    if (e == hipSuccess) e = hipStreamCreate(&P->aux);
    for (int b = 0; b < 2 && e == hipSuccess; ++b)
        e = hipEventCreateWithFlags(&P->table_free[b], hipEventDisableTiming);
    if (e != hipSuccess) {
        lbm_pool_destroy(P);
        return fail(LBM_EDEVICE, "pool set-up: %s", hipGetErrorString(e));
    }
    *out = P;
    return LBM_OK;
}

lbm_status lbm_pool_admit(lbm_pool* P, const lbm_params* pin, const double* rho0,
                          int64_t nsteps, int32_t* slot_out) {
    if (!P || !pin || !slot_out) return fail(LBM_EINVAL, "null argument");
    *slot_out = -1;
    if (nsteps < 0) return fail(LBM_EINVAL, "negative step count");
    lbm_params p = *pin;
    lbm_status st = lbm_params_resolve(&p);
    if (st != LBM_OK) return st;
    st = lbmhost::validate(p);
    if (st != LBM_OK) return st;
    if (p.precision != LBM_FP32_DEV)
        return fail(LBM_EINVAL, "the pool runs FP32 deviation storage only");
    lbmhost::Layout L;
    lbmhost::make_layout(p, &L);
    const size_t need = slot_bytes(L);
    if (P->used + need > P->cap)
        return fail(LBM_ENOMEM, "admission refused: %zu + %zu bytes exceed the %zu-byte cap",
                    P->used, need, P->cap);
    const size_t cells = (size_t)p.Nx * p.Ny;
    st = lbmhost::check_initial(p, rho0);
    if (st != LBM_OK) return st;
    PCHK(hipSetDevice(P->dev));
    st = ensure_mom(P, cells);
    if (st != LBM_OK) return st;

    int id = -1;
    for (size_t i = 0; i < P->slots.size(); ++i)
        if (!P->slots[i].used) {
            id = (int)i;
            break;
        }
    st = ensure_stat(P, id < 0 ? (int)P->slots.size() + 1 : id + 1);
    if (st != LBM_OK) return st;
    if (id < 0) {
        P->slots.emplace_back();
        id = (int)P->slots.size() - 1;
    }
    SlotState& s = P->slots[id];
    s = SlotState();
    s.p = p;
    s.L = L;
    int best = -1;
    for (size_t i = 0; i < P->spare.size(); ++i)
        if (P->spare[i].second >= need && (best < 0 || P->spare[i].second < P->spare[best].second))
            best = (int)i;
    hipError_t e = hipSuccess;
    if (best >= 0) {
        s.mem = P->spare[best].first;
        s.block = P->spare[best].second;
        P->spare.erase(P->spare.begin() + best);
    } else {
        e = hipMalloc(reinterpret_cast<void**>(&s.mem), need);
        if (e != hipSuccess && !P->spare.empty()) {
            (void)hipGetLastError();
            for (auto& b : P->spare) (void)hipFree(b.first);
            P->spare.clear();
            e = hipMalloc(reinterpret_cast<void**>(&s.mem), need);
        }
        if (e != hipSuccess) {
            (void)hipGetLastError();
            s = SlotState();
            return fail(LBM_ENOMEM, "slot allocation of %zu bytes failed", need);
        }
        s.block = need;
    }
    s.bytes = need;
    size_t o = 0;
    for (int b = 0; b < 2; ++b) {
        s.f[b] = reinterpret_cast<float*>(s.mem + o);
        o += lbmhost::align_up(9 * L.plane * 4);
    }
    for (int b = 0; b < 2; ++b) {
        s.T[b] = reinterpret_cast<float*>(s.mem + o);
        o += lbmhost::align_up(L.plane * 4);
    }
    lbmhost::fill_phys(p, s.k);
    lbmhost::fill_grid(p, L, seg_rows_for(P, s), s.g);
    s.steps_left = nsteps;
    s.used = true;
    P->used += need;
    // start-up on the aux stream: the density field goes through the moment
    // scratch, which only the aux stream uses
    std::vector<double> r0(cells, p.rho_v);
    if (rho0) std::copy(rho0, rho0 + cells, r0.begin());
    e = hipMemsetAsync(s.mem, 0, need, P->aux);
    if (e == hipSuccess)
        e = hipMemsetAsync(P->stat_dev + (size_t)id * kSlotStat, 0,
                           kSlotStat * sizeof(unsigned long long), P->aux);
    std::memset(P->stat_host + (size_t)id * kSlotStat, 0, kSlotStat * sizeof(unsigned long long));
    if (e == hipSuccess)
        e = hipMemcpyAsync(P->mom, r0.data(), cells * sizeof(double), hipMemcpyHostToDevice,
                           P->aux);
    if (e == hipSuccess)
        e = lbmk::launch_init_f32(s.g, s.k, P->mom, s.f[0], nullptr, s.T[0], P->aux);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.counted, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(s.ready, P->aux);
    // r0 is pageable host memory: the copy has completed when the call
    // returns, so the vector may go out of scope
    if (e != hipSuccess) {
        lbm_pool_release(P, id);
        return fail(LBM_EDEVICE, "slot start-up: %s", hipGetErrorString(e));
    }
    *slot_out = id;
    return LBM_OK;
}

lbm_status lbm_pool_run(lbm_pool* P, int32_t chunk) {
    if (!P) return fail(LBM_EINVAL, "null pool");
    if (chunk < 1) return fail(LBM_EINVAL, "chunk must be >= 1");
    PCHK(hipSetDevice(P->dev));
    // A slot whose steps have read a non-finite state (as of the last
    // counter copy that has landed) is retired: it takes no further steps
    // and lbm_pool_moments reports it with LBM_EUNSTABLE.  The other slots
    // are untouched: each reads and writes only its own memory.
    for (size_t i = 0; i < P->slots.size(); ++i) {
        SlotState& s = P->slots[i];
        if (s.used && s.steps_left > 0 && s.counted_recorded &&
            P->stat_host[i * kSlotStat] != 0ull && hipEventQuery(s.counted) == hipSuccess) {
            s.steps_left = 0;
            s.failed = true;
        }
    }
    std::vector<int> act;
    for (size_t i = 0; i < P->slots.size(); ++i)
        if (P->slots[i].used && P->slots[i].steps_left > 0) act.push_back((int)i);
    if (act.empty()) return LBM_OK;
    lbm_status st = ensure_table(P, (int)act.size());
    if (st != LBM_OK) return st;
    const int b = P->table_next;
    P->table_next ^= 1;
    PCHK(hipEventSynchronize(P->table_free[b]));  // the staging copy from two chunks ago
    lbmk::Slot* tab = P->table_host[b];
    int units = 0, longest = 0;
    bool ext = false;  // some slot needs the build with the optional features
    for (size_t j = 0; j < act.size(); ++j) {
        SlotState& s = P->slots[act[j]];
        ext = ext || (s.p.flags & (LBM_FRAME_T | LBM_FRAME_RHO | LBM_EOS_CS | LBM_OPEN_X |
                                   LBM_PHASE_PROPS | LBM_TOP_MIXED)) ||
              s.p.T_w_end > 0.0 || s.p.alpha_max > 0.0;
        if (!s.ready_waited) {
            PCHK(hipStreamWaitEvent(P->main, s.ready, 0));
            s.ready_waited = true;
        }
        const int take = (int)std::min<int64_t>(chunk, s.steps_left);
        lbmk::Slot& t = tab[j];
        t.g = s.g;
        t.k = s.k;
        t.mem = s.mem;
        for (int q = 0; q < 2; ++q) {
            t.off_f[q] = (unsigned)(reinterpret_cast<char*>(s.f[q]) - s.mem);
            t.off_T[q] = (unsigned)(reinterpret_cast<char*>(s.T[q]) - s.mem);
        }
        t.span = t.off_T[1] + (unsigned)(s.L.plane * 4);
        t.n0 = s.n;
        t.cur_f = s.cur_f;
        t.cur_T = s.cur_T;
        t.steps_left = take;
        t.unit_begin = units;
        t.stat = P->stat_dev + (size_t)act[j] * kSlotStat;
        units += s.g.n_units;
        longest = std::max(longest, take);
    }
    PCHK(hipMemcpyAsync(P->table_dev, tab, act.size() * sizeof(lbmk::Slot), hipMemcpyHostToDevice,
                        P->main));
    PCHK(hipEventRecord(P->table_free[b], P->main));
    for (int i = 0; i < longest; ++i)
        PCHK(lbmk::launch_step_batched(P->table_dev, (int)act.size(), units, i, ext, P->main));
    for (size_t j = 0; j < act.size(); ++j) {
        SlotState& s = P->slots[act[j]];
        const int take = (int)std::min<int64_t>(chunk, s.steps_left);
        s.n += take;
        s.steps_left -= take;
        s.cur_f ^= (take & 1);
        if (!(s.p.flags & LBM_FREEZE_T)) s.cur_T ^= (take & 1);
        PCHK(hipEventRecord(s.done, P->main));
    }
    // the counters as of the end of this chunk, for the next call's check
    PCHK(hipMemcpyAsync(P->stat_host, P->stat_dev,
                        P->slots.size() * kSlotStat * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, P->main));
    for (size_t j = 0; j < act.size(); ++j) {
        SlotState& s = P->slots[act[j]];
        if (!s.counted_recorded) {
            PCHK(hipEventRecord(s.counted, P->main));
            s.counted_recorded = true;
        }
    }
    P->steps_enqueued += longest;
    hipEvent_t ev = nullptr;
    if (!P->spare_events.empty()) {
        ev = P->spare_events.back();
        P->spare_events.pop_back();
    } else {
        PCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    PCHK(hipEventRecord(ev, P->main));
    P->chunk_events.push_back(ev);
    return LBM_OK;
}

lbm_status lbm_pool_wait(lbm_pool* P, int32_t max_pending) {
    if (!P) return fail(LBM_EINVAL, "null pool");
    if (max_pending < 0) max_pending = 0;
    PCHK(hipSetDevice(P->dev));
    while ((int32_t)P->chunk_events.size() > max_pending) {
        hipEvent_t ev = P->chunk_events.front();
        PCHK(hipEventSynchronize(ev));
        P->chunk_events.erase(P->chunk_events.begin());
        P->spare_events.push_back(ev);
    }
    return LBM_OK;
}

lbm_status lbm_pool_poll(lbm_pool* P, int32_t* done, int32_t max, int32_t* ndone) {
    if (!P || !ndone || (max > 0 && !done)) return fail(LBM_EINVAL, "null argument");
    *ndone = 0;
    for (size_t i = 0; i < P->slots.size() && *ndone < max; ++i) {
        SlotState& s = P->slots[i];
        if (!s.used || s.reported || s.steps_left > 0) continue;
        const hipError_t q = hipEventQuery(s.done);
        if (q == hipSuccess) {
            s.reported = true;
            done[(*ndone)++] = (int32_t)i;
        } else if (q != hipErrorNotReady) {
            return fail(LBM_EDEVICE, "slot %zu: %s", i, hipGetErrorString(q));
        }
    }
    return LBM_OK;
}

lbm_status lbm_pool_moments(lbm_pool* P, int32_t id, double* rho, double* ux, double* uy,
                            double* T) {
    SlotState* s = get_slot(P, id);
    if (!s) return fail(LBM_EINVAL, "no slot %d", id);
    PCHK(hipSetDevice(P->dev));
    // the slot's state after everything enqueued for it so far: `done`
    // marks the end of the last chunk that stepped it (a slot never stepped
    // has an unrecorded `done`, which waits for nothing)
    PCHK(hipStreamWaitEvent(P->aux, s->ready, 0));
    PCHK(hipStreamWaitEvent(P->aux, s->done, 0));
    const size_t cells = (size_t)s->p.Nx * s->p.Ny;
    double* m = P->mom;
    unsigned long long* nb = P->stat_dev + (size_t)P->stat_cap * kSlotStat;
    PCHK(hipMemsetAsync(nb, 0, sizeof(*nb), P->aux));
    PCHK(lbmk::launch_moments_f32(s->g, s->k, s->f[s->cur_f], nullptr, s->T[s->cur_T], m + 4 * cells,
                                  m, m + cells, m + 2 * cells, m + 3 * cells, s->n, nb, P->aux));
    double* outs[4] = {rho, ux, uy, T};
    for (int q = 0; q < 4; ++q)
        if (outs[q])
            PCHK(hipMemcpyAsync(outs[q], m + q * cells, cells * sizeof(double),
                                hipMemcpyDeviceToHost, P->aux));
    unsigned long long st[kSlotStat + 1];
    PCHK(hipMemcpyAsync(st, P->stat_dev + (size_t)id * kSlotStat,
                        kSlotStat * sizeof(unsigned long long), hipMemcpyDeviceToHost, P->aux));
    PCHK(hipMemcpyAsync(st + kSlotStat, nb, sizeof(*nb), hipMemcpyDeviceToHost, P->aux));
    PCHK(hipStreamSynchronize(P->aux));
    if (st[0] || st[kSlotStat])
        return fail(LBM_EUNSTABLE,
                    "slot %d: non-finite state (%llu node readings by its steps up to n = %lld, "
                    "%llu nodes at the read-out)%s", id, st[0], (long long)s->n, st[kSlotStat],
                    s->failed ? "; retired before its last step" : "");
    return LBM_OK;
}

lbm_status lbm_pool_slot_health(lbm_pool* P, int32_t id, int64_t* nonfinite,
                                int64_t* psi_clamps) {
    SlotState* s = get_slot(P, id);
    if (!s) return fail(LBM_EINVAL, "no slot %d", id);
    PCHK(hipSetDevice(P->dev));
    PCHK(hipStreamWaitEvent(P->aux, s->ready, 0));
    PCHK(hipStreamWaitEvent(P->aux, s->done, 0));
    unsigned long long st[kSlotStat];
    PCHK(hipMemcpyAsync(st, P->stat_dev + (size_t)id * kSlotStat, sizeof(st),
                        hipMemcpyDeviceToHost, P->aux));
    PCHK(hipStreamSynchronize(P->aux));
    if (nonfinite) *nonfinite = (int64_t)st[0];
    if (psi_clamps) *psi_clamps = (int64_t)st[1];
    return LBM_OK;
}

lbm_status lbm_pool_release(lbm_pool* P, int32_t id) {
    SlotState* s = get_slot(P, id);
    if (!s) return fail(LBM_EINVAL, "no slot %d", id);
    (void)hipSetDevice(P->dev);
    // nothing may still read or write the slot's memory: the last chunk that
    // included it and any read-out on the aux stream
    if (s->done) (void)hipEventSynchronize(s->done);
    (void)hipStreamSynchronize(P->aux);
    if (s->mem) P->spare.emplace_back(s->mem, s->block);
    if (s->ready) (void)hipEventDestroy(s->ready);
    if (s->done) (void)hipEventDestroy(s->done);
    if (s->counted) (void)hipEventDestroy(s->counted);
    P->used -= s->bytes;
    *s = SlotState();
    return LBM_OK;
}

lbm_status lbm_pool_destroy(lbm_pool* P) {
    if (!P) return LBM_OK;
    (void)hipSetDevice(P->dev);
    if (P->main) (void)hipStreamSynchronize(P->main);
    if (P->aux) (void)hipStreamSynchronize(P->aux);
    for (size_t i = 0; i < P->slots.size(); ++i)
        if (P->slots[i].used) lbm_pool_release(P, (int32_t)i);
    for (int b = 0; b < 2; ++b) {
        if (P->table_host[b]) (void)hipHostFree(P->table_host[b]);
        if (P->table_free[b]) (void)hipEventDestroy(P->table_free[b]);
    }
    for (auto& b : P->spare) (void)hipFree(b.first);
    for (hipEvent_t ev : P->chunk_events) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : P->spare_events) (void)hipEventDestroy(ev);
    if (P->table_dev) (void)hipFree(P->table_dev);
    if (P->mom) (void)hipFree(P->mom);
    if (P->stat_dev) (void)hipFree(P->stat_dev);
    if (P->stat_host) (void)hipHostFree(P->stat_host);
    if (P->aux) (void)hipStreamDestroy(P->aux);
    if (P->owns_main && P->main) (void)hipStreamDestroy(P->main);
    delete P;
    return LBM_OK;
}

lbm_status lbm_pool_info(const lbm_pool* P, int32_t* active, size_t* bytes_used,
                         size_t* cap_bytes) {
    if (!P) return fail(LBM_EINVAL, "null pool");
    int a = 0;
    for (const SlotState& s : P->slots)
        if (s.used) ++a;
    if (active) *active = a;
    if (bytes_used) *bytes_used = P->used;
    if (cap_bytes) *cap_bytes = P->cap;
    return LBM_OK;
}

int64_t lbm_pool_slot_time(const lbm_pool* P, int32_t id) {
    SlotState* s = get_slot(const_cast<lbm_pool*>(P), id);
    return s ? s->n : -1;
}

lbm_status lbm_pool_set_launch(lbm_pool* P, int32_t seg_rows) {
    if (!P) return fail(LBM_EINVAL, "null pool");
    P->seg_cap = seg_rows > 0 ? seg_rows : 0;
    if (seg_rows <= 0)
        for (int& t : P->seg_target) t = 0;
    for (SlotState& s : P->slots)
        if (s.used) lbmhost::fill_grid(s.p, s.L, seg_rows_for(P, s), s.g);
    return LBM_OK;
}

lbm_status lbm_pool_slot_launch(const lbm_pool* P, int32_t id, int32_t* seg_rows,
                                int32_t* waves) {
    const SlotState* s = get_slot(const_cast<lbm_pool*>(P), id);
    if (!s) return fail(LBM_EINVAL, "no slot %d", id);
    if (seg_rows) *seg_rows = s->g.seg_rows;
    if (waves) *waves = s->g.n_units;
    return LBM_OK;
}

lbm_status lbm_pool_autotune(lbm_pool* P, int32_t steps_per_trial, double* best_ms) {
    if (!P) return fail(LBM_EINVAL, "null pool");
    if (steps_per_trial < 1) return fail(LBM_EINVAL, "steps_per_trial must be >= 1");
    PCHK(hipSetDevice(P->dev));
    // the slots of the next chunk (those with steps left; all slots if none has)
    std::vector<int> act;
    for (size_t i = 0; i < P->slots.size(); ++i)
        if (P->slots[i].used && P->slots[i].steps_left > 0) act.push_back((int)i);
    if (act.empty())
        for (size_t i = 0; i < P->slots.size(); ++i)
            if (P->slots[i].used) act.push_back((int)i);
    if (act.empty()) return fail(LBM_EINVAL, "autotune needs admitted slots");
    PCHK(hipStreamSynchronize(P->main));
    PCHK(hipStreamSynchronize(P->aux));
    // Trials run on copies of the slots' memory, so the slots' states,
    // counters and time levels stay as they are.
    size_t total = 0;
    std::vector<size_t> at(act.size());
    for (size_t j = 0; j < act.size(); ++j) {
        at[j] = total;
        total += lbmhost::align_up(P->slots[act[j]].bytes);
    }
    const size_t stat_at = total;
    total += lbmhost::align_up(act.size() * kSlotStat * sizeof(unsigned long long));
    const size_t tab_at = total;
    total += act.size() * sizeof(lbmk::Slot);
    char* shadow = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&shadow), total) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LBM_ENOMEM, "autotune: no room for the %zu-byte trial copy", total);
    }
    std::vector<lbmk::Slot> tab(act.size());
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipError_t e = hipSuccess;
    for (size_t j = 0; j < act.size() && e == hipSuccess; ++j) {
        const SlotState& s = P->slots[act[j]];
        e = hipMemcpyAsync(shadow + at[j], s.mem, s.bytes, hipMemcpyDeviceToDevice, P->main);
    }
    if (e == hipSuccess) e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    bool ext = false;
    int present[kRowBuckets] = {};
    for (int id : act) {
        const SlotState& s = P->slots[id];
        ext = ext || (s.p.flags & (LBM_FRAME_T | LBM_FRAME_RHO | LBM_EOS_CS | LBM_OPEN_X |
                                   LBM_PHASE_PROPS | LBM_TOP_MIXED)) ||
              s.p.T_w_end > 0.0 || s.p.alpha_max > 0.0;
        present[row_bucket(s.L.rows)] = 1;
    }
    // time one policy (segment-height target per bucket) over the copies
    int trial_steps = steps_per_trial;
    auto trial = [&](const int* target, double* ms_out) -> hipError_t {
        int units = 0;
        for (size_t j = 0; j < act.size(); ++j) {
            const SlotState& s = P->slots[act[j]];
            const int t = target[row_bucket(s.L.rows)];
            lbmk::Slot& q = tab[j];
            q.k = s.k;
            lbmhost::fill_grid(s.p, s.L,
                               t > 0 ? balanced_seg_rows(s.L.rows, t)
                                     : lbmhost::default_seg_rows(s.p, s.L.rows, 14),
                               q.g);
            q.mem = shadow + at[j];
            for (int c = 0; c < 2; ++c) {
                q.off_f[c] = (unsigned)(reinterpret_cast<char*>(s.f[c]) - s.mem);
                q.off_T[c] = (unsigned)(reinterpret_cast<char*>(s.T[c]) - s.mem);
            }
            q.span = q.off_T[1] + (unsigned)(s.L.plane * 4);
            q.n0 = s.n;
            q.cur_f = s.cur_f;
            q.cur_T = s.cur_T;
            q.steps_left = trial_steps + 2;
            q.unit_begin = units;
            q.stat = reinterpret_cast<unsigned long long*>(shadow + stat_at) + j * kSlotStat;
            units += q.g.n_units;
        }
        auto* dtab = reinterpret_cast<lbmk::Slot*>(shadow + tab_at);
        hipError_t r = hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(lbmk::Slot),
                                      hipMemcpyHostToDevice, P->main);
        for (int i = 0; i < 2 && r == hipSuccess; ++i)
            r = lbmk::launch_step_batched(dtab, (int)act.size(), units, i, ext, P->main);
        if (r == hipSuccess) r = hipEventRecord(ev0, P->main);
        for (int i = 0; i < trial_steps && r == hipSuccess; ++i)
            r = lbmk::launch_step_batched(dtab, (int)act.size(), units, 2 + i, ext, P->main);
        if (r == hipSuccess) r = hipEventRecord(ev1, P->main);
        if (r == hipSuccess) r = hipEventSynchronize(ev1);
        float ms = 0.0f;
        if (r == hipSuccess) r = hipEventElapsedTime(&ms, ev0, ev1);
        *ms_out = ms / trial_steps;
        return r;
    };
    // Segment heights with seg + 10 a multiple of 6, from the default
    // heuristic's 14 rows up to whole slots.  First one height for every
    // bucket, then each bucket present in turn with the others fixed.
    const int cands[] = {8, 14, 20, 26, 32, 38, 44, 56, 68, 80, 104, 128, 182, 254, 1 << 20};
    int cur[kRowBuckets] = {};
    double best = 1e300;
    if (e == hipSuccess) e = trial(cur, &best);  // the default heuristic
    int pick[kRowBuckets];
    for (int c : cands) {
        if (e != hipSuccess) break;
        for (int& t : pick) t = c;
        double ms = 0.0;
        e = trial(pick, &ms);
        if (e == hipSuccess && ms < best) {
            best = ms;
            std::copy(pick, pick + kRowBuckets, cur);
        }
    }
    for (int b = 0; b < kRowBuckets && e == hipSuccess; ++b) {
        if (!present[b]) continue;
        std::copy(cur, cur + kRowBuckets, pick);
        int keep = cur[b];
        for (int c : cands) {
            if (e != hipSuccess || c == keep) continue;
            pick[b] = c;
            double ms = 0.0;
            e = trial(pick, &ms);
            if (e == hipSuccess && ms < best) {
                best = ms;
                cur[b] = c;
            }
        }
    }
    // Short trials resolve differences of about a per cent: the chosen policy
    // is kept only if it also beats the default heuristic over three times
    // the steps, each timed twice.
    bool tuned = false;
    for (int b = 0; b < kRowBuckets; ++b) tuned = tuned || cur[b] != 0;
    if (tuned && e == hipSuccess) {
        const int zero[kRowBuckets] = {};
        trial_steps = 3 * steps_per_trial;
        double tc = 0.0, td = 0.0, ms = 0.0;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
            e = trial(cur, &ms);
            tc += ms;
            if (e == hipSuccess) e = trial(zero, &ms);
            td += ms;
        }
        if (e == hipSuccess) {
            if (td <= tc) std::copy(zero, zero + kRowBuckets, cur);
            best = 0.5 * std::min(tc, td);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(P->main);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    (void)hipFree(shadow);
    if (e != hipSuccess) return fail(LBM_EDEVICE, "pool autotune: %s", hipGetErrorString(e));
    P->seg_cap = 0;
    std::copy(cur, cur + kRowBuckets, P->seg_target);
    for (SlotState& s : P->slots)
        if (s.used) lbmhost::fill_grid(s.p, s.L, seg_rows_for(P, s), s.g);
    if (best_ms) *best_ms = best;
    return LBM_OK;
}

lbm_status lbm_pool_synchronize(lbm_pool* P) {
    if (!P) return fail(LBM_EINVAL, "null pool");
    PCHK(hipSetDevice(P->dev));
    PCHK(hipStreamSynchronize(P->main));
    PCHK(hipStreamSynchronize(P->aux));
    return LBM_OK;
}

}  // extern "C"
