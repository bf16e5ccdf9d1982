// liborbit_hip: host orchestration and the C ABI declared in
// include/orbit_hip.h.  One translation unit (the kernel sources are
// included) so that every kernel is launched from the unit defining it.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>

#include "orbit_common.h"
#include "orbit_prep.hip"
#include "orbit_count.hip"
#include "orbit_combine.hip"
#include "orbit_sched.hip"
#include "../../include/orbit_hip.h"

namespace {

const int kMaxPhases = 24;
// auto: wave groups when the maps are at most this big and the out-degrees
// (bounded by the degeneracy) this small, i.e. when every source is light
const u32 kWaveGroupMaxMap = 4096;
const u32 kWaveGroupMaxOut = 64;
const u64 kMaxDynLds = 156 << 10;  // dynamic LDS per workgroup (160 KB per workgroup on gfx950)
// Per-source maps go to LDS (wave groups) when a workgroup's four slices and
// the kernel's other dynamic LDS fit in this many bytes: two workgroups per
// compute unit still fit in its 160 KB.
#ifndef LDS_MAP_BUDGET
#define LDS_MAP_BUDGET (76u << 10)
#endif
const u64 kLdsMapBudget = LDS_MAP_BUDGET;
// batches whose graphs have at most this many vertices peel in LDS (16
// bytes per vertex and workgroup)
#ifndef PEEL_LDS_MAX
#define PEEL_LDS_MAX 4096
#endif
const u32 kPeelLdsMax = PEEL_LDS_MAX;
const u32 kRelabelSortWg = 64;     // workgroups sorting the long rows of a relabelled CSR
thread_local float g_phase_ms[kMaxPhases];
thread_local const char *g_phase_name[kMaxPhases];
thread_local int g_nphase = 0;
thread_local u64 g_stats[7];

struct Buf {
    u64 off = 0, bytes = 0;
};

// Workspace layout.  Phase-1 buffers depend only on (n, m); phase-2
// buffers also on the triangle count, the degeneracy and the number of
// persistent workgroups.
struct Layout {
    // phase 1
    Buf state, deg, src, rev, rnd, pdeg, front, key, outdeg, outptr, outnbr, outslot, tcnt,
        triptr, bsum, gbase;
    // relabelling (ORB_RELABEL)
    Buf rl_rp, rl_ci, rl_order, rl_newid, rl_bin, rl_ndeg, rl_hist, rl_rp64, rl_queue, rl_bitmaps;
    u64 p1_end = 0;
    // phase 2
    Buf tri_c, tri_sab, tri_sac, tri_sbc, T, Tin, Tmid, tllen, tlptr, tlcur, tl, E7, E9, C4e,
        K4e, Q, K4t, Tv, N1, C4v, K4v, ni, vacc, cacc, feat, pred, sbin, shist, order, scratch;
    // k_max = 5: scratch of the 5-cycle kernel and of the second clique pass,
    // apart from the pair sweep's so that the three orbit groups can overlap
    Buf scratch_c5, scratch_clq;
    u64 total = 0;
    u64 stride = 0, stride_c5 = 0, stride_clq = 0;
    u32 nwg_c5 = 0;
    u32 nwg = 0;
    u32 per_wg = 1;  // execution groups (each with its own scratch) per workgroup
};

u64 align_up(u64 x, u64 a) { return (x + a - 1) / a * a; }

void place(u64 &cur, Buf &b, u64 bytes) {
    cur = align_up(cur, 256);
    b.off = cur;
    b.bytes = bytes;
    cur += bytes;
}

u64 nblocks_scan(u64 len) { return (len + SCAN_TILE - 1) / SCAN_TILE; }

bool wants_relabel(const orb_opts *opts) { return opts && (opts->flags & ORB_RELABEL); }

void layout_phase1(Layout &L, u32 n, u64 m, bool relabel = false) {
    const u64 M2 = 2 * m;
    u64 c = 0;
    place(c, L.state, sizeof(DevState));
    place(c, L.deg, 4ull * n);
    place(c, L.src, 4ull * M2);
    place(c, L.rev, 4ull * M2);
    place(c, L.rnd, 4ull * n);
    place(c, L.pdeg, 4ull * n);
    place(c, L.front, 8ull * n);
    place(c, L.key, 8ull * n);
    place(c, L.outdeg, 4ull * (n + 1));
    place(c, L.outptr, 8ull * (n + 1));
    place(c, L.outnbr, 4ull * (m + 1));
    place(c, L.outslot, 4ull * (m + 1));
    place(c, L.tcnt, 4ull * (m + 1));
    place(c, L.triptr, 8ull * (m + 1));
    u64 maxlen = M2 + 1 > (u64)n + 1 ? M2 + 1 : (u64)n + 1;
    place(c, L.bsum, 8ull * (nblocks_scan(maxlen) + 1));
    place(c, L.gbase, 4ull * n + 4);
    if (relabel) {
        place(c, L.rl_rp, 4ull * (n + 1));
        place(c, L.rl_ci, 4ull * M2 + 4);
        place(c, L.rl_order, 4ull * n + 4);
        place(c, L.rl_newid, 4ull * n + 4);
        place(c, L.rl_bin, 4ull * n + 4);
        place(c, L.rl_ndeg, 4ull * n + 4);
        place(c, L.rl_hist, 4ull * SCHED_BINS);
        place(c, L.rl_rp64, 8ull * (n + 1));
        place(c, L.rl_queue, 4ull * n + 4);
        place(c, L.rl_bitmaps, 4ull * kRelabelSortWg * ((n + 31) / 32 + 1));
    }
    L.p1_end = c;
}

// pair sweep: (sta, e2) records (16 bytes), ext (u64), touched (u32); wave groups add the
// per-wave global wheel maps and their touched lists (u32, 4 x n each)
u64 pair_stride(u32 n, bool wave_maps) {
    return 3 * align_up(8ull * n, 256) + align_up(4ull * n, 256) +
           (wave_maps ? 2 * align_up(4ull * WAVES_PER_WG * n, 256) : 0) + 256;
}
// 5-cycles: Wm (u32), P, CI (u64), touched (u32), mark (u8), C (u32), TO, SW
// (u64), jt (u32)
u64 c5_stride(u32 n) {
    return 4 * align_up(4ull * n, 256) + 4 * align_up(8ull * n, 256) + align_up(n, 256) + 256;
}
u64 clique_stride(u32 dmax) {
    u64 W = (dmax + 63) / 64;
    return align_up(4ull * dmax, 256) + 2 * 8ull * dmax * W + 2 * 8ull * dmax + 512;
}

// mapn: size of the per-source maps -- n, or the largest graph of a batch
// (maps are then indexed by position within the source's graph).
void layout_phase2(Layout &L, u32 n, u32 mapn, u64 m, u64 ntri, u32 dmax, int k_max,
                   bool ni_in_out, u32 nwg_req, u32 per_wg) {
    const u64 M2 = 2 * m;
    u64 c = L.p1_end;
    place(c, L.tri_c, 4ull * (ntri + 1));
    place(c, L.tri_sab, 4ull * (ntri + 1));
    place(c, L.tri_sac, 4ull * (ntri + 1));
    place(c, L.tri_sbc, 4ull * (ntri + 1));
    place(c, L.T, 4ull * M2 + 4);
    place(c, L.Tin, 4ull * M2 + 4);
    place(c, L.Tmid, 4ull * M2 + 4);
    place(c, L.tllen, 4ull * M2 + 4);
    place(c, L.tlptr, 8ull * (M2 + 1));
    place(c, L.tlcur, 4ull * M2 + 4);
    place(c, L.tl, 8ull * (3 * ntri + 1));
    place(c, L.E7, 8ull * M2 + 8);
    place(c, L.E9, 8ull * M2 + 8);
    place(c, L.C4e, 8ull * M2 + 8);
    place(c, L.K4e, 8ull * M2 + 8);
    place(c, L.Q, 8ull * M2 + 8);
    place(c, L.K4t, 4ull * (ntri + 1));
    place(c, L.Tv, 8ull * n + 8);
    place(c, L.N1, 8ull * n + 8);
    place(c, L.C4v, 8ull * n + 8);
    place(c, L.K4v, 8ull * n + 8);
    place(c, L.ni, ni_in_out ? 0 : 8ull * ORB_NORB * n + 8);
    place(c, L.vacc, 64ull * n + 64);
    place(c, L.cacc, 8ull * n + 8);
    place(c, L.feat, 12ull * n + 12);
    place(c, L.pred, 4ull * n + 4);
    place(c, L.sbin, 4ull * n + 4);
    place(c, L.shist, 4ull * SCHED_BINS);
    place(c, L.order, 4ull * n + 4);
    u64 stride = 8ull * mapn + 512;  // 4-cycle maps (and the long-list sort)
    if (k_max >= 5) {
        u64 ps = pair_stride(mapn, per_wg > 1);
        if (ps > stride) stride = ps;
    }
    u64 cs = clique_stride(dmax);
    if (cs > stride) stride = cs;
    stride = align_up(stride, 256);
    u32 nwg = nwg_req ? nwg_req : 512;
    // keep the per-source scratch within 48 GiB unless asked otherwise
    const u64 cap = 48ull << 30;
    while (!nwg_req && nwg > 64 && (u64)nwg * per_wg * stride > cap) nwg /= 2;
    L.nwg = nwg;
    L.per_wg = per_wg;
    L.stride = stride;
    // the overflow bound borrows the scratch for 6 doubles per vertex
    u64 sbytes = (u64)nwg * per_wg * stride;
    if (sbytes < 48ull * n + 256) sbytes = 48ull * n + 256;
    place(c, L.scratch, sbytes);
    if (k_max >= 5) {
        // the 5-cycle kernel runs at most 256 workgroups when its maps are
        // large (measured faster on big graphs)
        L.nwg_c5 = (mapn > 65536 && nwg > 256) ? 256 : nwg;
        L.stride_c5 = align_up(c5_stride(mapn), 256);
        L.stride_clq = align_up(cs, 256);
        place(c, L.scratch_c5, (u64)L.nwg_c5 * per_wg * L.stride_c5);
        place(c, L.scratch_clq, (u64)nwg * per_wg * L.stride_clq);
    }
    L.total = align_up(c, 256);
}

template <typename T>
T *at(void *ws, const Buf &b) {
    return (T *)((char *)ws + b.off);
}

int err_to_status(u32 e) {
    if (e & ERRB_ROWPTR) return ORB_E_OUT_OF_RANGE;
    if (e & ERRB_RANGE) return ORB_E_OUT_OF_RANGE;
    if (e & ERRB_LOOP) return ORB_E_SELF_LOOP;
    if (e & ERRB_DUP) return ORB_E_DUPLICATE;
    if (e & ERRB_ORDER) return ORB_E_NOT_SORTED;
    if (e & ERRB_ASYM) return ORB_E_ASYMMETRIC;
    if (e & (ERRB_VPTR | ERRB_CROSS)) return ORB_E_BATCH;
    if (e & ERRB_INTERNAL) return ORB_E_INTERNAL;
    return ORB_OK;
}

#define HCHK(x)                                   \
    do {                                          \
        hipError_t e_ = (x);                      \
        if (e_ != hipSuccess) return ORB_E_DEVICE; \
    } while (0)

// Byte ranges (within one workgroup's scratch) that a per-source kernel
// needs to be zero when it starts; it restores them to zero itself, but the
// lists it leaves behind are not zero, so the ranges are cleared before
// every such kernel.  Mirrors the device-side carving (base is 256-aligned).
unsigned grid_for(u64 items, unsigned per_block) {
    u64 g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (unsigned)g;
}
unsigned grid_waves(u64 items) { return grid_for(items * WAVE, WG); }

struct ZeroRange {
    u64 off, len;
};
int zero_ranges(int which, u32 n, bool wave_maps, ZeroRange *r) {
    const u64 a4 = align_up(4ull * n, 256), a8 = align_up(8ull * n, 256), a1 = align_up(n, 256);
    if (which == 0) {  // 4-cycles: cnt
        r[0] = {0, a4};
        return 1;
    }
    if (which == 1) {  // pair sweep: records, ext ... then the wave maps K
        r[0] = {0, 3 * a8};
        if (!wave_maps) return 1;
        r[1] = {3 * a8 + a4, align_up(4ull * WAVES_PER_WG * n, 256)};
        return 2;
    }
    // 5-cycles: Wm, P, CI, (touched), mark, C, TO, SW, (jt)
    r[0] = {0, a4 + 2 * a8};
    r[1] = {a4 + 2 * a8 + a4, a1 + a4 + 2 * a8};
    return 2;
}

int zero_scratch(int which, u32 mapn, unsigned char *scratch, u64 stride, const Layout &L,
                 u32 nwg, hipStream_t s) {
    ZeroRange r[2];
    int k = zero_ranges(which, mapn, L.per_wg > 1, r);
    for (int i = 0; i < k; i++)
        k_zero_rows<<<grid_for(r[i].len / 8 * nwg, WG), WG, 0, s>>>(scratch + r[i].off, stride,
                                                                   r[i].len / 8, nwg);
    HCHK(hipGetLastError());
    return ORB_OK;
}



// Lanes per vertex in the per-vertex kernels, from the mean degree: small
// groups for sparse low-degree graphs, whole waves otherwise.
int group_size(u32 n, u64 m) {
    const u64 mean_deg = n ? (2 * m) / n : 0;
    return mean_deg <= 8 ? 8 : mean_deg <= 16 ? 16 : 64;
}

// Launches the statement with the per-source execution group GPT.
#define WITH_GP(wave, ...)                                  \
    do {                                                    \
        if (wave) { using GPT = GpWave; __VA_ARGS__; }      \
        else { using GPT = GpWG; __VA_ARGS__; }             \
    } while (0)

// Launches the statement with the compile-time lane-group size GG = g.
#define WITH_GROUP(g, ...)                                      \
    do {                                                        \
        switch (g) {                                            \
            case 8: { constexpr int GG = 8; __VA_ARGS__; } break;   \
            case 16: { constexpr int GG = 16; __VA_ARGS__; } break; \
            case 32: { constexpr int GG = 32; __VA_ARGS__; } break; \
            default: { constexpr int GG = 64; __VA_ARGS__; } break; \
        }                                                       \
    } while (0)

// Kernels timed on their own streams (they may overlap): the pair sweep,
// the 5-cycles, the second clique pass with its triangle terms.
const int kTimedKernels = 3;
const char *const kTimedKernelName[kTimedKernels] = {"pairs", "c5", "clique2_k4terms"};
thread_local float g_kernel_ms[kTimedKernels];
thread_local int g_kernel_used = 0;

struct Timer {
    bool on;
    hipStream_t st;
    hipEvent_t ev[kMaxPhases + 1];
    hipEvent_t kev[2 * kTimedKernels];
    const char *names[kMaxPhases];
    int k = 0;
    int kused = 0;
    Timer(bool on_, hipStream_t s) : on(on_), st(s) {
        if (on) {
            for (int i = 0; i <= kMaxPhases; i++) (void)hipEventCreate(&ev[i]);
            for (int i = 0; i < 2 * kTimedKernels; i++) (void)hipEventCreate(&kev[i]);
            (void)hipEventRecord(ev[0], st);
        }
    }
    void kbegin(int i, hipStream_t s) {
        if (on) (void)hipEventRecord(kev[2 * i], s);
    }
    void kend(int i, hipStream_t s) {
        if (!on) return;
        (void)hipEventRecord(kev[2 * i + 1], s);
        kused |= 1 << i;
    }
    void mark(const char *name) {
        if (!on || k >= kMaxPhases) return;
        names[k] = name;
        (void)hipEventRecord(ev[k + 1], st);
        k++;
    }
    void finish() {
        if (!on) return;
        (void)hipEventSynchronize(ev[k]);
        g_kernel_used = kused;
        for (int i = 0; i < kTimedKernels; i++) {
            float ms = 0;
            if (kused >> i & 1) {
                (void)hipEventSynchronize(kev[2 * i + 1]);
                (void)hipEventElapsedTime(&ms, kev[2 * i], kev[2 * i + 1]);
            }
            g_kernel_ms[i] = ms;
        }
        g_nphase = k;
        for (int i = 0; i < k; i++) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
            g_phase_ms[i] = ms;
            g_phase_name[i] = names[i];
        }
    }
    ~Timer() {
        if (!on) return;
        for (int i = 0; i <= kMaxPhases; i++) (void)hipEventDestroy(ev[i]);
        for (int i = 0; i < 2 * kTimedKernels; i++) (void)hipEventDestroy(kev[i]);
    }
};

// exclusive scan of len values (u32 or u64) into out[0..len]
template <typename T>
int scan(const T *in, u64 len, u64 *out, u64 *bsum, DevState *st, hipStream_t s) {
    u64 nb = nblocks_scan(len ? len : 1);
    k_scan_reduce<T><<<(unsigned)nb, WG, 0, s>>>(in, len, bsum);
    k_scan_blocks<<<1, WG, 0, s>>>(bsum, nb, st);
    k_scan_final<T><<<(unsigned)nb, WG, 0, s>>>(in, len, bsum, out, st);
    HCHK(hipGetLastError());
    return ORB_OK;
}

int read_state(DevState *d, DevState *h, hipStream_t s) {
    HCHK(hipMemcpyAsync(h, d, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HCHK(hipStreamSynchronize(s));
    return ORB_OK;
}

// A plan: a graph of the whole count, captured after one ordinary run that
// fixed the data-dependent choices (peel launches, triangle count,
// degeneracy, largest graph of a batch).  While capturing, nothing is read
// back to the host.
struct Plan {
    bool capture = false;
    int peel_groups = 0;
    u64 ntri = 0;
    u32 maxlevel = 0, gmax = 0;
};

// Helper streams (default priority) and events of the overlapping orbit
// groups, one set per thread and device, created on first use and kept: a
// plan captured on this thread records them as branches of its graph.
struct GroupStreams {
    hipStream_t sb = nullptr;
    hipEvent_t fork = nullptr, jb = nullptr;
};
const int kMaxGroupDevices = 64;
thread_local GroupStreams g_group_streams[kMaxGroupDevices];

int group_streams(GroupStreams **out) {
    int dev = -1;
    HCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxGroupDevices) return ORB_E_DEVICE;
    GroupStreams &g = g_group_streams[dev];
    if (!g.sb) {
        HCHK(hipStreamCreateWithFlags(&g.sb, hipStreamNonBlocking));
        HCHK(hipEventCreateWithFlags(&g.fork, hipEventDisableTiming));
        HCHK(hipEventCreateWithFlags(&g.jb, hipEventDisableTiming));
    }
    *out = &g;
    return ORB_OK;
}

// zero n64 u64 words at p (a kernel, capturable)
int zero_u64(void *p, u64 n64, hipStream_t s) {
    if (!n64) return ORB_OK;
    k_fill_u64<<<grid_for(n64, WG), WG, 0, s>>>((u64 *)p, n64, 0);
    HCHK(hipGetLastError());
    return ORB_OK;
}

// Phase 1: validation, peeling, orientation and triangle counting.  Leaves
// ntri and the degeneracy in *hs.
int orient_and_count(const u32 *rp, const u32 *ci, u32 n, u64 m, void *ws, const Layout &L,
                     hipStream_t s, DevState *hs, Timer &tm, Plan *pl);

int run_phase1(const u32 *rp, const u32 *ci, u32 n, u64 m, const u64 *vptr, u32 B, void *ws,
               const Layout &L, hipStream_t s, DevState *hs, Timer &tm, Plan *pl) {
    const bool cap = pl && pl->capture;
    const u64 M2 = 2 * m;
    DevState *st = at<DevState>(ws, L.state);
    u32 *deg = at<u32>(ws, L.deg), *src = at<u32>(ws, L.src), *rev = at<u32>(ws, L.rev);
    u32 *rnd = at<u32>(ws, L.rnd), *front = at<u32>(ws, L.front);
    int *pdeg = at<int>(ws, L.pdeg);
    u64 *key = at<u64>(ws, L.key);
    u32 *outdeg = at<u32>(ws, L.outdeg), *outnbr = at<u32>(ws, L.outnbr),
        *outslot = at<u32>(ws, L.outslot), *tcnt = at<u32>(ws, L.tcnt);
    u64 *outptr = at<u64>(ws, L.outptr), *triptr = at<u64>(ws, L.triptr),
        *bsum = at<u64>(ws, L.bsum);

    int rc = zero_u64(st, sizeof(DevState) / 8, s);
    if (rc) return rc;
    k_check_rowptr<<<grid_for(n, WG), WG, 0, s>>>(rp, n, M2, st);
    HCHK(hipGetLastError());
    if (!cap) {
        rc = read_state(st, hs, s);
        if (rc) return rc;
        if (hs->err) return err_to_status(hs->err);
    }
    u32 *gbase = nullptr;
    if (vptr) {
        gbase = at<u32>(ws, L.gbase);
        k_batch_index<<<grid_waves(B), WG, 0, s>>>(vptr, B, n, gbase, st);
        if (cap) k_plan_guard<<<1, 64, 0, s>>>(st, 0, pl->gmax);
        HCHK(hipGetLastError());
        if (!cap) {
            rc = read_state(st, hs, s);
            if (rc) return rc;
            if (hs->err) return err_to_status(hs->err);
        }
    }
    if (n) {
        k_src_deg<<<grid_waves(n), WG, 0, s>>>(rp, n, src, deg);
        k_rev<<<grid_for(M2, WG), WG, 0, s>>>(rp, ci, src, gbase, n, M2, rev, st);
        HCHK(hipGetLastError());
    }
    if (!cap) {
        rc = read_state(st, hs, s);
        if (rc) return rc;
        if (hs->err) return err_to_status(hs->err);
    }
    tm.mark("validate");
    if (n == 0) return ORB_OK;

    // peeling.  A batch of graphs that fit in LDS peels in one launch, a
    // workgroup per graph; otherwise (step, advance) pairs are launched, with
    // a check for completion every 32
    const u32 gm = cap ? pl->gmax : hs->gmax;
    if (vptr && gm <= kPeelLdsMax) {
        const u32 cap_n = gm ? gm : 1;
        const u32 nwg = B < 4096 ? (B ? B : 1) : 4096;
        k_peel_graphs<<<nwg, WG, 16ull * cap_n, s>>>(vptr, B, n, rp, ci, deg, cap_n, rnd, st);
        HCHK(hipGetLastError());
        if (pl && !cap) pl->peel_groups = 1;
        if (cap) k_plan_guard<<<1, 64, 0, s>>>(st, 1, 0);
        k_rank_key<<<grid_for(n, WG), WG, 0, s>>>(rnd, n, key);
        tm.mark("peel");
        return orient_and_count(rp, ci, n, m, ws, L, s, hs, tm, pl);
    }
    k_peel_init<<<grid_for(n, WG), WG, 0, s>>>(deg, n, pdeg, rnd, st);
    HCHK(hipGetLastError());
    const unsigned gs = grid_for((u64)n, WG);
    const int gsz = group_size(n, m);
    for (int it = 0;; it++) {
        for (int k = 0; k < 32; k++) {
            WITH_GROUP(gsz, k_peel_step<GG><<<gs, WG, 0, s>>>(rp, ci, n, pdeg, rnd, front, st));
            k_peel_advance<<<1, 64, 0, s>>>(st);
        }
        HCHK(hipGetLastError());
        if (cap) {
            if (it + 1 >= pl->peel_groups) break;
            continue;
        }
        rc = read_state(st, hs, s);
        if (rc) return rc;
        if (hs->alive == 0) {
            if (pl) pl->peel_groups = it + 1;
            break;
        }
        if (it > (int)(4u * (u64)n / 32u + 1000000)) return ORB_E_INTERNAL;
    }
    if (cap) k_plan_guard<<<1, 64, 0, s>>>(st, 1, 0);
    k_rank_key<<<grid_for(n, WG), WG, 0, s>>>(rnd, n, key);
    tm.mark("peel");
    return orient_and_count(rp, ci, n, m, ws, L, s, hs, tm, pl);
}

// Orientation by the rank keys, out-lists, and the triangle count.
int orient_and_count(const u32 *rp, const u32 *ci, u32 n, u64 m, void *ws, const Layout &L,
                     hipStream_t s, DevState *hs, Timer &tm, Plan *pl) {
    const bool cap = pl && pl->capture;
    DevState *st = at<DevState>(ws, L.state);
    u32 *src = at<u32>(ws, L.src);
    u64 *key = at<u64>(ws, L.key);
    u32 *outdeg = at<u32>(ws, L.outdeg), *outnbr = at<u32>(ws, L.outnbr),
        *outslot = at<u32>(ws, L.outslot), *tcnt = at<u32>(ws, L.tcnt);
    u64 *outptr = at<u64>(ws, L.outptr), *triptr = at<u64>(ws, L.triptr),
        *bsum = at<u64>(ws, L.bsum);
    int rc = ORB_OK;
    k_outdeg<<<grid_waves(n), WG, 0, s>>>(rp, ci, key, n, outdeg);
    rc = scan<u32>(outdeg, n, outptr, bsum, st, s);
    if (rc) return rc;
    k_outfill<<<grid_waves(n), WG, 0, s>>>(rp, ci, key, n, outptr, outnbr, outslot);
    if (m) {
        k_tri_count<<<grid_for(m, WG), WG, 0, s>>>(src, outptr, outnbr, outslot, m, tcnt);
        rc = scan<u32>(tcnt, m, triptr, bsum, st, s);
        if (rc) return rc;
        k_save_ntri<<<1, 64, 0, s>>>(st);
        if (cap) k_plan_guard<<<1, 64, 0, s>>>(st, 2, pl->ntri);
    }
    HCHK(hipGetLastError());
    if (cap) {
        hs->ntri = pl->ntri;
        hs->maxlevel = pl->maxlevel;
        hs->gmax = pl->gmax;
    } else {
        rc = read_state(st, hs, s);
        if (rc) return rc;
        hs->ntri = m ? hs->scan_total : 0;
        if (pl) {
            pl->ntri = hs->ntri;
            pl->maxlevel = hs->maxlevel;
            pl->gmax = hs->gmax;
        }
    }
    tm.mark("orient");
    return ORB_OK;
}

// ORB_RELABEL: validate the caller's CSR (the checks of phase 1), then build
// the relabelled CSR (heaviest degree class first, rows sorted) in the
// workspace; phase 1 validates that one again.
int relabel_input(const u32 *rp, const u32 *ci, u32 n, u64 m, void *ws, const Layout &L,
                  hipStream_t s, DevState *hs, bool cap, const u32 **nrp_out,
                  const u32 **nci_out) {
    const u64 M2 = 2 * m;
    DevState *st = at<DevState>(ws, L.state);
    u32 *deg = at<u32>(ws, L.deg), *src = at<u32>(ws, L.src), *rev = at<u32>(ws, L.rev);
    u64 *bsum = at<u64>(ws, L.bsum);
    int rc = zero_u64(st, sizeof(DevState) / 8, s);
    if (rc) return rc;
    k_check_rowptr<<<grid_for(n, WG), WG, 0, s>>>(rp, n, M2, st);
    HCHK(hipGetLastError());
    if (!cap) {
        rc = read_state(st, hs, s);
        if (rc) return rc;
        if (hs->err) return err_to_status(hs->err);
    }
    k_src_deg<<<grid_waves(n), WG, 0, s>>>(rp, n, src, deg);
    k_rev<<<grid_for(M2, WG), WG, 0, s>>>(rp, ci, src, nullptr, n, M2, rev, st);
    HCHK(hipGetLastError());
    if (!cap) {
        rc = read_state(st, hs, s);
        if (rc) return rc;
        if (hs->err) return err_to_status(hs->err);
    }
    u32 *nrp = at<u32>(ws, L.rl_rp), *nci = at<u32>(ws, L.rl_ci);
    u32 *order = at<u32>(ws, L.rl_order), *newid = at<u32>(ws, L.rl_newid);
    u32 *bin = at<u32>(ws, L.rl_bin), *ndeg = at<u32>(ws, L.rl_ndeg);
    u32 *hist = at<u32>(ws, L.rl_hist), *queue = at<u32>(ws, L.rl_queue);
    u64 *nrp64 = at<u64>(ws, L.rl_rp64);
    rc = zero_u64(hist, SCHED_BINS / 2, s);
    if (rc) return rc;
    k_deg_bins<<<grid_for(n, WG), WG, 0, s>>>(deg, n, bin, hist);
    k_sched_offsets<<<1, 64, 0, s>>>(hist);
    k_sched_scatter<<<grid_for(n, WG), WG, 0, s>>>(bin, n, hist, order);
    k_relabel_index<<<grid_for(n, WG), WG, 0, s>>>(order, deg, n, newid, ndeg);
    HCHK(hipGetLastError());
    rc = scan<u32>(ndeg, n, nrp64, bsum, st, s);
    if (rc) return rc;
    k_relabel_fill<<<grid_waves(n), WG, 0, s>>>(rp, ci, order, newid, nrp64, n, nrp, nci);
    u32 *qlen = st->work + 14;
    k_row_sort_small<<<grid_waves(n), WG, 0, s>>>(nrp, n, nci, queue, qlen);
    k_row_sort_wg<<<kRelabelSortWg, WG, 0, s>>>(nrp, nci, queue, qlen, at<u32>(ws, L.rl_bitmaps), n);
    HCHK(hipGetLastError());
    *nrp_out = nrp;
    *nci_out = nci;
    return ORB_OK;
}

int count_impl(const u32 *rp, const u32 *ci, u32 n, u64 m, const u64 *vptr, u32 B, int k_max,
               u64 *counts, unsigned char *ovf, u64 *edge_out, void *ws,
               u64 ws_bytes, u64 *ws_required, hipStream_t s, const orb_opts *opts,
               bool query_only, Plan *pl = nullptr, u32 *nwg_fit = nullptr) {
    const u32 flags = opts ? opts->flags : 0u;
    const int K = orbit_num_orbits(k_max);
    if (!K) return ORB_E_INVALID_ARG;
    if (flags & ~(ORB_NONINDUCED | ORB_TIMING | ORB_RELABEL | ORB_SERIAL_GROUPS | ORB_ASYNC))
        return ORB_E_INVALID_ARG;
    Plan async_plan;
    if (flags & ORB_ASYNC) {  // the sizes of orbit_prepare; no host read back
        if (pl || query_only || !opts->sizes || (flags & ORB_TIMING)) return ORB_E_INVALID_ARG;
        async_plan.capture = true;
        async_plan.peel_groups = (int)opts->sizes->peel_groups;
        async_plan.ntri = opts->sizes->ntri;
        async_plan.maxlevel = opts->sizes->maxlevel;
        async_plan.gmax = opts->sizes->gmax;
        if (async_plan.peel_groups < 1 && n) return ORB_E_INVALID_ARG;
        pl = &async_plan;
    }
    const bool cap = pl && pl->capture;  // nothing is read back to the host
    const bool relabel = (flags & ORB_RELABEL) != 0;
    if (relabel && (vptr || opts->features_out || opts->steps_out)) return ORB_E_INVALID_ARG;
    if (edge_out && (relabel || vptr || k_max < 4)) return ORB_E_INVALID_ARG;
    const u32 sched = opts ? opts->schedule : ORB_SCHED_ID;
    if (sched > ORB_SCHED_MLP || (opts && opts->groups > ORB_GROUPS_WAVE))
        return ORB_E_INVALID_ARG;
    if (sched == ORB_SCHED_MLP && !opts->mlp_weights) return ORB_E_INVALID_ARG;
    if (2 * m >= (1ull << 32)) return ORB_E_INVALID_ARG;
    if (!rp || (m && !ci) || (!counts && !query_only && n)) return ORB_E_INVALID_ARG;
    Layout L;
    layout_phase1(L, n, m, relabel);
    if (ws_bytes < L.p1_end || !ws) {
        if (ws_required) *ws_required = L.p1_end;
        return ORB_E_WORKSPACE;
    }
    Timer tm((flags & ORB_TIMING) && !query_only && !cap, s);
    DevState hs;
    memset(&hs, 0, sizeof hs);
    const u32 *orig = nullptr;  // relabelled vertex -> caller's vertex
    const u32 *rp_in = rp, *ci_in = ci;  // the caller's graph
    if (relabel && n) {
        const u32 *nrp = nullptr, *nci = nullptr;
        int rc0 = relabel_input(rp, ci, n, m, ws, L, s, &hs, cap, &nrp, &nci);
        if (rc0) return rc0;
        rp = nrp;
        ci = nci;
        orig = at<u32>(ws, L.rl_order);
        tm.mark("relabel");
    }
    int rc = run_phase1(rp, ci, n, m, vptr, B, ws, L, s, &hs, tm, pl);
    if (rc) return rc;
    const u64 ntri = hs.ntri;
    const u32 dmax = hs.maxlevel + 1;
    const bool ni_in_out = (K == ORB_NORB) && !relabel;
    const u32 mapn = vptr ? (hs.gmax ? hs.gmax : 1) : n;
    // per-source execution groups: a wave per source for small maps (many
    // light sources), the whole workgroup per source otherwise
    const u32 greq = opts ? opts->groups : ORB_GROUPS_AUTO;
    const bool wave_groups =
        greq == ORB_GROUPS_WAVE ||
        (greq == ORB_GROUPS_AUTO && mapn <= kWaveGroupMaxMap && dmax <= kWaveGroupMaxOut);
    layout_phase2(L, n, mapn, m, ntri, dmax, k_max, ni_in_out, opts ? opts->num_wg : 0,
                  wave_groups ? WAVES_PER_WG : 1);
    if (nwg_fit) {  // fewer persistent workgroups until the workspace fits ws_bytes
        u32 w = L.nwg;
        while (L.total > ws_bytes && w > 1) {
            w /= 2;
            layout_phase2(L, n, mapn, m, ntri, dmax, k_max, ni_in_out, w,
                          wave_groups ? WAVES_PER_WG : 1);
        }
        *nwg_fit = L.nwg;
    }
    if (ws_required) *ws_required = L.total;
    if (query_only) return ORB_OK;
    if (L.total > ws_bytes) return ORB_E_WORKSPACE;
    if (n == 0) return ORB_OK;

    const u64 M2 = 2 * m;
    DevState *st = at<DevState>(ws, L.state);
    u32 *deg = at<u32>(ws, L.deg), *src = at<u32>(ws, L.src), *rev = at<u32>(ws, L.rev);
    u64 *key = at<u64>(ws, L.key);
    u32 *outnbr = at<u32>(ws, L.outnbr), *outslot = at<u32>(ws, L.outslot);
    u64 *outptr = at<u64>(ws, L.outptr), *triptr = at<u64>(ws, L.triptr),
        *bsum = at<u64>(ws, L.bsum);
    u32 *tri_c = at<u32>(ws, L.tri_c), *tri_sab = at<u32>(ws, L.tri_sab),
        *tri_sac = at<u32>(ws, L.tri_sac), *tri_sbc = at<u32>(ws, L.tri_sbc);
    u32 *T = at<u32>(ws, L.T), *Tin = at<u32>(ws, L.Tin), *Tmid = at<u32>(ws, L.Tmid),
        *tllen = at<u32>(ws, L.tllen), *tlcur = at<u32>(ws, L.tlcur);
    u64 *tlptr = at<u64>(ws, L.tlptr);
    uint2 *tl = at<uint2>(ws, L.tl);
    u64 *E7 = at<u64>(ws, L.E7), *E9 = at<u64>(ws, L.E9), *C4e = at<u64>(ws, L.C4e),
        *K4e = at<u64>(ws, L.K4e), *Q = at<u64>(ws, L.Q);
    u32 *K4t = at<u32>(ws, L.K4t);
    u64 *Tv = at<u64>(ws, L.Tv), *N1 = at<u64>(ws, L.N1), *C4v = at<u64>(ws, L.C4v),
        *K4v = at<u64>(ws, L.K4v);
    u64 *ni = ni_in_out ? counts : at<u64>(ws, L.ni);
    u64 *vacc = at<u64>(ws, L.vacc), *cacc = at<u64>(ws, L.cacc);
    unsigned char *scratch = at<unsigned char>(ws, L.scratch);
    const u32 *gbase = vptr ? at<u32>(ws, L.gbase) : nullptr;
    // LDS capacities: clique bit rows up to the largest out-degree, wheel
    // maps up to the largest map; the 5-cycle kernel runs at most 256
    // workgroups when its maps are large (measured faster on big graphs)
    // (out-degrees above the LDS capacity use bit rows in global scratch;
    // the capacity keeps every group's rows of a workgroup within 64 KB)
    u32 clq_d = dmax < CLQ_LDS_D ? dmax : CLQ_LDS_D;
    while (clq_d > 1 && 8ull * L.per_wg * clique_lds_words(clq_d) > kMaxDynLds) clq_d--;
    const size_t clq_lds = 8ull * L.per_wg * clique_lds_words(clq_d);
    const u32 pair_kl = ((mapn < PAIR_KMAP_LDS ? mapn : PAIR_KMAP_LDS) + 1) & ~1u;
    const size_t pair_lds = (size_t)WAVES_PER_WG * pair_kl * 6;
    const u32 c5_wg = L.nwg_c5;
    const u32 grp = L.nwg * L.per_wg, grp5 = c5_wg * L.per_wg;  // scratch rows in use
    // per-source maps in LDS (small maps, wave groups).  The 5-cycle kernel
    // keeps its maps in HBM: with them in LDS (49 bytes per vertex and
    // wave) it ran slower on the 100k-graph batch, two workgroups per
    // compute unit being too few for its chains of dependent loads.
    const u64 c4_lmw = c4_lds_words(mapn), pair_lmw = pair_lds_words(mapn);
    const u64 slices = 8ull * WAVES_PER_WG;
    const bool lm_c4 = wave_groups && slices * c4_lmw <= kLdsMapBudget;
    const bool lm_pairs = wave_groups && mapn <= pair_kl &&
                          pair_lds + slices * pair_lmw <= kLdsMapBudget;

    // zero the accumulators (the contiguous phase-2 region up to ni) and
    // the per-source scratch
    rc = zero_u64((char *)ws + L.T.off, (L.scratch.off - L.T.off) / 8, s);
    if (rc) return rc;
    rc = zero_u64(ni, (u64)ORB_NORB * n, s);
    if (rc) return rc;
    tm.mark("zero");
    if (ovf) {  // overflow flags on the caller's graph (scratch is free until the list sorts)
        double *oa = (double *)scratch, *ob = oa + 3ull * n;
        const int g = group_size(n, m);
        for (int pass = 0; pass < 3; pass++)
            WITH_GROUP(g, k_ovf<GG><<<grid_for((u64)n * GG, WG), WG, 0, s>>>(rp_in, ci_in, n, pass,
                                                                           oa, ob, ovf));
        HCHK(hipGetLastError());
        tm.mark("overflow");
    }

    // schedule of the per-source kernels
    float *feat = (opts && opts->features_out) ? opts->features_out : at<float>(ws, L.feat);
    const u32 *order = nullptr;
    if ((opts && opts->features_out) || sched != ORB_SCHED_ID) {
        k_features<<<grid_waves(n), WG, 0, s>>>(deg, outptr, outnbr, n, feat);
        HCHK(hipGetLastError());
    }
    if (sched != ORB_SCHED_ID) {
        float *pred = nullptr;
        if (sched == ORB_SCHED_MLP) {
            pred = at<float>(ws, L.pred);
            k_mlp_predict<<<grid_for(n, WG), WG, 0, s>>>(opts->mlp_weights, feat, n, pred);
        }
        u32 *sbin = at<u32>(ws, L.sbin), *shist = at<u32>(ws, L.shist);
        u32 *ord = at<u32>(ws, L.order);
        rc = zero_u64(shist, SCHED_BINS / 2, s);
        if (rc) return rc;
        k_sched_bins<<<grid_for(n, WG), WG, 0, s>>>(feat, pred, n, sbin, shist);
        k_sched_offsets<<<1, 64, 0, s>>>(shist);
        k_sched_scatter<<<grid_for(n, WG), WG, 0, s>>>(sbin, n, shist, ord);
        HCHK(hipGetLastError());
        order = ord;
    }
    u64 *steps_out = opts ? (u64 *)opts->steps_out : nullptr;
    if (steps_out) {
        rc = zero_u64(steps_out, n, s);
        if (rc) return rc;
    }
    tm.mark("schedule");

    if (ntri) {
        k_tri_fill<<<grid_for(m, WG), WG, 0, s>>>(src, outptr, outnbr, outslot, m, triptr, tri_c,
                                                  tri_sab, tri_sac, tri_sbc, st);
        k_tri_slots<<<grid_for(ntri, WG), WG, 0, s>>>(rev, ntri, tri_sab, tri_sac, tri_sbc, T, Tin,
                                                      Tmid, st);
        HCHK(hipGetLastError());
    }
    tm.mark("triangles");
    if (ntri && k_max >= 4) {
        k_tl_len<<<grid_for(M2, WG), WG, 0, s>>>(src, ci, T, M2, tllen);
        int rc2 = scan<u32>(tllen, M2, tlptr, bsum, st, s);
        if (rc2) return rc2;
        k_tl_fill<<<grid_for(ntri, WG), WG, 0, s>>>(src, ci, rev, ntri, tri_sab, tri_sac, tri_sbc,
                                                    tlptr, tlcur, tl, st);
        k_edge_e7e9<<<grid_for(M2, WG), WG, 0, s>>>(src, ci, rev, deg, T, tlptr, tl, M2, E7, E9, st);
        HCHK(hipGetLastError());
        if (k_max >= 5) {
            // lists sorted by third vertex for the pair sweep; the queue of
            // long lists reuses the (now free) list-length array, and the
            // long-list sort uses the per-source scratch before it is zeroed
            u32 *qlen = st->work + 15;
            k_tl_sort_small<<<grid_waves(M2), WG, 0, s>>>(src, ci, T, tlptr, tl, M2, tllen, qlen);
            k_tl_sort_wg<<<L.nwg, WG, 0, s>>>(rp, src, ci, T, tlptr, tl, tllen, qlen, scratch,
                                              L.stride, mapn, st);
            HCHK(hipGetLastError());
        }
    }
    tm.mark("tri_lists");
    const int gsz = group_size(n, m);
    WITH_GROUP(gsz, k_vert0<GG><<<grid_for((u64)n * GG, WG), WG, 0, s>>>(rp, ci, deg, T, n, Tv,
                                                                        N1));
    HCHK(hipGetLastError());
    u32 *work = st->work;
    int wi = 0;
    if (k_max >= 4) {
        if (!lm_c4) {
            rc = zero_scratch(0, mapn, scratch, L.stride, L, grp, s);
            if (rc) return rc;
        }
        tm.mark("zero_c4");
        if (lm_c4)
            k_c4<GpWave, true><<<L.nwg, WG, slices * c4_lmw, s>>>(
                rp, ci, rev, key, n, scratch, L.stride, work + wi++, order, mapn, gbase, c4_lmw,
                C4v, C4e, st);
        else
            WITH_GP(wave_groups, k_c4<GPT, false><<<L.nwg, WG, 0, s>>>(
                                     rp, ci, rev, key, n, scratch, L.stride, work + wi++, order,
                                     mapn, gbase, 0, C4v, C4e, st));
        HCHK(hipGetLastError());
        tm.mark("c4");
        if (ntri) {
            WITH_GP(wave_groups, k_clique<GPT><<<L.nwg, WG, clq_lds, s>>>(1, n, rev, outptr, outnbr, outslot, triptr, tri_c,
                                          tri_sbc, scratch, L.stride, dmax, clq_d, work + wi++, order, K4t, K4v, K4e,
                                          ni, st));
            HCHK(hipGetLastError());
        }
        tm.mark("cliques");
        if (ntri) {
            WITH_GROUP(gsz, k_trisweep<GG><<<grid_for((u64)n * GG, WG), WG, 0, s>>>(
                                rp, ci, rev, deg, T, tlptr, tl, Tv, N1, E7, E9, C4e, K4e, n,
                                ni));
            HCHK(hipGetLastError());
        }
        tm.mark("trisweep");
        if (edge_out) {
            k_edge_orbits<<<grid_for(M2, WAVE), WAVE, 0, s>>>(src, ci, deg, T, Tv, N1, C4e, E7, E9,
                                                            K4e, M2, edge_out);
            HCHK(hipGetLastError());
            tm.mark("edge_orbits");
        }
    }
    if (k_max >= 5) {
        // From here the three orbit groups of the 5-vertex patterns read only
        // finished data and write disjoint accumulators: the pair sweep
        // (wedges and diamonds), the 5-cycles, and the second clique pass with
        // its triangle terms.  Each has its own scratch; unless
        // ORB_SERIAL_GROUPS, the last two run one after the other on a helper
        // stream forked from and joined back into `s` by events, beside the
        // pair sweep.  (On two helper streams, all three at once, the counts
        // measured about 1 % slower.)
        const bool conc = !(flags & ORB_SERIAL_GROUPS);
        hipStream_t sb = s, sc = s;
        GroupStreams *gs = nullptr;
        unsigned char *scr_c5 = at<unsigned char>(ws, L.scratch_c5);
        unsigned char *scr_clq = at<unsigned char>(ws, L.scratch_clq);
        if (conc) {
            rc = group_streams(&gs);
            if (rc) return rc;
            sb = sc = gs->sb;
            HCHK(hipEventRecord(gs->fork, s));
            HCHK(hipStreamWaitEvent(sb, gs->fork, 0));
        }
        tm.kbegin(2, sc);
        if (ntri) {
            WITH_GP(wave_groups, k_clique<GPT><<<L.nwg, WG, clq_lds, sc>>>(2, n, rev, outptr, outnbr, outslot, triptr, tri_c,
                                          tri_sbc, scr_clq, L.stride_clq, dmax, clq_d, work + wi++, order, K4t, K4v, K4e,
                                          ni, st));
            k_tri_k4terms<<<grid_for(ntri, WG), WG, 0, sc>>>(src, ci, T, ntri, tri_c, tri_sab,
                                                             tri_sac, tri_sbc, K4t, ni, st);
            HCHK(hipGetLastError());
        }
        tm.kend(2, sc);
        if (!conc) tm.mark("clique2_k4terms");
        if (!lm_pairs) {
            rc = zero_scratch(1, mapn, scratch, L.stride, L, grp, s);
            if (rc) return rc;
        }
        if (!conc) tm.mark("zero_pairs");
        tm.kbegin(0, s);
        u64 *pcyc = opts ? (u64 *)opts->pass_cycles_out : nullptr;
        if (lm_pairs)
            k_pairs<GpWave, true><<<L.nwg, WG, pair_lds + slices * pair_lmw, s>>>(
                rp, ci, src, rev, deg, T, tlptr, tl, n, scratch, L.stride, work + wi++, order,
                mapn, gbase, pair_kl, pair_lmw, steps_out, pcyc, Q, vacc, st);
        else
            WITH_GP(wave_groups, k_pairs<GPT, false><<<L.nwg, WG, pair_lds, s>>>(
                                     rp, ci, src, rev, deg, T, tlptr, tl, n, scratch, L.stride,
                                     work + wi++, order, mapn, gbase, pair_kl, 0, steps_out,
                                     pcyc, Q, vacc, st));
        HCHK(hipGetLastError());
        tm.kend(0, s);
        if (!conc) tm.mark("pairs");
        rc = zero_scratch(2, mapn, scr_c5, L.stride_c5, L, grp5, sb);
        if (rc) return rc;
        if (!conc) tm.mark("zero_c5");
        tm.kbegin(1, sb);
        WITH_GP(wave_groups, k_c5<GPT><<<c5_wg, WG, 0, sb>>>(rp, ci, key, outptr, outnbr, outslot, T, Tin, Tmid, n, scr_c5,
                                  L.stride_c5, work + wi++, order, mapn, gbase, steps_out, cacc, st));
        HCHK(hipGetLastError());
        tm.kend(1, sb);
        if (conc) {
            HCHK(hipEventRecord(gs->jb, sb));
            HCHK(hipStreamWaitEvent(s, gs->jb, 0));
            tm.mark("groups");
        } else {
            tm.mark("c5");
        }
    }
    WITH_GROUP(gsz, k_vert1<GG><<<grid_for((u64)n * GG, WG), WG, 0, s>>>(
                        rp, ci, rev, deg, T, Tv, N1, C4v, K4v, C4e, K4e, E9, Q, vacc, cacc, n, ni));
    if (k_max >= 5)
        WITH_GROUP(gsz, k_vert2<GG><<<grid_for((u64)n * GG, WG), WG, 0, s>>>(rp, ci, deg, Tv, N1,
                                                                            n, ni));
    k_transform<<<grid_for(n, XF_ROWS), WAVE, 0, s>>>(ni, n, K, (flags & ORB_NONINDUCED) ? 0 : 1,
                                                     orig, counts);
    HCHK(hipGetLastError());
    tm.mark("combine");
    if (flags & ORB_TIMING) {
        k_stats<<<grid_for(M2 > n ? M2 : n, WG), WG, 0, s>>>(src, ci, deg, T, outptr, outnbr, n,
                                                             M2, st);
        HCHK(hipGetLastError());
    }
    if (cap) {  // the replay checks that it saw the sizes it was built for
        k_plan_check<<<1, 64, 0, s>>>(st, pl->ntri, pl->maxlevel, pl->gmax);
        HCHK(hipGetLastError());
        return ORB_OK;
    }
    rc = read_state(st, &hs, s);
    if (rc) return rc;
    tm.finish();
    if (flags & ORB_TIMING) {
        g_stats[0] = n; g_stats[1] = m; g_stats[2] = ntri; g_stats[3] = hs.maxlevel;
        g_stats[4] = hs.wedges; g_stats[5] = hs.diamonds; g_stats[6] = hs.paths3;
    }
    if (hs.err) return err_to_status(hs.err);
    return ORB_OK;
}

// ---- the entry point that allocates nothing: its workspace is a static
// device array.  Each GPU the library runs on holds its own copy for the
// life of the process.  In host code the array's name stands for a host-side
// stand-in, so the device address of the current GPU's copy is looked up
// once per device (hipGetSymbolAddress, with that device current) and only
// that address is ever handed to kernels.
#ifndef ORB_NOALLOC_BYTES
#define ORB_NOALLOC_BYTES (64ull << 20)
#endif
static __device__ __align__(256) unsigned char scratch[ORB_NOALLOC_BYTES];
const int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;

int scratch_of_current_device(void **out) {
    int dev = -1;
    HCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return ORB_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ORB_E_DEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return ORB_OK;
}

}  // namespace

extern "C" {

int orbit_num_orbits(int k_max) {
    switch (k_max) {
        case 3: return 4;
        case 4: return 15;
        case 5: return ORB_NORB;
        default: return 0;
    }
}

int orbit_count_ex(const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n, uint64_t m,
                   int k_max, uint64_t *counts, uint8_t *overflow_flags, void *workspace,
                   uint64_t ws_bytes, uint64_t *ws_required, void *stream,
                   const orb_opts *opts) {
    return count_impl(row_ptr, col_idx, n, m, nullptr, 0, k_max, (u64 *)counts, overflow_flags,
                      nullptr, workspace, ws_bytes, (u64 *)ws_required, (hipStream_t)stream, opts, false);
}

int orbit_prepare(const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n, uint64_t m,
                  int k_max, void *stream, const orb_opts *opts, uint64_t *bytes,
                  orb_sizes *sizes) {
    if (!bytes || !sizes || !orbit_num_orbits(k_max)) return ORB_E_INVALID_ARG;
    if (2 * m >= (1ull << 32)) return ORB_E_INVALID_ARG;
    if (opts && (opts->flags & ORB_ASYNC)) return ORB_E_INVALID_ARG;
    Layout L;
    layout_phase1(L, n, m, wants_relabel(opts));
    void *tmp = nullptr;
    if (hipMalloc(&tmp, L.p1_end) != hipSuccess) return ORB_E_DEVICE;
    u64 req = 0;
    Plan pl;
    int rc = count_impl(row_ptr, col_idx, n, m, nullptr, 0, k_max, nullptr, nullptr, nullptr, tmp,
                        L.p1_end, &req, (hipStream_t)stream, opts, true, &pl);
    (void)hipFree(tmp);
    if (rc) return rc;
    *bytes = req;
    sizes->ntri = pl.ntri;
    sizes->peel_groups = (uint32_t)pl.peel_groups;
    sizes->maxlevel = pl.maxlevel;
    sizes->gmax = pl.gmax;
    sizes->reserved = 0;
    return ORB_OK;
}

int orbit_count_status(const void *workspace, void *stream) {
    if (!workspace) return ORB_E_INVALID_ARG;
    DevState h;
    int rc = read_state((DevState *)workspace, &h, (hipStream_t)stream);
    if (rc) return rc;
    return h.err ? err_to_status(h.err) : ORB_OK;
}

int orbit_count_edges(const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n, uint64_t m,
                      int k_max, uint64_t *counts, uint64_t *edge_counts, void *workspace,
                      uint64_t ws_bytes, uint64_t *ws_required, void *stream,
                      const orb_opts *opts) {
    if (!edge_counts || k_max < 4) return ORB_E_INVALID_ARG;
    return count_impl(row_ptr, col_idx, n, m, nullptr, 0, k_max, (u64 *)counts, nullptr,
                      (u64 *)edge_counts, workspace, ws_bytes, (u64 *)ws_required,
                      (hipStream_t)stream, opts, false);
}

int orbit_num_patterns(int k_max) {
    switch (k_max) {
        case 3: return 3;
        case 4: return 9;
        case 5: return ORB_NPATTERN;
        default: return 0;
    }
}

int orbit_voc_summary(const uint64_t *counts, uint32_t n, int k_max, uint64_t *orbit_sums,
                      uint64_t *pattern_counts, uint64_t *hist, void *stream) {
    const int K = orbit_num_orbits(k_max);
    if (!K || !orbit_sums || !hist || (n && !counts)) return ORB_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    int rc = zero_u64(orbit_sums, 2ull * K, s);
    if (!rc) rc = zero_u64(hist, (u64)K * VOC_BINS, s);
    if (rc) return rc;
    if (n) {
        k_voc<<<grid_for((u64)n * K, WG), WG, 0, s>>>((const u64 *)counts, n, K,
                                                     (u64 *)orbit_sums, (u64 *)hist);
        HCHK(hipGetLastError());
    }
    if (pattern_counts) {
        k_voc_patterns<<<1, 64, 0, s>>>((const u64 *)orbit_sums, K, (u64 *)pattern_counts);
        HCHK(hipGetLastError());
    }
    return ORB_OK;
}

int orbit_count_noalloc(const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n,
                        uint64_t m, int k_max, uint64_t *counts, void *stream) {
    if (!orbit_num_orbits(k_max) || 2 * m >= (1ull << 32)) return ORB_E_INVALID_ARG;
    Layout L;
    layout_phase1(L, n, m);
    if (L.p1_end > ORB_NOALLOC_BYTES) return ORB_E_TOO_LARGE;
    void *ws = nullptr;
    int rc = scratch_of_current_device(&ws);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    // size the count for the static buffer (validates the graph on the way)
    u32 nwg = 0;
    u64 need = 0;
    rc = count_impl(row_ptr, col_idx, n, m, nullptr, 0, k_max, (u64 *)counts, nullptr, nullptr, ws,
                    ORB_NOALLOC_BYTES, &need, s, nullptr, true, nullptr, &nwg);
    if (rc) return rc;
    if (need > ORB_NOALLOC_BYTES) return ORB_E_TOO_LARGE;
    orb_opts o;
    memset(&o, 0, sizeof o);
    o.num_wg = nwg;
    o.flags = ORB_SERIAL_GROUPS;  // one stream: no helper stream is created
    return count_impl(row_ptr, col_idx, n, m, nullptr, 0, k_max, (u64 *)counts, nullptr, nullptr, ws,
                      ORB_NOALLOC_BYTES, nullptr, s, &o, false);
}

uint64_t orbit_noalloc_capacity(void) { return ORB_NOALLOC_BYTES; }

int orbit_workspace_query(const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n,
                          uint64_t m, int k_max, void *stream, const orb_opts *opts,
                          uint64_t *bytes) {
    if (!bytes || !orbit_num_orbits(k_max)) return ORB_E_INVALID_ARG;
    if (2 * m >= (1ull << 32)) return ORB_E_INVALID_ARG;
    Layout L;
    layout_phase1(L, n, m, wants_relabel(opts));
    void *tmp = nullptr;
    if (hipMalloc(&tmp, L.p1_end) != hipSuccess) return ORB_E_DEVICE;
    u64 req = 0;
    int rc = count_impl(row_ptr, col_idx, n, m, nullptr, 0, k_max, nullptr, nullptr, nullptr, tmp, L.p1_end, &req,
                        (hipStream_t)stream, opts, true);
    (void)hipFree(tmp);
    if (rc) return rc;
    *bytes = req;
    return ORB_OK;
}

int orbit_count(const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n, uint64_t m,
                int k_max, uint64_t *counts) {
    uint64_t need = 0;
    int rc = orbit_workspace_query(row_ptr, col_idx, n, m, k_max, nullptr, nullptr, &need);
    if (rc) return rc;
    // a workspace beyond the device's free memory is a size limit, not a
    // failed call (R-MAT scale 24 with edge factor 32 needs more than 288 GB)
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return ORB_E_DEVICE;
    if (need > free_b) return ORB_E_TOO_LARGE;
    void *ws = nullptr;
    if (hipMalloc(&ws, need ? need : 256) != hipSuccess) return ORB_E_DEVICE;
    rc = orbit_count_ex(row_ptr, col_idx, n, m, k_max, counts, nullptr, ws, need, nullptr,
                        nullptr, nullptr);
    (void)hipFree(ws);
    return rc;
}

int orbit_count_batched(const uint64_t *vptr, uint32_t num_graphs, const uint32_t *row_ptr,
                        const uint32_t *col_idx, uint32_t n, uint64_t m, int k_max,
                        uint64_t *counts, void *workspace, uint64_t ws_bytes,
                        uint64_t *ws_required, void *stream, const orb_opts *opts) {
    if (!vptr) return ORB_E_INVALID_ARG;
    return count_impl(row_ptr, col_idx, n, m, (const u64 *)vptr, num_graphs, k_max,
                      (u64 *)counts, nullptr, nullptr, workspace, ws_bytes, (u64 *)ws_required,
                      (hipStream_t)stream, opts, false);
}

int orbit_workspace_query_batched(const uint64_t *vptr, uint32_t num_graphs,
                                  const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n,
                                  uint64_t m, int k_max, void *stream, const orb_opts *opts,
                                  uint64_t *bytes) {
    if (!bytes || !vptr || !orbit_num_orbits(k_max)) return ORB_E_INVALID_ARG;
    if (2 * m >= (1ull << 32)) return ORB_E_INVALID_ARG;
    Layout L;
    layout_phase1(L, n, m);
    void *tmp = nullptr;
    if (hipMalloc(&tmp, L.p1_end) != hipSuccess) return ORB_E_DEVICE;
    u64 req = 0;
    int rc = count_impl(row_ptr, col_idx, n, m, (const u64 *)vptr, num_graphs, k_max, nullptr,
                        nullptr, nullptr, tmp, L.p1_end, &req, (hipStream_t)stream, opts, true);
    (void)hipFree(tmp);
    if (rc) return rc;
    *bytes = req;
    return ORB_OK;
}

int orbit_autotune(const uint64_t *vptr, uint32_t num_graphs, const uint32_t *row_ptr,
                   const uint32_t *col_idx, uint32_t n, uint64_t m, int k_max, uint64_t *counts,
                   void *workspace, uint64_t ws_bytes, void *stream, const orb_opts *base,
                   const uint32_t *nwg_candidates, int num_candidates, orb_opts *best,
                   float *best_ms) {
    if (!best || !nwg_candidates || num_candidates <= 0) return ORB_E_INVALID_ARG;
    orb_opts o;
    memset(&o, 0, sizeof o);
    if (base) o = *base;
    const u32 keep_flags = o.flags & ~ORB_TIMING;
    const u32 nsched = o.mlp_weights ? 3 : 2;
    hipStream_t s = (hipStream_t)stream;
    auto run = [&](const orb_opts &x, float *ms) -> int {
        int rc = count_impl(row_ptr, col_idx, n, m, (const u64 *)vptr, num_graphs, k_max,
                            (u64 *)counts, nullptr, nullptr, workspace, ws_bytes, nullptr, s, &x, false);
        if (rc) return rc;
        float t = 0;
        for (int i = 0; i < g_nphase; i++) t += g_phase_ms[i];
        *ms = t;
        return ORB_OK;
    };
    float bms = -1, ms = 0;
    orb_opts b = o;
    bool warm = false;
    for (int c = 0; c < num_candidates; c++) {
        for (u32 gr = ORB_GROUPS_WG; gr <= ORB_GROUPS_WAVE; gr++) {
            for (u32 sc = 0; sc < nsched; sc++) {
                orb_opts x = o;
                x.flags = keep_flags | ORB_TIMING;
                x.num_wg = nwg_candidates[c];
                x.schedule = sc;
                x.groups = gr;
                int rc = run(x, &ms);
                if (rc == ORB_E_WORKSPACE) break;  // this candidate does not fit
                if (rc) return rc;
                if (!warm) {  // the first run also loads the code and warms caches
                    warm = true;
                    rc = run(x, &ms);
                    if (rc) return rc;
                }
                if (bms < 0 || ms < bms) { bms = ms; b = x; }
            }
        }
    }
    if (bms < 0) return ORB_E_WORKSPACE;
    b.flags = keep_flags;
    *best = b;
    if (best_ms) *best_ms = bms;
    return ORB_OK;
}

struct orb_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    DevState *st = nullptr;  // device state inside the plan's workspace
};

int orbit_plan_create(const uint64_t *vptr, uint32_t num_graphs, const uint32_t *row_ptr,
                      const uint32_t *col_idx, uint32_t n, uint64_t m, int k_max,
                      uint64_t *counts, void *workspace, uint64_t ws_bytes, void *stream,
                      const orb_opts *opts, orb_plan **plan) {
    if (!plan) return ORB_E_INVALID_ARG;
    *plan = nullptr;
    orb_opts o;
    memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    o.flags &= ~ORB_TIMING;
    o.features_out = nullptr;
    o.steps_out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    // 1. an ordinary run validates the input and fixes the sizes
    Plan pl;
    int rc = count_impl(row_ptr, col_idx, n, m, (const u64 *)vptr, num_graphs, k_max,
                        (u64 *)counts, nullptr, nullptr, workspace, ws_bytes, nullptr, s, &o, false, &pl);
    if (rc) return rc;
    if (n == 0) return ORB_E_INVALID_ARG;  // nothing to capture
    // 2. the same launches, captured on a private stream
    hipStream_t cs = nullptr;
    HCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return ORB_E_DEVICE;
    }
    pl.capture = true;
    rc = count_impl(row_ptr, col_idx, n, m, (const u64 *)vptr, num_graphs, k_max,
                    (u64 *)counts, nullptr, nullptr, workspace, ws_bytes, nullptr, cs, &o, false, &pl);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : ORB_E_DEVICE;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return ORB_E_DEVICE;
    }
    orb_plan *p = new (std::nothrow) orb_plan;
    if (!p) {
        (void)hipGraphExecDestroy(ex);
        (void)hipGraphDestroy(g);
        return ORB_E_DEVICE;
    }
    Layout L;
    layout_phase1(L, n, m);
    p->graph = g;
    p->exec = ex;
    p->st = at<DevState>(workspace, L.state);
    *plan = p;
    return ORB_OK;
}

int orbit_plan_launch(orb_plan *plan, void *stream) {
    if (!plan) return ORB_E_INVALID_ARG;
    return hipGraphLaunch(plan->exec, (hipStream_t)stream) == hipSuccess ? ORB_OK : ORB_E_DEVICE;
}

int orbit_plan_status(orb_plan *plan, void *stream) {
    if (!plan) return ORB_E_INVALID_ARG;
    DevState h;
    int rc = read_state(plan->st, &h, (hipStream_t)stream);
    if (rc) return rc;
    return h.err ? err_to_status(h.err) : ORB_OK;
}

int orbit_plan_destroy(orb_plan *plan) {
    if (!plan) return ORB_OK;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    delete plan;
    return ORB_OK;
}

int orbit_mlp_init(float *weights, uint32_t seed, void *stream) {
    if (!weights) return ORB_E_INVALID_ARG;
    k_mlp_init<<<(MLP_NPARAM + WG - 1) / WG, WG, 0, (hipStream_t)stream>>>(weights, seed);
    return hipGetLastError() == hipSuccess ? ORB_OK : ORB_E_DEVICE;
}

int orbit_mlp_predict(const float *weights, const float *features, uint32_t count, float *out,
                      void *stream) {
    if (!weights || (count && (!features || !out))) return ORB_E_INVALID_ARG;
    if (!count) return ORB_OK;
    k_mlp_predict<<<grid_for(count, WG), WG, 0, (hipStream_t)stream>>>(weights, features, count,
                                                                        out);
    return hipGetLastError() == hipSuccess ? ORB_OK : ORB_E_DEVICE;
}

int orbit_mlp_grad(const float *weights, const float *features, const float *targets,
                   const uint64_t *steps, uint32_t count, float *grad, float *loss,
                   void *stream) {
    if (!weights || !features || !grad || !loss || !count || (!targets && !steps))
        return ORB_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    k_zero_f32<<<(MLP_NPARAM + WG - 1) / WG, WG, 0, s>>>(grad, MLP_NPARAM);
    k_zero_f32<<<1, WG, 0, s>>>(loss, 1);
    k_mlp_grad<<<grid_for((count + MLP_TILE - 1) / MLP_TILE, 1), WG, 0, s>>>(
        weights, features, targets, (const u64 *)steps, count, count, 1, 0, 0, grad, loss);
    return hipGetLastError() == hipSuccess ? ORB_OK : ORB_E_DEVICE;
}

int orbit_mlp_train(const float *features, const uint64_t *steps, uint32_t count,
                    float *weights, float *state, uint32_t iters, uint32_t batch, float lr,
                    uint32_t seed, void *stream) {
    if (!features || !steps || !weights || !state || !count || !batch) return ORB_E_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    float *m = state, *v = state + MLP_NPARAM, *grad = state + 2 * MLP_NPARAM;
    float *loss = state + 3 * MLP_NPARAM;
    k_zero_f32<<<(2 * MLP_NPARAM + WG - 1) / WG, WG, 0, s>>>(state, 2 * MLP_NPARAM);
    const unsigned gblocks = grid_for((batch + MLP_TILE - 1) / MLP_TILE, 1);
    for (uint32_t t = 1; t <= iters; t++) {
        k_zero_f32<<<(MLP_NPARAM + 1 + WG - 1) / WG, WG, 0, s>>>(grad, MLP_NPARAM + 1);
        k_mlp_grad<<<gblocks, WG, 0, s>>>(weights, features, nullptr, (const u64 *)steps, count,
                                          batch, 0, seed, t, grad, loss);
        k_mlp_adam<<<(MLP_NPARAM + WG - 1) / WG, WG, 0, s>>>(weights, grad, m, v, t, lr);
    }
    return hipGetLastError() == hipSuccess ? ORB_OK : ORB_E_DEVICE;
}

const char *orbit_strerror(int status) {
    switch (status) {
        case ORB_OK: return "ok";
        case ORB_E_INVALID_ARG: return "invalid argument";
        case ORB_E_NOT_SORTED: return "neighbour list not sorted";
        case ORB_E_SELF_LOOP: return "self-loop in input";
        case ORB_E_DUPLICATE: return "duplicate edge in input";
        case ORB_E_ASYMMETRIC: return "CSR is not symmetric";
        case ORB_E_OUT_OF_RANGE: return "index out of range or malformed row_ptr";
        case ORB_E_WORKSPACE: return "workspace too small";
        case ORB_E_DEVICE: return "HIP call failed";
        case ORB_E_INTERNAL: return "internal consistency check failed";
        case ORB_E_BATCH: return "batched input: bad graph offsets or an edge joining two graphs";
        case ORB_E_TOO_LARGE:
            return "graph needs more device memory than there is (orbit_count_noalloc's static "
                   "buffer, or the device's free memory for orbit_count)";
        default: return "unknown status";
    }
}

int orbit_last_stats(uint64_t *vals, int max_vals) {
    int k = max_vals < 7 ? max_vals : 7;
    for (int i = 0; i < k; i++) vals[i] = g_stats[i];
    return k;
}

int orbit_last_kernel_times(float *ms, const char **names, int max_kernels) {
    int k = 0;
    for (int i = 0; i < kTimedKernels && k < max_kernels; i++) {
        if (!(g_kernel_used >> i & 1)) continue;
        if (ms) ms[k] = g_kernel_ms[i];
        if (names) names[k] = kTimedKernelName[i];
        k++;
    }
    return k;
}

int orbit_last_phase_times(float *ms, const char **names, int max_phases) {
    int k = g_nphase < max_phases ? g_nphase : max_phases;
    for (int i = 0; i < k; i++) {
        if (ms) ms[i] = g_phase_ms[i];
        if (names) names[i] = g_phase_name[i];
    }
    return k;
}

}  // extern "C"
