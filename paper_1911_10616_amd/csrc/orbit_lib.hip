// liborbit_hip: host orchestration and the C ABI declared in
// include/orbit_hip.h.  One translation unit (the kernel sources are
// included) so that every kernel is launched from the unit defining it.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "orbit_common.h"
#include "orbit_prep.hip"
#include "orbit_count.hip"
#include "orbit_combine.hip"
#include "orbit_sched.hip"
#include "../../include/orbit_hip.h"

namespace {

const int kMaxPhases = 24;
thread_local float g_phase_ms[kMaxPhases];
thread_local const char *g_phase_name[kMaxPhases];
thread_local int g_nphase = 0;
thread_local u64 g_stats[6];

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
    u64 p1_end = 0;
    // phase 2
    Buf tri_c, tri_sab, tri_sac, tri_sbc, T, Tin, Tmid, tllen, tlptr, tlcur, tl, E7, E9, C4e,
        K4e, Q, K4t, Tv, N1, C4v, K4v, ni, feat, pred, sbin, shist, order, scratch;
    u64 total = 0;
    u64 stride = 0;
    u32 nwg = 0;
};

u64 align_up(u64 x, u64 a) { return (x + a - 1) / a * a; }

void place(u64 &cur, Buf &b, u64 bytes) {
    cur = align_up(cur, 256);
    b.off = cur;
    b.bytes = bytes;
    cur += bytes;
}

u64 nblocks_scan(u64 len) { return (len + SCAN_TILE - 1) / SCAN_TILE; }

void layout_phase1(Layout &L, u32 n, u64 m) {
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
    L.p1_end = c;
}

u64 pair_stride(u32 n) {
    // S u32, E/TA/TB u64, mark u8, touched u32, 4 wave maps + lists u32
    return align_up(4ull * n, 256) + 3 * align_up(8ull * n, 256) + align_up(n, 256) +
           align_up(4ull * n, 256) + 2 * align_up(4ull * WAVES_PER_WG * n, 256) + 256;
}
u64 clique_stride(u32 dmax) {
    u64 W = (dmax + 63) / 64;
    return align_up(4ull * dmax, 256) + 2 * 8ull * dmax * W + 2 * 8ull * dmax + 512;
}

// mapn: size of the per-source maps -- n, or the largest graph of a batch
// (maps are then indexed by position within the source's graph).
void layout_phase2(Layout &L, u32 n, u32 mapn, u64 m, u64 ntri, u32 dmax, int k_max,
                   bool ni_in_out, u32 nwg_req) {
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
    place(c, L.feat, 12ull * n + 12);
    place(c, L.pred, 4ull * n + 4);
    place(c, L.sbin, 4ull * n + 4);
    place(c, L.shist, 4ull * SCHED_BINS);
    place(c, L.order, 4ull * n + 4);
    u64 stride = 8ull * mapn + 512;  // 4-cycle maps (and the long-list sort)
    if (k_max >= 5) {
        u64 ps = pair_stride(mapn);
        if (ps > stride) stride = ps;
    }
    u64 cs = clique_stride(dmax);
    if (cs > stride) stride = cs;
    stride = align_up(stride, 256);
    u32 nwg = nwg_req ? nwg_req : 512;
    // keep the per-source scratch within 48 GiB unless asked otherwise
    const u64 cap = 48ull << 30;
    while (!nwg_req && nwg > 64 && (u64)nwg * stride > cap) nwg /= 2;
    L.nwg = nwg;
    L.stride = stride;
    place(c, L.scratch, (u64)nwg * stride);
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
struct ZeroRange {
    u64 off, len;
};
int zero_ranges(int which, u32 n, ZeroRange *r) {
    const u64 a4 = align_up(4ull * n, 256), a8 = align_up(8ull * n, 256), a1 = align_up(n, 256);
    if (which == 0) {  // 4-cycles: cnt
        r[0] = {0, a4};
        return 1;
    }
    if (which == 1) {  // pair sweep: S, E, TA, TB, mark ... then the wave maps K
        u64 kof = a4 + 3 * a8 + a1 + a4;
        r[0] = {0, a4 + 3 * a8 + a1};
        r[1] = {kof, align_up(4ull * WAVES_PER_WG * n, 256)};
        return 2;
    }
    // 5-cycles: Wm, P, CI, (touched), mark
    r[0] = {0, a4 + 2 * a8};
    r[1] = {a4 + 2 * a8 + a4, a1};
    return 2;
}

int zero_scratch(int which, u32 mapn, unsigned char *scratch, const Layout &L, u32 nwg,
                 hipStream_t s) {
    ZeroRange r[2];
    int k = zero_ranges(which, mapn, r);
    for (int i = 0; i < k; i++)
        HCHK(hipMemset2DAsync(scratch + r[i].off, L.stride, 0, r[i].len, nwg, s));
    return ORB_OK;
}

unsigned grid_for(u64 items, unsigned per_block) {
    u64 g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (unsigned)g;
}
unsigned grid_waves(u64 items) { return grid_for(items * WAVE, WG); }

struct Timer {
    bool on;
    hipStream_t st;
    hipEvent_t ev[kMaxPhases + 1];
    const char *names[kMaxPhases];
    int k = 0;
    Timer(bool on_, hipStream_t s) : on(on_), st(s) {
        if (on)
            for (int i = 0; i <= kMaxPhases; i++) (void)hipEventCreate(&ev[i]);
        if (on) (void)hipEventRecord(ev[0], st);
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
        g_nphase = k;
        for (int i = 0; i < k; i++) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
            g_phase_ms[i] = ms;
            g_phase_name[i] = names[i];
        }
    }
    ~Timer() {
        if (on)
            for (int i = 0; i <= kMaxPhases; i++) (void)hipEventDestroy(ev[i]);
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

struct Host {
    DevState st;
};

int read_state(DevState *d, DevState *h, hipStream_t s) {
    HCHK(hipMemcpyAsync(h, d, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HCHK(hipStreamSynchronize(s));
    return ORB_OK;
}

// Phase 1: validation, peeling, orientation and triangle counting.  Leaves
// ntri and the degeneracy in *hs.
int run_phase1(const u32 *rp, const u32 *ci, u32 n, u64 m, const u64 *vptr, u32 B, void *ws,
               const Layout &L, hipStream_t s, DevState *hs, Timer &tm) {
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

    HCHK(hipMemsetAsync(st, 0, sizeof(DevState), s));
    k_check_rowptr<<<grid_for(n, WG), WG, 0, s>>>(rp, n, M2, st);
    HCHK(hipGetLastError());
    int rc = read_state(st, hs, s);
    if (rc) return rc;
    if (hs->err) return err_to_status(hs->err);
    u32 *gbase = nullptr;
    if (vptr) {
        gbase = at<u32>(ws, L.gbase);
        k_batch_index<<<grid_waves(B), WG, 0, s>>>(vptr, B, n, gbase, st);
        HCHK(hipGetLastError());
        rc = read_state(st, hs, s);
        if (rc) return rc;
        if (hs->err) return err_to_status(hs->err);
    }
    if (n) {
        k_src_deg<<<grid_waves(n), WG, 0, s>>>(rp, n, src, deg);
        k_rev<<<grid_for(M2, WG), WG, 0, s>>>(rp, ci, src, gbase, n, M2, rev, st);
        HCHK(hipGetLastError());
    }
    rc = read_state(st, hs, s);
    if (rc) return rc;
    if (hs->err) return err_to_status(hs->err);
    tm.mark("validate");
    if (n == 0) return ORB_OK;

    // peeling: launch (step, advance) pairs; check for completion every 32
    k_peel_init<<<grid_for(n, WG), WG, 0, s>>>(deg, n, pdeg, rnd, st);
    HCHK(hipGetLastError());
    const unsigned gs = grid_for((u64)n, WG);
    for (int it = 0;; it++) {
        for (int k = 0; k < 32; k++) {
            k_peel_step<<<gs, WG, 0, s>>>(rp, ci, n, pdeg, rnd, front, st);
            k_peel_advance<<<1, 64, 0, s>>>(st);
        }
        HCHK(hipGetLastError());
        rc = read_state(st, hs, s);
        if (rc) return rc;
        if (hs->alive == 0) break;
        if (it > (int)(4u * (u64)n / 32u + 1000000)) return ORB_E_INTERNAL;
    }
    k_rank_key<<<grid_for(n, WG), WG, 0, s>>>(rnd, n, key);
    tm.mark("peel");

    k_outdeg<<<grid_waves(n), WG, 0, s>>>(rp, ci, key, n, outdeg);
    rc = scan<u32>(outdeg, n, outptr, bsum, st, s);
    if (rc) return rc;
    k_outfill<<<grid_waves(n), WG, 0, s>>>(rp, ci, key, n, outptr, outnbr, outslot);
    if (m) {
        k_tri_count<<<grid_for(m, WG), WG, 0, s>>>(src, outptr, outnbr, outslot, m, tcnt);
        rc = scan<u32>(tcnt, m, triptr, bsum, st, s);
        if (rc) return rc;
    }
    HCHK(hipGetLastError());
    rc = read_state(st, hs, s);
    if (rc) return rc;
    hs->ntri = m ? hs->scan_total : 0;
    tm.mark("orient");
    return ORB_OK;
}

int count_impl(const u32 *rp, const u32 *ci, u32 n, u64 m, const u64 *vptr, u32 B, int k_max,
               u64 *counts, void *ws,
               u64 ws_bytes, u64 *ws_required, hipStream_t s, const orb_opts *opts,
               bool query_only) {
    const u32 flags = opts ? opts->flags : 0u;
    const int K = orbit_num_orbits(k_max);
    if (!K) return ORB_E_INVALID_ARG;
    if (flags & ~(ORB_NONINDUCED | ORB_TIMING)) return ORB_E_INVALID_ARG;
    const u32 sched = opts ? opts->schedule : ORB_SCHED_ID;
    if (sched > ORB_SCHED_MLP || (opts && opts->reserved)) return ORB_E_INVALID_ARG;
    if (sched == ORB_SCHED_MLP && !opts->mlp_weights) return ORB_E_INVALID_ARG;
    if (2 * m >= (1ull << 32)) return ORB_E_INVALID_ARG;
    if (!rp || (m && !ci) || (!counts && !query_only && n)) return ORB_E_INVALID_ARG;
    Layout L;
    layout_phase1(L, n, m);
    if (ws_bytes < L.p1_end || !ws) {
        if (ws_required) *ws_required = L.p1_end;
        return ORB_E_WORKSPACE;
    }
    Timer tm((flags & ORB_TIMING) && !query_only, s);
    DevState hs;
    memset(&hs, 0, sizeof hs);
    int rc = run_phase1(rp, ci, n, m, vptr, B, ws, L, s, &hs, tm);
    if (rc) return rc;
    const u64 ntri = hs.ntri;
    const u32 dmax = hs.maxlevel + 1;
    const bool ni_in_out = (K == ORB_NORB);
    const u32 mapn = vptr ? (hs.gmax ? hs.gmax : 1) : n;
    layout_phase2(L, n, mapn, m, ntri, dmax, k_max, ni_in_out, opts ? opts->num_wg : 0);
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
    unsigned char *scratch = at<unsigned char>(ws, L.scratch);
    const u32 *gbase = vptr ? at<u32>(ws, L.gbase) : nullptr;

    // zero the accumulators (the contiguous phase-2 region up to ni) and
    // the per-source scratch
    HCHK(hipMemsetAsync((char *)ws + L.T.off, 0, L.scratch.off - L.T.off, s));
    HCHK(hipMemsetAsync(ni, 0, 8ull * ORB_NORB * n, s));
    tm.mark("zero");

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
        HCHK(hipMemsetAsync(shist, 0, 4ull * SCHED_BINS, s));
        k_sched_bins<<<grid_for(n, WG), WG, 0, s>>>(feat, pred, n, sbin, shist);
        k_sched_offsets<<<1, 64, 0, s>>>(shist);
        k_sched_scatter<<<grid_for(n, WG), WG, 0, s>>>(sbin, n, shist, ord);
        HCHK(hipGetLastError());
        order = ord;
    }
    u64 *steps_out = opts ? (u64 *)opts->steps_out : nullptr;
    if (steps_out) HCHK(hipMemsetAsync(steps_out, 0, 8ull * n, s));
    tm.mark("schedule");

    if (ntri) {
        k_tri_fill<<<grid_for(m, WG), WG, 0, s>>>(src, outptr, outnbr, outslot, m, triptr, tri_c,
                                                  tri_sab, tri_sac, tri_sbc);
        k_tri_slots<<<grid_for(ntri, WG), WG, 0, s>>>(rev, ntri, tri_sab, tri_sac, tri_sbc, T, Tin,
                                                      Tmid);
        HCHK(hipGetLastError());
    }
    tm.mark("triangles");
    if (ntri && k_max >= 4) {
        k_tl_len<<<grid_for(M2, WG), WG, 0, s>>>(src, ci, T, M2, tllen);
        int rc2 = scan<u32>(tllen, M2, tlptr, bsum, st, s);
        if (rc2) return rc2;
        k_tl_fill<<<grid_for(ntri, WG), WG, 0, s>>>(src, ci, rev, ntri, tri_sab, tri_sac, tri_sbc,
                                                    tlptr, tlcur, tl);
        k_edge_e7e9<<<grid_for(M2, WG), WG, 0, s>>>(src, ci, rev, deg, T, tlptr, tl, M2, E7, E9);
        HCHK(hipGetLastError());
        if (k_max >= 5) {
            // lists sorted by third vertex for the pair sweep; the queue of
            // long lists reuses the (now free) list-length array, and the
            // long-list sort uses the per-source scratch before it is zeroed
            u32 *qlen = st->work + 15;
            k_tl_sort_small<<<grid_waves(M2), WG, 0, s>>>(src, ci, T, tlptr, tl, M2, tllen, qlen);
            k_tl_sort_wg<<<L.nwg, WG, 0, s>>>(rp, src, ci, T, tlptr, tl, tllen, qlen, scratch,
                                              L.stride, mapn);
            HCHK(hipGetLastError());
        }
    }
    tm.mark("tri_lists");
    k_vert0<<<grid_waves(n), WG, 0, s>>>(rp, ci, deg, T, n, Tv, N1);
    HCHK(hipGetLastError());
    u32 *work = st->work;
    int wi = 0;
    if (k_max >= 4) {
        rc = zero_scratch(0, mapn, scratch, L, L.nwg, s);
        if (rc) return rc;
        tm.mark("zero_c4");
        k_c4<<<L.nwg, WG, 0, s>>>(rp, ci, rev, key, n, scratch, L.stride, work + wi++, order,
                                  mapn, gbase, C4v, C4e);
        HCHK(hipGetLastError());
        tm.mark("c4");
        if (ntri) {
            k_clique<<<L.nwg, WG, 0, s>>>(1, n, rev, outptr, outnbr, outslot, triptr, tri_c,
                                          tri_sbc, scratch, L.stride, dmax, work + wi++, order, K4t, K4v, K4e,
                                          ni, st);
            HCHK(hipGetLastError());
        }
        tm.mark("cliques");
        if (ntri) {
            k_trisweep<<<grid_waves(n), WG, 0, s>>>(rp, ci, src, rev, deg, T, tlptr, tl, Tv, N1,
                                                    E7, E9, C4e, K4e, n, ni);
            HCHK(hipGetLastError());
        }
        tm.mark("trisweep");
    }
    if (k_max >= 5) {
        if (ntri) {
            k_clique<<<L.nwg, WG, 0, s>>>(2, n, rev, outptr, outnbr, outslot, triptr, tri_c,
                                          tri_sbc, scratch, L.stride, dmax, work + wi++, order, K4t, K4v, K4e,
                                          ni, st);
            k_tri_k4terms<<<grid_for(ntri, WG), WG, 0, s>>>(src, ci, T, ntri, tri_c, tri_sab,
                                                            tri_sac, tri_sbc, K4t, ni);
            HCHK(hipGetLastError());
        }
        tm.mark("clique2_k4terms");
        rc = zero_scratch(1, mapn, scratch, L, L.nwg, s);
        if (rc) return rc;
        tm.mark("zero_pairs");
        k_pairs<<<L.nwg, WG, 0, s>>>(rp, ci, src, rev, deg, T, tlptr, tl, n, scratch, L.stride,
                                     work + wi++, order, mapn, gbase, steps_out, Q, ni);
        HCHK(hipGetLastError());
        tm.mark("pairs");
        rc = zero_scratch(2, mapn, scratch, L, L.nwg < 256 ? L.nwg : 256, s);
        if (rc) return rc;
        tm.mark("zero_c5");
        k_c5<<<L.nwg < 256 ? L.nwg : 256, WG, 0, s>>>(rp, ci, key, outptr, outnbr, outslot, Tin, Tmid, n, scratch,
                                  L.stride, work + wi++, order, mapn, gbase, steps_out, ni);
        HCHK(hipGetLastError());
        tm.mark("c5");
    }
    k_vert1<<<grid_waves(n), WG, 0, s>>>(rp, ci, rev, deg, T, Tv, N1, C4v, K4v, C4e, K4e, E9, Q,
                                         n, ni);
    if (k_max >= 5) k_vert2<<<grid_waves(n), WG, 0, s>>>(rp, ci, deg, Tv, N1, n, ni);
    k_transform<<<grid_for(n, WG), WG, 0, s>>>(ni, n, K, (flags & ORB_NONINDUCED) ? 0 : 1, counts);
    HCHK(hipGetLastError());
    tm.mark("combine");
    if (flags & ORB_TIMING) {
        k_stats<<<grid_for(M2 > n ? M2 : n, WG), WG, 0, s>>>(src, ci, deg, T, n, M2, st);
        HCHK(hipGetLastError());
    }
    rc = read_state(st, &hs, s);
    if (rc) return rc;
    tm.finish();
    if (flags & ORB_TIMING) {
        g_stats[0] = n; g_stats[1] = m; g_stats[2] = ntri; g_stats[3] = hs.maxlevel;
        g_stats[4] = hs.wedges; g_stats[5] = hs.diamonds;
    }
    if (hs.err) return err_to_status(hs.err);
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
                   int k_max, uint64_t *counts, void *workspace, uint64_t ws_bytes,
                   uint64_t *ws_required, void *stream, const orb_opts *opts) {
    return count_impl(row_ptr, col_idx, n, m, nullptr, 0, k_max, (u64 *)counts, workspace, ws_bytes,
                      (u64 *)ws_required, (hipStream_t)stream, opts, false);
}

int orbit_workspace_query(const uint32_t *row_ptr, const uint32_t *col_idx, uint32_t n,
                          uint64_t m, int k_max, void *stream, const orb_opts *opts,
                          uint64_t *bytes) {
    if (!bytes || !orbit_num_orbits(k_max)) return ORB_E_INVALID_ARG;
    if (2 * m >= (1ull << 32)) return ORB_E_INVALID_ARG;
    Layout L;
    layout_phase1(L, n, m);
    void *tmp = nullptr;
    if (hipMalloc(&tmp, L.p1_end) != hipSuccess) return ORB_E_DEVICE;
    u64 req = 0;
    int rc = count_impl(row_ptr, col_idx, n, m, nullptr, 0, k_max, nullptr, tmp, L.p1_end, &req,
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
    void *ws = nullptr;
    if (hipMalloc(&ws, need ? need : 256) != hipSuccess) return ORB_E_DEVICE;
    rc = orbit_count_ex(row_ptr, col_idx, n, m, k_max, counts, ws, need, nullptr, nullptr,
                        nullptr);
    (void)hipFree(ws);
    return rc;
}

int orbit_count_batched(const uint64_t *vptr, uint32_t num_graphs, const uint32_t *row_ptr,
                        const uint32_t *col_idx, uint32_t n, uint64_t m, int k_max,
                        uint64_t *counts, void *workspace, uint64_t ws_bytes,
                        uint64_t *ws_required, void *stream, const orb_opts *opts) {
    if (!vptr) return ORB_E_INVALID_ARG;
    return count_impl(row_ptr, col_idx, n, m, (const u64 *)vptr, num_graphs, k_max,
                      (u64 *)counts, workspace, ws_bytes, (u64 *)ws_required,
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
                        tmp, L.p1_end, &req, (hipStream_t)stream, opts, true);
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
                            (u64 *)counts, workspace, ws_bytes, nullptr, s, &x, false);
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
        for (u32 sc = 0; sc < nsched; sc++) {
            orb_opts x = o;
            x.flags = keep_flags | ORB_TIMING;
            x.num_wg = nwg_candidates[c];
            x.schedule = sc;
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
    if (bms < 0) return ORB_E_WORKSPACE;
    b.flags = keep_flags;
    *best = b;
    if (best_ms) *best_ms = bms;
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
        default: return "unknown status";
    }
}

int orbit_last_stats(uint64_t *vals, int max_vals) {
    int k = max_vals < 6 ? max_vals : 6;
    for (int i = 0; i < k; i++) vals[i] = g_stats[i];
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
