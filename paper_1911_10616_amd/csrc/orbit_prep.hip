// Preprocessing kernels: CSR validation, reverse slots, degeneracy peeling,
// orientation and prefix scans.
#include "orbit_common.h"

// ------------------------------------------------------------ validation
// row_ptr must start at 0, be monotone and end at 2m.
__global__ void k_check_rowptr(const u32 *rp, u32 n, u64 M2, DevState *st) {
    for (u64 u = GTID; u < n; u += GSTRIDE)
        if (rp[u] > rp[u + 1]) atomicOr(&st->err, ERRB_ROWPTR);
    if (GTID == 0 && (rp[0] != 0 || (u64)rp[n] != M2)) atomicOr(&st->err, ERRB_ROWPTR);
}

// src[s] = owner vertex of slot s; deg[u] = |N(u)|.  One wave per vertex.
__global__ void k_src_deg(const u32 *rp, u32 n, u32 *src, u32 *deg) {
    for (u64 u = GWAVE; u < n; u += NWAVES) {
        u32 b = rp[u], e = rp[u + 1];
        if (lane_id() == 0) deg[u] = e - b;
        for (u32 s = b + lane_id(); s < e; s += WAVE) src[s] = (u32)u;
    }
}

// Per slot s = (u,v): range, self-loop, order and duplicate checks, and the
// reverse slot rev[s] = position of u in N(v) (found by binary search; its
// absence means the CSR is not symmetric).
__global__ void k_rev(const u32 *rp, const u32 *ci, const u32 *src, const u32 *gbase, u32 n,
                      u64 M2, u32 *rev, DevState *st) {
    for (u64 s = GTID; s < M2; s += GSTRIDE) {
        u32 u = src[s], v = ci[s];
        rev[s] = (u32)s;
        if (v >= n) { atomicOr(&st->err, ERRB_RANGE); continue; }
        if (v == u) atomicOr(&st->err, ERRB_LOOP);
        if (gbase && gbase[u] != gbase[v]) atomicOr(&st->err, ERRB_CROSS);
        if (s + 1 < rp[u + 1]) {
            u32 w = ci[s + 1];
            if (w == v) atomicOr(&st->err, ERRB_DUP);
            else if (w < v) atomicOr(&st->err, ERRB_ORDER);
        }
        u32 b = rp[v], len = rp[v + 1] - b;
        u32 i = bfind(ci + b, len, u);
        if (i == UNSET) atomicOr(&st->err, ERRB_ASYM);
        else rev[s] = b + i;
    }
}

// Batched input: graph g owns vertices [vptr[g], vptr[g+1]).  Checks that
// the offsets start at 0, never decrease and end at n; records each
// vertex's first vertex gbase[v] and the largest graph.  One wave per graph.
__global__ void k_batch_index(const u64 *vptr, u32 B, u32 n, u32 *gbase, DevState *st) {
    if (GTID == 0 && (vptr[0] != 0 || vptr[B] != n)) atomicOr(&st->err, ERRB_VPTR);
    for (u64 g = GWAVE; g < B; g += NWAVES) {
        const u64 lo = vptr[g], hi = vptr[g + 1];
        if (hi < lo || hi > n) {
            if (lane_id() == 0) atomicOr(&st->err, ERRB_VPTR);
            continue;
        }
        for (u64 v = lo + lane_id(); v < hi; v += WAVE) gbase[v] = (u32)lo;
        if (lane_id() == 0) atomicMax(&st->gmax, (u32)(hi - lo));
    }
}

// ------------------------------------------------------------ peeling
// Bucketed k-core peeling.  Vertices are removed in rounds; every removed
// vertex gets the round id, and rank(u) = (round, id).  A round either
// scans for alive vertices whose remaining degree is <= level, or removes
// the current frontier and appends the neighbours whose degree drops to
// level.  An out-neighbour of u (higher rank) is alive when u is removed,
// so out-degrees are bounded by the degeneracy.
__global__ void k_peel_init(const u32 *deg, u32 n, int *pdeg, u32 *rnd, DevState *st) {
    for (u64 u = GTID; u < n; u += GSTRIDE) {
        pdeg[u] = (int)deg[u];
        rnd[u] = UNSET;
    }
    if (GTID == 0) {
        st->level = 0; st->round = 0; st->cur = 0;
        st->fsize[0] = 0; st->fsize[1] = 0;
        st->alive = n; st->minalive = 0xffffffffu; st->maxlevel = 0;
    }
}

// The frontier is processed by groups of G lanes per vertex (G from the
// mean degree).
template <int G>
__global__ void k_peel_step(const u32 *rp, const u32 *ci, u32 n, int *pdeg, u32 *rnd,
                            u32 *front, DevState *st) {
    const u32 cur = st->cur, nxt = cur ^ 1u;
    const u32 fs = st->fsize[cur];
    const int level = (int)st->level;
    const u32 round = st->round;
    if (st->alive == 0) return;
    if (fs == 0) {
        // every lane of a wave runs the same iterations, so the frontier
        // appends and the minimum are combined per wave (one atomic each)
        for (u64 base = GTID - lane_id(); base < n; base += GSTRIDE) {
            const u64 u = base + lane_id();
            bool take = false;
            u32 dmin = 0xffffffffu;
            if (u < n && rnd[u] == UNSET) {
                const int d = pdeg[u];
                if (d <= level) take = true;
                else dmin = (u32)d;
            }
            const u64 mask = __ballot(take);
            if (mask) {
                u32 basepos = 0;
                const u32 leader = (u32)__ffsll((long long)mask) - 1;
                if (lane_id() == leader) basepos = atomicAdd(&st->fsize[nxt], (u32)__popcll(mask));
                basepos = __shfl(basepos, (int)leader, WAVE);
                if (take) {
                    rnd[u] = round;
                    front[(u64)nxt * n + basepos + __popcll(mask & ((1ull << lane_id()) - 1ull))] =
                        (u32)u;
                }
            }
            for (int off = WAVE / 2; off > 0; off >>= 1) {
                const u32 o = __shfl_xor(dmin, off, WAVE);
                dmin = o < dmin ? o : dmin;
            }
            if (lane_id() == 0 && dmin != 0xffffffffu) atomicMin(&st->minalive, dmin);
        }
    } else {
        for (u64 i = GTID / G; i < fs; i += GSTRIDE / G) {
            u32 u = front[(u64)cur * n + i];
            for (u32 s = rp[u] + (threadIdx.x & (G - 1)); s < rp[u + 1]; s += G) {
                u32 w = ci[s];
                if (rnd[w] != UNSET) continue;
                int old = atomicSub(&pdeg[w], 1);
                if (old == level + 1) {
                    rnd[w] = round;
                    u32 pos = atomicAdd(&st->fsize[nxt], 1u);
                    front[(u64)nxt * n + pos] = w;
                }
            }
        }
    }
}

__global__ void k_peel_advance(DevState *st) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (st->alive == 0) return;
    u32 cur = st->cur, nxt = cur ^ 1u;
    u32 nf = st->fsize[nxt];
    if (nf > 0) {
        if (st->level > st->maxlevel) st->maxlevel = st->level;
        st->round += 1;
        st->alive -= nf;
    } else if (st->fsize[cur] == 0) {
        // an empty scan: jump to the smallest remaining degree
        u32 nl = st->level + 1;
        if (st->minalive != 0xffffffffu && st->minalive > nl) nl = st->minalive;
        st->level = nl;
    }
    st->minalive = 0xffffffffu;
    st->fsize[cur] = 0;
    st->cur = nxt;
}

// Batched input of small graphs: the same peeling, one workgroup per graph
// with the graph's remaining degrees, rounds and frontiers in LDS, so the
// whole batch peels in one launch instead of a launch pair per round.
// Rounds are numbered within each graph (edges never join two graphs, so
// only ranks within a graph are compared).  cap: the largest graph the
// launch's LDS holds; a larger one records an error.  Every loop ends: a
// pass removes a vertex, or raises the level (and the next pass removes
// one), or empties a frontier that an earlier pass filled -- at most 3 n
// passes for a graph of n vertices.
__global__ void __launch_bounds__(WG) k_peel_graphs(const u64 *vptr, u32 B, u32 n,
                                                    const u32 *rp, const u32 *ci,
                                                    const u32 *deg, u32 cap, u32 *rnd,
                                                    DevState *st) {
    extern __shared__ u32 pl_lds[];
    int *pd = (int *)pl_lds;           // remaining degree   [cap]
    u32 *rr = pl_lds + cap;            // round, or UNSET     [cap]
    u32 *fr = pl_lds + 2 * cap;        // frontiers           [2 cap]
    __shared__ u32 sh_fs[2], sh_min;
    if (st->err) return;
    for (u64 g = blockIdx.x; g < B; g += gridDim.x) {
        const u64 lo = vptr[g], hi = vptr[g + 1];
        if (hi <= lo) continue;
        if (hi > n || hi - lo > cap) {
            if (threadIdx.x == 0) atomicOr(&st->err, ERRB_INTERNAL);
            continue;
        }
        const u32 ng = (u32)(hi - lo);
        for (u32 i = threadIdx.x; i < ng; i += WG) {
            pd[i] = (int)deg[lo + i];
            rr[i] = UNSET;
        }
        if (threadIdx.x == 0) { sh_fs[0] = 0; sh_fs[1] = 0; }
        __syncthreads();
        u32 alive = ng, round = 0, level = 0, maxlevel = 0, cur = 0;
        for (u32 pass = 0; alive > 0; pass++) {
            if (pass > 4 * ng + 4) {  // cannot happen (see above)
                if (threadIdx.x == 0) atomicOr(&st->err, ERRB_INTERNAL);
                break;
            }
            const u32 nxt = cur ^ 1u;
            const u32 fs = sh_fs[cur];
            if (threadIdx.x == 0) sh_min = UNSET;
            __syncthreads();
            if (fs == 0) {  // scan for alive vertices of remaining degree <= level
                for (u32 i = threadIdx.x; i < ng; i += WG) {
                    if (rr[i] != UNSET) continue;
                    const int d = pd[i];
                    if (d <= (int)level) {
                        rr[i] = round;
                        fr[nxt * cap + atomicAdd(&sh_fs[nxt], 1u)] = i;
                    } else {
                        atomicMin(&sh_min, (u32)d);
                    }
                }
            } else {  // remove the frontier; append neighbours dropping to level
                for (u32 t = threadIdx.x; t < fs; t += WG) {
                    const u32 v = fr[cur * cap + t];
                    for (u32 s = rp[lo + v]; s < rp[lo + v + 1]; s++) {
                        const u32 w = ci[s] - (u32)lo;
                        if (w >= ng) {  // an edge leaving the graph (rejected earlier)
                            atomicOr(&st->err, ERRB_INTERNAL);
                            continue;
                        }
                        if (rr[w] != UNSET) continue;
                        if (atomicSub(&pd[w], 1) == (int)level + 1) {
                            rr[w] = round;
                            fr[nxt * cap + atomicAdd(&sh_fs[nxt], 1u)] = w;
                        }
                    }
                }
            }
            __syncthreads();
            const u32 nf = sh_fs[nxt];
            if (nf > 0) {
                if (level > maxlevel) maxlevel = level;
                round++;
                alive -= nf;
            } else if (fs == 0) {  // an empty scan: jump to the smallest remaining degree
                u32 nl = level + 1;
                if (sh_min != UNSET && sh_min > nl) nl = sh_min;
                level = nl;
            }
            __syncthreads();
            if (threadIdx.x == 0) sh_fs[cur] = 0;
            cur = nxt;
        }
        for (u32 i = threadIdx.x; i < ng; i += WG) rnd[lo + i] = rr[i];
        if (threadIdx.x == 0) atomicMax(&st->maxlevel, maxlevel);
        __syncthreads();
    }
}

// key[u] = (round << 32) | u : the total order used to orient edges
__global__ void k_rank_key(const u32 *rnd, u32 n, u64 *key) {
    for (u64 u = GTID; u < n; u += GSTRIDE) key[u] = ((u64)rnd[u] << 32) | u;
}

// ------------------------------------------------------------ orientation
// outdeg[u] = |{v in N(u) : key[v] > key[u]}|, one wave per vertex.
__global__ void k_outdeg(const u32 *rp, const u32 *ci, const u64 *key, u32 n, u32 *outdeg) {
    for (u64 u = GWAVE; u < n; u += NWAVES) {
        u64 ku = key[u];
        u32 cnt = 0;
        for (u32 s = rp[u] + lane_id(); s < rp[u + 1]; s += WAVE) cnt += key[ci[s]] > ku;
        cnt = wave_sum_u32(cnt);
        if (lane_id() == 0) outdeg[u] = cnt;
    }
}

// out-lists: the out-neighbours of u in ascending id order, their slots.
__global__ void k_outfill(const u32 *rp, const u32 *ci, const u64 *key, u32 n,
                          const u64 *out_ptr, u32 *out_nbr, u32 *out_slot) {
    for (u64 u = GWAVE; u < n; u += NWAVES) {
        u64 ku = key[u];
        u64 base = out_ptr[u];
        u32 b = rp[u], e = rp[u + 1];
        for (u32 s0 = b; s0 < e; s0 += WAVE) {
            u32 s = s0 + lane_id();
            bool f = s < e && key[ci[s]] > ku;
            u64 mask = __ballot(f);
            u32 pre = __popcll(mask & ((1ull << lane_id()) - 1ull));
            if (f) {
                out_nbr[base + pre] = ci[s];
                out_slot[base + pre] = s;
            }
            base += __popcll(mask);
        }
    }
}

// ------------------------------------------------------------ scans
// Exclusive scan of n32 (u32 or u64 input) into u64 out[0..len], out[len] =
// total.  Three launches: block sums, scan of the block sums in one
// workgroup, block-local scans.
#define SCAN_ITEMS 4
#define SCAN_TILE (WG * SCAN_ITEMS)

template <typename T>
__global__ void k_scan_reduce(const T *in, u64 len, u64 *bsum) {
    __shared__ u64 sh[WAVES_PER_WG];
    u64 base = (u64)blockIdx.x * SCAN_TILE;
    u64 acc = 0;
    for (int k = 0; k < SCAN_ITEMS; k++) {
        u64 i = base + (u64)k * WG + threadIdx.x;
        if (i < len) acc += (u64)in[i];
    }
    acc = wave_sum_u64(acc);
    if (lane_id() == 0) sh[wave_in_wg()] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 t = 0;
        for (int w = 0; w < WAVES_PER_WG; w++) t += sh[w];
        bsum[blockIdx.x] = t;
    }
}

__global__ void k_scan_blocks(u64 *bsum, u64 nb, DevState *st) {
    // one workgroup: sequential chunks of WG, exclusive scan in place
    __shared__ u64 sh[WG];
    __shared__ u64 carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (u64 c = 0; c < nb; c += WG) {
        u64 i = c + threadIdx.x;
        u64 v = i < nb ? bsum[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (u32 off = 1; off < WG; off <<= 1) {
            u64 t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        u64 incl = sh[threadIdx.x];
        if (i < nb) bsum[i] = carry + incl - v;
        __syncthreads();
        if (threadIdx.x == WG - 1) carry += incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) st->scan_total = carry;
}

template <typename T>
__global__ void k_scan_final(const T *in, u64 len, const u64 *bsum, u64 *out, const DevState *st) {
    __shared__ u64 wsum[WAVES_PER_WG];
    u64 base = (u64)blockIdx.x * SCAN_TILE;
    // each thread owns SCAN_ITEMS consecutive items
    u64 vals[SCAN_ITEMS];
    u64 acc = 0;
    for (int k = 0; k < SCAN_ITEMS; k++) {
        u64 i = base + (u64)threadIdx.x * SCAN_ITEMS + k;
        vals[k] = i < len ? (u64)in[i] : 0;
        acc += vals[k];
    }
    // inclusive scan of per-thread sums within the wave
    u64 x = acc;
    for (int off = 1; off < WAVE; off <<= 1) {
        u64 t = __shfl_up(x, off, WAVE);
        if ((int)lane_id() >= off) x += t;
    }
    if (lane_id() == WAVE - 1) wsum[wave_in_wg()] = x;
    __syncthreads();
    u64 woff = 0;
    for (u32 w = 0; w < wave_in_wg(); w++) woff += wsum[w];
    u64 run = bsum[blockIdx.x] + woff + x - acc;
    for (int k = 0; k < SCAN_ITEMS; k++) {
        u64 i = base + (u64)threadIdx.x * SCAN_ITEMS + k;
        if (i < len) out[i] = run;
        run += vals[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[len] = st->scan_total;
}


// canonical-slot triangle-list lengths: T[s] where src[s] < ci[s], else 0
__global__ void k_tl_len(const u32 *src, const u32 *ci, const u32 *T, u64 M2, u32 *len) {
    for (u64 s = GTID; s < M2; s += GSTRIDE) len[s] = src[s] < ci[s] ? T[s] : 0u;
}

__global__ void k_fill_u64(u64 *p, u64 len, u64 v) {
    for (u64 i = GTID; i < len; i += GSTRIDE) p[i] = v;
}
__global__ void k_fill_u32(u32 *p, u64 len, u32 v) {
    for (u64 i = GTID; i < len; i += GSTRIDE) p[i] = v;
}

// Zero `rows` rows of `width` u64 words, `pitch` bytes apart (the
// per-source scratch ranges; a kernel rather than a 2-D memset so that the
// whole count can be captured into a graph).
__global__ void k_zero_rows(unsigned char *base, u64 pitch, u64 width, u64 rows) {
    for (u64 i = GTID; i < width * rows; i += GSTRIDE) {
        const u64 r = i / width, w = i - r * width;
        ((u64 *)(base + r * pitch))[w] = 0;
    }
}

// Plans: the triangle count as left by the last scan of phase 1, and the
// check that a replayed graph saw the same sizes as the run it was built
// from (same peel completion, triangle count, degeneracy, largest graph).
__global__ void k_save_ntri(DevState *st) {
    if (GTID == 0) st->ntri = st->scan_total;
}
// Checks made during a replay, right after the step that fixes each size,
// so that no later kernel runs on sizes its buffers were not made for:
// what = 0: the largest graph of a batch is no larger than planned;
// what = 1: peeling finished within the planned launches;
// what = 2: the triangle count equals the planned one.
__global__ void k_plan_guard(DevState *st, int what, u64 expect) {
    if (GTID != 0) return;
    const bool bad = what == 0 ? st->gmax > expect
                   : what == 1 ? st->alive != 0
                               : st->scan_total != expect;
    if (bad) atomicOr(&st->err, ERRB_INTERNAL);
}
__global__ void k_plan_check(DevState *st, u64 ntri, u32 maxlevel, u32 gmax) {
    if (GTID == 0 && (st->alive != 0 || st->ntri != ntri || st->maxlevel != maxlevel ||
                      st->gmax != gmax))
        atomicOr(&st->err, ERRB_INTERNAL);
}

