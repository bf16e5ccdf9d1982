// Enumeration kernels: directed triangles and per-edge triangle lists,
// per-edge orbit quantities, 4-cycles, 4-/5-cliques, the pair sweep over
// wedges and diamonds, and 5-cycles.
#include "orbit_common.h"

// Orbit columns written by these kernels (non-induced accumulators).
#define NI(u, o) ni[(u64)(u) * ORB_NORB + (o)]

// ======================================================= directed triangles
// For every out-arc a->b (a before b in rank order) the common
// out-neighbours c of a and b: each triangle a<b<c is found once, from its
// two lowest-ranked vertices (the orientation of Fig. 5vertex-basis).
__device__ inline u32 arc_owner_of(const u32 *src, const u32 *out_slot, u64 p) {
    return src[out_slot[p]];
}

__global__ void k_tri_count(const u32 *src, const u64 *out_ptr, const u32 *out_nbr,
                            const u32 *out_slot, u64 m, u32 *tcnt) {
    for (u64 p = GTID; p < m; p += GSTRIDE) {
        u32 a = arc_owner_of(src, out_slot, p), b = out_nbr[p];
        u64 i = out_ptr[a], ie = out_ptr[a + 1], j = out_ptr[b], je = out_ptr[b + 1];
        u32 c = 0;
        while (i < ie && j < je) {
            u32 x = out_nbr[i], y = out_nbr[j];
            c += x == y;
            i += x <= y;
            j += y <= x;
        }
        tcnt[p] = c;
    }
}

// Triangle records, grouped by owner arc (a->b) and sorted by c:
// tri_c = c, tri_sab/sac/sbc = slots of (a,b), (a,c), (b,c).
// Writes nothing once an error is recorded (a replayed plan whose triangle
// count differs from the planned one must not write past its buffers).
__global__ void k_tri_fill(const u32 *src, const u64 *out_ptr, const u32 *out_nbr,
                           const u32 *out_slot, u64 m, const u64 *tri_ptr, u32 *tri_c,
                           u32 *tri_sab, u32 *tri_sac, u32 *tri_sbc, const DevState *st) {
    if (st->err) return;
    for (u64 p = GTID; p < m; p += GSTRIDE) {
        u32 a = arc_owner_of(src, out_slot, p), b = out_nbr[p];
        u64 i = out_ptr[a], ie = out_ptr[a + 1], j = out_ptr[b], je = out_ptr[b + 1];
        u64 w = tri_ptr[p];
        u32 sab = out_slot[p];
        while (i < ie && j < je) {
            u32 x = out_nbr[i], y = out_nbr[j];
            if (x == y) {
                tri_c[w] = x;
                tri_sab[w] = sab;
                tri_sac[w] = out_slot[i];
                tri_sbc[w] = out_slot[j];
                w++;
            }
            i += x <= y;
            j += y <= x;
        }
    }
}

// Per-slot triangle counts: T = all triangles on the edge, Tin = those
// whose third vertex precedes both ends (|N-(x) & N-(y)|), Tmid (on the
// slots of arc a->c) = those whose third vertex lies between (|N+(a) & N-(c)|).
// The kernels that read triangle records or lists do nothing once an error
// is recorded: after a size check failed the records were never written.
__global__ void k_tri_slots(const u32 *rev, u64 ntri, const u32 *tri_sab, const u32 *tri_sac,
                            const u32 *tri_sbc, u32 *T, u32 *Tin, u32 *Tmid, const DevState *st) {
    if (st->err) return;
    for (u64 t = GTID; t < ntri; t += GSTRIDE) {
        u32 sab = tri_sab[t], sac = tri_sac[t], sbc = tri_sbc[t];
        atomicAdd(&T[sab], 1u); atomicAdd(&T[rev[sab]], 1u);
        atomicAdd(&T[sac], 1u); atomicAdd(&T[rev[sac]], 1u);
        atomicAdd(&T[sbc], 1u); atomicAdd(&T[rev[sbc]], 1u);
        atomicAdd(&Tin[sbc], 1u); atomicAdd(&Tin[rev[sbc]], 1u);
        atomicAdd(&Tmid[sac], 1u); atomicAdd(&Tmid[rev[sac]], 1u);
    }
}

// Undirected per-edge triangle lists, stored once per edge at its canonical
// slot (the slot in the list of the smaller id).  Entry for third vertex x
// of edge (lo,hi): (slot of (lo,x), slot of (hi,x)).
__device__ inline void tl_push(u32 s_xy, u32 s_xz, u32 s_yz, const u32 *src, const u32 *ci,
                               const u32 *rev, const u64 *tl_ptr, u32 *tl_cur, uint2 *tl) {
    // edge (x,y) with third vertex z; s_xz = slot (x,z), s_yz = slot (y,z)
    u32 x = src[s_xy], y = ci[s_xy];
    u32 cs = x < y ? s_xy : rev[s_xy];
    uint2 e = x < y ? make_uint2(s_xz, s_yz) : make_uint2(s_yz, s_xz);
    u32 pos = atomicAdd(&tl_cur[cs], 1u);
    tl[tl_ptr[cs] + pos] = e;
}

__global__ void k_tl_fill(const u32 *src, const u32 *ci, const u32 *rev, u64 ntri,
                          const u32 *tri_sab, const u32 *tri_sac, const u32 *tri_sbc,
                          const u64 *tl_ptr, u32 *tl_cur, uint2 *tl, const DevState *st) {
    if (st->err) return;
    for (u64 t = GTID; t < ntri; t += GSTRIDE) {
        u32 sab = tri_sab[t], sac = tri_sac[t], sbc = tri_sbc[t];
        u32 sba = rev[sab], sca = rev[sac], scb = rev[sbc];
        tl_push(sab, sac, sbc, src, ci, rev, tl_ptr, tl_cur, tl);  // edge ab, third c
        tl_push(sac, sab, scb, src, ci, rev, tl_ptr, tl_cur, tl);  // edge ac, third b
        tl_push(sbc, sba, sca, src, ci, rev, tl_ptr, tl_cur, tl);  // edge bc, third a
    }
}

// Sorting the per-edge triangle lists by third vertex.  Within one list the
// third vertices are distinct, and both components of an entry grow with
// the third vertex's id (neighbour lists are ascending), so ordering by the
// first component orders the list by third vertex.  Lists of up to 64
// entries are sorted by one wave in registers (bitonic network over lanes);
// longer ones are queued for k_tl_sort_wg.
#ifndef TL_SORT_LDS
#define TL_SORT_LDS 4096
#endif
static_assert(TL_SORT_LDS >= 128 && (TL_SORT_LDS & (TL_SORT_LDS - 1)) == 0,
              "TL_SORT_LDS: a power of two >= 128");
__device__ inline u64 tl_key(uint2 e) { return ((u64)e.x << 32) | e.y; }
__device__ inline uint2 tl_unkey(u64 k) { return make_uint2((u32)(k >> 32), (u32)k); }

__global__ void k_tl_sort_small(const u32 *src, const u32 *ci, const u32 *T, const u64 *tl_ptr,
                                uint2 *tl, u64 M2, u32 *queue, u32 *qlen) {
    const u32 lane = lane_id();
    for (u64 s = GWAVE; s < M2; s += NWAVES) {
        if (src[s] > ci[s]) continue;  // the list lives at the canonical slot
        const u32 L = T[s];
        if (L < 2) continue;
        if (L > WAVE) {
            if (lane == 0) queue[atomicAdd(qlen, 1u)] = (u32)s;
            continue;
        }
        uint2 *p = tl + tl_ptr[s];
        u64 key = ~0ull;
        if (lane < L) key = tl_key(p[lane]);
        for (u32 k = 2; k <= WAVE; k <<= 1) {
            for (u32 j = k >> 1; j > 0; j >>= 1) {
                const u64 other = __shfl_xor(key, (int)j, WAVE);
                const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
                key = keep_min ? (key < other ? key : other) : (key > other ? key : other);
            }
        }
        if (lane < L) p[lane] = tl_unkey(key);
    }
}

// One workgroup per queued list.  Up to TL_SORT_LDS entries: bitonic sort in
// LDS.  Longer lists (both ends then have degree > TL_SORT_LDS): counting
// sort over positions in the shorter of the two neighbour lists -- a bitmap
// of occupied positions and the other component stored at its position in
// the workgroup's scratch, then ranks from a scan of the bitmap's popcounts.
__global__ void __launch_bounds__(WG) k_tl_sort_wg(const u32 *rp, const u32 *src, const u32 *ci,
                                                  const u32 *T, const u64 *tl_ptr, uint2 *tl,
                                                  const u32 *queue, const u32 *qlen,
                                                  unsigned char *scratch, u64 stride, u32 mapn,
                                                  const DevState *st) {
    __shared__ u64 sk[TL_SORT_LDS];
    __shared__ u32 part[WG];
    if (st->err) return;
    u32 *oth = (u32 *)(scratch + (u64)blockIdx.x * stride);          // mapn entries
    u32 *bm = (u32 *)align256((unsigned char *)(oth + mapn));        // ceil(mapn/32) words
    const u32 cnt = *qlen;
    for (u32 qi = blockIdx.x; qi < cnt; qi += gridDim.x) {
        const u32 s = queue[qi];
        const u32 L = T[s];
        uint2 *p = tl + tl_ptr[s];
        if (L <= TL_SORT_LDS) {
            u32 P = 128;
            while (P < L) P <<= 1;
            for (u32 i = threadIdx.x; i < P; i += WG) sk[i] = i < L ? tl_key(p[i]) : ~0ull;
            __syncthreads();
            for (u32 k = 2; k <= P; k <<= 1) {
                for (u32 j = k >> 1; j > 0; j >>= 1) {
                    for (u32 i = threadIdx.x; i < P; i += WG) {
                        const u32 ij = i ^ j;
                        if (ij > i) {
                            const u64 x = sk[i], y = sk[ij];
                            const bool asc = (i & k) == 0;
                            if ((x > y) == asc) { sk[i] = y; sk[ij] = x; }
                        }
                    }
                    __syncthreads();
                }
            }
            for (u32 i = threadIdx.x; i < L; i += WG) p[i] = tl_unkey(sk[i]);
            __syncthreads();
            continue;
        }
        const u32 lo = src[s], hi = ci[s];
        const u32 dlo = rp[lo + 1] - rp[lo], dhi = rp[hi + 1] - rp[hi];
        const bool by_lo = dlo <= dhi;
        const u32 base = by_lo ? rp[lo] : rp[hi];
        const u32 D = by_lo ? dlo : dhi;
        const u32 nw = (D + 31) / 32;
        for (u32 w = threadIdx.x; w < nw; w += WG) bm[w] = 0;
        __syncthreads();
        for (u32 i = threadIdx.x; i < L; i += WG) {
            const uint2 e = p[i];
            const u32 pos = (by_lo ? e.x : e.y) - base;
            atomicOr(&bm[pos >> 5], 1u << (pos & 31));
            oth[pos] = by_lo ? e.y : e.x;
        }
        __syncthreads();
        // each thread owns a contiguous run of bitmap words
        const u32 per = (nw + WG - 1) / WG;
        const u32 w0 = threadIdx.x * per, w1 = w0 + per < nw ? w0 + per : nw;
        u32 c = 0;
        for (u32 w = w0; w < w1; w++) c += __popc(bm[w]);
        part[threadIdx.x] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            u32 run = 0;
            for (u32 t = 0; t < WG; t++) { const u32 v = part[t]; part[t] = run; run += v; }
        }
        __syncthreads();
        u32 r = part[threadIdx.x];
        for (u32 w = w0; w < w1; w++) {
            u32 bits = bm[w];
            while (bits) {
                const u32 b = __ffs(bits) - 1;
                bits &= bits - 1;
                const u32 pos = w * 32 + b;
                const u32 mine = base + pos, other = oth[pos];
                p[r++] = by_lo ? make_uint2(mine, other) : make_uint2(other, mine);
            }
        }
        __syncthreads();
    }
}

// Triangle list of slot s = (u,v) as (slot(u,x), slot(v,x)) pairs.
struct TLView {
    const uint2 *p;
    u32 len;
    bool swap;
    __device__ inline uint2 get(u32 i) const {
        uint2 e = p[i];
        return swap ? make_uint2(e.y, e.x) : e;
    }
};
__device__ inline TLView tl_view(u32 s, const u32 *src, const u32 *ci, const u32 *rev,
                                 const u32 *T, const u64 *tl_ptr, const uint2 *tl) {
    TLView v;
    bool lo = src[s] < ci[s];
    u32 cs = lo ? s : rev[s];
    v.p = tl + tl_ptr[cs];
    v.len = T[s];
    v.swap = !lo;
    return v;
}

// Edge orbits of Lemma 4edgeorbit that need the triangle list:
// E7(u,v) = sum over triangles (u,v,x) of (d(x) - 2),
// E9<u,v> = sum over triangles (u,v,x) of (T(u,x) - 1)   [at slot (u,v)].
__global__ void k_edge_e7e9(const u32 *src, const u32 *ci, const u32 *rev, const u32 *deg,
                            const u32 *T, const u64 *tl_ptr, const uint2 *tl, u64 M2, u64 *E7,
                            u64 *E9, const DevState *st) {
    if (st->err) return;
    for (u64 s = GTID; s < M2; s += GSTRIDE) {
        TLView v = tl_view((u32)s, src, ci, rev, T, tl_ptr, tl);
        u64 e7 = 0, e9 = 0;
        for (u32 i = 0; i < v.len; i++) {
            uint2 e = v.get(i);
            e7 += (u64)deg[ci[e.x]] - 2;
            e9 += (u64)T[e.x] - 1;
        }
        E7[s] = e7;
        E9[s] = e9;
    }
}

// ======================================================= per-source kernels
// One workgroup per source vertex at a time (dynamic), with dense per-WG
// scratch arrays indexed by vertex id that are restored to zero after
// every source.
// Execution group of a per-source kernel: the whole workgroup works on one
// source (GpWG: heavy sources, big graphs), or each wave works on its own
// source with its own scratch (GpWave: many light sources, small graphs).
struct GpWG {
    static constexpr u32 size = WG, per_wg = 1, chunk = 1;
    __device__ static u32 id() { return 0; }
    __device__ static u32 rank() { return threadIdx.x; }
    __device__ static u64 global_id() { return blockIdx.x; }
    __device__ static void sync() { __syncthreads(); }
    __device__ static u64 sum(u64 v, u64 *sh) {
        v = wave_sum_u64(v);
        __syncthreads();
        if (lane_id() == 0) sh[wave_in_wg()] = v;
        __syncthreads();
        u64 t = 0;
        for (int w = 0; w < WAVES_PER_WG; w++) t += sh[w];
        return t;
    }
};
struct GpWave {
    static constexpr u32 size = WAVE, per_wg = WAVES_PER_WG, chunk = 16;
    __device__ static u32 id() { return wave_in_wg(); }
    __device__ static u32 rank() { return lane_id(); }
    __device__ static u64 global_id() { return (u64)blockIdx.x * per_wg + wave_in_wg(); }
    __device__ static void sync() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    }
    __device__ static u64 sum(u64 v, u64 *) { return wave_sum_u64(v); }
};

// The sources come from a queue: the i-th entry is order[i] (a schedule),
// or i itself when there is no schedule; n once the queue is empty.  A group
// takes GP::chunk consecutive entries per atomic on the shared counter (light
// sources would otherwise serialise on it).  q[0..1] = the group's current
// range of queue entries, q[2] = the source handed out; both start at 0.
// Once an error is recorded (st->err) the queue reads as empty from the next
// chunk on, so a replayed plan whose sizes no longer match its buffers stops
// early.
template <class GP>
__device__ inline u32 next_source(u32 *counter, u32 *q, const u32 *order, u32 n,
                                  const DevState *st) {
    GP::sync();
    if (GP::rank() == 0) {
        if (q[0] >= q[1]) {
            // the error word is looked at once per chunk (an agent-scope
            // load: it stays in the L2)
            const bool stop =
                __hip_atomic_load(&st->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            const u32 i = stop ? n : atomicAdd(counter, GP::chunk);
            q[0] = i;
            q[1] = i < n ? (n - i < GP::chunk ? n : i + GP::chunk) : i;
        }
        const u32 i = q[0];
        q[2] = i < q[1] ? (order ? order[i] : i) : n;
        q[0] = i + 1;
    }
    GP::sync();
    return q[2];
}

// Dynamic loop of a wave over [0, count): items are taken from an LDS
// counter, so a long item does not hold up the other waves' items.
template <typename F>
__device__ inline void wave_loop(u32 *counter, u32 count, F f) {
    for (;;) {
        u32 i = 0;
        if (lane_id() == 0) i = atomicAdd(counter, 1u);
        i = __shfl(i, 0, WAVE);
        if (i >= count) break;
        f(i);
    }
}

__device__ inline u64 block_sum_u64(u64 v, u64 *sh) {
    v = wave_sum_u64(v);
    __syncthreads();
    if (lane_id() == 0) sh[wave_in_wg()] = v;
    __syncthreads();
    u64 t = 0;
    for (int w = 0; w < WAVES_PER_WG; w++) t += sh[w];
    return t;
}

// ---- Per-source maps in LDS.  When a map (indexed by vertex within the
// source's graph) is small -- small graphs, and every graph of a batch of
// small graphs -- each wave of a wave-group kernel keeps its maps in its own
// slice of the workgroup's dynamic LDS (lmw u64 words per wave) instead of
// the per-group scratch in HBM.  The slices are cleared once when the
// workgroup starts; after that each source restores what it dirtied, as in
// HBM.  The pointers are formed from the LDS array by plain pointer
// arithmetic so that the compiler emits LDS instructions for them.
__device__ inline u64 *wave_lds_slice(u64 *dyn, u64 lmw) {
    return dyn + (u64)wave_in_wg() * lmw;
}
__device__ inline void clear_lds(u64 *p, u64 words) {
    for (u64 i = threadIdx.x; i < words; i += WG) p[i] = 0;
    __syncthreads();
}
// map entries rounded up so that the arrays after them stay 8-byte aligned
__host__ __device__ inline u32 map_even(u32 mapn) { return (mapn + 1) & ~1u; }
// u64 words per wave of each kernel's maps
__host__ __device__ inline u64 c4_lds_words(u32 mapn) { return map_even(mapn); }
__host__ __device__ inline u64 pair_lds_words(u32 mapn) { return 2ull * mapn + map_even(mapn) / 2; }

// ---- 4-cycles (Chiba-Nishizeki).  For every top vertex x: the wedges
// x - y - z with y and z before x in rank order; cnt[z] = number of such y.
// Every 4-cycle has a unique top x and opposite z; it adds C(cnt,2) to x and
// z, cnt-1 to each middle y, and cnt-1 to the edges (x,y) and (y,z).
// Gives C4(u) (orbit 8) and C4(e) (edge orbit E5).
// LM: the maps (cnt, touched) live in LDS (lmw words per wave).
template <class GP, bool LM>
__global__ void __launch_bounds__(WG) k_c4(const u32 *rp, const u32 *ci, const u32 *rev,
                                          const u64 *key, u32 n, unsigned char *scratch,
                                          u64 stride, u32 *work, const u32 *order, u32 mapn,
                                          const u32 *gbase, u64 lmw, u64 *C4v, u64 *C4e,
                                          const DevState *st) {
    __shared__ u32 sh_q_[GP::per_wg][3], sh_nt_[GP::per_wg], sh_next_[GP::per_wg];
    u32 *sh_q = sh_q_[GP::id()];
    if (GP::rank() == 0) { sh_q[0] = 0; sh_q[1] = 0; }
    u32 &sh_nt = sh_nt_[GP::id()];
    u32 &sh_next = sh_next_[GP::id()];
    __shared__ u64 sh_red[WAVES_PER_WG];
    static_assert(!LM || GP::per_wg > 1, "LDS maps are per wave");
    extern __shared__ u64 dyn_lds[];
    u32 *cnt, *touched;
    if constexpr (LM) {
        clear_lds(dyn_lds, WAVES_PER_WG * lmw);
        cnt = (u32 *)wave_lds_slice(dyn_lds, lmw);
        touched = cnt + map_even(mapn);
    } else {
        unsigned char *base = scratch + GP::global_id() * stride;
        cnt = (u32 *)base;
        touched = (u32 *)align256((unsigned char *)(cnt + mapn));
    }
    for (;;) {
        u32 x = next_source<GP>(work, sh_q, order, n, st);
        if (x >= n) break;
        const u32 vb = gbase ? gbase[x] : 0;  // maps are indexed within x's graph
        const u64 kx = key[x];
        const u32 bx = rp[x], dx = rp[x + 1] - bx;
        if (GP::rank() == 0) { sh_nt = 0; sh_next = 0; }
        GP::sync();
        wave_loop(&sh_next, dx, [&](u32 i) {
            u32 y = ci[bx + i];
            if (key[y] >= kx) return;
            for (u32 s = rp[y] + lane_id(); s < rp[y + 1]; s += WAVE) {
                u32 z = ci[s];
                if (z != x && key[z] < kx) {
                    u32 old = atomicAdd(&cnt[z - vb], 1u);
                    if (old == 0) touched[atomicAdd(&sh_nt, 1u)] = z;
                }
            }
        });
        GP::sync();
        const u32 nt = sh_nt;
        u64 loc = 0;
        for (u32 t = GP::rank(); t < nt; t += GP::size) {
            u32 z = touched[t];
            u64 v = c2(cnt[z - vb]);
            loc += v;
            atomic_add_u64(&C4v[z], v);
        }
        u64 tot = GP::sum(loc, sh_red);
        if (GP::rank() == 0) { atomic_add_u64(&C4v[x], tot); sh_next = 0; }
        GP::sync();
        wave_loop(&sh_next, dx, [&](u32 i) {
            u32 sxy = bx + i;
            u32 y = ci[sxy];
            if (key[y] >= kx) return;
            u64 acc = 0;
            for (u32 s = rp[y] + lane_id(); s < rp[y + 1]; s += WAVE) {
                u32 z = ci[s];
                if (z != x && key[z] < kx) {
                    u32 c = cnt[z - vb];
                    if (c > 1) {
                        acc += c - 1;
                        atomicAdd(&C4e[s], (u64)(c - 1));
                        atomicAdd(&C4e[rev[s]], (u64)(c - 1));
                    }
                }
            }
            acc = wave_sum_u64(acc);
            if (lane_id() == 0 && acc) {
                atomicAdd(&C4v[y], acc);
                atomicAdd(&C4e[sxy], acc);
                atomicAdd(&C4e[rev[sxy]], acc);
            }
        });
        GP::sync();
        for (u32 t = GP::rank(); t < nt; t += GP::size) cnt[touched[t] - vb] = 0;
    }
}

// ---- 4- and 5-cliques.  For a source a, G+(a) is the graph induced on its
// out-neighbours; its adjacency is held as bit rows (outm: out-neighbours,
// inm: in-neighbours within G+(a); the undirected row is their union).
// Every clique is counted once from its lowest-ranked vertex a: triangle
// records (a,b,c) give the 4-clique apexes inside N+(a) as (outm | inm)[b]
// & (outm | inm)[c] (and oriented ones as outm[b] & outm[c]); 5-cliques are the 4-cliques of
// G+(a).  Each oriented triangle x < y < z of G+(a) (a 4-clique a,x,y,z)
// credits x, y and z with up = |outm[x] & outm[y] & outm[z]| (the 4-cliques
// of G+(a) it is the bottom of) and z also with down = |inm[x] & inm[y] &
// inm[z]| (those it is the top of), so every member of every 4-clique of
// G+(a) -- every 5-clique through a -- is credited once without visiting
// the 5-cliques one by one.
//   pass 1: K4(u) (orbit 14), K4(e) (edge orbit E11), K4(t) per triangle
//           (apexes inside N+(a) plus one credit from each 4-clique whose
//           lowest vertex precedes the triangle), 5-cliques (orbit 72).
//   pass 2: orbit 70, sum over 4-cliques containing u of K4(opposite
//           triangle) - 1 (Theorem 5vertexorbit), needing the final K4(t).
#ifndef CLQ_LDS_D
#define CLQ_LDS_D 1024
#endif
// u64 words of one execution group's LDS rows for out-degrees up to d
__host__ __device__ inline u64 clique_lds_words(u32 d) {
    return 2ull * d + 2ull * d * ((d + 63) / 64) + (d + 1) / 2;
}

// Forward cursor over one triangle list: the keys it is asked for increase, so each search
// covers only the entries after the previous hit.
struct TriCursor {
    u64 base;
    u32 len;
    __device__ void open(u64 arc, const u64 *tri_ptr) {
        base = tri_ptr[arc];
        len = (u32)(tri_ptr[arc + 1] - base);
    }
    __device__ u64 find(u32 z, const u32 *tri_c, DevState *st) {
        u32 i = bfind(tri_c + base, len, z);
        if (i == UNSET) { atomicOr(&st->err, ERRB_INTERNAL); return base; }
        const u64 p = base + i;
        base = p + 1;
        len -= i + 1;
        return p;
    }
};
__device__ inline u64 arc_find(u32 x, u32 y, const u64 *out_ptr, const u32 *out_nbr,
                               DevState *st) {
    u64 b = out_ptr[x];
    u32 len = (u32)(out_ptr[x + 1] - b);
    u32 i = bfind(out_nbr + b, len, y);
    if (i == UNSET) { atomicOr(&st->err, ERRB_INTERNAL); return b; }
    return b + i;
}

template <class GP>
__global__ void __launch_bounds__(WG) k_clique(int pass, u32 n, const u32 *rev,
                                              const u64 *out_ptr, const u32 *out_nbr,
                                              const u32 *out_slot, const u64 *tri_ptr,
                                              const u32 *tri_c, const u32 *tri_sbc,
                                              unsigned char *scratch, u64 stride, u32 dcap,
                                              u32 lds_d, u32 *work, const u32 *order, u32 *K4t,
                                              u64 *K4v, u64 *K4e, u64 *ni, DevState *st) {
    __shared__ u32 sh_q_[GP::per_wg][3], sh_next_[GP::per_wg];
    u32 *sh_q = sh_q_[GP::id()];
    if (GP::rank() == 0) { sh_q[0] = 0; sh_q[1] = 0; }
    u32 &sh_next = sh_next_[GP::id()];
    __shared__ u64 sh_red[WAVES_PER_WG];
    // dynamic LDS: acc, acc5 [lds_d]; inm, outm [lds_d * lds_w]; nbr [lds_d]
    // (one such set per execution group)
    extern __shared__ u64 dyn_lds[];
    const u32 lds_w = (lds_d + 63) / 64;
    u64 *l_acc = dyn_lds + (u64)GP::id() * clique_lds_words(lds_d), *l_acc5 = l_acc + lds_d;
    u64 *l_inm = l_acc5 + lds_d, *l_out = l_inm + (u64)lds_d * lds_w;
    u32 *l_nbr = (u32 *)(l_out + (u64)lds_d * lds_w);
    unsigned char *gbase = scratch + GP::global_id() * stride;
    for (;;) {
        u32 a = next_source<GP>(work, sh_q, order, n, st);
        if (a >= n) break;
        const u64 pa = out_ptr[a];
        const u32 D = (u32)(out_ptr[a + 1] - pa);
        if (D < 2) continue;
        const u32 W = (D + 63) / 64;
        u32 *nbr;
        u64 *inm, *outm, *acc, *acc5;
        if (D <= lds_d) {
            nbr = l_nbr; inm = l_inm; outm = l_out; acc = l_acc; acc5 = l_acc5;
        } else {
            if (D > dcap) {  // cannot happen: out-degrees are bounded by the peel level
                if (GP::rank() == 0) atomicOr(&st->err, ERRB_INTERNAL);
                continue;
            }
            nbr = (u32 *)gbase;
            inm = (u64 *)align256((unsigned char *)(nbr + D));
            outm = inm + (u64)D * W;
            acc = outm + (u64)D * W;
            acc5 = acc + D;
        }
        for (u32 i = GP::rank(); i < D; i += GP::size) {
            nbr[i] = out_nbr[pa + i];
            acc[i] = 0;
            acc5[i] = 0;
        }
        // the in-rows serve pass 1 only
        for (u32 i = GP::rank(); i < D * W; i += GP::size) {
            outm[i] = 0;
            if (pass == 1) inm[i] = 0;
        }
        if (GP::rank() == 0) sh_next = 0;
        GP::sync();
        wave_loop(&sh_next, D, [&](u32 i) {
            u32 b = nbr[i];
            for (u64 q = out_ptr[b] + lane_id(); q < out_ptr[b + 1]; q += WAVE) {
                u32 j = bfind(nbr, D, out_nbr[q]);
                if (j != UNSET) {
                    atomicOr(&outm[(u64)i * W + j / 64], 1ull << (j % 64));
                    if (pass == 1) atomicOr(&inm[(u64)j * W + i / 64], 1ull << (i % 64));
                }
            }
        });
        GP::sync();
        const u64 r0 = tri_ptr[pa], r1 = tri_ptr[pa + D];
        u64 tot = 0, tot5 = 0;
        for (u64 r = r0 + GP::rank(); r < r1; r += GP::size) {
            // owner arc of record r: largest p in [pa, pa+D) with tri_ptr[p] <= r
            u32 lo = 0, hi = D;
            while (hi - lo > 1) {
                u32 mid = (lo + hi) >> 1;
                if (tri_ptr[pa + mid] <= r) lo = mid; else hi = mid;
            }
            const u32 i = lo;
            const u32 c = tri_c[r];
            const u32 j = bfind(nbr, D, c);
            if (j == UNSET) { atomicOr(&st->err, ERRB_INTERNAL); continue; }
            const u64 *ri = inm + (u64)i * W, *rj = inm + (u64)j * W;
            const u64 *oi = outm + (u64)i * W, *oj = outm + (u64)j * W;
            if (pass == 1) {
                // the undirected row is out | in
                u32 k = 0;
                for (u32 w = 0; w < W; w++) k += __popcll((ri[w] | oi[w]) & (rj[w] | oj[w]));
                if (k) {
                    atomicAdd(&K4t[r], k);
                    u32 sbc = tri_sbc[r];
                    atomicAdd(&K4e[sbc], (u64)k);
                    atomicAdd(&K4e[rev[sbc]], (u64)k);
                    atomicAdd(&acc[i], (u64)k);
                    atomicAdd(&acc[j], (u64)k);
                    tot += k;
                }
                const u32 b = nbr[i];
                // the apexes d come in increasing order, so the list of (b,c) is walked forward
                TriCursor cbc;
                bool open = false;
                for (u32 w = 0; w < W; w++) {
                    u64 msk = oi[w] & oj[w];
                    while (msk) {
                        u32 l = w * 64 + __ffsll((long long)msk) - 1;
                        msk &= msk - 1;
                        u32 d = nbr[l];
                        if (!open) {
                            cbc.open(arc_find(b, c, out_ptr, out_nbr, st), tri_ptr);
                            open = true;
                        }
                        // the triangle (b,c,d) gets this 4-clique as an apex a
                        atomicAdd(&K4t[cbc.find(d, tri_c, st)], 1u);
                        // the oriented triangle (i, j, l) of G+(a): up / down
                        const u64 *ol = outm + (u64)l * W, *il = inm + (u64)l * W;
                        u32 up = 0, down = 0;
                        for (u32 w2 = 0; w2 < W; w2++) {
                            up += __popcll(oi[w2] & oj[w2] & ol[w2]);
                            down += __popcll(ri[w2] & rj[w2] & il[w2]);
                        }
                        if (up) {
                            tot5 += up;
                            atomicAdd(&acc5[i], (u64)up);
                            atomicAdd(&acc5[j], (u64)up);
                        }
                        if (up + down) atomicAdd(&acc5[l], (u64)(up + down));
                    }
                }
            } else {
                const u32 b = nbr[i];
                const u64 kt_abc = (u64)K4t[r];
                // lists of (b,c), (a,c) and (a,b), each walked forward over increasing d
                TriCursor cbc, cac, cab;
                bool open = false;
                for (u32 w = 0; w < W; w++) {
                    u64 msk = oi[w] & oj[w];
                    while (msk) {
                        u32 l = w * 64 + __ffsll((long long)msk) - 1;
                        msk &= msk - 1;
                        u32 d = nbr[l];
                        if (!open) {
                            cbc.open(arc_find(b, c, out_ptr, out_nbr, st), tri_ptr);
                            cac.open(pa + j, tri_ptr);
                            cab.open(pa + i, tri_ptr);
                            open = true;
                        }
                        tot += (u64)K4t[cbc.find(d, tri_c, st)] - 1;
                        atomicAdd(&acc[i], (u64)K4t[cac.find(d, tri_c, st)] - 1);
                        atomicAdd(&acc[j], (u64)K4t[cab.find(d, tri_c, st)] - 1);
                        atomicAdd(&acc[l], kt_abc - 1);
                    }
                }
            }
        }
        GP::sync();
        u64 t4 = GP::sum(tot, sh_red);
        u64 t5 = pass == 1 ? GP::sum(tot5, sh_red) : 0;
        for (u32 i = GP::rank(); i < D; i += GP::size) {
            u32 v = nbr[i];
            if (pass == 1) {
                u64 h = acc[i] / 2;
                if (h) {
                    u32 s = out_slot[pa + i];
                    atomicAdd(&K4e[s], h);
                    atomicAdd(&K4e[rev[s]], h);
                    atomicAdd(&K4v[v], h);
                }
                atomic_add_u64(&NI(v, 72), acc5[i]);
            } else {
                atomic_add_u64(&NI(v, 70), acc[i]);
            }
        }
        if (GP::rank() == 0) {
            if (pass == 1) {
                atomic_add_u64(&K4v[a], t4 / 3);
                atomic_add_u64(&NI(a, 72), t5);
            } else {
                atomic_add_u64(&NI(a, 70), t4);
            }
        }
        GP::sync();
    }
}

// Orbits 66 and 71 from K4(t): each vertex u of triangle t = {u,v,x} gets
// C(K4(t),2) (orbit 71) and K4(t) (T(v,x) - 2) (orbit 66: the sum over the
// 4-cliques at u of T over the opposite triangle's edges, minus 6, regrouped
// by the triangle that the 4-clique shares with u).
__global__ void k_tri_k4terms(const u32 *src, const u32 *ci, const u32 *T, u64 ntri,
                              const u32 *tri_c, const u32 *tri_sab, const u32 *tri_sac,
                              const u32 *tri_sbc, const u32 *K4t, u64 *ni, const DevState *st) {
    if (st->err) return;
    for (u64 r = GTID; r < ntri; r += GSTRIDE) {
        u64 kt = K4t[r];
        if (!kt) continue;
        u32 sab = tri_sab[r];
        u32 a = src[sab], b = ci[sab], c = tri_c[r];
        u64 q = c2((i64)kt);
        atomic_add_u64(&NI(a, 71), q);
        atomic_add_u64(&NI(b, 71), q);
        atomic_add_u64(&NI(c, 71), q);
        atomic_add_u64(&NI(a, 66), kt * ((u64)T[tri_sbc[r]] - 2));
        atomic_add_u64(&NI(b, 66), kt * ((u64)T[tri_sac[r]] - 2));
        atomic_add_u64(&NI(c, 66), kt * ((u64)T[sab] - 2));
    }
}

// lanes of one wave see each other's LDS and memory writes after this
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// ---- pair sweep over wedges and diamonds (the undirected 2-hop sweep).
// For a source a and every b > a with s = |N(a) & N(b)| >= 2 (pairs with
// s <= 1 contribute to none of these orbits), with S = N(a) & N(b):
//   ta = sum_{y in S} T(a,y),  tb = sum_{y in S} T(y,b),  e = |E(S)|
// (edges inside S, i.e. the diamonds with tips a, b: D(a,b)).  Then
//   pair terms to a (and symmetrically to b), Theorem 5vertexorbit:
//     36: C(s,2)(d(b)-2)    50: C(s,3)    51: (tb - [a~b] s)(s-1)
//     63: e (s-2)
//   centre terms to y in S:  49: C(s-1,2)   62: e
//   chord terms (each diamond with tips a,b and chord (y,z)) to y and z:
//     64: s - 2
//   wheel terms: for y in N(a), K(a,y,b) = |N(a) & N(y) & N(b)| and
//     68: C(K,2) to a and to b;  Q(a,y) = sum_b C(K,2) (orbit 69 of y is half
//     the sum of Q over the arcs into y).
// The remaining subtractions (36: -N13, 51: -2 N12, 62: -N13) happen in the
// per-vertex combine.  a's share tb (s-1) of orbit 51 is summed wedge by
// wedge in the centre pass, T(y,b) (s-1) per wedge a - y - b, once s is
// final, so the wedge pass needs a single atomic per wedge.
// Profiling of the pair sweep: pass_cycles[k-1] accumulates the shader
// clock cycles that execution groups spend in pass k (1 wedges, 2 wheel
// maps, 3 pair terms, 4 centre terms); the group synchronises at each
// boundary so that the pass is complete.
template <class GP>
__device__ inline void pass_mark_g(u64 *pc, int k, u64 &t) {
    GP::sync();
    if (GP::rank() == 0) {
        const u64 now = clock64();
        if (k > 0) atomicAdd(&pc[k - 1], now - t);
        t = now;
    }
}
#define pass_mark(pc, k, t) pass_mark_g<GP>(pc, k, t)

// wheel maps of up to this many positions live in LDS (per wave); in
// workgroup execution groups the four waves' maps together hold one map of
// 6 x PAIR_KMAP_LDS positions for the arcs to larger neighbourhoods
#ifndef PAIR_KMAP_LDS
#define PAIR_KMAP_LDS 2048
#endif
// list entries a lane loads before it uses them (memory-level parallelism)
#ifndef UNR
#define UNR 4
#endif
// The pair sweep's per-vertex results go to a compact accumulator of eight
// words per vertex (one cache line; the combine copies them into the orbit
// columns) rather than into five lines of the 73-word rows.
#define VA_36 0
#define VA_50 1
#define VA_51 2
#define VA_63 3
#define VA_68 4
#define VA_64 5
#define VA_49 6
#define VA_62 7
#define VACC(u, k) vacc[(u64)(u) * 8 + (k)]

// Per-pair state of the source a, indexed by b (within b's graph):
//   sta[b]: bit 63 = [a ~ b].  While d(a) < 2^20, bits 40..62 hold s and
//           bits 0..39 hold ta (s <= d(a) < 2^20 and ta < d(a)^2 < 2^40), so
//           a wedge costs one atomic; for a source of higher degree bits
//           0..62 hold s and ext[b] holds ta.
//   e2[b]:  2 |E(S)|, summed from the wheel maps.
#define PS_ADJ (1ull << 63)
#define PS_SHIFT 40
#define PS_TA_MASK ((1ull << PS_SHIFT) - 1)
#define PS_WIDE_DEG (1u << 20)
// sta and e2 of one b are interleaved in a 16-byte record: the pair terms,
// the centre pass and the wheel drains read both, so each touches one line
// per b instead of two (measured 11 % faster on the Chung-Lu 1M graph).
struct PairState {
    u64 *sta, *e2, *ext;  // e2 = sta + 1
    u32 *touched;
    u32 *K, *tk;  // wave groups only: per-wave global wheel maps, WAVES_PER_WG x n each
    __device__ u64 &s(u32 i) const { return sta[2ull * i]; }
    __device__ u64 &e(u32 i) const { return e2[2ull * i]; }
};
// HBM layout: the records (16 n bytes), ext (8 n), touched (4 n), then in
// wave groups K and tk (4 WAVES_PER_WG n each), each part 256-aligned.
__device__ inline PairState pair_state(unsigned char *base, u32 n, bool wave_maps) {
    PairState p;
    p.sta = (u64 *)base;
    p.e2 = p.sta + 1;
    p.ext = (u64 *)(base + 2 * ((8ull * n + 255) & ~255ull));
    p.touched = (u32 *)align256((unsigned char *)(p.ext + n));
    p.K = wave_maps ? (u32 *)align256((unsigned char *)(p.touched + n)) : nullptr;
    p.tk = wave_maps ? (u32 *)align256((unsigned char *)(p.K + (u64)WAVES_PER_WG * n)) : nullptr;
    return p;
}
__device__ inline u64 ps_s(u64 v, bool wide) {
    return wide ? (v & ~PS_ADJ) : ((v & ~PS_ADJ) >> PS_SHIFT);
}

// Drain of one wheel-map entry: K = K(a,y,b) for the b at position pos of
// N(y) (slot by + pos).  Returns C(K,2) and adds K (s(a,b) - 2) to c64.
__device__ inline u64 wheel_drain(u32 kab, u32 b, u32 vb, const PairState &P, bool wide,
                                  u64 *vacc, u64 &c64) {
    const u64 v = c2((i64)kab);
    atomic_add_u64(&VACC(b, VA_68), v);
    atomicAdd(&P.e(b - vb), (u64)kab);
    c64 += (u64)kab * (ps_s(P.s(b - vb), wide) - 2);
    return v;
}

// Flat walk over up to 64 list parts held by the lanes of a wave: lane k
// holds part k (n_k entries, and whatever the caller stores for it in the
// wave's FlatLds).  The wave runs through the flat indices f = lane + 64 i,
// UNR per lane per step, so a long part is read with coalesced loads and
// short parts are read in parallel by different lanes -- a lane never waits
// for one list to end before loading from the next.  F(jv, ov, valid)
// receives UNR (part, offset) pairs; the parts of one lane only increase.
struct FlatLds {
    u32 pre[WAVE + 1];  // exclusive prefix sums of n_k; pre[64] = total
    u32 aux[WAVE];      // per part: caller data
    u64 ptr[WAVE];      // per part: caller data (a list base address)
};
template <typename F>
__device__ inline void flat_walk(FlatLds &L, u32 n_mine, F f) {
    const u32 lane = lane_id();
    u32 x = n_mine;
    for (int off = 1; off < WAVE; off <<= 1) {
        const u32 t = __shfl_up(x, off, WAVE);
        if ((int)lane >= off) x += t;
    }
    L.pre[lane + 1] = x;
    if (lane == 0) L.pre[0] = 0;
    const u32 total = __shfl(x, WAVE - 1, WAVE);
    wave_sync();
    u32 j = 0;
    for (u32 f0 = lane; f0 < total; f0 += UNR * WAVE) {
        u32 jv[UNR], ov[UNR];
        bool ok[UNR];
#pragma unroll
        for (int k = 0; k < UNR; k++) {
            const u32 fk = f0 + k * WAVE;
            ok[k] = fk < total;
            if (ok[k]) {
                while (fk >= L.pre[j + 1]) j++;
                jv[k] = j;
                ov[k] = fk - L.pre[j];
            }
        }
        f(jv, ov, ok);
    }
    wave_sync();
}

// LM: the pair state (sta, e2, touched) lives in LDS, lmw words per wave
// after the wheel maps (then every arc's wheel map is an LDS one).
template <class GP, bool LM>
__global__ void __launch_bounds__(WG) k_pairs(const u32 *rp, const u32 *ci, const u32 *src,
                                             const u32 *rev, const u32 *deg, const u32 *T,
                                             const u64 *tl_ptr, const uint2 *tl, u32 n,
                                             unsigned char *scratch, u64 stride, u32 *work,
                                             const u32 *order, u32 mapn, const u32 *gbase,
                                             u32 kl, u64 lmw, u64 *steps, u64 *pass_cycles,
                                             u64 *Q, u64 *vacc, const DevState *st) {
    constexpr bool kWaveGroups = GP::per_wg > 1;
    static_assert(!LM || kWaveGroups, "LDS maps are per wave");
    __shared__ u32 sh_q_[GP::per_wg][3], sh_nt_[GP::per_wg], sh_next_[GP::per_wg];
    u32 *sh_q = sh_q_[GP::id()];
    if (GP::rank() == 0) { sh_q[0] = 0; sh_q[1] = 0; }
    u32 &sh_nt = sh_nt_[GP::id()];
    u32 &sh_next = sh_next_[GP::id()];
    __shared__ u32 sh_ntk[WAVES_PER_WG];
    __shared__ u64 sh_red[WAVES_PER_WG];
    __shared__ u32 sh_hub[WG], sh_nhub;  // workgroup groups: this chunk's arcs to hubs
    __shared__ FlatLds sh_flat[WAVES_PER_WG];
    FlatLds &FL = sh_flat[wave_in_wg()];
    // per-arc centre sums of the flat walk (wave groups only; a token size
    // otherwise: three workgroups of hub wheel maps fill a CU's LDS)
    __shared__ u64 sh_cen[kWaveGroups ? WAVES_PER_WG : 1][2][kWaveGroups ? WAVE : 1];
    // dynamic LDS: per-wave wheel maps of kl positions (u32) and touched
    // lists (u16), kl <= PAIR_KMAP_LDS; in workgroup groups the same bytes
    // also serve as one map of hmax = 6 kl positions for the hub arcs
    extern __shared__ u64 dyn_lds[];
    u32 *l_k0 = (u32 *)dyn_lds;
    unsigned short *l_tk0 = (unsigned short *)(l_k0 + WAVES_PER_WG * kl);
    u32 *hmap = l_k0;
    const u32 hmax = 6 * kl;
    PairState P;
    u32 *Kw = nullptr, *tkw = nullptr;
    if constexpr (LM) {
        if (mapn > kl) {  // the launch must give every arc an LDS wheel map
            if (threadIdx.x == 0) atomicOr((u32 *)&st->err, ERRB_INTERNAL);
            return;
        }
        u64 *maps = dyn_lds + 3ull * kl;  // after the wheel maps (24 kl bytes)
        clear_lds(maps, WAVES_PER_WG * lmw);
        P.sta = wave_lds_slice(maps, lmw);
        P.e2 = P.sta + 1;
        P.ext = P.e2;  // wide sources cannot occur in maps this small
        P.touched = (u32 *)(P.sta + 2ull * mapn);
        P.K = P.tk = nullptr;
    } else {
        P = pair_state(scratch + GP::global_id() * stride, mapn, kWaveGroups);
        Kw = kWaveGroups ? P.K + (u64)wave_in_wg() * mapn : nullptr;
        tkw = kWaveGroups ? P.tk + (u64)wave_in_wg() * mapn : nullptr;
    }
    const u32 lane = lane_id();
    // every thread of the workgroup clears its share, then all wait (the
    // slices belong to different waves)
    for (u32 i = threadIdx.x; i < hmax; i += WG) hmap[i] = 0;
    if (threadIdx.x == 0) sh_nhub = 0;
    __syncthreads();
    for (;;) {
        const u32 a = next_source<GP>(work, sh_q, order, n, st);
        if (a >= n) break;
        const u32 vb = gbase ? gbase[a] : 0;  // maps are indexed within a's graph
        const u32 ba = rp[a], da = rp[a + 1] - ba;
        if (da < 2) continue;
        const u64 dega = da;
        const bool wide = !LM && da >= PS_WIDE_DEG;
        u64 nsteps = 0;  // loop iterations of this thread for this source
        u64 t_pass = 0;  // clock at the last pass boundary (profiling)
        for (u32 i = GP::rank(); i < da; i += GP::size) P.s(ci[ba + i] - vb) = PS_ADJ;
        if (GP::rank() == 0) { sh_nt = 0; sh_next = 0; }
        GP::sync();
        if (pass_cycles) pass_mark(pass_cycles, 0, t_pass);
        // wedges a - y - b, b > a: s and ta of the pair (a, b); UNR entries
        // per lane per step, whose loads and atomics are independent.  A
        // wave with a light source (d(a) <= 64) walks all its arcs' lists
        // at once, one list per lane, instead of one arc after another.
        const bool flat = kWaveGroups && da <= WAVE;
        if (flat) {
            u32 cnt = 0;
            if (lane < da) {
                const u32 y = ci[ba + lane];
                const u32 by = rp[y], ey = rp[y + 1];
                const u32 st0 = by + lbound(ci + by, ey - by, a + 1);
                cnt = ey - st0;
                FL.ptr[lane] = st0;
                FL.aux[lane] = T[ba + lane];
            }
            flat_walk(FL, cnt, [&](const u32 *jv, const u32 *ov, const bool *ok) {
                u32 bv[UNR];
                u64 old[UNR];
#pragma unroll
                for (int k = 0; k < UNR; k++) bv[k] = ok[k] ? ci[(u32)FL.ptr[jv[k]] + ov[k]] : UNSET;
#pragma unroll
                for (int k = 0; k < UNR; k++)
                    if (bv[k] != UNSET)
                        old[k] = atomicAdd(&P.s(bv[k] - vb), (1ull << PS_SHIFT) | FL.aux[jv[k]]);
#pragma unroll
                for (int k = 0; k < UNR; k++)
                    if (bv[k] != UNSET) {
                        nsteps++;
                        if (((old[k] & ~PS_ADJ) >> PS_SHIFT) == 0)
                            P.touched[atomicAdd(&sh_nt, 1u)] = bv[k];
                    }
            });
        } else wave_loop(&sh_next, da, [&](u32 iy) {
            const u32 say = ba + iy, y = ci[say];
            const u64 tay = T[say];
            const u32 by = rp[y], ey = rp[y + 1];
            const u32 st0 = by + lbound(ci + by, ey - by, a + 1);
            for (u32 s0 = st0 + lane; s0 < ey; s0 += UNR * WAVE) {
                u32 bv[UNR];
                u64 old[UNR];
#pragma unroll
                for (int k = 0; k < UNR; k++) {
                    const u32 s = s0 + k * WAVE;
                    bv[k] = s < ey ? ci[s] : UNSET;
                }
                if (!wide) {
#pragma unroll
                    for (int k = 0; k < UNR; k++)
                        if (bv[k] != UNSET)
                            old[k] = atomicAdd(&P.s(bv[k] - vb), (1ull << PS_SHIFT) | tay);
#pragma unroll
                    for (int k = 0; k < UNR; k++) old[k] = (old[k] & ~PS_ADJ) >> PS_SHIFT;
                } else {
#pragma unroll
                    for (int k = 0; k < UNR; k++)
                        if (bv[k] != UNSET) {
                            old[k] = atomicAdd(&P.s(bv[k] - vb), 1ull) & ~PS_ADJ;
                            atomicAdd(&P.ext[bv[k] - vb], tay);
                        }
                }
#pragma unroll
                for (int k = 0; k < UNR; k++)
                    if (bv[k] != UNSET) {
                        nsteps++;
                        if (old[k] == 0) P.touched[atomicAdd(&sh_nt, 1u)] = bv[k];
                    }
            }
        });
        GP::sync();
        if (GP::rank() == 0) sh_next = 0;
        GP::sync();
        if (pass_cycles) pass_mark(pass_cycles, 1, t_pass);
        // wheel maps of the arcs (a, y): K(a,y,b) = |N(a) & N(y) & N(b)| for
        // b > a, from the diamonds with tip a and chord (y,z) (z in the
        // triangle list of (a,y), b in the list of (y,z), which is sorted by
        // third vertex so the part with b > a is found by binary search).
        // Draining a map gives orbit 68 (C(K,2) to a and b), Q(a,y), the
        // doubled inner edge count E2(a,b) = sum_y K(a,y,b) = 2 |E(S)|, and
        // the chord terms of orbit 64: y gets K(a,y,b) (s(a,b) - 2), i.e.
        // s - 2 per diamond with chord (y,z) -- z gets its share when it is
        // the arc's end.  The map of (a, y) is indexed by b's position in
        // N(y): a wave's LDS map when d(y) <= kl; else, in workgroup groups,
        // the whole group's LDS map in windows of hmax positions (below), and
        // in wave groups the wave's global map.  The lists (y,z) of 64 z at
        // a time are walked flat.
        if (lane == 0) sh_ntk[wave_in_wg()] = 0;
        u64 l68 = 0;
        wave_loop(&sh_next, da, [&](u32 iy) {
            const u32 say = ba + iy, y = ci[say];
            if (T[say] == 0) return;
            const u32 by = rp[y], dy = rp[y + 1] - by;
            const bool inl = LM || dy <= kl;  // with LM, dy < mapn <= kl (checked at the start)
            if (!inl && !kWaveGroups) return;  // a hub arc: the whole group, below
            u32 *kc = inl ? l_k0 + wave_in_wg() * kl : Kw;
            unsigned short *tl_l = l_tk0 + wave_in_wg() * kl;
            TLView tv = tl_view(say, src, ci, rev, T, tl_ptr, tl);
            u32 *ntk = &sh_ntk[wave_in_wg()];
            // b > a  <=>  slot(y,b) >= ya, the first slot of N(y) above a
            const u32 ya = by + lbound(ci + by, dy, a + 1);
            for (u32 k0 = 0; k0 < tv.len; k0 += WAVE) {
                // each lane locates the part b > a of one list (y,z) ...
                const u32 kk = k0 + lane;
                u32 cnt = 0;
                if (kk < tv.len) {
                    const uint2 ez = tv.get(kk);  // (slot(a,z), slot(y,z))
                    const TLView tw = tl_view(ez.y, src, ci, rev, T, tl_ptr, tl);
                    u32 lo = 0, hi = tw.len;
                    while (lo < hi) {
                        const u32 mid = (lo + hi) >> 1;
                        if (tw.get(mid).x < ya) lo = mid + 1; else hi = mid;
                    }
                    cnt = tw.len - lo;
                    FL.ptr[lane] = (u64)(tw.p + lo);
                    FL.aux[lane] = tw.swap;
                }
                // ... then the wave walks those parts flat
                flat_walk(FL, cnt, [&](const u32 *jv, const u32 *ov, const bool *ok) {
                    uint2 ev[UNR];
#pragma unroll
                    for (int k = 0; k < UNR; k++)
                        if (ok[k]) ev[k] = ((const uint2 *)FL.ptr[jv[k]])[ov[k]];
#pragma unroll
                    for (int k = 0; k < UNR; k++) {
                        if (!ok[k]) continue;
                        const u32 pos = (FL.aux[jv[k]] ? ev[k].y : ev[k].x) - by;  // slot(y,b) - rp[y]
                        nsteps++;
                        const u32 old = atomicAdd(&kc[pos], 1u);
                        if (old == 0) {
                            const u32 t = atomicAdd(ntk, 1u);
                            if (inl) tl_l[t] = (unsigned short)pos; else tkw[t] = pos;
                        }
                    }
                });
            }
            wave_sync();
            const u32 m = *ntk;
            u64 q = 0, c64 = 0;
            for (u32 t = lane; t < m; t += WAVE) {
                const u32 pos = inl ? (u32)tl_l[t] : tkw[t];
                const u32 kab = atomicExch(&kc[pos], 0u);
                q += wheel_drain(kab, ci[by + pos], vb, P, wide, vacc, c64);
            }
            q = wave_sum_u64(q);
            c64 = wave_sum_u64(c64);
            if (lane == 0) {
                Q[say] = q;
                atomic_add_u64(&VACC(y, VA_64), c64);
                *ntk = 0;
            }
            l68 += q;
            wave_sync();
        });
        GP::sync();
        if (!kWaveGroups) {
            // arcs to hubs (d(y) > kl), one at a time by the whole group, in
            // windows of hmax positions of N(y): the lists (y,z) are sorted by
            // position, so a window is a sub-range of each, found by binary
            // search; a window is drained by a scan of its positions
            for (u32 c0 = 0; c0 < da; c0 += WG) {
                const u32 i = c0 + threadIdx.x;
                if (i < da) {
                    const u32 y = ci[ba + i];
                    if (T[ba + i] > 0 && rp[y + 1] - rp[y] > kl) sh_hub[atomicAdd(&sh_nhub, 1u)] = i;
                }
                __syncthreads();
                const u32 nh = sh_nhub;
                if (nh) {  // the touched lists' bytes become map positions: clear them
                    for (u32 w = threadIdx.x; w < WAVES_PER_WG * kl / 2; w += WG)
                        l_k0[WAVES_PER_WG * kl + w] = 0;
                    __syncthreads();
                }
                for (u32 h = 0; h < nh; h++) {
                    const u32 say = ba + sh_hub[h], y = ci[say];
                    const u32 by = rp[y], dy = rp[y + 1] - by;
                    const TLView tv = tl_view(say, src, ci, rev, T, tl_ptr, tl);
                    const u32 p0 = lbound(ci + by, dy, a + 1);  // first position with b > a
                    const u32 nbatch = (tv.len + WAVE - 1) / WAVE;
                    u64 q = 0, c64 = 0;
                    for (u32 w0 = p0; w0 < dy; w0 += hmax) {
                        const u32 w1 = dy - w0 < hmax ? dy : w0 + hmax;
                        if (threadIdx.x == 0) sh_next = 0;
                        __syncthreads();
                        wave_loop(&sh_next, nbatch, [&](u32 bi) {
                            const u32 kk = bi * WAVE + lane;
                            u32 cnt = 0;
                            if (kk < tv.len) {
                                const uint2 ez = tv.get(kk);  // (slot(a,z), slot(y,z))
                                const TLView tw = tl_view(ez.y, src, ci, rev, T, tl_ptr, tl);
                                // entries with position in [w0, w1)
                                u32 l = 0, r = tw.len;
                                while (l < r) {
                                    const u32 mid = (l + r) >> 1;
                                    if (tw.get(mid).x < by + w0) l = mid + 1; else r = mid;
                                }
                                const u32 lo = l;
                                r = tw.len;
                                if (w1 < dy) {
                                    while (l < r) {
                                        const u32 mid = (l + r) >> 1;
                                        if (tw.get(mid).x < by + w1) l = mid + 1; else r = mid;
                                    }
                                }
                                cnt = r - lo;
                                FL.ptr[lane] = (u64)(tw.p + lo);
                                FL.aux[lane] = tw.swap;
                            }
                            flat_walk(FL, cnt, [&](const u32 *jv, const u32 *ov, const bool *ok) {
                                uint2 ev[UNR];
#pragma unroll
                                for (int k = 0; k < UNR; k++)
                                    if (ok[k]) ev[k] = ((const uint2 *)FL.ptr[jv[k]])[ov[k]];
#pragma unroll
                                for (int k = 0; k < UNR; k++)
                                    if (ok[k]) {
                                        nsteps++;
                                        atomicAdd(&hmap[(FL.aux[jv[k]] ? ev[k].y : ev[k].x) - by - w0], 1u);
                                    }
                            });
                        });
                        __syncthreads();
                        for (u32 p = threadIdx.x; p < w1 - w0; p += WG) {
                            const u32 kab = hmap[p];
                            if (!kab) continue;
                            hmap[p] = 0;
                            q += wheel_drain(kab, ci[by + w0 + p], vb, P, wide, vacc, c64);
                        }
                        __syncthreads();
                    }
                    q = GP::sum(q, sh_red);
                    c64 = GP::sum(c64, sh_red);
                    if (threadIdx.x == 0) {
                        Q[say] = q;
                        atomic_add_u64(&VACC(y, VA_64), c64);
                    }
                    if (wave_in_wg() == 0) l68 += q;
                }
                __syncthreads();
                if (threadIdx.x == 0) sh_nhub = 0;
                __syncthreads();
            }
        }
        // l68 is uniform within each wave (computed from wave or group sums)
        if (lane == 0) atomic_add_u64(&VACC(a, VA_68), l68);
        if (pass_cycles) pass_mark(pass_cycles, 2, t_pass);
        // pair terms (e2 holds 2 e); a's tb (s-1) comes in the centre pass
        const u32 nt = sh_nt;
        u64 l36 = 0, l50 = 0, l51 = 0, l63 = 0;
        for (u32 t = GP::rank(); t < nt; t += GP::size) {
            const u32 b = P.touched[t];
            const u64 v = P.s(b - vb);
            const u64 s = ps_s(v, wide);
            if (s < 2) continue;
            const u64 adj = v >> 63;
            const u64 ta = wide ? P.ext[b - vb] : (v & PS_TA_MASK);
            const u64 e = P.e(b - vb) >> 1;
            const u64 cs2 = c2((i64)s), cs3 = c3((i64)s);
            l36 += cs2 * ((u64)deg[b] - 2);
            l50 += cs3;
            l51 -= adj * s * (s - 1);
            l63 += e * (s - 2);
            atomic_add_u64(&VACC(b, VA_36), cs2 * (dega - 2));
            atomic_add_u64(&VACC(b, VA_50), cs3);
            atomic_add_u64(&VACC(b, VA_51), (ta - adj * s) * (s - 1));
            atomic_add_u64(&VACC(b, VA_63), e * (s - 2));
        }
        l36 = GP::sum(l36, sh_red);
        l50 = GP::sum(l50, sh_red);
        l63 = GP::sum(l63, sh_red);
        if (GP::rank() == 0) {
            atomic_add_u64(&VACC(a, VA_36), l36);
            atomic_add_u64(&VACC(a, VA_50), l50);
            atomic_add_u64(&VACC(a, VA_63), l63);
            sh_next = 0;
        }
        GP::sync();
        if (pass_cycles) pass_mark(pass_cycles, 3, t_pass);
        // centre terms, and a's tb (s-1) wedge by wedge (light sources of
        // wave groups: all arcs at once, per-arc sums in LDS)
        if (flat) {
            u32 cnt = 0;
            u64 *c49 = sh_cen[wave_in_wg()][0], *c62 = sh_cen[wave_in_wg()][1];
            c49[lane] = 0;
            c62[lane] = 0;
            if (lane < da) {
                const u32 y = ci[ba + lane];
                const u32 by = rp[y], ey = rp[y + 1];
                const u32 st0 = by + lbound(ci + by, ey - by, a + 1);
                cnt = ey - st0;
                FL.ptr[lane] = st0;
            }
            flat_walk(FL, cnt, [&](const u32 *jv, const u32 *ov, const bool *ok) {
                u32 bv[UNR];
                u64 tv[UNR], sv[UNR], ev2[UNR];
#pragma unroll
                for (int k = 0; k < UNR; k++) {
                    const u32 s = ok[k] ? (u32)FL.ptr[jv[k]] + ov[k] : 0;
                    bv[k] = ok[k] ? ci[s] : UNSET;
                    tv[k] = ok[k] ? T[s] : 0;
                }
#pragma unroll
                for (int k = 0; k < UNR; k++)
                    if (bv[k] != UNSET) {
                        sv[k] = P.s(bv[k] - vb);
                        ev2[k] = P.e(bv[k] - vb);
                    }
#pragma unroll
                for (int k = 0; k < UNR; k++) {
                    if (bv[k] == UNSET) continue;
                    const u64 sb = ps_s(sv[k], wide);
                    nsteps++;
                    if (sb >= 2) {
                        atomicAdd(&c49[jv[k]], c2((i64)sb - 1));
                        atomicAdd(&c62[jv[k]], ev2[k] >> 1);
                        l51 += tv[k] * (sb - 1);
                    }
                }
            });
            if (lane < da) {
                const u32 y = ci[ba + lane];
                atomic_add_u64(&VACC(y, VA_49), c49[lane]);
                atomic_add_u64(&VACC(y, VA_62), c62[lane]);
            }
        } else wave_loop(&sh_next, da, [&](u32 iy) {
            const u32 say = ba + iy, y = ci[say];
            const u32 by = rp[y], ey = rp[y + 1];
            const u32 st0 = by + lbound(ci + by, ey - by, a + 1);
            u64 a49 = 0, a62 = 0;
            for (u32 s0 = st0 + lane; s0 < ey; s0 += UNR * WAVE) {
                u32 bv[UNR];
                u64 tv[UNR], sv[UNR], ev2[UNR];
#pragma unroll
                for (int k = 0; k < UNR; k++) {
                    const u32 s = s0 + k * WAVE;
                    bv[k] = s < ey ? ci[s] : UNSET;
                    tv[k] = s < ey ? T[s] : 0;
                }
#pragma unroll
                for (int k = 0; k < UNR; k++)
                    if (bv[k] != UNSET) {
                        sv[k] = P.s(bv[k] - vb);
                        ev2[k] = P.e(bv[k] - vb);
                    }
#pragma unroll
                for (int k = 0; k < UNR; k++) {
                    if (bv[k] == UNSET) break;
                    const u64 sb = ps_s(sv[k], wide);
                    nsteps++;
                    if (sb >= 2) {
                        a49 += c2((i64)sb - 1);
                        a62 += ev2[k] >> 1;
                        l51 += tv[k] * (sb - 1);
                    }
                }
            }
            a49 = wave_sum_u64(a49);
            a62 = wave_sum_u64(a62);
            if (lane == 0) {
                atomic_add_u64(&VACC(y, VA_49), a49);
                atomic_add_u64(&VACC(y, VA_62), a62);
            }
        });
        l51 = GP::sum(l51, sh_red);
        if (GP::rank() == 0) atomic_add_u64(&VACC(a, VA_51), l51);
        GP::sync();
        for (u32 t = GP::rank(); t < nt; t += GP::size) {
            const u32 b = P.touched[t];
            P.s(b - vb) = 0;
            P.e(b - vb) = 0;
            if (wide) P.ext[b - vb] = 0;
        }
        for (u32 i = GP::rank(); i < da; i += GP::size) P.s(ci[ba + i] - vb) = 0;
        if (pass_cycles) pass_mark(pass_cycles, 4, t_pass);
        if (steps) {  // per-source work, the training target of the scheduler
            u64 tot = GP::sum(nsteps, sh_red);
            if (GP::rank() == 0) atomic_add_u64(&steps[a], tot);  // the 5-cycle kernel may run alongside
        }
        GP::sync();
    }
}

// ---- 5-cycles (orbit 34): the procedure of the 5-cycle theorem.  Every
// 5-cycle has exactly one directed 3-path i <- j <- k -> l whose closing
// wedge i - w - l is not in-in (not both i->w and l->w).  For a source l:
//   W(i) = non-in-in wedges between l and i,  P(i) = directed 3-paths
//   from i to l.  Each 3-path credits i, j, k, l with
//   W(i) - [i~k] - [j~l] (removing w = k and w = j), and each non-in-in
//   wedge l - w - i credits w with P(i) minus the tailed triangles
//   (Fig. TaileTri): [w->i] Tin(w,l) + [w->l][w->i] (Tmid(w->i) - [l->i]).
// The sums over 3-paths are grouped by their middle vertex j instead of
// walking every path: with c(j) = |{k : k -> l, k -> j}| (j != l),
//   P(i)  = sum over j -> i, j != l, of c(j)                     (i != l)
//   CI(i) = sum of the corrections [k->i] + [j~l] over the paths to i
//         = sum_{k -> i, k -> l} (Tmid(k->i) - [l->i]) + sum_{j -> i} c(j) [j~l]
//           (the j with k -> j -> i are counted by Tmid of the arc k -> i)
//   credit of j = c(j) (SW(j) - d'(j) [j~l]) - sum_{k -> j, k -> l} (Tout(k->j) - [j->l])
//   credit of k = sum_{j in N+(k), j != l} (SW(j) - d'(j) [j~l] - Tout(k->j) + [j->l])
// with SW(j) = sum of W(i) over i in N+(j) \ {l}, d'(j) = |N+(j) \ {l}| and
// Tout(k->j) = |N+(k) & N+(j)| = T - Tin - Tmid of the arc (i in N+(j) with
// also k -> i is a triangle above both).  The work per source drops from
// the number of 3-paths to the out-lists of the distinct middle vertices.
struct C5Scratch {
    u32 *Wm, *C, *touched, *jt;
    u64 *P, *CI, *TO, *SW;
    unsigned char *mark;
};
// Per-list values and sums of a wave's flat walks over a light source's
// lists (wave groups).
struct C5Flat {
    u64 acc[WAVE], acc2[WAVE], kw[WAVE];
    u32 tin[WAVE], cnt[WAVE];
};
// Layout (each array 256-aligned): Wm, P, CI | touched | mark | C, TO, SW | jt.
// The first, third and fourth groups must be zero when a source starts.
__device__ inline C5Scratch c5_scratch(unsigned char *base, u32 n) {
    C5Scratch c;
    c.Wm = (u32 *)base;
    c.P = (u64 *)align256((unsigned char *)(c.Wm + n));
    c.CI = (u64 *)align256((unsigned char *)(c.P + n));
    c.touched = (u32 *)align256((unsigned char *)(c.CI + n));
    c.mark = align256((unsigned char *)(c.touched + n));
    c.C = (u32 *)align256(c.mark + n);
    c.TO = (u64 *)align256((unsigned char *)(c.C + n));
    c.SW = (u64 *)align256((unsigned char *)(c.TO + n));
    c.jt = (u32 *)align256((unsigned char *)(c.SW + n));
    return c;
}

template <class GP>
__global__ void __launch_bounds__(WG) k_c5(const u32 *rp, const u32 *ci, const u64 *key,
                                          const u64 *out_ptr, const u32 *out_nbr,
                                          const u32 *out_slot, const u32 *T, const u32 *Tin,
                                          const u32 *Tmid, u32 n, unsigned char *scratch,
                                          u64 stride, u32 *work, const u32 *order, u32 mapn,
                                          const u32 *gbase, u64 *steps, u64 *cacc,
                                          const DevState *st) {
    __shared__ u32 sh_q_[GP::per_wg][3], sh_nt_[GP::per_wg], sh_nj_[GP::per_wg],
        sh_next_[GP::per_wg];
    u32 *sh_q = sh_q_[GP::id()];
    if (GP::rank() == 0) { sh_q[0] = 0; sh_q[1] = 0; }
    u32 &sh_nt = sh_nt_[GP::id()];
    u32 &sh_nj = sh_nj_[GP::id()];
    u32 &sh_next = sh_next_[GP::id()];
    __shared__ u64 sh_red[WAVES_PER_WG];
    C5Scratch C = c5_scratch(scratch + GP::global_id() * stride, mapn);
    const u32 lane = lane_id();
    // light sources of wave groups walk all their lists at once (one list
    // per lane, flat), with per-list values and sums in LDS
    constexpr bool kWaveGroups = GP::per_wg > 1;
    constexpr u32 kF = kWaveGroups ? WAVES_PER_WG : 1;
    __shared__ FlatLds sh_flat[kF];
    __shared__ C5Flat sh_c5f[kF];
    FlatLds &FL = sh_flat[kWaveGroups ? wave_in_wg() : 0];
    C5Flat &F = sh_c5f[kWaveGroups ? wave_in_wg() : 0];
    for (;;) {
        const u32 l = next_source<GP>(work, sh_q, order, n, st);
        if (l >= n) break;
        const u32 vb = gbase ? gbase[l] : 0;  // maps are indexed within l's graph
        const u32 bl = rp[l], dl = rp[l + 1] - bl;
        if (dl < 2) continue;
        const u64 kl = key[l];
        u64 nsteps = 0;  // loop iterations of this thread for this source
        const bool flat = kWaveGroups && dl <= WAVE;
        for (u32 i = GP::rank(); i < dl; i += GP::size) C.mark[ci[bl + i] - vb] = 1;
        if (GP::rank() == 0) { sh_nt = 0; sh_nj = 0; sh_next = 0; }
        GP::sync();
        // pass 1: non-in-in wedges l - w - i; for every in-neighbour k of l,
        // each out-arc k -> x (x != l): c(x), the Tout part of x's credit,
        // and the Tmid part of CI(x)
        if (flat) {
            u32 w = 0, cnt = 0;
            u64 kw = 0;
            if (lane < dl) {  // the wedge ends of w: N+(w) if l -> w, else N(w)
                w = ci[bl + lane];
                kw = key[w];
                const u64 b = kw > kl ? out_ptr[w] : rp[w];
                cnt = (u32)((kw > kl ? out_ptr[w + 1] : (u64)rp[w + 1]) - b);
                FL.ptr[lane] = (u64)((kw > kl ? out_nbr : ci) + b);
            }
            flat_walk(FL, cnt, [&](const u32 *jv, const u32 *ov, const bool *ok) {
                u32 iv[UNR];
#pragma unroll
                for (int k = 0; k < UNR; k++) iv[k] = ok[k] ? ((const u32 *)FL.ptr[jv[k]])[ov[k]] : l;
#pragma unroll
                for (int k = 0; k < UNR; k++)
                    if (ok[k]) {
                        nsteps++;
                        if (iv[k] != l) atomicAdd(&C.Wm[iv[k] - vb], 1u);
                    }
            });
            cnt = 0;
            if (lane < dl && kw < kl) {  // w -> l: w plays k, its out-arcs k -> x
                cnt = (u32)(out_ptr[w + 1] - out_ptr[w]);
                FL.ptr[lane] = out_ptr[w];
            }
            flat_walk(FL, cnt, [&](const u32 *jv, const u32 *ov, const bool *ok) {
#pragma unroll
                for (int k = 0; k < UNR; k++) {
                    if (!ok[k]) continue;
                    const u64 q = FL.ptr[jv[k]] + ov[k];
                    const u32 x = out_nbr[q];
                    nsteps++;
                    if (x == l) continue;
                    const u32 sq = out_slot[q];
                    const u32 ts = T[sq], ti = Tin[sq], tm = Tmid[sq];
                    const bool adj = C.mark[x - vb] != 0;
                    const u64 kx = key[x];
                    const u32 xl = adj && kx < kl, lx = adj && kx > kl;  // x -> l, l -> x
                    if (atomicAdd(&C.C[x - vb], 1u) == 0) C.jt[atomicAdd(&sh_nj, 1u)] = x;
                    const u64 to = (u64)(ts - ti - tm) - xl;
                    if (to) atomicAdd(&C.TO[x - vb], to);
                    const u64 cm = (u64)tm - lx;
                    if (cm) atomicAdd(&C.CI[x - vb], cm);
                }
            });
        } else wave_loop(&sh_next, dl, [&](u32 iw) {
            const u32 w = ci[bl + iw];
            if (key[w] > kl) {  // l -> w, then w -> i
                for (u64 q = out_ptr[w] + lane; q < out_ptr[w + 1]; q += WAVE) {
                    atomicAdd(&C.Wm[out_nbr[q] - vb], 1u);
                    nsteps++;
                }
                return;
            }
            // w -> l, then any i ~ w
            for (u32 s = rp[w] + lane; s < rp[w + 1]; s += WAVE) {
                const u32 i = ci[s];
                if (i != l) atomicAdd(&C.Wm[i - vb], 1u);
                nsteps++;
            }
            const u32 k = w;
            for (u64 q = out_ptr[k] + lane; q < out_ptr[k + 1]; q += WAVE) {
                const u32 x = out_nbr[q];
                nsteps++;
                if (x == l) continue;
                const u32 s = out_slot[q];
                const u32 ts = T[s], ti = Tin[s], tm = Tmid[s];
                const bool adj = C.mark[x - vb] != 0;
                const u64 kx = key[x];
                const u32 xl = adj && kx < kl, lx = adj && kx > kl;  // x -> l, l -> x
                if (atomicAdd(&C.C[x - vb], 1u) == 0) C.jt[atomicAdd(&sh_nj, 1u)] = x;
                const u64 to = (u64)(ts - ti - tm) - xl;
                if (to) atomicAdd(&C.TO[x - vb], to);
                const u64 cm = (u64)tm - lx;
                if (cm) atomicAdd(&C.CI[x - vb], cm);
            }
        });
        GP::sync();
        if (GP::rank() == 0) sh_next = 0;
        GP::sync();
        // pass 1b: every middle vertex j reached: P(i) += c(j) and
        // CI(i) += c(j) [j~l] for i in N+(j) \ {l}; SW(j); credit of j
        const u32 nj = sh_nj;
        if (flat) {  // 64 middle vertices at a time, one out-list per lane
            for (u32 t0 = 0; t0 < nj; t0 += WAVE) {
                const u32 t = t0 + lane;
                u32 j = 0, cnt = 0;
                u64 cj = 0;
                bool mj = false;
                F.acc[lane] = 0;
                F.cnt[lane] = 0;
                if (t < nj) {
                    j = C.jt[t];
                    cj = C.C[j - vb];
                    mj = C.mark[j - vb] != 0;
                    FL.ptr[lane] = out_ptr[j];
                    FL.aux[lane] = (u32)cj | (mj ? 0x80000000u : 0u);  // c(j) <= d(l) < 2^31
                    cnt = (u32)(out_ptr[j + 1] - out_ptr[j]);
                }
                flat_walk(FL, cnt, [&](const u32 *jv, const u32 *ov, const bool *ok) {
#pragma unroll
                    for (int k = 0; k < UNR; k++) {
                        if (!ok[k]) continue;
                        const u32 i = out_nbr[FL.ptr[jv[k]] + ov[k]];
                        nsteps++;
                        if (i == l) continue;
                        const u32 aux = FL.aux[jv[k]];
                        const u64 cjk = aux & 0x7fffffffu;
                        if (atomicAdd(&C.P[i - vb], cjk) == 0) C.touched[atomicAdd(&sh_nt, 1u)] = i;
                        if (aux >> 31) atomicAdd(&C.CI[i - vb], cjk);
                        atomicAdd(&F.acc[jv[k]], (u64)C.Wm[i - vb]);
                        atomicAdd(&F.cnt[jv[k]], 1u);
                    }
                });
                if (t < nj) {
                    const u64 sw = F.acc[lane], dj = F.cnt[lane];
                    C.SW[j - vb] = sw;
                    atomic_add_u64(&cacc[j], cj * (sw - (mj ? dj : 0)) - C.TO[j - vb]);
                }
                wave_sync();
            }
        } else wave_loop(&sh_next, nj, [&](u32 t) {
            const u32 j = C.jt[t];
            const u64 cj = C.C[j - vb];
            const bool mj = C.mark[j - vb] != 0;
            u64 sw = 0, dj = 0;
            for (u64 q = out_ptr[j] + lane; q < out_ptr[j + 1]; q += WAVE) {
                const u32 i = out_nbr[q];
                nsteps++;
                if (i == l) continue;
                if (atomicAdd(&C.P[i - vb], cj) == 0) C.touched[atomicAdd(&sh_nt, 1u)] = i;
                if (mj) atomicAdd(&C.CI[i - vb], cj);
                sw += C.Wm[i - vb];
                dj++;
            }
            sw = wave_sum_u64(sw);
            dj = wave_sum_u64(dj);
            if (lane == 0) {
                C.SW[j - vb] = sw;
                atomic_add_u64(&cacc[j], cj * (sw - (mj ? dj : 0)) - C.TO[j - vb]);
            }
        });
        GP::sync();
        if (GP::rank() == 0) sh_next = 0;
        GP::sync();
        // pass 2: credits of w per wedge, and of k per out-arc k -> j
        if (flat) {
            u32 w = 0, cnt = 0;
            u64 kw = 0;
            F.acc[lane] = 0;
            F.acc2[lane] = 0;
            if (lane < dl) {  // the wedge ends of w, as in pass 1
                w = ci[bl + lane];
                kw = key[w];
                F.kw[lane] = kw;
                F.tin[lane] = Tin[bl + lane];
                FL.aux[lane] = kw > kl;
                FL.ptr[lane] = kw > kl ? out_ptr[w] : (u64)rp[w];
                cnt = (u32)((kw > kl ? out_ptr[w + 1] : (u64)rp[w + 1]) - FL.ptr[lane]);
            }
            flat_walk(FL, cnt, [&](const u32 *jv, const u32 *ov, const bool *ok) {
#pragma unroll
                for (int k = 0; k < UNR; k++) {
                    if (!ok[k]) continue;
                    const u32 pj = jv[k];
                    const u64 idx = FL.ptr[pj] + ov[k];
                    const u64 tin = F.tin[pj];
                    if (FL.aux[pj]) {  // l -> w -> i
                        const u64 p = C.P[out_nbr[idx] - vb];
                        if (p) atomicAdd(&F.acc[pj], p - tin);
                    } else {  // w -> l
                        const u32 i = ci[idx];
                        if (i == l) continue;
                        const u64 p = C.P[i - vb];
                        if (!p) continue;
                        u64 corr = 0;
                        const u64 ki = key[i];
                        if (ki > F.kw[pj]) {  // w -> i
                            const bool li = C.mark[i - vb] && ki > kl;  // l -> i
                            corr = tin + (u64)Tmid[idx] - (li ? 1 : 0);
                        }
                        atomicAdd(&F.acc[pj], p - corr);
                    }
                }
            });
            cnt = 0;
            if (lane < dl && kw < kl) {  // w plays k: its out-arcs k -> j, j != l
                cnt = (u32)(out_ptr[w + 1] - out_ptr[w]);
                FL.ptr[lane] = out_ptr[w];
            }
            flat_walk(FL, cnt, [&](const u32 *jv, const u32 *ov, const bool *ok) {
#pragma unroll
                for (int k = 0; k < UNR; k++) {
                    if (!ok[k]) continue;
                    const u64 q = FL.ptr[jv[k]] + ov[k];
                    const u32 j = out_nbr[q];
                    if (j == l) continue;
                    const u32 sq = out_slot[q];
                    const bool mj = C.mark[j - vb] != 0;
                    const u32 jl = mj && key[j] < kl;  // j -> l
                    const u64 dj = (out_ptr[j + 1] - out_ptr[j]) - jl;
                    const u64 tout = (u64)T[sq] - Tin[sq] - Tmid[sq];
                    atomicAdd(&F.acc2[jv[k]], C.SW[j - vb] - (mj ? dj : 0) - tout + jl);
                }
            });
            if (lane < dl) atomic_add_u64(&cacc[w], F.acc[lane] + F.acc2[lane]);
        } else wave_loop(&sh_next, dl, [&](u32 iw) {
            const u32 slw = bl + iw;
            const u32 w = ci[slw];
            const u64 kw = key[w];
            const u64 tin = Tin[slw];
            u64 accw = 0;
            if (kw > kl) {  // l -> w -> i
                for (u64 q = out_ptr[w] + lane; q < out_ptr[w + 1]; q += WAVE) {
                    const u64 p = C.P[out_nbr[q] - vb];
                    if (p) accw += p - tin;  // w -> i holds; w -> l does not
                }
            } else {  // w -> l
                for (u32 s = rp[w] + lane; s < rp[w + 1]; s += WAVE) {
                    const u32 i = ci[s];
                    if (i == l) continue;
                    const u64 p = C.P[i - vb];
                    if (!p) continue;
                    u64 corr = 0;
                    if (key[i] > kw) {  // w -> i
                        const bool li = C.mark[i - vb] && key[i] > kl;  // l -> i
                        corr = tin + (u64)Tmid[s] - (li ? 1 : 0);
                    }
                    accw += p - corr;
                }
                // w plays k: its out-arcs k -> j, j != l
                const u32 k = w;
                u64 acck = 0;
                for (u64 q = out_ptr[k] + lane; q < out_ptr[k + 1]; q += WAVE) {
                    const u32 j = out_nbr[q];
                    if (j == l) continue;
                    const u32 s = out_slot[q];
                    const bool mj = C.mark[j - vb] != 0;
                    const u32 jl = mj && key[j] < kl;  // j -> l
                    const u64 dj = (out_ptr[j + 1] - out_ptr[j]) - jl;
                    const u64 tout = (u64)T[s] - Tin[s] - Tmid[s];
                    acck += C.SW[j - vb] - (mj ? dj : 0) - tout + jl;
                }
                acck = wave_sum_u64(acck);
                if (lane == 0) atomic_add_u64(&cacc[k], acck);
            }
            accw = wave_sum_u64(accw);
            if (lane == 0) atomic_add_u64(&cacc[w], accw);
        });
        GP::sync();
        // credits of i (summed over its 3-paths) and of l
        const u32 nt = sh_nt;
        u64 accl = 0;
        for (u32 t = GP::rank(); t < nt; t += GP::size) {
            const u32 i = C.touched[t];
            const u64 v = C.P[i - vb] * (u64)C.Wm[i - vb] - C.CI[i - vb];
            accl += v;
            atomic_add_u64(&cacc[i], v);
        }
        accl = GP::sum(accl, sh_red);
        if (GP::rank() == 0) atomic_add_u64(&cacc[l], accl);
        if (steps) {
            const u64 tot = GP::sum(nsteps, sh_red);
            if (GP::rank() == 0) atomic_add_u64(&steps[l], tot);  // the pair sweep may run alongside
        }
        GP::sync();
        // reset: P, CI of the 3-path ends; C, TO, SW of the middle vertices;
        // Wm of every wedge end
        for (u32 t = GP::rank(); t < nt; t += GP::size) {
            const u32 i = C.touched[t];
            C.P[i - vb] = 0;
            C.CI[i - vb] = 0;
        }
        for (u32 t = GP::rank(); t < nj; t += GP::size) {
            const u32 j = C.jt[t];
            C.C[j - vb] = 0;
            C.TO[j - vb] = 0;
            C.SW[j - vb] = 0;
        }
        if (GP::rank() == 0) sh_next = 0;
        GP::sync();
        if (flat) {
            u32 cnt = 0;
            if (lane < dl) {
                const u32 w = ci[bl + lane];
                const bool lw = key[w] > kl;
                const u64 b = lw ? out_ptr[w] : rp[w];
                cnt = (u32)((lw ? out_ptr[w + 1] : (u64)rp[w + 1]) - b);
                FL.ptr[lane] = (u64)((lw ? out_nbr : ci) + b);
            }
            flat_walk(FL, cnt, [&](const u32 *jv, const u32 *ov, const bool *ok) {
#pragma unroll
                for (int k = 0; k < UNR; k++)
                    if (ok[k]) C.Wm[((const u32 *)FL.ptr[jv[k]])[ov[k]] - vb] = 0;
            });
        } else wave_loop(&sh_next, dl, [&](u32 iw) {
            const u32 w = ci[bl + iw];
            if (key[w] > kl) {
                for (u64 q = out_ptr[w] + lane; q < out_ptr[w + 1]; q += WAVE) C.Wm[out_nbr[q] - vb] = 0;
            } else {
                for (u32 s = rp[w] + lane; s < rp[w + 1]; s += WAVE) C.Wm[ci[s] - vb] = 0;
            }
        });
        for (u32 i = GP::rank(); i < dl; i += GP::size) C.mark[ci[bl + i] - vb] = 0;
        GP::sync();
    }
}
