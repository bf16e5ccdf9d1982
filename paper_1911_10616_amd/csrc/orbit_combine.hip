// Per-vertex kernels: neighbour sums, the triangle sweep, the orbit
// equations of Lemma 4vertexorbit and Theorem 5vertexorbit, and the
// non-induced -> induced transform.
#include "orbit_common.h"
#include "orbit_tables.h"

#define NI(u, o) ni[(u64)(u) * ORB_NORB + (o)]

// The per-vertex kernels run one group of G consecutive lanes per vertex
// (G = 8..64, chosen from the mean degree): low-degree graphs then use
// all lanes of a wave and reduce over fewer steps.
template <int G> __device__ inline u32 glane() { return threadIdx.x & (G - 1); }
template <int G> __device__ inline u64 group_sum_u64(u64 v) {
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}
// Every lane of a wave runs the same number of iterations (vertex u of a
// group past n is inactive: empty neighbour range, no stores), so the
// group reductions always see all of their lanes.
#define GROUP_LOOP(G, u, n)                                                              \
    for (u64 u##_base = (GTID / WAVE) * (WAVE / (G)); u##_base < (n);                   \
         u##_base += (GSTRIDE / WAVE) * (WAVE / (G)))                                   \
        for (u64 u = u##_base + lane_id() / (G), u##_once = 0; u##_once < 1; u##_once++)
#define GROUP_VALID(u, n) ((u) < (n))

// Tv(u) = number of triangles at u (half the sum of T over u's edges);
// N1(u) = sum over neighbours v of (d(v) - 1) (orbit 1).
template <int G>
__global__ void k_vert0(const u32 *rp, const u32 *ci, const u32 *deg, const u32 *T, u32 n,
                        u64 *Tv, u64 *N1) {
    GROUP_LOOP(G, u, n) {
        u64 t = 0, n1 = 0;
        for (u32 s = (u < n ? rp[u] : 0) + glane<G>(); s < (u < n ? rp[u + 1] : 0); s += G) {
            t += T[s];
            n1 += (u64)deg[ci[s]] - 1;
        }
        t = group_sum_u64<G>(t);
        n1 = group_sum_u64<G>(n1);
        if (glane<G>() == 0 && u < n) { Tv[u] = t / 2; N1[u] = n1; }
    }
}

// Triangle sweep: for every triangle {u,v,x} at u, the summands of the
// orbit equations that sum over triangles (Lemma 4vertexorbit orbit 12;
// Theorem 5vertexorbit orbits 25, 26, 29, 32, 43, 46, 48, 52, 53, 54, 59,
// 61, 65).  Each triangle is visited from the slot (u,v) with v < x.
template <int G>
__global__ void k_trisweep(const u32 *rp, const u32 *ci, const u32 *rev,
                           const u32 *deg, const u32 *T, const u64 *tl_ptr, const uint2 *tl,
                           const u64 *Tv, const u64 *N1, const u64 *E7, const u64 *E9,
                           const u64 *C4e, const u64 *K4e, u32 n, u64 *ni) {
    GROUP_LOOP(G, u, n) {
        u64 a12 = 0, a25 = 0, a26 = 0, a29 = 0, a32 = 0, a43 = 0, a46 = 0, a48 = 0, a52 = 0,
            a53 = 0, a54 = 0, a59 = 0, a61 = 0, a65 = 0;
        const u64 du = u < n ? deg[u] : 0;
        for (u32 s = (u < n ? rp[u] : 0) + glane<G>(); s < (u < n ? rp[u + 1] : 0); s += G) {
            const u32 v = ci[s];
            const u32 tuv = T[s];
            if (tuv == 0) continue;
            const bool lo = (u32)u < v;
            const uint2 *p = tl + tl_ptr[lo ? s : rev[s]];
            const u64 dv = deg[v];
            const u64 c4uv = C4e[s];
            for (u32 k = 0; k < tuv; k++) {
                uint2 e = p[k];
                const u32 sux = lo ? e.x : e.y, svx = lo ? e.y : e.x;
                const u32 x = ci[sux];
                if (x < v) continue;
                const u32 sxv = rev[svx];
                const u64 dx = deg[x];
                const u64 tvx = T[svx], tux = T[sux];
                a12 += tvx - 1;
                a25 += (dv - 2) * (dx - 2);
                a26 += (du - 2) * ((dv - 2) + (dx - 2));
                a29 += N1[v] + N1[x];
                a32 += c2((i64)dv - 2) + c2((i64)dx - 2);
                a43 += (Tv[v] - 1) + (Tv[x] - 1);
                a46 += E7[svx];
                a48 += ((u64)tuv - 1) * (dx - 2) + (tux - 1) * (dv - 2);
                a52 += C4e[svx];
                a53 += c4uv + C4e[sux];
                a54 += c2((i64)tvx - 1);
                a59 += E9[sxv] + E9[svx];
                a61 += ((u64)tuv - 1) * (tux - 1);
                a65 += K4e[svx];
            }
        }
        a12 = group_sum_u64<G>(a12); a25 = group_sum_u64<G>(a25); a26 = group_sum_u64<G>(a26);
        a29 = group_sum_u64<G>(a29); a32 = group_sum_u64<G>(a32); a43 = group_sum_u64<G>(a43);
        a46 = group_sum_u64<G>(a46); a48 = group_sum_u64<G>(a48); a52 = group_sum_u64<G>(a52);
        a53 = group_sum_u64<G>(a53); a54 = group_sum_u64<G>(a54); a59 = group_sum_u64<G>(a59);
        a61 = group_sum_u64<G>(a61); a65 = group_sum_u64<G>(a65);
        if (glane<G>() == 0 && u < n) {
            NI(u, 12) = a12; NI(u, 25) = a25; NI(u, 26) = a26; NI(u, 29) = a29;
            NI(u, 32) = a32; NI(u, 43) = a43; NI(u, 46) = a46; NI(u, 48) = a48;
            NI(u, 52) = a52; NI(u, 53) = a53; NI(u, 54) = a54; NI(u, 59) = a59;
            NI(u, 61) = a61; NI(u, 65) = a65;
        }
    }
}

// First-order neighbour sums and the final orbits 0..14 (Lemma
// 4vertexorbit).  Temporary sums that later equations need are parked in
// the columns of the orbits they feed (28, 31, 37, 56, 60).  Orbit 69 of u
// is half the sum, over arcs (v,u), of Q(v,u); the sum is even and is
// accumulated in 128 bits so that the halving is exact modulo 2^64.
template <int G>
__global__ void k_vert1(const u32 *rp, const u32 *ci, const u32 *rev, const u32 *deg,
                        const u32 *T, const u64 *Tv, const u64 *N1, const u64 *C4v,
                        const u64 *K4v, const u64 *C4e, const u64 *K4e, const u64 *E9,
                        const u64 *Q, const u64 *vacc, const u64 *cacc, u32 n, u64 *ni) {
    GROUP_LOOP(G, u, n) {
        const u64 du = u < n ? deg[u] : 0;
        u64 s4 = 0, n6 = 0, n9 = 0, n10 = 0, n13 = 0, s28 = 0, s31 = 0, n22 = 0, s37 = 0,
            n40 = 0, n41 = 0, n55 = 0, s56 = 0, n57 = 0, s60 = 0, n67 = 0, qlo = 0, qhi = 0;
        for (u32 s = (u < n ? rp[u] : 0) + glane<G>(); s < (u < n ? rp[u + 1] : 0); s += G) {
            const u32 v = ci[s];
            const u64 dv = deg[v];
            const u64 t = T[s];
            const u32 r = rev[s];
            const u64 tv = Tv[v];
            s4 += N1[v];
            n6 += c2((i64)dv - 1);
            n9 += tv - t;
            n10 += t * (dv - 2);
            n13 += c2((i64)t);
            s28 += tv;
            s31 += (dv - 1) * tv;
            n22 += c3((i64)dv - 1);
            s37 += C4e[s] * (dv - 2);
            n40 += E9[r] * (dv - 3);
            n41 += c2((i64)t) * (dv - 3);
            n55 += c3((i64)t);
            s56 += K4v[v];
            n57 += K4e[s] * (dv - 3);
            s60 += E9[r] * (t - 1);
            n67 += K4e[s] * (t - 2);
            u64 q = Q[r];
            qlo += q;
            qhi += qlo < q;
        }
        s4 = group_sum_u64<G>(s4); n6 = group_sum_u64<G>(n6); n9 = group_sum_u64<G>(n9);
        n10 = group_sum_u64<G>(n10); n13 = group_sum_u64<G>(n13); s28 = group_sum_u64<G>(s28);
        s31 = group_sum_u64<G>(s31); n22 = group_sum_u64<G>(n22); s37 = group_sum_u64<G>(s37);
        n40 = group_sum_u64<G>(n40); n41 = group_sum_u64<G>(n41); n55 = group_sum_u64<G>(n55);
        s56 = group_sum_u64<G>(s56); n57 = group_sum_u64<G>(n57); s60 = group_sum_u64<G>(s60);
        n67 = group_sum_u64<G>(n67);
        // 128-bit sum of Q: add the lane partials pairwise with carries
        for (int off = G / 2; off > 0; off >>= 1) {
            u64 olo = __shfl_xor(qlo, off, WAVE), ohi = __shfl_xor(qhi, off, WAVE);
            u64 nlo = qlo + olo;
            qhi = qhi + ohi + (nlo < qlo);
            qlo = nlo;
        }
        if (glane<G>() == 0 && u < n) {
            const u64 n1 = N1[u], t = Tv[u];
            const u64 n2 = c2((i64)du), n3 = t;
            NI(u, 0) = du;
            NI(u, 1) = n1;
            NI(u, 2) = n2;
            NI(u, 3) = n3;
            NI(u, 4) = s4 - 2 * n2 - 2 * n3;
            NI(u, 5) = n1 * (du - 1) - 2 * n3;
            NI(u, 6) = n6;
            NI(u, 7) = c3((i64)du);
            NI(u, 8) = C4v[u];
            NI(u, 9) = n9;
            NI(u, 10) = n10;
            NI(u, 11) = t * (du - 2);
            NI(u, 13) = n13;
            NI(u, 14) = K4v[u];
            NI(u, 22) = n22;
            NI(u, 28) = s28;
            NI(u, 31) = s31;
            NI(u, 37) = s37;
            NI(u, 40) = n40;
            NI(u, 41) = n41;
            NI(u, 55) = n55;
            NI(u, 56) = s56;
            NI(u, 57) = n57;
            NI(u, 60) = s60;
            NI(u, 67) = n67;
            NI(u, 69) = (qlo >> 1) | (qhi << 63);
            // pair sweep and 5-cycle results (zero when those kernels did not run)
            const u64 *va = vacc + u * 8;
            NI(u, 36) = va[0];
            NI(u, 50) = va[1];
            NI(u, 51) = va[2];
            NI(u, 63) = va[3];
            NI(u, 68) = va[4];
            NI(u, 64) = va[5];
            NI(u, 49) = va[6];
            NI(u, 62) = va[7];
            NI(u, 34) = cacc[u];
        }
    }
}

// Second-order neighbour sums and every remaining equation of Theorem
// 5vertexorbit (with the corrected forms of orbits 19, 20, 21, 35, 40, 64,
// 66, 68, 69 that the transcribed equations need), finishing the
// non-induced counts of orbits 15..72 of u.  Reads only columns 4..13 of
// the neighbours' rows, and writes only columns 15..72 of its own row.
template <int G>
__global__ void k_vert2(const u32 *rp, const u32 *ci, const u32 *deg, const u64 *Tv,
                        const u64 *N1, u32 n, u64 *ni) {
    GROUP_LOOP(G, u, n) {
        u64 s15 = 0, s18 = 0, s19 = 0, s24 = 0, s27 = 0, s35 = 0, s39 = 0, s45 = 0;
        for (u32 s = (u < n ? rp[u] : 0) + glane<G>(); s < (u < n ? rp[u + 1] : 0); s += G) {
            const u64 *r = ni + (u64)ci[s] * ORB_NORB;
            s15 += r[4];
            s19 += r[5];
            s18 += r[6];
            s35 += r[8];
            s27 += r[9];
            s24 += r[10];
            s45 += r[12];
            s39 += r[13];
        }
        s15 = group_sum_u64<G>(s15); s18 = group_sum_u64<G>(s18); s19 = group_sum_u64<G>(s19);
        s24 = group_sum_u64<G>(s24); s27 = group_sum_u64<G>(s27); s35 = group_sum_u64<G>(s35);
        s39 = group_sum_u64<G>(s39); s45 = group_sum_u64<G>(s45);
        if (glane<G>() != 0 || u >= n) continue;
        u64 *R = ni + u * ORB_NORB;
        const u64 d = deg[u];
        const u64 n1 = N1[u], t = Tv[u];
        const u64 n3 = R[3], n4 = R[4], n5 = R[5], n6 = R[6], n7 = R[7], n8 = R[8], n9 = R[9],
                  n10 = R[10], n11 = R[11], n12 = R[12], n13 = R[13], n14 = R[14];
        R[15] = s15 - n5 - 2 * n11 - 2 * n8;
        R[16] = n4 * (d - 1) - n10 - 2 * n8;
        R[17] = c2((i64)n1) - n3 - n6 - n8 - n10;
        R[18] = s18 - 3 * n7 - n10;
        R[19] = s19 - n4 - n5 - n10;
        R[20] = (d - 1) * n6 - n10;
        R[21] = c2((i64)d - 1) * n1 - 2 * n11;
        // R[22] final from the first-order sums
        R[23] = c4((i64)d);
        R[24] = s24 - n10 - 2 * n11 - 2 * n12;
        R[25] = R[25] - n12;
        R[26] = R[26] - 2 * n13;
        R[27] = s27 - n11 - 2 * n13;
        R[28] = (d - 1) * R[28] - 2 * n3 - 2 * n11 - 2 * n12;
        R[29] = R[29] - 4 * n3 - n10 - 2 * n11 - 2 * n12 - 2 * n13;
        R[30] = t * n1 - 2 * n3 - n10 - 2 * n13;
        R[31] = R[31] - 2 * n9 - n10 - 2 * n3;
        // R[32] final from the triangle sweep
        R[33] = t * c2((i64)d - 2);
        // R[34] final from the 5-cycle kernel
        R[35] = s35 - 2 * n8 - n13;
        R[36] = R[36] - n13;
        R[37] = R[37] - 2 * n12;
        R[38] = n8 * (d - 2) - n13;
        R[39] = s39 - n13 - 2 * n12;
        // R[40], R[41] final from the first-order sums
        R[42] = (d - 3) * n13;
        R[43] = R[43] - 2 * n12 - 2 * n13;
        R[44] = c2((i64)t) - n13;
        R[45] = s45 - 2 * n13 - 3 * n14;
        R[46] = R[46] - n11 - 3 * n14;
        R[47] = n12 * (d - 2) - 3 * n14;
        R[48] = R[48] - 6 * n14;
        // R[49], R[50] final from the pair sweep
        R[51] = R[51] - 2 * n12;
        R[52] = R[52] - 2 * n13;
        R[53] = R[53] - 2 * n13 - 2 * n12;
        // R[54], R[55] final
        R[56] = R[56] - 3 * n14;
        // R[57] final
        R[58] = n14 * (d - 3);
        R[59] = R[59] - 2 * n13 - 6 * n14;
        R[60] = R[60] - 6 * n14;
        R[61] = R[61] - 3 * n14;
        R[62] = R[62] - n13;
        // R[63], R[64] final from the pair sweep
        R[65] = R[65] - 3 * n14;
        // R[66]..R[72] final (66, 71: triangle 4-clique terms; 67, 69:
        // first-order sums; 68: wheel maps; 70, 72: clique passes)
    }
}

// Induced counts: I = Ainv N per row, block by block; Ainv is unit upper
// triangular, so row i only reads columns >= i and can be overwritten in
// increasing order.  One wave per tile of 64 rows: the rows are read into
// LDS with coalesced loads, each lane transforms one row in registers (a
// row's 73 words are 584 bytes apart from the next lane's, so the LDS reads
// are spread over all banks), and the first K columns go out with coalesced
// stores (out may alias ni when K == 73).
#define XF_ROWS 64
// With a relabelling, row r of ni belongs to vertex orig[r] of the caller's
// graph and is written there (orig == NULL: the identity).
__global__ void __launch_bounds__(WAVE) k_transform(u64 *ni, u32 n, int K, int induced,
                                                    const u32 *orig, u64 *out) {
    __shared__ u64 tile[XF_ROWS * ORB_NORB];
    const u32 lane = threadIdx.x;
    for (u64 base = (u64)blockIdx.x * XF_ROWS; base < n; base += (u64)gridDim.x * XF_ROWS) {
        const u32 rows = n - base < XF_ROWS ? (u32)(n - base) : XF_ROWS;
        const u64 *src = ni + base * ORB_NORB;
        for (u32 i = lane; i < rows * ORB_NORB; i += WAVE) tile[i] = src[i];
        __syncthreads();
        if (induced && lane < rows) {
            // the row in registers: with both loops unrolled every column
            // index and coefficient of the table is a constant
            u64 *T = tile + (u64)lane * ORB_NORB;
            u64 R[ORB_NORB];
#pragma unroll
            for (int c = 0; c < ORB_NORB; c++) R[c] = T[c];
#pragma unroll
            for (int i = 0; i < ORB_NORB; i++) {
                if (i < K) {
                    u64 acc = 0;
#pragma unroll
                    for (int k = ORB_AINV_PTR[i]; k < ORB_AINV_PTR[i + 1]; k++)
                        acc += (u64)(i64)ORB_AINV_VAL[k] * R[ORB_AINV_COL[k]];
                    R[i] = acc;
                }
            }
#pragma unroll
            for (int c = 0; c < ORB_NORB; c++) T[c] = R[c];
        }
        __syncthreads();
        u64 *dst = out + base * K;
        if (orig) {
            for (u32 i = lane; i < rows * (u32)K; i += WAVE) {
                const u32 r = i / K, c = i % K;
                out[(u64)orig[base + r] * K + c] = tile[r * ORB_NORB + c];
            }
        } else if (K == ORB_NORB) {
            for (u32 i = lane; i < rows * ORB_NORB; i += WAVE) dst[i] = tile[i];
        } else {
            for (u32 i = lane; i < rows * (u32)K; i += WAVE)
                dst[i] = tile[(i / K) * ORB_NORB + i % K];
        }
        __syncthreads();
    }
}

// Work statistics (reported with per-phase timing): wedges = sum of C(d,2)
// over vertices, diamonds = sum of C(T(e),2) over edges, and the directed
// 3-paths the 5-cycle kernel walks, i <- j <- k with k -> l for a source l:
// sum over k of d+(k) * sum_{j in N+(k)} d+(j).
__global__ void k_stats(const u32 *src, const u32 *ci, const u32 *deg, const u32 *T,
                        const u64 *out_ptr, const u32 *out_nbr, u32 n, u64 M2, DevState *st) {
    u64 w = 0, d = 0, p3 = 0;
    for (u64 u = GTID; u < n; u += GSTRIDE) {
        w += c2((i64)deg[u]);
        const u64 b = out_ptr[u], e = out_ptr[u + 1];
        u64 f = 0;
        for (u64 q = b; q < e; q++) {
            const u32 j = out_nbr[q];
            f += out_ptr[j + 1] - out_ptr[j];
        }
        p3 += (e - b) * f;
    }
    for (u64 s = GTID; s < M2; s += GSTRIDE)
        if (src[s] < ci[s]) d += c2((i64)T[s]);
    w = wave_sum_u64(w);
    d = wave_sum_u64(d);
    p3 = wave_sum_u64(p3);
    if (lane_id() == 0) {
        atomic_add_u64(&st->wedges, w);
        atomic_add_u64(&st->diamonds, d);
        atomic_add_u64(&st->paths3, p3);
    }
}

// ---- overflow flags.  Counts are exact modulo 2^64; a row is certainly
// exact when every non-induced count of the vertex is below 2^63.  Bound:
// a non-induced copy of a k-vertex pattern at u is a connected k-vertex
// subgraph containing u; it contains a spanning tree, and at most
// 2^(C(k,2)-k+1) subgraphs on one vertex set share a tree (64, 8, 2 for
// k = 5, 4, 3).  The k-vertex trees containing u number at most the sum over
// the rooted tree shapes with k vertices of hom(shape, G; root -> u) divided
// by the shape's root-fixing automorphisms, and those homomorphism counts
// are nested neighbour sums of degrees:
//   pass 0: s1 = sum_{v~u} d(v),  q1 = sum d(v)^2,  c1 = sum d(v)^3
//   pass 1: s2 = sum_{v~u} s1(v), q2 = sum q1(v),   r1 = sum d(v) s1(v)
//   pass 2: s3 = sum_{v~u} s2(v), then
//     B3 = s1 + d^2/2
//     B4 = s2 + q1/2 + d s1 + d^3/6
//     B5 = s3 + q2/2 + r1 + c1/6 + d s2 + d q1/2 + s1^2/2 + d^2 s1/2 + d^4/24
//   flag = 64 B5 + 8 B4 + 2 B3 + d >= 2^63 (less a relative margin that
//   covers the fp64 rounding of the sums).
template <int G> __device__ inline double group_sum_f64(double v) {
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}
template <int G>
__global__ void k_ovf(const u32 *rp, const u32 *ci, u32 n, int pass, double *a, double *b,
                      unsigned char *flags) {
    GROUP_LOOP(G, u, n) {
        double x0 = 0, x1 = 0, x2 = 0;
        for (u32 s = (u < n ? rp[u] : 0) + glane<G>(); s < (u < n ? rp[u + 1] : 0); s += G) {
            const u32 v = ci[s];
            const double dv = (double)(rp[v + 1] - rp[v]);
            if (pass == 0) {
                x0 += dv; x1 += dv * dv; x2 += dv * dv * dv;
            } else if (pass == 1) {
                const double s1v = a[(u64)v * 3];
                x0 += s1v; x1 += a[(u64)v * 3 + 1]; x2 += dv * s1v;
            } else {
                x0 += b[(u64)v * 3];
            }
        }
        x0 = group_sum_f64<G>(x0);
        x1 = group_sum_f64<G>(x1);
        x2 = group_sum_f64<G>(x2);
        if (glane<G>() != 0 || u >= n) continue;
        if (pass == 0) {
            a[u * 3] = x0; a[u * 3 + 1] = x1; a[u * 3 + 2] = x2;
        } else if (pass == 1) {
            b[u * 3] = x0; b[u * 3 + 1] = x1; b[u * 3 + 2] = x2;
        } else {
            const double d = (double)(rp[u + 1] - rp[u]);
            const double s1 = a[u * 3], q1 = a[u * 3 + 1], c1 = a[u * 3 + 2];
            const double s2 = b[u * 3], q2 = b[u * 3 + 1], r1 = b[u * 3 + 2], s3 = x0;
            const double B3 = s1 + d * d / 2;
            const double B4 = s2 + q1 / 2 + d * s1 + d * d * d / 6;
            const double B5 = s3 + q2 / 2 + r1 + c1 / 6 + d * s2 + d * q1 / 2 + s1 * s1 / 2 +
                              d * d * s1 / 2 + d * d * d * d / 24;
            const double bound = 64 * B5 + 8 * B4 + 2 * B3 + d;
            flags[u] = bound >= 9223372036854775808.0 * (1.0 - 1e-9) ? 1 : 0;
        }
    }
}

// ---- edge orbit counts (Lemma 4edgeorbit).  At every slot s = (u, v):
// E_i<u,v> for i = 0..11, u the endpoint in the vertex orbit of larger
// index (slot (v, u) holds the other orientation):
//   E0 = d(u)-1                     E1 = T(u,v)
//   E2 = sum_{x in N(u)\v} (d(x)-1) - T(u,v) = N1(u) - (d(v)-1) - T(u,v)
//   E3 = (d(u)-1)(d(v)-1) - T(u,v)  E4 = C(d(u)-1, 2)     E5 = C4(u,v)
//   E6 = T(u) - T(u,v)              E7 = sum over triangles (u,v,x) of d(x)-2
//   E8 = T(u,v)(d(u)-2)             E9 = sum over triangles (u,v,x) of T(u,x)-1
//   E10 = C(T(u,v), 2)              E11 = K4(u,v)
// One wave per 64 slots; the 64 x 12 words go through LDS so that the rows
// are written with contiguous stores.
#define NEORB 12
__global__ void __launch_bounds__(WAVE) k_edge_orbits(const u32 *src, const u32 *ci,
                                                      const u32 *deg, const u32 *T,
                                                      const u64 *Tv, const u64 *N1,
                                                      const u64 *C4e, const u64 *E7,
                                                      const u64 *E9, const u64 *K4e, u64 M2,
                                                      u64 *E) {
    __shared__ u64 tile[WAVE * NEORB];
    const u32 lane = threadIdx.x;
    for (u64 base = (u64)blockIdx.x * WAVE; base < M2; base += (u64)gridDim.x * WAVE) {
        const u64 s = base + lane;
        const u32 rows = M2 - base < WAVE ? (u32)(M2 - base) : WAVE;
        if (s < M2) {
            const u32 u = src[s], v = ci[s];
            const u64 du = deg[u], dv = deg[v], t = T[s];
            u64 *o = tile + (u64)lane * NEORB;
            o[0] = du - 1;
            o[1] = t;
            o[2] = N1[u] - (dv - 1) - t;
            o[3] = (du - 1) * (dv - 1) - t;
            o[4] = c2((i64)du - 1);
            o[5] = C4e[s];
            o[6] = Tv[u] - t;
            o[7] = E7[s];
            o[8] = t * (du - 2);
            o[9] = E9[s];
            o[10] = c2((i64)t);
            o[11] = K4e[s];
        }
        __syncthreads();
        u64 *dst = E + base * NEORB;
        for (u32 i = lane; i < rows * NEORB; i += WAVE) dst[i] = tile[i];
        __syncthreads();
    }
}

// ---- VOC distributions and global pattern counts (the paper's
// experiments section, "VOC distributions"; Figs. orb70CCD, orb17CCD,
// H9CCD).  Per orbit o of the K columns:
//   sums[2o], sums[2o+1]: low and high 64 bits of sum_u counts[u][o];
//   hist[o * 65 + b]: number of vertices whose count has bit length b
//     (b = 0 for a zero count, else 2^(b-1) <= count < 2^b), so that the
//     complementary cumulative distribution -- the fraction of vertices
//     with count >= x -- is exact at x = 2^(b-1): sum_{b' >= b} hist / n.
// Elements are read row by row (coalesced); each workgroup keeps its
// histogram and sums in LDS and flushes them once.  A 64-bit add returns
// the old value, so its carry into the high word is known exactly.
#define VOC_BINS 65
__device__ inline void add_u128(u64 *lo, u64 *hi, u64 v) {
    if (!v) return;
    const u64 old = atomicAdd(lo, v);
    if (old + v < old) atomicAdd(hi, 1ull);
}
__global__ void __launch_bounds__(WG) k_voc(const u64 *counts, u32 n, int K, u64 *sums,
                                           u64 *hist) {
    __shared__ u32 lh[ORB_NORB * VOC_BINS];
    __shared__ u64 ls[ORB_NORB * 2];
    for (u32 i = threadIdx.x; i < (u32)K * VOC_BINS; i += WG) lh[i] = 0;
    for (u32 i = threadIdx.x; i < (u32)K * 2; i += WG) ls[i] = 0;
    __syncthreads();
    const u64 total = (u64)n * K;
    for (u64 i = GTID; i < total; i += GSTRIDE) {
        const u32 o = (u32)(i % K);
        const u64 c = counts[i];
        const u32 b = c ? 64 - __clzll((long long)c) : 0;
        atomicAdd(&lh[o * VOC_BINS + b], 1u);
        add_u128(&ls[2 * o], &ls[2 * o + 1], c);
    }
    __syncthreads();
    for (u32 i = threadIdx.x; i < (u32)K * VOC_BINS; i += WG)
        if (lh[i]) atomicAdd(&hist[i], (u64)lh[i]);
    for (u32 o = threadIdx.x; o < (u32)K; o += WG) {
        add_u128(&sums[2 * o], &sums[2 * o + 1], ls[2 * o]);
        if (ls[2 * o + 1]) atomicAdd(&sums[2 * o + 1], ls[2 * o + 1]);
    }
}

// 128-bit value (hi, lo) divided by a small d, by 32-bit limbs
__device__ inline void div_u128_small(u64 hi, u64 lo, u32 d, u64 *qhi, u64 *qlo) {
    const u32 limb[4] = {(u32)(hi >> 32), (u32)hi, (u32)(lo >> 32), (u32)lo};
    u32 q[4];
    u64 r = 0;
    for (int i = 0; i < 4; i++) {
        const u64 x = (r << 32) | limb[i];
        q[i] = (u32)(x / d);
        r = x % d;
    }
    *qhi = ((u64)q[0] << 32) | q[1];
    *qlo = ((u64)q[2] << 32) | q[3];
}

// Copies of each pattern: the sum over vertices of one of its orbits
// divided by the number of pattern vertices in that orbit (every induced
// copy puts that many vertices in the orbit); the first orbit of each
// pattern is used.  pats[2h], pats[2h+1] = low, high 64 bits.
__global__ void k_voc_patterns(const u64 *sums, int K, u64 *pats) {
    if (GTID != 0) return;
    int last = -1;
    for (int o = 0; o < K; o++) {
        const int h = ORB_ORBIT_PATTERN[o];
        if (h == last) continue;
        last = h;
        u64 qh, ql;
        div_u128_small(sums[2 * o + 1], sums[2 * o], ORB_ORBIT_SIZE[o], &qh, &ql);
        pats[2 * h] = ql;
        pats[2 * h + 1] = qh;
    }
}
