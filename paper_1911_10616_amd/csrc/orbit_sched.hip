// Work scheduling for the per-source kernels: per-vertex cost features, a
// small multilayer perceptron (3 -> 32 -> 32 -> 1, ReLU, fp32) that predicts
// the log2 step count of a source from its out-degree profile, its training
// kernels (mini-batch gradient of the mean squared error, Adam), and the
// binning of vertices by predicted cost into a heaviest-first queue.  The
// schedule only changes the order in which sources are processed; every
// count is an integer sum, so the results are identical under any order.
#include "orbit_common.h"

// Parameter layout (1217 floats): W1[32][3], b1[32], W2[32][32], b2[32],
// W3[32], b3.
#define MLP_IN 3
#define MLP_H 32
#define MLP_OFF_W1 0
#define MLP_OFF_B1 (MLP_OFF_W1 + MLP_H * MLP_IN)
#define MLP_OFF_W2 (MLP_OFF_B1 + MLP_H)
#define MLP_OFF_B2 (MLP_OFF_W2 + MLP_H * MLP_H)
#define MLP_OFF_W3 (MLP_OFF_B2 + MLP_H)
#define MLP_OFF_B3 (MLP_OFF_W3 + MLP_H)
#define MLP_NPARAM (MLP_OFF_B3 + 1)
#define SCHED_BINS 128

// Counter-based hash (splitmix64 finaliser) for initialisation and batches.
__host__ __device__ inline u64 mix64(u64 x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__device__ inline float unit_float(u64 h) { return (float)(h >> 40) * (1.0f / 16777216.0f); }

// features[u] = (log2(1+d+(u)), log2(1 + sum_{w in N+(u)} d+(w)), log2(1+d(u)))
__global__ void k_features(const u32 *deg, const u64 *out_ptr, const u32 *out_nbr, u32 n,
                           float *feat) {
    for (u64 u = GWAVE; u < n; u += NWAVES) {
        const u64 b = out_ptr[u], e = out_ptr[u + 1];
        u64 s = 0;
        for (u64 q = b + lane_id(); q < e; q += WAVE) {
            const u32 w = out_nbr[q];
            s += out_ptr[w + 1] - out_ptr[w];
        }
        s = wave_sum_u64(s);
        if (lane_id() == 0) {
            feat[u * 3 + 0] = log2f(1.0f + (float)(e - b));
            feat[u * 3 + 1] = log2f(1.0f + (float)s);
            feat[u * 3 + 2] = log2f(1.0f + (float)deg[u]);
        }
    }
}

// He-style initialisation from the hash of (seed, index).
__global__ void k_mlp_init(float *w, u32 seed) {
    for (u32 i = (u32)GTID; i < MLP_NPARAM; i += (u32)GSTRIDE) {
        float fan_in = i < MLP_OFF_B1 ? (float)MLP_IN : i < MLP_OFF_W3 ? (float)MLP_H : (float)MLP_H;
        bool bias = (i >= MLP_OFF_B1 && i < MLP_OFF_W2) || (i >= MLP_OFF_B2 && i < MLP_OFF_W3) ||
                    i == MLP_OFF_B3;
        float r = unit_float(mix64(((u64)seed << 32) ^ i)) * 2.0f - 1.0f;  // [-1, 1)
        w[i] = bias ? 0.0f : r * sqrtf(6.0f / fan_in);
    }
}

__device__ inline float mlp_forward(const float *W, const float *x, float *h1, float *h2) {
    for (int j = 0; j < MLP_H; j++) {
        float a = W[MLP_OFF_B1 + j];
        for (int i = 0; i < MLP_IN; i++) a += W[MLP_OFF_W1 + j * MLP_IN + i] * x[i];
        h1[j] = a > 0.0f ? a : 0.0f;
    }
    for (int j = 0; j < MLP_H; j++) {
        float a = W[MLP_OFF_B2 + j];
        for (int i = 0; i < MLP_H; i++) a += W[MLP_OFF_W2 + j * MLP_H + i] * h1[i];
        h2[j] = a > 0.0f ? a : 0.0f;
    }
    float y = W[MLP_OFF_B3];
    for (int i = 0; i < MLP_H; i++) y += W[MLP_OFF_W3 + i] * h2[i];
    return y;
}

__global__ void __launch_bounds__(WG) k_mlp_predict(const float *w, const float *feat, u32 count,
                                                   float *out) {
    __shared__ float W[MLP_NPARAM];
    for (u32 i = threadIdx.x; i < MLP_NPARAM; i += WG) W[i] = w[i];
    __syncthreads();
    float h1[MLP_H], h2[MLP_H];
    for (u64 s = GTID; s < count; s += GSTRIDE) out[s] = mlp_forward(W, feat + 3 * s, h1, h2);
}

// Gradient of L = (1/N) sum_s (y_s - t_s)^2 over the samples of a batch
// (sample s of step `step` is hash(seed, step, s) mod count, or s itself
// when full_batch).  The first MLP_TILE threads each run one sample forward
// and backward and keep its activations and back-propagated errors in LDS;
// the whole workgroup then forms the weight gradients as sums over the
// tile's samples (each thread owns a few parameters) and adds them to grad
// with one atomic per parameter.
#define MLP_TILE 64
// Targets come either as floats or as step counts s (target log2(1+s)).
__global__ void __launch_bounds__(WG) k_mlp_grad(const float *w, const float *feat,
                                                const float *target, const u64 *steps,
                                                u32 count, u32 batch, u32 full_batch, u32 seed,
                                                u32 step, float *grad, float *loss) {
    __shared__ float W[MLP_NPARAM];
    __shared__ float sx[MLP_TILE][MLP_IN];
    __shared__ float sh1[MLP_TILE][MLP_H + 1];
    __shared__ float sd2[MLP_TILE][MLP_H + 1];
    __shared__ float sd1[MLP_TILE][MLP_H + 1];
    __shared__ float sh2[MLP_TILE][MLP_H + 1];
    __shared__ float sdy[MLP_TILE];
    for (u32 i = threadIdx.x; i < MLP_NPARAM; i += WG) W[i] = w[i];
    __syncthreads();
    const float inv_n = 1.0f / (float)batch;
    for (u64 base = (u64)blockIdx.x * MLP_TILE; base < batch; base += (u64)gridDim.x * MLP_TILE) {
        const u32 t = threadIdx.x;
        const u64 k = base + t;
        float x[MLP_IN] = {0, 0, 0};
        float h1[MLP_H], h2[MLP_H];
        float dy = 0.0f;
        if (t < MLP_TILE && k < batch) {
            u64 sidx = full_batch ? k : mix64(((u64)seed << 40) ^ ((u64)step << 20) ^ k) % count;
            for (int i = 0; i < MLP_IN; i++) x[i] = feat[3 * sidx + i];
            float y = mlp_forward(W, x, h1, h2);
            float tv = target ? target[sidx] : log2f(1.0f + (float)steps[sidx]);
            float diff = y - tv;
            dy = 2.0f * diff * inv_n;
            atomicAdd(loss, diff * diff * inv_n);
        } else {
            for (int j = 0; j < MLP_H; j++) { h1[j] = 0.0f; h2[j] = 0.0f; }
        }
        // back-propagate to the hidden layers
        if (t < MLP_TILE) {
            float d2[MLP_H];
            for (int j = 0; j < MLP_H; j++) d2[j] = h2[j] > 0.0f ? dy * W[MLP_OFF_W3 + j] : 0.0f;
            for (int i = 0; i < MLP_H; i++) {
                float a = 0.0f;
                for (int j = 0; j < MLP_H; j++) a += W[MLP_OFF_W2 + j * MLP_H + i] * d2[j];
                sd1[t][i] = h1[i] > 0.0f ? a : 0.0f;
                sh1[t][i] = h1[i];
                sd2[t][i] = d2[i];
                sh2[t][i] = h2[i];
            }
            for (int i = 0; i < MLP_IN; i++) sx[t][i] = x[i];
            sdy[t] = dy;
        }
        __syncthreads();
        // weight gradients summed over the tile's samples
        for (u32 p = threadIdx.x; p < MLP_NPARAM; p += WG) {
            float g = 0.0f;
            if (p < MLP_OFF_B1) {
                const u32 j = p / MLP_IN, i = p % MLP_IN;
                for (int s = 0; s < MLP_TILE; s++) g += sd1[s][j] * sx[s][i];
            } else if (p < MLP_OFF_W2) {
                const u32 j = p - MLP_OFF_B1;
                for (int s = 0; s < MLP_TILE; s++) g += sd1[s][j];
            } else if (p < MLP_OFF_B2) {
                const u32 q = p - MLP_OFF_W2, j = q / MLP_H, i = q % MLP_H;
                for (int s = 0; s < MLP_TILE; s++) g += sd2[s][j] * sh1[s][i];
            } else if (p < MLP_OFF_W3) {
                const u32 j = p - MLP_OFF_B2;
                for (int s = 0; s < MLP_TILE; s++) g += sd2[s][j];
            } else if (p < MLP_OFF_B3) {
                const u32 i = p - MLP_OFF_W3;
                for (int s = 0; s < MLP_TILE; s++) g += sdy[s] * sh2[s][i];
            } else {
                for (int s = 0; s < MLP_TILE; s++) g += sdy[s];
            }
            if (g != 0.0f) atomicAdd(&grad[p], g);
        }
        __syncthreads();
    }
}

// Adam update of all parameters (step index t >= 1); m and v hold the
// moment estimates.
__global__ void k_mlp_adam(float *w, const float *grad, float *m, float *v, u32 t, float lr) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float bc1 = 1.0f - powf(b1, (float)t), bc2 = 1.0f - powf(b2, (float)t);
    for (u32 i = (u32)GTID; i < MLP_NPARAM; i += (u32)GSTRIDE) {
        const float g = grad[i];
        const float mi = b1 * m[i] + (1.0f - b1) * g;
        const float vi = b2 * v[i] + (1.0f - b2) * g * g;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

__global__ void k_zero_f32(float *p, u32 len) {
    for (u32 i = (u32)GTID; i < len; i += (u32)GSTRIDE) p[i] = 0.0f;
}

// Predicted (or static) cost -> bin; histogram; heaviest-first queue.
// static schedule: cost = log2(1+d(u)) + log2(1+d+(u)) (degree thresholds);
// learned schedule: cost = the network's prediction.
__device__ inline u32 cost_bin(float c) {
    float b = c * 4.0f;
    if (!(b > 0.0f)) return 0;
    if (b >= (float)(SCHED_BINS - 1)) return SCHED_BINS - 1;
    return (u32)b;
}

__global__ void k_sched_bins(const float *feat, const float *pred, u32 n, u32 *bin,
                             u32 *hist) {
    __shared__ u32 h[SCHED_BINS];
    for (u32 i = threadIdx.x; i < SCHED_BINS; i += WG) h[i] = 0;
    __syncthreads();
    for (u64 u = GTID; u < n; u += GSTRIDE) {
        float c = pred ? pred[u] : feat[3 * u + 2] + feat[3 * u + 0];
        u32 b = cost_bin(c);
        bin[u] = b;
        atomicAdd(&h[b], 1u);
    }
    __syncthreads();
    for (u32 i = threadIdx.x; i < SCHED_BINS; i += WG)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// exclusive offsets with the heaviest bin first (single workgroup)
__global__ void k_sched_offsets(u32 *hist) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    u32 run = 0;
    for (int b = SCHED_BINS - 1; b >= 0; b--) {
        u32 c = hist[b];
        hist[b] = run;
        run += c;
    }
}

__global__ void k_sched_scatter(const u32 *bin, u32 n, u32 *cursor, u32 *order) {
    for (u64 u = GTID; u < n; u += GSTRIDE) order[atomicAdd(&cursor[bin[u]], 1u)] = (u32)u;
}

// ---- relabelling (ORB_RELABEL): vertices renumbered heaviest first, by the
// same degree classes as the static schedule (bins of 4 log2(1+d)), so that
// the hubs' rows, maps and per-vertex data sit together.  The counts are
// computed on the relabelled graph and written back to the original ids.
__global__ void k_deg_bins(const u32 *deg, u32 n, u32 *bin, u32 *hist) {
    __shared__ u32 h[SCHED_BINS];
    for (u32 i = threadIdx.x; i < SCHED_BINS; i += WG) h[i] = 0;
    __syncthreads();
    for (u64 u = GTID; u < n; u += GSTRIDE) {
        const u32 b = cost_bin(log2f(1.0f + (float)deg[u]));
        bin[u] = b;
        atomicAdd(&h[b], 1u);
    }
    __syncthreads();
    for (u32 i = threadIdx.x; i < SCHED_BINS; i += WG)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// newid[order[i]] = i; ndeg[i] = d(order[i])
__global__ void k_relabel_index(const u32 *order, const u32 *deg, u32 n, u32 *newid,
                                u32 *ndeg) {
    for (u64 i = GTID; i < n; i += GSTRIDE) {
        const u32 u = order[i];
        newid[u] = (u32)i;
        ndeg[i] = deg[u];
    }
}

// row i of the relabelled CSR: the new ids of the neighbours of order[i]
// (unsorted; k_row_sort_* sort every row), one wave per row
__global__ void k_relabel_fill(const u32 *rp, const u32 *ci, const u32 *order,
                               const u32 *newid, const u64 *nrp64, u32 n, u32 *nrp,
                               u32 *nci) {
    for (u64 i = GWAVE; i < n; i += NWAVES) {
        const u32 u = order[i];
        const u32 b = rp[u], e = rp[u + 1];
        const u64 o = nrp64[i];
        if (lane_id() == 0) {
            nrp[i] = (u32)o;
            if (i + 1 == n) nrp[n] = (u32)nrp64[n];
        }
        for (u32 s = b + lane_id(); s < e; s += WAVE) nci[o + (s - b)] = newid[ci[s]];
    }
}

// Sorting the rows of the relabelled CSR: rows of up to 64 entries by one
// wave in registers (bitonic over lanes); longer rows are queued for
// k_row_sort_wg.
__global__ void k_row_sort_small(const u32 *nrp, u32 n, u32 *nci, u32 *queue, u32 *qlen) {
    const u32 lane = lane_id();
    for (u64 i = GWAVE; i < n; i += NWAVES) {
        const u32 b = nrp[i], L = nrp[i + 1] - b;
        if (L < 2) continue;
        if (L > WAVE) {
            if (lane == 0) queue[atomicAdd(qlen, 1u)] = (u32)i;
            continue;
        }
        u32 key = 0xffffffffu;
        if (lane < L) key = nci[b + lane];
        for (u32 k = 2; k <= WAVE; k <<= 1) {
            for (u32 j = k >> 1; j > 0; j >>= 1) {
                const u32 other = __shfl_xor(key, (int)j, WAVE);
                const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
                key = keep_min ? (key < other ? key : other) : (key > other ? key : other);
            }
        }
        if (lane < L) nci[b + lane] = key;
    }
}

// One workgroup per queued row: up to 4096 entries by bitonic sort in LDS;
// longer rows (ids distinct, below n) by marking a bitmap of n bits in the
// workgroup's scratch and reading the marked ids back in order.
#ifndef ROW_SORT_LDS
#define ROW_SORT_LDS 4096
#endif
__global__ void __launch_bounds__(WG) k_row_sort_wg(const u32 *nrp, u32 *nci, const u32 *queue,
                                                   const u32 *qlen, u32 *bitmaps, u32 n) {
    __shared__ u32 sk[ROW_SORT_LDS];
    __shared__ u32 part[WG];
    const u32 nw = (n + 31) / 32;
    u32 *bm = bitmaps + (u64)blockIdx.x * nw;
    const u32 cnt = *qlen;
    for (u32 qi = blockIdx.x; qi < cnt; qi += gridDim.x) {
        const u32 row = queue[qi];
        const u32 b = nrp[row], L = nrp[row + 1] - b;
        u32 *p = nci + b;
        if (L <= ROW_SORT_LDS) {
            u32 P = 128;
            while (P < L) P <<= 1;
            for (u32 i = threadIdx.x; i < P; i += WG) sk[i] = i < L ? p[i] : 0xffffffffu;
            __syncthreads();
            for (u32 k = 2; k <= P; k <<= 1) {
                for (u32 j = k >> 1; j > 0; j >>= 1) {
                    for (u32 i = threadIdx.x; i < P; i += WG) {
                        const u32 ij = i ^ j;
                        if (ij > i) {
                            const u32 x = sk[i], y = sk[ij];
                            const bool asc = (i & k) == 0;
                            if ((x > y) == asc) { sk[i] = y; sk[ij] = x; }
                        }
                    }
                    __syncthreads();
                }
            }
            for (u32 i = threadIdx.x; i < L; i += WG) p[i] = sk[i];
            __syncthreads();
            continue;
        }
        for (u32 w = threadIdx.x; w < nw; w += WG) bm[w] = 0;
        __syncthreads();
        for (u32 i = threadIdx.x; i < L; i += WG) {
            const u32 v = p[i];
            atomicOr(&bm[v >> 5], 1u << (v & 31));
        }
        __syncthreads();
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
                const u32 bb = __ffs(bits) - 1;
                bits &= bits - 1;
                p[r++] = w * 32 + bb;
            }
        }
        __syncthreads();
    }
}

