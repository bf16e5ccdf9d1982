// Device-side helpers shared by the orbit-counting kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef unsigned long long u64;
typedef uint32_t u32;
typedef long long i64;

#define ORB_NORB 73
#define WG 256
#define WAVE 64
#define WAVES_PER_WG (WG / WAVE)
#define UNSET 0xffffffffu

// error bits written by kernels into DevState::err
#define ERRB_RANGE 0x1u
#define ERRB_LOOP 0x2u
#define ERRB_DUP 0x4u
#define ERRB_ORDER 0x8u
#define ERRB_ASYM 0x10u
#define ERRB_ROWPTR 0x20u
#define ERRB_INTERNAL 0x40u
#define ERRB_CROSS 0x80u     // batched input: an edge joins two graphs
#define ERRB_VPTR 0x100u     // batched input: malformed graph offsets

// Small block of device state shared by the phases of one call.
struct DevState {
    u32 err;
    u32 level;      // peeling: current core level
    u32 round;      // peeling: round id given to vertices appended now
    u32 cur;        // peeling: frontier buffer being consumed
    u32 fsize[2];   // peeling: frontier sizes
    u32 alive;      // peeling: vertices not yet removed
    u32 minalive;   // peeling: smallest remaining degree seen by a scan
    u32 maxlevel;   // peeling: largest level at which a vertex was removed
    u32 gmax;       // batched input: largest graph (vertices)
    u32 work[16];   // dynamic work counters of the per-source kernels
    u64 ntri;       // number of triangles
    u64 scan_total; // total of the last exclusive scan
    u64 wedges;     // sum over vertices of C(d,2)
    u64 diamonds;   // sum over edges of C(T(e),2)
    u64 paths3;     // directed 3-paths walked by the 5-cycle kernel
};

// ---------------------------------------------------------------- binomials
// C(x,k) for k <= 4, exact modulo 2^64: the product of k consecutive
// integers is divisible by k!, so each divisor is taken out of a factor
// that it divides before the (wrapping) multiplication.  C(x,k) = 0 for
// x < k, including negative x.
__host__ __device__ inline u64 c2(i64 x) {
    if (x < 2) return 0;
    u64 a = (u64)x, b = (u64)(x - 1);
    if ((a & 1) == 0) a >>= 1; else b >>= 1;
    return a * b;
}
__host__ __device__ inline u64 c3(i64 x) {
    if (x < 3) return 0;
    u64 f[3] = {(u64)x, (u64)(x - 1), (u64)(x - 2)};
    for (int i = 0; i < 3; i++) if (f[i] % 3 == 0) { f[i] /= 3; break; }
    for (int i = 0; i < 3; i++) if ((f[i] & 1) == 0) { f[i] >>= 1; break; }
    return f[0] * f[1] * f[2];
}
__host__ __device__ inline u64 c4(i64 x) {
    if (x < 4) return 0;
    u64 f[4] = {(u64)x, (u64)(x - 1), (u64)(x - 2), (u64)(x - 3)};
    for (int i = 0; i < 4; i++) if (f[i] % 3 == 0) { f[i] /= 3; break; }
    int q = -1;
    for (int i = 0; i < 4; i++) if ((f[i] & 3) == 0) { f[i] >>= 2; q = i; break; }
    for (int i = 0; i < 4; i++) if (i != q && (f[i] & 1) == 0) { f[i] >>= 1; break; }
    return f[0] * f[1] * f[2] * f[3];
}

// ------------------------------------------------------------- wave helpers
__device__ inline u32 lane_id() { return threadIdx.x & (WAVE - 1); }
__device__ inline u32 wave_in_wg() { return threadIdx.x / WAVE; }

__device__ inline u64 wave_sum_u64(u64 v) {
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}
__device__ inline u32 wave_sum_u32(u32 v) {
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// lower_bound over a sorted u32 array: first index in [0,len) with a[i] >= key
__device__ inline u32 lbound(const u32 *a, u32 len, u32 key) {
    u32 lo = 0, hi = len;
    while (lo < hi) {
        u32 mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}
// index of key in sorted a[0,len), or UNSET
__device__ inline u32 bfind(const u32 *a, u32 len, u32 key) {
    u32 i = lbound(a, len, key);
    return (i < len && a[i] == key) ? i : UNSET;
}

__device__ inline unsigned char *align256(unsigned char *p) {
    return (unsigned char *)(((uintptr_t)p + 255) & ~(uintptr_t)255);
}

__device__ inline void atomic_add_u64(u64 *p, u64 v) {
    if (v) atomicAdd(p, v);
}

// grid-stride helpers
#define GTID ((u64)blockIdx.x * blockDim.x + threadIdx.x)
#define GSTRIDE ((u64)gridDim.x * blockDim.x)
#define GWAVE (GTID / WAVE)
#define NWAVES (GSTRIDE / WAVE)
