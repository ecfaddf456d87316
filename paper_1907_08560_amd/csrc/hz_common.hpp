// hz_common.hpp -- shared device/host helpers of the GHSVD library (gfx950).
//
// Complex values live in HBM as interleaved (re, im) pairs: double2 for
// complex128, float2 for complex64.  All matrices are column-major.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ghsvd.h"

namespace ghsvd {

// ----------------------------------------------------------------------------
// Complex arithmetic on double2 / float2.
// ----------------------------------------------------------------------------
__host__ __device__ __forceinline__ double2 cmk(double r, double i) { return make_double2(r, i); }
__host__ __device__ __forceinline__ double2 cadd(double2 a, double2 b) { return cmk(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ double2 csub(double2 a, double2 b) { return cmk(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
    return cmk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ __forceinline__ double2 cconj(double2 a) { return cmk(a.x, -a.y); }
__host__ __device__ __forceinline__ double2 cscale(double2 a, double s) { return cmk(a.x * s, a.y * s); }
__host__ __device__ __forceinline__ double cnorm2(double2 a) { return a.x * a.x + a.y * a.y; }

__device__ __forceinline__ float2 fmk(float r, float i) { return make_float2(r, i); }

// ----------------------------------------------------------------------------
// Wavefront (64 lanes) and workgroup reductions, fixed order (deterministic).
// ----------------------------------------------------------------------------
constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Sums NV values over the workgroup; every thread gets the totals.  `lds`
// must hold NV * (blockDim.x / 64) doubles.  Contains two __syncthreads().
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k * nw + wid] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += lds[k * nw + w];
        v[k] = s;
    }
    __syncthreads();
}

// (value, index) argmax over the workgroup: largest value, smallest index on ties.
// `lds_v` / `lds_i` hold blockDim.x / 64 entries.  Every thread gets the result.
__device__ __forceinline__ void block_argmax(double &v, int &idx, double *lds_v, int *lds_i) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(v, off, kWave);
        const int oi = __shfl_xor(idx, off, kWave);
        if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
    }
    if (lane == 0) { lds_v[wid] = v; lds_i[wid] = idx; }
    __syncthreads();
    v = lds_v[0];
    idx = lds_i[0];
    for (int w = 1; w < nw; ++w) {
        const double ov = lds_v[w];
        const int oi = lds_i[w];
        if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
    }
    __syncthreads();
}

// ----------------------------------------------------------------------------
// Host helpers.
// ----------------------------------------------------------------------------
#define GHSVD_HIP(call)                                                   \
    do {                                                                  \
        hipError_t e_ = (call);                                           \
        if (e_ != hipSuccess) return GHSVD_EDEVICE;                       \
    } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over a caller workspace.
struct Carver {
    char *base;
    size_t used;
    size_t cap;
    template <typename T>
    T *take(size_t count) {
        used = align_up(used, 256);
        T *p = reinterpret_cast<T *>(base ? base + used : nullptr);
        used += count * sizeof(T);
        return p;
    }
    bool ok() const { return used <= cap; }
};

// Leading dimension (in complex elements) used for internal copies: rows
// rounded up to a multiple of 8 elements (128 bytes for complex128).
inline int pad_ld(int rows) { return (rows + 7) / 8 * 8; }

// Global-address-space view of a device array.  Kernels reach the matrices
// through pointers stored in descriptors, whose address space the compiler
// cannot see, so plain accesses become flat instructions; those also count
// against the LDS wait counter, which makes every wait for an LDS or
// cross-lane result wait for outstanding memory loads as well.  Accesses
// through GPtr are global (vector-memory) instructions.  Elements move as
// builtin vectors (the HIP vector types only support the generic address
// space).
#define GHSVD_GLOBAL __attribute__((address_space(1)))
typedef double gvec_d2 __attribute__((ext_vector_type(2)));
typedef float gvec_f2 __attribute__((ext_vector_type(2)));
template <typename T>
struct GVec {
    using type = T;
};
template <>
struct GVec<double2> {
    using type = gvec_d2;
};
template <>
struct GVec<float2> {
    using type = gvec_f2;
};
__device__ __forceinline__ double2 gv_from(gvec_d2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ float2 gv_from(gvec_f2 v) { return make_float2(v.x, v.y); }
template <typename T>
__device__ __forceinline__ T gv_from(T v) {
    return v;
}
__device__ __forceinline__ gvec_d2 gv_to(double2 t) {
    gvec_d2 v;
    v.x = t.x;
    v.y = t.y;
    return v;
}
__device__ __forceinline__ gvec_f2 gv_to(float2 t) {
    gvec_f2 v;
    v.x = t.x;
    v.y = t.y;
    return v;
}
template <typename T>
__device__ __forceinline__ T gv_to(T t) {
    return t;
}

template <typename T>
struct GPtr {
    using V = typename GVec<T>::type;
    GHSVD_GLOBAL V *p = nullptr;
    GPtr() = default;
    __device__ explicit GPtr(const T *q) : p((GHSVD_GLOBAL V *)(q)) {}
    __device__ GPtr operator+(long i) const {
        GPtr r;
        r.p = p + i;
        return r;
    }
    __device__ T ld(long i) const { return gv_from(p[i]); }
    __device__ void st(long i, const T &t) const { p[i] = gv_to(t); }
};

// The round-robin ordering: pair of slot k at step s for N (even) players
// (0 <= s < N - 1, 0 <= k < N / 2; the sums below stay within one period,
// so a conditional subtraction replaces the integer modulo).
__host__ __device__ __forceinline__ void rr_pair(int N, int s, int k, int &p, int &q) {
    int i, j;
    if (k == 0) {
        i = N - 1;
        j = s;
    } else {
        const int M = N - 1;
        i = s + k;
        if (i >= M) i -= M;
        j = s - k;
        if (j < 0) j += M;
    }
    p = i < j ? i : j;
    q = i < j ? j : i;
}

}  // namespace ghsvd
