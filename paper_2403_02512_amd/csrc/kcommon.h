// Device-side helpers shared by the HIP translation units of the qsv library:
// complex arithmetic on interleaved (re, im) pairs, index expansion (insert
// zero bits, paper Alg. 2), DPP wavefront reductions with a fixed summation
// order, and the per-device dynamic-LDS attribute.
#pragma once

#include <atomic>

#include "qsv_internal.h"

namespace qsv {

// Raise a kernel's dynamic-LDS limit to the CU's 160 KiB, once per device (the
// attribute is per device; `done` holds one bit per device id).
inline hipError_t allow_big_lds(const void* fn, std::atomic<uint64_t>& done) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = 1ull << (dev & 63);
    if (done.load() & bit) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess) done.fetch_or(bit);
    return e;
}

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * b + c
template <typename T>
__device__ __forceinline__ cx<T> cmad(cx<T> a, cx<T> b, cx<T> c) {
    return {c.re + a.re * b.re - a.im * b.im, c.im + a.re * b.im + a.im * b.re};
}
// Im(conj(l) * v) in FP64
template <typename T>
__device__ __forceinline__ double im_conj_mul(cx<T> l, cx<T> v) {
    return (double)l.re * (double)v.im - (double)l.im * (double)v.re;
}

// acc + Im(conj(l) v) as two fused multiply-adds
template <typename T>
__device__ __forceinline__ double acc_im_conj_mul(double acc, cx<T> l, cx<T> v) {
    return __builtin_fma((double)l.re, (double)v.im, __builtin_fma(-(double)l.im, (double)v.re, acc));
}

// Store of one amplitude.  nt: a non-temporal (streaming) store, which asks
// the caches not to keep the line: the state is written once per pass and
// not read again before it is evicted (the paper's streaming stores, Sec.
// 3.1).  nt is uniform across the launch, so the branch is a scalar one.
template <typename T>
__device__ __forceinline__ void st_amp(cx<T>* p, cx<T> v, bool nt) {
    if (nt) {
        typedef T V2 __attribute__((ext_vector_type(2)));
        V2 x;
        x.x = v.re;
        x.y = v.im;
        __builtin_nontemporal_store(x, reinterpret_cast<V2*>(p));
    } else {
        *p = v;
    }
}

__device__ __forceinline__ uint64_t expand_idx(uint64_t k, const Expand& e) {
    uint64_t r = k & e.m[0];
    for (int i = 1; i < e.nm; ++i) r |= (k << i) & e.m[i];
    return r;
}

// v of the lane `shift` below in the same 16-lane row (0 past the row start):
// DPP row_shr on both halves of the double, no LDS traffic
template <int SHIFT>
__device__ __forceinline__ double row_shr(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x110 + SHIFT, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x110 + SHIFT, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// The value of lane Q of this lane's group of four (DPP quad_perm broadcast).
template <int Q>
__device__ __forceinline__ double quad_lane(double v) {
    constexpr int ctrl = Q | (Q << 2) | (Q << 4) | (Q << 6);
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int Q>
__device__ __forceinline__ float quad_lane(float v) {
    constexpr int ctrl = Q | (Q << 2) | (Q << 4) | (Q << 6);
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctrl, 0xF, 0xF, false));
}

__device__ __forceinline__ double lane_value(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the 64 lanes (every lane active), returned to all lanes: in-row
// prefix sums by DPP leave each row's total in its lane 15; the four row
// totals are read as uniform values.  Fixed order, so reproducible.
__device__ __forceinline__ double wave_sum(double v) {
    v += row_shr<1>(v);
    v += row_shr<2>(v);
    v += row_shr<4>(v);
    v += row_shr<8>(v);
    return (lane_value(v, 15) + lane_value(v, 31)) + (lane_value(v, 47) + lane_value(v, 63));
}

// *p += v in LDS without waiting for the old value (ds_add_f64, no return):
// one lane per accumulator adds in program order, so the sum keeps its
// order and the result is reproducible; a barrier completes the adds.
__device__ __forceinline__ void lds_add(double* p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Adds the block-wide sum of v to *dst (one thread writes).  Every thread of
// the block must call it; fixed summation order, so results are reproducible.
__device__ __forceinline__ void block_add(double v, double* red, double* dst, int tid, int nthr) {
    if (nthr >= 64) {
        v = wave_sum(v);
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < (nthr >> 6); ++w) s += red[w];
            *dst += s;
        }
    } else {
        red[tid] = v;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < nthr; ++w) s += red[w];
            *dst += s;
        }
    }
    __syncthreads();
}

template <typename T>
struct M2T {
    cx<T> a, b, c, d;
};
template <typename T>
__device__ __forceinline__ M2T<T> to_t(const Mat2& m) {
    return {{(T)m.re[0], (T)m.im[0]}, {(T)m.re[1], (T)m.im[1]}, {(T)m.re[2], (T)m.im[2]}, {(T)m.re[3], (T)m.im[3]}};
}

}  // namespace qsv
