// HIP kernels of the qsv hot path for gfx950 (CDNA4, wave64).
//
//  k_init    psi = |basis>                                    (write-only stream)
//  k_gate1   2x2 on amplitude pairs at the target's bit stride, optionally
//            controlled (paper Alg. 1 / Alg. 2): classes dense, diagonal,
//            anti-diagonal
//  k_diag1   one phase on the amplitudes whose target and control bits are
//            fixed: PhaseShift/Z/S/T and their controlled forms scale only
//            the |1> amplitudes, so they read and write half the vector
//            (Sec. 2.1.1, Listing 1)
//  k_gate2   4x4 on amplitude quads (Ising gates, SWAP, Givens rotations);
//            k_gate2_lanes: one lane per amplitude when a target is among
//            the lowest index bits (quad exchange by DPP)
//  k_gatek   2^k x 2^k on 2^k-tuples, k = 3..5, one tuple per thread
//  k_tile    (k_tile.h, instantiated in tile_*.hip) LDS-staged pass: a tile
//            of 2^b amplitudes spanning b index bits (always including the
//            lowest ones, for coalescing) takes a whole list of gates,
//            diagonal phase layers and adjoint inner products per HBM round
//            trip; one or two vectors (phi, lambda)
//  k_pauli   Pauli-sum expectation value / lambda = H psi, FP64 accumulation
//            and wavefront-shuffle block reductions
//  k_reduce  deterministic FP64 reduction of per-block partials
//
// Index conventions: wire w is index bit n-1-w; matrix index bit k-1-i
// belongs to target i.
#include "kcommon.h"

namespace qsv {

const char* const kKernelNames[KK_COUNT] = {"init",  "gate1", "diag1",        "gate2",        "gatek", "tile1",
                                            "tile2", "pauli_expval", "pauli_lambda", "reduce", "copy",  "probs", "sparse_expval",
                                            "sample", "dense"};

// ------------------------------------------------------------------ init

template <typename T>
__global__ __launch_bounds__(256) void k_init(cx<T>* __restrict__ psi, uint64_t N, uint64_t basis) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        cx<T> v;
        v.re = i == basis ? T(1) : T(0);
        v.im = T(0);
        psi[i] = v;
    }
}

template <typename T>
hipError_t launch_init(hipStream_t s, void* psi, uint64_t N, uint64_t basis) {
    uint64_t blocks = (N + 1023) / 1024;
    if (blocks > (1u << 20)) blocks = 1u << 20;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(k_init<T>, dim3((unsigned)blocks), dim3(256), 0, s, (cx<T>*)psi, N, basis);
    return hipGetLastError();
}

// ------------------------------------------------------------------ single-qubit streaming kernels

constexpr int G1_ITEMS = 2;

template <typename T, int CLS>
__global__ __launch_bounds__(256) void k_gate1(cx<T>* __restrict__ psi, uint64_t n_items, Expand ex,
                                               uint64_t setmask, uint64_t tbit, Mat2 mat, int nt) {
    const M2T<T> m = to_t<T>(mat);
    const uint64_t k0 = (uint64_t)blockIdx.x * (256 * G1_ITEMS) + threadIdx.x;
    uint64_t i0[G1_ITEMS];
    cx<T> a0[G1_ITEMS], a1[G1_ITEMS];
#pragma unroll
    for (int r = 0; r < G1_ITEMS; ++r) {
        const uint64_t k = k0 + (uint64_t)r * 256;
        i0[r] = k < n_items ? (expand_idx(k, ex) | setmask) : ~0ull;
        if (k < n_items) {
            a0[r] = psi[i0[r]];
            a1[r] = psi[i0[r] | tbit];
        }
    }
#pragma unroll
    for (int r = 0; r < G1_ITEMS; ++r) {
        if (i0[r] == ~0ull) continue;
        cx<T> b0, b1;
        if (CLS == MC_DENSE) {
            b0 = cmad(m.a, a0[r], cmul(m.b, a1[r]));
            b1 = cmad(m.c, a0[r], cmul(m.d, a1[r]));
        } else if (CLS == MC_DIAG) {
            b0 = cmul(m.a, a0[r]);
            b1 = cmul(m.d, a1[r]);
        } else {  // anti-diagonal
            b0 = cmul(m.b, a1[r]);
            b1 = cmul(m.c, a0[r]);
        }
        st_amp(psi + i0[r], b0, nt);
        st_amp(psi + (i0[r] | tbit), b1, nt);
    }
}

template <typename T>
hipError_t launch_gate1(hipStream_t s, void* psi, uint64_t n_items, const Expand& ex, uint64_t setmask,
                        uint64_t tbit, int cls, const Mat2& m, bool nt) {
    const uint64_t blocks = (n_items + 256 * G1_ITEMS - 1) / (256 * G1_ITEMS);
    dim3 g((unsigned)blocks), b(256);
    if (cls == MC_DIAG)
        hipLaunchKernelGGL((k_gate1<T, MC_DIAG>), g, b, 0, s, (cx<T>*)psi, n_items, ex, setmask, tbit, m, (int)nt);
    else if (cls == MC_ANTI)
        hipLaunchKernelGGL((k_gate1<T, MC_ANTI>), g, b, 0, s, (cx<T>*)psi, n_items, ex, setmask, tbit, m, (int)nt);
    else
        hipLaunchKernelGGL((k_gate1<T, MC_DENSE>), g, b, 0, s, (cx<T>*)psi, n_items, ex, setmask, tbit, m, (int)nt);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void k_diag1(cx<T>* __restrict__ psi, uint64_t n_items, Expand ex,
                                               uint64_t setmask, double dre, double dim, int nt) {
    const cx<T> d = {(T)dre, (T)dim};
    const uint64_t k0 = (uint64_t)blockIdx.x * (256 * 4) + threadIdx.x;
    uint64_t idx[4];
    cx<T> a[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const uint64_t k = k0 + (uint64_t)r * 256;
        idx[r] = k < n_items ? (expand_idx(k, ex) | setmask) : ~0ull;
        if (k < n_items) a[r] = psi[idx[r]];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (idx[r] != ~0ull) st_amp(psi + idx[r], cmul(d, a[r]), nt);
}

template <typename T>
hipError_t launch_diag1(hipStream_t s, void* psi, uint64_t n_items, const Expand& ex, uint64_t setmask,
                        double dre, double dim, bool nt) {
    const uint64_t blocks = (n_items + 1023) / 1024;
    hipLaunchKernelGGL(k_diag1<T>, dim3((unsigned)blocks), dim3(256), 0, s, (cx<T>*)psi, n_items, ex, setmask,
                       dre, dim, (int)nt);
    return hipGetLastError();
}

// ------------------------------------------------------------------ two-qubit streaming kernel

template <typename T, int CLS>
__device__ __forceinline__ void gate2_quad(cx<T>* __restrict__ psi, uint64_t i, uint64_t b0, uint64_t b1,
                                           const Mat4& mat, int nt);

template <typename T, int CLS>
__global__ __launch_bounds__(256) void k_gate2(cx<T>* __restrict__ psi, uint64_t n_items, Expand ex,
                                               uint64_t setmask, uint64_t b0, uint64_t b1, Mat4 mat, int nt) {
    // grid-stride: a launch holds fewer than 2^32 threads
    for (uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x; k < n_items; k += (uint64_t)gridDim.x * 256)
        gate2_quad<T, CLS>(psi, expand_idx(k, ex) | setmask, b0, b1, mat, nt);
}

template <typename T, int CLS>
__device__ __forceinline__ void gate2_quad(cx<T>* __restrict__ psi, uint64_t i, uint64_t b0, uint64_t b1,
                                           const Mat4& mat, int nt) {
    const uint64_t idx[4] = {i, i | b1, i | b0, i | b0 | b1};
    if (CLS == MC_MID) {  // only |01>, |10> mix; |00>, |11> untouched
        const cx<T> x1 = psi[idx[1]], x2 = psi[idx[2]];
        const cx<T> m11 = {(T)mat.re[5], (T)mat.im[5]}, m12 = {(T)mat.re[6], (T)mat.im[6]};
        const cx<T> m21 = {(T)mat.re[9], (T)mat.im[9]}, m22 = {(T)mat.re[10], (T)mat.im[10]};
        st_amp(psi + idx[1], cmad(m11, x1, cmul(m12, x2)), nt);
        st_amp(psi + idx[2], cmad(m21, x1, cmul(m22, x2)), nt);
        return;
    }
    cx<T> a[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = psi[idx[j]];
    if (CLS == MC_DIAG) {
#pragma unroll
        for (int j = 0; j < 4; ++j) st_amp(psi + idx[j], cmul(cx<T>{(T)mat.re[j * 5], (T)mat.im[j * 5]}, a[j]), nt);
        return;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        cx<T> acc = {T(0), T(0)};
#pragma unroll
        for (int j = 0; j < 4; ++j) acc = cmad(cx<T>{(T)mat.re[r * 4 + j], (T)mat.im[r * 4 + j]}, a[j], acc);
        st_amp(psi + idx[r], acc, nt);
    }
}

// A matrix entry of the by-value kernel argument as a wave-uniform register
// value.  Selecting between such values per lane stays a register select; a
// select between the argument's own elements is turned into an indexed access,
// which copies the whole matrix to per-lane scratch memory.
__device__ __forceinline__ double uniform_value(double x) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double select4(int q, double a, double b, double c, double d) {
    const double lo = (q & 1) ? b : a, hi = (q & 1) ? d : c;
    return (q & 2) ? hi : lo;
}

// The same 4x4 update with one lane per amplitude: the four lanes of a DPP
// quad hold one quad's amplitudes (lane q: index bits b0 b1 = q >> 1, q & 1)
// and exchange them by quad_perm broadcasts.  For targets among the lowest
// index bits the quad-per-lane form strides its loads by the quad size
// (several passes over each cache line per instruction); here consecutive
// lanes read consecutive amplitudes.
template <typename T, int CLS>
__global__ __launch_bounds__(256) void k_gate2_lanes(cx<T>* __restrict__ psi, uint64_t n_items, Expand ex,
                                                     uint64_t setmask, uint64_t b0, uint64_t b1, Mat4 mat, int nt) {
    const int q = (int)(threadIdx.x & 3);
    // this lane's row of the matrix (row q; the diagonal entry only for a
    // diagonal matrix), built once
    constexpr int NJ = CLS == MC_DIAG ? 1 : 4;
    cx<T> row[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int c0 = CLS == MC_DIAG ? 0 : j, st = CLS == MC_DIAG ? 5 : 4;
        row[j] = {(T)select4(q, uniform_value(mat.re[c0]), uniform_value(mat.re[st + c0]),
                             uniform_value(mat.re[2 * st + c0]), uniform_value(mat.re[3 * st + c0])),
                  (T)select4(q, uniform_value(mat.im[c0]), uniform_value(mat.im[st + c0]),
                             uniform_value(mat.im[2 * st + c0]), uniform_value(mat.im[3 * st + c0]))};
    }
    // grid-stride (a launch holds fewer than 2^32 threads); the stride is a
    // multiple of 4, so a quad's four lanes share the item and leave together
    for (uint64_t gid = (uint64_t)blockIdx.x * 256 + threadIdx.x; (gid >> 2) < n_items;
         gid += (uint64_t)gridDim.x * 256) {
        const uint64_t i = expand_idx(gid >> 2, ex) | setmask | ((q & 2) ? b0 : 0) | ((q & 1) ? b1 : 0);
        const cx<T> v = psi[i];
        if constexpr (CLS == MC_DIAG) {
            st_amp(psi + i, cmul(row[0], v), nt);
        } else {
            // the quad's four amplitudes, broadcast from their lanes
            cx<T> acc = cmul(row[0], cx<T>{quad_lane<0>(v.re), quad_lane<0>(v.im)});
            acc = cmad(row[1], cx<T>{quad_lane<1>(v.re), quad_lane<1>(v.im)}, acc);
            acc = cmad(row[2], cx<T>{quad_lane<2>(v.re), quad_lane<2>(v.im)}, acc);
            acc = cmad(row[3], cx<T>{quad_lane<3>(v.re), quad_lane<3>(v.im)}, acc);
            st_amp(psi + i, acc, nt);
        }
    }
}

template <typename T>
hipError_t launch_gate2(hipStream_t s, void* psi, uint64_t n_items, const Expand& ex, uint64_t setmask, uint64_t b0,
                        uint64_t b1, int cls, const Mat4& m, bool nt) {
    const uint64_t blocks = std::min<uint64_t>((n_items + 255) / 256, 1u << 22);
    dim3 g((unsigned)blocks), b(256);
    // a target among the three lowest index bits (one cache line holds 8
    // complex128 amplitudes): one lane per amplitude
    const bool low = ((b0 | b1) & 7) != 0 && cls != MC_MID;
    if (low) {
        const uint64_t lanes = 4 * n_items;
        dim3 gl((unsigned)std::min<uint64_t>((lanes + 255) / 256, 1u << 22));
        if (cls == MC_DIAG)
            hipLaunchKernelGGL((k_gate2_lanes<T, MC_DIAG>), gl, b, 0, s, (cx<T>*)psi, n_items, ex, setmask, b0, b1,
                               m, (int)nt);
        else
            hipLaunchKernelGGL((k_gate2_lanes<T, MC_DENSE>), gl, b, 0, s, (cx<T>*)psi, n_items, ex, setmask, b0, b1,
                               m, (int)nt);
        return hipGetLastError();
    }
    if (cls == MC_MID)
        hipLaunchKernelGGL((k_gate2<T, MC_MID>), g, b, 0, s, (cx<T>*)psi, n_items, ex, setmask, b0, b1, m, (int)nt);
    else if (cls == MC_DIAG)
        hipLaunchKernelGGL((k_gate2<T, MC_DIAG>), g, b, 0, s, (cx<T>*)psi, n_items, ex, setmask, b0, b1, m, (int)nt);
    else
        hipLaunchKernelGGL((k_gate2<T, MC_DENSE>), g, b, 0, s, (cx<T>*)psi, n_items, ex, setmask, b0, b1, m,
                           (int)nt);
    return hipGetLastError();
}

// ------------------------------------------------------------------ k-qubit streaming kernel

struct TBits {
    int32_t tb[6];
};

template <typename T, int K>
__global__ __launch_bounds__(256) void k_gatek(cx<T>* __restrict__ psi, uint64_t n_items, Expand ex,
                                               uint64_t setmask, TBits tb, const cx<T>* __restrict__ mat, int nt) {
    constexpr int D = 1 << K;
    const uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= n_items) return;
    const uint64_t base = expand_idx(k, ex) | setmask;
    uint64_t off[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        uint64_t o = 0;
#pragma unroll
        for (int i = 0; i < K; ++i)
            if ((j >> (K - 1 - i)) & 1) o |= 1ull << tb.tb[i];
        off[j] = o;
    }
    cx<T> a[D];
#pragma unroll
    for (int j = 0; j < D; ++j) a[j] = psi[base | off[j]];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        cx<T> acc = {T(0), T(0)};
#pragma unroll
        for (int j = 0; j < D; ++j) acc = cmad(mat[r * D + j], a[j], acc);
        st_amp(psi + (base | off[r]), acc, nt);
    }
}

// Dense k-qubit matrix (k <= 6) whose targets all lie in the lowest six index
// bits: a wavefront owns an aligned chunk of 64 amplitudes, which holds whole
// tuples.  Every lane loads one amplitude (coalesced) into LDS and computes
// one output - the row given by its own target bits - from the tuple's
// inputs (LDS reads shared by the lanes of a tuple) and its matrix row (LDS,
// rows padded by one entry against bank conflicts).  Chunks are enumerated by
// ex / setmask over the index bits above bit 5 (controls there); controls in
// the chunk are per lane (lcm / lcv).
template <typename T>
__global__ __launch_bounds__(256) void k_gatek_low(cx<T>* __restrict__ psi, uint64_t n_chunks, Expand ex,
                                                   uint64_t setmask, TBits tb, int k, uint32_t lcm, uint32_t lcv,
                                                   const cx<T>* __restrict__ mat, int nt) {
    extern __shared__ __align__(16) unsigned char gk_smem[];
    const int dim = 1 << k, stride = dim + 1;
    cx<T>* m = reinterpret_cast<cx<T>*>(gk_smem);
    cx<T>* buf = m + dim * stride;
    for (int e = threadIdx.x; e < dim * dim; e += 256) m[(e / dim) * stride + (e % dim)] = mat[e];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t tmask = 0;
    int row = 0;
    for (int i = 0; i < k; ++i) {
        tmask |= 1u << tb.tb[i];
        row = (row << 1) | ((lane >> tb.tb[i]) & 1);
    }
    const uint32_t base_t = (uint32_t)lane & ~tmask;
    const bool on = ((uint32_t)lane & lcm) == lcv;
    cx<T>* wb = buf + wave * 64;
    const cx<T>* mr = m + row * stride;
    __syncthreads();
    // the block walks 4 chunks per step, one per wavefront, in lockstep
    for (uint64_t c0 = (uint64_t)blockIdx.x * 4; c0 < n_chunks; c0 += (uint64_t)gridDim.x * 4) {
        const uint64_t c = c0 + wave;
        const bool live = c < n_chunks;
        const uint64_t base = live ? ((expand_idx(c, ex) | setmask) << 6) : 0;
        if (live) wb[lane] = psi[base + lane];
        __syncthreads();
        if (live) {
            cx<T> acc = {T(0), T(0)};
            for (int j = 0; j < dim; ++j) {
                uint32_t o = base_t;
                for (int i = 0; i < k; ++i)
                    if ((j >> (k - 1 - i)) & 1) o |= 1u << tb.tb[i];
                acc = cmad(mr[j], wb[o], acc);
            }
            if (on) st_amp(psi + base + lane, acc, nt);
        }
        __syncthreads();
    }
}

template <typename T>
hipError_t launch_gatek_low(hipStream_t s, void* psi, uint64_t n_chunks, const Expand& ex, uint64_t setmask, int k,
                            const int32_t* tbits, uint32_t lcm, uint32_t lcv, const void* mat, bool nt) {
    if (k < 1 || k > 6) return hipErrorInvalidValue;
    TBits tb;
    for (int i = 0; i < 6; ++i) tb.tb[i] = i < k ? tbits[i] : 0;
    const int dim = 1 << k;
    const size_t lds = ((size_t)dim * (dim + 1) + 256) * sizeof(cx<T>);
    static std::atomic<uint64_t> lds_raised{0};
    if (lds > 65536) {
        hipError_t e = allow_big_lds((const void*)k_gatek_low<T>, lds_raised);
        if (e != hipSuccess) return e;
    }
    uint64_t blocks = (n_chunks + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_gatek_low<T>, dim3((unsigned)(blocks ? blocks : 1)), dim3(256), lds, s, (cx<T>*)psi,
                       n_chunks, ex, setmask, tb, k, lcm, lcv, (const cx<T>*)mat, (int)nt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gatek(hipStream_t s, void* psi, uint64_t n_items, const Expand& ex, uint64_t setmask, int k,
                        const int32_t* tbits, const void* mat, bool nt) {
    TBits tb;
    for (int i = 0; i < 6; ++i) tb.tb[i] = i < k ? tbits[i] : 0;
    const uint64_t blocks = (n_items + 255) / 256;
    dim3 g((unsigned)blocks), b(256);
    const cx<T>* m = (const cx<T>*)mat;
    switch (k) {
    case 3: hipLaunchKernelGGL((k_gatek<T, 3>), g, b, 0, s, (cx<T>*)psi, n_items, ex, setmask, tb, m, (int)nt); break;
    case 4: hipLaunchKernelGGL((k_gatek<T, 4>), g, b, 0, s, (cx<T>*)psi, n_items, ex, setmask, tb, m, (int)nt); break;
    case 5: hipLaunchKernelGGL((k_gatek<T, 5>), g, b, 0, s, (cx<T>*)psi, n_items, ex, setmask, tb, m, (int)nt); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ dense k-qubit matrices, LDS-staged

// A dense 2^K x 2^K matrix (K = 3..6) on any K target bits.  A tile is the
// 2^(K+6) amplitudes that agree outside the targets and the six lowest index
// bits that are neither targets nor controls (the lane bits): 64 tuples of
// 2^K amplitudes.  Controls always lie outside the tile and are enumerated by
// ex / setmask, so no lane tests a control.
//
//  load:    the tile in ascending tile-bit order (global order, so loads are
//           coalesced runs) into LDS at c = (j << 6) | l for element j of
//           tuple l, with one pad slot per 64 (address c + (c >> 6)), which
//           keeps both the load's and the compute's LDS accesses conflict-free
//           whichever bits are targets;
//  compute: wave w of the NT / 64 waves takes rows [w R, (w+1) R) of every
//           tuple, R = 2^K / (NT / 64), lane = tuple: each input read from
//           LDS feeds R complex MACs whose matrix entries are wave-uniform
//           (scalar loads).  The host stores the matrix as (wave, column j,
//           row) so a wave's entries for one input are contiguous, and the
//           next column's input and entries are fetched before the current
//           column's MACs, so their latency hides behind the arithmetic;
//  store:   outputs back to LDS, then coalesced stores.
// FLOPs per amplitude 8 * 2^K: memory-bound up to K = 5 in complex128 and
// FP64-ALU-bound at K = 6, which runs 512 threads (four waves per SIMD with
// two blocks per CU, so at most 128 VGPRs) to keep the FMA pipes fed.
template <typename T, int K, int NT>
__global__ __launch_bounds__(NT, 4) void k_dense(cx<T>* __restrict__ psi, const DenseArgs a,
                                                         const cx<T>* __restrict__ mat, int nt) {
    constexpr int D = 1 << K;          // tuple size
    constexpr int NW = NT / 64;        // waves
    constexpr int RW = D / NW;         // rows per wave
    constexpr int NE = D * 64;         // tile elements
    constexpr int RL = NE / NT;        // elements per thread in load / store
    constexpr int LB = NT == 512 ? 9 : 8;
    extern __shared__ __align__(16) unsigned char dn_smem[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(dn_smem);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // the thread's load/store slots: tile-local index tid + r * NT; both maps
    // (to the global offset and to the compact LDS index) are bit deposits,
    // linear over GF(2), so the tid part and the r part combine by OR
    uint64_t goff = 0;
    uint32_t coff = 0;
#pragma unroll
    for (int i = 0; i < LB; ++i)
        if ((tid >> i) & 1) {
            goff |= 1ull << a.sb[i];
            coff |= 1u << a.cb[i];
        }
    const cx<T>* mw = mat + (size_t)wave * D * RW;
    for (uint64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        const uint64_t base = expand_idx(tile, a.outer) | a.setmask;
        constexpr int LC = RL < 4 ? RL : 4;  // loads in flight per thread per chunk
#pragma unroll
        for (int r0 = 0; r0 < RL; r0 += LC) {
            cx<T> v[LC];
#pragma unroll
            for (int r = 0; r < LC; ++r) v[r] = psi[base | goff | a.goff_hi[r0 + r]];
#pragma unroll
            for (int r = 0; r < LC; ++r) {
                const uint32_t c = coff | a.coff_hi[r0 + r];
                lds[c + (c >> 6)] = v[r];
            }
        }
        __syncthreads();
        cx<T> acc[RW];
#pragma unroll
        for (int q = 0; q < RW; ++q) acc[q] = {T(0), T(0)};
        cx<T> x = lds[lane];
        cx<T> m[RW];
#pragma unroll
        for (int q = 0; q < RW; ++q) m[q] = mw[q];
        for (int j = 0; j < D; ++j) {
            // next column's input and entries first (the last fetch re-reads
            // column D - 1, in bounds, unused)
            const int jn = j + 1 < D ? j + 1 : j;
            const cx<T> xn = lds[(jn << 6) + lane + jn];
            cx<T> mn[RW];
#pragma unroll
            for (int q = 0; q < RW; ++q) mn[q] = mw[(size_t)jn * RW + q];
#pragma unroll
            for (int q = 0; q < RW; ++q) acc[q] = cmad(m[q], x, acc[q]);
            x = xn;
#pragma unroll
            for (int q = 0; q < RW; ++q) m[q] = mn[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            const int row = wave * RW + q;
            lds[(row << 6) + lane + row] = acc[q];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const uint32_t c = coff | a.coff_hi[r];
            st_amp(psi + (base | goff | a.goff_hi[r]), lds[c + (c >> 6)], nt);
        }
        __syncthreads();
    }
}

// The 6-qubit complex128 case on the FP64 matrix cores: the tile's product
// OUT[r][t] = sum_j M[r][j] X[j][t] (64 rows, 64 tuples, 64 columns) as real
// 16x16x4 products, Re += Mr Xr - Mi Xi and Im += Mr Xi + Mi Xr.  Wave w of
// 8 owns the 16-row block w / 2 and the 32 tuples of half w % 2; its A
// operands (its 16 rows of Mr and Mi, one double per lane per 4-column step)
// stay in registers for the whole launch, the B operands (X, one complex per
// lane per step and tuple block) come from the same padded LDS layout as the
// vector form, and the accumulators hold 16 x 16 blocks (four doubles per
// lane).  Operand layout of v_mfma_f64_16x16x4f64, wave64: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and receives D[4 (l / 16) + v][l % 16]
// in element v of its accumulator.  Load, layout and store are those of
// k_dense<double, 6, 512>; the matrix is read from the same per-wave layout.
typedef double v4d __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(512, 2) void k_dense6_mfma(cx<double>* __restrict__ psi, const DenseArgs a,
                                                        const cx<double>* __restrict__ mat, int nt) {
    constexpr int D = 64, NT = 512, RW = 8, RL = 8, LB = 9;
    extern __shared__ __align__(16) unsigned char dm_smem[];
    cx<double>* lds = reinterpret_cast<cx<double>*>(dm_smem);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rb = wave >> 1, th = wave & 1;
    uint64_t goff = 0;
    uint32_t coff = 0;
#pragma unroll
    for (int i = 0; i < LB; ++i)
        if ((tid >> i) & 1) {
            goff |= 1ull << a.sb[i];
            coff |= 1u << a.cb[i];
        }
    // A operands for the whole launch: M[16 rb + lane % 16][4 s + lane / 16];
    // row r, column j sits at ((r / RW) * D + j) * RW + r % RW
    double ar[16], ai[16];
    {
        const int r = 16 * rb + (lane & 15);
#pragma unroll
        for (int st = 0; st < 16; ++st) {
            const int j = 4 * st + (lane >> 4);
            const cx<double> m = mat[((size_t)(r / RW) * D + j) * RW + (r % RW)];
            ar[st] = m.re;
            ai[st] = m.im;
        }
    }
    for (uint64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        const uint64_t base = expand_idx(tile, a.outer) | a.setmask;
#pragma unroll
        for (int r0 = 0; r0 < RL; r0 += 4) {
            cx<double> v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = psi[base | goff | a.goff_hi[r0 + r]];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t c = coff | a.coff_hi[r0 + r];
                lds[c + (c >> 6)] = v[r];
            }
        }
        __syncthreads();
        v4d cre[2], cim[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            cre[b] = v4d{0.0, 0.0, 0.0, 0.0};
            cim[b] = v4d{0.0, 0.0, 0.0, 0.0};
        }
#pragma unroll
        for (int st = 0; st < 16; ++st) {
            const int k = 4 * st + (lane >> 4);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int t = 32 * th + 16 * b + (lane & 15);
                const cx<double> x = lds[k * 65 + t];
                cre[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[st], x.re, cre[b], 0, 0, 0);
                cre[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[st], -x.im, cre[b], 0, 0, 0);
                cim[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[st], x.im, cim[b], 0, 0, 0);
                cim[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[st], x.re, cim[b], 0, 0, 0);
            }
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // accumulator element v of lane l is D[4 v + l / 16][l % 16]
                const int r = 16 * rb + 4 * v + (lane >> 4), t = 32 * th + 16 * b + (lane & 15);
                lds[r * 65 + t] = cx<double>{cre[b][v], cim[b][v]};
            }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RL; ++r) {
            const uint32_t c = coff | a.coff_hi[r];
            st_amp(psi + (base | goff | a.goff_hi[r]), lds[c + (c >> 6)], nt);
        }
        __syncthreads();
    }
}

size_t dense_lds_bytes(int k, int elem_bytes) { return (size_t)(64 << k) * 65 / 64 * elem_bytes; }

template <typename T>
hipError_t launch_dense(hipStream_t s, void* psi, const DenseArgs& a, const void* mat, bool nt, bool mfma) {
    const size_t lds = dense_lds_bytes(a.k, (int)sizeof(cx<T>));
    uint64_t blocks = a.n_tiles < 4096 ? a.n_tiles : 4096;
    if (blocks == 0) return hipSuccess;
    if constexpr (sizeof(T) == 8) {
        if (mfma && a.k == 6) {
            static std::atomic<uint64_t> mf_raised{0};
            hipError_t e = allow_big_lds((const void*)k_dense6_mfma, mf_raised);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_dense6_mfma, dim3((unsigned)blocks), dim3(512), lds, s, (cx<double>*)psi, a,
                               (const cx<double>*)mat, (int)nt);
            return hipGetLastError();
        }
    }
    const cx<T>* m = (const cx<T>*)mat;
    static std::atomic<uint64_t> lds_raised{0};
#define QSV_DN(KV, NTV)                                                                                          \
    {                                                                                                            \
        if (lds > 65536) {                                                                                       \
            hipError_t e = allow_big_lds((const void*)k_dense<T, KV, NTV>, lds_raised);                         \
            if (e != hipSuccess) return e;                                                                       \
        }                                                                                                        \
        hipLaunchKernelGGL((k_dense<T, KV, NTV>), dim3((unsigned)blocks), dim3(NTV), lds, s, (cx<T>*)psi, a, m, \
                           (int)nt);                                                                             \
    }                                                                                                            \
    break;
    switch (a.k) {
    case 3: QSV_DN(3, 256)
    case 4: QSV_DN(4, 256)
    case 5: QSV_DN(5, 256)
    case 6: QSV_DN(6, 512)
    default: return hipErrorInvalidValue;
    }
#undef QSV_DN
    return hipGetLastError();
}

int dense_threads(int k) { return k == 6 ? 512 : 256; }

// ------------------------------------------------------------------ tile passes (tile_*.hip)

int tile_lds_bytes(int b, bool two, int elem_bytes, int nslots, int zt_n, int n_zop, int n_outer) {
    const int nthr = 1 << (b < 8 ? b : 8);
    const int nacc = nthr >= 64 ? nthr / 16 : 1;
    const int acc = ((64 + nslots * nacc) * 8 + 15) & ~15;
    // grouped Z-parity ops: per-op columns of the tile-number bits and the
    // current tile's parity bits (8-byte words after the phase tables)
    const int zt = (zt_n * elem_bytes + 7) & ~7;
    return (two ? 2 : 1) * (1 << b) * elem_bytes + acc + zt + n_zop * (n_outer + 1) * 8;
}

template <typename T>
hipError_t launch_tile(hipStream_t s, bool two, bool generic, const void* phi_src, void* phi, void* lam,
                       const TileArgs& a, const TOp* ops, const void* coef, const uint64_t* words, double* partials,
                       int grid, int nthr, int R, size_t lds_bytes) {
    if (two)
        return launch_tile_v<T, true>(s, generic, phi_src, phi, lam, a, ops, coef, words, partials, grid, nthr, R,
                                      lds_bytes);
    return launch_tile_v<T, false>(s, generic, phi_src, phi, lam, a, ops, coef, words, partials, grid, nthr, R,
                                   lds_bytes);
}

template <typename T>
hipError_t launch_tile_batch(hipStream_t s, bool two, bool generic, const TileEntry* entries,
                             const int32_t* blk_entry, const TileArgs* args, const TOp* ops, const void* coef,
                             const uint64_t* words, double* partials, int blocks, int nthr, int R, size_t lds) {
    if (two)
        return launch_tile_batch_v<T, true>(s, generic, entries, blk_entry, args, ops, coef, words, partials, blocks,
                                            nthr, R, lds);
    return launch_tile_batch_v<T, false>(s, generic, entries, blk_entry, args, ops, coef, words, partials, blocks,
                                         nthr, R, lds);
}

// ------------------------------------------------------------------ Pauli sums

// (P psi)_i = i^{nY} (-1)^{popcount((i ^ x) & z)} psi_{i ^ x}; terms sharing
// an x mask share the load of psi_{i ^ x}.  Accumulation in FP64.
//
// Groups flagged with a table slot (at most two per observable, chosen by the
// host for many-term groups) skip the term loop: the parity vector of the
// source index s = i ^ x is linear over GF(2) in s, so for the grid-stride
// index i = base0 + it * stride it is (the thread's constant part) XOR (the
// iteration's uniform part), each an XOR of per-bit columns; the group's
// weight is then the sum of one 256-entry table lookup per byte of it.

// Table state of one block: LDS offsets, parity columns and the thread's
// constant parity part of (up to) two table groups.
// Two table slots, as named fields: the slot of a group is a runtime value,
// and an array indexed by it would live in per-lane scratch memory.
struct LutState {
    int nslot;
    int toff0, toff1;                   // the slots' table offsets in LDS
    const uint64_t* cols0;              // per index bit: its parity part
    const uint64_t* cols1;
    uint64_t pthr0, pthr1;              // this thread's parity parts
};
struct LutIter {
    uint64_t p0, p1;  // the iteration's parity parts of slots 0 and 1
};

// Copy the observable's byte tables into LDS and set up the parity parts for
// the block's first index base0 (every thread must call it; ends with a
// barrier).
__device__ __forceinline__ void lut_setup(LutState& L, const PauliGroupDev* __restrict__ groups, int n_groups,
                                          const uint64_t* __restrict__ aux, cx<double>* tabs, uint64_t base0) {
    L.nslot = 0;
    L.toff0 = L.toff1 = 0;
    L.cols0 = L.cols1 = nullptr;
    L.pthr0 = L.pthr1 = 0;
    int tot = 0;
    for (int g = 0; g < n_groups; ++g) {
        const PauliGroupDev gr = groups[g];
        if (gr.lut < 0) continue;
        const cx<double>* src = reinterpret_cast<const cx<double>*>(aux + gr.lut_off);
        for (int e = threadIdx.x; e < gr.nb * 256; e += blockDim.x) tabs[tot * 256 + e] = src[e];
        const uint64_t* cl = aux + gr.col_off;
        uint64_t p = 0;
        const uint64_t s0 = base0 ^ gr.x;  // the source index without the iteration's bits
        for (int k = 0; k < 64; ++k)
            if ((s0 >> k) & 1) p ^= cl[k];
        if (gr.lut & 1) {
            L.toff1 = tot * 256;
            L.cols1 = cl;
            L.pthr1 = p;
        } else {
            L.toff0 = tot * 256;
            L.cols0 = cl;
            L.pthr0 = p;
        }
        tot += gr.nb;
        ++L.nslot;
    }
    __syncthreads();
}

// Weight sum_t w_t (-1)^{parity(src & z_t)} of one group at source index src
// (it: the iteration's parity parts of the table groups).
template <typename T>
__device__ __forceinline__ void group_weight(const PauliGroupDev& gr, uint64_t src,
                                             const PauliTermDev* __restrict__ terms, const LutState& L,
                                             const cx<double>* tabs, const LutIter& it, double& sr,
                                             double& si) {
    sr = 0.0;
    si = 0.0;
    if (gr.lut >= 0) {
        const bool s1 = gr.lut & 1;
        const uint64_t p = s1 ? (L.pthr1 ^ it.p1) : (L.pthr0 ^ it.p0);
        const cx<double>* tb = tabs + (s1 ? L.toff1 : L.toff0);
        for (int b = 0; b < gr.nb; ++b) {
            const cx<double> e = tb[b * 256 + (int)((p >> (8 * b)) & 255)];
            sr += e.re;
            si += e.im;
        }
    } else {
        for (int t = gr.t0; t < gr.t0 + gr.nt; ++t) {
            const PauliTermDev tm = terms[t];
            const bool neg = __popcll(src & tm.z) & 1;
            sr += neg ? -tm.wre : tm.wre;
            si += neg ? -tm.wim : tm.wim;
        }
    }
}

// (H psi)_i accumulated over the observable's groups.  The gathers psi[i ^ x]
// of four groups are issued before any of them is used, so their latencies
// overlap (observables of many single-term groups are gather-latency bound).
template <typename T>
__device__ __forceinline__ void pauli_row(const cx<T>* __restrict__ psi, uint64_t i, cx<T> pi,
                                          const PauliGroupDev* __restrict__ groups, int n_groups,
                                          const PauliTermDev* __restrict__ terms, const LutState& L,
                                          const cx<double>* tabs, const LutIter& it, double& ar, double& ai) {
    ar = 0.0;
    ai = 0.0;
    constexpr int U = 4;
    int g = 0;
    for (; g + U <= n_groups; g += U) {
        cx<T> ps[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t x = groups[g + u].x;
            ps[u] = x ? psi[i ^ x] : pi;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const PauliGroupDev gr = groups[g + u];
            double sr, si;
            group_weight<T>(gr, i ^ gr.x, terms, L, tabs, it, sr, si);
            ar += sr * (double)ps[u].re - si * (double)ps[u].im;
            ai += sr * (double)ps[u].im + si * (double)ps[u].re;
        }
    }
    for (; g < n_groups; ++g) {
        const PauliGroupDev gr = groups[g];
        const cx<T> ps = gr.x ? psi[i ^ gr.x] : pi;
        double sr, si;
        group_weight<T>(gr, i ^ gr.x, terms, L, tabs, it, sr, si);
        ar += sr * (double)ps.re - si * (double)ps.im;
        ai += sr * (double)ps.im + si * (double)ps.re;
    }
}

// the iteration's uniform parity parts: columns of the iteration's bits
__device__ __forceinline__ LutIter lut_iter(const LutState& L, uint64_t it, int lstride) {
    LutIter o = {0, 0};
    if (L.cols0)
        for (uint64_t r = it; r; r &= r - 1) o.p0 ^= L.cols0[lstride + __ffsll((unsigned long long)r) - 1];
    if (L.cols1)
        for (uint64_t r = it; r; r &= r - 1) o.p1 ^= L.cols1[lstride + __ffsll((unsigned long long)r) - 1];
    return o;
}

// One thread's share of an observable sweep: indices base0, base0 + stride,
// ... below N.  The diagonal loads psi[i] of U indices are issued together
// (one 16-byte load per index would leave the sweep latency bound), then the
// rows are formed in index order, so the sums keep their order.
template <typename T, bool WRITE, bool NORM2>
__device__ __forceinline__ void pauli_sweep(const cx<T>* __restrict__ psi, cx<T>* __restrict__ lam, uint64_t N,
                                            uint64_t base0, uint64_t stride, int lstride,
                                            const PauliGroupDev* __restrict__ groups, int n_groups,
                                            const PauliTermDev* __restrict__ terms, const LutState& L,
                                            const cx<double>* tabs, double& dot, double& nrm) {
    constexpr int U = 4;
    auto row = [&](uint64_t i, uint64_t it, cx<T> pi) {
        const LutIter itp = lut_iter(L, it, lstride);
        double ar, ai;
        pauli_row<T>(psi, i, pi, groups, n_groups, terms, L, tabs, itp, ar, ai);
        if (WRITE) lam[i] = cx<T>{(T)ar, (T)ai};
        dot += (double)pi.re * ar + (double)pi.im * ai;
        if (NORM2) nrm += ar * ar + ai * ai;
    };
    uint64_t i = base0, it = 0;
    for (; i + (U - 1) * stride < N; i += U * stride, it += U) {
        cx<T> pv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) pv[u] = psi[i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) row(i + u * stride, it + u, pv[u]);
    }
    for (; i < N; i += stride, ++it) row(i, it, psi[i]);
}

template <typename T, bool WRITE, bool NORM2>
__global__ __launch_bounds__(256) void k_pauli(const cx<T>* __restrict__ psi, cx<T>* __restrict__ lam, uint64_t N,
                                               const PauliGroupDev* __restrict__ groups, int n_groups,
                                               const PauliTermDev* __restrict__ terms,
                                               const uint64_t* __restrict__ aux, double* __restrict__ partials) {
    __shared__ double red[64];
    extern __shared__ __align__(16) unsigned char pauli_smem[];
    cx<double>* tabs = reinterpret_cast<cx<double>*>(pauli_smem);
    const uint64_t base0 = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * 256;  // a power of two
    const int lstride = __ffsll((unsigned long long)stride) - 1;
    LutState L;
    lut_setup(L, groups, n_groups, aux, tabs, base0);
    double dot = 0.0, nrm = 0.0;
    pauli_sweep<T, WRITE, NORM2>(psi, lam, N, base0, stride, lstride, groups, n_groups, terms, L, tabs, dot, nrm);
    double tot = 0.0;
    block_add(dot, red, &tot, threadIdx.x, 256);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
    if (NORM2) {  // ||H psi||^2 for the variance
        double t2 = 0.0;
        block_add(nrm, red, &t2, threadIdx.x, 256);
        if (threadIdx.x == 0) partials[gridDim.x + blockIdx.x] = t2;
    }
}

int pauli_grid(uint64_t N) {
    uint64_t g = (N + 255) / 256;
    if (g > 4096) g = 4096;
    return (int)(g ? g : 1);
}

template <typename T>
hipError_t launch_pauli(hipStream_t s, bool write_lambda, bool norm2, const void* psi, void* lam, uint64_t N,
                        const PauliGroupDev* groups, int n_groups, const PauliTermDev* terms, const uint64_t* aux,
                        int lut_tables, double* partials, int grid) {
    const size_t lds = (size_t)lut_tables * 256 * sizeof(cx<double>);
    if (norm2)
        hipLaunchKernelGGL((k_pauli<T, false, true>), dim3(grid), dim3(256), lds, s, (const cx<T>*)psi, (cx<T>*)lam,
                           N, groups, n_groups, terms, aux, partials);
    else if (write_lambda)
        hipLaunchKernelGGL((k_pauli<T, true, false>), dim3(grid), dim3(256), lds, s, (const cx<T>*)psi, (cx<T>*)lam,
                           N, groups, n_groups, terms, aux, partials);
    else
        hipLaunchKernelGGL((k_pauli<T, false, false>), dim3(grid), dim3(256), lds, s, (const cx<T>*)psi,
                           (cx<T>*)lam, N, groups, n_groups, terms, aux, partials);
    return hipGetLastError();
}

// Batched Pauli sums: block b serves entry blk_entry[2b] (one circuit) as its
// block blk_entry[2b + 1], with that circuit's byte tables (if any) in LDS.
template <typename T, bool WRITE>
__global__ __launch_bounds__(256) void k_pauli_batch(const PauliEntry* __restrict__ entries,
                                                     const int32_t* __restrict__ blk_entry,
                                                     const PauliGroupDev* __restrict__ groups,
                                                     const PauliTermDev* __restrict__ terms,
                                                     const uint64_t* __restrict__ aux,
                                                     double* __restrict__ partials) {
    __shared__ double red[64];
    extern __shared__ __align__(16) unsigned char pauli_smem[];
    cx<double>* tabs = reinterpret_cast<cx<double>*>(pauli_smem);
    const PauliEntry& en = entries[blk_entry[2 * blockIdx.x]];
    const cx<T>* __restrict__ psi = (const cx<T>*)en.psi;
    cx<T>* __restrict__ lam = (cx<T>*)en.lam;
    const uint64_t blk = (uint64_t)blk_entry[2 * blockIdx.x + 1];
    const PauliGroupDev* gp = groups + en.g0;
    const uint64_t base0 = blk * 256 + threadIdx.x;
    const uint64_t stride = (uint64_t)en.nblk * 256;  // a power of two
    const int lstride = __ffsll((unsigned long long)stride) - 1;
    LutState L;
    lut_setup(L, gp, en.ng, aux, tabs, base0);
    double dot = 0.0, nrm = 0.0;
    pauli_sweep<T, WRITE, false>(psi, lam, en.N, base0, stride, lstride, gp, en.ng, terms, L, tabs, dot, nrm);
    double tot = 0.0;
    block_add(dot, red, &tot, threadIdx.x, 256);
    if (threadIdx.x == 0) partials[en.part_off + blk] = tot;
}

template <typename T>
hipError_t launch_pauli_batch(hipStream_t s, bool write_lambda, const PauliEntry* entries, const int32_t* blk_entry,
                              const PauliGroupDev* groups, const PauliTermDev* terms, const uint64_t* aux,
                              int lut_tables, double* partials, int blocks) {
    const size_t lds = (size_t)lut_tables * 256 * sizeof(cx<double>);
    if (write_lambda)
        hipLaunchKernelGGL((k_pauli_batch<T, true>), dim3(blocks), dim3(256), lds, s, entries, blk_entry, groups,
                           terms, aux, partials);
    else
        hipLaunchKernelGGL((k_pauli_batch<T, false>), dim3(blocks), dim3(256), lds, s, entries, blk_entry, groups,
                           terms, aux, partials);
    return hipGetLastError();
}

// ------------------------------------------------------------------ marginal probabilities

// Block (x, y) sums |psi_i|^2 over its share of the indices whose measured
// wires hold bin (bin0 + y): i = (rest with zeros at the measured bits) | binbits.
template <typename T>
__global__ __launch_bounds__(256) void k_probs(const cx<T>* __restrict__ psi, uint64_t n_rest, Expand ex,
                                               const uint64_t* __restrict__ binbits, int bin0,
                                               double* __restrict__ partials) {
    __shared__ double red[64];
    const int bin = bin0 + (int)blockIdx.y;
    const uint64_t bb = binbits[bin];
    double sum = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x; r < n_rest; r += stride) {
        const cx<T> a = psi[expand_idx(r, ex) | bb];
        sum += (double)a.re * a.re + (double)a.im * a.im;
    }
    double tot = 0.0;
    block_add(sum, red, &tot, threadIdx.x, 256);
    if (threadIdx.x == 0) partials[(uint64_t)bin * gridDim.x + blockIdx.x] = tot;
}

template <typename T>
hipError_t launch_probs(hipStream_t s, const void* psi, uint64_t n_rest, const Expand& ex, const uint64_t* binbits,
                        int n_bins, int gx, double* partials) {
    for (int b0 = 0; b0 < n_bins; b0 += 32768) {
        const int nb = n_bins - b0 < 32768 ? n_bins - b0 : 32768;
        hipLaunchKernelGGL(k_probs<T>, dim3(gx, nb), dim3(256), 0, s, (const cx<T>*)psi, n_rest, ex, binbits, b0,
                           partials);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------------------ shot sampling

// |psi|^2 summed over each chunk of 2^clog2 amplitudes (one block per chunk).
template <typename T>
__global__ __launch_bounds__(256) void k_chunk_norms(const cx<T>* __restrict__ psi, int clog2,
                                                     double* __restrict__ sums) {
    __shared__ double red[64];
    const uint64_t len = 1ull << clog2, base = (uint64_t)blockIdx.x << clog2;
    double s = 0.0;
    for (uint64_t j = threadIdx.x; j < len; j += 256) {
        const cx<T> a = psi[base + j];
        s += (double)a.re * a.re + (double)a.im * a.im;
    }
    double tot = 0.0;
    block_add(s, red, &tot, threadIdx.x, 256);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One wavefront per sample: inside chunk chunk[k], the first index whose
// running |psi|^2 sum exceeds resid[k].  Lanes own consecutive segments; a
// lane-ordered prefix over the segment totals picks the segment, whose lane
// then walks it.  Where rounding leaves no index above resid, the last
// amplitude with non-zero probability of the last non-empty segment is taken,
// so only indices of non-zero probability are ever returned.
template <typename T>
__global__ __launch_bounds__(256) void k_sample(const cx<T>* __restrict__ psi, int clog2,
                                                const int64_t* __restrict__ chunk, const double* __restrict__ resid,
                                                uint64_t* __restrict__ out, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= n) return;  // uniform per wavefront
    const uint64_t len = 1ull << clog2;
    const uint64_t seg = len >= 64 ? len >> 6 : 1;
    const uint64_t base = (uint64_t)chunk[k] << clog2;
    const uint64_t lo = (uint64_t)lane * seg;
    double s = 0.0;
    if (lo < len)
        for (uint64_t j = 0; j < seg; ++j) {
            const cx<T> a = psi[base + lo + j];
            s += (double)a.re * a.re + (double)a.im * a.im;
        }
    double incl = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    double excl = __shfl_up(incl, 1, 64);
    if (lane == 0) excl = 0.0;
    const double r = resid[k];
    const uint64_t hit = __ballot(incl > r);
    int pick;
    if (hit) {
        pick = __ffsll((unsigned long long)hit) - 1;
    } else {
        const uint64_t nz = __ballot(s > 0.0);
        pick = nz ? 63 - __clzll((long long)nz) : 0;
    }
    if (lane == pick) {
        double acc = excl;
        uint64_t idx = lo, last_nz = lo;
        bool found = false;
        for (uint64_t j = 0; j < seg && lo + j < len; ++j) {
            const cx<T> a = psi[base + lo + j];
            const double p = (double)a.re * a.re + (double)a.im * a.im;
            if (p > 0.0) last_nz = lo + j;
            acc += p;
            if (acc > r) {
                idx = lo + j;
                found = true;
                break;
            }
        }
        out[k] = base + (found ? idx : last_nz);
    }
}

template <typename T>
hipError_t launch_chunk_norms(hipStream_t s, const void* psi, int clog2, uint64_t n_chunks, double* sums) {
    hipLaunchKernelGGL(k_chunk_norms<T>, dim3((unsigned)n_chunks), dim3(256), 0, s, (const cx<T>*)psi, clog2, sums);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sample(hipStream_t s, const void* psi, int clog2, const int64_t* chunk, const double* resid,
                         uint64_t* out, int64_t n) {
    const int64_t blocks = (n + 3) / 4;
    for (int64_t b0 = 0; b0 < blocks; b0 += (1 << 30)) {
        const int64_t nb = blocks - b0 < (1 << 30) ? blocks - b0 : (1 << 30);
        const int64_t k0 = b0 * 4;
        hipLaunchKernelGGL(k_sample<T>, dim3((unsigned)nb), dim3(256), 0, s, (const cx<T>*)psi, clog2, chunk + k0,
                           resid + k0, out + k0, n - k0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------------------ sparse Hamiltonian

// <psi|S|psi> for a CSR matrix S (rows = basis indices): one row per thread,
// FP64 accumulation of conj(psi_i) * sum_j S_ij psi_j; real and imaginary
// block partials at partials[b] and partials[grid + b].
template <typename T>
__global__ __launch_bounds__(256) void k_sparse(const cx<T>* __restrict__ psi, uint64_t N,
                                                const int64_t* __restrict__ row_ptr,
                                                const int64_t* __restrict__ col,
                                                const double* __restrict__ val, double* __restrict__ partials) {
    __shared__ double red[64];
    double sr = 0.0, si = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += stride) {
        double vr = 0.0, vi = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            const cx<T> a = psi[col[k]];
            const double mr = val[2 * k], mi = val[2 * k + 1];
            vr += mr * (double)a.re - mi * (double)a.im;
            vi += mr * (double)a.im + mi * (double)a.re;
        }
        const cx<T> p = psi[i];
        sr += (double)p.re * vr + (double)p.im * vi;
        si += (double)p.re * vi - (double)p.im * vr;
    }
    double tr = 0.0, ti = 0.0;
    block_add(sr, red, &tr, threadIdx.x, 256);
    block_add(si, red, &ti, threadIdx.x, 256);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = tr;
        partials[gridDim.x + blockIdx.x] = ti;
    }
}

template <typename T>
hipError_t launch_sparse(hipStream_t s, const void* psi, uint64_t N, const int64_t* row_ptr, const int64_t* col,
                         const double* val, double* partials, int grid) {
    hipLaunchKernelGGL(k_sparse<T>, dim3(grid), dim3(256), 0, s, (const cx<T>*)psi, N, row_ptr, col, val, partials);
    return hipGetLastError();
}

// ------------------------------------------------------------------ allocation-free scratch

// Device scratch of the allocation-free entry point (qsv_expval_noalloc): its
// Pauli tables, per-block partials and results live here instead of in
// buffers the library allocates.  Every device that loads the library holds
// its own copy until the process ends; calls that overlap on one device share
// it (and race).  Host code never names the array: it uses the address
// returned below, taken once per device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

// The scratch's address on the current device (the caller keeps it per device).
hipError_t noalloc_scratch_address(void** ptr) { return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch)); }

// ------------------------------------------------------------------ deterministic reduction

__global__ __launch_bounds__(256) void k_reduce(const double* __restrict__ partials, int n_blocks,
                                                double* __restrict__ out) {
    __shared__ double red[64];
    const int slot = blockIdx.x;
    double s = 0.0;
    for (int j = threadIdx.x; j < n_blocks; j += 256) s += partials[(uint64_t)slot * n_blocks + j];
    double tot = 0.0;
    block_add(s, red, &tot, threadIdx.x, 256);
    if (threadIdx.x == 0) out[slot] = tot;
}

// Batched reduction: block b sums partials[re[b].off + j], j < re[b].n, into out[re[b].out].
__global__ __launch_bounds__(256) void k_reduce_batch(const ReduceEntry* __restrict__ re,
                                                      const double* __restrict__ partials, double* __restrict__ out) {
    __shared__ double red[64];
    const ReduceEntry e = re[blockIdx.x];
    double s = 0.0;
    for (int j = threadIdx.x; j < e.n; j += 256) s += partials[e.off + j];
    double tot = 0.0;
    block_add(s, red, &tot, threadIdx.x, 256);
    if (threadIdx.x == 0) out[e.out] = tot;
}

hipError_t launch_reduce_batch(hipStream_t s, const ReduceEntry* re, int n, const double* partials, double* out) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_batch, dim3(n), dim3(256), 0, s, re, partials, out);
    return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t s, const double* partials, int n_blocks, int n_slots, double* out) {
    if (n_slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3(n_slots), dim3(256), 0, s, partials, n_blocks, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ instantiations

#define QSV_INST(T)                                                                                              \
    template hipError_t launch_init<T>(hipStream_t, void*, uint64_t, uint64_t);                                 \
    template hipError_t launch_gate1<T>(hipStream_t, void*, uint64_t, const Expand&, uint64_t, uint64_t, int,   \
                                        const Mat2&, bool);                                                     \
    template hipError_t launch_diag1<T>(hipStream_t, void*, uint64_t, const Expand&, uint64_t, double, double,  \
                                        bool);                                                                  \
    template hipError_t launch_gate2<T>(hipStream_t, void*, uint64_t, const Expand&, uint64_t, uint64_t,        \
                                        uint64_t, int, const Mat4&, bool);                                      \
    template hipError_t launch_gatek<T>(hipStream_t, void*, uint64_t, const Expand&, uint64_t, int,             \
                                        const int32_t*, const void*, bool);                                     \
    template hipError_t launch_gatek_low<T>(hipStream_t, void*, uint64_t, const Expand&, uint64_t, int,         \
                                            const int32_t*, uint32_t, uint32_t, const void*, bool);             \
    template hipError_t launch_dense<T>(hipStream_t, void*, const DenseArgs&, const void*, bool, bool);        \
    template hipError_t launch_tile<T>(hipStream_t, bool, bool, const void*, void*, void*, const TileArgs&, const TOp*,      \
                                       const void*, const uint64_t*, double*, int, int, int, size_t);           \
    template hipError_t launch_pauli<T>(hipStream_t, bool, bool, const void*, void*, uint64_t,                  \
                                        const PauliGroupDev*, int, const PauliTermDev*, const uint64_t*, int,  \
                                        double*, int);                                                          \
    template hipError_t launch_probs<T>(hipStream_t, const void*, uint64_t, const Expand&, const uint64_t*, int, \
                                        int, double*);                                                          \
    template hipError_t launch_tile_batch<T>(hipStream_t, bool, bool, const TileEntry*, const int32_t*,        \
                                             const TileArgs*, const TOp*, const void*, const uint64_t*, double*, \
                                             int, int, int, size_t);                                            \
    template hipError_t launch_pauli_batch<T>(hipStream_t, bool, const PauliEntry*, const int32_t*,             \
                                              const PauliGroupDev*, const PauliTermDev*, const uint64_t*, int,  \
                                              double*, int);                                                    \
    template hipError_t launch_sparse<T>(hipStream_t, const void*, uint64_t, const int64_t*, const int64_t*,    \
                                         const double*, double*, int);                                          \
    template hipError_t launch_chunk_norms<T>(hipStream_t, const void*, int, uint64_t, double*);              \
    template hipError_t launch_sample<T>(hipStream_t, const void*, int, const int64_t*, const double*,          \
                                         uint64_t*, int64_t);

QSV_INST(double)
QSV_INST(float)

}  // namespace qsv
