// The LDS-staged tile pass (one vector for gate application, two vectors for
// the adjoint sweep) and its batched form.  Templates only: each tile_*.hip
// translation unit instantiates one (precision, vector count) pair, so the
// heavy register-group code compiles in parallel.
#pragma once

#include "kcommon.h"

namespace qsv {

// ------------------------------------------------------------------ LDS-tiled fused pass

// LDS position of tile element t: bits 4..7 are XOR-ed into bits 0..3, so
// that threads reading subcubes whose group bits include the lowest tile bits
// (a lane stride of 16 elements) spread over all banks.  A bijection on any
// tile size.
__device__ __forceinline__ uint32_t sw(uint32_t t) { return t ^ ((t >> 4) & 15u); }

// One op of a tile pass.  tp/tl: the phi/lambda tiles in LDS (tl only when
// TWO).  The thread owns tile elements t = tid + r * nthr, r < R; pair and
// quad ops address any element of the tile.
template <typename T, bool TWO, int R>
struct TileCtx {
    cx<T>* tp;
    cx<T>* tl;
    double* red;
    double* sacc;
    const cx<T>* coef;
    const uint64_t* words;
    uint64_t base, offlo, tile;
    const uint64_t* offhi;
    int n_outer;
    const cx<T>* ztab;  // the pass's phase tables, in LDS
    // parity bits of the current tile's base index for each grouped Z-parity
    // op (LDS, by the op's tb[5])
    const uint64_t* zpar;
    int tid, nthr, nwaves;
    int nacc;  // slot accumulator entries per slot: one per 16-lane row (or 1)
};

template <typename T, bool TWO, int R>
__device__ __forceinline__ void tile_apply1(const TileCtx<T, TWO, R>& c, const TOp& op) {
    const int q = op.tb[0];
    const uint32_t qb = 1u << q, lo = qb - 1;
    const cx<T> m0 = c.coef[op.coff], m1 = c.coef[op.coff + 1], m2 = c.coef[op.coff + 2], m3 = c.coef[op.coff + 3];
    const int half = (c.nthr * R) >> 1;
    const int cls = op.cls;
    for (int p = c.tid; p < half; p += c.nthr) {
        const uint32_t t0 = (((uint32_t)p & ~lo) << 1) | ((uint32_t)p & lo), t1 = t0 | qb;
        if ((t0 & op.lcmask) != op.lcval) continue;
#pragma unroll
        for (int v = 0; v < (TWO ? 2 : 1); ++v) {
            cx<T>* t = v ? c.tl : c.tp;
            const uint32_t s0 = sw(t0), s1 = sw(t1);
            const cx<T> a0 = t[s0], a1 = t[s1];
            if (cls == MC_DIAG) {
                t[s0] = cmul(m0, a0);
                t[s1] = cmul(m3, a1);
            } else if (cls == MC_ANTI) {
                t[s0] = cmul(m1, a1);
                t[s1] = cmul(m2, a0);
            } else {
                t[s0] = cmad(m0, a0, cmul(m1, a1));
                t[s1] = cmad(m2, a0, cmul(m3, a1));
            }
        }
    }
}

template <typename T, bool TWO, int R>
__device__ __forceinline__ void tile_apply2(const TileCtx<T, TWO, R>& c, const TOp& op) {
    const uint32_t b0 = 1u << op.tb[0], b1 = 1u << op.tb[1];
    const uint32_t plo = b0 < b1 ? b0 : b1, phi = b0 < b1 ? b1 : b0;
    const int quarter = (c.nthr * R) >> 2;
    const cx<T>* m = c.coef + op.coff;
    const int cls = op.cls;
    for (int p = c.tid; p < quarter; p += c.nthr) {
        uint32_t t = (((uint32_t)p & ~(plo - 1)) << 1) | ((uint32_t)p & (plo - 1));
        t = ((t & ~(phi - 1)) << 1) | (t & (phi - 1));
        if ((t & op.lcmask) != op.lcval) continue;
        const uint32_t idx[4] = {sw(t), sw(t | b1), sw(t | b0), sw(t | b0 | b1)};
#pragma unroll
        for (int v = 0; v < (TWO ? 2 : 1); ++v) {
            cx<T>* tt = v ? c.tl : c.tp;
            if (cls == MC_MID) {
                const cx<T> x1 = tt[idx[1]], x2 = tt[idx[2]];
                tt[idx[1]] = cmad(m[5], x1, cmul(m[6], x2));
                tt[idx[2]] = cmad(m[9], x1, cmul(m[10], x2));
            } else if (cls == MC_DIAG) {
#pragma unroll
                for (int j = 0; j < 4; ++j) tt[idx[j]] = cmul(m[j * 5], tt[idx[j]]);
            } else {
                cx<T> a[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) a[j] = tt[idx[j]];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    cx<T> acc = {T(0), T(0)};
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc = cmad(m[r * 4 + j], a[j], acc);
                    tt[idx[r]] = acc;
                }
            }
        }
    }
}

__device__ __forceinline__ uint32_t spread_bits(int j, int k, const int32_t* tb) {
    uint32_t o = 0;
    for (int i = 0; i < k; ++i)
        if ((j >> (k - 1 - i)) & 1) o |= 1u << tb[i];
    return o;
}

// k-qubit matrix (any k) on tile bits tb[0..k-1]: every thread computes
// output values into registers, then all threads write back after a barrier.
// With at most one tuple per thread (k >= log2 R), a thread owns R rows of one
// tuple: tuple = tid mod T, rows from (tid / T) * R, so the rows - and the
// matrix entries read - are uniform across a wavefront when T >= 64 (scalar
// loads), and each input is read from LDS once per thread.  Otherwise each
// element computes its own row.
template <typename T, bool TWO, int R>
__device__ __forceinline__ void tile_applyk(const TileCtx<T, TWO, R>& c, const TOp& op) {
    const int k = op.k, dim = 1 << k;
    const int tsz = c.nthr * R;
    const int ntup = tsz >> k;
    cx<T> ap[R], al[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        ap[r] = {T(0), T(0)};
        al[r] = {T(0), T(0)};
    }
    if (ntup <= c.nthr) {
        // sorted target bits (k <= 8, uniform), then the tuple's base index
        int srt[8];
        for (int i = 0; i < k; ++i) srt[i] = op.tb[i];
        for (int i = 1; i < k; ++i)
            for (int j = i; j > 0 && srt[j - 1] > srt[j]; --j) {
                const int t = srt[j];
                srt[j] = srt[j - 1];
                srt[j - 1] = t;
            }
        uint32_t tb = (uint32_t)(c.tid & (ntup - 1));
        for (int i = 0; i < k; ++i) {
            const uint32_t q = (uint32_t)srt[i];
            tb = ((tb >> q) << (q + 1)) | (tb & ((1u << q) - 1));
        }
        const int row0 = (c.tid / ntup) * R;
        const bool on = (tb & op.lcmask) == op.lcval;
        for (int j = 0; j < dim; ++j) {
            const uint32_t sj = sw(tb | spread_bits(j, k, op.tb));
            const cx<T> x = c.tp[sj];
            const cx<T> xl = TWO ? c.tl[sj] : x;
            const cx<T>* mcol = c.coef + op.coff + (size_t)row0 * dim + j;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const cx<T> mm = mcol[(size_t)r * dim];
                ap[r] = cmad(mm, x, ap[r]);
                if (TWO) al[r] = cmad(mm, xl, al[r]);
            }
        }
        __syncthreads();
        if (on) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t so = sw(tb | spread_bits(row0 + r, k, op.tb));
                c.tp[so] = ap[r];
                if (TWO) c.tl[so] = al[r];
            }
        }
        return;
    }
    uint32_t tmask = 0;
    for (int i = 0; i < k; ++i) tmask |= 1u << op.tb[i];
    int row[R];
    uint32_t gb[R];
    bool on[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t t = c.tid + r * c.nthr;
        int rw = 0;
        for (int i = 0; i < k; ++i) rw = (rw << 1) | ((t >> op.tb[i]) & 1);
        row[r] = rw;
        gb[r] = t & ~tmask;
        on[r] = (t & op.lcmask) == op.lcval;
    }
    for (int j = 0; j < dim; ++j) {
        const uint32_t sp = spread_bits(j, k, op.tb);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const cx<T> mm = c.coef[op.coff + row[r] * dim + j];
            ap[r] = cmad(mm, c.tp[sw(gb[r] | sp)], ap[r]);
            if (TWO) al[r] = cmad(mm, c.tl[sw(gb[r] | sp)], al[r]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (!on[r]) continue;
        const uint32_t t = c.tid + r * c.nthr;
        c.tp[sw(t)] = ap[r];
        if (TWO) c.tl[sw(t)] = al[r];
    }
}

template <typename T, bool TWO, int R>
__device__ __forceinline__ void tile_diag(const TileCtx<T, TWO, R>& c, const TOp& op) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint64_t g = c.base | c.offlo | c.offhi[r];
        if ((g & op.gcmask) != op.gcval) continue;
        int j = 0;
        for (int i = 0; i < op.k; ++i) j = (j << 1) | (int)((g >> op.tb[i]) & 1);
        const cx<T> d = c.coef[op.coff + j];
        const int t = c.tid + r * c.nthr;
        c.tp[sw(t)] = cmul(d, c.tp[sw(t)]);
        if (TWO) c.tl[sw(t)] = cmul(d, c.tl[sw(t)]);
    }
}

// Parity bits (bit j = parity of base & z_j) of this tile's base index: the
// map is linear over GF(2), so it is the XOR of the host's per-outer-bit
// columns over the set bits of the tile number (uniform, scalar unit).
__device__ __forceinline__ uint64_t tile_parity(uint64_t tile, const uint64_t* __restrict__ cols, int n_outer) {
    uint64_t p = 0;
    for (int k = 0; k < n_outer; ++k)
        if ((tile >> k) & 1) p ^= cols[k];
    return p;
}

// Z-parity rotation group: the odd-parity bit mask of g = base|offlo|offhi[r]
// is the XOR of the three parts' masks (parity is linear over GF(2)); the
// per-thread and per-r parts are precomputed on the host.
template <typename T, bool TWO, int R>
__device__ __forceinline__ void tile_zphase(const TileCtx<T, TWO, R>& c, const TOp& op) {
    const uint64_t* w = c.words + op.woff;
    const uint64_t pb = tile_parity(c.tile, w + op.m + c.nthr + R, c.n_outer);
    const uint64_t pl = w[op.m + c.tid] ^ pb;
    const uint64_t* ph = w + op.m + c.nthr;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int cnt = (int)__popcll(pl ^ ph[r]);
        const cx<T> d = c.coef[op.coff + cnt];
        const int t = c.tid + r * c.nthr;
        c.tp[sw(t)] = cmul(d, c.tp[sw(t)]);
        if (TWO) c.tl[sw(t)] = cmul(d, c.tl[sw(t)]);
    }
}

template <typename T, bool TWO, int R>
__device__ __forceinline__ void tile_dot(const TileCtx<T, TWO, R>& c, const TOp& op) {
    if constexpr (TWO) {
        double acc = 0.0;
        const cx<T>* G = c.coef + op.coff;
        if (op.kind == OP_DOT1) {
            const uint32_t qb = 1u << op.tb[0], lo = qb - 1;
            const int half = (c.nthr * R) >> 1;
            for (int p = c.tid; p < half; p += c.nthr) {
                const uint32_t t0 = (((uint32_t)p & ~lo) << 1) | ((uint32_t)p & lo), t1 = t0 | qb;
                if ((t0 & op.lcmask) != op.lcval) continue;
                const cx<T> p0 = c.tp[sw(t0)], p1 = c.tp[sw(t1)];
                acc += im_conj_mul(c.tl[sw(t0)], cmad(G[0], p0, cmul(G[1], p1)));
                acc += im_conj_mul(c.tl[sw(t1)], cmad(G[2], p0, cmul(G[3], p1)));
            }
        } else if (op.kind == OP_DOT2 || op.kind == OP_DOTK) {
            const int k = op.k, dim = 1 << k;
            uint32_t tmask = 0;
            for (int i = 0; i < k; ++i) tmask |= 1u << op.tb[i];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint32_t t = c.tid + r * c.nthr;
                if ((t & op.lcmask) != op.lcval) continue;
                int rw = 0;
                for (int i = 0; i < k; ++i) rw = (rw << 1) | ((t >> op.tb[i]) & 1);
                const uint32_t gb = t & ~tmask;
                cx<T> v = {T(0), T(0)};
                for (int j = 0; j < dim; ++j) v = cmad(G[rw * dim + j], c.tp[sw(gb | spread_bits(j, k, op.tb))], v);
                acc += im_conj_mul(c.tl[sw(t)], v);
            }
        } else if (op.kind == OP_DOTDIAG) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint64_t g = c.base | c.offlo | c.offhi[r];
                if ((g & op.gcmask) != op.gcval) continue;
                int j = 0;
                for (int i = 0; i < op.k; ++i) j = (j << 1) | (int)((g >> op.tb[i]) & 1);
                const int t = c.tid + r * c.nthr;
                acc += im_conj_mul(c.tl[sw(t)], cmul(G[j], c.tp[sw(t)]));
            }
        } else {  // OP_DOTZSUM: generator sum_j Z^{z_j}, eigenvalue m - 2 * (odd count)
            const uint64_t* w = c.words + op.woff;
            const uint64_t pb = tile_parity(c.tile, w + op.m + c.nthr + R, c.n_outer);
            const uint64_t pl = w[op.m + c.tid] ^ pb;
            const uint64_t* ph = w + op.m + c.nthr;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int cnt = (int)__popcll(pl ^ ph[r]);
                const int t = c.tid + r * c.nthr;
                acc += (double)(op.m - 2 * cnt) * im_conj_mul(c.tl[sw(t)], c.tp[sw(t)]);
            }
        }
        block_add(acc, c.red, c.sacc + op.slot * c.nacc, c.tid, c.nthr);
    }
}


// ------------------------------------------------------------------ register subcube groups
//
// A GROUP op names GB tile bits Q.  The tile splits into 2^(b-GB) subcubes
// of 2^GB elements that agree on the other tile bits; each thread loads whole
// subcubes from LDS into registers, runs every sub-op of the group on them
// (1- and 2-qubit matrices on bits of Q, diagonal phases on any global bits,
// adjoint inner products), and writes them back once: one LDS round trip per
// group instead of one per gate.  Element e of a subcube is tile index
// tc | eo[e], eo[e] = sum of bit i of e shifted to Q[i].

// 2x2 update of one register pair, specialised by matrix class
template <typename T, int CLS>
__device__ __forceinline__ void bfly(const cx<T>* m, cx<T>& x0, cx<T>& x1) {
    const cx<T> a0 = x0, a1 = x1;
    if (CLS == MC_PX) {  // exactly X: the pair trades places (no arithmetic)
        x0 = a1;
        x1 = a0;
    } else if (CLS == MC_ANTI) {
        x0 = cmul(m[1], a1);
        x1 = cmul(m[2], a0);
    } else if (CLS == MC_REAL) {
        const T m0 = m[0].re, m1 = m[1].re, m2 = m[2].re, m3 = m[3].re;
        x0 = {m0 * a0.re + m1 * a1.re, m0 * a0.im + m1 * a1.im};
        x1 = {m2 * a0.re + m3 * a1.re, m2 * a0.im + m3 * a1.im};
    } else if (CLS == MC_DIAG) {
        x0 = cmul(m[0], a0);
        x1 = cmul(m[3], a1);
    } else if (CLS == MC_RIRI_D) {  // [[1, i p], [i q, 1]]: one FMA per component
        const T p = m[1].im, q = m[2].im;
        x0 = {a0.re - p * a1.im, a0.im + p * a1.re};
        x1 = {a1.re - q * a0.im, a1.im + q * a0.re};
    } else if (CLS == MC_RIRI_O) {  // [[u, i], [i, v]]
        const T u = m[0].re, v = m[3].re;
        x0 = {u * a0.re - a1.im, u * a0.im + a1.re};
        x1 = {v * a1.re - a0.im, v * a1.im + a0.re};
    } else if (CLS == MC_REAL_D) {  // [[1, p], [q, 1]]
        const T p = m[1].re, q = m[2].re;
        x0 = {a0.re + p * a1.re, a0.im + p * a1.im};
        x1 = {a1.re + q * a0.re, a1.im + q * a0.im};
    } else if (CLS == MC_REAL_O) {  // [[u, -1], [1, v]]
        const T u = m[0].re, v = m[3].re;
        x0 = {u * a0.re - a1.re, u * a0.im - a1.im};
        x1 = {a0.re + v * a1.re, a0.im + v * a1.im};
    } else if (CLS == MC_RIRI) {  // [[r0, i q1], [i q2, r3]]
        const T r0 = m[0].re, q1 = m[1].im, q2 = m[2].im, r3 = m[3].re;
        x0 = {r0 * a0.re - q1 * a1.im, r0 * a0.im + q1 * a1.re};
        x1 = {r3 * a1.re - q2 * a0.im, r3 * a1.im + q2 * a0.re};
    } else {
        x0 = cmad(m[0], a0, cmul(m[1], a1));
        x1 = cmad(m[2], a0, cmul(m[3], a1));
    }
}

template <typename T, bool TWO, int GB, int P, int CLS, bool CTRL>
__device__ __forceinline__ void g_apply1(cx<T>* a, cx<T>* l, const cx<T>* mg, uint32_t tc, const uint32_t* eo,
                                         uint32_t lcm, uint32_t lcv) {
    const cx<T> m[4] = {mg[0], mg[1], mg[2], mg[3]};
#pragma unroll
    for (int e0 = 0; e0 < (1 << GB); ++e0) {
        if (e0 & (1 << P)) continue;
        const int e1 = e0 | (1 << P);
        if (CTRL && ((tc | eo[e0]) & lcm) != lcv) continue;
        bfly<T, CLS>(m, a[e0], a[e1]);
        if (TWO) bfly<T, CLS>(m, l[e0], l[e1]);
    }
}

template <typename T, bool TWO, int GB, int P0, int P1, int CLS, bool CTRL>
__device__ __forceinline__ void g_apply2(cx<T>* a, cx<T>* l, const cx<T>* m, uint32_t tc, const uint32_t* eo,
                                         uint32_t lcm, uint32_t lcv) {
#pragma unroll
    for (int e = 0; e < (1 << GB); ++e) {
        if (e & ((1 << P0) | (1 << P1))) continue;
        if (CTRL && ((tc | eo[e]) & lcm) != lcv) continue;
        const int id[4] = {e, e | (1 << P1), e | (1 << P0), e | (1 << P0) | (1 << P1)};
#pragma unroll
        for (int v = 0; v < (TWO ? 2 : 1); ++v) {
            cx<T>* x = v ? l : a;
            if (CLS == MC_MID) {
                const cx<T> x1 = x[id[1]], x2 = x[id[2]];
                x[id[1]] = cmad(m[5], x1, cmul(m[6], x2));
                x[id[2]] = cmad(m[9], x1, cmul(m[10], x2));
            } else {
                const cx<T> y[4] = {x[id[0]], x[id[1]], x[id[2]], x[id[3]]};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    cx<T> acc = cmul(m[r * 4], y[0]);
#pragma unroll
                    for (int j = 1; j < 4; ++j) acc = cmad(m[r * 4 + j], y[j], acc);
                    x[id[r]] = acc;
                }
            }
        }
    }
}

template <typename T, int GB, int P, int CLS, bool CTRL>
__device__ __forceinline__ double g_dot1(const cx<T>* a, const cx<T>* l, const cx<T>* G, uint32_t tc,
                                         const uint32_t* eo, uint32_t lcm, uint32_t lcv) {
    const cx<T> g0 = G[0], g1 = G[1], g2 = G[2], g3 = G[3];
    double acc = 0.0;
#pragma unroll
    for (int e0 = 0; e0 < (1 << GB); ++e0) {
        if (e0 & (1 << P)) continue;
        const int e1 = e0 | (1 << P);
        if (CTRL && ((tc | eo[e0]) & lcm) != lcv) continue;
        // the X, Y and diagonal classes accumulate in fused multiply-add chains
        if (CLS == MC_PX) {         // G = X: Im(l0* p1) + Im(l1* p0)
            acc = acc_im_conj_mul(acc_im_conj_mul(acc, l[e0], a[e1]), l[e1], a[e0]);
        } else if (CLS == MC_DIAG) {  // G = diag(g0, g3), real
            acc = __builtin_fma((double)g0.re, im_conj_mul(l[e0], a[e0]), acc);
            acc = __builtin_fma((double)g3.re, im_conj_mul(l[e1], a[e1]), acc);
        } else if (CLS == MC_PY) {  // G = Y: Re(l1* p0) - Re(l0* p1)
            acc = __builtin_fma((double)l[e1].re, (double)a[e0].re, acc);
            acc = __builtin_fma((double)l[e1].im, (double)a[e0].im, acc);
            acc = __builtin_fma(-(double)l[e0].re, (double)a[e1].re, acc);
            acc = __builtin_fma(-(double)l[e0].im, (double)a[e1].im, acc);
        } else {
            acc += im_conj_mul(l[e0], cmad(g0, a[e0], cmul(g1, a[e1])));
            acc += im_conj_mul(l[e1], cmad(g2, a[e0], cmul(g3, a[e1])));
        }
    }
    return acc;
}

template <typename T, int GB, int P0, int P1, bool CTRL>
__device__ __forceinline__ double g_dot2(const cx<T>* a, const cx<T>* l, const cx<T>* G, uint32_t tc,
                                         const uint32_t* eo, uint32_t lcm, uint32_t lcv) {
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < (1 << GB); ++e) {
        if (e & ((1 << P0) | (1 << P1))) continue;
        if (CTRL && ((tc | eo[e]) & lcm) != lcv) continue;
        const int id[4] = {e, e | (1 << P1), e | (1 << P0), e | (1 << P0) | (1 << P1)};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            cx<T> v = cmul(G[r * 4], a[id[0]]);
#pragma unroll
            for (int j = 1; j < 4; ++j) v = cmad(G[r * 4 + j], a[id[j]], v);
            acc += im_conj_mul(l[id[r]], v);
        }
    }
    return acc;
}

// register accumulators of the group's inner products, selected by a runtime
// index through a switch so they stay in registers
struct DotAcc {
    double v[GROUP_MAX_DOTS];
    __device__ __forceinline__ void add(int i, double x) {
        switch (i) {
        case 0: v[0] += x; break;
        case 1: v[1] += x; break;
        case 2: v[2] += x; break;
        case 3: v[3] += x; break;
        case 4: v[4] += x; break;
        case 5: v[5] += x; break;
        case 6: v[6] += x; break;
        default: v[7] += x; break;
        }
    }
    __device__ __forceinline__ double get(int i) const {
        switch (i) {
        case 0: return v[0];
        case 1: return v[1];
        case 2: return v[2];
        case 3: return v[3];
        case 4: return v[4];
        case 5: return v[5];
        case 6: return v[6];
        default: return v[7];
        }
    }
};

// One layer of one-qubit ops over every group position.  Ops on different
// positions commute (and so do a generator on one position and a matrix on
// another, for the inner products), so the layer runs positions in a fixed
// order as straight-line code: no per-gate dispatch, and the register arrays
// flow through without merges.  Per position p the coefficients are
// [generator (GCLS == DENSE or DIAG only)] then the 2x2 matrix.
template <typename T, bool TWO, int GB, int CLS, int GCLS, int P, typename Sink>
__device__ __forceinline__ void g_layer_pos(cx<T>* a, cx<T>* l, const cx<T>* m, uint32_t dmask, Sink& sink) {
    constexpr int NC = (GCLS == MC_DENSE || GCLS == MC_DIAG) ? 8 : 4;
    const cx<T>* mp = m + P * NC;
    if constexpr (TWO && GCLS >= 0) {
        if (dmask & (1u << P)) sink(P, g_dot1<T, GB, P, GCLS, false>(a, l, mp, 0, nullptr, 0, 0));
    }
    // unconditional: positions without a gate hold the identity, which keeps
    // the layer branch-free (a skipped position would merge two versions of
    // the register arrays)
    g_apply1<T, TWO, GB, P, CLS, false>(a, l, mp + NC - 4, 0, nullptr, 0, 0);
}

// sink(p, v) receives this thread's inner product at position p (where bit p
// of dmask is set), right after it is computed
template <typename T, bool TWO, int GB, int CLS, int GCLS, typename Sink>
__device__ __forceinline__ void g_layer(cx<T>* a, cx<T>* l, const cx<T>* m, uint32_t dmask, Sink& sink) {
    g_layer_pos<T, TWO, GB, CLS, GCLS, 0>(a, l, m, dmask, sink);
    if constexpr (GB > 1) g_layer_pos<T, TWO, GB, CLS, GCLS, 1>(a, l, m, dmask, sink);
    if constexpr (GB > 2) g_layer_pos<T, TWO, GB, CLS, GCLS, 2>(a, l, m, dmask, sink);
    if constexpr (GB > 3) g_layer_pos<T, TWO, GB, CLS, GCLS, 3>(a, l, m, dmask, sink);
}

#define QSV_P1_CASES(F)                                  \
    switch (p0) {                                        \
    case 0: F(0); break;                                 \
    case 1: if constexpr (GB > 1) { F(1); } break;       \
    case 2: if constexpr (GB > 2) { F(2); } break;       \
    case 3: if constexpr (GB > 3) { F(3); } break;       \
    default: break;                                      \
    }
#define QSV_P2_CASE(A, B, F) \
    case A * 4 + B: if constexpr (GB > A && GB > B) { F(A, B); } break;
#define QSV_P2_CASES(F)                                                                          \
    switch (p0 * 4 + p1) {                                                                       \
    QSV_P2_CASE(0, 1, F) QSV_P2_CASE(0, 2, F) QSV_P2_CASE(0, 3, F) QSV_P2_CASE(1, 0, F)          \
    QSV_P2_CASE(1, 2, F) QSV_P2_CASE(1, 3, F) QSV_P2_CASE(2, 0, F) QSV_P2_CASE(2, 1, F)          \
    QSV_P2_CASE(2, 3, F) QSV_P2_CASE(3, 0, F) QSV_P2_CASE(3, 1, F) QSV_P2_CASE(3, 2, F)          \
    default: break;                                                                              \
    }

// ZP: the tile parities of the grouped Z-parity ops are in LDS (c.zpar);
// otherwise they are formed from the columns at each use.
template <typename T, bool TWO, int R, int GB, bool ZP = true>
__device__ __forceinline__ void tile_group(const TileCtx<T, TWO, R>& c, const TOp& g, const TOp* __restrict__ subs,
                                           int b) {
    constexpr int E = 1 << GB;
    const int nsub = (c.nthr * R) >> GB;
    const uint64_t* w = c.words + g.woff;
    uint32_t eo[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        uint32_t o = 0;
#pragma unroll
        for (int i = 0; i < GB; ++i)
            if ((e >> i) & 1) o |= 1u << g.tb[i];
        eo[e] = o;
    }
    // sw() is linear over GF(2) and tc, eo[e] have disjoint bits, so the
    // LDS slot of element e is sw(tc) ^ sw(eo[e]) (a uniform XOR)
    uint32_t swe[E];
#pragma unroll
    for (int e = 0; e < E; ++e) swe[e] = sw(eo[e]);
    DotAcc acc;
#pragma unroll
    for (int d = 0; d < GROUP_MAX_DOTS; ++d) acc.v[d] = 0.0;
    const int nq = b - GB;
    const bool need_gc = g.aux != 0;  // the group holds position-dependent diagonals
    // every thread runs the same number of subcubes (all lanes active inside
    // the loop): layers reduce their inner products right away, per 16-lane
    // row by DPP, into the row's own slot accumulator
    const bool inloop = c.nthr >= 64 && nsub >= c.nthr;
    auto row_flush = [&](double v, int slot) {
        v += row_shr<1>(v);
        v += row_shr<2>(v);
        v += row_shr<4>(v);
        v += row_shr<8>(v);
        if ((c.tid & 15) == 15) lds_add(&c.sacc[slot * c.nacc + (c.tid >> 4)], v);
    };
#pragma unroll 1
    for (int sc = c.tid; sc < nsub; sc += c.nthr) {
        uint32_t tc = (uint32_t)sc;
#pragma unroll
        for (int i = 0; i < GB; ++i) {  // Q ascending: insert a zero at each Q bit
            const uint32_t q = (uint32_t)g.tb[i];
            tc = ((tc >> q) << (q + 1)) | (tc & ((1u << q) - 1));
        }
        uint64_t gc = c.base;
        if (need_gc)
            for (int j = 0; j < nq; ++j)
                if ((sc >> j) & 1) gc |= 1ull << w[E + j];
        // two vectors: the per-subcube parity word of the group's first
        // Z-parity op (tb[4] of the group op) is loaded before the subcube, so
        // its latency overlaps the LDS reads (one vector: no registers to spare)
        uint64_t wz0 = 0;
        if (TWO && g.tb[4] >= 0) wz0 = c.words[subs[g.tb[4]].woff + subs[g.tb[4]].m + sc];
        auto zbits = [&](const TOp& s, int si) {
            const uint64_t* z = c.words + s.woff;
            const uint64_t w = (TWO && si == g.tb[4]) ? wz0 : z[s.m + sc];
            uint64_t t;
            if constexpr (ZP) t = c.zpar[s.tb[5]];
            else t = tile_parity(c.tile, z + s.m + nsub + E, c.n_outer);
            return t ^ w;
        };
        const uint32_t stc = sw(tc);
        cx<T> a[E], l[TWO ? E : 1];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            a[e] = c.tp[stc ^ swe[e]];
            if (TWO) l[e] = c.tl[stc ^ swe[e]];
        }
        for (int si = 0; si < g.m; ++si) {
            const TOp& s = subs[si];
            const bool local = s.kind == OP_APPLY1 || s.kind == OP_APPLY2 || s.kind == OP_DOT1 || s.kind == OP_DOT2;
            if (local && (c.base & s.gcmask) != s.gcval) continue;
            const cx<T>* m = c.coef + s.coff;
            const int p0 = s.tb[0], p1 = s.tb[1];
            switch (s.kind) {
            case OP_APPLY1: {
                const bool ctrl = s.lcmask != 0;
                if (ctrl && s.cls == MC_PX) {
#define F(P) g_apply1<T, TWO, GB, P, MC_PX, true>(a, l, m, tc, eo, s.lcmask, s.lcval)
                    QSV_P1_CASES(F)
#undef F
                } else if (ctrl) {
#define F(P) g_apply1<T, TWO, GB, P, MC_DENSE, true>(a, l, m, tc, eo, s.lcmask, s.lcval)
                    QSV_P1_CASES(F)
#undef F
                } else if (s.cls == MC_PX) {
#define F(P) g_apply1<T, TWO, GB, P, MC_PX, false>(a, l, m, tc, eo, 0, 0)
                    QSV_P1_CASES(F)
#undef F
                } else if (s.cls == MC_ANTI) {
#define F(P) g_apply1<T, TWO, GB, P, MC_ANTI, false>(a, l, m, tc, eo, 0, 0)
                    QSV_P1_CASES(F)
#undef F
                } else if (s.cls == MC_REAL) {
#define F(P) g_apply1<T, TWO, GB, P, MC_REAL, false>(a, l, m, tc, eo, 0, 0)
                    QSV_P1_CASES(F)
#undef F
                } else if (s.cls == MC_RIRI) {
#define F(P) g_apply1<T, TWO, GB, P, MC_RIRI, false>(a, l, m, tc, eo, 0, 0)
                    QSV_P1_CASES(F)
#undef F
                } else if (s.cls == MC_DIAG) {
#define F(P) g_apply1<T, TWO, GB, P, MC_DIAG, false>(a, l, m, tc, eo, 0, 0)
                    QSV_P1_CASES(F)
#undef F
                } else {
#define F(P) g_apply1<T, TWO, GB, P, MC_DENSE, false>(a, l, m, tc, eo, 0, 0)
                    QSV_P1_CASES(F)
#undef F
                }
            } break;
            case OP_APPLY2:
                if (s.lcmask) {
                    if (s.cls == MC_MID) {
#define F(A, B) g_apply2<T, TWO, GB, A, B, MC_MID, true>(a, l, m, tc, eo, s.lcmask, s.lcval)
                        QSV_P2_CASES(F)
#undef F
                    } else {
#define F(A, B) g_apply2<T, TWO, GB, A, B, MC_DENSE, true>(a, l, m, tc, eo, s.lcmask, s.lcval)
                        QSV_P2_CASES(F)
#undef F
                    }
                } else if (s.cls == MC_MID) {
#define F(A, B) g_apply2<T, TWO, GB, A, B, MC_MID, false>(a, l, m, tc, eo, 0, 0)
                    QSV_P2_CASES(F)
#undef F
                } else {
#define F(A, B) g_apply2<T, TWO, GB, A, B, MC_DENSE, false>(a, l, m, tc, eo, 0, 0)
                    QSV_P2_CASES(F)
#undef F
                }
                break;
            case OP_LAYER1: {
                // template GCLS: -1 without inner products, else the generator's class
                const uint32_t gcode = TWO ? s.lcval : (uint32_t)LG_NONE;
                // every lane active here: reduce per row at once; otherwise
                // keep the sums for the flush after the loop
                int ai = s.aux;
                auto sink = [&](int p, double v) {
                    if (inloop) row_flush(v, s.tb[p]);
                    else acc.add(ai++, v);
                };
#define L(C, G) g_layer<T, TWO, GB, C, G>(a, l, m, s.lcmask, sink)
                if (gcode == LG_NONE) {
                    if (s.cls == MC_RIRI_D) L(MC_RIRI_D, -1);
                    else if (s.cls == MC_RIRI_O) L(MC_RIRI_O, -1);
                    else if (s.cls == MC_REAL_D) L(MC_REAL_D, -1);
                    else if (s.cls == MC_REAL_O) L(MC_REAL_O, -1);
                    else if (s.cls == MC_REAL) L(MC_REAL, -1);
                    else if (s.cls == MC_RIRI) L(MC_RIRI, -1);
                    else if (s.cls == MC_DIAG) L(MC_DIAG, -1);
                    else L(MC_DENSE, -1);
                } else if constexpr (TWO) {
                    if (gcode == LG_X) {
                        if (s.cls == MC_RIRI_D) L(MC_RIRI_D, MC_PX);
                        else if (s.cls == MC_RIRI_O) L(MC_RIRI_O, MC_PX);
                        else if (s.cls == MC_REAL) L(MC_REAL, MC_PX);
                        else if (s.cls == MC_RIRI) L(MC_RIRI, MC_PX);
                        else L(MC_DENSE, MC_PX);
                    } else if (gcode == LG_Y) {
                        if (s.cls == MC_REAL_D) L(MC_REAL_D, MC_PY);
                        else if (s.cls == MC_REAL_O) L(MC_REAL_O, MC_PY);
                        else if (s.cls == MC_REAL) L(MC_REAL, MC_PY);
                        else if (s.cls == MC_RIRI) L(MC_RIRI, MC_PY);
                        else L(MC_DENSE, MC_PY);
                    } else if (gcode == LG_DIAG) {
                        if (s.cls == MC_REAL) L(MC_REAL, MC_DIAG);
                        else if (s.cls == MC_RIRI) L(MC_RIRI, MC_DIAG);
                        else if (s.cls == MC_DIAG) L(MC_DIAG, MC_DIAG);
                        else L(MC_DENSE, MC_DIAG);
                    } else {
                        if (s.cls == MC_REAL) L(MC_REAL, MC_DENSE);
                        else if (s.cls == MC_RIRI) L(MC_RIRI, MC_DENSE);
                        else if (s.cls == MC_DIAG) L(MC_DIAG, MC_DENSE);
                        else L(MC_DENSE, MC_DENSE);
                    }
                }
#undef L
            } break;
            case OP_DIAG:
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const uint64_t gi = gc | w[e];
                    if ((gi & s.gcmask) != s.gcval) continue;
                    int j = 0;
                    for (int i = 0; i < s.k; ++i) j = (j << 1) | (int)((gi >> s.tb[i]) & 1);
                    const cx<T> d = m[j];
                    a[e] = cmul(d, a[e]);
                    if (TWO) l[e] = cmul(d, l[e]);
                }
                break;
            case OP_ZPHASE: {
                const uint64_t* z = c.words + s.woff;
                const uint64_t pc = zbits(s, si);
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const cx<T> d = c.ztab[s.aux + (int)__popcll(pc ^ z[s.m + nsub + e])];
                    a[e] = cmul(d, a[e]);
                    if (TWO) l[e] = cmul(d, l[e]);
                }
            } break;
            case OP_ZPHDOT:
                if constexpr (TWO) {
                    const uint64_t* z = c.words + s.woff;
                    const uint64_t pc = zbits(s, si);
                    double v = 0.0;
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const int cnt = (int)__popcll(pc ^ z[s.m + nsub + e]);
                        v = __builtin_fma((double)(s.m - 2 * cnt), im_conj_mul(l[e], a[e]), v);
                        const cx<T> d = c.ztab[s.lcval + cnt];
                        a[e] = cmul(d, a[e]);
                        l[e] = cmul(d, l[e]);
                    }
                    if (inloop) row_flush(v, s.slot);
                    else acc.add(s.aux, v);
                }
                break;
            default:
                if constexpr (TWO) {
                    double v = 0.0;
                    if (s.kind == OP_DOT1) {
                        if (s.lcmask) {
#define F(P) v = g_dot1<T, GB, P, MC_DENSE, true>(a, l, m, tc, eo, s.lcmask, s.lcval)
                            QSV_P1_CASES(F)
#undef F
                        } else if (s.cls == MC_PX) {
#define F(P) v = g_dot1<T, GB, P, MC_PX, false>(a, l, m, tc, eo, 0, 0)
                            QSV_P1_CASES(F)
#undef F
                        } else if (s.cls == MC_PY) {
#define F(P) v = g_dot1<T, GB, P, MC_PY, false>(a, l, m, tc, eo, 0, 0)
                            QSV_P1_CASES(F)
#undef F
                        } else if (s.cls == MC_DIAG) {
#define F(P) v = g_dot1<T, GB, P, MC_DIAG, false>(a, l, m, tc, eo, 0, 0)
                            QSV_P1_CASES(F)
#undef F
                        } else {
#define F(P) v = g_dot1<T, GB, P, MC_DENSE, false>(a, l, m, tc, eo, 0, 0)
                            QSV_P1_CASES(F)
#undef F
                        }
                    } else if (s.kind == OP_DOT2) {
                        if (s.lcmask) {
#define F(A, B) v = g_dot2<T, GB, A, B, true>(a, l, m, tc, eo, s.lcmask, s.lcval)
                            QSV_P2_CASES(F)
#undef F
                        } else {
#define F(A, B) v = g_dot2<T, GB, A, B, false>(a, l, m, tc, eo, 0, 0)
                            QSV_P2_CASES(F)
#undef F
                        }
                    } else if (s.kind == OP_DOTDIAG) {
#pragma unroll
                        for (int e = 0; e < E; ++e) {
                            const uint64_t gi = gc | w[e];
                            if ((gi & s.gcmask) != s.gcval) continue;
                            int j = 0;
                            for (int i = 0; i < s.k; ++i) j = (j << 1) | (int)((gi >> s.tb[i]) & 1);
                            v += im_conj_mul(l[e], cmul(m[j], a[e]));
                        }
                    } else {  // OP_DOTZSUM
                        const uint64_t* z = c.words + s.woff;
                        const uint64_t pc = zbits(s, si);
#pragma unroll
                        for (int e = 0; e < E; ++e)
                            v = __builtin_fma((double)(s.m - 2 * (int)__popcll(pc ^ z[s.m + nsub + e])),
                                              im_conj_mul(l[e], a[e]), v);
                    }
                    if (inloop) row_flush(v, s.slot);
                    else acc.add(s.aux, v);
                }
                break;
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            c.tp[stc ^ swe[e]] = a[e];
            if (TWO) c.tl[stc ^ swe[e]] = l[e];
        }
    }
    if constexpr (TWO) {
        // flush: per-wave sums into the wave's accumulator (no barrier when
        // the block is made of whole waves)
        // per 16-lane row: DPP prefix sums leave the row's total in its last
        // lane, which adds it to the row's own accumulator (no cross-row
        // traffic; the block sums the rows once at the end)
        auto flush = [&](int ai, int slot) {
            double v = acc.get(ai);
            if (c.nthr >= 64) {
                v += row_shr<1>(v);
                v += row_shr<2>(v);
                v += row_shr<4>(v);
                v += row_shr<8>(v);
                if ((c.tid & 15) == 15) lds_add(&c.sacc[slot * c.nacc + (c.tid >> 4)], v);
            } else {
                block_add(v, c.red, c.sacc + slot * c.nacc, c.tid, c.nthr);
            }
        };
        for (int si = 0; si < g.m; ++si) {
            const TOp& s = subs[si];
            if (s.kind == OP_LAYER1) {
                if (inloop) continue;  // reduced inside the loop
                int ai = s.aux;
                for (int p = 0; p < GB; ++p)
                    if (s.lcmask & (1u << p)) flush(ai++, s.tb[p]);
                continue;
            }
            if ((s.kind < OP_DOT1 || s.kind == OP_DOTK || s.kind > OP_DOTZSUM) && s.kind != OP_ZPHDOT) continue;
            if (inloop) continue;  // reduced inside the loop
            flush(s.aux, s.slot);
        }
    }
}

// The first tile of a warp-specialised block, loaded into LDS buffer buf.
template <typename T, bool TWO, int R>
__device__ __forceinline__ void tile_to_lds(cx<T>* buf, uint32_t stid, const cx<T>* phi_src, const cx<T>* lam,
                                            const TileArgs& a, uint64_t offlo, uint64_t tile, bool synth) {
    constexpr int NT = 256;
    const uint64_t base = expand_idx(tile, a.outer) | offlo;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint64_t g = base | a.offhi[r];
        cx<T> v;
        if (synth) {
            v.re = g == a.basis ? T(1) : T(0);
            v.im = T(0);
        } else {
            v = phi_src[g];
        }
        buf[stid + r * NT] = v;
        if (TWO) buf[NT * R + stid + r * NT] = lam[g];
    }
}

// GEN: the pass also holds standalone ops (k-qubit matrices, or a tile too
// small for groups); group-only passes compile without those code paths,
// which keeps their register footprint (and so their occupancy) lower.
// One block's share of a tile pass: tiles blk, blk + nblk, ... of the pass
// described by a.  phi_src is where phi is read from (phi itself, or the
// post-circuit state for an out-of-place first adjoint pass); with
// TILE_SYNTH the tile is synthesised as the basis state a.basis instead.
// LAMZ: the first reverse pass of a diagonal, uniform-coefficient observable
// (TILE_LAMZ), compiled separately so that the other passes carry none of it.
template <typename T, bool TWO, int LR, bool GEN, bool LAMZ = false>
__device__ __forceinline__ void tile_body(const cx<T>* phi_src, cx<T>* phi,
                                          cx<T>* __restrict__ lam, const TileArgs& a, const TOp* __restrict__ ops,
                                          const cx<T>* __restrict__ coef, const uint64_t* __restrict__ words,
                                          double* __restrict__ partials, uint64_t blk, uint64_t nblk) {
    constexpr int R = 1 << LR;
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    // tiles of more than 256 elements always run 256 threads: a compile-time
    // block size turns every per-element LDS offset into an immediate
    const int nthr = LR > 0 ? 256 : (int)blockDim.x;
    const int tsz = nthr * R;
    // LDS slot of the thread's element r: sw(tid + r * nthr) = sw(tid) + r * nthr
    // (r * nthr only has bits at or above bit 8 when R > 1)
    const uint32_t stid = sw((uint32_t)tid);
    TileCtx<T, TWO, R> c;
    c.tp = reinterpret_cast<cx<T>*>(smem);
    c.tl = c.tp + (TWO ? tsz : 0);
    c.red = reinterpret_cast<double*>(smem + (TWO ? 2 : 1) * (size_t)tsz * sizeof(cx<T>));
    c.sacc = c.red + 64;
    c.coef = coef;
    c.words = words;
    c.offhi = a.offhi;
    c.n_outer = a.n_outer;
    c.tid = tid;
    c.nthr = nthr;
    c.nwaves = nthr >= 64 ? nthr >> 6 : 1;
    c.nacc = nthr >= 64 ? nthr >> 4 : 1;
    constexpr bool lamz = TWO && LAMZ;
    const int nsl = a.nslots + (lamz ? 1 : 0);  // slot accumulators, with <H> last
    {
        // phase tables after the per-wave slot accumulators, 16-byte aligned
        const size_t off = (64 + (size_t)nsl * c.nacc) * sizeof(double);
        cx<T>* zt = reinterpret_cast<cx<T>*>(reinterpret_cast<unsigned char*>(c.red) + ((off + 15) & ~(size_t)15));
        for (int i = tid; i < a.zt_n; i += nthr) zt[i] = coef[a.zt_off + i];
        c.ztab = zt;
    }
    // grouped Z-parity ops: their columns (tile-number bit j -> parity bits)
    // in LDS once per block, then per tile the parity bits of its base index
    uint64_t* zcol = reinterpret_cast<uint64_t*>(
        (reinterpret_cast<uintptr_t>(c.ztab + a.zt_n) + 7) & ~(uintptr_t)7);
    uint64_t* zpar = zcol + (size_t)a.n_zop * a.n_outer;
    c.zpar = zpar;
    if (a.n_zop > 0) {
        constexpr int GBv = TWO ? GROUP_BITS_TWO : GROUP_BITS_ONE;
        const int nsub = tsz >> GBv;
        for (int oi = 0; oi < a.nops; ++oi) {
            const TOp& op = ops[a.op0 + oi];
            if (op.kind != OP_GROUP) continue;
            for (int si = 0; si < op.m; ++si) {
                const TOp& s = ops[a.op0 + oi + 1 + si];
                if (s.kind != OP_ZPHASE && s.kind != OP_DOTZSUM && s.kind != OP_ZPHDOT) continue;
                const uint64_t* cols = words + s.woff + s.m + nsub + (1 << GBv);
                for (int j = tid; j < a.n_outer; j += nthr) zcol[(size_t)s.tb[5] * a.n_outer + j] = cols[j];
            }
            oi += op.m;
        }
        __syncthreads();
    }
    uint64_t offlo = 0;
    for (int j = 0; j < a.nthr_log2; ++j) offlo |= (uint64_t)((tid >> j) & 1) << a.sb[j];
    c.offlo = offlo;
    for (int s = tid; s < nsl * c.nacc; s += nthr) c.sacc[s] = 0.0;
    if constexpr (lamz) __syncthreads();  // the <H> slot is added to before the first barrier of the tile loop
    const bool synth = (a.flags & TILE_SYNTH) != 0;

    // TILE_LAMZ: lambda_g = c (m - 2 |odd parities of g|) phi_g and <H> = sum
    // of conj(phi_g) lambda_g; the parity bits of g are the XOR of the tile's,
    // the thread's and the register slot's parts (linear over GF(2)).  Each
    // tile's <H> share goes to slot accumulator a.nslots (reduced per row like
    // the inner products), so nothing stays live across the groups.
    const uint64_t* lw = words + a.lamz_woff;

    for (uint64_t tile = blk; tile < a.n_tiles; tile += nblk) {
        const uint64_t base = expand_idx(tile, a.outer);
        c.base = base;
        c.tile = tile;
        const uint64_t lam_par = lamz ? tile_parity(tile, lw + nthr + R, a.n_outer) ^ lw[tid] : 0;
        double ev = 0.0;
        // global -> LDS in chunks of LCH elements per thread: LCH loads in
        // flight per thread without keeping all R values live in registers
        constexpr int LCH = R < 8 ? R : 8;
        for (int r0 = 0; r0 < R; r0 += LCH) {
            cx<T> vp[LCH], vl[LCH];
#pragma unroll
            for (int r = 0; r < LCH; ++r) {
                const uint64_t g = base | offlo | a.offhi[r0 + r];
                if (synth) {
                    vp[r].re = g == a.basis ? T(1) : T(0);
                    vp[r].im = T(0);
                } else {
                    vp[r] = phi_src[g];
                }
                if (TWO && !lamz) vl[r] = lam[g];
            }
            if (lamz) {
#pragma unroll
                for (int r = 0; r < LCH; ++r) {
                    const int w = a.lamz_m - 2 * (int)__popcll(lam_par ^ lw[nthr + r0 + r]);
                    const T s = (T)(a.lamz_c * (double)w);
                    vl[r] = {s * vp[r].re, s * vp[r].im};
                    ev = __builtin_fma((double)w, (double)vp[r].re * vp[r].re + (double)vp[r].im * vp[r].im, ev);
                }
            }
#pragma unroll
            for (int r = 0; r < LCH; ++r) {
                c.tp[stid + (r0 + r) * nthr] = vp[r];
                if (TWO) c.tl[stid + (r0 + r) * nthr] = vl[r];
            }
        }
        if (lamz && nthr >= 64) {  // this tile's <H> share, per 16-lane row
            ev += row_shr<1>(ev);
            ev += row_shr<2>(ev);
            ev += row_shr<4>(ev);
            ev += row_shr<8>(ev);
            if ((tid & 15) == 15) lds_add(&c.sacc[a.nslots * c.nacc + (tid >> 4)], ev * a.lamz_c);
        } else if (lamz) {
            block_add(ev * a.lamz_c, c.red, c.sacc + a.nslots * c.nacc, tid, nthr);
        }
        for (int k = tid; k < a.n_zop; k += nthr) {
            const uint64_t* col = zcol + (size_t)k * a.n_outer;
            uint64_t p = 0;
#pragma unroll 4
            for (int j = 0; j < a.n_outer; ++j) p ^= ((tile >> j) & 1) ? col[j] : 0ull;
            zpar[k] = p;
        }
        __syncthreads();
        for (int oi = 0; oi < a.nops; ++oi) {
            const TOp& op = ops[a.op0 + oi];
            if ((op.kind <= OP_APPLYK || (op.kind >= OP_DOT1 && op.kind <= OP_DOTK)) &&
                (base & op.gcmask) != op.gcval)
                continue;  // outer controls fail for this whole tile (uniform)
            if (op.kind == OP_GROUP) {
                tile_group<T, TWO, R, TWO ? GROUP_BITS_TWO : GROUP_BITS_ONE>(c, op, ops + a.op0 + oi + 1, a.b);
                oi += op.m;
                __syncthreads();
                continue;
            }
            if constexpr (GEN) {
                switch (op.kind) {
                case OP_APPLY1: tile_apply1(c, op); break;
                case OP_APPLY2: tile_apply2(c, op); break;
                case OP_APPLYK: tile_applyk(c, op); break;
                case OP_DIAG: tile_diag(c, op); break;
                case OP_ZPHASE: tile_zphase(c, op); break;
                default: tile_dot(c, op); break;
                }
            }
            __syncthreads();
        }
        const bool nt = (a.flags & TILE_NT) != 0;
        const T osc = (T)a.out_scale;
        const bool scaled = osc != T(1);  // factored layers in the pass
        for (int r0 = 0; r0 < R; r0 += LCH) {
#pragma unroll
            for (int r = 0; r < LCH; ++r) {
                const uint64_t g = base | offlo | a.offhi[r0 + r];
                cx<T> vp = c.tp[stid + (r0 + r) * nthr];
                if (scaled) vp = {vp.re * osc, vp.im * osc};
                st_amp(phi + g, vp, nt);
                if (TWO) {
                    cx<T> vl = c.tl[stid + (r0 + r) * nthr];
                    if (scaled) vl = {vl.re * osc, vl.im * osc};
                    st_amp(lam + g, vl, nt);
                }
            }
        }
        __syncthreads();
    }
    __syncthreads();
    for (int s = tid; s < a.nslots; s += nthr) {
        double v = 0.0;
        for (int w = 0; w < c.nacc; ++w) v += c.sacc[s * c.nacc + w];
        partials[(uint64_t)s * nblk + blk] = v;
    }
    if (lamz && tid == 0) {  // <H>: partial row nslots
        double v = 0.0;
        for (int w = 0; w < c.nacc; ++w) v += c.sacc[a.nslots * c.nacc + w];
        partials[(uint64_t)a.nslots * nblk + blk] = v;
    }
}

template <typename T, bool TWO, int LR, bool GEN>
__global__ __launch_bounds__(256, 2) void k_tile(const cx<T>* phi_src, cx<T>* phi, cx<T>* __restrict__ lam,
                                                 const TileArgs a, const TOp* __restrict__ ops,
                                                 const cx<T>* __restrict__ coef, const uint64_t* __restrict__ words,
                                                 double* __restrict__ partials) {
    tile_body<T, TWO, LR, GEN>(phi_src, phi, lam, a, ops, coef, words, partials, blockIdx.x, gridDim.x);
}

// The first reverse pass with lambda formed from phi (TILE_LAMZ).
template <typename T, int LR>
__global__ __launch_bounds__(256, 2) void k_tile_lamz(const cx<T>* phi_src, cx<T>* phi, cx<T>* __restrict__ lam,
                                                      const TileArgs a, const TOp* __restrict__ ops,
                                                      const cx<T>* __restrict__ coef,
                                                      const uint64_t* __restrict__ words,
                                                      double* __restrict__ partials) {
    tile_body<T, true, LR, false, true>(phi_src, phi, lam, a, ops, coef, words, partials, blockIdx.x, gridDim.x);
}

// Warp-specialised form of a group-only pass (every top-level op is a
// register group, so each op costs exactly one barrier): 512 threads, waves
// 0-3 compute, waves 4-7 load, with two tile buffers in LDS.  While the
// compute waves run tile i from one buffer, the load waves fetch tile i+1
// (global -> registers -> LDS) into the other; both sides execute the same
// barriers (one per group, one per tile), so HBM reads overlap the groups
// and neither side waits for the other except at the tile boundary.  The
// compute waves write tile i back at its end (stores do not block).
// LDS: buffer 0, buffer 1 (phi, then lambda when TWO), then the reduction
// area, slot accumulators and phase tables as in tile_body.
template <typename T, bool TWO, int LR>
__device__ __forceinline__ void tile_body_ws(const cx<T>* phi_src, cx<T>* phi, cx<T>* __restrict__ lam,
                                             const TileArgs& a, const TOp* __restrict__ ops,
                                             const cx<T>* __restrict__ coef, const uint64_t* __restrict__ words,
                                             double* __restrict__ partials, uint64_t blk, uint64_t nblk) {
    constexpr int R = 1 << LR;
    constexpr int NT = 256;  // compute threads (and load threads)
    constexpr int TSZ = NT * R;
    constexpr size_t VB = (size_t)(TWO ? 2 : 1) * TSZ * sizeof(cx<T>);  // one buffer
    extern __shared__ __align__(16) unsigned char smem[];
    const int tid = threadIdx.x;
    const bool loader = tid >= NT;
    const int lt = tid & (NT - 1);
    const uint32_t stid = sw((uint32_t)lt);
    cx<T>* buf0 = reinterpret_cast<cx<T>*>(smem);
    cx<T>* buf1 = reinterpret_cast<cx<T>*>(smem + VB);
    TileCtx<T, TWO, R> c;
    c.red = reinterpret_cast<double*>(smem + 2 * VB);
    c.sacc = c.red + 64;
    c.coef = coef;
    c.words = words;
    c.offhi = a.offhi;
    c.n_outer = a.n_outer;
    c.tid = lt;
    c.nthr = NT;
    c.nwaves = NT >> 6;
    c.nacc = NT >> 4;
    {
        const size_t off = (64 + (size_t)a.nslots * c.nacc) * sizeof(double);
        cx<T>* zt = reinterpret_cast<cx<T>*>(reinterpret_cast<unsigned char*>(c.red) + ((off + 15) & ~(size_t)15));
        for (int i = tid; i < a.zt_n; i += 2 * NT) zt[i] = coef[a.zt_off + i];
        c.ztab = zt;
    }
    c.zpar = nullptr;  // tile parities from the columns per use (tile_group<..., false>)
    uint64_t offlo = 0;
    for (int j = 0; j < 8; ++j) offlo |= (uint64_t)((lt >> j) & 1) << a.sb[j];
    c.offlo = offlo;
    for (int s = tid; s < a.nslots * c.nacc; s += 2 * NT) c.sacc[s] = 0.0;
    const bool synth = (a.flags & TILE_SYNTH) != 0;

    if (loader) {
        if (blk < a.n_tiles) tile_to_lds<T, TWO, R>(buf0, stid, phi_src, lam, a, offlo, blk, synth);
        __syncthreads();
        int cur = 0;
        for (uint64_t tile = blk; tile < a.n_tiles; tile += nblk) {
            const bool more = tile + nblk < a.n_tiles;
            // phi then (TWO) lambda values of the next tile, one array so that
            // all of them stay in registers
            constexpr int NV = (TWO ? 2 : 1) * R;
            cx<T> v[NV];
            const uint64_t nbase = expand_idx(more ? tile + nblk : tile, a.outer) | offlo;
            if (more) {
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    const uint64_t g = nbase | a.offhi[q % R];
                    if (q >= R) {
                        v[q] = lam[g];
                    } else if (synth) {
                        v[q].re = g == a.basis ? T(1) : T(0);
                        v[q].im = T(0);
                    } else {
                        v[q] = phi_src[g];
                    }
                }
            }
            // the compute side's barriers: one per group
            for (int oi = 0; oi < a.nops; ++oi) {
                oi += ops[a.op0 + oi].m;
                __syncthreads();
            }
            if (more) {
                cx<T>* nb = cur ? buf0 : buf1;
#pragma unroll
                for (int q = 0; q < NV; ++q) nb[(q >= R ? TSZ : 0) + stid + (q % R) * NT] = v[q];
            }
            __syncthreads();
            cur ^= 1;
        }
    } else {
        __syncthreads();
        int cur = 0;
        const bool nt = (a.flags & TILE_NT) != 0;
        for (uint64_t tile = blk; tile < a.n_tiles; tile += nblk) {
            const uint64_t base = expand_idx(tile, a.outer);
            c.base = base;
            c.tile = tile;
            c.tp = cur ? buf1 : buf0;
            c.tl = c.tp + (TWO ? TSZ : 0);
            for (int oi = 0; oi < a.nops; ++oi) {
                const TOp& op = ops[a.op0 + oi];
                tile_group<T, TWO, R, TWO ? GROUP_BITS_TWO : GROUP_BITS_ONE, false>(c, op, ops + a.op0 + oi + 1,
                                                                                    a.b);
                oi += op.m;
                __syncthreads();
            }
            const T osc = (T)a.out_scale;
            const bool scaled = osc != T(1);  // factored layers in the pass
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const uint64_t g = base | offlo | a.offhi[r];
                cx<T> vp = c.tp[stid + r * NT];
                if (scaled) vp = {vp.re * osc, vp.im * osc};
                st_amp(phi + g, vp, nt);
                if (TWO) {
                    cx<T> vl = c.tl[stid + r * NT];
                    if (scaled) vl = {vl.re * osc, vl.im * osc};
                    st_amp(lam + g, vl, nt);
                }
            }
            __syncthreads();
            cur ^= 1;
        }
    }
    __syncthreads();
    if (!loader)
        for (int s = lt; s < a.nslots; s += NT) {
            double v = 0.0;
            for (int w = 0; w < c.nacc; ++w) v += c.sacc[s * c.nacc + w];
            partials[(uint64_t)s * nblk + blk] = v;
        }
}

template <typename T, bool TWO, int LR>
__global__ __launch_bounds__(512, 1) void k_tile_ws(const cx<T>* phi_src, cx<T>* phi, cx<T>* __restrict__ lam,
                                                    const TileArgs a, const TOp* __restrict__ ops,
                                                    const cx<T>* __restrict__ coef,
                                                    const uint64_t* __restrict__ words,
                                                    double* __restrict__ partials) {
    tile_body_ws<T, TWO, LR>(phi_src, phi, lam, a, ops, coef, words, partials, blockIdx.x, gridDim.x);
}

// Batched passes: block b serves entry blk_entry[2b] (one circuit's pass) as
// its block blk_entry[2b + 1].
template <typename T, bool TWO, int LR, bool GEN>
__global__ __launch_bounds__(256, 2) void k_tile_batch(const TileEntry* __restrict__ entries,
                                                       const int32_t* __restrict__ blk_entry,
                                                       const TileArgs* __restrict__ args, const TOp* __restrict__ ops,
                                                       const cx<T>* __restrict__ coef,
                                                       const uint64_t* __restrict__ words,
                                                       double* __restrict__ partials) {
    const TileEntry& e = entries[blk_entry[2 * blockIdx.x]];
    tile_body<T, TWO, LR, GEN>((const cx<T>*)e.phi_src, (cx<T>*)e.phi, (cx<T>*)e.lam, args[e.args], ops, coef, words,
                               partials + e.part_off, (uint64_t)blk_entry[2 * blockIdx.x + 1], e.nblk);
}


template <typename T, bool TWO, int LR, bool GEN>
static hipError_t launch_tile_lr(hipStream_t s, const void* phi_src, void* phi, void* lam, const TileArgs& a,
                                 const TOp* ops, const void* coef, const uint64_t* words, double* partials, int grid,
                                 int nthr, size_t lds) {
    if constexpr (TWO && (LR == 3 || LR == 4) && !GEN) {
        if (a.flags & TILE_LAMZ) {
            static std::atomic<uint64_t> lz_raised{0};
            if (lds > 65536) {
                hipError_t e = allow_big_lds((const void*)k_tile_lamz<T, LR>, lz_raised);
                if (e != hipSuccess) return e;
            }
            hipLaunchKernelGGL((k_tile_lamz<T, LR>), dim3(grid), dim3(nthr), lds, s, (const cx<T>*)phi_src,
                               (cx<T>*)phi, (cx<T>*)lam, a, ops, (const cx<T>*)coef, words, partials);
            return hipGetLastError();
        }
    }
    if constexpr (LR >= 3 && !GEN) {
        if (a.flags & TILE_WS) {
            // warp-specialised form (the host sized the grid and the LDS for it)
            static std::atomic<uint64_t> ws_raised{0};
            hipError_t e = allow_big_lds((const void*)k_tile_ws<T, TWO, LR>, ws_raised);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_tile_ws<T, TWO, LR>), dim3(grid), dim3(512), lds, s, (const cx<T>*)phi_src,
                               (cx<T>*)phi, (cx<T>*)lam, a, ops, (const cx<T>*)coef, words, partials);
            return hipGetLastError();
        }
    }
    static std::atomic<uint64_t> lds_raised{0};
    if (lds > 65536) {
        hipError_t e = allow_big_lds((const void*)k_tile<T, TWO, LR, GEN>, lds_raised);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_tile<T, TWO, LR, GEN>), dim3(grid), dim3(nthr), lds, s, (const cx<T>*)phi_src, (cx<T>*)phi,
                       (cx<T>*)lam, a, ops, (const cx<T>*)coef, words, partials);
    return hipGetLastError();
}

template <typename T, bool TWO, bool GEN>
static hipError_t launch_tile_two(hipStream_t s, const void* phi_src, void* phi, void* lam, const TileArgs& a,
                                  const TOp* ops, const void* coef, const uint64_t* words, double* partials, int grid,
                                  int nthr, int R, size_t lds) {
    switch (R) {
    case 1: return launch_tile_lr<T, TWO, 0, GEN>(s, phi_src, phi, lam, a, ops, coef, words, partials, grid, nthr, lds);
    case 2: return launch_tile_lr<T, TWO, 1, GEN>(s, phi_src, phi, lam, a, ops, coef, words, partials, grid, nthr, lds);
    case 4: return launch_tile_lr<T, TWO, 2, GEN>(s, phi_src, phi, lam, a, ops, coef, words, partials, grid, nthr, lds);
    case 8: return launch_tile_lr<T, TWO, 3, GEN>(s, phi_src, phi, lam, a, ops, coef, words, partials, grid, nthr, lds);
    case 16: return launch_tile_lr<T, TWO, 4, GEN>(s, phi_src, phi, lam, a, ops, coef, words, partials, grid, nthr, lds);
    case 32: return launch_tile_lr<T, TWO, 5, GEN>(s, phi_src, phi, lam, a, ops, coef, words, partials, grid, nthr, lds);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, bool TWO>
hipError_t launch_tile_v(hipStream_t s, bool generic, const void* phi_src, void* phi, void* lam, const TileArgs& a,
                         const TOp* ops, const void* coef, const uint64_t* words, double* partials, int grid,
                         int nthr, int R, size_t lds_bytes) {
    if (generic)
        return launch_tile_two<T, TWO, true>(s, phi_src, phi, lam, a, ops, coef, words, partials, grid, nthr, R,
                                             lds_bytes);
    return launch_tile_two<T, TWO, false>(s, phi_src, phi, lam, a, ops, coef, words, partials, grid, nthr, R,
                                          lds_bytes);
}

template <typename T, bool TWO, int LR, bool GEN>
static hipError_t launch_tile_batch_lr(hipStream_t s, const TileEntry* entries, const int32_t* blk_entry,
                                       const TileArgs* args, const TOp* ops, const void* coef, const uint64_t* words,
                                       double* partials, int blocks, int nthr, size_t lds) {
    static std::atomic<uint64_t> lds_raised{0};
    if (lds > 65536) {
        hipError_t e = allow_big_lds((const void*)k_tile_batch<T, TWO, LR, GEN>, lds_raised);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_tile_batch<T, TWO, LR, GEN>), dim3(blocks), dim3(nthr), lds, s, entries, blk_entry, args,
                       ops, (const cx<T>*)coef, words, partials);
    return hipGetLastError();
}

template <typename T, bool TWO, bool GEN>
static hipError_t launch_tile_batch_two(hipStream_t s, const TileEntry* entries, const int32_t* blk_entry,
                                        const TileArgs* args, const TOp* ops, const void* coef,
                                        const uint64_t* words, double* partials, int blocks, int nthr, int R,
                                        size_t lds) {
#define QSV_TB(LRV) launch_tile_batch_lr<T, TWO, LRV, GEN>(s, entries, blk_entry, args, ops, coef, words, partials, \
                                                           blocks, nthr, lds)
    switch (R) {
    case 1: return QSV_TB(0);
    case 2: return QSV_TB(1);
    case 4: return QSV_TB(2);
    case 8: return QSV_TB(3);
    case 16: return QSV_TB(4);
    case 32: return QSV_TB(5);
    default: return hipErrorInvalidValue;
    }
#undef QSV_TB
}

template <typename T, bool TWO>
hipError_t launch_tile_batch_v(hipStream_t s, bool generic, const TileEntry* entries, const int32_t* blk_entry,
                               const TileArgs* args, const TOp* ops, const void* coef, const uint64_t* words,
                               double* partials, int blocks, int nthr, int R, size_t lds) {
    if (generic)
        return launch_tile_batch_two<T, TWO, true>(s, entries, blk_entry, args, ops, coef, words, partials, blocks,
                                                   nthr, R, lds);
    return launch_tile_batch_two<T, TWO, false>(s, entries, blk_entry, args, ops, coef, words, partials, blocks,
                                                nthr, R, lds);
}

}  // namespace qsv
