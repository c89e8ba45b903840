// Internal declarations of the qsv library (host runtime <-> HIP kernels).
// Nothing here is part of the C ABI; see include/qsv.h for that.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "qsv.h"

namespace qsv {

using cd = std::complex<double>;

// ------------------------------------------------------------------ device descriptors

// Insert zero bits at sorted positions p_0 < .. < p_{m-1} of an index k:
// r = (k & m[0]) | ((k << 1) & m[1]) | .. | ((k << m) & m[m]), where m[i]
// keeps the output bits strictly between p_{i-1} and p_i (paper Alg. 2 and
// its getMasks helper, read with the corrections listed in the design notes).
struct Expand {
    uint64_t m[16];
    int32_t nm;  // number of masks = inserted positions + 1
    int32_t pad;
};

Expand make_expand(const std::vector<int>& sorted_positions);

enum TOpKind : int32_t {
    OP_APPLY1 = 1,  // 2x2 on local tile bit tb[0]
    OP_APPLY2,      // 4x4 on local tile bits tb[0] (msb), tb[1]
    OP_APPLYK,      // 2^k x 2^k on local tile bits tb[0..k-1]
    OP_DIAG,        // diagonal on global index bits tb[0..k-1]; table at coff
    OP_ZPHASE,      // exp(-i a/2 sum_j Z^{z_j}) via a phase table over the odd-parity count
    OP_DOT1,        // slot += Im <lam|G|phi> for G on local bit tb[0]
    OP_DOT2,
    OP_DOTK,
    OP_DOTDIAG,     // slot += Im <lam|D|phi> for diagonal D on global bits
    OP_DOTZSUM,     // slot += Im <lam| sum_j Z^{z_j} |phi>
    OP_GROUP,       // the next m ops act inside register subcubes over the k tile bits tb[0..k-1]
    OP_LAYER1,      // in a group: for each group position p ascending, an optional inner
                    // product with a one-qubit generator on p (bit p of lcmask; slot tb[p];
                    // generator class code lcval, LayerGen), then the 2x2 matrix of class cls on p
                    // (bit p of m: the layer has a gate on p; elsewhere the table
                    // holds the identity)
    OP_ZPHDOT       // in a group: DOTZSUM then ZPHASE over the same Z strings, one parity
                    // count per element (slot, aux and the parity words as DOTZSUM; phase
                    // table at coff, at lcval inside the pass's table in LDS).  The inner
                    // product is the same before and after the phase, which multiplies
                    // phi and lambda alike by a unit-modulus diagonal
};

// Matrix classes.  DENSE/DIAG/ANTI/MID are used by every kernel; the finer
// classes only by the register-group ops (elsewhere they run as DENSE):
// REAL = all entries real (H, RY), RIRI = real diagonal and imaginary
// off-diagonal (RX), PX / PY = exactly Pauli X / Y (inner-product generators).
enum MatClass : int32_t { MC_DENSE = 0, MC_DIAG = 1, MC_ANTI = 2, MC_MID = 3, MC_REAL = 4, MC_RIRI = 5, MC_PX = 6,
                          MC_PY = 7,
                          // factored layer classes (scaled so that one entry pair is exactly 1 or +-i; the
                          // common factor is carried as a tile-wide scale): RIRI_D [[1, i p], [i q, 1]],
                          // RIRI_O [[u, i], [i, v]], REAL_D [[1, p], [q, 1]], REAL_O [[u, -1], [1, v]]
                          MC_RIRI_D = 8, MC_RIRI_O = 9, MC_REAL_D = 10, MC_REAL_O = 11 };

struct TOp {
    int32_t kind, cls, k, slot;
    int32_t tb[6];
    uint32_t lcmask, lcval;  // controls on local tile-index bits
    uint64_t gcmask, gcval;  // controls on global index bits
    int64_t coff;            // complex offset into the coefficient table
    int64_t woff;            // u64 offset into the word table (ZPHASE/DOTZSUM)
    int32_t m;               // parity masks (ZPHASE/DOTZSUM); sub-op count (GROUP)
    int32_t aux;             // register accumulator of a DOT inside a group
};

// Register subcube width of the grouped tile ops (elements per subcube = 2^GB)
constexpr int GROUP_BITS_ONE = 4;  // one vector
constexpr int GROUP_BITS_TWO = 3;  // phi and lambda
constexpr int GROUP_MAX_DOTS = 8;

constexpr int TILE_MAX_R_LOG2 = 5;   // at most 32 elements per thread
constexpr int TILE_THREADS = 256;

struct TileArgs {
    Expand outer;           // tile number -> base index (zeros at the tile bits)
    uint64_t n_tiles;
    uint64_t offhi[1 << TILE_MAX_R_LOG2];  // deposit of (r * nthr) into the tile bits
    int32_t sb[16];         // tile bits, ascending (tile-local bit j <-> global bit sb[j])
    int32_t b;              // tile bits
    int32_t nthr_log2;
    int32_t op0, nops;
    int32_t nslots;
    int32_t zt_n;           // phase-table entries copied to LDS at kernel start
    int64_t zt_off;         // their offset in the coefficient table
    int32_t flags;          // TILE_SYNTH: phi tiles start as the basis state `basis`
    int32_t n_outer;        // index bits outside the tile (bits of the tile number)
    uint64_t basis;
    int32_t n_zop;          // Z-parity ops inside register groups (their tb[5] numbers them)
    int32_t lamz_m;         // TILE_LAMZ: number of Z strings of the observable
    double out_scale;       // the pass's factored layers leave the tile scaled by 1 / out_scale
    // TILE_LAMZ (first reverse pass, observable = c * sum of lamz_m Z strings):
    // lambda is formed from the loaded phi instead of read, and <H> goes to
    // partial row nslots.  Words at lamz_woff: per thread, per register slot
    // and per tile-number bit, the parity bits of the observable's masks.
    int64_t lamz_woff;
    double lamz_c;
};
constexpr int32_t TILE_SYNTH = 1;
constexpr int32_t TILE_NT = 2;  // write back with non-temporal stores
constexpr int32_t TILE_WS = 4;  // warp-specialised kernel form (two tile buffers, 512 threads)
constexpr int32_t TILE_LAMZ = 8;  // lambda = H phi formed in the load (diagonal, uniform-coefficient H)

// A dense k-qubit matrix on a tile of 2^(k+6) amplitudes: the k targets and
// six lane bits (the lowest index bits that are neither targets nor
// controls).  Tile-local bit i (ascending global bit order) is global bit
// sb[i] and bit cb[i] of the compact LDS index (j << 6) | lane.
struct DenseArgs {
    Expand outer;        // tile number -> base index (zeros at tile bits and controls)
    uint64_t setmask;    // control values
    uint64_t n_tiles;
    uint64_t goff_hi[16];  // global offset of tile-local index r * (block size)
    uint32_t coff_hi[16];  // compact index of tile-local index r * (block size)
    int32_t sb[12], cb[12];
    int32_t k, pad;
};

// One circuit's pass inside a batched launch (nblk blocks; the launch's block
// table maps each workgroup to (entry, local block)).
struct TileEntry {
    const void* phi_src;
    void* phi;
    void* lam;
    int64_t part_off;  // first partial of this entry (slot-major, nblk per slot)
    int32_t args, nblk, pad0, pad1;
};
struct PauliEntry {
    const void* psi;
    void* lam;
    uint64_t N;
    int64_t part_off;
    int32_t g0, ng, nblk, pad;
};
struct ReduceEntry {
    int64_t off;
    int32_t n, out;
};

struct PauliGroupDev {
    uint64_t x;
    int32_t t0, nt;
    // Byte-table evaluation for groups with many terms: the group's weight at
    // source index s is sum_t w_t (-1)^{parity(s & z_t)}; the parity vector
    // (bit t) is linear in s, so it is the XOR of per-index-bit columns, and
    // the weight is the sum over its bytes of 256-entry tables.
    int32_t lut;      // -1: term loop; else table slot (0 or 1) of this observable
    int32_t nb;       // byte tables (ceil(nt / 8))
    int64_t lut_off;  // first complex entry of the tables in the aux array (in doubles)
    int64_t col_off;  // first of the 64 per-index-bit parity columns in the aux array
};
// generator class code of a LAYER1 op (its lcval)
enum LayerGen : uint32_t { LG_NONE = 0, LG_X = 1, LG_Y = 2, LG_DENSE = 3, LG_DIAG = 4 };
constexpr int PAULI_LUT_MIN_TERMS = 16;
constexpr int PAULI_LUT_MAX_TABLES = 12;  // 12 x 256 x 16 B = 48 KiB of LDS
struct PauliTermDev {
    uint64_t z;
    double wre, wim;  // coeff * i^{popcount(x & z)}
};

// ------------------------------------------------------------------ kernel families (profiling)

enum KernelKind : int {
    KK_INIT = 0, KK_GATE1, KK_DIAG1, KK_GATE2, KK_GATEK, KK_TILE1, KK_TILE2,
    KK_PAULI, KK_PAULI_LAMBDA, KK_REDUCE, KK_COPY, KK_PROBS, KK_SPARSE, KK_SAMPLE, KK_DENSE, KK_COUNT
};
extern const char* const kKernelNames[KK_COUNT];

// ------------------------------------------------------------------ launchers (kernels.hip)
// T is double (QSV_C128) or float (QSV_C64); every pointer is device memory.

struct Mat2 { double re[4], im[4]; };
struct Mat4 { double re[16], im[16]; };

template <typename T> hipError_t launch_init(hipStream_t s, void* psi, uint64_t N, uint64_t basis);
// nt: non-temporal (streaming) stores
template <typename T> hipError_t launch_gate1(hipStream_t s, void* psi, uint64_t n_items, const Expand& ex,
                                              uint64_t setmask, uint64_t tbit, int cls, const Mat2& m, bool nt);
template <typename T> hipError_t launch_diag1(hipStream_t s, void* psi, uint64_t n_items, const Expand& ex,
                                              uint64_t setmask, double dre, double dim, bool nt);
template <typename T> hipError_t launch_gate2(hipStream_t s, void* psi, uint64_t n_items, const Expand& ex,
                                              uint64_t setmask, uint64_t b0, uint64_t b1, int cls, const Mat4& m,
                                              bool nt);
template <typename T> hipError_t launch_gatek_low(hipStream_t s, void* psi, uint64_t n_chunks, const Expand& ex,
                                                  uint64_t setmask, int k, const int32_t* tbits, uint32_t lcm,
                                                  uint32_t lcv, const void* mat, bool nt);
template <typename T> hipError_t launch_gatek(hipStream_t s, void* psi, uint64_t n_items, const Expand& ex,
                                              uint64_t setmask, int k, const int32_t* tbits, const void* mat,
                                              bool nt);
// mfma: the 6-qubit complex128 case on the FP64 matrix cores (k_dense6_mfma)
template <typename T> hipError_t launch_dense(hipStream_t s, void* psi, const DenseArgs& a, const void* mat, bool nt,
                                              bool mfma);
size_t dense_lds_bytes(int k, int elem_bytes);
int dense_threads(int k);  // block size of the dense kernel for k targets
template <typename T> hipError_t launch_tile(hipStream_t s, bool two, bool generic, const void* phi_src, void* phi,
                                             void* lam, const TileArgs& a,
                                             const TOp* ops, const void* coef, const uint64_t* words,
                                             double* partials, int grid, int nthr, int R, size_t lds_bytes);
// per (precision, one or two vectors): defined in k_tile.h, instantiated in tile_*.hip
template <typename T, bool TWO> hipError_t launch_tile_v(hipStream_t s, bool generic, const void* phi_src, void* phi,
                                                         void* lam, const TileArgs& a, const TOp* ops,
                                                         const void* coef, const uint64_t* words, double* partials,
                                                         int grid, int nthr, int R, size_t lds_bytes);
template <typename T, bool TWO> hipError_t launch_tile_batch_v(hipStream_t s, bool generic, const TileEntry* entries,
                                                               const int32_t* blk_entry, const TileArgs* args,
                                                               const TOp* ops, const void* coef,
                                                               const uint64_t* words, double* partials, int blocks,
                                                               int nthr, int R, size_t lds);
template <typename T> hipError_t launch_tile_batch(hipStream_t s, bool two, bool generic, const TileEntry* entries,
                                                   const int32_t* blk_entry, const TileArgs* args, const TOp* ops,
                                                   const void* coef, const uint64_t* words, double* partials,
                                                   int blocks, int nthr, int R, size_t lds_bytes);
template <typename T> hipError_t launch_pauli_batch(hipStream_t s, bool write_lambda, const PauliEntry* entries,
                                                    const int32_t* blk_entry, const PauliGroupDev* groups,
                                                    const PauliTermDev* terms, const uint64_t* aux, int lut_tables,
                                                    double* partials, int blocks);
hipError_t launch_reduce_batch(hipStream_t s, const ReduceEntry* re, int n, const double* partials, double* out);
template <typename T> hipError_t launch_pauli(hipStream_t s, bool write_lambda, bool norm2, const void* psi,
                                              void* lam, uint64_t N, const PauliGroupDev* groups, int n_groups,
                                              const PauliTermDev* terms, const uint64_t* aux, int lut_tables,
                                              double* partials, int grid);
template <typename T> hipError_t launch_sparse(hipStream_t s, const void* psi, uint64_t N, const int64_t* row_ptr,
                                               const int64_t* col, const double* val, double* partials, int grid);
template <typename T> hipError_t launch_chunk_norms(hipStream_t s, const void* psi, int clog2, uint64_t n_chunks,
                                                    double* sums);
template <typename T> hipError_t launch_sample(hipStream_t s, const void* psi, int clog2, const int64_t* chunk,
                                               const double* resid, uint64_t* out, int64_t n);
template <typename T> hipError_t launch_probs(hipStream_t s, const void* psi, uint64_t n_rest, const Expand& ex,
                                              const uint64_t* binbits, int n_bins, int gx, double* partials);
hipError_t launch_reduce(hipStream_t s, const double* partials, int n_blocks, int n_slots, double* out);

// Scratch of the allocation-free entry point: a static device array of this
// size in kernels.hip; its device address is taken once per device.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)8 << 20;
hipError_t noalloc_scratch_address(void** ptr);

int tile_lds_bytes(int b, bool two, int elem_bytes, int nslots, int zt_n, int n_zop = 0, int n_outer = 0);
int pauli_grid(uint64_t N);

// ------------------------------------------------------------------ host gate model (gates.cpp)

// One unitary factor: matrix m (2^k x 2^k, first target = msb) on targets tw,
// applied when every control wire cw[j] holds cv[j].
struct Factor {
    int k = 0;
    int tw[8] = {0};
    int nc = 0;
    int cw[8] = {0};
    int cv[8] = {0};
    std::vector<cd> m;
    // derivative of a trainable angle slot: contribution to d/dparams[param]
    // is coef * Im<lam|G|phi> with G on the targets under the same controls
    bool has_dot = false;
    int param = -1;
    double coef = 0.0;
    std::vector<cd> g;
    // exp(-i zangle/2 Z..Z) on the targets without controls (RZ, IsingZZ, MultiRZ)
    bool zrot = false;
    double zangle = 0.0;
    // the angle symbolically: zscale * params[zparam] (zparam < 0: constant)
    int zparam = -1;
    double zscale = 0.0;
    int src_op = -1;
};

// Expand op into factors.  decompose: split Rot/U3/CRot into their one-angle
// factors and attach derivative data (adjoint); otherwise one factor per op.
void op_factors(const qsv_op& op, const double* params, const double* matrices, bool decompose,
                std::vector<Factor>& out);

int gate_own_wires(int gate);   // 0 = variable width; -1 = unknown gate
int gate_n_angles(int gate);

// ------------------------------------------------------------------ planner (plan.cpp)

struct Item {
    bool dot;        // generator inner product (else apply factor matrix)
    bool zrot = false;  // Z-parity rotation (a phase table in the tile pass's LDS)
    int f;           // factor index
    uint64_t xbits;  // index bits the item mixes (targets of a non-diagonal matrix)
    uint64_t zbits;  // index bits it acts on diagonally (controls, diagonal targets)
};

struct Pass {
    uint64_t S = 0;           // tile bits (global index bit mask)
    std::vector<int> items;   // execution order
};

struct PlanOptions {
    int b = 12;          // tile bits
    int low = 4;         // coalescing low bits kept in every tile
    bool fusion = true;
    bool layers = true;  // one-qubit runs inside register groups as LAYER1 sub-ops
    int max_scan = 2048; // look-ahead window of the greedy planner
    bool ws = false;     // warp-specialised tile passes where they fit (TILE_WS)
    // LDS a tile pass may spend beyond its tile: each inner product holds a
    // slot accumulator (slot_bytes), each Z-parity rotation at most two
    // phase-table entries (ztab_bytes); a pass closes before exceeding it
    int64_t slot_bytes = 0, ztab_bytes = 0, lds_budget = INT64_MAX;
};

constexpr int LDS_PER_CU = 160 * 1024;
// Group-only tile passes of >= 2048 amplitudes run warp-specialised (load
// waves fill a second tile buffer while compute waves run the first) when
// both buffers fit the CU's LDS: one persistent block per CU of the MI355X.
constexpr int TILE_WS_GRID = 256;

std::vector<Pass> plan_passes(const std::vector<Item>& items, int n, const PlanOptions& opt);
Item make_item(const Factor& f, bool dot, int fidx, int n);

}  // namespace qsv
