// C-ABI entry points of libqsv: context/state lifetime, validation, lowering
// of planned passes into kernel launches, expectation values and the adjoint
// Jacobian (paper Sec. 2.1-2.2; the adjoint method of Jones & Gacon cited in
// Sec. 2.1 and Sec. 3.1.1).
#include <algorithm>
#include <array>
#include <chrono>
#include <atomic>
#include <exception>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>

#include "qsv_internal.h"

using namespace qsv;

// ------------------------------------------------------------------ errors

namespace {
thread_local std::string g_thread_err;

struct QsvError : std::runtime_error {
    qsv_status st;
    QsvError(qsv_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};

[[noreturn]] void fail(qsv_status s, const std::string& m) { throw QsvError(s, m); }

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) fail(QSV_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCHK(x) hip_check((x), #x)

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};
}  // namespace

struct qsv_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    int64_t opt_fusion = 1, opt_tile_bits = 0, opt_tile_bits_adj = 0, opt_low_bits = 0, opt_profile = 0,
            opt_nontemporal = 0, opt_layers = 1, opt_tile_ws = 0, opt_dense_mfma = 0;
    void* scratch = nullptr;  // this device's allocation-free scratch (qsv_expval_noalloc)
    // fault injection for tests of the error paths (QSV_OPT_TEST_*)
    int64_t test_alloc_limit = 0, test_fail_launch = 0;
    DevBuf ops, coef, words, partials, slots, pgroups, pterms, paux, ws0, ws1, binbits, csr_ptr, csr_col, csr_val,
        smp_chunk, smp_resid, smp_out;
    void* pin = nullptr;
    size_t pin_bytes = 0;
    hipEvent_t pin_ev = nullptr;
    bool pin_pending = false;
    struct Rec {
        int kind;
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> ev_pool;
    int64_t st_launch[KK_COUNT] = {0};
    double st_ms[KK_COUNT] = {0}, st_bytes[KK_COUNT] = {0};
};

struct qsv_state {
    qsv_ctx* ctx;
    int n;
    qsv_dtype dt;
    void* ptr;
    bool owned;
};

namespace {

template <typename F>
qsv_status guard(qsv_ctx* ctx, F&& f) {
    try {
        f();
        return QSV_OK;
    } catch (const QsvError& e) {
        g_thread_err = e.what();
        if (ctx) ctx->err = e.what();
        return e.st;
    } catch (const std::bad_alloc&) {
        g_thread_err = "host allocation failed";
        if (ctx) ctx->err = g_thread_err;
        return QSV_ERR_OOM;
    } catch (const std::exception& e) {
        g_thread_err = e.what();
        if (ctx) ctx->err = e.what();
        return QSV_ERR_ARG;
    }
}

void set_device(qsv_ctx* c) { HIPCHK(hipSetDevice(c->device)); }

// hipMalloc, except that with QSV_OPT_TEST_ALLOC_LIMIT set an allocation
// above the limit fails as if the device were out of memory.
hipError_t dev_malloc(qsv_ctx* c, void** p, size_t bytes) {
    if (c->test_alloc_limit > 0 && bytes > (size_t)c->test_alloc_limit) return hipErrorOutOfMemory;
    return hipMalloc(p, bytes);
}

void ensure(qsv_ctx* c, DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (b.bytes >= bytes) return;
    if (b.p) {
        HIPCHK(hipStreamSynchronize(c->stream));
        HIPCHK(hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    const size_t want = std::max(bytes, (size_t)4096);
    hipError_t e = dev_malloc(c, &b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(QSV_ERR_OOM, "device allocation of " + std::to_string(want) + " bytes failed");
    }
    b.bytes = want;
}

void release(DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

// Stage host data into pinned memory and copy it to the device buffers, all
// asynchronous on the context stream.  The pinned area is reused only after
// the previous copies out of it completed.
struct Upload {
    DevBuf* dst;
    const void* src;
    size_t bytes;
};
void upload(qsv_ctx* c, std::initializer_list<Upload> ups) {
    size_t total = 0;
    for (auto& u : ups) total += (u.bytes + 255) & ~(size_t)255;
    if (c->pin_pending) {
        HIPCHK(hipEventSynchronize(c->pin_ev));
        c->pin_pending = false;
    }
    if (c->pin_bytes < total) {
        if (c->pin) HIPCHK(hipHostFree(c->pin));
        c->pin = nullptr;
        const size_t want = std::max(total, (size_t)1 << 20);
        if (hipHostMalloc(&c->pin, want, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            c->pin_bytes = 0;
            fail(QSV_ERR_OOM, "pinned host allocation failed");
        }
        c->pin_bytes = want;
    }
    size_t off = 0;
    for (auto& u : ups) {
        if (!u.bytes) continue;
        ensure(c, *u.dst, u.bytes);
        char* p = (char*)c->pin + off;
        std::memcpy(p, u.src, u.bytes);
        HIPCHK(hipMemcpyAsync(u.dst->p, p, u.bytes, hipMemcpyHostToDevice, c->stream));
        off += (u.bytes + 255) & ~(size_t)255;
    }
    HIPCHK(hipEventRecord(c->pin_ev, c->stream));
    c->pin_pending = true;
}

hipEvent_t get_event(qsv_ctx* c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    return e;
}

// Times one launch when profiling is on.
struct Timed {
    qsv_ctx* c;
    int kind;
    double bytes;
    hipEvent_t a = nullptr;
    Timed(qsv_ctx* c_, int k, double by) : c(c_), kind(k), bytes(by) {
        if (c->test_fail_launch > 0 && --c->test_fail_launch == 0)
            fail(QSV_ERR_HIP, std::string("injected failure of a ") + qsv::kKernelNames[kind] +
                                  " launch (QSV_OPT_TEST_FAIL_LAUNCH)");
        if (c->opt_profile) {
            a = get_event(c);
            HIPCHK(hipEventRecord(a, c->stream));
        }
    }
    void done(hipError_t launch_err) {
        hip_check(launch_err, qsv::kKernelNames[kind]);
        if (a) {
            hipEvent_t b = get_event(c);
            HIPCHK(hipEventRecord(b, c->stream));
            c->recs.push_back({kind, a, b, bytes});
            a = nullptr;
        }
    }
};

void flush_stats(qsv_ctx* c) {
    if (c->recs.empty()) return;
    HIPCHK(hipStreamSynchronize(c->stream));
    for (auto& r : c->recs) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
        c->st_launch[r.kind] += 1;
        c->st_ms[r.kind] += ms;
        c->st_bytes[r.kind] += r.bytes;
        c->ev_pool.push_back(r.a);
        c->ev_pool.push_back(r.b);
    }
    c->recs.clear();
}

// ------------------------------------------------------------------ validation

void validate_ops_impl(int n, const qsv_op* ops, size_t n_ops, size_t n_params, size_t n_mat, const double* params,
                       const double* matrices) {
    if (n < 1 || n > QSV_MAX_QUBITS) fail(QSV_ERR_ARG, "n_qubits out of range");
    if (n_ops && !ops) fail(QSV_ERR_ARG, "ops is NULL");
    for (size_t i = 0; i < n_ops; ++i) {
        const qsv_op& o = ops[i];
        const std::string at = " (op " + std::to_string(i) + ")";
        const int own = gate_own_wires(o.gate);
        if (own < 0) fail(QSV_ERR_UNSUPPORTED, "unknown gate id " + std::to_string(o.gate) + at);
        if (o.n_wires < 1 || o.n_wires > QSV_MAX_OP_WIRES || o.n_wires > n)
            fail(QSV_ERR_WIRE, "bad wire count" + at);
        if (o.n_ctrls < 0 || o.n_ctrls >= o.n_wires) fail(QSV_ERR_WIRE, "bad control count" + at);
        if (o.n_ctrls < 32 && (o.ctrl_values >> o.n_ctrls) != 0) fail(QSV_ERR_ARG, "ctrl_values has bits beyond n_ctrls" + at);
        const int k = o.n_wires - o.n_ctrls;
        if (own > 0 && k != own) fail(QSV_ERR_WIRE, "gate takes " + std::to_string(own) + " own wires" + at);
        if (o.gate == QSV_GATE_UNITARY && k > 6) fail(QSV_ERR_UNSUPPORTED, "QubitUnitary wider than 6 wires" + at);
        for (int a = 0; a < o.n_wires; ++a) {
            if (o.wires[a] < 0 || o.wires[a] >= n) fail(QSV_ERR_WIRE, "wire out of range" + at);
            for (int b = 0; b < a; ++b)
                if (o.wires[a] == o.wires[b]) fail(QSV_ERR_WIRE, "repeated wire" + at);
        }
        for (int s = 0; s < gate_n_angles(o.gate); ++s) {
            if (o.param[s] < -1 || (o.param[s] >= 0 && (size_t)o.param[s] >= n_params))
                fail(QSV_ERR_PARAM, "parameter index out of range" + at);
            if (o.param[s] >= 0 && !params) fail(QSV_ERR_ARG, "params is NULL" + at);
        }
        if (o.gate == QSV_GATE_UNITARY) {
            const size_t d = (size_t)1 << (2 * k);
            if (!matrices) fail(QSV_ERR_ARG, "matrices is NULL" + at);
            if (o.matrix_offset < 0 || (size_t)o.matrix_offset + d > n_mat)
                fail(QSV_ERR_PARAM, "matrix_offset out of range" + at);
        }
    }
}

void validate_obs_impl(int n, const qsv_pauli_sum* obs, size_t n_obs) {
    if (n_obs && !obs) fail(QSV_ERR_ARG, "observables are NULL");
    const uint64_t all = n >= 64 ? ~0ull : ((1ull << n) - 1);
    for (size_t o = 0; o < n_obs; ++o) {
        const qsv_pauli_sum& h = obs[o];
        if (h.n_terms < 0) fail(QSV_ERR_ARG, "negative term count");
        if (h.n_terms && (!h.coeff || !h.x_mask || !h.z_mask)) fail(QSV_ERR_ARG, "observable arrays are NULL");
        for (int64_t t = 0; t < h.n_terms; ++t)
            if ((h.x_mask[t] | h.z_mask[t]) & ~all) fail(QSV_ERR_WIRE, "Pauli mask beyond n_qubits");
    }
}

qsv_ctx* state_ctx(qsv_state* s) {
    if (!s) fail(QSV_ERR_ARG, "state is NULL");
    return s->ctx;
}

size_t elem_bytes(qsv_dtype d) { return d == QSV_C128 ? 16 : 8; }

// ------------------------------------------------------------------ lowering

struct Step {
    enum Type { TILE, GATE1, DIAG1, GATE2, GATEK, GATEK_LOW, DENSE } type = TILE;
    // tile
    TileArgs ta{};
    int grid = 1, nthr = 1, R = 1;
    size_t lds = 0;
    int nslots = 0, slot_base = 0;
    bool generic = false;  // the pass holds standalone (non-group) tile ops
    // streaming gate
    Expand ex{};
    uint64_t n_items = 0, setmask = 0, tbit = 0, b0 = 0, b1 = 0;
    int cls = 0, k = 0;
    int32_t tb[6] = {0};
    uint32_t lcm = 0, lcv = 0;  // GATEK_LOW: controls inside the 64-amplitude chunk
    Mat2 m2{};
    Mat4 m4{};
    int64_t coff = 0;
    double dre = 0, dim = 0;
    DenseArgs da{};  // DENSE
    double bytes = 0;
};

struct Program {
    std::vector<TOp> tops;
    std::vector<cd> coef;
    std::vector<uint64_t> words;
    std::vector<Step> steps;
    std::vector<std::pair<int, double>> slot_param;  // global slot -> (param, coef)
    size_t max_partials = 0;
};

int classify1(const std::vector<cd>& m) {
    if (m[1] == 0.0 && m[2] == 0.0) return MC_DIAG;
    if (m[0] == 0.0 && m[3] == 0.0) return MC_ANTI;
    bool real = true;
    for (int j = 0; j < 4; ++j) real = real && m[j].imag() == 0.0;
    if (real) return MC_REAL;
    if (m[0].imag() == 0.0 && m[3].imag() == 0.0 && m[1].real() == 0.0 && m[2].real() == 0.0) return MC_RIRI;
    return MC_DENSE;
}

// generator classes of one-target inner products
int classify_gen1(const std::vector<cd>& g) {
    if (g[0] == 0.0 && g[3] == 0.0 && g[1] == 1.0 && g[2] == 1.0) return MC_PX;
    if (g[0] == 0.0 && g[3] == 0.0 && g[1] == cd(0.0, -1.0) && g[2] == cd(0.0, 1.0)) return MC_PY;
    // real diagonal (Z, the |1><1| projector of PhaseShift)
    if (g[1] == 0.0 && g[2] == 0.0 && g[0].imag() == 0.0 && g[3].imag() == 0.0) return MC_DIAG;
    return MC_DENSE;
}

int classify2(const std::vector<cd>& m) {
    bool diag = true;
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            if (r != c && m[r * 4 + c] != 0.0) diag = false;
    if (diag) return MC_DIAG;
    bool mid = m[0] == 1.0 && m[15] == 1.0;
    for (int j = 0; j < 4 && mid; ++j) {
        if (j != 0 && (m[0 * 4 + j] != 0.0 || m[j * 4 + 0] != 0.0)) mid = false;
        if (j != 3 && (m[3 * 4 + j] != 0.0 || m[j * 4 + 3] != 0.0)) mid = false;
    }
    return mid ? MC_MID : MC_DENSE;
}

std::vector<cd> maybe_dag(const std::vector<cd>& m, int dim, bool d) {
    if (!d) return m;
    std::vector<cd> o(m.size());
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c) o[(size_t)c * dim + r] = std::conj(m[(size_t)r * dim + c]);
    return o;
}

uint64_t wire_bit(int n, int w) { return 1ull << (n - 1 - w); }

uint64_t deposit(uint64_t v, const int* sb, int nb) {
    uint64_t o = 0;
    for (int j = 0; j < nb; ++j)
        if ((v >> j) & 1) o |= 1ull << sb[j];
    return o;
}

uint64_t parity_bits_host(uint64_t x, const std::vector<uint64_t>& z) {
    uint64_t p = 0;
    for (size_t j = 0; j < z.size(); ++j) p |= (uint64_t)(__builtin_popcountll(x & z[j]) & 1) << j;
    return p;
}

int tile_grid(uint64_t n_tiles) { return (int)std::min<uint64_t>(n_tiles, 4096); }

// One lowered tile operation before grouping.
struct Proto {
    enum Kind { APPLY, DOT, DIAG, DOTDIAG, ZPHASE, DOTZSUM } kind;
    int f = -1;                  // factor
    std::vector<uint64_t> z;     // Z-parity masks (ZPHASE / DOTZSUM)
    double angle = 0.0;          // ZPHASE
    uint32_t tbits = 0;          // tile-local bits mixed (APPLY / DOT)
    uint32_t dbits = 0;          // tile-local bits acted on diagonally (controls, diagonal targets)
    int k = 0;                   // targets
    bool is_dot() const { return kind == DOT || kind == DOTDIAG || kind == DOTZSUM; }
};

// Reorder the protos of a grouped pass so that fewer register groups are
// needed: list scheduling that keeps every pair of non-commuting protos in
// order (one mixes a bit the other mixes or acts on diagonally; two inner
// products always commute, and so do two diagonal ops) and, at each step,
// takes the first ready proto (in the original order) whose mixed bits fit
// the open group; a group closes when no ready proto fits.  Keeping the
// original order where possible keeps runs on distinct positions together, so
// they still form layers.  Passes with a standalone wide matrix keep their
// order.
std::vector<Proto> schedule_groups(const std::vector<Proto>& pr, int GB) {
    const size_t P = pr.size();
    for (const Proto& p : pr)
        if ((p.kind == Proto::APPLY || p.kind == Proto::DOT) && p.k > 2) return pr;
    auto is_dot = [](const Proto& p) { return p.kind == Proto::DOT || p.kind == Proto::DOTDIAG || p.kind == Proto::DOTZSUM; };
    std::vector<int> npred(P, 0);
    std::vector<std::vector<int>> succ(P);
    for (size_t i = 0; i < P; ++i)
        for (size_t j = i + 1; j < P; ++j) {
            if (is_dot(pr[i]) && is_dot(pr[j])) continue;
            const uint32_t ai = pr[i].tbits | pr[i].dbits, aj = pr[j].tbits | pr[j].dbits;
            if ((pr[i].tbits & aj) || (pr[j].tbits & ai)) {
                succ[i].push_back((int)j);
                ++npred[j];
            }
        }
    std::vector<Proto> out;
    out.reserve(P);
    std::vector<char> done(P, 0);
    uint32_t Q = 0;
    while (out.size() < P) {
        // the first ready op (original order) that fits the open group
        int pick = -1;
        for (size_t i = 0; i < P; ++i) {
            if (done[i] || npred[i]) continue;
            if (__builtin_popcount(Q | pr[i].tbits) <= GB) {
                pick = (int)i;
                break;
            }
        }
        if (pick < 0) {  // nothing fits the open group: start a new one
            Q = 0;
            continue;
        }
        done[pick] = 1;
        Q |= pr[pick].tbits;
        out.push_back(pr[pick]);
        for (int j : succ[pick]) --npred[j];
    }
    return out;
}

// Lower one planned pass into a k_tile step.
void lower_tile(Program& P, const std::vector<Factor>& F, const std::vector<Item>& items, const Pass& pass, int n,
                bool two, bool dagger, size_t eb, bool layers = true, bool ws = false) {
    Step st;
    st.type = Step::TILE;
    int sb[16], b = 0;
    for (int bit = 0; bit < n; ++bit)
        if ((pass.S >> bit) & 1) sb[b++] = bit;
    int rank[64];
    for (int j = 0; j < b; ++j) rank[sb[j]] = j;
    const int nthr_log2 = std::min(b, 8);
    const int nthr = 1 << nthr_log2, R = 1 << (b - nthr_log2);
    if (R > (1 << TILE_MAX_R_LOG2)) fail(QSV_ERR_UNSUPPORTED, "tile too large");
    TileArgs& a = st.ta;
    std::memset(&a, 0, sizeof a);
    a.out_scale = 1.0;
    // Factored layers (classes RIRI_D/O, REAL_D/O) run a scaled copy of their
    // matrices, so the tile holds the true amplitudes divided by tscale (the
    // product of the factors applied so far in the pass, the same for every
    // tile and for phi and lambda); an inner product taken at that point is
    // tscale^2 times too small, which its slot coefficient undoes, and the
    // write-back multiplies by the final tscale.
    double tscale = 1.0;
    a.outer = make_expand(std::vector<int>(sb, sb + b));
    a.n_tiles = 1ull << (n - b);
    for (int r = 0; r < R; ++r) a.offhi[r] = deposit((uint64_t)r << nthr_log2, sb, b);
    for (int j = 0; j < b; ++j) a.sb[j] = sb[j];
    a.b = b;
    a.n_outer = n - b;
    a.nthr_log2 = nthr_log2;
    a.op0 = (int)P.tops.size();
    st.nthr = nthr;
    st.R = R;
    st.grid = tile_grid(a.n_tiles);
    st.slot_base = (int)P.slot_param.size();

    // order: inside each run of diagonal items, inner products first, then
    // un-applies (diagonal matrices commute)
    std::vector<int> order;
    {
        size_t i = 0;
        const auto& it = pass.items;
        while (i < it.size()) {
            if (items[it[i]].xbits) {
                order.push_back(it[i]);
                ++i;
                continue;
            }
            size_t j = i;
            while (j < it.size() && !items[it[j]].xbits) ++j;
            for (size_t q = i; q < j; ++q)
                if (items[it[q]].dot) order.push_back(it[q]);
            for (size_t q = i; q < j; ++q)
                if (!items[it[q]].dot) order.push_back(it[q]);
            i = j;
        }
    }

    // protos, merging Z-parity rotations of equal angle and inner products of
    // equal (param, coefficient)
    std::vector<Proto> protos;
    std::vector<std::pair<int, double>> proto_slot;  // for dot protos
    auto zmask_of = [&](const Factor& g) {
        uint64_t zm = 0;
        for (int i = 0; i < g.k; ++i) zm |= wire_bit(n, g.tw[i]);
        return zm;
    };
    auto local_mask = [&](uint64_t global) {
        uint32_t m = 0;
        for (int j = 0; j < b; ++j)
            if ((global >> sb[j]) & 1) m |= 1u << j;
        return m;
    };
    size_t q = 0;
    while (q < order.size()) {
        const Item& it = items[order[q]];
        const Factor& f = F[it.f];
        Proto pr;
        pr.f = it.f;
        pr.k = f.k;
        pr.dbits = local_mask(it.zbits);
        if (!it.xbits && f.zrot && (it.dot || true)) {
            size_t e = q;
            if (it.dot) {
                pr.kind = Proto::DOTZSUM;
                while (e < order.size() && pr.z.size() < 64) {
                    const Item& jt = items[order[e]];
                    const Factor& g = F[jt.f];
                    if (!(jt.dot && !jt.xbits && g.zrot && g.param == f.param && g.coef == f.coef)) break;
                    pr.z.push_back(zmask_of(g));
                    pr.dbits |= local_mask(jt.zbits);
                    ++e;
                }
            } else {
                pr.kind = Proto::ZPHASE;
                pr.angle = dagger ? -f.zangle : f.zangle;
                while (e < order.size() && pr.z.size() < 64) {
                    const Item& jt = items[order[e]];
                    const Factor& g = F[jt.f];
                    // merge rotations with the same symbolic angle (parameter
                    // and scale), or equal constant angles: the grouping does
                    // not depend on the parameter values
                    const bool same = f.zparam >= 0 ? (g.zparam == f.zparam && g.zscale == f.zscale)
                                                    : (g.zparam < 0 && g.zangle == f.zangle);
                    if (!(!jt.dot && !jt.xbits && g.zrot && same)) break;
                    pr.z.push_back(zmask_of(g));
                    pr.dbits |= local_mask(jt.zbits);
                    ++e;
                }
            }
            protos.push_back(pr);
            q = e;
            continue;
        }
        const int tbit0 = n - 1 - f.tw[0];
        if (!it.xbits && f.k == 1 && f.nc == 0 && ((pass.S >> tbit0) & 1)) {
            // an uncontrolled one-qubit diagonal (PhaseShift, the phase factors
            // of U3 / Rot) on a tile bit: a 2x2 matrix on a group position, so
            // it runs in register layers instead of evaluating its global
            // index per element
            pr.kind = it.dot ? Proto::DOT : Proto::APPLY;
            pr.tbits = 1u << rank[tbit0];
        } else if (!it.xbits) {
            if (f.k > 6) fail(QSV_ERR_UNSUPPORTED, "diagonal factor wider than 6 targets");
            pr.kind = it.dot ? Proto::DOTDIAG : Proto::DIAG;
        } else {
            if (f.k > 6) fail(QSV_ERR_UNSUPPORTED, "factor wider than 6 targets");
            pr.kind = it.dot ? Proto::DOT : Proto::APPLY;
            for (int i = 0; i < f.k; ++i) pr.tbits |= 1u << rank[n - 1 - f.tw[i]];
        }
        protos.push_back(pr);
        ++q;
    }

    const int GB = two ? GROUP_BITS_TWO : GROUP_BITS_ONE;
    const bool grouped = b >= GB;
    if (grouped && layers) protos = schedule_groups(protos, GB);
    const int nsub = grouped ? (1 << (b - GB)) : 0;
    int nslots = 0;
    // phase tables of the pass, appended contiguously after emission (the
    // kernel copies them to LDS once per launch)
    std::vector<cd> ztab;
    std::vector<std::pair<size_t, int>> zpatch;  // (tops index, offset in ztab)

    auto controls = [&](const Factor& f, TOp& op, bool local_ok) {
        op.lcmask = op.lcval = 0;
        op.gcmask = op.gcval = 0;
        for (int j = 0; j < f.nc; ++j) {
            const uint64_t bit = wire_bit(n, f.cw[j]);
            const int p = n - 1 - f.cw[j];
            if (local_ok && ((pass.S >> p) & 1)) {
                op.lcmask |= 1u << rank[p];
                if (f.cv[j]) op.lcval |= 1u << rank[p];
            } else {
                op.gcmask |= bit;
                if (f.cv[j]) op.gcval |= bit;
            }
        }
    };
    // Emit one proto.  In a group (Q = group bits ascending, tile-local) the
    // targets of local ops are positions in Q and Z-parity tables are indexed
    // by subcube and element; standalone ops use the per-thread / per-r layout.
    auto emit = [&](const Proto& pr, const std::vector<int>* Q, int& dslot) {
        // a Z-parity rotation right after the inner product of the same Z
        // strings in a group joins it (one parity count per element)
        if (Q && pr.kind == Proto::ZPHASE && !P.tops.empty() && P.tops.back().kind == OP_DOTZSUM &&
            P.tops.back().m == (int)pr.z.size() &&
            std::equal(pr.z.begin(), pr.z.end(), P.words.begin() + P.tops.back().woff)) {
            const int m = (int)pr.z.size();
            P.tops.back().kind = OP_ZPHDOT;
            zpatch.push_back({P.tops.size() - 1, (int)ztab.size()});
            for (int cnt = 0; cnt <= m; ++cnt) ztab.push_back(std::exp(cd(0.0, -0.5 * pr.angle * (m - 2 * cnt))));
            return;
        }
        TOp op;
        std::memset(&op, 0, sizeof op);
        op.k = pr.k;
        op.slot = -1;
        op.coff = (int64_t)P.coef.size();
        if (pr.is_dot()) {
            op.slot = nslots++;
            const Factor& f = F[pr.f];
            P.slot_param.push_back({f.param, f.coef * tscale * tscale});
            if (Q) op.aux = dslot++;
        }
        if (pr.kind == Proto::ZPHASE || pr.kind == Proto::DOTZSUM) {
            op.kind = pr.kind == Proto::ZPHASE ? OP_ZPHASE : OP_DOTZSUM;
            op.m = (int)pr.z.size();
            op.woff = (int64_t)P.words.size();
            for (auto x : pr.z) P.words.push_back(x);
            if (Q) {
                op.tb[5] = a.n_zop++;  // its tile-parity slot in LDS
                // per subcube: parity bits of the subcube's global offset;
                // per element: of the element's offset inside the subcube
                std::vector<int> nonq;
                for (int j = 0; j < b; ++j)
                    if (std::find(Q->begin(), Q->end(), j) == Q->end()) nonq.push_back(sb[j]);
                for (int sc = 0; sc < nsub; ++sc) {
                    uint64_t off = 0;
                    for (size_t j = 0; j < nonq.size(); ++j)
                        if ((sc >> j) & 1) off |= 1ull << nonq[j];
                    P.words.push_back(parity_bits_host(off, pr.z));
                }
                for (int e = 0; e < (1 << GB); ++e) {
                    uint64_t off = 0;
                    for (int i = 0; i < GB; ++i)
                        if ((e >> i) & 1) off |= 1ull << sb[(*Q)[i]];
                    P.words.push_back(parity_bits_host(off, pr.z));
                }
            } else {
                for (int t = 0; t < nthr; ++t)
                    P.words.push_back(parity_bits_host(deposit((uint64_t)t, sb, nthr_log2), pr.z));
                for (int r = 0; r < R; ++r) P.words.push_back(parity_bits_host(a.offhi[r], pr.z));
            }
            // per index bit outside the tile (ascending = bit k of the tile
            // number): its parity column; the tile base's parity bits are the
            // XOR of the columns of the tile number's set bits (linear over GF(2))
            for (int g = 0; g < n; ++g)
                if (!((pass.S >> g) & 1)) P.words.push_back(parity_bits_host(1ull << g, pr.z));
            if (pr.kind == Proto::ZPHASE) {
                const int m = (int)pr.z.size();
                zpatch.push_back({P.tops.size(), (int)ztab.size()});
                for (int cnt = 0; cnt <= m; ++cnt)
                    ztab.push_back(std::exp(cd(0.0, -0.5 * pr.angle * (m - 2 * cnt))));
            }
            P.tops.push_back(op);
            return;
        }
        const Factor& f = F[pr.f];
        const int dim = 1 << f.k;
        const bool dot = pr.is_dot();
        if (pr.kind == Proto::DIAG || pr.kind == Proto::DOTDIAG) {
            op.kind = dot ? OP_DOTDIAG : OP_DIAG;
            for (int i = 0; i < f.k; ++i) op.tb[i] = n - 1 - f.tw[i];
            controls(f, op, false);
            const std::vector<cd>& src = dot ? f.g : f.m;
            for (int j = 0; j < dim; ++j) {
                const cd d = src[(size_t)j * dim + j];
                P.coef.push_back((!dot && dagger) ? std::conj(d) : d);
            }
            P.tops.push_back(op);
            return;
        }
        controls(f, op, true);
        const std::vector<cd> mm = dot ? f.g : maybe_dag(f.m, dim, dagger);
        if (Q) {
            for (int i = 0; i < f.k; ++i) {
                const int tl = rank[n - 1 - f.tw[i]];
                op.tb[i] = (int)(std::find(Q->begin(), Q->end(), tl) - Q->begin());
            }
        } else {
            for (int i = 0; i < f.k; ++i) op.tb[i] = rank[n - 1 - f.tw[i]];
        }
        if (!dot && Q && f.k == 1 && P.tops.back().kind == OP_APPLY1) {
            // right after a one-qubit matrix on the same position with the same
            // controls (in this group: the group op precedes its sub-ops): one
            // matrix, the product (the earlier one acts first)
            TOp& pv = P.tops.back();
            if (pv.tb[0] == op.tb[0] && pv.lcmask == op.lcmask && pv.lcval == op.lcval && pv.gcmask == op.gcmask &&
                pv.gcval == op.gcval) {
                cd* m0 = &P.coef[(size_t)pv.coff];
                const cd p[4] = {mm[0] * m0[0] + mm[1] * m0[2], mm[0] * m0[1] + mm[1] * m0[3],
                                 mm[2] * m0[0] + mm[3] * m0[2], mm[2] * m0[1] + mm[3] * m0[3]};
                const std::vector<cd> pm(p, p + 4);
                for (int j = 0; j < 4; ++j) m0[j] = p[j];
                pv.cls = classify1(pm);
                if (pv.cls == MC_ANTI && p[1] == 1.0 && p[2] == 1.0) pv.cls = MC_PX;
                return;
            }
        }
        if (dot) {
            op.kind = f.k == 1 ? OP_DOT1 : (f.k == 2 ? OP_DOT2 : OP_DOTK);
            if (Q && f.k == 1) op.cls = classify_gen1(mm);
        } else {
            op.kind = f.k == 1 ? OP_APPLY1 : (f.k == 2 ? OP_APPLY2 : OP_APPLYK);
            op.cls = f.k == 1 ? classify1(mm) : (f.k == 2 ? classify2(mm) : MC_DENSE);
            // grouped kernels: dense / anti / mid, and diagonal for one qubit
            if (Q && op.cls == MC_DIAG && f.k != 1) op.cls = MC_DENSE;
            // exactly X (a CNOT's target): a register swap in a group
            if (Q && f.k == 1 && op.cls == MC_ANTI && mm[1] == 1.0 && mm[2] == 1.0) op.cls = MC_PX;
        }
        for (auto& x : mm) P.coef.push_back(x);
        P.tops.push_back(op);
    };

    st.generic = !grouped;
    if (!grouped) {
        int dummy = 0;
        for (const Proto& pr : protos) emit(pr, nullptr, dummy);
    } else {
        // greedy groups: consecutive protos whose mixed bits fit in GB bits
        size_t i = 0;
        while (i < protos.size()) {
            const Proto& p0 = protos[i];
            if ((p0.kind == Proto::APPLY || p0.kind == Proto::DOT) && p0.k > 2) {
                st.generic = true;
                int dummy = 0;
                emit(p0, nullptr, dummy);  // standalone k-qubit matrix
                ++i;
                continue;
            }
            uint32_t qmask = 0;
            int ndots = 0;
            size_t e = i;
            while (e < protos.size()) {
                const Proto& pr = protos[e];
                if ((pr.kind == Proto::APPLY || pr.kind == Proto::DOT) && pr.k > 2) break;
                const uint32_t nq = qmask | pr.tbits;
                if (__builtin_popcount(nq) > GB) break;
                if (pr.is_dot() && ndots == GROUP_MAX_DOTS) break;
                qmask = nq;
                ndots += pr.is_dot();
                ++e;
            }
            // pad Q with the highest free tile bits (keeps lanes on low bits)
            for (int j = b - 1; __builtin_popcount(qmask) < GB && j >= 0; --j) qmask |= 1u << j;
            std::vector<int> Q;
            for (int j = 0; j < b; ++j)
                if ((qmask >> j) & 1) Q.push_back(j);
            TOp gop;
            std::memset(&gop, 0, sizeof gop);
            gop.kind = OP_GROUP;
            gop.k = GB;
            for (int t = 0; t < GB; ++t) gop.tb[t] = Q[t];
            gop.m = (int)(e - i);
            gop.slot = -1;
            gop.tb[4] = gop.tb[5] = -1;  // set below: the first two Z-parity sub-ops
            // aux = 1: some sub-op needs the global index of each element
            for (size_t x = i; x < e; ++x)
                if (protos[x].kind == Proto::DIAG || protos[x].kind == Proto::DOTDIAG) gop.aux = 1;
            gop.woff = (int64_t)P.words.size();
            for (int el = 0; el < (1 << GB); ++el) {
                uint64_t off = 0;
                for (int t = 0; t < GB; ++t)
                    if ((el >> t) & 1) off |= 1ull << sb[Q[t]];
                P.words.push_back(off);
            }
            for (int j = 0; j < b; ++j)
                if (!((qmask >> j) & 1)) P.words.push_back((uint64_t)sb[j]);
            const size_t gidx = P.tops.size();
            P.tops.push_back(gop);
            int dslot = 0;
            if (!layers) {
                for (size_t x = i; x < e; ++x) emit(protos[x], &Q, dslot);
            } else {
                // runs of uncontrolled one-qubit matrices and inner products
                // on distinct group positions become one LAYER1 sub-op (ops on
                // different positions commute, so the layer may run them in
                // position order)
                auto pos_of = [&](const Proto& pr) {
                    const int tl = rank[n - 1 - F[pr.f].tw[0]];
                    return (int)(std::find(Q.begin(), Q.end(), tl) - Q.begin());
                };
                auto layer_ok = [&](const Proto& pr) {
                    return (pr.kind == Proto::APPLY || pr.kind == Proto::DOT) && pr.k == 1 && F[pr.f].nc == 0;
                };
                int lg[4] = {-1, -1, -1, -1}, ld[4] = {-1, -1, -1, -1};
                std::vector<size_t> run;
                auto flush_layer = [&]() {
                    if (run.empty()) return;
                    int npos = 0, only = -1;
                    for (int p = 0; p < GB; ++p)
                        if (lg[p] >= 0 || ld[p] >= 0) ++npos, only = p;
                    if (npos == 1) {  // one position: its inner product and matrix as plain ops
                        if (ld[only] >= 0) emit(protos[ld[only]], &Q, dslot);
                        if (lg[only] >= 0) emit(protos[lg[only]], &Q, dslot);
                    } else {
                        TOp op;
                        std::memset(&op, 0, sizeof op);
                        op.kind = OP_LAYER1;
                        op.k = 1;
                        op.slot = -1;
                        op.aux = dslot;
                        bool real = true, riri = true, diag = true;
                        int gcls = LG_NONE;
                        std::vector<cd> mats[4], gens[4];
                        for (int p = 0; p < GB; ++p) {
                            op.tb[p] = -1;
                            mats[p] = {1.0, 0.0, 0.0, 1.0};
                            if (lg[p] >= 0) {
                                mats[p] = maybe_dag(F[protos[lg[p]].f].m, 2, dagger);
                                op.m |= 1 << p;
                            }
                            const auto& m = mats[p];
                            real = real && m[0].imag() == 0 && m[1].imag() == 0 && m[2].imag() == 0 &&
                                   m[3].imag() == 0;
                            riri = riri && m[0].imag() == 0 && m[3].imag() == 0 && m[1].real() == 0 &&
                                   m[2].real() == 0;
                            diag = diag && m[1] == 0.0 && m[2] == 0.0;
                            gens[p] = {0.0, 0.0, 0.0, 0.0};
                            if (ld[p] >= 0) {
                                const Factor& f = F[protos[ld[p]].f];
                                gens[p] = f.g;
                                const int cg = classify_gen1(f.g);
                                const int c = cg == MC_PX ? LG_X
                                            : cg == MC_PY ? LG_Y
                                            : cg == MC_DIAG ? LG_DIAG : LG_DENSE;
                                gcls = gcls == LG_NONE ? c : (gcls == c ? c : LG_DENSE);
                                op.lcmask |= 1u << p;
                                op.tb[p] = nslots++;
                                P.slot_param.push_back({f.param, f.coef});
                                ++dslot;
                            }
                        }
                        op.cls = real ? MC_REAL : (riri ? MC_RIRI : (diag ? MC_DIAG : MC_DENSE));
                        // Factored form of an RX- or RY-like layer (every
                        // position, identities included, with equal diagonal
                        // entries): divide each position's matrix by its
                        // diagonal entry (D form, |entry| >= 1/2) or by its
                        // off-diagonal entry (O form, no identities), so that
                        // one FMA per component applies it; the factors go
                        // into the pass's scale.  Slot coefficients of the
                        // layer's inner products get the scale before their
                        // position's matrix.
                        std::vector<double> fac(GB, 1.0);
                        const bool fr = op.cls == MC_RIRI && (gcls == LG_NONE || gcls == LG_X);
                        const bool fy = op.cls == MC_REAL && (gcls == LG_NONE || gcls == LG_Y);
                        if (fr || fy) {
                            bool dok = true, ook = true;
                            double prod_d = 1.0, prod_o = 1.0;
                            for (int p = 0; p < GB; ++p) {
                                const auto& m = mats[p];
                                const bool eqd = m[0] == m[3] && m[0].imag() == 0.0;
                                dok = dok && eqd && std::abs(m[0].real()) >= 0.5;
                                prod_d *= std::abs(m[0].real());
                                // O: RIRI needs m01 == m10 = i q; REAL needs m01 == -m10
                                const double off = fr ? m[2].imag() : m[2].real();
                                const bool offok = fr ? (m[1] == m[2]) : (m[1] == -m[2]);
                                ook = ook && eqd && offok && std::abs(off) >= 0.5;
                                prod_o *= std::abs(off);
                            }
                            // keep the pass scale well inside both precisions' range
                            dok = dok && tscale * prod_d >= 1e-18;
                            ook = ook && tscale * prod_o >= 1e-18;
                            if (dok || ook) {
                                for (int p = 0; p < GB; ++p) {
                                    auto& m = mats[p];
                                    const cd f = dok ? m[0] : (fr ? cd(m[2].imag(), 0.0) : m[2]);
                                    fac[p] = f.real();
                                    for (auto& x : m) x /= f;
                                    // exact unit entries (the kernel does not read them)
                                    if (dok) m[0] = m[3] = 1.0;
                                    else if (fr) m[1] = m[2] = cd(0.0, 1.0);
                                    else m[1] = -1.0, m[2] = 1.0;
                                }
                                op.cls = fr ? (dok ? MC_RIRI_D : MC_RIRI_O) : (dok ? MC_REAL_D : MC_REAL_O);
                            }
                        }
                        // the kernel takes each position's inner product, then
                        // applies its matrix: slot scales in that order
                        {
                            size_t sp = P.slot_param.size();
                            for (int p = 0; p < GB; ++p)
                                if (ld[p] >= 0) --sp;
                            for (int p = 0; p < GB; ++p) {
                                if (ld[p] >= 0) P.slot_param[sp++].second *= tscale * tscale;
                                tscale *= fac[p];
                            }
                        }
                        op.lcval = (uint32_t)gcls;
                        op.coff = (int64_t)P.coef.size();
                        for (int p = 0; p < GB; ++p) {
                            if (gcls == LG_DENSE || gcls == LG_DIAG)
                                for (auto x : gens[p]) P.coef.push_back(x);
                            for (auto x : mats[p]) P.coef.push_back(x);
                        }
                        P.tops.push_back(op);
                    }
                    run.clear();
                    for (int p = 0; p < 4; ++p) lg[p] = ld[p] = -1;
                };
                // Layers by depth (as-soon-as-possible levels).  Each
                // position's layer ops form units (an optional inner product,
                // then an optional matrix); a unit's level is one above the
                // level of the last op on its position, and any other op's
                // level is one above the last ops on the positions it touches
                // (all positions for diagonal and Z-parity ops).  Ops of one
                // level touch disjoint positions and so commute, and an inner
                // product on one position is unchanged by gates on others
                // (they act on phi and lambda alike and commute with its
                // generator), so emitting by level -- the level's units as one
                // layer, then its other ops -- is exact.  U3 / Rot
                // decompositions then give full PhaseShift, RY or RZ layers
                // instead of one layer per gate, and a CNOT only orders the
                // two positions it touches.
                auto posmask = [&](uint32_t bits) {
                    uint32_t m = 0;
                    for (int t = 0; t < GB; ++t)
                        if ((bits >> Q[t]) & 1) m |= 1u << t;
                    return m;
                };
                std::vector<int> lvl(GB, -1), open_dot(GB, -1);
                std::vector<std::pair<int, size_t>> order;  // (level, proto)
                for (size_t x = i; x < e; ++x) {
                    const Proto& pr = protos[x];
                    int level;
                    if (layer_ok(pr)) {
                        const int p = pos_of(pr);
                        if (pr.kind == Proto::APPLY && open_dot[p] >= 0) {
                            level = lvl[p];  // the matrix after this unit's inner product
                            open_dot[p] = -1;
                        } else {
                            level = lvl[p] + 1;
                            lvl[p] = level;
                            open_dot[p] = pr.kind == Proto::DOT ? (int)x : -1;
                        }
                    } else {
                        const bool local = (pr.kind == Proto::APPLY || pr.kind == Proto::DOT) && pr.k <= 2;
                        const uint32_t S = local ? posmask(pr.tbits | pr.dbits) : (1u << GB) - 1;
                        level = 0;
                        for (int p = 0; p < GB; ++p)
                            if ((S >> p) & 1) level = std::max(level, lvl[p] + 1);
                        for (int p = 0; p < GB; ++p)
                            if ((S >> p) & 1) {
                                lvl[p] = level;
                                open_dot[p] = -1;
                            }
                    }
                    order.push_back({level, x});
                }
                std::stable_sort(order.begin(), order.end(),
                                 [](const std::pair<int, size_t>& u, const std::pair<int, size_t>& v) {
                                     return u.first < v.first;
                                 });
                // matrix classes a unit's matrix fits (bit 0 real, 1 RIRI,
                // 2 diagonal; all for no matrix) and its generator code
                auto unit_fits = [&](int app) {
                    if (app < 0) return 7u;
                    const std::vector<cd> m = maybe_dag(F[protos[app].f].m, 2, dagger);
                    uint32_t fl = 0;
                    if (m[0].imag() == 0 && m[1].imag() == 0 && m[2].imag() == 0 && m[3].imag() == 0) fl |= 1;
                    if (m[0].imag() == 0 && m[3].imag() == 0 && m[1].real() == 0 && m[2].real() == 0) fl |= 2;
                    if (m[1] == 0.0 && m[2] == 0.0) fl |= 4;
                    return fl;
                };
                auto unit_gen = [&](int dot) {
                    if (dot < 0) return (int)LG_NONE;
                    const int cg = classify_gen1(F[protos[dot].f].g);
                    return cg == MC_PX ? (int)LG_X : cg == MC_PY ? (int)LG_Y : cg == MC_DIAG ? (int)LG_DIAG : (int)LG_DENSE;
                };
                // the class a layer gets from its fits (real, then RIRI, then diagonal)
                auto fit_class = [](uint32_t fl) { return fl & 1 ? 1 : fl & 2 ? 2 : fl & 4 ? 4 : 0; };
                for (size_t q = 0; q < order.size();) {
                    size_t q1 = q;
                    while (q1 < order.size() && order[q1].first == order[q].first) ++q1;
                    int udot[4] = {-1, -1, -1, -1}, uapp[4] = {-1, -1, -1, -1};
                    for (size_t r = q; r < q1; ++r) {
                        const size_t x = order[r].second;
                        if (!layer_ok(protos[x])) continue;
                        const int p = pos_of(protos[x]);
                        if (protos[x].kind == Proto::DOT) udot[p] = (int)x;
                        else uapp[p] = (int)x;
                    }
                    // the level's units (distinct positions) as layers of one
                    // matrix and generator class each; a unit joins a layer
                    // when that keeps the layer's classes
                    bool done[4] = {false, false, false, false};
                    for (int p0 = 0; p0 < GB; ++p0) {
                        if (done[p0] || (udot[p0] < 0 && uapp[p0] < 0)) continue;
                        uint32_t fl = unit_fits(uapp[p0]);
                        int gen = unit_gen(udot[p0]);
                        for (int p = p0; p < GB; ++p) {
                            if (done[p] || (udot[p] < 0 && uapp[p] < 0)) continue;
                            const uint32_t nf = fl & unit_fits(uapp[p]);
                            const int g = unit_gen(udot[p]);
                            if (p != p0) {
                                if (fit_class(nf) != fit_class(fl) && fit_class(fl) != 0) continue;
                                if (gen != LG_NONE && g != LG_NONE && g != gen) continue;
                            }
                            fl = nf;
                            if (gen == LG_NONE) gen = g;
                            done[p] = true;
                            if (udot[p] >= 0) {
                                ld[p] = udot[p];
                                run.push_back((size_t)udot[p]);
                            }
                            if (uapp[p] >= 0) {
                                lg[p] = uapp[p];
                                run.push_back((size_t)uapp[p]);
                            }
                        }
                        flush_layer();
                    }
                    for (size_t r = q; r < q1; ++r)
                        if (!layer_ok(protos[order[r].second])) emit(protos[order[r].second], &Q, dslot);
                    q = q1;
                }
            }
            P.tops[gidx].m = (int)(P.tops.size() - gidx - 1);
            {
                int nz = 0;
                for (int si = 0; si < P.tops[gidx].m && nz < 2; ++si) {
                    const int k = P.tops[gidx + 1 + si].kind;
                    if (k == OP_ZPHASE || k == OP_DOTZSUM || k == OP_ZPHDOT) P.tops[gidx].tb[4 + nz++] = si;
                }
            }
            i = e;
        }
    }
    a.nops = (int)P.tops.size() - a.op0;
    a.nslots = nslots;
    a.out_scale = tscale;
    a.zt_off = (int64_t)P.coef.size();
    a.zt_n = (int)ztab.size();
    for (auto& zp : zpatch) {
        TOp& t = P.tops[zp.first];
        t.coff = a.zt_off + zp.second;
        if (t.kind == OP_ZPHDOT) t.lcval = (uint32_t)zp.second;  // aux is its inner-product index
        else t.aux = zp.second;
    }
    for (auto& x : ztab) P.coef.push_back(x);
    st.nslots = nslots;
    st.lds = (size_t)tile_lds_bytes(b, two, (int)eb, nslots, a.zt_n, a.n_zop, a.n_outer);
    if (st.lds > (size_t)LDS_PER_CU)  // the planner's budget keeps passes below this
        fail(QSV_ERR_UNSUPPORTED, "tile pass needs more LDS than a CU has");
    {
        // the warp-specialised form needs a second tile buffer
        const size_t lds_ws = st.lds + (size_t)(two ? 2 : 1) * ((size_t)1 << b) * eb;
        if (ws && !st.generic && nthr == 256 && R >= 8 && lds_ws <= (size_t)LDS_PER_CU) {
            a.flags |= TILE_WS;
            st.lds = lds_ws;
            st.grid = (int)std::min<uint64_t>(a.n_tiles, TILE_WS_GRID);
        }
    }
    st.bytes = (double)(two ? 4 : 2) * (double)((uint64_t)1 << n) * (double)eb;
    P.max_partials = std::max(P.max_partials, (size_t)nslots * st.grid);
    P.steps.push_back(st);
}

// Lower a one-factor forward pass into a streaming kernel when one fits.
bool lower_single(Program& P, const Factor& f, int n, size_t eb, int low_bits) {
    const int dim = 1 << f.k;
    std::vector<int> pos;
    uint64_t setmask = 0;
    for (int j = 0; j < f.nc; ++j) {
        pos.push_back(n - 1 - f.cw[j]);
        if (f.cv[j]) setmask |= wire_bit(n, f.cw[j]);
    }
    for (int i = 0; i < f.k; ++i) pos.push_back(n - 1 - f.tw[i]);
    std::sort(pos.begin(), pos.end());
    const double N = (double)((uint64_t)1 << n);
    Step st;
    st.n_items = (uint64_t)1 << (n - (int)pos.size());
    st.ex = make_expand(pos);
    st.setmask = setmask;
    const double frac = std::ldexp(1.0, -f.nc);
    if (f.k == 1) {
        const int cls = classify1(f.m);
        st.tbit = wire_bit(n, f.tw[0]);
        if (cls == MC_DIAG && f.m[0] == 1.0) {
            st.type = Step::DIAG1;
            st.setmask |= st.tbit;
            st.dre = f.m[3].real();
            st.dim = f.m[3].imag();
            st.bytes = N * eb * frac;  // read + write of half the (controlled) vector
        } else {
            st.type = Step::GATE1;
            st.cls = cls;
            for (int j = 0; j < 4; ++j) {
                st.m2.re[j] = f.m[j].real();
                st.m2.im[j] = f.m[j].imag();
            }
            st.bytes = 2.0 * N * eb * frac;
        }
    } else if (f.k >= 3 && f.k <= 6 && n - f.nc >= f.k + 6) {
        // LDS-staged dense matrix: targets plus six lane bits per tile
        st.type = Step::DENSE;
        DenseArgs& d = st.da;
        d.k = f.k;
        uint64_t used = 0;
        for (int p : pos) used |= 1ull << p;
        std::vector<int> lane;
        for (int p = 0; p < n && (int)lane.size() < 6; ++p)
            if (!((used >> p) & 1)) lane.push_back(p);
        std::vector<int> tbits;  // tile bits ascending
        for (int i = 0; i < f.k; ++i) tbits.push_back(n - 1 - f.tw[i]);
        for (int p : lane) tbits.push_back(p);
        std::sort(tbits.begin(), tbits.end());
        for (int i = 0; i < f.k + 6; ++i) {
            d.sb[i] = tbits[i];
            const auto li = std::find(lane.begin(), lane.end(), tbits[i]);
            if (li != lane.end()) {
                d.cb[i] = (int)(li - lane.begin());
            } else {
                int t = 0;
                while (n - 1 - f.tw[t] != tbits[i]) ++t;
                d.cb[i] = 6 + (f.k - 1 - t);  // target 0 is the matrix index's msb
            }
        }
        const int nt = dense_threads(f.k), lb = nt == 512 ? 9 : 8;
        const int rl = (64 << f.k) / nt;
        for (int r = 0; r < rl; ++r) {
            uint64_t g = 0;
            uint32_t cc = 0;
            for (int i = lb; i < f.k + 6; ++i)
                if (((r << lb) >> i) & 1) {
                    g |= 1ull << d.sb[i];
                    cc |= 1u << d.cb[i];
                }
            d.goff_hi[r] = g;
            d.coff_hi[r] = cc;
        }
        std::vector<int> outer_pos = tbits;
        for (int j = 0; j < f.nc; ++j) outer_pos.push_back(n - 1 - f.cw[j]);
        std::sort(outer_pos.begin(), outer_pos.end());
        d.outer = make_expand(outer_pos);
        d.setmask = setmask;
        d.n_tiles = (uint64_t)1 << (n - (int)outer_pos.size());
        // the kernel's matrix layout: (wave w, column j, row q of the wave's
        // dim / waves rows), so one input's entries are contiguous per wave
        st.coff = (int64_t)P.coef.size();
        const int nw = nt / 64, rw = dim / nw;
        for (int w = 0; w < nw; ++w)
            for (int j = 0; j < dim; ++j)
                for (int q = 0; q < rw; ++q) P.coef.push_back(f.m[(size_t)(w * rw + q) * dim + j]);
        st.bytes = 2.0 * N * eb * frac;
    } else if (f.k == 2) {
        st.type = Step::GATE2;
        st.cls = classify2(f.m);
        st.b0 = wire_bit(n, f.tw[0]);
        st.b1 = wire_bit(n, f.tw[1]);
        for (int j = 0; j < 16; ++j) {
            st.m4.re[j] = f.m[j].real();
            st.m4.im[j] = f.m[j].imag();
        }
        st.bytes = (st.cls == MC_MID ? 1.0 : 2.0) * N * eb * frac;
    } else if (f.k == 3 && n >= 6 && [&] {
                   for (int i = 0; i < f.k; ++i)
                       if (n - 1 - f.tw[i] >= 6) return false;
                   return true;
               }()) {
        // targets in the lowest six bits: one wavefront per aligned chunk of 64
        // (measured faster than one tuple per thread for k = 3; for k >= 4 the
        // per-lane matrix rows make it LDS-bound, so those keep the other paths)
        (void)low_bits;
        st.type = Step::GATEK_LOW;
        st.k = f.k;
        for (int i = 0; i < f.k; ++i) st.tb[i] = n - 1 - f.tw[i];
        std::vector<int> hi;
        uint64_t set_hi = 0;
        st.lcm = st.lcv = 0;
        for (int j = 0; j < f.nc; ++j) {
            const int p = n - 1 - f.cw[j];
            if (p >= 6) {
                hi.push_back(p - 6);
                if (f.cv[j]) set_hi |= 1ull << (p - 6);
            } else {
                st.lcm |= 1u << p;
                if (f.cv[j]) st.lcv |= 1u << p;
            }
        }
        std::sort(hi.begin(), hi.end());
        st.ex = make_expand(hi);
        st.setmask = set_hi;
        st.n_items = (uint64_t)1 << (n - 6 - (int)hi.size());
        st.coff = (int64_t)P.coef.size();
        for (int j = 0; j < dim * dim; ++j) P.coef.push_back(f.m[j]);
        st.bytes = 2.0 * N * eb * std::ldexp(1.0, -(int)hi.size());
    } else if (f.k <= 5) {
        st.type = Step::GATEK;
        st.k = f.k;
        for (int i = 0; i < f.k; ++i) st.tb[i] = n - 1 - f.tw[i];
        st.coff = (int64_t)P.coef.size();
        for (int j = 0; j < dim * dim; ++j) P.coef.push_back(f.m[j]);
        st.bytes = 2.0 * N * eb * frac;
    } else {
        return false;
    }
    P.steps.push_back(st);
    return true;
}

PlanOptions plan_opts(int64_t tile_bits, int64_t low_bits, int64_t fusion, qsv_dtype dt, bool two,
                      int64_t layers = 1) {
    PlanOptions o;
    const bool c128 = dt == QSV_C128;
    const int eb = c128 ? 16 : 8;
    int b = (int)tile_bits;
    if (b <= 0) b = two ? (c128 ? 11 : 12) : (c128 ? 12 : 13);
    b = std::min(b, 8 + TILE_MAX_R_LOG2);
    // the tile itself must leave room in the CU's LDS for the pass's slot
    // accumulators and phase tables
    while (b > 1 && tile_lds_bytes(b, two, eb, 0, 0) > LDS_PER_CU - 8192) --b;
    o.b = b;
    o.low = low_bits > 0 ? (int)low_bits : (c128 ? 4 : 5);
    o.fusion = fusion != 0;
    o.layers = layers != 0;
    const int nthr = 1 << std::min(b, 8);
    o.slot_bytes = 8 * (nthr >= 64 ? nthr / 16 : 1);
    // two phase-table entries, and (grouped) the op's tile-number columns
    // and current tile parity
    o.ztab_bytes = 2 * eb + 8 * (QSV_MAX_QUBITS + 1);
    o.lds_budget = LDS_PER_CU - tile_lds_bytes(b, two, eb, 0, 0) - 16;
    return o;
}

PlanOptions plan_opts(qsv_ctx* c, qsv_dtype dt, bool two) {
    PlanOptions o = plan_opts(two ? c->opt_tile_bits_adj : c->opt_tile_bits, c->opt_low_bits, c->opt_fusion, dt,
                              two, c->opt_layers);
    o.ws = c->opt_tile_ws != 0;
    return o;
}

Program build_program(const PlanOptions& po, const std::vector<Factor>& F, const std::vector<Item>& items, int n,
                      qsv_dtype dt, bool two, bool dagger, bool allow_streaming = true) {
    Program P;
    const size_t eb = elem_bytes(dt);
    std::vector<Pass> passes = plan_passes(items, n, po);
    for (const Pass& p : passes) {
        if (allow_streaming && !two && p.items.size() == 1 && !items[p.items[0]].dot) {
            if (lower_single(P, F[items[p.items[0]].f], n, eb, po.low)) continue;
        }
        lower_tile(P, F, items, p, n, two, dagger, eb, po.layers, po.ws);
    }
    return P;
}

template <typename T>
struct DevT {};

// Launch every step of a program on (phi, lam).  Slot sums land in
// slots + slot_offset + step.slot_base.
// phi_src: where the first step reads phi from (the program then runs out of
// place for its first pass; nullptr: phi itself).  The first step must then be
// a tile pass.
void run_program(qsv_ctx* c, const Program& P, qsv_dtype dt, int n, void* phi, void* lam, double* slots,
                 int slot_offset, const void* phi_src = nullptr, double* lamz_ev = nullptr) {
    const bool c128 = dt == QSV_C128;
    const size_t cb = c128 ? 16 : 8;
    if (phi_src && (P.steps.empty() || P.steps[0].type != Step::TILE))
        fail(QSV_ERR_UNSUPPORTED, "out-of-place program without a leading tile pass");
    for (const Step& st : P.steps) {
        if (st.type == Step::TILE) {
            const void* src = (phi_src && &st == &P.steps[0]) ? phi_src : phi;
            Timed t(c, lam ? KK_TILE2 : KK_TILE1, st.bytes);
            TileArgs ta = st.ta;
            if (c->opt_nontemporal) ta.flags |= TILE_NT;
            hipError_t e = c128 ? launch_tile<double>(c->stream, lam != nullptr, st.generic, src, phi, lam, ta,
                                                      (const TOp*)c->ops.p, c->coef.p, (const uint64_t*)c->words.p,
                                                      (double*)c->partials.p, st.grid, st.nthr, st.R, st.lds)
                                : launch_tile<float>(c->stream, lam != nullptr, st.generic, src, phi, lam, ta,
                                                     (const TOp*)c->ops.p, c->coef.p, (const uint64_t*)c->words.p,
                                                     (double*)c->partials.p, st.grid, st.nthr, st.R, st.lds);
            t.done(e);
            if (st.nslots) {
                Timed tr(c, KK_REDUCE, 8.0 * st.nslots * st.grid);
                tr.done(launch_reduce(c->stream, (const double*)c->partials.p, st.grid, st.nslots,
                                      slots + slot_offset + st.slot_base));
            }
            if ((st.ta.flags & TILE_LAMZ) && lamz_ev) {  // <H> from the pass that formed lambda
                Timed tr(c, KK_REDUCE, 8.0 * st.grid);
                tr.done(launch_reduce(c->stream, (const double*)c->partials.p + (size_t)st.nslots * st.grid,
                                      st.grid, 1, lamz_ev));
            }
            continue;
        }
        const int kind = st.type == Step::GATE1 ? KK_GATE1
                         : st.type == Step::DIAG1 ? KK_DIAG1
                         : st.type == Step::GATE2 ? KK_GATE2
                         : st.type == Step::DENSE ? KK_DENSE : KK_GATEK;  // GATEK and GATEK_LOW
        Timed t(c, kind, st.bytes);
        hipError_t e = hipSuccess;
        const bool nt = c->opt_nontemporal != 0;
        switch (st.type) {
        case Step::GATE1:
            e = c128 ? launch_gate1<double>(c->stream, phi, st.n_items, st.ex, st.setmask, st.tbit, st.cls, st.m2, nt)
                     : launch_gate1<float>(c->stream, phi, st.n_items, st.ex, st.setmask, st.tbit, st.cls, st.m2, nt);
            break;
        case Step::DIAG1:
            e = c128 ? launch_diag1<double>(c->stream, phi, st.n_items, st.ex, st.setmask, st.dre, st.dim, nt)
                     : launch_diag1<float>(c->stream, phi, st.n_items, st.ex, st.setmask, st.dre, st.dim, nt);
            break;
        case Step::GATE2:
            e = c128 ? launch_gate2<double>(c->stream, phi, st.n_items, st.ex, st.setmask, st.b0, st.b1, st.cls, st.m4,
                                            nt)
                     : launch_gate2<float>(c->stream, phi, st.n_items, st.ex, st.setmask, st.b0, st.b1, st.cls, st.m4,
                                           nt);
            break;
        case Step::GATEK_LOW:
            e = c128 ? launch_gatek_low<double>(c->stream, phi, st.n_items, st.ex, st.setmask, st.k, st.tb, st.lcm,
                                                st.lcv, (const char*)c->coef.p + st.coff * cb, nt)
                     : launch_gatek_low<float>(c->stream, phi, st.n_items, st.ex, st.setmask, st.k, st.tb, st.lcm,
                                               st.lcv, (const char*)c->coef.p + st.coff * cb, nt);
            break;
        case Step::GATEK:
            e = c128 ? launch_gatek<double>(c->stream, phi, st.n_items, st.ex, st.setmask, st.k, st.tb,
                                            (const char*)c->coef.p + st.coff * cb, nt)
                     : launch_gatek<float>(c->stream, phi, st.n_items, st.ex, st.setmask, st.k, st.tb,
                                           (const char*)c->coef.p + st.coff * cb, nt);
            break;
        case Step::DENSE:
            e = c128 ? launch_dense<double>(c->stream, phi, st.da, (const char*)c->coef.p + st.coff * cb, nt,
                                            c->opt_dense_mfma != 0)
                     : launch_dense<float>(c->stream, phi, st.da, (const char*)c->coef.p + st.coff * cb, nt, false);
            break;
        default:
            break;
        }
        t.done(e);
    }
}

// Host coefficient table in the state's precision.
std::vector<char> coef_bytes(const std::vector<cd>& coef, qsv_dtype dt) {
    std::vector<char> out;
    if (dt == QSV_C128) {
        out.resize(coef.size() * 16);
        std::memcpy(out.data(), coef.data(), out.size());
    } else {
        out.resize(coef.size() * 8);
        float* f = (float*)out.data();
        for (size_t i = 0; i < coef.size(); ++i) {
            f[2 * i] = (float)coef[i].real();
            f[2 * i + 1] = (float)coef[i].imag();
        }
    }
    return out;
}

// Pauli sums -> grouped device tables (one entry range per observable).
struct PauliTables {
    std::vector<PauliGroupDev> groups;
    std::vector<PauliTermDev> terms;
    std::vector<uint64_t> aux;                    // byte tables (complex FP64) and parity columns
    std::vector<std::pair<int, int>> obs_groups;  // (first group, count)
    std::vector<int> n_x_groups;                  // groups with x != 0
    std::vector<int> lut_tables;                  // byte tables per observable (LDS of its launch)
};

// allow_lut: groups of many terms (the largest two with 16..64 terms, at most
// 12 byte tables) are evaluated by table lookups in k_pauli.
void add_pauli(PauliTables& T, const qsv_pauli_sum& h, double scale, bool allow_lut = true) {
    std::map<uint64_t, std::vector<int64_t>> by_x;
    for (int64_t t = 0; t < h.n_terms; ++t) by_x[h.x_mask[t]].push_back(t);
    const int g0 = (int)T.groups.size();
    int nx = 0;
    for (auto& kv : by_x) {
        PauliGroupDev g;
        std::memset(&g, 0, sizeof g);
        g.x = kv.first;
        g.t0 = (int)T.terms.size();
        g.nt = (int)kv.second.size();
        g.lut = -1;
        if (g.x) ++nx;
        for (int64_t t : kv.second) {
            const uint64_t z = h.z_mask[t];
            const int ny = __builtin_popcountll(g.x & z) & 3;
            // i^ny
            const double c = h.coeff[t] * scale;
            PauliTermDev tm;
            tm.z = z;
            tm.wre = ny == 0 ? c : (ny == 2 ? -c : 0.0);
            tm.wim = ny == 1 ? c : (ny == 3 ? -c : 0.0);
            T.terms.push_back(tm);
        }
        T.groups.push_back(g);
    }
    int tables = 0;
    if (allow_lut) {
        std::vector<int> cand;
        for (int gi = g0; gi < (int)T.groups.size(); ++gi)
            if (T.groups[gi].nt >= PAULI_LUT_MIN_TERMS && T.groups[gi].nt <= 64) cand.push_back(gi);
        std::sort(cand.begin(), cand.end(), [&](int a, int b) { return T.groups[a].nt > T.groups[b].nt; });
        int slot = 0;
        for (int gi : cand) {
            PauliGroupDev& g = T.groups[gi];
            const int nb = (g.nt + 7) / 8;
            if (slot == 2 || tables + nb > PAULI_LUT_MAX_TABLES) continue;
            g.lut = slot++;
            g.nb = nb;
            if (T.aux.size() & 1) T.aux.push_back(0);  // 16-byte aligned complex entries
            g.lut_off = (int64_t)T.aux.size();
            for (int b = 0; b < nb; ++b)
                for (int v = 0; v < 256; ++v) {
                    double re = 0.0, im = 0.0;
                    for (int j = 0; j < 8 && 8 * b + j < g.nt; ++j) {
                        const PauliTermDev& tm = T.terms[g.t0 + 8 * b + j];
                        const double sgn = ((v >> j) & 1) ? -1.0 : 1.0;
                        re += sgn * tm.wre;
                        im += sgn * tm.wim;
                    }
                    uint64_t ur, ui;
                    std::memcpy(&ur, &re, 8);
                    std::memcpy(&ui, &im, 8);
                    T.aux.push_back(ur);
                    T.aux.push_back(ui);
                }
            g.col_off = (int64_t)T.aux.size();
            for (int k = 0; k < 64; ++k) {
                uint64_t col = 0;
                for (int t = 0; t < g.nt; ++t)
                    if ((T.terms[g.t0 + t].z >> k) & 1) col |= 1ull << t;
                T.aux.push_back(col);
            }
            tables += nb;
        }
    }
    T.obs_groups.push_back({g0, (int)T.groups.size() - g0});
    T.n_x_groups.push_back(nx);
    T.lut_tables.push_back(tables);
}

// expval (or lambda) of observable o into slots[out_slot]
// norm2: also ||H psi||^2 into slot[1] (variance), without writing lambda
void run_pauli(qsv_ctx* c, qsv_dtype dt, int n, const PauliTables& T, int o, const void* psi, void* lam, double* slot,
               bool norm2 = false) {
    const uint64_t N = 1ull << n;
    const int grid = pauli_grid(N);
    const double eb = (double)elem_bytes(dt);
    const double bytes = (1.0 + T.n_x_groups[o] + (lam ? 1.0 : 0.0)) * (double)N * eb;
    ensure(c, c->partials, (size_t)grid * 16);
    const PauliGroupDev* g = (const PauliGroupDev*)c->pgroups.p + T.obs_groups[o].first;
    const PauliTermDev* tm = (const PauliTermDev*)c->pterms.p;
    Timed t(c, lam ? KK_PAULI_LAMBDA : KK_PAULI, bytes);
    const uint64_t* aux = (const uint64_t*)c->paux.p;
    t.done(dt == QSV_C128 ? launch_pauli<double>(c->stream, lam != nullptr, norm2, psi, lam, N, g,
                                                 T.obs_groups[o].second, tm, aux, T.lut_tables[o],
                                                 (double*)c->partials.p, grid)
                          : launch_pauli<float>(c->stream, lam != nullptr, norm2, psi, lam, N, g,
                                                T.obs_groups[o].second, tm, aux, T.lut_tables[o],
                                                (double*)c->partials.p, grid));
    Timed tr(c, KK_REDUCE, 8.0 * grid);
    tr.done(launch_reduce(c->stream, (const double*)c->partials.p, grid, norm2 ? 2 : 1, slot));
}

void upload_program(qsv_ctx* c, const Program& P, qsv_dtype dt, const PauliTables* T) {
    std::vector<char> cf = coef_bytes(P.coef, dt);
    if (T)
        upload(c, {{&c->ops, P.tops.data(), P.tops.size() * sizeof(TOp)},
                   {&c->coef, cf.data(), cf.size()},
                   {&c->words, P.words.data(), P.words.size() * 8},
                   {&c->pgroups, T->groups.data(), T->groups.size() * sizeof(PauliGroupDev)},
                   {&c->pterms, T->terms.data(), T->terms.size() * sizeof(PauliTermDev)},
                   {&c->paux, T->aux.data(), T->aux.size() * 8}});
    else
        upload(c, {{&c->ops, P.tops.data(), P.tops.size() * sizeof(TOp)},
                   {&c->coef, cf.data(), cf.size()},
                   {&c->words, P.words.data(), P.words.size() * 8}});
    ensure(c, c->partials, std::max<size_t>(P.max_partials, 1) * 8);
}

std::vector<Factor> forward_factors(const qsv_op* ops, size_t n_ops, const double* params, const double* matrices,
                                    bool decompose) {
    std::vector<Factor> F;
    for (size_t i = 0; i < n_ops; ++i) {
        const size_t f0 = F.size();
        op_factors(ops[i], params, matrices, decompose, F);
        for (size_t j = f0; j < F.size(); ++j) F[j].src_op = (int)i;
    }
    return F;
}

// Reverse sweep items: for each factor from the last, its generator inner
// product (if it carries a trainable angle) and then its un-apply.
std::vector<Item> adjoint_items(const std::vector<Factor>& F, int n) {
    std::vector<Item> items;
    for (int i = (int)F.size() - 1; i >= 0; --i) {
        if (F[i].has_dot) items.push_back(make_item(F[i], true, i, n));
        items.push_back(make_item(F[i], false, i, n));
    }
    return items;
}

std::vector<Item> forward_items(const std::vector<Factor>& F, int n) {
    std::vector<Item> items;
    for (size_t i = 0; i < F.size(); ++i) items.push_back(make_item(F[i], false, (int)i, n));
    return items;
}

// The adjoint sweep for one combined observable set.  rows: n_rows Pauli
// sums; each gets its own lambda and sweep (or one combined lambda for the
// VJP).  out_rows[r * n_params + p] receives d<H_r>/dp, expv[r] = <H_r>.
void adjoint_impl(qsv_state* s, const qsv_op* ops, size_t n_ops, const double* params, size_t n_params,
                  const double* matrices, const std::vector<const qsv_pauli_sum*>& rows,
                  const std::vector<double>& row_scale_vjp, bool vjp, double* out, double* expv, uint32_t flags) {
    qsv_ctx* c = s->ctx;
    const int n = s->n;
    const uint64_t N = 1ull << n;
    const size_t eb = elem_bytes(s->dt);
    const size_t n_rows = vjp ? 1 : rows.size();
    if ((flags & QSV_ADJ_INPLACE) && n_rows > 1)
        fail(QSV_ERR_ARG, "QSV_ADJ_INPLACE needs a single observable (or the VJP form)");

    std::vector<Factor> F = forward_factors(ops, n_ops, params, matrices, true);
    std::vector<Item> items = adjoint_items(F, n);
    Program P = build_program(plan_opts(c, s->dt, true), F, items, n, s->dt, true, true);
    const size_t nslot = P.slot_param.size();

    // An observable that is c times a sum of Z strings (a diagonal H with one
    // coefficient, e.g. a MaxCut cost) needs no separate lambda = H psi pass:
    // the first reverse pass forms lambda = c (m - 2 |odd parities|) phi from
    // the tile it loads and sums <H> on the way (one full read and write of
    // the state fewer).
    bool lamz = false;
    // (the kernel form exists for the default two-vector tiles: 8 or 16
    // elements per thread, group-only passes)
    if (!vjp && n_rows == 1 && !P.steps.empty() && P.steps[0].type == Step::TILE &&
        !(P.steps[0].ta.flags & TILE_WS) && !P.steps[0].generic && (P.steps[0].R == 8 || P.steps[0].R == 16) &&
        P.steps[0].nthr == 256) {
        const qsv_pauli_sum* h = rows[0];
        lamz = h->n_terms > 0 && h->n_terms <= 64;
        for (int64_t t = 0; t < h->n_terms && lamz; ++t)
            lamz = h->x_mask[t] == 0 && h->coeff[t] == h->coeff[0];
        if (lamz) {
            Step& s0 = P.steps[0];
            TileArgs& a = s0.ta;
            std::vector<uint64_t> zm(h->z_mask, h->z_mask + h->n_terms);
            a.flags |= TILE_LAMZ;
            a.lamz_m = (int32_t)h->n_terms;
            a.lamz_c = h->coeff[0];
            a.lamz_woff = (int64_t)P.words.size();
            const int nthr = 1 << a.nthr_log2, R = 1 << (a.b - a.nthr_log2);
            uint64_t S = 0;
            for (int j = 0; j < a.b; ++j) S |= 1ull << a.sb[j];
            for (int t = 0; t < nthr; ++t) P.words.push_back(parity_bits_host(deposit((uint64_t)t, a.sb, a.nthr_log2), zm));
            for (int r = 0; r < R; ++r) P.words.push_back(parity_bits_host(a.offhi[r], zm));
            for (int g = 0; g < n; ++g)
                if (!((S >> g) & 1)) P.words.push_back(parity_bits_host(1ull << g, zm));
            s0.bytes -= (double)N * eb;  // lambda is not read
            P.max_partials = std::max(P.max_partials, (size_t)(s0.nslots + 1) * s0.grid);
            // one more slot accumulator (the <H> sums) in LDS
            s0.lds = (size_t)tile_lds_bytes(a.b, true, (int)eb, s0.nslots + 1, a.zt_n, a.n_zop, a.n_outer);
            if (s0.lds > (size_t)LDS_PER_CU) fail(QSV_ERR_UNSUPPORTED, "tile pass needs more LDS than a CU has");
        }
    }

    PauliTables T;
    if (vjp) {
        // lambda = sum_o cot_o H_o psi: one table with scaled coefficients
        std::vector<double> co;
        std::vector<uint64_t> xs, zs;
        for (size_t o = 0; o < rows.size(); ++o)
            for (int64_t t = 0; t < rows[o]->n_terms; ++t) {
                co.push_back(rows[o]->coeff[t] * row_scale_vjp[o]);
                xs.push_back(rows[o]->x_mask[t]);
                zs.push_back(rows[o]->z_mask[t]);
            }
        qsv_pauli_sum h{(int64_t)co.size(), co.data(), xs.data(), zs.data()};
        add_pauli(T, h, 1.0);
        for (auto* r : rows) add_pauli(T, *r, 1.0);  // for the expvals
    } else {
        for (auto* r : rows) add_pauli(T, *r, 1.0);
    }
    upload_program(c, P, s->dt, &T);

    // workspace: lambda, and phi unless the state itself is consumed
    const bool inplace = (flags & QSV_ADJ_INPLACE) != 0;
    ensure(c, c->ws0, N * eb);
    if (!inplace) ensure(c, c->ws1, N * eb);
    void* lam = c->ws0.p;
    void* phi = inplace ? s->ptr : c->ws1.p;
    const size_t n_ev = vjp ? rows.size() : n_rows;
    ensure(c, c->slots, (n_rows * nslot + n_ev + 1) * 8);
    double* slots = (double*)c->slots.p;
    double* evslots = slots + n_rows * nslot;

    if (vjp && expv)
        for (size_t o = 0; o < rows.size(); ++o) run_pauli(c, s->dt, n, T, (int)(o + 1), s->ptr, nullptr, evslots + o);
    for (size_t r = 0; r < n_rows; ++r) {
        if (!lamz)
            run_pauli(c, s->dt, n, T, (int)r, s->ptr, lam, vjp ? slots + n_rows * nslot + rows.size() : evslots + r);
        // out of place: the first pass reads the state and writes phi (no copy)
        const bool oop = !inplace && !P.steps.empty();
        if (!inplace && P.steps.empty()) {
            Timed t(c, KK_COPY, 2.0 * N * eb);
            t.done(hipMemcpyAsync(phi, s->ptr, N * eb, hipMemcpyDeviceToDevice, c->stream));
        }
        run_program(c, P, s->dt, n, phi, lam, slots, (int)(r * nslot), oop ? s->ptr : nullptr,
                    lamz ? evslots + r : nullptr);
    }
    std::vector<double> host(n_rows * nslot + n_ev + 1);
    HIPCHK(hipMemcpyAsync(host.data(), slots, host.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (size_t r = 0; r < n_rows; ++r) {
        double* row = out + r * n_params;
        std::fill(row, row + n_params, 0.0);
        for (size_t q = 0; q < nslot; ++q) row[P.slot_param[q].first] += P.slot_param[q].second * host[r * nslot + q];
    }
    if (expv) {
        for (size_t o = 0; o < n_ev; ++o) expv[o] = host[n_rows * nslot + o];
    }
}

}  // namespace

// ------------------------------------------------------------------ helpers used by kernels' callers

Expand qsv::make_expand(const std::vector<int>& pos) {
    Expand e;
    std::memset(&e, 0, sizeof e);
    const int m = (int)pos.size();
    if (m + 1 > 16) fail(QSV_ERR_UNSUPPORTED, "too many inserted bits");
    auto ones_below = [](int p) -> uint64_t { return p >= 64 ? ~0ull : ((1ull << p) - 1); };
    if (m == 0) {
        e.m[0] = ~0ull;
        e.nm = 1;
        return e;
    }
    e.m[0] = ones_below(pos[0]);
    for (int i = 1; i < m; ++i) e.m[i] = ones_below(pos[i]) & ~ones_below(pos[i - 1] + 1);
    e.m[m] = ~ones_below(pos[m - 1] + 1);
    e.nm = m + 1;
    return e;
}

// ------------------------------------------------------------------ C ABI

extern "C" {

const char* qsv_version(void) { return "qsv 0.1.0 (gfx950)"; }

const char* qsv_status_string(int st) {
    switch (st) {
    case QSV_OK: return "ok";
    case QSV_ERR_ARG: return "invalid argument";
    case QSV_ERR_WIRE: return "invalid wire";
    case QSV_ERR_DTYPE: return "dtype mismatch";
    case QSV_ERR_OOM: return "out of memory";
    case QSV_ERR_HIP: return "HIP runtime error";
    case QSV_ERR_UNSUPPORTED: return "unsupported";
    case QSV_ERR_PARAM: return "invalid parameter index";
    default: return "unknown status";
    }
}

const char* qsv_thread_last_error(void) { return g_thread_err.c_str(); }

int qsv_device_count(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

int qsv_kernel_kinds(void) { return KK_COUNT; }
const char* qsv_kernel_name(int kind) { return kind >= 0 && kind < KK_COUNT ? kKernelNames[kind] : ""; }

namespace {
// Device address of the allocation-free scratch, taken once per device (with
// that device current) at the first context created on it.
std::mutex g_scratch_mu;
void* g_scratch[64] = {nullptr};

void* scratch_for_device(int device) {
    if (device < 0 || device >= 64) fail(QSV_ERR_UNSUPPORTED, "device id beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        void* p = nullptr;
        hipError_t e = noalloc_scratch_address(&p);
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            fail(QSV_ERR_HIP, std::string("hipGetSymbolAddress of the scratch failed: ") + hipGetErrorString(e));
        }
        g_scratch[device] = p;
    }
    return g_scratch[device];
}
}  // namespace

qsv_status qsv_ctx_create(int device, void* hip_stream, qsv_ctx** out) {
    return guard(nullptr, [&] {
        if (!out) fail(QSV_ERR_ARG, "out is NULL");
        *out = nullptr;
        int nd = qsv_device_count();
        if (device < 0 || device >= nd) fail(QSV_ERR_ARG, "no HIP device " + std::to_string(device));
        std::unique_ptr<qsv_ctx> c(new qsv_ctx);
        c->device = device;
        set_device(c.get());
        if (hip_stream) {
            c->stream = (hipStream_t)hip_stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
        HIPCHK(hipEventCreateWithFlags(&c->pin_ev, hipEventDisableTiming));
        c->scratch = scratch_for_device(device);
        *out = c.release();
    });
}

void qsv_ctx_destroy(qsv_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (DevBuf* b : {&c->ops, &c->coef, &c->words, &c->partials, &c->slots, &c->pgroups, &c->pterms, &c->paux, &c->ws0, &c->ws1,
                      &c->binbits, &c->csr_ptr, &c->csr_col, &c->csr_val, &c->smp_chunk, &c->smp_resid, &c->smp_out})
        release(*b);
    if (c->pin) (void)hipHostFree(c->pin);
    for (auto& r : c->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->pin_ev) (void)hipEventDestroy(c->pin_ev);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char* qsv_last_error(const qsv_ctx* c) { return c ? c->err.c_str() : g_thread_err.c_str(); }

qsv_status qsv_ctx_set_stream(qsv_ctx* c, void* hip_stream) {
    return guard(c, [&] {
        if (!c) fail(QSV_ERR_ARG, "ctx is NULL");
        set_device(c);
        HIPCHK(hipStreamSynchronize(c->stream));
        if (c->own_stream) HIPCHK(hipStreamDestroy(c->stream));
        if (hip_stream) {
            c->stream = (hipStream_t)hip_stream;
            c->own_stream = false;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
    });
}

qsv_status qsv_ctx_synchronize(qsv_ctx* c) {
    return guard(c, [&] {
        if (!c) fail(QSV_ERR_ARG, "ctx is NULL");
        set_device(c);
        HIPCHK(hipStreamSynchronize(c->stream));
    });
}

qsv_status qsv_ctx_set_option(qsv_ctx* c, int option, int64_t v) {
    return guard(c, [&] {
        if (!c) fail(QSV_ERR_ARG, "ctx is NULL");
        switch (option) {
        case QSV_OPT_FUSION: c->opt_fusion = v != 0; break;
        case QSV_OPT_TILE_BITS:
            if (v < 0 || v > 8 + TILE_MAX_R_LOG2) fail(QSV_ERR_ARG, "tile bits out of range");
            c->opt_tile_bits = v;
            break;
        case QSV_OPT_TILE_BITS_ADJ:
            if (v < 0 || v > 8 + TILE_MAX_R_LOG2) fail(QSV_ERR_ARG, "tile bits out of range");
            c->opt_tile_bits_adj = v;
            break;
        case QSV_OPT_LOW_BITS:
            if (v < 0 || v > 8) fail(QSV_ERR_ARG, "low bits out of range");
            c->opt_low_bits = v;
            break;
        case QSV_OPT_PROFILE: c->opt_profile = v != 0; break;
        case QSV_OPT_NONTEMPORAL: c->opt_nontemporal = v != 0; break;
        case QSV_OPT_LAYERS: c->opt_layers = v != 0; break;
        case QSV_OPT_TILE_WS: c->opt_tile_ws = v != 0; break;
        case QSV_OPT_DENSE_MFMA: c->opt_dense_mfma = v != 0; break;
        case QSV_OPT_TEST_ALLOC_LIMIT:
            if (v < 0) fail(QSV_ERR_ARG, "allocation limit must be >= 0");
            c->test_alloc_limit = v;
            break;
        case QSV_OPT_TEST_FAIL_LAUNCH:
            if (v < 0) fail(QSV_ERR_ARG, "launch count must be >= 0");
            c->test_fail_launch = v;
            break;
        default: fail(QSV_ERR_ARG, "unknown option");
        }
    });
}

qsv_status qsv_ctx_get_option(qsv_ctx* c, int option, int64_t* v) {
    return guard(c, [&] {
        if (!c || !v) fail(QSV_ERR_ARG, "NULL argument");
        switch (option) {
        case QSV_OPT_FUSION: *v = c->opt_fusion; break;
        case QSV_OPT_TILE_BITS: *v = c->opt_tile_bits; break;
        case QSV_OPT_TILE_BITS_ADJ: *v = c->opt_tile_bits_adj; break;
        case QSV_OPT_LOW_BITS: *v = c->opt_low_bits; break;
        case QSV_OPT_PROFILE: *v = c->opt_profile; break;
        case QSV_OPT_NONTEMPORAL: *v = c->opt_nontemporal; break;
        case QSV_OPT_LAYERS: *v = c->opt_layers; break;
        case QSV_OPT_TILE_WS: *v = c->opt_tile_ws; break;
        case QSV_OPT_DENSE_MFMA: *v = c->opt_dense_mfma; break;
        case QSV_OPT_TEST_ALLOC_LIMIT: *v = c->test_alloc_limit; break;
        case QSV_OPT_TEST_FAIL_LAUNCH: *v = c->test_fail_launch; break;
        default: fail(QSV_ERR_ARG, "unknown option");
        }
    });
}

qsv_status qsv_ctx_workspace_bytes(qsv_ctx* c, size_t* out) {
    return guard(c, [&] {
        if (!c || !out) fail(QSV_ERR_ARG, "NULL argument");
        size_t t = 0;
        for (DevBuf* b : {&c->ops, &c->coef, &c->words, &c->partials, &c->slots, &c->pgroups, &c->pterms, &c->paux, &c->ws0, &c->ws1,
                          &c->binbits, &c->csr_ptr, &c->csr_col, &c->csr_val, &c->smp_chunk, &c->smp_resid, &c->smp_out})
            t += b->bytes;
        *out = t;
    });
}

qsv_status qsv_ctx_release_workspace(qsv_ctx* c) {
    return guard(c, [&] {
        if (!c) fail(QSV_ERR_ARG, "ctx is NULL");
        set_device(c);
        HIPCHK(hipStreamSynchronize(c->stream));
        release(c->ws0);
        release(c->ws1);
        release(c->partials);
    });
}

qsv_status qsv_ctx_kernel_stats(qsv_ctx* c, int kind, int64_t* launches, double* ms, double* bytes) {
    return guard(c, [&] {
        if (!c) fail(QSV_ERR_ARG, "ctx is NULL");
        if (kind < 0 || kind >= KK_COUNT) fail(QSV_ERR_ARG, "bad kernel kind");
        set_device(c);
        flush_stats(c);
        if (launches) *launches = c->st_launch[kind];
        if (ms) *ms = c->st_ms[kind];
        if (bytes) *bytes = c->st_bytes[kind];
    });
}

qsv_status qsv_ctx_reset_stats(qsv_ctx* c) {
    return guard(c, [&] {
        if (!c) fail(QSV_ERR_ARG, "ctx is NULL");
        set_device(c);
        flush_stats(c);
        for (int k = 0; k < KK_COUNT; ++k) {
            c->st_launch[k] = 0;
            c->st_ms[k] = 0;
            c->st_bytes[k] = 0;
        }
    });
}

qsv_status qsv_state_create(qsv_ctx* c, int n, qsv_dtype dt, qsv_state** out) {
    return guard(c, [&] {
        if (!c || !out) fail(QSV_ERR_ARG, "NULL argument");
        *out = nullptr;
        if (n < 1 || n > QSV_MAX_QUBITS) fail(QSV_ERR_ARG, "n_qubits out of range");
        if (dt != QSV_C64 && dt != QSV_C128) fail(QSV_ERR_DTYPE, "unknown dtype");
        set_device(c);
        const size_t bytes = ((size_t)1 << n) * elem_bytes(dt);
        void* p = nullptr;
        if (dev_malloc(c, &p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            fail(QSV_ERR_OOM, "state allocation of " + std::to_string(bytes) + " bytes failed");
        }
        std::unique_ptr<qsv_state> s(new qsv_state{c, n, dt, p, true});
        Timed t(c, KK_INIT, (double)bytes);
        t.done(dt == QSV_C128 ? launch_init<double>(c->stream, p, 1ull << n, 0)
                              : launch_init<float>(c->stream, p, 1ull << n, 0));
        *out = s.release();
    });
}

qsv_status qsv_state_wrap(qsv_ctx* c, int n, qsv_dtype dt, void* dev_ptr, qsv_state** out) {
    return guard(c, [&] {
        if (!c || !out || !dev_ptr) fail(QSV_ERR_ARG, "NULL argument");
        *out = nullptr;
        if (n < 1 || n > QSV_MAX_QUBITS) fail(QSV_ERR_ARG, "n_qubits out of range");
        if (dt != QSV_C64 && dt != QSV_C128) fail(QSV_ERR_DTYPE, "unknown dtype");
        if ((uintptr_t)dev_ptr % elem_bytes(dt)) fail(QSV_ERR_ARG, "device pointer misaligned");
        *out = new qsv_state{c, n, dt, dev_ptr, false};
    });
}

void qsv_state_destroy(qsv_state* s) {
    if (!s) return;
    if (s->owned && s->ptr) {
        (void)hipSetDevice(s->ctx->device);
        (void)hipStreamSynchronize(s->ctx->stream);
        (void)hipFree(s->ptr);
    }
    delete s;
}

int qsv_state_n_qubits(const qsv_state* s) { return s ? s->n : 0; }
void* qsv_state_device_ptr(const qsv_state* s) { return s ? s->ptr : nullptr; }

qsv_status qsv_state_reset(qsv_state* s, uint64_t basis) {
    qsv_ctx* c = s ? s->ctx : nullptr;
    return guard(c, [&] {
        state_ctx(s);
        if (basis >> s->n) fail(QSV_ERR_ARG, "basis index out of range");
        set_device(c);
        const uint64_t N = 1ull << s->n;
        Timed t(c, KK_INIT, (double)(N * elem_bytes(s->dt)));
        t.done(s->dt == QSV_C128 ? launch_init<double>(c->stream, s->ptr, N, basis)
                                 : launch_init<float>(c->stream, s->ptr, N, basis));
    });
}

qsv_status qsv_state_copy(qsv_state* dst, const qsv_state* src) {
    qsv_ctx* c = dst ? dst->ctx : nullptr;
    return guard(c, [&] {
        if (!dst || !src) fail(QSV_ERR_ARG, "NULL state");
        if (dst->n != src->n) fail(QSV_ERR_ARG, "qubit counts differ");
        if (dst->dt != src->dt) fail(QSV_ERR_DTYPE, "dtypes differ");
        set_device(c);
        const size_t bytes = ((size_t)1 << dst->n) * elem_bytes(dst->dt);
        Timed t(c, KK_COPY, 2.0 * bytes);
        t.done(hipMemcpyAsync(dst->ptr, src->ptr, bytes, hipMemcpyDeviceToDevice, c->stream));
    });
}

qsv_status qsv_state_to_host(const qsv_state* s, void* host) {
    qsv_ctx* c = s ? s->ctx : nullptr;
    return guard(c, [&] {
        if (!s || !host) fail(QSV_ERR_ARG, "NULL argument");
        set_device(c);
        const size_t bytes = ((size_t)1 << s->n) * elem_bytes(s->dt);
        HIPCHK(hipStreamSynchronize(c->stream));
        HIPCHK(hipMemcpy(host, s->ptr, bytes, hipMemcpyDeviceToHost));
    });
}

qsv_status qsv_state_from_host(qsv_state* s, const void* host) {
    qsv_ctx* c = s ? s->ctx : nullptr;
    return guard(c, [&] {
        if (!s || !host) fail(QSV_ERR_ARG, "NULL argument");
        set_device(c);
        const size_t bytes = ((size_t)1 << s->n) * elem_bytes(s->dt);
        HIPCHK(hipStreamSynchronize(c->stream));
        HIPCHK(hipMemcpy(s->ptr, host, bytes, hipMemcpyHostToDevice));
    });
}

qsv_status qsv_validate_ops(int n, const qsv_op* ops, size_t n_ops, size_t n_params, size_t n_mat) {
    return guard(nullptr, [&] {
        // parameters/matrices presence is checked by the hot-path calls
        static const double dummy = 0.0;
        validate_ops_impl(n, ops, n_ops, n_params, n_mat, &dummy, &dummy);
    });
}

qsv_status qsv_validate_obs(int n, const qsv_pauli_sum* obs, size_t n_obs) {
    return guard(nullptr, [&] {
        if (n < 1 || n > QSV_MAX_QUBITS) fail(QSV_ERR_ARG, "n_qubits out of range");
        validate_obs_impl(n, obs, n_obs);
    });
}

qsv_status qsv_plan_json(int n, qsv_dtype dt, const qsv_op* ops, size_t n_ops, const double* params,
                         size_t n_params, const double* matrices, size_t n_mat, int adjoint, int tile_bits,
                         int low_bits, int fusion, char* out, size_t cap, size_t* needed) {
    return guard(nullptr, [&] {
        validate_ops_impl(n, ops, n_ops, n_params, n_mat, params, matrices);
        if (dt != QSV_C64 && dt != QSV_C128) fail(QSV_ERR_DTYPE, "unknown dtype");
        if (tile_bits < 0 || tile_bits > 8 + TILE_MAX_R_LOG2 || low_bits < 0 || low_bits > 8)
            fail(QSV_ERR_ARG, "tile options out of range");
        const bool two = adjoint != 0;
        std::vector<Factor> F = forward_factors(ops, n_ops, params, matrices, two);
        std::vector<Item> items = two ? adjoint_items(F, n) : forward_items(F, n);
        Program P = build_program(plan_opts(tile_bits, low_bits, fusion != 0, dt, two, fusion != 2), F, items, n, dt,
                                  two, two);
        std::string js;
        char buf[512];
        auto add = [&](const char* fmt, auto... a) {
            std::snprintf(buf, sizeof buf, fmt, a...);
            js += buf;
        };
        js += "{\"steps\":[";
        for (size_t i = 0; i < P.steps.size(); ++i) {
            const Step& st = P.steps[i];
            if (i) js += ",";
            static const char* names[] = {"tile", "gate1", "diag1", "gate2", "gatek", "gatek_low", "dense"};
            add("{\"type\":\"%s\",\"bytes\":%.17g", names[st.type], st.bytes);
            if (st.type == Step::DENSE) {
                const DenseArgs& d = st.da;
                add(",\"k\":%d,\"nthr\":%d,\"coff\":%lld,\"n_tiles\":%llu,\"setmask\":%llu,\"sb\":[", d.k,
                    dense_threads(d.k), (long long)st.coff, (unsigned long long)d.n_tiles,
                    (unsigned long long)d.setmask);
                for (int j = 0; j < d.k + 6; ++j) add(j ? ",%d" : "%d", d.sb[j]);
                js += "],\"cb\":[";
                for (int j = 0; j < d.k + 6; ++j) add(j ? ",%d" : "%d", d.cb[j]);
                js += "],\"goff_hi\":[";
                const int rl = (64 << d.k) / dense_threads(d.k);
                for (int r = 0; r < rl; ++r) add(r ? ",%llu" : "%llu", (unsigned long long)d.goff_hi[r]);
                js += "],\"coff_hi\":[";
                for (int r = 0; r < rl; ++r) add(r ? ",%u" : "%u", d.coff_hi[r]);
                js += "],\"outer\":[";
                for (int j = 0; j < d.outer.nm; ++j) add(j ? ",%llu" : "%llu", (unsigned long long)d.outer.m[j]);
                js += "]";
            } else if (st.type == Step::TILE) {
                const TileArgs& a = st.ta;
                add(",\"b\":%d,\"nthr\":%d,\"R\":%d,\"grid\":%d,\"op0\":%d,\"nops\":%d,\"nslots\":%d,\"slot_base\":%d,"
                    "\"generic\":%d,\"n_tiles\":%llu,\"n_outer\":%d,\"lds\":%zu,\"flags\":%d,"
                    "\"out_scale\":%.17g,\"zt_off\":%lld,\"zt_n\":%d,\"sb\":[",
                    a.b, st.nthr, st.R, st.grid, a.op0, a.nops, a.nslots, st.slot_base, (int)st.generic,
                    (unsigned long long)a.n_tiles, a.n_outer, st.lds, a.flags, a.out_scale, (long long)a.zt_off,
                    a.zt_n);
                for (int j = 0; j < a.b; ++j) add(j ? ",%d" : "%d", a.sb[j]);
                js += "],\"offhi\":[";
                for (int r = 0; r < st.R; ++r) add(r ? ",%llu" : "%llu", (unsigned long long)a.offhi[r]);
                js += "],\"outer\":[";
                for (int j = 0; j < a.outer.nm; ++j) add(j ? ",%llu" : "%llu", (unsigned long long)a.outer.m[j]);
                js += "]";
            } else {
                add(",\"n_items\":%llu,\"setmask\":%llu,\"tbit\":%llu,\"b0\":%llu,\"b1\":%llu,\"cls\":%d,\"k\":%d,"
                    "\"coff\":%lld,\"dre\":%.17g,\"dim\":%.17g,\"tb\":[%d,%d,%d,%d,%d,%d],\"ex\":[",
                    (unsigned long long)st.n_items, (unsigned long long)st.setmask, (unsigned long long)st.tbit,
                    (unsigned long long)st.b0, (unsigned long long)st.b1, st.cls, st.k, (long long)st.coff, st.dre,
                    st.dim, st.tb[0], st.tb[1], st.tb[2], st.tb[3], st.tb[4], st.tb[5]);
                for (int j = 0; j < st.ex.nm; ++j) add(j ? ",%llu" : "%llu", (unsigned long long)st.ex.m[j]);
                js += "],\"m2\":[";
                for (int j = 0; j < 4; ++j) add(j ? ",%.17g,%.17g" : "%.17g,%.17g", st.m2.re[j], st.m2.im[j]);
                js += "],\"m4\":[";
                for (int j = 0; j < 16; ++j) add(j ? ",%.17g,%.17g" : "%.17g,%.17g", st.m4.re[j], st.m4.im[j]);
                add("],\"lcm\":%u,\"lcv\":%u", st.lcm, st.lcv);
            }
            js += "}";
        }
        js += "],\"tops\":[";
        for (size_t i = 0; i < P.tops.size(); ++i) {
            const TOp& o = P.tops[i];
            add("%s{\"kind\":%d,\"cls\":%d,\"k\":%d,\"slot\":%d,\"tb\":[%d,%d,%d,%d,%d,%d],\"lcmask\":%u,\"lcval\":%u,"
                "\"gcmask\":%llu,\"gcval\":%llu,\"coff\":%lld,\"woff\":%lld,\"m\":%d,\"aux\":%d}",
                i ? "," : "", o.kind, o.cls, o.k, o.slot, o.tb[0], o.tb[1], o.tb[2], o.tb[3], o.tb[4], o.tb[5],
                o.lcmask, o.lcval, (unsigned long long)o.gcmask, (unsigned long long)o.gcval, (long long)o.coff,
                (long long)o.woff, o.m, o.aux);
        }
        js += "],\"coef\":[";
        for (size_t i = 0; i < P.coef.size(); ++i)
            add(i ? ",%.17g,%.17g" : "%.17g,%.17g", P.coef[i].real(), P.coef[i].imag());
        js += "],\"words\":[";
        for (size_t i = 0; i < P.words.size(); ++i) add(i ? ",%llu" : "%llu", (unsigned long long)P.words[i]);
        js += "],\"slot_param\":[";
        for (size_t i = 0; i < P.slot_param.size(); ++i)
            add(i ? ",[%d,%.17g]" : "[%d,%.17g]", P.slot_param[i].first, P.slot_param[i].second);
        js += "]}";
        if (needed) *needed = js.size() + 1;
        if (out && cap) {
            const size_t k = std::min(cap - 1, js.size());
            std::memcpy(out, js.data(), k);
            out[k] = 0;
        }
    });
}

qsv_status qsv_plan_stats(int n, qsv_dtype dt, const qsv_op* ops, size_t n_ops, const double* params,
                          size_t n_params, const double* matrices, size_t n_mat, int adjoint, int tile_bits,
                          int low_bits, int fusion, int64_t* n_passes, int64_t* n_tile_passes,
                          int64_t* n_kernel_ops, double* alg_bytes) {
    return guard(nullptr, [&] {
        validate_ops_impl(n, ops, n_ops, n_params, n_mat, params, matrices);
        if (dt != QSV_C64 && dt != QSV_C128) fail(QSV_ERR_DTYPE, "unknown dtype");
        if (tile_bits < 0 || tile_bits > 8 + TILE_MAX_R_LOG2 || low_bits < 0 || low_bits > 8)
            fail(QSV_ERR_ARG, "tile options out of range");
        const bool two = adjoint != 0;
        std::vector<Factor> F = forward_factors(ops, n_ops, params, matrices, two);
        std::vector<Item> items = two ? adjoint_items(F, n) : forward_items(F, n);
        Program P = build_program(plan_opts(tile_bits, low_bits, fusion != 0, dt, two, fusion != 2), F, items, n, dt,
                                  two, two);
        int64_t tiles = 0;
        double bytes = 0;
        for (const Step& st : P.steps) {
            tiles += st.type == Step::TILE;
            bytes += st.bytes;
        }
        if (n_passes) *n_passes = (int64_t)P.steps.size();
        if (n_tile_passes) *n_tile_passes = tiles;
        if (n_kernel_ops) *n_kernel_ops = (int64_t)P.tops.size();
        if (alg_bytes) *alg_bytes = bytes;
    });
}

qsv_status qsv_apply(qsv_state* s, const qsv_op* ops, size_t n_ops, const double* params, size_t n_params,
                     const double* matrices, size_t n_mat) {
    qsv_ctx* c = s ? s->ctx : nullptr;
    return guard(c, [&] {
        state_ctx(s);
        validate_ops_impl(s->n, ops, n_ops, n_params, n_mat, params, matrices);
        if (!n_ops) return;
        set_device(c);
        std::vector<Factor> F = forward_factors(ops, n_ops, params, matrices, false);
        std::vector<Item> items = forward_items(F, s->n);
        Program P = build_program(plan_opts(c, s->dt, false), F, items, s->n, s->dt, false, false);
        upload_program(c, P, s->dt, nullptr);
        run_program(c, P, s->dt, s->n, s->ptr, nullptr, nullptr, 0);
    });
}

qsv_status qsv_expval(qsv_state* s, const qsv_pauli_sum* obs, size_t n_obs, double* out) {
    qsv_ctx* c = s ? s->ctx : nullptr;
    return guard(c, [&] {
        state_ctx(s);
        validate_obs_impl(s->n, obs, n_obs);
        if (n_obs && !out) fail(QSV_ERR_ARG, "out is NULL");
        if (!n_obs) return;
        set_device(c);
        PauliTables T;
        for (size_t o = 0; o < n_obs; ++o) add_pauli(T, obs[o], 1.0);
        upload(c, {{&c->pgroups, T.groups.data(), T.groups.size() * sizeof(PauliGroupDev)},
                   {&c->pterms, T.terms.data(), T.terms.size() * sizeof(PauliTermDev)},
                   {&c->paux, T.aux.data(), T.aux.size() * 8}});
        ensure(c, c->slots, n_obs * 8);
        for (size_t o = 0; o < n_obs; ++o) run_pauli(c, s->dt, s->n, T, (int)o, s->ptr, nullptr, (double*)c->slots.p + o);
        HIPCHK(hipMemcpyAsync(out, c->slots.p, n_obs * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    });
}


qsv_status qsv_expval_noalloc(qsv_state* s, const qsv_pauli_sum* obs, size_t n_obs, double* out) {
    qsv_ctx* c = s ? s->ctx : nullptr;
    return guard(c, [&] {
        state_ctx(s);
        validate_obs_impl(s->n, obs, n_obs);
        if (n_obs && !out) fail(QSV_ERR_ARG, "out is NULL");
        if (!n_obs) return;
        set_device(c);
        char* base = (char*)c->scratch;
        if (!base) fail(QSV_ERR_HIP, "no scratch address for this context's device");
        PauliTables T;
        for (size_t o = 0; o < n_obs; ++o) add_pauli(T, obs[o], 1.0);
        const uint64_t N = 1ull << s->n;
        const int grid = pauli_grid(N);
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        const size_t gb = T.groups.size() * sizeof(PauliGroupDev), tb = T.terms.size() * sizeof(PauliTermDev),
                     ab = T.aux.size() * 8;
        const size_t off_g = 0, off_t = al(off_g + gb), off_a = al(off_t + tb), off_p = al(off_a + ab),
                     off_s = al(off_p + (size_t)grid * 8), total = off_s + n_obs * 8;
        if (total > NOALLOC_SCRATCH_BYTES)
            fail(QSV_ERR_ARG, "observables need " + std::to_string(total) + " bytes of scratch; the allocation-free "
                              "entry point has " + std::to_string(NOALLOC_SCRATCH_BYTES));
        if (gb) HIPCHK(hipMemcpyAsync(base + off_g, T.groups.data(), gb, hipMemcpyHostToDevice, c->stream));
        if (tb) HIPCHK(hipMemcpyAsync(base + off_t, T.terms.data(), tb, hipMemcpyHostToDevice, c->stream));
        if (ab) HIPCHK(hipMemcpyAsync(base + off_a, T.aux.data(), ab, hipMemcpyHostToDevice, c->stream));
        const PauliGroupDev* groups = (const PauliGroupDev*)(base + off_g);
        const PauliTermDev* terms = (const PauliTermDev*)(base + off_t);
        const uint64_t* aux = (const uint64_t*)(base + off_a);
        double* partials = (double*)(base + off_p);
        double* slots = (double*)(base + off_s);
        for (size_t o = 0; o < n_obs; ++o) {
            // every block writes its partial and the reduction writes the
            // slot, so nothing in the scratch needs clearing between calls
            const PauliGroupDev* g = groups + T.obs_groups[o].first;
            HIPCHK(s->dt == QSV_C128
                       ? launch_pauli<double>(c->stream, false, false, s->ptr, nullptr, N, g, T.obs_groups[o].second,
                                              terms, aux, T.lut_tables[o], partials, grid)
                       : launch_pauli<float>(c->stream, false, false, s->ptr, nullptr, N, g, T.obs_groups[o].second,
                                             terms, aux, T.lut_tables[o], partials, grid));
            HIPCHK(launch_reduce(c->stream, partials, grid, 1, slots + o));
        }
        HIPCHK(hipMemcpyAsync(out, slots, n_obs * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    });
}

qsv_status qsv_var(qsv_state* s, const qsv_pauli_sum* obs, size_t n_obs, double* out) {
    qsv_ctx* c = s ? s->ctx : nullptr;
    return guard(c, [&] {
        state_ctx(s);
        validate_obs_impl(s->n, obs, n_obs);
        if (n_obs && !out) fail(QSV_ERR_ARG, "out is NULL");
        if (!n_obs) return;
        set_device(c);
        PauliTables T;
        for (size_t o = 0; o < n_obs; ++o) add_pauli(T, obs[o], 1.0);
        upload(c, {{&c->pgroups, T.groups.data(), T.groups.size() * sizeof(PauliGroupDev)},
                   {&c->pterms, T.terms.data(), T.terms.size() * sizeof(PauliTermDev)},
                   {&c->paux, T.aux.data(), T.aux.size() * 8}});
        ensure(c, c->slots, n_obs * 16);
        for (size_t o = 0; o < n_obs; ++o)
            run_pauli(c, s->dt, s->n, T, (int)o, s->ptr, nullptr, (double*)c->slots.p + 2 * o, true);
        std::vector<double> h(2 * n_obs);
        HIPCHK(hipMemcpyAsync(h.data(), c->slots.p, h.size() * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (size_t o = 0; o < n_obs; ++o) out[o] = h[2 * o + 1] - h[2 * o] * h[2 * o];
    });
}

qsv_status qsv_expval_sparse(qsv_state* s, const int64_t* row_ptr, const int64_t* col, const double* values,
                             int64_t nnz, double* out) {
    qsv_ctx* c = s ? s->ctx : nullptr;
    return guard(c, [&] {
        state_ctx(s);
        if (!row_ptr || !out || (nnz && (!col || !values))) fail(QSV_ERR_ARG, "NULL argument");
        const uint64_t N = 1ull << s->n;
        if (row_ptr[0] != 0 || row_ptr[N] != nnz || nnz < 0) fail(QSV_ERR_ARG, "row_ptr must run from 0 to nnz");
        for (uint64_t i = 0; i < N; ++i)
            if (row_ptr[i + 1] < row_ptr[i]) fail(QSV_ERR_ARG, "row_ptr not monotone");
        for (int64_t k = 0; k < nnz; ++k)
            if (col[k] < 0 || (uint64_t)col[k] >= N) fail(QSV_ERR_ARG, "column index out of range");
        set_device(c);
        upload(c, {{&c->csr_ptr, row_ptr, (N + 1) * 8}, {&c->csr_col, col, (size_t)nnz * 8},
                   {&c->csr_val, values, (size_t)nnz * 16}});
        const int grid = pauli_grid(N);
        ensure(c, c->partials, (size_t)grid * 16);
        ensure(c, c->slots, 16);
        {
            Timed t(c, KK_SPARSE, (double)(N * elem_bytes(s->dt)) + 24.0 * nnz + 8.0 * (N + 1));
            t.done(s->dt == QSV_C128
                       ? launch_sparse<double>(c->stream, s->ptr, N, (const int64_t*)c->csr_ptr.p,
                                               (const int64_t*)c->csr_col.p, (const double*)c->csr_val.p,
                                               (double*)c->partials.p, grid)
                       : launch_sparse<float>(c->stream, s->ptr, N, (const int64_t*)c->csr_ptr.p,
                                              (const int64_t*)c->csr_col.p, (const double*)c->csr_val.p,
                                              (double*)c->partials.p, grid));
        }
        Timed tr(c, KK_REDUCE, 16.0 * grid);
        tr.done(launch_reduce(c->stream, (const double*)c->partials.p, grid, 2, (double*)c->slots.p));
        HIPCHK(hipMemcpyAsync(out, c->slots.p, 16, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    });
}

qsv_status qsv_probs(qsv_state* s, const int32_t* wires, int n_wires, double* out) {
    qsv_ctx* c = s ? s->ctx : nullptr;
    return guard(c, [&] {
        state_ctx(s);
        const int n = s->n;
        if (!wires || !out) fail(QSV_ERR_ARG, "NULL argument");
        if (n_wires < 1 || n_wires > std::min(n, 20)) fail(QSV_ERR_ARG, "n_wires must be in [1, min(n, 20)]");
        std::vector<int> pos;
        for (int j = 0; j < n_wires; ++j) {
            if (wires[j] < 0 || wires[j] >= n) fail(QSV_ERR_WIRE, "wire out of range");
            for (int i = 0; i < j; ++i)
                if (wires[i] == wires[j]) fail(QSV_ERR_WIRE, "repeated wire");
            pos.push_back(n - 1 - wires[j]);
        }
        set_device(c);
        const int nb = 1 << n_wires;
        std::vector<uint64_t> bb(nb);
        for (int b = 0; b < nb; ++b) {
            uint64_t x = 0;
            for (int j = 0; j < n_wires; ++j)  // first listed wire = most significant bit of the bin
                if ((b >> (n_wires - 1 - j)) & 1) x |= 1ull << pos[j];
            bb[b] = x;
        }
        std::vector<int> sorted = pos;
        std::sort(sorted.begin(), sorted.end());
        const Expand ex = make_expand(sorted);
        const uint64_t n_rest = 1ull << (n - n_wires);
        const int gx = (int)std::max<uint64_t>(1, std::min<uint64_t>((n_rest + 1023) / 1024,
                                                                    std::max(1, 4096 / nb)));
        upload(c, {{&c->binbits, bb.data(), bb.size() * 8}});
        ensure(c, c->partials, (size_t)nb * gx * 8);
        ensure(c, c->slots, (size_t)nb * 8);
        {
            Timed t(c, KK_PROBS, (double)((1ull << n) * elem_bytes(s->dt)));
            t.done(s->dt == QSV_C128 ? launch_probs<double>(c->stream, s->ptr, n_rest, ex, (const uint64_t*)c->binbits.p,
                                                            nb, gx, (double*)c->partials.p)
                                     : launch_probs<float>(c->stream, s->ptr, n_rest, ex, (const uint64_t*)c->binbits.p,
                                                           nb, gx, (double*)c->partials.p));
        }
        Timed tr(c, KK_REDUCE, 8.0 * nb * gx);
        tr.done(launch_reduce(c->stream, (const double*)c->partials.p, gx, nb, (double*)c->slots.p));
        HIPCHK(hipMemcpyAsync(out, c->slots.p, (size_t)nb * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    });
}

qsv_status qsv_sample(qsv_state* s, const double* u, size_t n_samples, uint64_t* out) {
    qsv_ctx* c = s ? s->ctx : nullptr;
    return guard(c, [&] {
        state_ctx(s);
        if (n_samples == 0) return;
        if (!u || !out) fail(QSV_ERR_ARG, "NULL argument");
        for (size_t k = 0; k < n_samples; ++k)
            if (!(u[k] >= 0.0 && u[k] < 1.0)) fail(QSV_ERR_ARG, "uniforms must lie in [0, 1)");
        const int n = s->n;
        // chunks of >= 64 amplitudes, at most 2^16 of them
        const int clog2 = n <= 6 ? n : std::max(6, n - 16);
        const uint64_t n_chunks = 1ull << (n - clog2);
        set_device(c);
        ensure(c, c->partials, n_chunks * 8);
        const bool c128 = s->dt == QSV_C128;
        {
            Timed t(c, KK_SAMPLE, (double)((1ull << n) * elem_bytes(s->dt)));
            t.done(c128 ? launch_chunk_norms<double>(c->stream, s->ptr, clog2, n_chunks, (double*)c->partials.p)
                        : launch_chunk_norms<float>(c->stream, s->ptr, clog2, n_chunks, (double*)c->partials.p));
        }
        std::vector<double> cs(n_chunks);
        HIPCHK(hipMemcpyAsync(cs.data(), c->partials.p, n_chunks * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        // inclusive running sums over chunks in index order
        std::vector<double> incl(n_chunks);
        double run = 0.0;
        size_t last_nz = 0;
        for (uint64_t i = 0; i < n_chunks; ++i) {
            run += cs[i];
            incl[i] = run;
            if (cs[i] > 0.0) last_nz = i;
        }
        if (!(run > 0.0)) fail(QSV_ERR_ARG, "the state has zero norm");
        std::vector<int64_t> ch(n_samples);
        std::vector<double> rs(n_samples);
        for (size_t k = 0; k < n_samples; ++k) {
            const double t = u[k] * run;
            size_t j = (size_t)(std::upper_bound(incl.begin(), incl.end(), t) - incl.begin());
            if (j >= n_chunks) j = last_nz;  // t rounded up to the total
            ch[k] = (int64_t)j;
            rs[k] = t - (j ? incl[j - 1] : 0.0);
        }
        upload(c, {{&c->smp_chunk, ch.data(), n_samples * 8}, {&c->smp_resid, rs.data(), n_samples * 8}});
        ensure(c, c->smp_out, n_samples * 8);
        {
            Timed t(c, KK_SAMPLE, (double)n_samples * 64.0 * (double)((1ull << clog2) / 64 + 1) *
                                      (double)elem_bytes(s->dt));
            t.done(c128 ? launch_sample<double>(c->stream, s->ptr, clog2, (const int64_t*)c->smp_chunk.p,
                                                (const double*)c->smp_resid.p, (uint64_t*)c->smp_out.p,
                                                (int64_t)n_samples)
                        : launch_sample<float>(c->stream, s->ptr, clog2, (const int64_t*)c->smp_chunk.p,
                                               (const double*)c->smp_resid.p, (uint64_t*)c->smp_out.p,
                                               (int64_t)n_samples));
        }
        HIPCHK(hipMemcpyAsync(out, c->smp_out.p, n_samples * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    });
}

qsv_status qsv_adjoint_jacobian(qsv_state* s, const qsv_op* ops, size_t n_ops, const double* params, size_t n_params,
                                const double* matrices, size_t n_mat, const qsv_pauli_sum* obs, size_t n_obs,
                                double* jac, double* expval, uint32_t flags) {
    qsv_ctx* c = s ? s->ctx : nullptr;
    return guard(c, [&] {
        state_ctx(s);
        validate_ops_impl(s->n, ops, n_ops, n_params, n_mat, params, matrices);
        validate_obs_impl(s->n, obs, n_obs);
        if (n_obs == 0) return;
        if (n_params && !jac) fail(QSV_ERR_ARG, "jac is NULL");
        if (flags & ~QSV_ADJ_INPLACE) fail(QSV_ERR_ARG, "unknown flags");
        set_device(c);
        std::vector<const qsv_pauli_sum*> rows;
        for (size_t o = 0; o < n_obs; ++o) rows.push_back(&obs[o]);
        std::vector<double> jtmp(n_obs * std::max<size_t>(n_params, 1));
        adjoint_impl(s, ops, n_ops, params, n_params, matrices, rows, {}, false, jtmp.data(), expval, flags);
        if (n_params) std::memcpy(jac, jtmp.data(), n_obs * n_params * 8);
    });
}

qsv_status qsv_adjoint_vjp(qsv_state* s, const qsv_op* ops, size_t n_ops, const double* params, size_t n_params,
                           const double* matrices, size_t n_mat, const qsv_pauli_sum* obs, size_t n_obs,
                           const double* cot, double* grad, double* expval, uint32_t flags) {
    qsv_ctx* c = s ? s->ctx : nullptr;
    return guard(c, [&] {
        state_ctx(s);
        validate_ops_impl(s->n, ops, n_ops, n_params, n_mat, params, matrices);
        validate_obs_impl(s->n, obs, n_obs);
        if (n_obs == 0) return;
        if (!cot) fail(QSV_ERR_ARG, "cotangent is NULL");
        if (n_params && !grad) fail(QSV_ERR_ARG, "grad is NULL");
        if (flags & ~QSV_ADJ_INPLACE) fail(QSV_ERR_ARG, "unknown flags");
        set_device(c);
        std::vector<const qsv_pauli_sum*> rows;
        std::vector<double> sc;
        for (size_t o = 0; o < n_obs; ++o) {
            rows.push_back(&obs[o]);
            sc.push_back(cot[o]);
        }
        std::vector<double> g(std::max<size_t>(n_params, 1));
        adjoint_impl(s, ops, n_ops, params, n_params, matrices, rows, sc, true, g.data(), expval, flags);
        if (n_params) std::memcpy(grad, g.data(), n_params * 8);
    });
}

}  // extern "C"

// ------------------------------------------------------------------ batched circuits
//
// Many independent circuits of uneven width (paper Sec. 4.1 and 4.2: batches
// of circuits and observables distributed as tasks) run as one sequence of
// batched launches: launch s carries pass s of every circuit that has one,
// each block serving one (circuit, pass) entry.  States live in one pooled
// allocation; the first forward pass synthesises |0..0> instead of reading a
// reset state, and the first adjoint pass reads the post-circuit state and
// writes phi, so no copy pass is needed.  All tables (ops, coefficients,
// entries) travel in one host->device copy; with QSV_BATCH_GRAPH the whole
// sequence is captured once in a HIP graph and replayed for new parameters.

struct qsv_batch {
    qsv_ctx* ctx = nullptr;
    qsv_dtype dt = QSV_C128;
    std::vector<int> n;
    std::vector<std::vector<qsv_op>> ops;
    std::vector<size_t> n_params, p_off;
    std::vector<double> matrices;
    size_t n_mat = 0;
    std::vector<std::vector<double>> ocoef;
    std::vector<std::vector<uint64_t>> ox, oz;
    DevBuf pool, tables, partials, results;
    std::vector<size_t> off_psi, off_phi, off_lam;
    void* stage_in = nullptr;
    size_t stage_in_bytes = 0;
    void* stage_out = nullptr;
    size_t stage_out_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t graph_key = 0;
    bool graph_grad = false;
};

namespace {

uint64_t fnv(uint64_t h, const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h;
}

// Block table of a batched launch, XCD-aware: the GPU hands workgroup b to
// XCD b mod 8 and each XCD has its own L2, so every block of a circuit goes to
// the circuit's home XCD, where its state then stays cached across the
// launches of the batch.  ents: (entry, blocks, home XCD).  Returns (entry,
// local block) pairs in launch order; a position whose XCD has no blocks left
// takes one from the fullest queue.
constexpr int N_XCD = 8;
std::vector<int32_t> xcd_block_table(const std::vector<std::array<int32_t, 3>>& ents) {
    std::vector<std::vector<std::pair<int32_t, int32_t>>> q(N_XCD);
    size_t total = 0;
    for (const auto& e : ents) {
        auto& qq = q[(size_t)e[2] % N_XCD];
        for (int32_t b = e[1] - 1; b >= 0; --b) qq.push_back({e[0], b});  // popped from the back: ascending
        total += (size_t)e[1];
    }
    std::vector<int32_t> out;
    out.reserve(2 * total);
    for (size_t b = 0; b < total; ++b) {
        size_t x = b % N_XCD;
        if (q[x].empty())
            for (size_t y = 0; y < (size_t)N_XCD; ++y)
                if (q[y].size() > q[x].size()) x = y;
        out.push_back(q[x].back().first);
        out.push_back(q[x].back().second);
        q[x].pop_back();
    }
    return out;
}

// Home XCD of each circuit: longest-processing-time assignment by state
// size, so the XCDs get about equal shares of the batch.
std::vector<int32_t> xcd_homes(const std::vector<int>& n) {
    std::vector<size_t> order(n.size());
    for (size_t i = 0; i < n.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return n[a] > n[b]; });
    std::vector<double> load(N_XCD, 0.0);
    std::vector<int32_t> home(n.size(), 0);
    for (size_t i : order) {
        int x = 0;
        for (int y = 1; y < N_XCD; ++y)
            if (load[y] < load[x]) x = y;
        home[i] = x;
        load[x] += std::ldexp(1.0, n[i]);
    }
    return home;
}

struct BatchLaunch {
    enum { TILE, PAULI, REDUCE } kind;
    bool two = false, generic = false;
    int R = 1, nthr = 256, blocks = 0;
    size_t lds = 0;
    int lut_tables = 0;                   // PAULI: most byte tables of one circuit (LDS)
    size_t entries_off = 0, blk_off = 0;  // byte offsets in the table buffer
    int n_entries = 0;
    double bytes = 0;
};

struct BatchPlan {
    std::vector<char> tab;           // the device table image
    size_t off_tops = 0, off_coef = 0, off_words = 0, off_args = 0, off_pg = 0, off_pt = 0, off_re = 0;
    size_t off_aux = 0;
    int n_reduce = 0;
    std::vector<BatchLaunch> launches;
    size_t n_partials = 0, n_results = 0;
    std::vector<std::vector<std::pair<int, double>>> slot_param;  // per circuit
    std::vector<size_t> slot_base;                                // per circuit, in results
    uint64_t key = 0;                                             // structure hash (all but coefficients)
};

template <typename V>
size_t append_bytes(std::vector<char>& tab, const std::vector<V>& v) {
    const size_t off = (tab.size() + 255) & ~(size_t)255;
    tab.resize(off + v.size() * sizeof(V));
    if (!v.empty()) std::memcpy(tab.data() + off, v.data(), v.size() * sizeof(V));
    return off;
}

// Run f(0..n-1) on up to 16 host threads; the first exception is rethrown.
template <typename Fn>
void parallel_for(size_t n, Fn f) {
    const size_t hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>({hw, 16, (n + 7) / 8});
    if (nt <= 1) {
        for (size_t i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<size_t> next{0};
    std::vector<std::exception_ptr> err(nt);
    std::vector<std::thread> th;
    for (size_t t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            try {
                for (size_t i; (i = next.fetch_add(1)) < n;) f(i);
            } catch (...) {
                err[t] = std::current_exception();
                next = n;
            }
        });
    for (auto& x : th) x.join();
    for (auto& e : err)
        if (e) std::rethrow_exception(e);
}

BatchPlan plan_batch(qsv_batch* B, const double* params, bool grad) {
    BatchPlan bp;
    qsv_ctx* c = B->ctx;
    const size_t nc = B->n.size();
    const size_t eb = elem_bytes(B->dt);
    std::vector<TOp> tops;
    std::vector<cd> coef;
    std::vector<uint64_t> words;
    std::vector<TileArgs> args;
    struct StepRef {
        int args_idx, grid, R, nthr, nslots, slot_base;
        size_t lds;
        bool generic;
        double bytes;
        int64_t part_off;
    };
    std::vector<std::vector<StepRef>> fwd(nc), adj(nc);
    size_t n_part = 0;
    bp.slot_param.resize(nc);
    bp.slot_base.resize(nc);
    size_t n_res = nc;  // expvals first
    auto append_program = [&](Program& P, std::vector<StepRef>& out, bool synth_first) {
        const size_t tb = tops.size(), cb = coef.size(), wb = words.size();
        for (TOp op : P.tops) {
            op.coff += (int64_t)cb;
            op.woff += (int64_t)wb;
            tops.push_back(op);
        }
        coef.insert(coef.end(), P.coef.begin(), P.coef.end());
        words.insert(words.end(), P.words.begin(), P.words.end());
        for (size_t i = 0; i < P.steps.size(); ++i) {
            const Step& st = P.steps[i];
            TileArgs a = st.ta;
            a.op0 += (int)tb;
            a.zt_off += (int64_t)cb;
            if (synth_first && i == 0) {
                a.flags |= TILE_SYNTH;
                a.basis = 0;
            }
            StepRef r{(int)args.size(), st.grid, st.R, st.nthr, st.nslots, st.slot_base, st.lds, st.generic,
                      st.bytes, (int64_t)n_part};
            n_part += (size_t)st.nslots * st.grid;
            args.push_back(a);
            out.push_back(r);
        }
    };
    // per-circuit planning and lowering is independent: spread it over host threads
    std::vector<Program> Pf(nc), Pb(nc);
    parallel_for(nc, [&](size_t ci) {
        const int n = B->n[ci];
        const double* pp = params + B->p_off[ci];
        const auto& ops = B->ops[ci];
        std::vector<Factor> F = forward_factors(ops.data(), ops.size(), pp, B->matrices.data(), false);
        std::vector<Item> it = forward_items(F, n);
        PlanOptions po = plan_opts(c, B->dt, false);
        po.ws = false;  // the batched kernel runs the classic form
        Pf[ci] = build_program(po, F, it, n, B->dt, false, false, false);
        if (Pf[ci].steps.empty()) {  // no gates: one empty pass that writes |0..0>
            Pass p;
            const int b = std::min(po.b, n);
            p.S = (b >= 64 ? ~0ull : ((1ull << b) - 1));
            lower_tile(Pf[ci], F, it, p, n, false, false, eb);
        }
        if (grad && B->n_params[ci]) {
            std::vector<Factor> Fa = forward_factors(ops.data(), ops.size(), pp, B->matrices.data(), true);
            std::vector<Item> ia = adjoint_items(Fa, n);
            PlanOptions pa = plan_opts(c, B->dt, true);
            pa.ws = false;  // the batched kernel runs the classic form
            Pb[ci] = build_program(pa, Fa, ia, n, B->dt, true, true, false);
        }
    });
    for (size_t ci = 0; ci < nc; ++ci) {
        append_program(Pf[ci], fwd[ci], true);
        if (grad && B->n_params[ci]) {
            bp.slot_param[ci] = Pb[ci].slot_param;
            bp.slot_base[ci] = n_res;
            n_res += Pb[ci].slot_param.size();
            append_program(Pb[ci], adj[ci], false);
        }
    }
    // Pauli tables (one observable per circuit)
    PauliTables T;
    for (size_t ci = 0; ci < nc; ++ci) {
        qsv_pauli_sum h{(int64_t)B->ocoef[ci].size(), B->ocoef[ci].data(), B->ox[ci].data(), B->oz[ci].data()};
        add_pauli(T, h, 1.0);
    }
    std::vector<char>& tab = bp.tab;
    std::vector<char> coef_b = coef_bytes(coef, B->dt);
    bp.off_tops = append_bytes(tab, tops);
    bp.off_coef = append_bytes(tab, coef_b);
    bp.off_words = append_bytes(tab, words);
    bp.off_args = append_bytes(tab, args);
    bp.off_pg = append_bytes(tab, T.groups);
    bp.off_pt = append_bytes(tab, T.terms);
    bp.off_aux = append_bytes(tab, T.aux);
    const uintptr_t pool = (uintptr_t)B->pool.p;
    std::vector<ReduceEntry> reds;
    const std::vector<int32_t> home = xcd_homes(B->n);
    auto tile_launches = [&](std::vector<std::vector<StepRef>>& steps, bool two) {
        size_t max_steps = 0;
        for (auto& v : steps) max_steps = std::max(max_steps, v.size());
        for (size_t si = 0; si < max_steps; ++si) {
            // group the circuits' si-th passes by kernel variant
            std::map<std::tuple<int, int, bool>, std::vector<size_t>> groups;
            for (size_t ci = 0; ci < nc; ++ci)
                if (si < steps[ci].size()) {
                    const StepRef& r = steps[ci][si];
                    groups[{r.R, r.nthr, r.generic}].push_back(ci);
                }
            for (auto& kv : groups) {
                BatchLaunch L;
                L.kind = BatchLaunch::TILE;
                L.two = two;
                L.R = std::get<0>(kv.first);
                L.nthr = std::get<1>(kv.first);
                L.generic = std::get<2>(kv.first);
                std::vector<TileEntry> ents;
                std::vector<std::array<int32_t, 3>> eb;
                for (size_t ci : kv.second) {
                    const StepRef& r = steps[ci][si];
                    TileEntry e;
                    std::memset(&e, 0, sizeof e);
                    void* psi = (void*)(pool + B->off_psi[ci]);
                    if (two) {
                        e.phi_src = si == 0 ? psi : (void*)(pool + B->off_phi[ci]);
                        e.phi = (void*)(pool + B->off_phi[ci]);
                        e.lam = (void*)(pool + B->off_lam[ci]);
                    } else {
                        e.phi_src = psi;
                        e.phi = psi;
                        e.lam = nullptr;
                    }
                    e.part_off = r.part_off;
                    e.args = r.args_idx;
                    e.nblk = r.grid;
                    eb.push_back({(int32_t)ents.size(), r.grid, home[ci]});
                    ents.push_back(e);
                    L.lds = std::max(L.lds, r.lds);
                    L.bytes += r.bytes;
                    // slot sums: result index = circuit's slot base + step's first slot + local slot
                    for (int sl = 0; sl < r.nslots; ++sl)
                        reds.push_back({r.part_off + (int64_t)sl * r.grid, r.grid,
                                        (int32_t)(bp.slot_base[ci] + (size_t)(r.slot_base + sl))});
                }
                const std::vector<int32_t> blk = xcd_block_table(eb);
                L.blocks = (int)(blk.size() / 2);
                L.n_entries = (int)ents.size();
                L.entries_off = append_bytes(tab, ents);
                L.blk_off = append_bytes(tab, blk);
                bp.launches.push_back(L);
            }
        }
    };
    tile_launches(fwd, false);
    // <H> (and lambda = H psi when differentiating), one entry per circuit
    {
        BatchLaunch L;
        L.kind = BatchLaunch::PAULI;
        L.two = grad;
        std::vector<PauliEntry> ents;
        std::vector<std::array<int32_t, 3>> ebl;
        for (size_t ci = 0; ci < nc; ++ci) {
            const uint64_t N = 1ull << B->n[ci];
            PauliEntry e;
            std::memset(&e, 0, sizeof e);
            e.psi = (void*)(pool + B->off_psi[ci]);
            e.lam = grad ? (void*)(pool + B->off_lam[ci]) : nullptr;
            e.N = N;
            e.g0 = T.obs_groups[ci].first;
            e.ng = T.obs_groups[ci].second;
            e.nblk = std::max(1, std::min(pauli_grid(N), 256));
            e.part_off = (int64_t)n_part;
            reds.push_back({(int64_t)n_part, e.nblk, (int32_t)ci});
            L.lut_tables = std::max(L.lut_tables, T.lut_tables[ci]);
            n_part += (size_t)e.nblk;
            ebl.push_back({(int32_t)ents.size(), e.nblk, home[ci]});
            ents.push_back(e);
            L.bytes += (1.0 + T.n_x_groups[ci] + (grad ? 1.0 : 0.0)) * (double)N * eb;
        }
        const std::vector<int32_t> blk = xcd_block_table(ebl);
        L.blocks = (int)(blk.size() / 2);
        L.n_entries = (int)ents.size();
        L.entries_off = append_bytes(tab, ents);
        L.blk_off = append_bytes(tab, blk);
        bp.launches.push_back(L);
    }
    if (grad) tile_launches(adj, true);
    bp.n_reduce = (int)reds.size();
    bp.off_re = append_bytes(tab, reds);
    bp.n_partials = std::max<size_t>(n_part, 1);
    bp.n_results = n_res;
    // structure key: everything but the coefficient values
    uint64_t h = 1469598103934665603ull;
    h = fnv(h, tab.data(), bp.off_coef);
    h = fnv(h, tab.data() + bp.off_words, tab.size() - bp.off_words);
    h = fnv(h, &grad, sizeof grad);
    bp.key = h;
    return bp;
}

void pin_grow(void** p, size_t* have, size_t want) {
    if (*have >= want) return;
    if (*p) HIPCHK(hipHostFree(*p));
    *p = nullptr;
    *have = 0;
    if (hipHostMalloc(p, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        fail(QSV_ERR_OOM, "pinned host allocation failed");
    }
    *have = want;
}

// Enqueue the whole batch on the context stream (uploads, launches, download).
void enqueue_batch(qsv_batch* B, const BatchPlan& bp) {
    qsv_ctx* c = B->ctx;
    hipStream_t st = c->stream;
    HIPCHK(hipMemcpyAsync(B->tables.p, B->stage_in, bp.tab.size(), hipMemcpyHostToDevice, st));
    const char* T = (const char*)B->tables.p;
    const bool c128 = B->dt == QSV_C128;
    double* part = (double*)B->partials.p;
    for (const BatchLaunch& L : bp.launches) {
        hipError_t e = hipSuccess;
        if (L.kind == BatchLaunch::TILE) {
            Timed t(c, L.two ? KK_TILE2 : KK_TILE1, L.bytes);
            e = c128 ? launch_tile_batch<double>(st, L.two, L.generic, (const TileEntry*)(T + L.entries_off),
                                                 (const int32_t*)(T + L.blk_off), (const TileArgs*)(T + bp.off_args),
                                                 (const TOp*)(T + bp.off_tops), T + bp.off_coef,
                                                 (const uint64_t*)(T + bp.off_words), part, L.blocks, L.nthr, L.R,
                                                 L.lds)
                     : launch_tile_batch<float>(st, L.two, L.generic, (const TileEntry*)(T + L.entries_off),
                                                (const int32_t*)(T + L.blk_off), (const TileArgs*)(T + bp.off_args),
                                                (const TOp*)(T + bp.off_tops), T + bp.off_coef,
                                                (const uint64_t*)(T + bp.off_words), part, L.blocks, L.nthr, L.R,
                                                L.lds);
            t.done(e);
        } else {
            Timed t(c, L.two ? KK_PAULI_LAMBDA : KK_PAULI, L.bytes);
            e = c128 ? launch_pauli_batch<double>(st, L.two, (const PauliEntry*)(T + L.entries_off),
                                                  (const int32_t*)(T + L.blk_off),
                                                  (const PauliGroupDev*)(T + bp.off_pg),
                                                  (const PauliTermDev*)(T + bp.off_pt),
                                                  (const uint64_t*)(T + bp.off_aux), L.lut_tables, part, L.blocks)
                     : launch_pauli_batch<float>(st, L.two, (const PauliEntry*)(T + L.entries_off),
                                                 (const int32_t*)(T + L.blk_off),
                                                 (const PauliGroupDev*)(T + bp.off_pg),
                                                 (const PauliTermDev*)(T + bp.off_pt),
                                                 (const uint64_t*)(T + bp.off_aux), L.lut_tables, part, L.blocks);
            t.done(e);
        }
    }
    {
        Timed t(c, KK_REDUCE, 8.0 * bp.n_partials);
        t.done(launch_reduce_batch(st, (const ReduceEntry*)(T + bp.off_re), bp.n_reduce, part,
                                   (double*)B->results.p));
    }
    HIPCHK(hipMemcpyAsync(B->stage_out, B->results.p, bp.n_results * 8, hipMemcpyDeviceToHost, st));
}

}  // namespace

extern "C" {

qsv_status qsv_batch_create(qsv_ctx* c, qsv_dtype dt, size_t n_circuits, const int32_t* n_qubits, const qsv_op* ops,
                            const size_t* op_offsets, const size_t* n_params, const double* matrices,
                            size_t n_matrix_elems, const qsv_pauli_sum* obs, qsv_batch** out) {
    return guard(c, [&] {
        if (!c || !out || !n_qubits || !op_offsets || !n_params || !obs) fail(QSV_ERR_ARG, "NULL argument");
        *out = nullptr;
        if (dt != QSV_C64 && dt != QSV_C128) fail(QSV_ERR_DTYPE, "unknown dtype");
        if (n_circuits == 0) fail(QSV_ERR_ARG, "empty batch");
        static const double dummy = 0.0;
        std::unique_ptr<qsv_batch> B(new qsv_batch);
        B->ctx = c;
        B->dt = dt;
        size_t poff = 0, soff = 0;
        const size_t eb = elem_bytes(dt);
        for (size_t i = 0; i < n_circuits; ++i) {
            const int n = n_qubits[i];
            if (n < 1 || n > QSV_MAX_QUBITS) fail(QSV_ERR_ARG, "n_qubits out of range (circuit " + std::to_string(i) + ")");
            if (op_offsets[i + 1] < op_offsets[i]) fail(QSV_ERR_ARG, "op_offsets not monotone");
            const size_t no = op_offsets[i + 1] - op_offsets[i];
            validate_ops_impl(n, ops + op_offsets[i], no, n_params[i], n_matrix_elems, &dummy,
                              matrices ? matrices : &dummy);
            validate_obs_impl(n, &obs[i], 1);
            B->n.push_back(n);
            B->ops.emplace_back(ops + op_offsets[i], ops + op_offsets[i + 1]);
            B->n_params.push_back(n_params[i]);
            B->p_off.push_back(poff);
            poff += n_params[i];
            B->ocoef.emplace_back(obs[i].coeff, obs[i].coeff + obs[i].n_terms);
            B->ox.emplace_back(obs[i].x_mask, obs[i].x_mask + obs[i].n_terms);
            B->oz.emplace_back(obs[i].z_mask, obs[i].z_mask + obs[i].n_terms);
            const size_t bytes = (((size_t)1 << n) * eb + 255) & ~(size_t)255;
            B->off_psi.push_back(soff);
            B->off_phi.push_back(soff + bytes);
            B->off_lam.push_back(soff + 2 * bytes);
            soff += 3 * bytes;
        }
        B->p_off.push_back(poff);
        if (matrices && n_matrix_elems) B->matrices.assign(matrices, matrices + 2 * n_matrix_elems);
        else B->matrices.assign(2, 0.0);
        B->n_mat = n_matrix_elems;
        set_device(c);
        ensure(c, B->pool, soff);
        *out = B.release();
    });
}

void qsv_batch_destroy(qsv_batch* B) {
    if (!B) return;
    (void)hipSetDevice(B->ctx->device);
    (void)hipStreamSynchronize(B->ctx->stream);
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    for (DevBuf* b : {&B->pool, &B->tables, &B->partials, &B->results}) release(*b);
    if (B->stage_in) (void)hipHostFree(B->stage_in);
    if (B->stage_out) (void)hipHostFree(B->stage_out);
    delete B;
}

qsv_status qsv_batch_run(qsv_batch* B, const double* params, double* expval, double* grad, uint32_t flags) {
    qsv_ctx* c = B ? B->ctx : nullptr;
    return guard(c, [&] {
        if (!B || !expval) fail(QSV_ERR_ARG, "NULL argument");
        if (flags & ~(uint32_t)QSV_BATCH_GRAPH) fail(QSV_ERR_ARG, "unknown flags");
        if (B->p_off.back() && !params) fail(QSV_ERR_ARG, "params is NULL");
        static const double dummy = 0.0;
        const double* pp = params ? params : &dummy;
        const bool want_grad = grad != nullptr;
        set_device(c);
        BatchPlan bp = plan_batch(B, pp, want_grad);
        const bool use_graph = (flags & QSV_BATCH_GRAPH) != 0;
        const bool same = use_graph && B->exec && B->graph_key == bp.key && B->graph_grad == want_grad;
        if (!same) {
            // (re)allocate device and staging buffers: pointers baked into a
            // graph must stay valid, so a new structure rebuilds the graph
            HIPCHK(hipStreamSynchronize(c->stream));
            if (B->exec) HIPCHK(hipGraphExecDestroy(B->exec));
            if (B->graph) HIPCHK(hipGraphDestroy(B->graph));
            B->exec = nullptr;
            B->graph = nullptr;
            ensure(c, B->tables, bp.tab.size());
            ensure(c, B->partials, bp.n_partials * 8);
            ensure(c, B->results, bp.n_results * 8);
            pin_grow(&B->stage_in, &B->stage_in_bytes, bp.tab.size());
            pin_grow(&B->stage_out, &B->stage_out_bytes, bp.n_results * 8);
        }
        std::memcpy(B->stage_in, bp.tab.data(), bp.tab.size());
        if (use_graph) {
            if (!same) {
                HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
                const int64_t prof = c->opt_profile;
                c->opt_profile = 0;  // no event records inside the graph
                try {
                    enqueue_batch(B, bp);
                } catch (...) {
                    c->opt_profile = prof;
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(c->stream, &g);
                    if (g) (void)hipGraphDestroy(g);
                    throw;
                }
                c->opt_profile = prof;
                HIPCHK(hipStreamEndCapture(c->stream, &B->graph));
                HIPCHK(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
                B->graph_key = bp.key;
                B->graph_grad = want_grad;
            }
            HIPCHK(hipGraphLaunch(B->exec, c->stream));
        } else {
            enqueue_batch(B, bp);
        }
        HIPCHK(hipStreamSynchronize(c->stream));
        const double* res = (const double*)B->stage_out;
        const size_t nc = B->n.size();
        for (size_t ci = 0; ci < nc; ++ci) expval[ci] = res[ci];
        if (want_grad) {
            for (size_t ci = 0; ci < nc; ++ci) {
                double* g = grad + B->p_off[ci];
                std::fill(g, g + B->n_params[ci], 0.0);
                const auto& sp = bp.slot_param[ci];
                for (size_t q = 0; q < sp.size(); ++q) g[sp[q].first] += sp[q].second * res[bp.slot_base[ci] + q];
            }
        }
    });
}

}  // extern "C"

// ------------------------------------------------------------------ tile-width tuner

extern "C" qsv_status qsv_autotune(qsv_state* s, const qsv_op* ops, size_t n_ops, const double* params,
                                   size_t n_params, const double* matrices, size_t n_mat, const qsv_pauli_sum* obs,
                                   size_t n_obs, int32_t* tile_bits, int32_t* tile_bits_adj) {
    qsv_ctx* c = s ? s->ctx : nullptr;
    return guard(c, [&] {
        state_ctx(s);
        validate_ops_impl(s->n, ops, n_ops, n_params, n_mat, params, matrices);
        validate_obs_impl(s->n, obs, n_obs);
        if (!tile_bits || !tile_bits_adj) fail(QSV_ERR_ARG, "NULL argument");
        set_device(c);
        const bool c128 = s->dt == QSV_C128;
        const int n = s->n;
        auto check = [&](qsv_status st) {
            if (st != QSV_OK) fail(st, c->err);
        };
        auto seconds = [&](auto&& fn) {
            fn();  // warm-up (plans, uploads, first-launch costs)
            check(qsv_ctx_synchronize(c));
            double best = 1e300;
            for (int rep = 0; rep < 2; ++rep) {
                const auto t0 = std::chrono::steady_clock::now();
                fn();
                check(qsv_ctx_synchronize(c));
                best = std::min(best, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
            }
            return best;
        };
        const int64_t keep_f = c->opt_tile_bits, keep_a = c->opt_tile_bits_adj;
        const int64_t keep_layers = c->opt_layers, keep_low = c->opt_low_bits;
        // candidates: tiles from 2^10 amplitudes up to the LDS limit of two
        // blocks (one vector) or one block (two vectors) per CU, capped at n
        const int fmax = std::min(n, c128 ? 13 : 13), amax = std::min(n, c128 ? 12 : 13);
        int best_f = 0, best_a = 0;
        try {
            double tb = 1e300;
            for (int b = std::min(fmax, 10); b <= fmax; ++b) {
                c->opt_tile_bits = b;
                const double t = seconds([&] {
                    check(qsv_state_reset(s, 0));
                    check(qsv_apply(s, ops, n_ops, params, n_params, matrices, n_mat));
                });
                if (t < tb) tb = t, best_f = b;
            }
            c->opt_tile_bits = best_f;
            check(qsv_state_reset(s, 0));
            check(qsv_apply(s, ops, n_ops, params, n_params, matrices, n_mat));
            if (n_obs && n_params) {
                std::vector<double> jac(n_obs * n_params), ev(n_obs);
                double ta = 1e300;
                for (int b = std::min(amax, 9); b <= amax; ++b) {
                    c->opt_tile_bits_adj = b;
                    const double t = seconds([&] {
                        check(qsv_adjoint_jacobian(s, ops, n_ops, params, n_params, matrices, n_mat, obs, n_obs,
                                                   jac.data(), ev.data(), 0));
                    });
                    if (t < ta) ta = t, best_a = b;
                }
            }
            // then the fusion form at those widths: one-qubit layers on or
            // off, and the number of lowest index bits every pass keeps in
            // its tile (the default, one fewer, one more), timed on the whole
            // program (forward, and the adjoint sweep when it is given)
            c->opt_tile_bits_adj = best_a ? best_a : keep_a;
            const int low_def = c128 ? 4 : 5;
            double tbest = 1e300;
            int64_t best_layers = 1, best_low = 0;
            std::vector<double> jac2(n_obs * n_params), ev2(n_obs);
            for (int64_t layers : {1, 0})
                for (int64_t low : {(int64_t)0, (int64_t)low_def - 1, (int64_t)low_def + 1}) {
                    c->opt_layers = layers;
                    c->opt_low_bits = low;
                    const double t = seconds([&] {
                        check(qsv_state_reset(s, 0));
                        check(qsv_apply(s, ops, n_ops, params, n_params, matrices, n_mat));
                        if (n_obs && n_params)
                            check(qsv_adjoint_jacobian(s, ops, n_ops, params, n_params, matrices, n_mat, obs,
                                                       n_obs, jac2.data(), ev2.data(), 0));
                    });
                    if (t < tbest) tbest = t, best_layers = layers, best_low = low;
                }
            c->opt_layers = best_layers;
            c->opt_low_bits = best_low;
        } catch (...) {
            c->opt_tile_bits = keep_f;
            c->opt_tile_bits_adj = keep_a;
            c->opt_layers = keep_layers;
            c->opt_low_bits = keep_low;
            throw;
        }
        c->opt_tile_bits = best_f;
        c->opt_tile_bits_adj = best_a ? best_a : keep_a;
        *tile_bits = (int32_t)c->opt_tile_bits;
        *tile_bits_adj = (int32_t)c->opt_tile_bits_adj;
    });
}
