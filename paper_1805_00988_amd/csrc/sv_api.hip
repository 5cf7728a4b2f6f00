// Host side of libsv.so: argument validation, state handles, the gate table
// for sv_op records, single-gate dispatch, the tile-pass scheduler of sv_run,
// and the reductions' host results.
#include "sv_internal.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

struct sv_state {
    int n = 0;
    int dtype = 0;
    void *amps = nullptr;
    bool owned = false;
    hipStream_t stream = nullptr;
    int device = 0;
    double *d_red = nullptr;          // kReduceBlocks partials + 1 total
    double *h_result = nullptr;       // pinned, 8 doubles
    // staging arena: per-call records (tile-pass gates, block matrices,
    // MFMA operand fragments) written to pinned host memory and copied once
    // per call to the device arena on the handle's stream
    char *d_arena = nullptr;
    char *h_arena = nullptr;
    size_t arena_cap = 0;
    hipEvent_t stage_done = nullptr;  // last copy out of h_arena
    bool stage_pending = false;
    // per-launch timing (sv_timing): event pairs around each kernel launch
    struct Rec {
        int kid;
        double bytes, flops;
        hipEvent_t a, b;
    };
    double *d_scratch = nullptr;      // adjoint partial sums
    size_t scratch_cap = 0;           // in doubles
    bool timing = false;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    size_t pool_used = 0;
};

namespace sv {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

static int hip_fail(hipError_t e, const char *where) {
    return fail(SV_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define SV_HIP(call)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return hip_fail(e_, #call);                                          \
    } while (0)

// ----------------------------------------------------------- launch timing
enum KernelId { K_INIT, K_GATE1, K_GATE2, K_SCALE, K_TILE, K_PROBS, K_EXPECT, K_FUSED, K_ADJOINT,
                K_MEASURE, K_COUNT };
static const char *kKernelNames[K_COUNT] = {"init_basis", "gate1_stream", "gate2_stream",
                                            "scale_subspace", "tile_pass", "probabilities",
                                            "expectation", "fused_block", "adjoint_step", "measurement"};

static hipEvent_t take_event(sv_state *h) {
    if (h->pool_used == h->pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->pool.push_back(e);
    }
    return h->pool[h->pool_used++];
}

// Brackets one kernel launch with events on the handle's stream when timing
// is on; 'bytes' is the algorithmic HBM traffic of the launch and 'flops'
// its algorithmic floating-point operations.
struct Timed {
    sv_state *h;
    int kid;
    double bytes, flops;
    hipEvent_t a = nullptr;
    Timed(sv_state *h_, int kid_, double bytes_, double flops_ = 0.0)
        : h(h_), kid(kid_), bytes(bytes_), flops(flops_) {
        if (h->timing && (a = take_event(h)) != nullptr) (void)hipEventRecord(a, h->stream);
    }
    ~Timed() {
        if (!a) return;
        hipEvent_t b = take_event(h);
        if (!b) return;
        (void)hipEventRecord(b, h->stream);
        h->recs.push_back({kid, bytes, flops, a, b});
    }
};

static double state_bytes(const sv_state *h) {
    return (double)(1ull << h->n) * (h->dtype == SV_C64 ? 8.0 : 16.0);
}

// ------------------------------------------------------------ gate table
// H X Y Z S T per the gate table of Sec. 1.3.2; rotations exp(-i theta P/2);
// U1 = diag(1, e^{i theta}).  Output: 4 complex entries, row-major, (re, im).
static bool named_matrix(int kind, double th, double *U) {
    const double c = std::cos(0.5 * th), s = std::sin(0.5 * th);
    const double h = 0.70710678118654752440;
    double m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    switch (kind) {
    case SV_GATE_H: m[0] = h; m[2] = h; m[4] = h; m[6] = -h; break;
    case SV_GATE_X: m[2] = 1; m[4] = 1; break;
    case SV_GATE_Y: m[3] = -1; m[5] = 1; break;
    case SV_GATE_Z: m[0] = 1; m[6] = -1; break;
    case SV_GATE_S: m[0] = 1; m[7] = 1; break;
    case SV_GATE_T: m[0] = 1; m[6] = h; m[7] = h; break;
    case SV_GATE_RX: m[0] = c; m[3] = -s; m[5] = -s; m[6] = c; break;
    case SV_GATE_RY: m[0] = c; m[2] = -s; m[4] = s; m[6] = c; break;
    case SV_GATE_RZ: m[0] = c; m[1] = -s; m[6] = c; m[7] = s; break;
    case SV_GATE_U1: m[0] = 1; m[6] = std::cos(th); m[7] = std::sin(th); break;
    default: return false;
    }
    std::memcpy(U, m, sizeof(m));
    return true;
}

// A gate in canonical form: k targets, controls, 2^k x 2^k matrix.
struct Gate {
    int k;
    int t[2];
    uint64_t ctrl;
    double U[32];
    uint64_t tmask() const { return (1ull << t[0]) | (k == 2 ? (1ull << t[1]) : 0ull); }
    uint64_t qmask() const { return tmask() | ctrl; }
};

static int check_gate(int n, int k, const int *targets, uint64_t ctrl, const double *U) {
    if (!targets || !U) return fail(SV_EINVAL, "NULL targets or matrix");
    if (k != 1 && k != 2) return fail(SV_EINVAL, "k must be 1 or 2");
    uint64_t seen = 0;
    for (int j = 0; j < k; ++j) {
        if (targets[j] < 0 || targets[j] >= n)
            return fail(SV_EINVAL, "target qubit " + std::to_string(targets[j]) + " outside [0, n)");
        if (seen & (1ull << targets[j])) return fail(SV_EINVAL, "duplicate target qubits");
        seen |= 1ull << targets[j];
    }
    if (n < 64 && (ctrl >> n) != 0) return fail(SV_EINVAL, "control mask has bits >= n");
    if (ctrl & seen) return fail(SV_EINVAL, "a control qubit is also a target");
    for (int i = 0; i < 2 * (1 << (2 * k)); ++i)
        if (!std::isfinite(U[i])) return fail(SV_EINVAL, "matrix entry is not finite");
    return SV_OK;
}

static int op_to_gate(int n, const sv_op &op, const double *params, int n_params, Gate *g) {
    double th = op.theta;
    if (op.param_index >= 0) {
        if (!params || op.param_index >= n_params)
            return fail(SV_EINVAL, "param_index outside the parameter vector");
        th = params[op.param_index];
    }
    g->ctrl = op.ctrl_mask;
    if (op.kind == SV_GATE_MATRIX) {
        if (op.n_targets != 1 && op.n_targets != 2)
            return fail(SV_EINVAL, "matrix op needs 1 or 2 targets");
        g->k = op.n_targets;
        g->t[0] = op.targets[0];
        g->t[1] = op.n_targets == 2 ? op.targets[1] : -1;
        std::memcpy(g->U, op.matrix, sizeof(double) * 2 * (1 << (2 * g->k)));
    } else {
        if (op.n_targets != 1) return fail(SV_EINVAL, "named gates take one target");
        g->k = 1;
        g->t[0] = op.targets[0];
        g->t[1] = -1;
        if (!named_matrix(op.kind, th, g->U))
            return fail(SV_EINVAL, "unknown gate kind " + std::to_string(op.kind));
    }
    return check_gate(n, g->k, g->t, g->ctrl, g->U);
}

// ---------------------------------------------------------------- buffers
static int ensure_arena(sv_state *h, size_t bytes) {
    if (bytes <= h->arena_cap) return SV_OK;
    size_t cap = std::max<size_t>(1 << 16, h->arena_cap);
    while (cap < bytes) cap *= 2;
    if (h->stage_pending) SV_HIP(hipEventSynchronize(h->stage_done));
    // the old device arena may still be read by queued kernels: drain first
    SV_HIP(hipStreamSynchronize(h->stream));
    h->stage_pending = false;
    if (h->d_arena) SV_HIP(hipFree(h->d_arena));
    if (h->h_arena) SV_HIP(hipHostFree(h->h_arena));
    h->d_arena = nullptr;
    h->h_arena = nullptr;
    h->arena_cap = 0;
    SV_HIP(hipMalloc((void **)&h->d_arena, cap));
    SV_HIP(hipHostMalloc((void **)&h->h_arena, cap, hipHostMallocDefault));
    h->arena_cap = cap;
    return SV_OK;
}

// Copy the staged bytes to the device arena on the handle's stream.  Kernels
// queued earlier that read the arena finish before the copy (stream order).
static int upload_arena(sv_state *h, size_t bytes) {
    SV_HIP(hipMemcpyAsync(h->d_arena, h->h_arena, bytes, hipMemcpyHostToDevice, h->stream));
    SV_HIP(hipEventRecord(h->stage_done, h->stream));
    h->stage_pending = true;
    return SV_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int stage_wait(sv_state *h) {
    if (h->stage_pending) SV_HIP(hipEventSynchronize(h->stage_done));
    h->stage_pending = false;
    return SV_OK;
}

// ------------------------------------------------------- single-gate path
static bool is_one(const double *z) { return z[0] == 1.0 && z[1] == 0.0; }
static bool is_zero(const double *z) { return z[0] == 0.0 && z[1] == 0.0; }

static int vbits_of(int dtype) { return dtype == SV_C64 ? 1 : 0; }

// Tile pass holding one gate (used for two-qubit gates on qubit 0 of a
// complex64 state, whose pair partner is inside a 16-byte vector).
static int tile_single(sv_state *h, const Gate &g);

static double gate_flops_per_amp(const Gate &g);

static int apply_one(sv_state *h, const Gate &g) {
    if (g.k == 1) {
        const double *U = g.U;
        if (is_zero(U + 2) && is_zero(U + 4)) {
            if (is_one(U) && is_one(U + 6)) return SV_OK; // identity
            if (is_one(U)) {
                const uint64_t mask = g.ctrl | (1ull << g.t[0]);
                Timed tm(h, K_SCALE, 2.0 * state_bytes(h) / (double)(1ull << __builtin_popcountll(mask)),
                         6.0 * (double)(1ull << h->n) / (double)(1ull << __builtin_popcountll(mask)));
                SV_HIP(launch_scale(h->amps, h->n, h->dtype, mask, U + 6, h->stream));
                return SV_OK;
            }
        }
        Timed tm(h, K_GATE1, 2.0 * state_bytes(h) / (double)(1ull << __builtin_popcountll(g.ctrl)),
                 gate_flops_per_amp(g) * (double)(1ull << h->n));
        SV_HIP(launch_gate1(h->amps, h->n, h->dtype, g.t[0], g.ctrl, g.U, h->stream));
        return SV_OK;
    }
    const int vb = vbits_of(h->dtype);
    if (g.t[0] >= vb && g.t[1] >= vb) {
        Timed tm(h, K_GATE2, 2.0 * state_bytes(h) / (double)(1ull << __builtin_popcountll(g.ctrl)),
                 gate_flops_per_amp(g) * (double)(1ull << h->n));
        SV_HIP(launch_gate2(h->amps, h->n, h->dtype, g.t[0], g.t[1], g.ctrl, g.U, h->stream));
        return SV_OK;
    }
    return tile_single(h, g);
}

// ------------------------------------------------------------- tile passes
struct Pass {
    std::vector<int> gates; // indices into the gate list, in application order
    uint64_t S = 0;         // qubits staged in the tile
};

static void tile_layout(int n, int mmax, int lmin, uint64_t needed, TileSpec *sp) {
    // low block of L >= lmin qubits plus the needed qubits above it; the
    // scheduler guarantees lmin + popcount(needed >> lmin) <= mmax.  L then
    // grows while the tile has room, absorbing needed qubits it passes.
    int L = std::min(lmin, n);
    int K = __builtin_popcountll(needed >> L);
    while (L + K < mmax && L < n) {
        ++L;
        K = __builtin_popcountll(L < 64 ? needed >> L : 0);
    }
    sp->L = L;
    sp->K = 0;
    uint64_t hi = L < 64 ? (needed >> L) << L : 0;
    while (hi) {
        const int b = __builtin_ctzll(hi);
        hi &= hi - 1;
        sp->high[sp->K++] = b;
    }
}

static int local_bit(const TileSpec &sp, int q) {
    if (q < sp.L) return q;
    for (int i = 0; i < sp.K; ++i)
        if (sp.high[i] == q) return sp.L + i;
    return -1;
}

// Qubits a tile layout holds.
static uint64_t tile_qubits(const TileSpec &sp) {
    uint64_t S = sp.L >= 64 ? ~0ull : ((1ull << sp.L) - 1ull);
    for (int i = 0; i < sp.K; ++i) S |= 1ull << sp.high[i];
    return S;
}

// A tile pass compiled for the device: tile layout, register sweeps and the
// sweeps' gate records (stored consecutively in sweep order).
struct PassCode {
    TileSpec sp{};
    int m = 0;
    double flops_per_amp = 0.0; // algorithmic flops of the pass per state amplitude
    bool two_qubit = false;     // holds SK_2Q records
    bool lane_phases = false;   // holds SK_LPH records
    uint32_t direct = 0;        // kDirectFirst / kDirectLast (launch_tile)
    std::vector<TileSweep> sweeps;
    std::vector<TileGate> gates; // records in sweep order (host form)
    std::vector<std::vector<char>> tables; // SK_PTAB payloads (descriptors and tables)
    std::vector<char> recs;      // the same, packed for the device (pack_records)
    size_t bytes() const { return align256(sweeps.size() * sizeof(TileSweep)) + recs.size(); }
};

// Bytes of matrix data a record reads on the device.
static size_t record_payload(const TileGate &r, bool f32) {
    const size_t c = f32 ? 8 : 16; // one complex entry
    switch (r.kind) {
    case SK_2Q: return 16 * c;
    case SK_GEN: case SK_REAL: case SK_RIMAG: case SK_PARAM: return 4 * c;
    case SK_DIAG: case SK_DIAGR: return 2 * c;
    case SK_PHASE: case SK_LPH: return (size_t)r.b1 * (8 + c); // b1 entries of (condition, phase)
    default: return 0; // SK_SWAP, SK_FLUSH
    }
}

// Pack the records (each cut after its entries, 8-byte aligned sizes) and
// point every sweep at its first record.
static void pack_records(PassCode &pc, bool f32) {
    pc.recs.clear();
    size_t gi = 0;
    for (TileSweep &S : pc.sweeps) {
        S.rec_off = (int32_t)pc.recs.size();
        for (int k = 0; k < S.n_gates; ++k, ++gi) {
            TileGate r = pc.gates[gi];
            if (r.kind == SK_PTAB) { // head, then its payload (index in m[0])
                uint64_t ti;
                std::memcpy(&ti, r.m, 8);
                const std::vector<char> &pl = pc.tables[ti];
                r.size = (int32_t)(kRecordHead + pl.size());
                const char *src = reinterpret_cast<const char *>(&r);
                pc.recs.insert(pc.recs.end(), src, src + kRecordHead);
                pc.recs.insert(pc.recs.end(), pl.begin(), pl.end());
                continue;
            }
            const size_t sz = ((size_t)kRecordHead + record_payload(r, f32) + 7) & ~(size_t)7;
            r.size = (int32_t)sz;
            const char *src = reinterpret_cast<const char *>(&r);
            pc.recs.insert(pc.recs.end(), src, src + sz);
        }
    }
    pc.recs.resize(pc.recs.size() + kRecordTail, 0);
}

static bool is_diag1(const Gate &g) { return g.k == 1 && is_zero(g.U + 2) && is_zero(g.U + 4); }

static bool is_x(const Gate &g) {
    const double x[8] = {0, 0, 1, 0, 1, 0, 0, 0};
    return g.k == 1 && std::memcmp(g.U, x, sizeof(x)) == 0;
}

// Controls of a gate: bits outside the tile go to the record (tested once
// per tile on its base index); the local bits inside the tile are returned.
static uint32_t encode_controls(const TileSpec &sp, uint64_t ctrl, TileGate *r) {
    uint32_t cin = 0;
    for (uint64_t c = ctrl; c; c &= c - 1) {
        const int b = __builtin_ctzll(c);
        const int lb = local_bit(sp, b);
        if (lb >= 0) cin |= 1u << lb;
        else r->cout |= 1ull << b;
    }
    return cin;
}

// Tile bits of register index j of a sweep over the local positions qset.
static uint32_t register_bits(const std::vector<int> &qset, int j) {
    uint32_t f = 0;
    for (size_t b = 0; b < qset.size(); ++b)
        if ((j >> b) & 1) f |= 1u << qset[b];
    return f;
}

// Split the in-tile controls cin of a record into the per-lane part and the
// register-index mask: amask gets every j with no bit of 'skip' set (the low
// index of a pair or quad), with 'need' set, and whose register bits hold
// the register controls.
static void encode_sweep_masks(const std::vector<int> &qset, uint32_t cin, uint32_t skip, uint32_t need,
                               TileGate *r) {
    const uint32_t fall = register_bits(qset, (1 << qset.size()) - 1);
    const uint32_t cr = cin & fall;
    r->lane = cin & ~fall;
    r->amask = 0;
    for (int j = 0; j < (1 << qset.size()); ++j)
        if (!(j & skip) && (j & need) == need && (register_bits(qset, j) & cr) == cr) r->amask |= 1u << j;
}

// Store n complex entries (re, im interleaved, FP64) in the record in the
// state's precision.
static void put_matrix(TileGate &r, const double *U, int n, bool f32) {
    if (!f32) {
        std::memcpy(r.m, U, sizeof(double) * 2 * n);
        return;
    }
    float *f = reinterpret_cast<float *>(r.m);
    for (int i = 0; i < 2 * n; ++i) f[i] = (float)U[i];
}

// Algorithmic floating-point operations per updated amplitude of a gate:
// general 2x2 complex matvec 14 (two complex products and a sum per
// output), real 2x2 6, diagonal 6 (3 on average for a phase gate, which
// changes half of the amplitudes), swap 0, general 4x4 30.  A gate with c
// controls updates 2^-c of the state.
static double gate_flops_per_amp(const Gate &g) {
    double f;
    if (is_diag1(g)) f = is_one(g.U) ? 3.0 : 6.0;
    else if (g.k == 1) {
        bool real = true;
        for (int i = 0; i < 4; ++i) real = real && g.U[2 * i + 1] == 0.0;
        f = is_x(g) ? 0.0 : (real ? 6.0 : 14.0);
    } else f = 30.0;
    return f / (double)(1ull << __builtin_popcountll(g.ctrl));
}

static TileGate encode_sweep_gate(const TileSpec &sp, const std::vector<int> &qset, const Gate &g,
                                  bool f32) {
    TileGate r;
    std::memset(&r, 0, sizeof(r));
    const uint32_t cin = encode_controls(sp, g.ctrl, &r);
    auto pos = [&](int q) {
        const int lb = local_bit(sp, q);
        for (size_t j = 0; j < qset.size(); ++j)
            if (qset[j] == lb) return (int)j;
        return -1;
    };
    if (is_diag1(g)) {
        const double d[4] = {g.U[0], g.U[1], g.U[6], g.U[7]};
        const int p = pos(g.t[0]);
        put_matrix(r, d, 2, f32);
        if (p >= 0) {
            // on a register position: a phase gate (d0 = 1) leaves the
            // amplitudes with the target bit clear alone
            r.kind = SK_DIAGR;
            r.b0 = p;
            encode_sweep_masks(qset, cin, 0, is_one(g.U) ? 1u << p : 0u, &r);
        } else {
            r.kind = SK_DIAG;
            r.b0 = local_bit(sp, g.t[0]);
            encode_sweep_masks(qset, cin, 0, 0, &r);
        }
        return r;
    }
    if (g.k == 1) {
        r.b0 = pos(g.t[0]);
        bool real = true;
        for (int i = 0; i < 4; ++i) real = real && g.U[2 * i + 1] == 0.0;
        // real diagonal, imaginary off-diagonal: half the arithmetic of a general matrix
        const bool rimag = g.U[1] == 0.0 && g.U[7] == 0.0 && g.U[2] == 0.0 && g.U[4] == 0.0;
        encode_sweep_masks(qset, cin, 1u << r.b0, 0, &r);
        // an exchange with per-lane controls runs as selects (complex64) or
        // as the real matrix X (complex128)
        r.kind = is_x(g) && (r.lane == 0 || f32) ? SK_SWAP : (real ? SK_REAL : (rimag ? SK_RIMAG : SK_GEN));
        put_matrix(r, g.U, 4, f32);
        return r;
    }
    r.kind = SK_2Q;
    const int p0 = pos(g.t[0]), p1 = pos(g.t[1]);
    if (p0 < p1) {
        r.b0 = p0;
        r.b1 = p1;
        put_matrix(r, g.U, 16, f32);
    } else { // bit 0 of the matrix index must name the lower position: swap index bits
        r.b0 = p1;
        r.b1 = p0;
        double u[32];
        auto sw = [](int i) { return ((i & 1) << 1) | ((i >> 1) & 1); };
        for (int row = 0; row < 4; ++row)
            for (int col = 0; col < 4; ++col) {
                const int src = sw(row) * 4 + sw(col), dst = row * 4 + col;
                u[2 * dst] = g.U[2 * src];
                u[2 * dst + 1] = g.U[2 * src + 1];
            }
        put_matrix(r, u, 16, f32);
    }
    encode_sweep_masks(qset, cin, (1u << r.b0) | (1u << r.b1), 0, &r);
    return r;
}

// Phases gathered for one (slot, per-lane mask): each entry multiplies the
// tile's factor by its phase when the tile's global index holds all bits of
// its condition (bits outside the tile).  Entries whose conditions lie in a
// window of at most kPtabBits consecutive index bits are replaced by a table
// over that window: entry x is the product of the window's phases whose
// condition holds for index bits x (the product formed in FP64, rounded
// once), so the device takes one table entry per window instead of testing
// and multiplying every phase.  Entries without a condition fold into the
// first table.  Windows cover at least two entries; the rest stay a list.
struct PhaseEntry {
    uint64_t cond;
    std::complex<double> ph;
};
struct PhaseWindow {
    int shift, bits;
    std::vector<std::complex<double>> tab;
};
static void phase_windows(const std::vector<PhaseEntry> &ents, std::vector<PhaseWindow> *wins,
                          std::vector<PhaseEntry> *rest) {
    std::complex<double> k0 = 1.0;
    bool has0 = false;
    std::vector<PhaseEntry> cond;
    for (const PhaseEntry &e : ents) {
        if (e.cond == 0) {
            k0 *= e.ph;
            has0 = true;
        } else {
            cond.push_back(e);
        }
    }
    std::stable_sort(cond.begin(), cond.end(), [](const PhaseEntry &a, const PhaseEntry &b) {
        return __builtin_ctzll(a.cond) < __builtin_ctzll(b.cond);
    });
    std::vector<char> used(cond.size(), 0);
    for (size_t i = 0; i < cond.size(); ++i) {
        if (used[i]) continue;
        const int s = __builtin_ctzll(cond[i].cond);
        if ((cond[i].cond >> s) >= (1ull << kPtabBits)) { // wider than a window
            rest->push_back(cond[i]);
            used[i] = 1;
            continue;
        }
        std::vector<size_t> in;
        uint64_t span = 0;
        for (size_t j = i; j < cond.size(); ++j)
            if (!used[j] && (cond[j].cond >> s) < (1ull << kPtabBits)) {
                in.push_back(j);
                span |= cond[j].cond >> s;
            }
        if (in.size() < 2) {
            rest->push_back(cond[i]);
            used[i] = 1;
            continue;
        }
        PhaseWindow w;
        w.shift = s;
        w.bits = 64 - __builtin_clzll(span);
        w.tab.assign((size_t)1 << w.bits, 1.0);
        for (size_t j : in) {
            used[j] = 1;
            const uint64_t c = cond[j].cond >> s;
            for (uint64_t x = 0; x < w.tab.size(); ++x)
                if ((x & c) == c) w.tab[x] *= cond[j].ph;
        }
        wins->push_back(std::move(w));
    }
    if (has0) {
        if (!wins->empty()) {
            for (auto &z : (*wins)[0].tab) z *= k0;
        } else {
            rest->push_back({0, k0});
        }
    }
}

// Group the pass's gates (in order) into sweeps of at most W register
// qubits; diagonal one-qubit gates join the current sweep whatever their
// target, since they act per amplitude.
// Probe of a parametrised gate in an adjoint pass: slot within the pass and
// the 2x2 probe matrix (complex, interleaved).
struct Probe {
    int slot;
    double M[8];
};

static TileGate encode_probe(const TileSpec &sp, const std::vector<int> &qset, const Gate &g, const Probe &pr,
                             bool f32) {
    TileGate r;
    std::memset(&r, 0, sizeof(r));
    const uint32_t cin = encode_controls(sp, g.ctrl, &r);
    // the probes of RX, RY, RZ and U1 have their own kinds (no matrix)
    auto is_m = [&](const double *m) { return std::memcmp(pr.M, m, sizeof(pr.M)) == 0; };
    const double mx[8] = {0, 0, 1, 0, 1, 0, 0, 0}, my[8] = {0, 0, 0, -1, 0, 1, 0, 0};
    const double mz[8] = {1, 0, 0, 0, 0, 0, -1, 0}, mp[8] = {0, 0, 0, 0, 0, 0, 1, 0};
    r.kind = is_m(mx) ? SK_PROBE_X : is_m(my) ? SK_PROBE_Y : is_m(mz) ? SK_PROBE_Z : is_m(mp) ? SK_PROBE_P1 : SK_PARAM;
    const int lb = local_bit(sp, g.t[0]);
    r.b0 = (int)(std::find(qset.begin(), qset.end(), lb) - qset.begin());
    r.b1 = pr.slot;
    encode_sweep_masks(qset, cin, 1u << r.b0, 0, &r);
    if (r.kind == SK_PARAM) put_matrix(r, pr.M, 4, f32);
    return r;
}

// Group the pass's gates (in order) into sweeps of at most W register
// qubits; diagonal one-qubit gates join the current sweep whatever their
// target, since they act per amplitude.  With probes (adjoint passes), a
// parametrised gate needs its target in registers and is encoded as a probe
// record followed by its own record.
// shortest run of phase gates gathered into per-lane factors (a flush costs
// about as much as applying three of them one by one)
constexpr int kMinPhaseRun = 4;

static PassCode compile_pass(const TileSpec &sp, const std::vector<const Gate *> &gs, int sweep_w, bool f32,
                             const std::vector<const Probe *> *probes = nullptr, bool lph_f32 = false) {
    PassCode pc;
    pc.sp = sp;
    pc.m = sp.L + sp.K;
    const int W = std::min(pc.m, sweep_w);
    std::vector<int> qset;
    std::vector<size_t> cur;
    auto probe_of = [&](size_t i) -> const Probe * { return probes ? (*probes)[i] : nullptr; };
    auto close = [&]() {
        if (cur.empty()) return;
        // free register positions come from the top of the tile, leaving the
        // low tile bits to the lanes (contiguous accesses)
        for (int b = pc.m - 1; (int)qset.size() < W && b >= 0; --b)
            if (std::find(qset.begin(), qset.end(), b) == qset.end()) qset.push_back(b);
        std::sort(qset.begin(), qset.end());
        TileSweep sw{};
        sw.n_gates = 0;
        const uint32_t fall = register_bits(qset, (1 << qset.size()) - 1);
        // Phase gates whose condition holds at most one register bit are
        // gathered into per-lane factors (all diagonal gates commute) when at
        // least kMinPhaseRun of them follow each other; a flush applies them.
        // Diagonal gates whose target lies outside the tile (their factor is
        // uniform over the tile's lanes for each value of the target) are
        // always gathered.
        std::vector<int> slot(cur.size(), -1);
        auto outside = [&](const Gate &g) { return is_diag1(g) && local_bit(sp, g.t[0]) < 0; };
        if (!probes) {
            for (size_t a = 0; a < cur.size();) {
                size_t b = a;
                while (b < cur.size()) {
                    const Gate &g = *gs[cur[b]];
                    if (!is_diag1(g) || !(is_one(g.U) || outside(g))) break;
                    TileGate tmp{};
                    const int lt = local_bit(sp, g.t[0]);
                    const uint32_t cond = encode_controls(sp, g.ctrl, &tmp) | (lt >= 0 ? 1u << lt : 0u);
                    const uint32_t reg = cond & fall;
                    if (__builtin_popcount(reg) > 1) break;
                    int s = W;
                    for (int q = 0; q < W; ++q)
                        if (reg == (1u << qset[q])) s = q;
                    slot[b] = s;
                    ++b;
                }
                if (b - a < (size_t)kMinPhaseRun)
                    for (size_t c = a; c < b; ++c)
                        if (!outside(*gs[cur[c]])) slot[c] = -1;
                a = b == a ? a + 1 : b;
            }
        }
        // A gathered run emits one record per (slot, per-lane mask) with the
        // list of its gates' outside-tile conditions and phases (the factor
        // of the tile is the product of the phases whose condition holds),
        // then a flush.
        uint32_t pending = 0;
        std::vector<std::pair<std::pair<int, uint32_t>, std::vector<std::pair<uint64_t, std::array<double, 2>>>>>
            groups;
        const size_t entry_bytes = 8 + (f32 ? 8 : 16);
        const int max_entries = (int)(sizeof(TileGate::m) / entry_bytes);
        auto flush = [&]() {
            if (!pending) return;
            // groups conditioned on one lane bit and nothing outside the
            // tile: one SK_LPH record per slot lists (bit, phase) for all of
            // them, so the lanes walk one record instead of one per bit.
            // Complex64 passes carry them only when launched on the kernel
            // instances compiled with them (lph_f32, full sweep width): in
            // the common instance the extra record kind slowed the other
            // passes more than it saved
            std::vector<std::vector<std::pair<uint32_t, std::complex<double>>>> lph(W + 1);
            std::vector<char> in_lph(groups.size(), 0);
            const bool use_lph = !f32 || (lph_f32 && W == kSweepW);
            for (size_t gi = 0; gi < groups.size() && use_lph; ++gi) {
                const auto &grp = groups[gi];
                const uint32_t lm = grp.first.second;
                if (__builtin_popcount(lm) != 1) continue;
                bool inside = true;
                std::complex<double> ph = 1.0;
                for (const auto &e : grp.second) {
                    inside = inside && e.first == 0;
                    ph *= std::complex<double>(e.second[0], e.second[1]);
                }
                if (!inside) continue;
                lph[grp.first.first].push_back({lm, ph});
                in_lph[gi] = 1;
            }
            for (int slot_i = 0; slot_i <= W; ++slot_i) {
                const auto &ents = lph[slot_i];
                if (ents.size() < 2) { // a single bit stays an SK_PHASE record
                    for (size_t gi = 0; gi < groups.size(); ++gi)
                        if (in_lph[gi] && groups[gi].first.first == slot_i) in_lph[gi] = 0;
                    continue;
                }
                for (size_t e0 = 0; e0 < ents.size(); e0 += (size_t)max_entries) {
                    pc.lane_phases = true;
                    TileGate r{};
                    r.kind = SK_LPH;
                    r.b0 = slot_i;
                    r.amask = 1;
                    const size_t ne = std::min(ents.size() - e0, (size_t)max_entries);
                    r.b1 = (int32_t)ne;
                    char *dst = reinterpret_cast<char *>(r.m);
                    for (size_t e = 0; e < ne; ++e, dst += entry_bytes) {
                        const uint64_t lm = ents[e0 + e].first;
                        std::memcpy(dst, &lm, 8);
                        const std::complex<double> z = ents[e0 + e].second;
                        if (f32) {
                            const float f[2] = {(float)z.real(), (float)z.imag()};
                            std::memcpy(dst + 8, f, 8);
                        } else {
                            const double f[2] = {z.real(), z.imag()};
                            std::memcpy(dst + 8, f, 16);
                        }
                    }
                    pc.gates.push_back(r);
                    ++sw.n_gates;
                }
            }
            for (size_t gi = 0; gi < groups.size(); ++gi) {
                if (in_lph[gi]) continue;
                const auto &grp = groups[gi];
                std::vector<PhaseEntry> all, ents_l;
                for (const auto &e : grp.second) all.push_back({e.first, {e.second[0], e.second[1]}});
                std::vector<PhaseWindow> wins;
                phase_windows(all, &wins, &ents_l);
                // tables: kPtabWindows windows per record, their descriptors
                // in the kPtabDesc bytes after the head, then the entry 1 (unused
                // windows point at it) and the tables
                auto put = [f32](std::vector<char> &pl, std::complex<double> z) {
                    if (f32) {
                        const float f[2] = {(float)z.real(), (float)z.imag()};
                        pl.insert(pl.end(), reinterpret_cast<const char *>(f), reinterpret_cast<const char *>(f) + 8);
                    } else {
                        const double f[2] = {z.real(), z.imag()};
                        pl.insert(pl.end(), reinterpret_cast<const char *>(f),
                                  reinterpret_cast<const char *>(f) + 16);
                    }
                };
                for (size_t w0 = 0; w0 < wins.size(); w0 += (size_t)kPtabWindows) {
                    const size_t nw = std::min(wins.size() - w0, (size_t)kPtabWindows);
                    std::vector<char> pl(kPtabDesc, 0);
                    put(pl, 1.0);
                    for (size_t w = 0; w < nw; ++w) {
                        const PhaseWindow &pw = wins[w0 + w];
                        const uint32_t d[4] = {(uint32_t)pw.shift, (1u << pw.bits) - 1u,
                                               (uint32_t)(pl.size() - kPtabDesc), 0u};
                        std::memcpy(pl.data() + 16 * w, d, 16);
                        for (const auto &z : pw.tab) put(pl, z);
                    }
                    TileGate r{};
                    r.kind = SK_PTAB;
                    r.b0 = grp.first.first;
                    r.b1 = (int32_t)nw;
                    r.lane = grp.first.second;
                    r.amask = 1;
                    const uint64_t ti = pc.tables.size();
                    std::memcpy(r.m, &ti, 8);
                    pc.tables.push_back(std::move(pl));
                    pc.gates.push_back(r);
                    ++sw.n_gates;
                }
                std::vector<std::pair<uint64_t, std::array<double, 2>>> ents;
                for (const PhaseEntry &e : ents_l) ents.push_back({e.cond, {e.ph.real(), e.ph.imag()}});
                for (size_t e0 = 0; e0 < ents.size(); e0 += (size_t)max_entries) {
                    TileGate r{};
                    r.kind = SK_PHASE;
                    r.b0 = grp.first.first;
                    r.lane = grp.first.second;
                    r.amask = 1;
                    const size_t ne = std::min(ents.size() - e0, (size_t)max_entries);
                    r.b1 = (int32_t)ne;
                    char *dst = reinterpret_cast<char *>(r.m);
                    for (size_t e = 0; e < ne; ++e, dst += entry_bytes) {
                        std::memcpy(dst, &ents[e0 + e].first, 8);
                        const double *ph = ents[e0 + e].second.data();
                        if (f32) {
                            const float f[2] = {(float)ph[0], (float)ph[1]};
                            std::memcpy(dst + 8, f, 8);
                        } else {
                            std::memcpy(dst + 8, ph, 16);
                        }
                    }
                    pc.gates.push_back(r);
                    ++sw.n_gates;
                }
            }
            groups.clear();
            TileGate r{};
            r.kind = SK_FLUSH;
            r.amask = pending;
            pc.gates.push_back(r);
            ++sw.n_gates;
            pending = 0;
        };
        for (size_t ci = 0; ci < cur.size(); ++ci) {
            const size_t i = cur[ci];
            if (slot[ci] >= 0) {
                const Gate &g = *gs[i];
                TileGate r{};
                const int lt = local_bit(sp, g.t[0]);
                const uint32_t cond = encode_controls(sp, g.ctrl, &r) | (lt >= 0 ? 1u << lt : 0u);
                const std::pair<int, uint32_t> key{slot[ci], cond & ~fall};
                auto it = std::find_if(groups.begin(), groups.end(), [&](const auto &x) { return x.first == key; });
                if (it == groups.end()) {
                    groups.push_back({key, {}});
                    it = groups.end() - 1;
                }
                if (lt >= 0) {
                    it->second.push_back({r.cout, {g.U[6], g.U[7]}});
                } else {
                    // target outside the tile: diag(d0, d1) = d0 on the
                    // condition, times d1 / d0 where the target is 1
                    const std::complex<double> d0{g.U[0], g.U[1]}, d1{g.U[6], g.U[7]};
                    if (!is_one(g.U)) it->second.push_back({r.cout, {d0.real(), d0.imag()}});
                    const std::complex<double> q = is_one(g.U) ? d1 : d1 / d0;
                    it->second.push_back({r.cout | (1ull << g.t[0]), {q.real(), q.imag()}});
                }
                pending |= 1u << slot[ci];
                pc.flops_per_amp += gate_flops_per_amp(g);
                continue;
            }
            flush();
            if (const Probe *pr = probe_of(i)) {
                pc.gates.push_back(encode_probe(sp, qset, *gs[i], *pr, f32));
                ++sw.n_gates;
                // probe: Im<lam|M|psi> over the gate's pairs, 8 flops per amplitude
                pc.flops_per_amp += 8.0 / (double)(1ull << __builtin_popcountll(gs[i]->ctrl));
            }
            pc.gates.push_back(encode_sweep_gate(sp, qset, *gs[i], f32));
            pc.two_qubit = pc.two_qubit || pc.gates.back().kind == SK_2Q;
            ++sw.n_gates;
            pc.flops_per_amp += (probes ? 2.0 : 1.0) * gate_flops_per_amp(*gs[i]);
        }
        flush();
        for (int j = 0; j < kSweepW; ++j) sw.qpos[j] = j < W ? qset[j] : 0;
        pc.sweeps.push_back(sw);
        cur.clear();
        qset.clear();
    };
    // Each sweep takes the gates, in order, whose targets fit its register
    // set, and also looks past a gate that does not fit: a later gate may
    // join the sweep if it shares no qubit with any gate left behind (gates
    // on disjoint qubits commute; a probe's value is unchanged by moving a
    // gate on other qubits across it, since that gate and its inverse cancel
    // around the probe's Pauli).  Fewer sweeps mean fewer exchanges of the
    // tile through LDS.
    std::vector<char> done(gs.size(), 0);
    size_t first = 0;
    while (first < gs.size()) {
        uint64_t blocked = 0; // qubits of the gates left behind by this sweep
        for (size_t i = first; i < gs.size(); ++i) {
            if (done[i]) continue;
            const Gate *g = gs[i];
            const uint64_t qm = g->qmask();
            if (qm & blocked) {
                blocked |= qm;
                continue;
            }
            if (is_diag1(*g) && !probe_of(i)) {
                cur.push_back(i);
                done[i] = 1;
                continue;
            }
            std::vector<int> need;
            for (int j = 0; j < g->k; ++j) {
                const int lb = local_bit(sp, g->t[j]);
                if (std::find(qset.begin(), qset.end(), lb) == qset.end()) need.push_back(lb);
            }
            if ((int)(qset.size() + need.size()) > W) {
                blocked |= qm;
                continue;
            }
            qset.insert(qset.end(), need.begin(), need.end());
            cur.push_back(i);
            done[i] = 1;
        }
        // the first open gate fits an empty register set whenever W >= k;
        // should it not, it still gets a sweep of its own (the loop ends)
        if (cur.empty() && !done[first]) {
            for (int j = 0; j < gs[first]->k; ++j) qset.push_back(local_bit(sp, gs[first]->t[j]));
            cur.push_back(first);
            done[first] = 1;
        }
        close();
        while (first < gs.size() && done[first]) ++first;
    }
    pack_records(pc, f32);
    // the first and last sweeps read / write the state directly (measured
    // faster than staging the tile through LDS for every register layout,
    // most when the register positions leave the low tile bits to the lanes)
    pc.direct = kDirectFirst | kDirectLast;
    return pc;
}

// Write a compiled pass into the host arena at 'off' (256-aligned).
static void stage_pass(sv_state *h, const PassCode &pc, size_t off) {
    std::memcpy(h->h_arena + off, pc.sweeps.data(), pc.sweeps.size() * sizeof(TileSweep));
    std::memcpy(h->h_arena + off + align256(pc.sweeps.size() * sizeof(TileSweep)), pc.recs.data(),
                pc.recs.size());
}

static int launch_pass(sv_state *h, const PassCode &pc, size_t off) {
    const TileSweep *sw = reinterpret_cast<const TileSweep *>(h->d_arena + off);
    const char *gt = h->d_arena + off + align256(pc.sweeps.size() * sizeof(TileSweep));
    Timed tm(h, K_TILE, 2.0 * state_bytes(h), pc.flops_per_amp * (double)(1ull << h->n));
    SV_HIP(launch_tile(h->amps, h->n, h->dtype, pc.sp, sw, (int)pc.sweeps.size(), gt, pc.two_qubit, pc.lane_phases,
                       pc.direct, h->stream));
    return SV_OK;
}

static int tile_single(sv_state *h, const Gate &g) {
    TileSpec sp{};
    tile_layout(h->n, std::min(h->n, tile_max_qubits(h->dtype)), std::min(h->n, 6), g.tmask(), &sp);
    std::vector<const Gate *> one{&g};
    const PassCode pc = compile_pass(sp, one, sweep_width(h->dtype), h->dtype == SV_C64);
    int rc = ensure_arena(h, pc.bytes());
    if (rc) return rc;
    if ((rc = stage_wait(h))) return rc;
    stage_pass(h, pc, 0);
    if ((rc = upload_arena(h, pc.bytes()))) return rc;
    return launch_pass(h, pc, 0);
}

// Greedy, commutation-aware grouping: scan the unscheduled gates in order;
// a gate joins the current pass if it does not touch a qubit of an earlier
// gate left behind, and its targets fit in the tile (low block plus at most
// kmax further qubits).  Gates left behind block their qubits for the rest
// of the scan, so every pair of gates sharing a qubit keeps its order.
// Gates a pass with tile qubits S would take, in order: a gate joins if it
// shares no qubit with a gate left behind and S holds the qubits it needs.
static int pass_gates(const std::vector<uint64_t> &tm, const std::vector<uint64_t> &qm, uint64_t all,
                      const std::vector<char> &done, size_t first, uint64_t S, Pass *take) {
    uint64_t blocked = 0;
    int cnt = 0;
    for (size_t i = first; i < tm.size(); ++i) {
        if (done[i]) continue;
        if ((qm[i] & blocked) || (tm[i] & ~S)) {
            blocked |= qm[i];
            if (blocked == all) break; // every later gate shares a qubit with one left behind
            continue;
        }
        ++cnt;
        if (take) take->gates.push_back((int)i);
    }
    return cnt;
}

// Greedy tile set: the qubits beyond the low block are taken in the order
// the gates first need them, while they fit.
static uint64_t greedy_tile_set(const std::vector<uint64_t> &tm, const std::vector<uint64_t> &qm, uint64_t all,
                                const std::vector<char> &done, size_t first, uint64_t low, int kmax) {
    uint64_t S = low, blocked = 0;
    int used = 0;
    for (size_t i = first; i < tm.size() && blocked != all; ++i) {
        if (done[i]) continue;
        if (qm[i] & blocked) {
            blocked |= qm[i];
            continue;
        }
        const uint64_t need = tm[i] & ~S;
        const int nn = __builtin_popcountll(need);
        if (used + nn <= kmax) {
            S |= need;
            used += nn;
        } else {
            blocked |= qm[i];
        }
    }
    return S;
}

// Lookahead tile set: the qubits beyond the low block are added one at a
// time, among those needed by the first gates that do not fit yet (at most
// 12 candidates), each time the one that lets the pass take the most gates;
// the first addition takes the candidate of rank 'rank' instead of the best.
// *count receives the gates the pass takes.
static uint64_t lookahead_tile_set(const std::vector<uint64_t> &tm, const std::vector<uint64_t> &qm, uint64_t all,
                                   const std::vector<char> &done, size_t first, uint64_t low, int kmax, int rank,
                                   int *count) {
    uint64_t S = low;
    int c = pass_gates(tm, qm, all, done, first, S, nullptr);
    std::vector<std::pair<int, uint64_t>> sc;
    for (int used = 0; used < kmax; ++used) {
        uint64_t cand = 0, blocked = 0;
        for (size_t i = first; i < tm.size() && __builtin_popcountll(cand) < 12 && blocked != all; ++i) {
            if (done[i]) continue;
            if (qm[i] & blocked) {
                blocked |= qm[i];
                continue;
            }
            if (tm[i] & ~S) {
                cand |= tm[i] & ~S;
                blocked |= qm[i];
            }
        }
        sc.clear();
        for (uint64_t cc = cand; cc; cc &= cc - 1) {
            const uint64_t q = cc & (~cc + 1);
            sc.push_back({pass_gates(tm, qm, all, done, first, S | q, nullptr), q});
        }
        std::sort(sc.begin(), sc.end(), [](const std::pair<int, uint64_t> &x, const std::pair<int, uint64_t> &y) {
            return x.first > y.first || (x.first == y.first && x.second < y.second);
        });
        const size_t pick = used == 0 ? (size_t)rank : 0;
        if (sc.size() <= pick || sc[pick].first <= c) break;
        S |= sc[pick].second;
        c = sc[pick].first;
    }
    *count = c;
    return S;
}

// Commutation-aware pass scheduler.  Every pass holds the low lmin qubits
// and up to mmax - lmin others.  Level 0 (greedy): the others are taken in
// the order the gates first need them.  Level 1: the pass takes the greedy
// set or the lookahead set, whichever takes more gates.  Level 2: the pass's
// tile set is chosen among the greedy set and kLookRanks lookahead sets (the
// best first addition and the next best ones) by the gates this pass and the
// next one would take together (the next pass chosen as at level 1).  On the
// random circuits of the benchmark: 48 -> 39 -> 33 passes at 32 qubits,
// 36 -> 31 -> 28 at 30 qubits; level 2 costs about six times the host time
// of level 1 (about 11 ms for the 32-qubit circuit).  The scans stop once
// every qubit is blocked by a gate left behind.
constexpr int kLookRanks = 9;
static std::vector<Pass> schedule_masks(const std::vector<uint64_t> &tm, const std::vector<uint64_t> &qm,
                                        int mmax, int lmin, int lookahead = 0) {
    std::vector<Pass> passes;
    std::vector<char> done(tm.size(), 0);
    size_t first = 0;
    const uint64_t low = lmin >= 64 ? ~0ull : ((1ull << lmin) - 1ull);
    const int kmax = std::max(0, mmax - lmin);
    uint64_t all = 0; // every qubit some gate touches
    for (uint64_t m : qm) all |= m;
    auto next_first = [&](const std::vector<char> &d, size_t f) {
        while (f < tm.size() && d[f]) ++f;
        return f;
    };
    while (first < tm.size()) {
        uint64_t S = greedy_tile_set(tm, qm, all, done, first, low, kmax);
        if (lookahead == 1) {
            int cl;
            const uint64_t Sl = lookahead_tile_set(tm, qm, all, done, first, low, kmax, 0, &cl);
            if (cl >= pass_gates(tm, qm, all, done, first, S, nullptr)) S = Sl;
        } else if (lookahead >= 2) {
            std::vector<uint64_t> cands = {S};
            for (int r = 0; r < kLookRanks; ++r) {
                int c;
                const uint64_t Sr = lookahead_tile_set(tm, qm, all, done, first, low, kmax, r, &c);
                if (std::find(cands.begin(), cands.end(), Sr) == cands.end()) cands.push_back(Sr);
            }
            int best = -1;
            std::vector<char> d2;
            for (uint64_t Sc : cands) {
                Pass p;
                const int c1 = pass_gates(tm, qm, all, done, first, Sc, &p);
                d2 = done;
                for (int gi : p.gates) d2[(size_t)gi] = 1;
                const size_t f2 = next_first(d2, first);
                int c2 = 0;
                if (f2 < tm.size()) {
                    int cl;
                    lookahead_tile_set(tm, qm, all, d2, f2, low, kmax, 0, &cl);
                    const int cg = pass_gates(tm, qm, all, d2, f2, greedy_tile_set(tm, qm, all, d2, f2, low, kmax), nullptr);
                    c2 = std::max(cl, cg);
                }
                if (c1 + c2 > best) {
                    best = c1 + c2;
                    S = Sc;
                }
            }
        }
        Pass p;
        p.S = S;
        pass_gates(tm, qm, all, done, first, S, &p);
        for (int gi : p.gates) done[(size_t)gi] = 1;
        passes.push_back(std::move(p));
        first = next_first(done, first);
    }
    return passes;
}

// Tile qubits a gate of a plain tile pass needs: its targets, except for
// phase gates diag(1, e^{i phi}) with any controls (symmetric in their
// qubits: the target can be any of them, and with none in the tile the
// factor is uniform per tile) and uncontrolled one-qubit diagonal gates
// (uniform per tile for each value of the target), which need none.
static uint64_t tile_need(const Gate &g) {
    if (is_diag1(g) && (is_one(g.U) || g.ctrl == 0)) return 0;
    return g.tmask();
}

// outside_diag: let the gates tile_need exempts leave their targets out of
// the tile (sv_run's passes; the batch and adjoint passes keep every target
// in the tile).
static std::vector<Pass> schedule(const std::vector<Gate> &gs, int n, int mmax, int lmin,
                                  bool outside_diag = false, int lookahead = 0) {
    (void)n;
    std::vector<uint64_t> tm(gs.size()), qm(gs.size());
    for (size_t i = 0; i < gs.size(); ++i) {
        tm[i] = outside_diag ? tile_need(gs[i]) : gs[i].tmask();
        qm[i] = gs[i].qmask();
    }
    return schedule_masks(tm, qm, mmax, lmin, lookahead);
}

// Scheduler level for a state: the passes of larger states cost more GPU
// time, so they get the more thorough (and slower) lookahead; small states
// keep the greedy schedule, whose host time is a few microseconds per pass.
static int lookahead_level_for(int n, int dtype) {
    const double b = std::ldexp(dtype == SV_C64 ? 8.0 : 16.0, n);
    return b >= 4.0 * (1ull << 30) ? 2 : (b >= 256.0 * (1ull << 20) ? 1 : 0);
}
static int lookahead_level(const sv_state *h) { return lookahead_level_for(h->n, h->dtype); }

// A phase gate of a pass with its target outside the tile and a control
// inside: the same gate with that control as the target (the gate is
// symmetric in its qubits), so that only phase gates with no qubit in the
// tile keep an outside target.
static Gate retarget_phase(const Gate &g, uint64_t S) {
    Gate r = g;
    const uint64_t in = g.ctrl & S;
    if (is_diag1(g) && is_one(g.U) && !((S >> g.t[0]) & 1ull) && in) {
        const int t = __builtin_ctzll(in);
        r.ctrl = (g.ctrl | (1ull << g.t[0])) & ~(1ull << t);
        r.t[0] = t;
    }
    return r;
}

// A single gate that the streamed kernels cannot take: a two-qubit gate with
// a target inside a 16-byte complex64 vector.
static bool needs_tile(int dtype, const Gate &g) {
    const int vb = vbits_of(dtype);
    return g.k == 2 && (g.t[0] < vb || g.t[1] < vb);
}

// Tile size and low block of sv_run's plain passes: runs of 128 complex64 /
// 64 complex128 amplitudes (shorter runs cut the number of passes but cost
// more per pass, measured).
static int plain_tile_qubits(int n, int dtype) { return std::min(n, tile_max_qubits(dtype)); }
static int plain_low_qubits(int n, int dtype) { return std::min(n, dtype == SV_C64 ? 7 : 6); }

static int run_gates(sv_state *h, const std::vector<Gate> &gs, int mode) {
    if (mode == SV_RUN_PER_GATE) {
        for (const Gate &g : gs) {
            const int rc = apply_one(h, g);
            if (rc) return rc;
        }
        return SV_OK;
    }
    const int mmax = plain_tile_qubits(h->n, h->dtype), lmin = plain_low_qubits(h->n, h->dtype);
    std::vector<Pass> passes = schedule(gs, h->n, mmax, lmin, true, lookahead_level(h));
    // compile every tiled pass, stage all of them, upload once, launch in order
    std::vector<PassCode> code(passes.size());
    std::vector<size_t> offs(passes.size(), 0);
    std::vector<char> tiled(passes.size(), 0);
    size_t total = 0;
    for (size_t pi = 0; pi < passes.size(); ++pi) {
        const Pass &p = passes[pi];
        tiled[pi] = p.gates.size() > 1 || (p.gates.size() == 1 && needs_tile(h->dtype, gs[p.gates[0]]));
        if (!tiled[pi]) continue;
        uint64_t needed = 0;
        for (int gi : p.gates) needed |= tile_need(gs[gi]);
        TileSpec sp{};
        tile_layout(h->n, mmax, lmin, needed, &sp);
        std::vector<Gate> local;
        local.reserve(p.gates.size());
        for (int gi : p.gates) local.push_back(retarget_phase(gs[gi], tile_qubits(sp)));
        std::vector<const Gate *> ptrs;
        for (const Gate &g : local) ptrs.push_back(&g);
        code[pi] = compile_pass(sp, ptrs, sweep_width(h->dtype), h->dtype == SV_C64, nullptr, true);
        offs[pi] = total;
        total += align256(code[pi].bytes());
    }
    if (total) {
        int rc = ensure_arena(h, total);
        if (rc) return rc;
        if ((rc = stage_wait(h))) return rc;
        for (size_t pi = 0; pi < passes.size(); ++pi)
            if (tiled[pi]) stage_pass(h, code[pi], offs[pi]);
        if ((rc = upload_arena(h, total))) return rc;
    }
    for (size_t pi = 0; pi < passes.size(); ++pi) {
        const Pass &p = passes[pi];
        if (p.gates.empty()) continue;
        const int rc = tiled[pi] ? launch_pass(h, code[pi], offs[pi]) : apply_one(h, gs[p.gates[0]]);
        if (rc) return rc;
    }
    return SV_OK;
}


// ================================================================ fusion
// A dense block: qubits ascending (bit j of the matrix index <-> q[j]) and its
// 2^k x 2^k matrix, row-major, FP64.
// In a fused tile pass a block may also depend on qubits outside the tile
// (vmask, at most kMaxVariantQubits): the diagonal gates fused into it reduce,
// for each value v of those qubits, to diagonals on the block's own qubits,
// and var[v] is the block's matrix for that value (bit i of v = the i-th
// lowest qubit of vmask).
struct Block {
    int k = 0;
    int q[5] = {0, 0, 0, 0, 0};
    std::vector<std::complex<double>> M;
    int n_gates = 0;
    uint64_t vmask = 0;
    std::vector<std::vector<std::complex<double>>> var;
};

// Left-multiply M (a matrix on the block's qubits) by gate g embedded in
// them: each column of M is a 2^k-amplitude vector and g acts on it as on a
// state.
static void absorb_into(const Block &b, std::vector<std::complex<double>> &M, const Gate &g) {
    const int D = 1 << b.k;
    auto local = [&](int q) {
        for (int j = 0; j < b.k; ++j)
            if (b.q[j] == q) return j;
        return -1;
    };
    uint32_t lctrl = 0;
    for (uint64_t c = g.ctrl; c; c &= c - 1) lctrl |= 1u << local(__builtin_ctzll(c));
    std::complex<double> G[16];
    for (int i = 0; i < (1 << (2 * g.k)); ++i) G[i] = {g.U[2 * i], g.U[2 * i + 1]};
    if (g.k == 1) {
        const int t = local(g.t[0]);
        for (int a = 0; a < D; ++a) {
            if ((a >> t) & 1) continue;
            if (((uint32_t)a & lctrl) != lctrl) continue;
            const int c = a | (1 << t);
            for (int col = 0; col < D; ++col) {
                const std::complex<double> x0 = M[(size_t)a * D + col], x1 = M[(size_t)c * D + col];
                M[(size_t)a * D + col] = G[0] * x0 + G[1] * x1;
                M[(size_t)c * D + col] = G[2] * x0 + G[3] * x1;
            }
        }
    } else {
        const int t0 = local(g.t[0]), t1 = local(g.t[1]);
        for (int a = 0; a < D; ++a) {
            if (((a >> t0) & 1) || ((a >> t1) & 1)) continue;
            if (((uint32_t)a & lctrl) != lctrl) continue;
            const int idx[4] = {a, a | (1 << t0), a | (1 << t1), a | (1 << t0) | (1 << t1)};
            for (int col = 0; col < D; ++col) {
                std::complex<double> x[4], y[4];
                for (int r = 0; r < 4; ++r) x[r] = M[(size_t)idx[r] * D + col];
                for (int r = 0; r < 4; ++r) {
                    y[r] = 0;
                    for (int c = 0; c < 4; ++c) y[r] += G[4 * r + c] * x[c];
                }
                for (int r = 0; r < 4; ++r) M[(size_t)idx[r] * D + col] = y[r];
            }
        }
    }
}

static void absorb(Block &b, const Gate &g) {
    absorb_into(b, b.M, g);
    b.n_gates += 1;
}

// Whether g's matrix is diagonal (then g multiplies each basis state by a
// phase and commutes with every other diagonal gate).
static bool is_diag_gate(const Gate &g) {
    const int D = 1 << g.k;
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c)
            if (r != c && !is_zero(g.U + 2 * (r * D + c))) return false;
    return true;
}

// Left-multiply M by the diagonal gate g with the block's outside qubits
// (vmask) fixed to variant v: basis state a of the block's qubits is scaled
// by g's diagonal entry at the targets' values when all controls are 1.
static void absorb_phase(const Block &b, std::vector<std::complex<double>> &M, const Gate &g, uint32_t v) {
    const int D = 1 << b.k;
    auto value = [&](int q, int a) -> uint32_t {
        for (int j = 0; j < b.k; ++j)
            if (b.q[j] == q) return ((uint32_t)a >> j) & 1u;
        const int rank = __builtin_popcountll(b.vmask & ((1ull << q) - 1ull));
        return (v >> rank) & 1u;
    };
    const int Dg = 1 << g.k;
    for (int a = 0; a < D; ++a) {
        bool on = true;
        for (uint64_t c = g.ctrl; c; c &= c - 1) on = on && value(__builtin_ctzll(c), a);
        if (!on) continue;
        const uint32_t r = value(g.t[0], a) | (g.k == 2 ? value(g.t[1], a) << 1 : 0u);
        const std::complex<double> d{g.U[2 * (r * Dg + r)], g.U[2 * (r * Dg + r) + 1]};
        for (int col = 0; col < D; ++col) M[(size_t)a * D + col] *= d;
    }
}

// Commutation-aware greedy fusion: scan the unplaced gates in order; a gate
// joins the open block if it touches no qubit of a gate left behind earlier
// in the scan and the block's qubit set (targets and controls) stays within
// k_max; otherwise its qubits are blocked for the rest of the scan.  Gates
// that share a qubit therefore keep their relative order.
static std::vector<Block> fuse(const std::vector<Gate> &gs, int k_max) {
    std::vector<Block> out;
    std::vector<char> done(gs.size(), 0);
    size_t first = 0;
    while (first < gs.size()) {
        uint64_t set = 0, blocked = 0;
        std::vector<int> members;
        for (size_t i = first; i < gs.size(); ++i) {
            if (done[i]) continue;
            const uint64_t gq = gs[i].qmask();
            if (gq & blocked) {
                blocked |= gq;
                continue;
            }
            if (__builtin_popcountll(set | gq) <= k_max) {
                set |= gq;
                members.push_back((int)i);
                done[i] = 1;
            } else {
                blocked |= gq;
            }
        }
        Block b;
        for (uint64_t m = set; m; m &= m - 1) b.q[b.k++] = __builtin_ctzll(m);
        const int D = 1 << b.k;
        b.M.assign((size_t)D * D, 0.0);
        for (int i = 0; i < D; ++i) b.M[(size_t)i * D + i] = 1.0;
        for (int gi : members) absorb(b, gs[gi]);
        out.push_back(std::move(b));
        while (first < gs.size() && done[first]) ++first;
    }
    return out;
}

// Fusion of one tile pass's gates, the tile holding qubits S.  Every qubit
// of a non-diagonal gate is in the tile; a diagonal gate may also act on
// qubits outside it, which no other gate of the pass touches except other
// diagonal gates (all of which commute), so only a gate's qubits inside the
// tile order it against the others and count towards k_max.  Its qubits
// outside the tile join the block's variant qubits (at most
// kMaxVariantQubits; the scheduler lets only diagonal gates of at most that
// many qubits leave the tile).
static std::vector<Block> fuse_tile(const std::vector<Gate> &gs, int k_max, uint64_t S) {
    std::vector<Block> out;
    std::vector<char> done(gs.size(), 0);
    size_t first = 0;
    while (first < gs.size()) {
        uint64_t set = 0, vset = 0, blocked = 0;
        std::vector<int> members;
        for (size_t i = first; i < gs.size(); ++i) {
            if (done[i]) continue;
            const uint64_t gin = gs[i].qmask() & S, gout = gs[i].qmask() & ~S;
            if (gin & blocked) {
                blocked |= gin;
                continue;
            }
            if (__builtin_popcountll(set | gin) <= k_max && __builtin_popcountll(vset | gout) <= kMaxVariantQubits) {
                set |= gin;
                vset |= gout;
                members.push_back((int)i);
                done[i] = 1;
            } else {
                blocked |= gin;
            }
        }
        Block b;
        for (uint64_t m = set; m; m &= m - 1) b.q[b.k++] = __builtin_ctzll(m);
        b.vmask = vset;
        const int D = 1 << b.k;
        std::vector<std::complex<double>> I((size_t)D * D, 0.0);
        for (int i = 0; i < D; ++i) I[(size_t)i * D + i] = 1.0;
        b.var.assign((size_t)1 << __builtin_popcountll(vset), I);
        for (uint32_t v = 0; v < b.var.size(); ++v)
            for (int gi : members) {
                if (gs[gi].qmask() & ~S) absorb_phase(b, b.var[v], gs[gi], v);
                else absorb_into(b, b.var[v], gs[gi]);
            }
        b.n_gates = (int)members.size();
        out.push_back(std::move(b));
        while (first < gs.size() && done[first]) ++first;
    }
    return out;
}

// ---------------------------------------------- MFMA operand fragments
static uint16_t bf16_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u); // round to nearest even (finite inputs)
    return (uint16_t)(u >> 16);
}
static float bf16_value(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// B operand of the two real GEMMs (K_total = 2D rows, D columns):
//   part 0 (Re Y): rows [0,D) Re U^T, rows [D,2D) -Im U^T
//   part 1 (Im Y): rows [0,D) Im U^T, rows [D,2D)  Re U^T
static float bpart(const std::complex<double> *U, int D, int part, int krow, int col) {
    const bool top = krow < D;
    const std::complex<double> u = U[(size_t)col * D + (top ? krow : krow - D)];
    if (part == 0) return (float)(top ? u.real() : -u.imag());
    return (float)(top ? u.imag() : u.real());
}

// Bytes of the fragment buffer for (k, prec).
static size_t frag_bytes(int k, int prec) {
    if (prec == SV_PREC_FP32) return (size_t)2 * (k == 5 ? 32 : 8) * 64 * 4;
    return (size_t)2 * (k == 5 ? 4 : 1) * 2 * 64 * 16;
}

// Split-BF16 orders the K rows (amplitude, re/im) interleaved: row 2a + c
// multiplies component c of amplitude a.
static float bpart_interleaved(const std::complex<double> *U, int D, int part, int krow, int col) {
    const std::complex<double> u = U[(size_t)col * D + (krow >> 1)];
    const bool re = (krow & 1) == 0;
    if (part == 0) return (float)(re ? u.real() : -u.imag());
    return (float)(re ? u.imag() : u.real());
}

// Lay out U in the per-lane order the MFMA kernels load (see k_fused.hip).
static void make_fragments(const std::complex<double> *U, int k, int prec, char *out) {
    const int D = 1 << k;
    if (prec == SV_PREC_FP32) {
        float *f = reinterpret_cast<float *>(out);
        const int rows = k == 5 ? 32 : 16, per = k == 5 ? 2 : 4, KS = 2 * D / per;
        for (int p = 0; p < 2; ++p)
            for (int st = 0; st < KS; ++st)
                for (int lane = 0; lane < 64; ++lane)
                    f[(p * KS + st) * 64 + lane] =
                        bpart(U, D, p, per * st + lane / rows, lane % rows);
    } else {
        uint16_t *f = reinterpret_cast<uint16_t *>(out);
        const int rows = k == 5 ? 32 : 16, KS = k == 5 ? 4 : 1;
        for (int p = 0; p < 2; ++p)
            for (int st = 0; st < KS; ++st)
                for (int lane = 0; lane < 64; ++lane)
                    for (int e = 0; e < 8; ++e) {
                        const int krow = (512 / rows) * st + 8 * (lane / rows) + e;
                        const float x = bpart_interleaved(U, D, p, krow, lane % rows);
                        const uint16_t hi = bf16_bits(x);
                        const uint16_t lo = bf16_bits(x - bf16_value(hi));
                        f[(((p * KS + st) * 2 + 0) * 64 + lane) * 8 + e] = hi;
                        f[(((p * KS + st) * 2 + 1) * 64 + lane) * 8 + e] = lo;
                    }
    }
}

// FP64 MFMA operand (complex128 blocks): frag[((p * NT + nt) * KS + s) * 64 + lane]
// = B_p[4s + lane/16][16nt + lane%16], NT = D/16, KS = D/2.
static size_t frag64_bytes(int k) {
    const int D = 1 << k;
    return (size_t)2 * (D / 16) * (D / 2) * 64 * sizeof(double);
}

static void make_fragments64(const std::complex<double> *U, int k, char *out) {
    const int D = 1 << k, NT = D / 16, KS = D / 2;
    double *f = reinterpret_cast<double *>(out);
    for (int p = 0; p < 2; ++p)
        for (int nt = 0; nt < NT; ++nt)
            for (int st = 0; st < KS; ++st)
                for (int lane = 0; lane < 64; ++lane) {
                    const int krow = 4 * st + lane / 16, col = 16 * nt + lane % 16;
                    const bool top = krow < D;
                    const std::complex<double> u = U[(size_t)col * D + (top ? krow : krow - D)];
                    const double val = p == 0 ? (top ? u.real() : -u.imag()) : (top ? u.imag() : u.real());
                    f[((p * NT + nt) * KS + st) * 64 + lane] = val;
                }
}

static bool mfma64_ok(const sv_state *h, int k) {
    if (h->dtype != SV_C128 || (k != 4 && k != 5)) return false;
    const int m = std::min(h->n, fused_tile_qubits(h->dtype));
    return m >= k && ((1u << m) >> k) % 16 == 0;
}

// Whether a k-qubit MFMA block can run on this state (whole wave-tiles).
static bool mfma_ok(const sv_state *h, int k, int prec) {
    if (prec == SV_PREC_NATIVE || h->dtype != SV_C64 || (k != 4 && k != 5)) return false;
    const int m = std::min(h->n, fused_tile_qubits(h->dtype));
    const int rows = k == 5 ? 32 : 16;
    return m >= k && ((1u << m) >> k) % rows == 0;
}

// A fused tile pass: the tile layout, the uniform block width k of its
// blocks (narrower blocks are padded with identity qubits), whether it runs
// on the matrix cores, and its blocks' positions and padded matrices.
struct FusedPass {
    // a pass of the fused path runs either its dense blocks on the matrix
    // cores (below) or, where the cost model prefers it, its gates as plain
    // register sweeps on the same tile (k_tile, 'code')
    bool plain = false;
    PassCode code;
    double cost = 0.0; // modelled time, ms per 2^30 amplitudes
    TileSpec sp{};
    int m = 0;
    double flops_per_amp = 0.0; // 8 * 2^k per block of k qubits (complex matvec as real flops)
    int k = 0;
    int engine = SV_PREC_NATIVE;
    uint32_t direct = 0; // kDirectFirst / kDirectLast (matrix cores)
    std::vector<DenseBlock> blocks;
    // per block, its padded matrix for each variant of its outside qubits
    std::vector<std::vector<std::vector<std::complex<double>>>> mats;
};

// engine: the launch_dense_pass precision code of a pass (SV_PREC_NATIVE =
// vector ALUs, SV_PREC_FP32 / SV_PREC_SPLIT_BF16 = complex64 matrix cores,
// kPrecMfma64 = complex128 on the FP64 matrix cores).
static bool is_mfma(int engine) { return engine != SV_PREC_NATIVE; }

static size_t dense_frag_bytes(const sv_state *h, int k, int engine) {
    if (engine == kPrecMfma64) return align256(frag64_bytes(k));
    if (engine != SV_PREC_NATIVE) return align256(frag_bytes(k, engine));
    return align256(((size_t)1 << (2 * k)) * (h->dtype == SV_C64 ? 8 : 16));
}

// MFMA rows (groups per wave-tile) of an engine at block width k
static int mfma_rows(int k, int engine) { return engine == kPrecMfma64 ? 16 : (k == 5 ? 32 : 16); }

// operand plus, for the matrix cores, the LDS offset tables
// (qoff[2^k], goff_lo[rows], goff_hi[2^(m-k) / rows]) and the same tables of
// global offsets
static size_t dense_tab_entries(int k, int m, int engine) {
    const size_t rows = (size_t)mfma_rows(k, engine);
    return ((size_t)1 << k) + rows + (((size_t)1 << (m - k)) / rows);
}
static size_t dense_op_bytes(const sv_state *h, int k, int m, int engine, size_t n_variants) {
    size_t b = n_variants * dense_frag_bytes(h, k, engine);
    if (is_mfma(engine)) {
        b += align256(dense_tab_entries(k, m, engine) * sizeof(uint32_t));
        b += align256(dense_tab_entries(k, m, engine) * sizeof(uint64_t));
    }
    return b;
}

// Global index offset (from the tile's base) of local tile index l.
static uint64_t tile_global_offset(const TileSpec &sp, uint32_t l) {
    uint64_t g = l & ((1u << sp.L) - 1u);
    for (int i = 0; i < sp.K; ++i)
        if ((l >> (sp.L + i)) & 1u) g |= 1ull << sp.high[i];
    return g;
}

static size_t fused_pass_bytes(const sv_state *h, const FusedPass &fp) {
    if (fp.plain) return fp.code.bytes();
    size_t b = align256(fp.blocks.size() * sizeof(DenseBlock));
    for (const auto &vs : fp.mats) b += dense_op_bytes(h, fp.k, fp.m, fp.engine, vs.size());
    return b;
}

// Embed a k-qubit matrix in K qubits (extra index bits k..K-1 act as identity).
static std::vector<std::complex<double>> pad_matrix(const std::vector<std::complex<double>> &M, int k, int K) {
    const int d = 1 << k, D = 1 << K;
    std::vector<std::complex<double>> P((size_t)D * D, 0.0);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c)
            if ((r >> k) == (c >> k)) P[(size_t)r * D + c] = M[(size_t)(r & (d - 1)) * d + (c & (d - 1))];
    return P;
}

// Shortest contiguous run (low tile qubits) of a fused pass: 32 amplitudes
// (256 bytes complex64, 512 complex128).  A fused pass needs every qubit of
// a non-diagonal gate in its tile, so short runs leave room for more of
// them: the 30-qubit depth-40 CZ circuit takes 31 passes with these runs,
// 33 and 38 with runs of 64 and 128.
static int fused_lmin(const sv_state *h) { return std::min(h->n, 5); }

// One fused pass over the blocks bs[idx] in the tile layout sp (which holds
// all their qubits).  Blocks run on the matrix cores in the requested
// precision (the state's own for SV_PREC_NATIVE) whenever the tile holds
// whole wave-tiles; narrower blocks are then padded to 4 qubits.
static FusedPass build_fused_pass(const sv_state *h, const TileSpec &sp, const std::vector<Block> &bs,
                                  const std::vector<int> &idx, int prec) {
    FusedPass fp;
    int kmax = 1;
    for (int bi : idx) kmax = std::max(kmax, bs[bi].k);
    fp.sp = sp;
    fp.m = fp.sp.L + fp.sp.K;
    const int K = std::max(4, kmax);
    if (h->dtype == SV_C64) {
        const int p32 = prec == SV_PREC_NATIVE ? SV_PREC_FP32 : prec;
        fp.engine = mfma_ok(h, K, p32) ? p32 : SV_PREC_NATIVE;
    } else {
        fp.engine = mfma64_ok(h, K) ? kPrecMfma64 : SV_PREC_NATIVE;
    }
    fp.k = fp.engine == SV_PREC_NATIVE ? kmax : K;
    // the matrix-core kernels read the first block's operands from the state
    // and write the last block's results back to it
    if (is_mfma(fp.engine)) fp.direct = kDirectFirst | kDirectLast;
    for (int bi : idx) {
        const Block &B = bs[bi];
        DenseBlock db{};
        db.bp.k = fp.k;
        uint32_t used = 0;
        for (int j = 0; j < B.k; ++j) {
            db.bp.qpos[j] = local_bit(fp.sp, B.q[j]);
            used |= 1u << db.bp.qpos[j];
        }
        // padding qubits: the highest tile positions the block does not use
        for (int j = B.k, pos = fp.m - 1; j < fp.k; ++j) {
            while ((used >> pos) & 1u) --pos;
            db.bp.qpos[j] = pos;
            used |= 1u << pos;
        }
        db.bp.ng = 0;
        for (int b = 0; b < fp.m; ++b)
            if (!((used >> b) & 1u)) db.bp.gpos[db.bp.ng++] = b;
        db.vmask = B.vmask;
        fp.blocks.push_back(db);
        std::vector<std::vector<std::complex<double>>> vs;
        for (const auto &M : B.var.empty() ? std::vector<std::vector<std::complex<double>>>{B.M} : B.var)
            vs.push_back(B.k == fp.k ? M : pad_matrix(M, B.k, fp.k));
        fp.mats.push_back(std::move(vs));
        fp.flops_per_amp += 8.0 * (double)(1 << B.k);
    }
    return fp;
}

// Passes for a list of blocks (each: qubits q[0..k-1], matrix M), grouped
// by the tile scheduler.
static std::vector<FusedPass> compile_fused(const sv_state *h, const std::vector<Block> &bs, int prec) {
    const int mmax = std::min(h->n, fused_tile_qubits(h->dtype));
    std::vector<uint64_t> tm(bs.size());
    for (size_t b = 0; b < bs.size(); ++b) {
        tm[b] = 0;
        for (int j = 0; j < bs[b].k; ++j) tm[b] |= 1ull << bs[b].q[j];
    }
    std::vector<FusedPass> out;
    for (const Pass &p : schedule_masks(tm, tm, mmax, fused_lmin(h), lookahead_level(h))) {
        uint64_t needed = 0;
        for (int bi : p.gates) needed |= tm[bi];
        TileSpec sp{};
        tile_layout(h->n, mmax, fused_lmin(h), needed, &sp);
        out.push_back(build_fused_pass(h, sp, bs, p.gates, prec));
    }
    return out;
}


// Tile-aware fusion of a gate list: the tile scheduler first groups the
// gates into passes, then each pass's gates are fused into blocks of at most
// k_max qubits, so all blocks of a pass share one trip of the state through
// LDS.  Every qubit of a non-diagonal gate, controls included, must be in
// the tile; a diagonal gate of at most kMaxVariantQubits qubits needs none
// of its qubits there (those outside select a variant of its block's
// matrix per tile).
// Cost model of one pass, in ms per 2^30 amplitudes, fitted to kernel times
// measured on the MI355X (30-qubit complex64 fusion workload and the 32-qubit
// complex64 headline passes; complex128 scaled by its measured per-amplitude
// ratio).  A matrix-core pass costs its streaming floor plus a share per
// block by width and engine; a plain pass its floor plus shares per sweep
// (LDS exchange and barrier), per record, per gathered phase and per vector
// ALU operation.  It only ranks the alternatives of one pass.
static double fused_pass_cost(const sv_state *h, const FusedPass &fp) {
    const bool c64 = h->dtype == SV_C64;
    double t = c64 ? 3.4 : 6.5;
    for (const DenseBlock &db : fp.blocks) {
        const int k = db.bp.k;
        switch (fp.engine) {
        case SV_PREC_SPLIT_BF16: t += k <= 4 ? 0.34 : 0.65; break;
        case SV_PREC_FP32: t += k <= 4 ? 0.77 : 1.83; break;
        case kPrecMfma64: t += k <= 4 ? 1.5 : 3.2; break;
        default: t += c64 ? 0.12 * (1 << k) : 0.25 * (1 << k); break; // vector ALUs
        }
    }
    return t;
}

static double plain_pass_cost(const sv_state *h, const PassCode &pc) {
    double valu = 0.0, entries = 0.0;
    const int D = 1 << std::min(pc.m, sweep_width(h->dtype));
    for (const TileGate &r : pc.gates) {
        const int en = __builtin_popcount(r.amask);
        switch (r.kind) {
        case SK_GEN: valu += 16 + 16 * en; break;
        case SK_REAL: case SK_RIMAG: valu += 8 + 8 * en; break;
        case SK_SWAP: valu += 2 * en; break;
        case SK_DIAG: case SK_DIAGR: valu += 8 + 4 * en; break;
        case SK_2Q: valu += 64 * en; break;
        case SK_PHASE: valu += 6 + 6 * r.b1; entries += r.b1; break;
        case SK_PTAB: valu += 6 + 6 * r.b1; entries += r.b1; break;
        case SK_LPH: valu += 6 + 8 * r.b1; entries += r.b1; break;
        case SK_FLUSH: valu += 4.0 * D * __builtin_popcount(r.amask); break;
        default: break;
        }
    }
    const double t = 1.31 + 0.58 * (double)pc.sweeps.size() + 0.057 * (double)pc.gates.size() + 0.017 * entries +
                     4.4e-5 * valu;
    return h->dtype == SV_C64 ? t : 2.5 * t;
}

static std::vector<FusedPass> compile_fused_gates(const sv_state *h, const std::vector<Gate> &gs, int k_max,
                                                  int prec, int *n_blocks) {
    const int mmax = std::min(h->n, fused_tile_qubits(h->dtype));
    std::vector<uint64_t> tm(gs.size()), qm(gs.size());
    for (size_t i = 0; i < gs.size(); ++i) {
        qm[i] = gs[i].qmask();
        const bool outside_ok = is_diag_gate(gs[i]) && __builtin_popcountll(qm[i]) <= kMaxVariantQubits;
        tm[i] = outside_ok ? 0 : qm[i];
    }
    std::vector<FusedPass> out;
    *n_blocks = 0;
    for (const Pass &p : schedule_masks(tm, qm, mmax, fused_lmin(h), lookahead_level(h))) {
        uint64_t needed = 0;
        std::vector<Gate> sub;
        sub.reserve(p.gates.size());
        for (int gi : p.gates) {
            needed |= tm[gi];
            sub.push_back(gs[gi]);
        }
        TileSpec sp{};
        tile_layout(h->n, mmax, fused_lmin(h), needed, &sp);
        const uint64_t S = tile_qubits(sp);
        // candidates: blocks of at most k_max qubits, of at most 4 (when
        // k_max is 5), and the pass's gates as plain sweeps; the cheapest
        // by the cost model runs
        FusedPass best;
        int best_blocks = 0;
        best.cost = 1e300;
        // fuse_tile needs every gate's tile qubits to fit one block
        int widest = 1;
        for (const Gate &g : sub) widest = std::max(widest, __builtin_popcountll(g.qmask() & S));
        std::vector<int> widths{k_max};
        if (k_max == 5 && widest <= 4) widths.push_back(4);
        for (int kk : widths) {
            const std::vector<Block> bs = fuse_tile(sub, kk, S);
            std::vector<int> idx(bs.size());
            for (size_t b = 0; b < bs.size(); ++b) idx[b] = (int)b;
            FusedPass fp = build_fused_pass(h, sp, bs, idx, prec);
            fp.cost = fused_pass_cost(h, fp);
            if (fp.cost < best.cost) {
                best = std::move(fp);
                best_blocks = (int)bs.size();
            }
        }
        const int mtile = sp.L + sp.K;
        bool plain_ok = mtile <= tile_launch_qubits(h->dtype);
        std::vector<Gate> local;
        local.reserve(sub.size());
        for (const Gate &g : sub) {
            local.push_back(retarget_phase(g, S));
            plain_ok = plain_ok && (tile_need(local.back()) & ~S) == 0 && !needs_tile(h->dtype, g);
        }
        if (plain_ok) {
            std::vector<const Gate *> ptrs;
            for (const Gate &g : local) ptrs.push_back(&g);
            FusedPass fp;
            fp.plain = true;
            fp.sp = sp;
            fp.m = mtile;
            fp.code = compile_pass(sp, ptrs, sweep_width(h->dtype), h->dtype == SV_C64, nullptr, true);
            fp.cost = plain_pass_cost(h, fp.code);
            if (fp.cost < best.cost) {
                best = std::move(fp);
                best_blocks = 0;
            }
        }
        out.push_back(std::move(best));
        *n_blocks += best_blocks;
    }
    return out;
}

// LDS layout of the complex64 matrix-core passes, which address their tile
// only through the offset tables (their first block reads the state and
// their last writes it, so the tile is never staged by the device's own
// swizzle): the low 5 bits of a tile index (32 amplitudes, one row of the
// 64 banks) are XOR-ed with a fixed linear function of the higher bits.  The
// constants were chosen with a bank-conflict model of the blocks' operand
// and result accesses (64 lanes in two phases of 32, 2 banks per amplitude)
// over every position of a 4- or 5-qubit block in a 13-qubit tile: 2.5 LDS
// cycles per access on average and 4 at worst, against 4.3 and 16 for the
// gate tile's fold (2 is conflict-free).
static uint32_t mfma_swizzle_c64(uint32_t l) {
    static const uint32_t H[8] = {29, 19, 30, 7, 11, 27, 31, 22};
    uint32_t h = 0;
    for (int i = 0; i < 8; ++i)
        if ((l >> (5 + i)) & 1u) h ^= H[i];
    return l ^ h;
}

// Write a fused pass (block records, then per block its operand variants
// and offset tables) at 'off'; operand offsets are relative to the arena
// base.
static void stage_fused(sv_state *h, FusedPass &fp, size_t off) {
    const size_t fb = dense_frag_bytes(h, fp.k, fp.engine);
    const int ab = h->dtype == SV_C64 ? 8 : 16;
    size_t opo = off + align256(fp.blocks.size() * sizeof(DenseBlock));
    for (size_t b = 0; b < fp.blocks.size(); ++b) {
        DenseBlock &db = fp.blocks[b];
        const size_t nvar = fp.mats[b].size();
        db.op_off = (int64_t)opo;
        db.vstride = (int64_t)fb;
        db.tab_off = 0;
        db.gtab_off = 0;
        for (size_t v = 0; v < nvar; ++v) {
            char *dst = h->h_arena + opo + v * fb;
            const std::vector<std::complex<double>> &Mv = fp.mats[b][v];
            const std::complex<double> *U = Mv.data();
            if (fp.engine == kPrecMfma64) {
                make_fragments64(U, fp.k, dst);
            } else if (fp.engine != SV_PREC_NATIVE) {
                make_fragments(U, fp.k, fp.engine, dst);
            } else if (h->dtype == SV_C64) {
                float *f = reinterpret_cast<float *>(dst);
                for (size_t i = 0; i < Mv.size(); ++i) {
                    f[2 * i] = (float)U[i].real();
                    f[2 * i + 1] = (float)U[i].imag();
                }
            } else {
                double *d = reinterpret_cast<double *>(dst);
                for (size_t i = 0; i < Mv.size(); ++i) {
                    d[2 * i] = U[i].real();
                    d[2 * i + 1] = U[i].imag();
                }
            }
        }
        const size_t tabs = opo + nvar * fb;
        if (is_mfma(fp.engine)) {
            db.tab_off = (int64_t)tabs;
            uint32_t *qoff = reinterpret_cast<uint32_t *>(h->h_arena + tabs);
            uint32_t *goff = qoff + (1u << fp.k);
            auto deposit = [](uint32_t x, const int *pos, int nb) {
                uint32_t r = 0;
                for (int i = 0; i < nb; ++i)
                    if ((x >> i) & 1u) r |= 1u << pos[i];
                return r;
            };
            const uint32_t rows = (uint32_t)mfma_rows(fp.k, fp.engine);
            uint32_t *ghi = goff + rows;
            const bool own = h->dtype == SV_C64 && fp.direct == (kDirectFirst | kDirectLast) && fp.m <= 13;
            auto swz = [&](uint32_t l) { return own ? mfma_swizzle_c64(l) : lds_swizzle(l, ab); };
            for (uint32_t j = 0; j < (1u << fp.k); ++j) qoff[j] = swz(deposit(j, db.bp.qpos, fp.k));
            for (uint32_t g = 0; g < rows; ++g) goff[g] = swz(deposit(g, db.bp.gpos, db.bp.ng));
            for (uint32_t w = 0; w < (1u << (fp.m - fp.k)) / rows; ++w)
                ghi[w] = swz(deposit(w * rows, db.bp.gpos, db.bp.ng));
            // the same tables as global offsets
            db.gtab_off = (int64_t)(tabs + align256(dense_tab_entries(fp.k, fp.m, fp.engine) * sizeof(uint32_t)));
            uint64_t *gq = reinterpret_cast<uint64_t *>(h->h_arena + db.gtab_off);
            uint64_t *gg = gq + (1u << fp.k);
            for (uint32_t j = 0; j < (1u << fp.k); ++j) gq[j] = tile_global_offset(fp.sp, deposit(j, db.bp.qpos, fp.k));
            for (uint32_t g = 0; g < rows; ++g) gg[g] = tile_global_offset(fp.sp, deposit(g, db.bp.gpos, db.bp.ng));
            for (uint32_t w = 0; w < (1u << (fp.m - fp.k)) / rows; ++w)
                gg[rows + w] = tile_global_offset(fp.sp, deposit(w * rows, db.bp.gpos, db.bp.ng));
        }
        opo += dense_op_bytes(h, fp.k, fp.m, fp.engine, nvar);
    }
    std::memcpy(h->h_arena + off, fp.blocks.data(), fp.blocks.size() * sizeof(DenseBlock));
}

static int launch_fused(sv_state *h, const FusedPass &fp, size_t off) {
    if (fp.plain) return launch_pass(h, fp.code, off);
    Timed tm(h, K_FUSED, 2.0 * state_bytes(h), fp.flops_per_amp * (double)(1ull << h->n));
    SV_HIP(launch_dense_pass(h->amps, h->n, h->dtype, fp.sp, fp.k,
                             reinterpret_cast<const DenseBlock *>(h->d_arena + off), (int)fp.blocks.size(),
                             h->d_arena, fp.engine, fp.direct, h->stream));
    return SV_OK;
}

// Stage, upload and launch a sequence of fused passes.
static int run_fused_passes(sv_state *h, std::vector<FusedPass> &fps) {
    std::vector<size_t> offs(fps.size());
    size_t total = 0;
    for (size_t i = 0; i < fps.size(); ++i) {
        offs[i] = total;
        total += align256(fused_pass_bytes(h, fps[i]));
    }
    int rc = ensure_arena(h, total);
    if (rc) return rc;
    if ((rc = stage_wait(h))) return rc;
    for (size_t i = 0; i < fps.size(); ++i) {
        if (fps[i].plain) stage_pass(h, fps[i].code, offs[i]);
        else stage_fused(h, fps[i], offs[i]);
    }
    if ((rc = upload_arena(h, total))) return rc;
    for (size_t i = 0; i < fps.size(); ++i)
        if ((rc = launch_fused(h, fps[i], offs[i]))) return rc;
    return SV_OK;
}

static int parse_ops(const sv_state *h, int n, const sv_op *ops, int n_ops, const double *params,
                     int n_params, std::vector<Gate> &gs) {
    (void)h;
    if (n_ops < 0 || (n_ops > 0 && !ops)) return fail(SV_EINVAL, "bad op list");
    gs.resize((size_t)n_ops);
    for (int i = 0; i < n_ops; ++i) {
        const int rc = op_to_gate(n, ops[i], params, n_params, &gs[i]);
        if (rc) return fail(rc, "op " + std::to_string(i) + ": " + g_last_error);
    }
    return SV_OK;
}


// ================================================================ adjoint
static Gate dagger(const Gate &g) {
    Gate d = g;
    const int D = 1 << g.k;
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) {
            d.U[2 * (c * D + r)] = g.U[2 * (r * D + c)];
            d.U[2 * (c * D + r) + 1] = -g.U[2 * (r * D + c) + 1];
        }
    return d;
}

// Probe M and factor f of a parametrised gate: dU/dtheta = c M U gives the
// gradient term f * Im <lam| M |psi> (R_P = exp(-i theta P/2): M = P, f = 1;
// U1 = diag(1, e^{i theta}): M = |1><1|, f = -2).
static bool probe_of(int kind, double *M, double *f) {
    for (int i = 0; i < 8; ++i) M[i] = 0.0;
    switch (kind) {
    case SV_GATE_RX: M[2] = 1; M[4] = 1; *f = 1.0; return true;
    case SV_GATE_RY: M[3] = -1; M[5] = 1; *f = 1.0; return true;
    case SV_GATE_RZ: M[0] = 1; M[6] = -1; *f = 1.0; return true;
    case SV_GATE_U1: M[6] = 1; *f = -2.0; return true;
    default: return false;
    }
}

static int ensure_scratch(sv_state *h, size_t doubles) {
    if (doubles <= h->scratch_cap) return SV_OK;
    SV_HIP(hipStreamSynchronize(h->stream));
    if (h->d_scratch) SV_HIP(hipFree(h->d_scratch));
    h->d_scratch = nullptr;
    h->scratch_cap = 0;
    SV_HIP(hipMalloc((void **)&h->d_scratch, doubles * sizeof(double)));
    h->scratch_cap = doubles;
    return SV_OK;
}


// ================================================================ batches
struct BatchProgram {
    std::vector<BatchCircuit> circuits;
    std::vector<BatchPass> passes;
    std::vector<TileSweep> sweeps;
    std::vector<char> recs; // packed records of all passes
    bool two_qubit = false;
    std::vector<int32_t> order;
    size_t state_bytes = 0;
};

// Fusion width of a batch program: fw = 0 keeps the gates; fw = 1 or 2
// multiplies, greedily in circuit order, gates into blocks of at most fw
// qubits (targets and controls; a gate may move ahead only past gates on
// other qubits, as in fuse()), each block becoming one 2x2 or 4x4 gate.  A
// block of a single gate keeps that gate (its cheaper record kind), and a
// gate wider than fw passes through on its own.
static std::vector<Gate> fuse_for_batch(const std::vector<Gate> &gs, int fw) {
    if (fw <= 0) return gs;
    std::vector<Gate> out;
    std::vector<char> done(gs.size(), 0);
    size_t first = 0;
    while (first < gs.size()) {
        if (__builtin_popcountll(gs[first].qmask()) > fw) {
            out.push_back(gs[first]);
            done[first] = 1;
        } else {
            uint64_t set = 0, blocked = 0;
            std::vector<int> members;
            for (size_t i = first; i < gs.size(); ++i) {
                if (done[i]) continue;
                const uint64_t gq = gs[i].qmask();
                if ((gq & blocked) || __builtin_popcountll(set | gq) > fw) {
                    blocked |= gq;
                    continue;
                }
                set |= gq;
                members.push_back((int)i);
                done[i] = 1;
            }
            if (members.size() == 1) {
                out.push_back(gs[members[0]]);
            } else {
                Block b;
                for (uint64_t m = set; m; m &= m - 1) b.q[b.k++] = __builtin_ctzll(m);
                const int D = 1 << b.k;
                b.M.assign((size_t)D * D, 0.0);
                for (int i = 0; i < D; ++i) b.M[(size_t)i * D + i] = 1.0;
                for (int gi : members) absorb(b, gs[gi]);
                Gate g{};
                g.k = b.k;
                g.t[0] = b.q[0];
                g.t[1] = b.k == 2 ? b.q[1] : -1;
                g.ctrl = 0;
                for (size_t i = 0; i < b.M.size(); ++i) {
                    g.U[2 * i] = b.M[i].real();
                    g.U[2 * i + 1] = b.M[i].imag();
                }
                out.push_back(g);
            }
        }
        while (first < gs.size() && done[first]) ++first;
    }
    return out;
}

// Compile every circuit into tile passes for tiles of at most mmax qubits
// and sweeps of sweep_w register qubits.
static BatchProgram compile_batch(const std::vector<int> &widths,
                                  const std::vector<std::vector<Gate>> &circ, int dtype, int mmax,
                                  int sweep_w, bool keep) {
    BatchProgram bp;
    const size_t el = dtype == SV_C64 ? 8 : 16;
    std::vector<double> cost(widths.size());
    for (size_t i = 0; i < widths.size(); ++i) {
        const int w = widths[i];
        const int m = std::min(w, mmax);
        const int lmin = std::min(w, dtype == SV_C64 ? 7 : 6);
        std::vector<Pass> passes;
        if (w <= mmax) {
            Pass p;
            for (size_t g = 0; g < circ[i].size(); ++g) p.gates.push_back((int)g);
            passes.push_back(p);
        } else {
            passes = schedule(circ[i], w, m, lmin);
        }
        if (passes.empty()) passes.push_back(Pass{}); // a circuit without gates still reduces |0>
        BatchCircuit c{};
        c.w = w;
        c.n_passes = (int)passes.size();
        c.pass_off = (int)bp.passes.size();
        c.keep = keep ? 1 : 0;
        c.state_off = 0;
        if (passes.size() > 1 || keep) {
            c.state_off = (int64_t)bp.state_bytes;
            bp.state_bytes += align256(((size_t)1 << w) * el);
        }
        for (const Pass &p : passes) {
            uint64_t needed = 0;
            std::vector<const Gate *> ptrs;
            for (int gi : p.gates) {
                needed |= circ[i][gi].tmask();
                ptrs.push_back(&circ[i][gi]);
            }
            TileSpec sp{};
            if (w <= mmax) {
                sp.L = w;
                sp.K = 0;
            } else {
                tile_layout(w, m, lmin, needed, &sp);
            }
            PassCode pc = compile_pass(sp, ptrs, sweep_w, dtype == SV_C64);
            if (pc.sweeps.empty()) {
                // a circuit without gates still needs one sweep: the batch
                // kernel synthesises |0...0> and reduces in a sweep's registers
                TileSweep sw{};
                const int W = std::min(pc.m, sweep_w);
                for (int b = 0; b < W; ++b) sw.qpos[b] = pc.m - W + b;
                sw.rec_off = 0;
                pc.sweeps.push_back(sw);
            }
            BatchPass q{};
            q.sp = sp;
            q.n_sweeps = (int)pc.sweeps.size();
            q.sweep_off = (int)bp.sweeps.size();
            q.gate_off = (int)bp.recs.size();
            bp.passes.push_back(q);
            bp.sweeps.insert(bp.sweeps.end(), pc.sweeps.begin(), pc.sweeps.end());
            bp.recs.insert(bp.recs.end(), pc.recs.begin(), pc.recs.end());
            bp.two_qubit = bp.two_qubit || pc.two_qubit;
        }
        bp.circuits.push_back(c);
        cost[i] = std::ldexp((double)(circ[i].size() + 1) * (double)passes.size(), w);
    }
    bp.order.resize(widths.size());
    for (size_t i = 0; i < widths.size(); ++i) bp.order[i] = (int32_t)i;
    std::stable_sort(bp.order.begin(), bp.order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    return bp;
}

} // namespace sv

struct sv_batch {
    int n = 0;
    int dtype = 0;
    int flags = 0;
    uint64_t zmask = 0;
    hipStream_t stream = nullptr;
    std::vector<int> widths;
    std::vector<std::vector<sv::Gate>> circ;
    // device program
    char *d_prog = nullptr;
    void *d_states = nullptr;
    double *d_out = nullptr;
    unsigned int *d_counter = nullptr;
    sv::BatchArgs args{};
    std::vector<int64_t> state_off;
    std::vector<int> n_passes;
    int tile_m = 0, sweep_w = 0, grid = 0, fuse_w = 0;
    bool two_qubit = false; // the program holds SK_2Q records
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace sv {

static void batch_release_program(sv_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_prog) (void)hipFree(b->d_prog);
    if (b->d_states) (void)hipFree(b->d_states);
    b->exec = nullptr;
    b->graph = nullptr;
    b->d_prog = nullptr;
    b->d_states = nullptr;
}

// Build, upload and capture the batch program for (tile_m, sweep_w, grid).
static int batch_prepare(sv_batch *b, int tile_m, int sweep_w, int grid, int fuse_w) {
    // the kernel is instantiated for sweeps of exactly sweep_w register
    // qubits: a circuit narrower than that would have no register groups
    const int wnarrow = *std::min_element(b->widths.begin(), b->widths.end());
    if (sweep_w > wnarrow || sweep_w > tile_m)
        return fail(SV_EINVAL, "sweep width " + std::to_string(sweep_w) + " exceeds the narrowest circuit (" +
                                   std::to_string(wnarrow) + " qubits) or the tile");
    SV_HIP(hipStreamSynchronize(b->stream));
    batch_release_program(b);
    const bool keep = (b->flags & SV_BATCH_KEEP_STATES) != 0;
    std::vector<std::vector<Gate>> fused;
    if (fuse_w > 0) {
        fused.reserve(b->circ.size());
        for (const auto &c : b->circ) fused.push_back(fuse_for_batch(c, fuse_w));
    }
    BatchProgram bp = compile_batch(b->widths, fuse_w > 0 ? fused : b->circ, b->dtype, tile_m, sweep_w, keep);
    const size_t o_c = 0;
    const size_t o_p = align256(o_c + bp.circuits.size() * sizeof(BatchCircuit));
    const size_t o_s = align256(o_p + bp.passes.size() * sizeof(BatchPass));
    const size_t o_g = align256(o_s + bp.sweeps.size() * sizeof(TileSweep));
    const size_t o_o = align256(o_g + bp.recs.size());
    const size_t total = align256(o_o + bp.order.size() * sizeof(int32_t));
    size_t free_b = 0, total_b = 0;
    SV_HIP(hipMemGetInfo(&free_b, &total_b));
    if (total + bp.state_bytes + (64u << 20) > free_b)
        return fail(SV_ENOMEM, "batch program and states exceed free device memory");
    SV_HIP(hipMalloc((void **)&b->d_prog, total));
    if (bp.state_bytes) SV_HIP(hipMalloc(&b->d_states, bp.state_bytes));
    std::vector<char> host(total, 0);
    std::memcpy(host.data() + o_c, bp.circuits.data(), bp.circuits.size() * sizeof(BatchCircuit));
    std::memcpy(host.data() + o_p, bp.passes.data(), bp.passes.size() * sizeof(BatchPass));
    std::memcpy(host.data() + o_s, bp.sweeps.data(), bp.sweeps.size() * sizeof(TileSweep));
    std::memcpy(host.data() + o_g, bp.recs.data(), bp.recs.size());
    std::memcpy(host.data() + o_o, bp.order.data(), bp.order.size() * sizeof(int32_t));
    SV_HIP(hipMemcpy(b->d_prog, host.data(), total, hipMemcpyHostToDevice));
    BatchArgs &a = b->args;
    a.circuits = reinterpret_cast<const BatchCircuit *>(b->d_prog + o_c);
    a.passes = reinterpret_cast<const BatchPass *>(b->d_prog + o_p);
    a.sweeps = reinterpret_cast<const TileSweep *>(b->d_prog + o_s);
    a.recs = b->d_prog + o_g;
    a.order = reinterpret_cast<const int32_t *>(b->d_prog + o_o);
    a.counter = b->d_counter;
    a.states = b->d_states;
    a.out = b->d_out;
    a.n_circuits = b->n;
    a.zmask = b->zmask;
    b->state_off.resize(b->n);
    b->n_passes.resize(b->n);
    for (int i = 0; i < b->n; ++i) {
        b->state_off[i] = bp.circuits[i].state_off;
        b->n_passes[i] = bp.circuits[i].n_passes;
    }
    b->tile_m = tile_m;
    b->sweep_w = sweep_w;
    b->grid = grid;
    b->fuse_w = fuse_w;
    b->two_qubit = bp.two_qubit;
    // one eager launch (sets kernel attributes, checks the launch), then capture
    SV_HIP(launch_batch(a, b->dtype, sweep_w, tile_m, grid, b->two_qubit, b->stream));
    SV_HIP(hipStreamSynchronize(b->stream));
    // capture on a private stream (the caller's may be the null stream, which
    // cannot be captured); the graph is launched on the caller's stream
    hipStream_t cap = nullptr;
    SV_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t e0 = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e0 != hipSuccess) {
        (void)hipStreamDestroy(cap);
        return hip_fail(e0, "hipStreamBeginCapture");
    }
    hipError_t e = launch_batch(a, b->dtype, sweep_w, tile_m, grid, b->two_qubit, cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cap, &g);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return hip_fail(e, "launch_batch (capture)");
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    b->graph = g;
    SV_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    return SV_OK;
}

static int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

} // namespace sv

using namespace sv;

// ===================================================================== C ABI
extern "C" {

const char *sv_last_error(void) { return g_last_error.c_str(); }

const char *sv_version(void) { return "svsim-gfx950 0.1"; }

size_t sv_state_bytes(int n_qubits, int dtype) {
    if (n_qubits < 1 || n_qubits > 40) return 0;
    if (dtype != SV_C64 && dtype != SV_C128) return 0;
    return (size_t(1) << n_qubits) * (dtype == SV_C64 ? 8 : 16);
}

int sv_alloc(int n_qubits, int dtype, void *dev_buf, void *hip_stream, sv_handle *out) {
    if (!out) return fail(SV_EINVAL, "NULL output handle");
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > 40) return fail(SV_EINVAL, "n_qubits must be in [1, 40]");
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "dtype must be SV_C64 or SV_C128");
    if (dev_buf && (reinterpret_cast<uintptr_t>(dev_buf) & 15u))
        return fail(SV_EINVAL, "dev_buf must be 16-byte aligned");
    const size_t bytes = sv_state_bytes(n_qubits, dtype);
    sv_state *h = new sv_state();
    h->n = n_qubits;
    h->dtype = dtype;
    h->stream = (hipStream_t)hip_stream;
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "hipGetDevice");
    }
    if (!dev_buf) {
        size_t free_b = 0, total_b = 0;
        e = hipMemGetInfo(&free_b, &total_b);
        if (e != hipSuccess) {
            delete h;
            return hip_fail(e, "hipMemGetInfo");
        }
        if (bytes + (64u << 20) > free_b) {
            delete h;
            return fail(SV_ENOMEM, "state of " + std::to_string(bytes) + " bytes exceeds free device memory");
        }
        e = hipMalloc(&h->amps, bytes);
        if (e != hipSuccess) {
            delete h;
            return fail(SV_ENOMEM, std::string("hipMalloc of the state failed: ") + hipGetErrorString(e));
        }
        h->owned = true;
    } else {
        h->amps = dev_buf;
    }
    int rc = SV_OK;
    if ((e = hipMalloc((void **)&h->d_red, sizeof(double) * (kReduceBlocks + 1))) != hipSuccess ||
        (e = hipHostMalloc((void **)&h->h_result, sizeof(double) * 8, hipHostMallocDefault)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&h->stage_done, hipEventDisableTiming)) != hipSuccess ||
        (e = launch_init_basis(h->amps, h->n, h->dtype, 0, h->stream)) != hipSuccess) {
        rc = hip_fail(e, "sv_alloc");
        sv_free(h);
        return rc;
    }
    *out = h;
    return SV_OK;
}

int sv_free(sv_handle h) {
    if (!h) return fail(SV_EINVAL, "NULL handle");
    hipStreamSynchronize(h->stream);
    if (h->owned && h->amps) hipFree(h->amps);
    if (h->d_red) hipFree(h->d_red);
    if (h->h_result) hipHostFree(h->h_result);
    if (h->d_scratch) hipFree(h->d_scratch);
    if (h->d_arena) hipFree(h->d_arena);
    if (h->h_arena) hipHostFree(h->h_arena);
    if (h->stage_done) hipEventDestroy(h->stage_done);
    for (hipEvent_t e : h->pool) hipEventDestroy(e);
    delete h;
    return SV_OK;
}

int sv_set_basis(sv_handle h, uint64_t x) {
    if (!h) return fail(SV_EINVAL, "NULL handle");
    if (h->n < 64 && (x >> h->n) != 0) return fail(SV_EINVAL, "basis index >= 2^n");
    Timed tm(h, K_INIT, state_bytes(h));
    SV_HIP(launch_init_basis(h->amps, h->n, h->dtype, x, h->stream));
    return SV_OK;
}

int sv_set_stream(sv_handle h, void *hip_stream) {
    if (!h) return fail(SV_EINVAL, "NULL handle");
    int rc = stage_wait(h);
    if (rc) return rc;
    SV_HIP(hipStreamSynchronize(h->stream));
    h->stream = (hipStream_t)hip_stream;
    return SV_OK;
}

int sv_sync(sv_handle h) {
    if (!h) return fail(SV_EINVAL, "NULL handle");
    SV_HIP(hipStreamSynchronize(h->stream));
    return SV_OK;
}

void *sv_data(sv_handle h) { return h ? h->amps : nullptr; }

int sv_apply_gate(sv_handle h, int k, const int *targets, uint64_t ctrl_mask, const double *U) {
    if (!h) return fail(SV_EINVAL, "NULL handle");
    int rc = check_gate(h->n, k, targets, ctrl_mask, U);
    if (rc) return rc;
    Gate g;
    g.k = k;
    g.t[0] = targets[0];
    g.t[1] = k == 2 ? targets[1] : -1;
    g.ctrl = ctrl_mask;
    std::memcpy(g.U, U, sizeof(double) * 2 * (1 << (2 * k)));
    return apply_one(h, g);
}

int sv_run(sv_handle h, const sv_op *ops, int n_ops, const double *params, int n_params, int mode) {
    if (!h) return fail(SV_EINVAL, "NULL handle");
    if (n_ops < 0 || (n_ops > 0 && !ops)) return fail(SV_EINVAL, "bad op list");
    if (mode != SV_RUN_PER_GATE && mode != SV_RUN_TILED) return fail(SV_EINVAL, "unknown run mode");
    std::vector<Gate> gs((size_t)n_ops);
    for (int i = 0; i < n_ops; ++i) {
        const int rc = op_to_gate(h->n, ops[i], params, n_params, &gs[i]);
        if (rc) return fail(rc, "op " + std::to_string(i) + ": " + g_last_error);
    }
    return run_gates(h, gs, mode);
}

int sv_probabilities(sv_handle h, void *dev_out, double *host_norm) {
    if (!h) return fail(SV_EINVAL, "NULL handle");
    {
        Timed tm(h, K_PROBS, state_bytes(h) * (dev_out ? 1.5 : 1.0));
        SV_HIP(launch_probabilities(h->amps, h->n, h->dtype, dev_out, h->d_red, kReduceBlocks,
                                    h->d_red + kReduceBlocks, h->stream));
    }
    if (host_norm) {
        SV_HIP(hipMemcpyAsync(h->h_result, h->d_red + kReduceBlocks, sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
        SV_HIP(hipStreamSynchronize(h->stream));
        *host_norm = h->h_result[0];
    }
    return SV_OK;
}

int sv_expectation(sv_handle h, int n_terms, const uint64_t *z_masks, const double *coeffs,
                   double *host_out) {
    if (!h) return fail(SV_EINVAL, "NULL handle");
    if (n_terms < 1 || n_terms > kMaxTerms) return fail(SV_EINVAL, "n_terms must be in [1, 64]");
    if (!z_masks || !coeffs || !host_out) return fail(SV_EINVAL, "NULL argument");
    for (int j = 0; j < n_terms; ++j)
        if (h->n < 64 && (z_masks[j] >> h->n) != 0) return fail(SV_EINVAL, "Z mask has bits >= n");
    {
        Timed tm(h, K_EXPECT, state_bytes(h));
        SV_HIP(launch_expectation(h->amps, h->n, h->dtype, n_terms, z_masks, coeffs, h->d_red,
                                  kReduceBlocks, h->d_red + kReduceBlocks, h->stream));
    }
    SV_HIP(hipMemcpyAsync(h->h_result, h->d_red + kReduceBlocks, sizeof(double),
                          hipMemcpyDeviceToHost, h->stream));
    SV_HIP(hipStreamSynchronize(h->stream));
    *host_out = h->h_result[0];
    return SV_OK;
}

int sv_expectation_noalloc(const void *dev_amps, int n_qubits, int dtype, int n_terms, const uint64_t *z_masks,
                           const double *coeffs, double *dev_out, void *hip_stream) {
    if (!dev_amps || !dev_out || !z_masks || !coeffs) return fail(SV_EINVAL, "NULL argument");
    if (n_qubits < 1 || n_qubits > 40) return fail(SV_EINVAL, "n_qubits must be in [1, 40]");
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "dtype must be SV_C64 or SV_C128");
    if (reinterpret_cast<uintptr_t>(dev_amps) & 15u) return fail(SV_EINVAL, "dev_amps must be 16-byte aligned");
    if (reinterpret_cast<uintptr_t>(dev_out) & 7u) return fail(SV_EINVAL, "dev_out must be 8-byte aligned");
    if (n_terms < 1 || n_terms > kMaxTerms)
        return fail(SV_EINVAL, "n_terms must be in [1, 64] (the terms travel as kernel arguments)");
    for (int j = 0; j < n_terms; ++j)
        if (n_qubits < 64 && (z_masks[j] >> n_qubits) != 0) return fail(SV_EINVAL, "Z mask has bits >= n");
    SV_HIP(launch_expectation_static(dev_amps, n_qubits, dtype, n_terms, z_masks, coeffs, dev_out,
                                     (hipStream_t)hip_stream));
    return SV_OK;
}

// ============================================================ measurement
static int measure_positions(const sv_state *h, uint64_t mask, MeasurePos *mp) {
    if (mask == 0) return fail(SV_EINVAL, "empty qubit mask");
    if (h->n < 64 && (mask >> h->n) != 0) return fail(SV_EINVAL, "qubit mask has bits >= n");
    const int k = __builtin_popcountll(mask);
    if (k > kMaxMeasureQubits) return fail(SV_EINVAL, "at most 6 qubits per measurement");
    mp->k = 0;
    for (uint64_t m = mask; m; m &= m - 1) mp->pos[mp->k++] = __builtin_ctzll(m);
    return SV_OK;
}

// FP64 outcome probabilities of the qubits in mp, in outcome order.
static int marginals_of(sv_state *h, const MeasurePos &mp, std::vector<double> &out) {
    const int G = marginal_blocks(h->n, h->dtype), nb = 1 << mp.k;
    int rc = ensure_scratch(h, (size_t)nb * G + nb);
    if (rc) return rc;
    {
        Timed tm(h, K_MEASURE, state_bytes(h), 2.0 * (double)(1ull << h->n));
        SV_HIP(launch_marginals(h->amps, h->n, h->dtype, mp, h->d_scratch, h->stream));
    }
    SV_HIP(launch_sum_slots(h->d_scratch, nb, G, h->d_scratch + (size_t)nb * G, h->stream));
    out.assign(nb, 0.0);
    SV_HIP(hipMemcpyAsync(out.data(), h->d_scratch + (size_t)nb * G, nb * sizeof(double), hipMemcpyDeviceToHost,
                          h->stream));
    SV_HIP(hipStreamSynchronize(h->stream));
    return SV_OK;
}

static int collapse_onto(sv_state *h, uint64_t mask, uint64_t want, double p) {
    Timed tm(h, K_MEASURE, 2.0 * state_bytes(h), 2.0 * (double)(1ull << h->n));
    SV_HIP(launch_collapse(h->amps, h->n, h->dtype, mask, want, 1.0 / std::sqrt(p), h->stream));
    return SV_OK;
}

int sv_marginals(sv_handle h, uint64_t mask, double *host_out) {
    if (!h || !host_out) return fail(SV_EINVAL, "NULL argument");
    MeasurePos mp{};
    int rc = measure_positions(h, mask, &mp);
    if (rc) return rc;
    std::vector<double> m;
    if ((rc = marginals_of(h, mp, m))) return rc;
    std::memcpy(host_out, m.data(), m.size() * sizeof(double));
    return SV_OK;
}

int sv_collapse(sv_handle h, uint64_t mask, uint64_t value, double *host_prob) {
    if (!h) return fail(SV_EINVAL, "NULL handle");
    if (h->n < 64 && (mask >> h->n) != 0) return fail(SV_EINVAL, "qubit mask has bits >= n");
    const uint64_t want = value & mask;
    const int G = marginal_blocks(h->n, h->dtype);
    int rc = ensure_scratch(h, (size_t)G + 1);
    if (rc) return rc;
    {
        Timed tm(h, K_MEASURE, state_bytes(h), 2.0 * (double)(1ull << h->n));
        SV_HIP(launch_masked_prob(h->amps, h->n, h->dtype, mask, want, h->d_scratch, h->stream));
    }
    SV_HIP(launch_sum_slots(h->d_scratch, 1, G, h->d_scratch + G, h->stream));
    double p = 0.0;
    SV_HIP(hipMemcpyAsync(&p, h->d_scratch + G, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    SV_HIP(hipStreamSynchronize(h->stream));
    if (host_prob) *host_prob = p;
    if (!(p > 0.0)) return fail(SV_EINVAL, "the outcome has probability 0");
    return collapse_onto(h, mask, want, p);
}

int sv_measure(sv_handle h, uint64_t mask, double u, uint64_t *host_value, double *host_prob) {
    if (!h || !host_value) return fail(SV_EINVAL, "NULL argument");
    if (!(u >= 0.0 && u < 1.0)) return fail(SV_EINVAL, "u must be in [0, 1)");
    MeasurePos mp{};
    int rc = measure_positions(h, mask, &mp);
    if (rc) return rc;
    std::vector<double> m;
    if ((rc = marginals_of(h, mp, m))) return rc;
    // inverse CDF over the outcomes in index order
    double total = 0.0;
    for (double x : m) total += x;
    if (!(total > 0.0)) return fail(SV_EINVAL, "the state has norm 0");
    const double t = u * total;
    double c = 0.0;
    int o = -1, last = 0;
    for (int i = 0; i < (int)m.size(); ++i) {
        c += m[i];
        if (m[i] > 0.0) last = i;
        if (c > t) {
            o = i;
            break;
        }
    }
    if (o < 0) o = last;
    uint64_t v = 0;
    for (int i = 0; i < mp.k; ++i)
        if ((o >> i) & 1) v |= 1ull << mp.pos[i];
    *host_value = v;
    if (host_prob) *host_prob = m[o];
    return collapse_onto(h, mask, v, m[o]);
}

int sv_sample(sv_handle h, int n_samples, const double *uniforms, uint64_t *host_out) {
    if (!h) return fail(SV_EINVAL, "NULL handle");
    if (n_samples < 0 || n_samples > (1 << 24)) return fail(SV_EINVAL, "n_samples must be in [0, 2^24]");
    if (n_samples == 0) return SV_OK;
    if (!uniforms || !host_out) return fail(SV_EINVAL, "NULL argument");
    for (int i = 0; i < n_samples; ++i)
        if (!(uniforms[i] >= 0.0 && uniforms[i] < 1.0)) return fail(SV_EINVAL, "uniforms must be in [0, 1)");
    const int bl = sample_block_log(h->n);
    const size_t B = (size_t)1 << (h->n - bl), S = (size_t)n_samples;
    int rc = ensure_scratch(h, B + 3 * S);
    if (rc) return rc;
    double *d_sums = h->d_scratch;
    int64_t *d_blk = reinterpret_cast<int64_t *>(h->d_scratch + B);
    double *d_tgt = h->d_scratch + B + S;
    uint64_t *d_out = reinterpret_cast<uint64_t *>(h->d_scratch + B + 2 * S);
    {
        Timed tm(h, K_MEASURE, state_bytes(h), 2.0 * (double)(1ull << h->n));
        SV_HIP(launch_block_sums(h->amps, h->n, h->dtype, bl, d_sums, h->stream));
    }
    std::vector<double> sums(B), pre(B + 1);
    SV_HIP(hipMemcpyAsync(sums.data(), d_sums, B * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    SV_HIP(hipStreamSynchronize(h->stream));
    pre[0] = 0.0;
    for (size_t b = 0; b < B; ++b) pre[b + 1] = pre[b] + sums[b];
    const double total = pre[B];
    if (!(total > 0.0)) return fail(SV_EINVAL, "the state has norm 0");
    // block of each sample: the first block whose cumulative end exceeds the
    // target (the last block with mass if rounding leaves none)
    size_t last_nz = 0;
    for (size_t b = 0; b < B; ++b)
        if (sums[b] > 0.0) last_nz = b;
    std::vector<int64_t> blk(S);
    std::vector<double> tgt(S);
    for (size_t i = 0; i < S; ++i) {
        const double t = uniforms[i] * total;
        size_t b = (size_t)(std::upper_bound(pre.begin() + 1, pre.end(), t) - (pre.begin() + 1));
        if (b >= B) b = last_nz;
        blk[i] = (int64_t)b;
        tgt[i] = t - pre[b];
    }
    SV_HIP(hipMemcpyAsync(d_blk, blk.data(), S * sizeof(int64_t), hipMemcpyHostToDevice, h->stream));
    SV_HIP(hipMemcpyAsync(d_tgt, tgt.data(), S * sizeof(double), hipMemcpyHostToDevice, h->stream));
    {
        Timed tm(h, K_MEASURE, 0.0, 0.0);
        SV_HIP(launch_sample_scan(h->amps, h->dtype, bl, n_samples, d_blk, d_tgt, d_out, h->stream));
    }
    SV_HIP(hipMemcpyAsync(host_out, d_out, S * sizeof(uint64_t), hipMemcpyDeviceToHost, h->stream));
    SV_HIP(hipStreamSynchronize(h->stream));
    return SV_OK;
}

int sv_timing(sv_handle h, int enable) {
    if (!h) return fail(SV_EINVAL, "NULL handle");
    SV_HIP(hipStreamSynchronize(h->stream));
    h->recs.clear();
    h->pool_used = 0;
    h->timing = enable != 0;
    return SV_OK;
}

int sv_timing_read(sv_handle h, sv_kernel_stat *out, int cap, int *n_out) {
    if (!h || !n_out || (cap > 0 && !out)) return fail(SV_EINVAL, "NULL argument");
    SV_HIP(hipStreamSynchronize(h->stream));
    sv_kernel_stat acc[K_COUNT];
    std::memset(acc, 0, sizeof(acc));
    for (const auto &r : h->recs) {
        float ms = 0.0f;
        SV_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        acc[r.kid].launches += 1;
        acc[r.kid].total_ms += ms;
        acc[r.kid].bytes += r.bytes;
        acc[r.kid].flops += r.flops;
    }
    int n = 0;
    for (int k = 0; k < K_COUNT; ++k) {
        if (acc[k].launches == 0) continue;
        if (n < cap) {
            out[n] = acc[k];
            std::snprintf(out[n].name, sizeof(out[n].name), "%s", kKernelNames[k]);
        }
        ++n;
    }
    *n_out = n;
    h->recs.clear();
    h->pool_used = 0;
    return n > cap ? fail(SV_EINVAL, "cap too small") : SV_OK;
}

int sv_apply_fused(sv_handle h, int k, const int *qubits, const double *U, int prec) {
    if (!h) return fail(SV_EINVAL, "NULL handle");
    if (!qubits || !U) return fail(SV_EINVAL, "NULL qubits or matrix");
    if (k < 1 || k > 5) return fail(SV_EINVAL, "k must be in [1, 5]");
    if (k > h->n) return fail(SV_EINVAL, "k exceeds the register size");
    if (prec != SV_PREC_NATIVE && prec != SV_PREC_FP32 && prec != SV_PREC_SPLIT_BF16)
        return fail(SV_EINVAL, "unknown precision");
    uint64_t seen = 0;
    for (int j = 0; j < k; ++j) {
        if (qubits[j] < 0 || qubits[j] >= h->n) return fail(SV_EINVAL, "qubit outside [0, n)");
        if (seen & (1ull << qubits[j])) return fail(SV_EINVAL, "duplicate qubits");
        seen |= 1ull << qubits[j];
    }
    const int D = 1 << k;
    for (int i = 0; i < 2 * D * D; ++i)
        if (!std::isfinite(U[i])) return fail(SV_EINVAL, "matrix entry is not finite");
    if (prec != SV_PREC_NATIVE && h->dtype != SV_C64)
        return fail(SV_EUNSUPPORTED, "FP32 and split-BF16 blocks need a complex64 state");
    Block B;
    B.k = k;
    for (int j = 0; j < k; ++j) B.q[j] = qubits[j];
    B.M.resize((size_t)D * D);
    for (int i = 0; i < D * D; ++i) B.M[i] = {U[2 * i], U[2 * i + 1]};
    std::vector<FusedPass> fps = compile_fused(h, std::vector<Block>{B}, prec);
    return run_fused_passes(h, fps);
}

int sv_fuse(int n_qubits, const sv_op *ops, int n_ops, const double *params, int n_params,
            int k_max, int max_blocks, int *block_k, int *block_qubits, double *block_mats,
            int *block_gates, int *n_blocks) {
    if (n_qubits < 1 || n_qubits > 40) return fail(SV_EINVAL, "n_qubits must be in [1, 40]");
    if (k_max < 1 || k_max > 5) return fail(SV_EINVAL, "k_max must be in [1, 5]");
    if (!n_blocks || max_blocks < 0 || (max_blocks > 0 && (!block_k || !block_qubits || !block_mats || !block_gates)))
        return fail(SV_EINVAL, "NULL output");
    std::vector<Gate> gs;
    int rc = parse_ops(nullptr, n_qubits, ops, n_ops, params, n_params, gs);
    if (rc) return rc;
    for (const Gate &g : gs)
        if (__builtin_popcountll(g.qmask()) > k_max)
            return fail(SV_EINVAL, "a gate touches more qubits than k_max");
    std::vector<Block> bs = fuse(gs, k_max);
    *n_blocks = (int)bs.size();
    if ((int)bs.size() > max_blocks) return fail(SV_EINVAL, "more blocks than max_blocks");
    for (size_t b = 0; b < bs.size(); ++b) {
        const Block &B = bs[b];
        const int D = 1 << B.k;
        block_k[b] = B.k;
        block_gates[b] = B.n_gates;
        for (int j = 0; j < 5; ++j) block_qubits[b * 5 + j] = j < B.k ? B.q[j] : -1;
        double *m = block_mats + b * 2 * 32 * 32;
        for (int i = 0; i < D * D; ++i) {
            m[2 * i] = B.M[i].real();
            m[2 * i + 1] = B.M[i].imag();
        }
    }
    return SV_OK;
}

int sv_schedule(int n_qubits, int dtype, const sv_op *ops, int n_ops, const double *params, int n_params,
                int level, int max_passes, int *gate_pass, uint64_t *pass_qubits, int *n_passes) {
    if (n_qubits < 1 || n_qubits > 40) return fail(SV_EINVAL, "n_qubits must be in [1, 40]");
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "dtype must be SV_C64 or SV_C128");
    if (level < -1 || level > 2) return fail(SV_EINVAL, "level must be in [-1, 2]");
    if (!n_passes || max_passes < 0 || (n_ops > 0 && !gate_pass) || (max_passes > 0 && !pass_qubits))
        return fail(SV_EINVAL, "NULL output");
    std::vector<Gate> gs;
    int rc = parse_ops(nullptr, n_qubits, ops, n_ops, params, n_params, gs);
    if (rc) return rc;
    const int mmax = plain_tile_qubits(n_qubits, dtype), lmin = plain_low_qubits(n_qubits, dtype);
    const int lv = level < 0 ? lookahead_level_for(n_qubits, dtype) : level;
    const std::vector<Pass> passes = schedule(gs, n_qubits, mmax, lmin, true, lv);
    *n_passes = (int)passes.size();
    if ((int)passes.size() > max_passes) return fail(SV_EINVAL, "more passes than max_passes");
    for (size_t pi = 0; pi < passes.size(); ++pi) {
        const Pass &p = passes[pi];
        uint64_t needed = 0;
        for (int gi : p.gates) {
            gate_pass[gi] = (int)pi;
            needed |= tile_need(gs[(size_t)gi]);
        }
        // the tile run_gates builds for the pass, or 0 for a single gate it streams
        const bool tiled = p.gates.size() > 1 || (p.gates.size() == 1 && needs_tile(dtype, gs[(size_t)p.gates[0]]));
        TileSpec sp{};
        if (tiled) tile_layout(n_qubits, mmax, lmin, needed, &sp);
        pass_qubits[pi] = tiled ? tile_qubits(sp) : 0;
    }
    return SV_OK;
}

int sv_run_fused(sv_handle h, const sv_op *ops, int n_ops, const double *params, int n_params,
                 int k_max, int prec, int *n_blocks_out) {
    if (!h) return fail(SV_EINVAL, "NULL handle");
    if (k_max < 1 || k_max > 5) return fail(SV_EINVAL, "k_max must be in [1, 5]");
    if (prec != SV_PREC_NATIVE && prec != SV_PREC_FP32 && prec != SV_PREC_SPLIT_BF16)
        return fail(SV_EINVAL, "unknown precision");
    std::vector<Gate> gs;
    int rc = parse_ops(h, h->n, ops, n_ops, params, n_params, gs);
    if (rc) return rc;
    const int kk = std::min(k_max, h->n);
    for (const Gate &g : gs)
        if (__builtin_popcountll(g.qmask()) > kk)
            return fail(SV_EINVAL, "a gate touches more qubits than k_max");
    int nb = 0;
    std::vector<FusedPass> fps = compile_fused_gates(h, gs, kk, prec, &nb);
    if ((rc = run_fused_passes(h, fps))) return rc;
    if (n_blocks_out) *n_blocks_out = nb;
    return SV_OK;
}

int sv_fused_tune(sv_handle h, const sv_op *ops, int n_ops, const double *params, int n_params, int k_max,
                  int prec_mask, int reps, int *k_out, int *prec_out, double *ms_out) {
    if (!h || !k_out || !prec_out) return fail(SV_EINVAL, "NULL argument");
    if (k_max < 0 || k_max > 5) return fail(SV_EINVAL, "k_max must be in [0, 5]");
    if (reps < 1) reps = 1;
    std::vector<Gate> gs;
    int rc = parse_ops(h, h->n, ops, n_ops, params, n_params, gs);
    if (rc) return rc;
    int widest = 1;
    for (const Gate &g : gs) widest = std::max(widest, __builtin_popcountll(g.qmask()));
    // candidates: plain tile passes (k = 0), then fused widths 4 and 5 in
    // the allowed arithmetic (complex64: FP32 and split-BF16 matrix cores;
    // complex128: its own precision)
    std::vector<std::pair<int, int>> cand{{0, SV_PREC_NATIVE}};
    const std::vector<int> precs = h->dtype == SV_C64 ? std::vector<int>{SV_PREC_FP32, SV_PREC_SPLIT_BF16}
                                                      : std::vector<int>{SV_PREC_NATIVE};
    for (int k = 4; k <= std::min(k_max, std::min(h->n, 5)); ++k)
        for (int p : precs)
            if (((prec_mask >> p) & 1) && widest <= k) cand.push_back({k, p});
    // every candidate starts from the handle's present state, kept in a copy
    const size_t bytes = (size_t)state_bytes(h);
    size_t free_b = 0, total_b = 0;
    SV_HIP(hipMemGetInfo(&free_b, &total_b));
    if (bytes + (64u << 20) > free_b) return fail(SV_ENOMEM, "no room for a copy of the state");
    void *saved = nullptr;
    SV_HIP(hipMalloc(&saved, bytes));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rc = SV_OK;
    double best = 1e300;
    int bk = 0, bp = SV_PREC_NATIVE;
    auto run_one = [&](int k, int p) -> int {
        if (k == 0) return run_gates(h, gs, SV_RUN_TILED);
        int nb = 0;
        std::vector<FusedPass> fps = compile_fused_gates(h, gs, k, p, &nb);
        return run_fused_passes(h, fps);
    };
    hipError_t e = hipMemcpyAsync(saved, h->amps, bytes, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) rc = hip_fail(e, "sv_fused_tune");
    for (size_t c = 0; c < cand.size() && !rc; ++c) {
        double t_min = 1e300;
        for (int r = 0; r <= reps && !rc; ++r) { // the first run is untimed (warm-up)
            e = hipMemcpyAsync(h->amps, saved, bytes, hipMemcpyDeviceToDevice, h->stream);
            if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
            if (e != hipSuccess) { rc = hip_fail(e, "sv_fused_tune"); break; }
            if ((rc = run_one(cand[c].first, cand[c].second))) break;
            float ms = 0.0f;
            e = hipEventRecord(e1, h->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) { rc = hip_fail(e, "sv_fused_tune"); break; }
            if (r > 0) t_min = std::min(t_min, (double)ms);
        }
        if (!rc && t_min < best) {
            best = t_min;
            bk = cand[c].first;
            bp = cand[c].second;
        }
    }
    if (!rc) {
        e = hipMemcpyAsync(h->amps, saved, bytes, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) rc = hip_fail(e, "sv_fused_tune");
    } else {
        (void)hipMemcpyAsync(h->amps, saved, bytes, hipMemcpyDeviceToDevice, h->stream);
        (void)hipStreamSynchronize(h->stream);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(saved);
    if (rc) return rc;
    *k_out = bk;
    *prec_out = bp;
    if (ms_out) *ms_out = best;
    return SV_OK;
}

int sv_adjoint_grad(sv_handle h, sv_handle lam, const sv_op *ops, int n_ops, const double *params,
                    int n_params, int n_terms, const uint64_t *z_masks, const double *coeffs,
                    double *host_loss, double *host_grad) {
    if (!h || !lam) return fail(SV_EINVAL, "NULL handle");
    if (h == lam || h->amps == lam->amps) return fail(SV_EINVAL, "work handle must be distinct");
    if (h->n != lam->n || h->dtype != lam->dtype) return fail(SV_EINVAL, "work handle differs in size or dtype");
    if (n_terms < 1 || n_terms > kMaxTerms) return fail(SV_EINVAL, "n_terms must be in [1, 64]");
    if (!z_masks || !coeffs || !host_loss) return fail(SV_EINVAL, "NULL argument");
    if (n_params < 0 || (n_params > 0 && (!params || !host_grad))) return fail(SV_EINVAL, "bad parameter vector");
    for (int j = 0; j < n_terms; ++j)
        if (h->n < 64 && (z_masks[j] >> h->n) != 0) return fail(SV_EINVAL, "Z mask has bits >= n");
    std::vector<Gate> gs;
    int rc = parse_ops(h, h->n, ops, n_ops, params, n_params, gs);
    if (rc) return rc;
    int n_param_gates = 0;
    for (int i = 0; i < n_ops; ++i) {
        if (ops[i].param_index < 0) continue;
        double M[8], f;
        if (ops[i].kind == SV_GATE_MATRIX || !probe_of(ops[i].kind, M, &f))
            return fail(SV_EINVAL, "op " + std::to_string(i) + ": only RX RY RZ U1 can carry a parameter");
        ++n_param_gates;
    }
    // reverse list: undo of every gate (last first), parametrised ones with a probe
    std::vector<Gate> rev;
    std::vector<Probe> probes_store;
    std::vector<int> rev_param;   // param_index of each reversed gate, -1 if fixed
    std::vector<double> rev_factor;
    rev.reserve(gs.size());
    probes_store.reserve(gs.size());
    for (int g = n_ops - 1; g >= 0; --g) {
        rev.push_back(dagger(gs[g]));
        rev_param.push_back(ops[g].param_index);
        double M[8] = {0, 0, 0, 0, 0, 0, 0, 0}, f = 0.0;
        if (ops[g].param_index >= 0) probe_of(ops[g].kind, M, &f);
        rev_factor.push_back(f);
        Probe pr{};
        std::memcpy(pr.M, M, sizeof(M));
        probes_store.push_back(pr);
    }
    const int mmax = std::min(h->n, adjoint_tile_qubits(h->dtype));
    const int lmin = std::min(h->n, h->dtype == SV_C64 ? 7 : 6);
    const int B = (int)std::min<uint64_t>((uint64_t)adjoint_blocks(), 1ull << (h->n - mmax));
    std::vector<Pass> passes = schedule(rev, h->n, mmax, lmin);
    // split passes holding more parametrised gates than one launch accumulates
    std::vector<Pass> split;
    for (const Pass &p : passes) {
        Pass cur;
        int np = 0;
        for (int gi : p.gates) {
            if (rev_param[gi] >= 0 && np == kMaxAdjSlots) {
                split.push_back(cur);
                cur = Pass{};
                np = 0;
            }
            cur.gates.push_back(gi);
            if (rev_param[gi] >= 0) ++np;
        }
        if (!cur.gates.empty()) split.push_back(cur);
    }
    // compile: slots numbered globally in sweep order
    std::vector<PassCode> code(split.size());
    std::vector<int> slot0(split.size()), nslot(split.size());
    std::vector<int> slot_param, slot_rev;
    std::vector<size_t> offs(split.size());
    size_t total = 0;
    for (size_t pi = 0; pi < split.size(); ++pi) {
        uint64_t needed = 0;
        std::vector<const Gate *> ptrs;
        std::vector<const Probe *> prs;
        slot0[pi] = (int)slot_param.size();
        int ns = 0;
        for (int gi : split[pi].gates) {
            needed |= rev[gi].tmask();
            ptrs.push_back(&rev[gi]);
            if (rev_param[gi] >= 0) {
                probes_store[gi].slot = ns++;
                prs.push_back(&probes_store[gi]);
                slot_param.push_back(rev_param[gi]);
                slot_rev.push_back(gi);
            } else {
                prs.push_back(nullptr);
            }
        }
        nslot[pi] = ns;
        TileSpec sp{};
        tile_layout(h->n, mmax, lmin, needed, &sp);
        code[pi] = compile_pass(sp, ptrs, sweep_width(h->dtype), h->dtype == SV_C64, &prs);
        offs[pi] = total;
        total += align256(code[pi].bytes());
    }
    const size_t n_slots = slot_param.size();
    const size_t loss_n = (size_t)adjoint_blocks();
    if ((rc = ensure_scratch(h, loss_n + n_slots * B + 1 + n_slots))) return rc;
    double *partials = h->d_scratch;                       // loss partials, then slot partials
    double *sums = h->d_scratch + loss_n + n_slots * B;    // loss, then one sum per slot
    hipStream_t saved = lam->stream;
    SV_HIP(hipStreamSynchronize(saved));
    lam->stream = h->stream; // every launch of the sweep is ordered on h's stream
    auto restore = [&](int code_) {
        lam->stream = saved;
        return code_;
    };
    {
        Timed tm(h, K_ADJOINT, 2.0 * state_bytes(h));
        hipError_t e = launch_adjoint_init(h->amps, lam->amps, h->n, h->dtype, n_terms, z_masks, coeffs,
                                           partials, h->stream);
        if (e != hipSuccess) return restore(hip_fail(e, "launch_adjoint_init"));
    }
    if (total) {
        if ((rc = ensure_arena(h, total))) return restore(rc);
        if ((rc = stage_wait(h))) return restore(rc);
        for (size_t pi = 0; pi < split.size(); ++pi) stage_pass(h, code[pi], offs[pi]);
        if ((rc = upload_arena(h, total))) return restore(rc);
    }
    for (size_t pi = 0; pi < split.size(); ++pi) {
        const PassCode &pc = code[pi];
        const TileSweep *sw = reinterpret_cast<const TileSweep *>(h->d_arena + offs[pi]);
        const char *gt = h->d_arena + offs[pi] + align256(pc.sweeps.size() * sizeof(TileSweep));
        Timed tm(h, K_ADJOINT, 4.0 * state_bytes(h), pc.flops_per_amp * (double)(1ull << h->n));
        hipError_t e = launch_adjoint_tile(h->amps, lam->amps, h->n, h->dtype, pc.sp, sw, (int)pc.sweeps.size(), gt,
                                           slot0[pi], nslot[pi], partials + loss_n, B, pc.two_qubit, h->stream);
        if (e != hipSuccess) return restore(hip_fail(e, "launch_adjoint_tile"));
    }
    hipError_t e = launch_sum_slots(partials, 1, (int)loss_n, sums, h->stream);
    if (e == hipSuccess) e = launch_sum_slots(partials + loss_n, (int)n_slots, B, sums + 1, h->stream);
    if (e != hipSuccess) return restore(hip_fail(e, "launch_sum_slots"));
    std::vector<double> out(n_slots + 1);
    e = hipMemcpyAsync(out.data(), sums, out.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return restore(hip_fail(e, "adjoint result copy"));
    *host_loss = out[0];
    for (int p = 0; p < n_params; ++p) host_grad[p] = 0.0;
    for (size_t sl = 0; sl < n_slots; ++sl) host_grad[slot_param[sl]] += rev_factor[slot_rev[sl]] * out[sl + 1];
    return restore(SV_OK);
}

int sv_batch_create(int n_circuits, const int *widths, const int64_t *op_offsets, const sv_op *ops,
                    const double *params, int n_params, int dtype, uint64_t z_mask, int flags,
                    void *hip_stream, sv_batch_handle *out) {
    if (!out) return fail(SV_EINVAL, "NULL output handle");
    *out = nullptr;
    if (n_circuits < 1 || !widths || !op_offsets) return fail(SV_EINVAL, "bad batch description");
    if (dtype != SV_C64 && dtype != SV_C128) return fail(SV_EINVAL, "dtype must be SV_C64 or SV_C128");
    const int wmin = sweep_width(dtype);
    if (op_offsets[0] != 0) return fail(SV_EINVAL, "op_offsets[0] must be 0");
    if (op_offsets[n_circuits] > 0 && !ops) return fail(SV_EINVAL, "NULL ops");
    int wmax = 0;
    for (int i = 0; i < n_circuits; ++i) {
        if (widths[i] < wmin || widths[i] > 30)
            return fail(SV_EINVAL, "circuit width outside [" + std::to_string(wmin) + ", 30]");
        if (op_offsets[i + 1] < op_offsets[i]) return fail(SV_EINVAL, "op_offsets must not decrease");
        wmax = std::max(wmax, widths[i]);
    }
    if (wmax < 64 && (z_mask >> wmax) != 0) return fail(SV_EINVAL, "Z mask has bits beyond every width");
    sv_batch *b = new sv_batch();
    b->n = n_circuits;
    b->dtype = dtype;
    b->flags = flags;
    b->zmask = z_mask;
    b->stream = (hipStream_t)hip_stream;
    b->widths.assign(widths, widths + n_circuits);
    b->circ.resize(n_circuits);
    for (int i = 0; i < n_circuits; ++i) {
        std::vector<Gate> &gs = b->circ[i];
        const int64_t lo = op_offsets[i], hi = op_offsets[i + 1];
        gs.resize((size_t)(hi - lo));
        for (int64_t j = lo; j < hi; ++j) {
            const int rc = op_to_gate(widths[i], ops[j], params, n_params, &gs[(size_t)(j - lo)]);
            if (rc) {
                delete b;
                return fail(rc, "circuit " + std::to_string(i) + " op " + std::to_string(j - lo) + ": " + g_last_error);
            }
        }
    }
    hipError_t e;
    if ((e = hipMalloc((void **)&b->d_out, sizeof(double) * n_circuits)) != hipSuccess ||
        (e = hipMalloc((void **)&b->d_counter, 256)) != hipSuccess) {
        sv_batch_free(b);
        return hip_fail(e, "sv_batch_create");
    }
    const int rc = batch_prepare(b, batch_tile_qubits(dtype), sweep_width(dtype), 2 * device_cus(), 0);
    if (rc) {
        const std::string msg = g_last_error;
        sv_batch_free(b);
        return fail(rc, msg);
    }
    *out = b;
    return SV_OK;
}

int sv_batch_run(sv_batch_handle b) {
    if (!b || !b->exec) return fail(SV_EINVAL, "NULL or unprepared batch");
    SV_HIP(hipGraphLaunch(b->exec, b->stream));
    return SV_OK;
}

int sv_batch_results(sv_batch_handle b, double *host_out) {
    if (!b || !host_out) return fail(SV_EINVAL, "NULL argument");
    SV_HIP(hipMemcpyAsync(host_out, b->d_out, sizeof(double) * b->n, hipMemcpyDeviceToHost, b->stream));
    SV_HIP(hipStreamSynchronize(b->stream));
    return SV_OK;
}

void *sv_batch_output(sv_batch_handle b) { return b ? b->d_out : nullptr; }

int sv_batch_state(sv_batch_handle b, int i, void *host_out) {
    if (!b || !host_out || i < 0 || i >= b->n) return fail(SV_EINVAL, "bad argument");
    if (!(b->flags & SV_BATCH_KEEP_STATES)) return fail(SV_EINVAL, "batch was created without SV_BATCH_KEEP_STATES");
    const size_t bytes = ((size_t)1 << b->widths[i]) * (b->dtype == SV_C64 ? 8 : 16);
    SV_HIP(hipStreamSynchronize(b->stream));
    SV_HIP(hipMemcpy(host_out, (char *)b->d_states + b->state_off[i], bytes, hipMemcpyDeviceToHost));
    return SV_OK;
}

int sv_batch_tune(sv_batch_handle b, int reps, int *tile_m, int *sweep_w, int *grid, int *fuse_w,
                  double *best_ms) {
    if (!b) return fail(SV_EINVAL, "NULL batch");
    if (reps < 1) reps = 1;
    const int cus = device_cus();
    const int mtop = batch_tile_qubits(b->dtype);
    const int ws[2] = {3, 4};
    const int ms[3] = {mtop, mtop - 1, mtop - 2};
    const int gs[2] = {cus, 2 * cus};
    double best = 1e300;
    int bm = mtop, bw = sweep_width(b->dtype), bg = 2 * cus, bf = 0;
    hipEvent_t e0, e1;
    SV_HIP(hipEventCreate(&e0));
    SV_HIP(hipEventCreate(&e1));
    int rc = SV_OK;
    const int wnarrow = *std::min_element(b->widths.begin(), b->widths.end());
    for (int fw = 0; fw <= 2 && !rc; ++fw)
    for (int wi = 0; wi < 2 && !rc; ++wi)
        for (int mi = 0; mi < 3 && !rc; ++mi)
            for (int gi = 0; gi < 2 && !rc; ++gi) {
                // sweeps wider than the narrowest circuit are not candidates
                if (ws[wi] > wnarrow) continue;
                if ((rc = batch_prepare(b, ms[mi], ws[wi], gs[gi], fw))) break;
                float ms_run = 0.0f;
                hipError_t e = hipEventRecord(e0, b->stream);
                for (int r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(b->exec, b->stream);
                if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e == hipSuccess) e = hipEventElapsedTime(&ms_run, e0, e1);
                if (e != hipSuccess) {
                    rc = hip_fail(e, "sv_batch_tune");
                    break;
                }
                const double t = ms_run / reps;
                if (t < best) {
                    best = t;
                    bm = ms[mi];
                    bw = ws[wi];
                    bg = gs[gi];
                    bf = fw;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if ((rc = batch_prepare(b, bm, bw, bg, bf))) return rc;
    if (tile_m) *tile_m = bm;
    if (sweep_w) *sweep_w = bw;
    if (grid) *grid = bg;
    if (fuse_w) *fuse_w = bf;
    if (best_ms) *best_ms = best;
    return SV_OK;
}

int sv_batch_config(sv_batch_handle b, int tile_m, int sweep_w, int grid, int fuse_w) {
    if (!b) return fail(SV_EINVAL, "NULL batch");
    const int mtop = batch_tile_qubits(b->dtype);
    if (tile_m < mtop - 2 || tile_m > mtop) return fail(SV_EINVAL, "tile qubits outside the tuner's range");
    if (sweep_w != 3 && sweep_w != 4) return fail(SV_EINVAL, "sweep width must be 3 or 4");
    if (grid < 1 || grid > 64 * device_cus()) return fail(SV_EINVAL, "grid outside [1, 64 per CU]");
    if (fuse_w < 0 || fuse_w > 2) return fail(SV_EINVAL, "fusion width must be 0, 1 or 2");
    return batch_prepare(b, tile_m, sweep_w, grid, fuse_w);
}

int sv_batch_free(sv_batch_handle b) {
    if (!b) return fail(SV_EINVAL, "NULL batch");
    (void)hipStreamSynchronize(b->stream);
    batch_release_program(b);
    if (b->d_out) (void)hipFree(b->d_out);
    if (b->d_counter) (void)hipFree(b->d_counter);
    delete b;
    return SV_OK;
}

} // extern "C"
