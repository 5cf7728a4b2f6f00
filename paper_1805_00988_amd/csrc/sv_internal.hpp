// Internal definitions shared by the translation units of libsv.so.
// Device-side complex arithmetic, gate records for on-chip tile passes and
// the launcher prototypes the host API dispatches to.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/sv.h"

namespace sv {

// ---------------------------------------------------------------- complex
template <typename T>
struct cpx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}

// a*b + c
template <typename T>
__device__ __forceinline__ cpx<T> cfma(cpx<T> a, cpx<T> b, cpx<T> c) {
    return {fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}

template <typename T>
__device__ __forceinline__ T norm2(cpx<T> a) {
    return fma(a.re, a.re, a.im * a.im);
}

// 2x2 gate by value (kernel argument), row-major [[m0, m1], [m2, m3]].
template <typename T>
struct Mat2 {
    cpx<T> m[4];
};

template <typename T>
struct Mat4 {
    cpx<T> m[16];
};

// ------------------------------------------------- nontemporal accesses
// 16-byte loads and stores for kernels that touch every byte of the state
// once per launch (streamed gates, reductions): marked nontemporal so they
// do not displace reusable lines in the caches (measured 5-10 % faster for
// the in-place update and read-only streams of a 32 GiB state).
typedef float f32x4_nt __attribute__((ext_vector_type(4)));
typedef double f64x2_nt __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float4 ld_nt(const float4 *p) {
    const f32x4_nt v = __builtin_nontemporal_load(reinterpret_cast<const f32x4_nt *>(p));
    return float4{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ double2 ld_nt(const double2 *p) {
    const f64x2_nt v = __builtin_nontemporal_load(reinterpret_cast<const f64x2_nt *>(p));
    return double2{v.x, v.y};
}
__device__ __forceinline__ void st_nt(float4 *p, float4 v) {
    const f32x4_nt w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<f32x4_nt *>(p));
}
__device__ __forceinline__ void st_nt(double2 *p, double2 v) {
    const f64x2_nt w = {v.x, v.y};
    __builtin_nontemporal_store(w, reinterpret_cast<f64x2_nt *>(p));
}

// ------------------------------------------------------ index enumeration
// Positions (ascending) at which a zero bit is inserted into an enumeration
// index, and the bits OR-ed in afterwards.  This maps a dense counter onto
// the set of indices that have fixed values in those positions.
constexpr int kMaxInsert = 10;
struct Enum {
    int n_pos;
    int pos[kMaxInsert];
    uint64_t set;   // bits forced to 1 after insertion (control bits)
    uint64_t check; // further control bits, checked instead of enumerated
};

__device__ __forceinline__ uint64_t insert_zero(uint64_t i, int p) {
    const uint64_t low = (1ull << p) - 1ull;
    return (i & low) | ((i & ~low) << 1);
}

__device__ __forceinline__ uint64_t expand(const Enum &e, uint64_t i) {
    for (int k = 0; k < e.n_pos; ++k) i = insert_zero(i, e.pos[k]);
    return i | e.set;
}

// ------------------------------------------------------ tile-pass records
// A gate applied inside an on-chip tile.  Local bit positions refer to the
// tile's own index: bits [0, L) are qubits 0..L-1, bit L+i is the i-th extra
// (high) tile qubit.  Within a sweep (see tile_sweep.hpp) b0/b1 are positions
// among the sweep's register qubits, except for SK_DIAG, where b0 is the
// target's local bit.
enum SweepKind : int32_t {
    SK_GEN = 1,   // general 2x2 on sweep position b0
    SK_REAL = 2,  // real 2x2 (m[0], m[2], m[4], m[6] hold the entries)
    SK_DIAG = 3,  // diag(d0, d1) on tile bit b0 outside the registers; m: d0, d1
    SK_SWAP = 4,  // X: exchange the pair (per-lane controls: complex64 only)
    SK_2Q = 5,    // 4x4 on sweep positions b0 < b1 (bit 0 of the matrix index <-> b0)
    SK_PARAM = 6, // adjoint sweep: add Im<lam|M|psi> for M (entries 0-3) on position b0
                  // to slot b1; the undo of the gate follows as its own record
    SK_DIAGR = 7, // diag(d0, d1) on sweep position b0; m: d0, d1
    SK_RIMAG = 8, // 2x2 on sweep position b0 with real diagonal and imaginary
                  // off-diagonal entries (RX, Y); m: the four complex entries
    SK_PHASE = 9, // b1 phases gathered into a per-lane factor: the record's
                  // entries are (uint64 condition outside the tile, complex phase);
                  // the product of the phases whose condition holds for the tile
                  // multiplies slot b0 (sweep position p: the amplitudes with
                  // register bit p set, or W: all) in lanes whose group holds
                  // 'lane'; amask 1
    SK_FLUSH = 10, // multiply every amplitude by its gathered factors (slot W for
                   // all, slot p for those with register bit p) and reset the
                   // slots in amask
    // SK_PARAM for the probes of the rotations and the phase gate: M is
    // Pauli X, Y, Z or the projector |1><1|, whose Im<lam|M|psi> over a
    // pair needs two to four products instead of a 2x2 product (no matrix)
    SK_PROBE_X = 11,
    SK_PROBE_Y = 12,
    SK_PROBE_Z = 13,
    SK_PROBE_P1 = 14,
    // phases gathered as SK_PHASE, taken from tables: kPtabWindows windows
    // of consecutive global index bits, described in the kPtabDesc bytes
    // after the head by (uint32 shift, mask, byte offset, unused); the
    // tables follow, the first entry of that area being 1 (the table of an
    // unused window: shift 0, mask 0, offset 0); the tile's factor is the
    // product over the windows of the entry at offset + ((base >> shift) &
    // mask) entries; b1 counts the windows used; slot b0, 'lane' and amask
    // as SK_PHASE
    SK_PTAB = 15,
    // phases on lane bits (complex128 streams only): b1 entries of (uint64
    // tile-bit mask of one bit, complex phase) laid out as SK_PHASE's; a
    // lane's factor is the product of the phases whose bit its group holds;
    // slot b0, amask 1
    SK_LPH = 16
};
constexpr int kPtabBits = 6;    // widest window of a phase table
// windows per SK_PTAB record (four would hold more scalar registers than
// the tile kernels can spare without spilling more of them)
constexpr int kPtabWindows = 2;
constexpr int kPtabDesc = 16 * kPtabWindows; // descriptor bytes after the record head
// Controls inside the tile are split by where they sit in the sweep: bits
// on tile positions outside the registers ('lane') are constant over one
// lane's group and tested per lane; bits on register positions only select
// register indices and are folded, with the gate's own pattern, into
// 'amask': bit j is set for every register index j the record starts an
// update at (the low index of each pair or quad whose controls hold; for a
// diagonal gate every amplitude whose factor can differ from 1).
// On the device the records of a pass form one packed byte stream: each is
// this layout cut after the matrix entries its kind reads (record_entries),
// 'size' bytes long, so that a pass's records stay in the scalar data cache
// while every wave walks them; the stream ends with kRecordTail zero bytes
// (the record head is read as one 96-byte block).
struct TileGate {
    int32_t kind;
    int32_t b0, b1;
    uint32_t lane;     // control bits on tile positions outside the registers
    uint32_t amask;    // register indices updated (see above)
    int32_t size;      // bytes of the packed record
    uint64_t cout;     // control bits outside the tile (global positions)
    double m[32];      // matrix entries, complex interleaved: FP64, or FP32 packed into
                       // the first half of the storage for complex64 states
};
constexpr int kRecordHead = 32, kRecordTail = 96;

constexpr int kSweepW = 4; // tile qubits held in registers per sweep (fewer for tiny tiles)
struct TileSweep {
    int32_t n_gates;       // records of this sweep, stored consecutively
    int32_t qpos[kSweepW]; // ascending local positions held in registers
    int32_t rec_off;       // byte offset of its first record in the pass's stream
    int32_t pad[2];
};

// LDS swizzle of a tile index, linear over XOR (and its own inverse): the
// positions within one 128-byte LDS row (16 complex64 or 8 complex128
// amplitudes) are XOR-ed with a fold of the higher index bits, so lanes
// whose amplitudes differ in arbitrary tile bits spread over the banks.
// The shifts were chosen with a bank-conflict model of a sweep's register
// groups over every set of register positions (64 banks, 32-lane phases):
// 3.2 LDS cycles per access on average for complex64 and 5.0 for
// complex128, against 4.1 and 5.7 for shifts (s, 2s, 3s).
__host__ __device__ inline uint32_t lds_swizzle(uint32_t l, int amp_bytes) {
    if (amp_bytes == 8) return l ^ (((l >> 4) ^ (l >> 5) ^ (l >> 7)) & 15u);
    return l ^ (((l >> 3) ^ (l >> 4) ^ (l >> 5)) & 7u);
}

constexpr int kMaxTileHigh = 8; // extra tile qubits beyond the low block
struct TileSpec {
    int L;                    // low qubits 0..L-1 are in the tile
    int K;                    // number of extra high qubits
    int high[kMaxTileHigh];   // ascending
};

// --------------------------------------------------------------- status
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

// ------------------------------------------------------------ launchers
// All return hipError_t of the launch.  'amps' is the state buffer.
hipError_t launch_init_basis(void *amps, int n, int dtype, uint64_t x, hipStream_t s);
hipError_t launch_gate1(void *amps, int n, int dtype, int t, uint64_t ctrl, const double *U,
                        hipStream_t s);
hipError_t launch_gate2(void *amps, int n, int dtype, int t0, int t1, uint64_t ctrl,
                        const double *U, hipStream_t s);
hipError_t launch_scale(void *amps, int n, int dtype, uint64_t set_mask, const double *factor,
                        hipStream_t s);
// two_qubit: the pass holds SK_2Q records (selects the kernel instance with that
// path).  direct: kDirectFirst / kDirectLast let the first sweep read its
// register groups straight from the state / the last sweep write them straight
// back instead of staging the tile through LDS (worth it when the sweep's
// register positions leave the lowest tile bits to the lanes, so that a
// wave's accesses stay contiguous).
constexpr uint32_t kDirectFirst = 1, kDirectLast = 2;
hipError_t launch_tile(void *amps, int n, int dtype, const TileSpec &spec, const TileSweep *dev_sweeps,
                       int n_sweeps, const char *dev_recs, bool two_qubit, bool lane_phases, uint32_t direct,
                       hipStream_t s);
int tile_max_qubits(int dtype);
int tile_launch_qubits(int dtype);
int batch_tile_qubits(int dtype);
int sweep_width(int dtype);
// Dense blocks of a fused tile pass: positions of the block's qubits in the
// tile (bit j of the matrix index <-> qpos[j]) and of the remaining tile bits
// (group index), and the byte offset of the block's operand (the matrix in
// the state's precision, or MFMA operand fragments) from the pass's base.
struct BlockPos {
    int k;
    int qpos[6];
    int gpos[16];
    int ng;
};
// tab_off: byte offset of the block's LDS offset tables (matrix cores only):
// uint32 qoff[2^k] = swizzled LDS offset of matrix index j deposited at
// qpos, then goff_lo[R] and goff_hi[2^(m-k) / R] = the same for group index
// g (g < R) and g = w * R deposited at gpos, R the kernel's MFMA rows.  The
// maps are linear over XOR, so the offset of (group w*R + i, index j) is
// goff_hi[w] ^ goff_lo[i] ^ qoff[j].  gtab_off: the same three tables as
// uint64 global index offsets from the tile's base (OR-combined), for the
// blocks that read or write the state directly.
// vmask: qubits outside the tile on which the block's matrix depends (the
// diagonal gates fused into it may act on qubits the tile does not hold;
// within one tile those qubits are fixed, so the gate reduces to a diagonal
// on the block's own qubits).  The operand of variant v, bit i of v = value
// of the i-th lowest qubit of vmask in the tile's base index, starts at
// op_off + v * vstride.
constexpr int kMaxVariantQubits = 4;
struct DenseBlock {
    BlockPos bp;
    int32_t pad;
    int64_t op_off;
    int64_t tab_off;
    int64_t gtab_off;
    uint64_t vmask;
    int64_t vstride;
};
// launch_dense_pass precision code for complex128 blocks on the FP64 matrix cores
constexpr int kPrecMfma64 = 100;
// direct (matrix cores): kDirectFirst / kDirectLast let the first block read
// the state and the last block write it without staging the tile in LDS
hipError_t launch_dense_pass(void *amps, int n, int dtype, const TileSpec &sp, int k,
                             const DenseBlock *dev_blocks, int n_blocks, const char *dev_base, int prec,
                             uint32_t direct, hipStream_t s);
int fused_tile_qubits(int dtype);
hipError_t launch_probabilities(const void *amps, int n, int dtype, void *dev_out,
                                double *dev_partials, int n_partials, double *dev_total,
                                hipStream_t s);
constexpr int kMaxTerms = 64;
hipError_t launch_expectation(const void *amps, int n, int dtype, int n_terms,
                              const uint64_t *masks, const double *coeffs, double *dev_partials,
                              int n_partials, double *dev_total, hipStream_t s);
constexpr int kReduceBlocks = 8192;
// sv_expectation on a caller's state with its partial sums in the library's
// static device array (no allocation); the same kernels and grid as
// launch_expectation with kReduceBlocks partials
hipError_t launch_expectation_static(const void *amps, int n, int dtype, int n_terms,
                                     const uint64_t *masks, const double *coeffs, double *dev_total,
                                     hipStream_t s);

// ------------------------------------------------------------- batches
struct BatchCircuit {
    int32_t w;         // qubits
    int32_t n_passes;
    int32_t pass_off;
    int32_t keep;      // store the final state
    int64_t state_off; // byte offset of the state in the batch's state buffer
};
struct BatchPass {
    TileSpec sp;
    int32_t n_sweeps;
    int32_t sweep_off;
    int32_t gate_off;      // byte offset of the pass's records in the stream
    int32_t pad;
};
struct BatchArgs {
    const BatchCircuit *circuits;
    const BatchPass *passes;
    const TileSweep *sweeps;
    const char *recs;
    const int32_t *order;
    unsigned int *counter;
    void *states;
    double *out;
    int n_circuits;
    uint64_t zmask;
};
hipError_t launch_batch(const BatchArgs &args, int dtype, int sweep_w, int tile_m, int grid, bool two_qubit,
                        hipStream_t s);

// ----------------------------------------------------------- measurement
constexpr int kMaxMeasureQubits = 6;
struct MeasurePos {
    int k;                        // measured qubits
    int pos[kMaxMeasureQubits];   // ascending; outcome bit i = qubit pos[i]
};
int marginal_blocks(int n, int dtype);
// partials[b * marginal_blocks + g]: workgroup g's sum of outcome b
hipError_t launch_marginals(const void *amps, int n, int dtype, const MeasurePos &mp, double *partials,
                            hipStream_t s);
// partials[g], marginal_blocks workgroups: sum of |psi_x|^2 over (x & mask) == want
hipError_t launch_masked_prob(const void *amps, int n, int dtype, uint64_t mask, uint64_t want,
                              double *partials, hipStream_t s);
// psi_x *= (x & mask) == want ? scale : 0
hipError_t launch_collapse(void *amps, int n, int dtype, uint64_t mask, uint64_t want, double scale,
                           hipStream_t s);
// sampling: blocks of 2^sample_block_log(n) amplitudes
int sample_block_log(int n);
hipError_t launch_block_sums(const void *amps, int n, int dtype, int block_log, double *sums, hipStream_t s);
hipError_t launch_sample_scan(const void *amps, int dtype, int block_log, int n_samples, const int64_t *blk,
                              const double *target, uint64_t *out, hipStream_t s);

int adjoint_blocks();
hipError_t launch_adjoint_init(const void *psi, void *lam, int n, int dtype, int n_terms,
                               const uint64_t *masks, const double *coeffs, double *partials,
                               hipStream_t s);
hipError_t launch_sum_slots(const double *partials, int n_slots, int n_blocks, double *out,
                            hipStream_t s);
// One tile pass of the adjoint sweep over psi and lam (both staged in LDS).
// Probes of the pass's parametrised gates accumulate per workgroup and are
// written to partials[(slot0 + i) * n_blocks + workgroup] for i < n_slots.
hipError_t launch_adjoint_tile(void *psi, void *lam, int n, int dtype, const TileSpec &spec,
                               const TileSweep *dev_sweeps, int n_sweeps, const char *dev_recs,
                               int slot0, int n_slots, double *partials, int n_blocks, bool two_qubit,
                               hipStream_t s);
int adjoint_tile_qubits(int dtype);
constexpr int kMaxAdjSlots = 128;

} // namespace sv
