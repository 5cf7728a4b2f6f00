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
// (high) tile qubit.
enum TileGateKind : int32_t { TG_1Q = 1, TG_2Q = 2, TG_DIAG = 3 };
struct TileGate {
    int32_t kind;
    int32_t b0, b1;    // local target bits (b1 unused for 1q)
    uint32_t cin;      // control bits inside the tile (local positions)
    uint64_t cout;     // control bits outside the tile (global positions)
    double m[32];      // 1q: 4 complex, 2q: 16 complex, diag: d0, d1 (2 complex)
};

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
hipError_t launch_tile(void *amps, int n, int dtype, const TileSpec &spec, const TileGate *dev_gates,
                       int n_gates, hipStream_t s);
int tile_max_qubits(int dtype);
hipError_t launch_dense(void *amps, int n, int dtype, const TileSpec &sp, int k, const int *qubits,
                        const void *dev_mat, int prec, hipStream_t s);
int fused_tile_qubits(int dtype);

hipError_t launch_probabilities(const void *amps, int n, int dtype, void *dev_out,
                                double *dev_partials, int n_partials, double *dev_total,
                                hipStream_t s);
constexpr int kMaxTerms = 64;
hipError_t launch_expectation(const void *amps, int n, int dtype, int n_terms,
                              const uint64_t *masks, const double *coeffs, double *dev_partials,
                              int n_partials, double *dev_total, hipStream_t s);
constexpr int kReduceBlocks = 1024;

int adjoint_blocks();
hipError_t launch_adjoint_init(const void *psi, void *lam, int n, int dtype, int n_terms,
                               const uint64_t *masks, const double *coeffs, double *partials,
                               hipStream_t s);
hipError_t launch_adjoint_param(void *psi, void *lam, int n, int dtype, int t, uint64_t ctrl,
                                const double *udag, const double *probe, double *partials,
                                hipStream_t s);
hipError_t launch_sum_slots(const double *partials, int n_slots, int n_blocks, double *out,
                            hipStream_t s);

} // namespace sv
