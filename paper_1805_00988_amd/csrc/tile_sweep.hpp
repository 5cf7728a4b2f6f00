// Applying a run of gates to a tile of amplitudes staged in LDS.
//
// A tile holds 2^m amplitudes (local index l, m <= 13).  The gates of a pass
// are grouped by the host into sweeps: a sweep names W = 4 local qubit
// positions and a list of gates whose targets lie among them (diagonal
// gates may target any tile position).  For each sweep every thread takes
// groups of 2^W amplitudes that differ only in those positions, holds them
// in registers, applies the sweep's gates in order and writes them back, so
// the tile crosses LDS once per sweep instead of once per gate.
//
// LDS addresses are swizzled (lds_swizzle): positions within one 128-byte
// LDS row (16 complex64 or 8 complex128 amplitudes) are XOR-ed with a fold of
// the row index, so the lanes of a wave, whose groups differ in arbitrary
// tile bits, spread over the banks.
#pragma once

#include "sv_internal.hpp"

namespace sv {


template <typename T>
__device__ __forceinline__ uint32_t lds_phys(uint32_t l) {
    return lds_swizzle(l, 2 * (int)sizeof(T));
}

// ------------------------------------------------------------ tile staging
// 16-byte vectors of amplitudes: two complex64 or one complex128.
template <typename T>
struct Amp16;
template <>
struct Amp16<float> {
    using type = float4;
    static constexpr int bits = 1;
};
template <>
struct Amp16<double> {
    using type = double2;
    static constexpr int bits = 0;
};

// Offset of local amplitude l from the tile's base index: the low L bits in
// place, bit L + i at global position high[i].  The map is linear over the
// OR of parts with disjoint bits.
__device__ __forceinline__ uint64_t tile_offset(const TileSpec &sp, uint32_t l) {
    uint64_t g = l & ((1u << sp.L) - 1u);
    const uint32_t hi = l >> sp.L;
#pragma unroll
    for (int i = 0; i < kMaxTileHigh; ++i) {
        if (i >= sp.K) break;
        if ((hi >> i) & 1u) g |= 1ull << sp.high[i];
    }
    return g;
}

// Copy a tile of tsize amplitudes between the state and the swizzled LDS
// tile with NTH threads.  Thread t moves the 16-byte vectors at local index
// t*VA + r*STRIDE (VA amplitudes per vector, STRIDE = NTH*VA) for rounds r;
// U rounds are issued before any of their results is used, so a lane keeps
// U memory accesses in flight.  Both addresses split into a per-thread part
// and a wave-uniform per-round part (disjoint bits, combined by OR / XOR).
template <typename T, int NTH, int U>
__device__ __forceinline__ void tile_load(const typename Amp16<T>::type *__restrict__ v, cpx<T> *lds,
                                          const TileSpec &sp, uint64_t base, uint32_t tsize) {
    constexpr int vb = Amp16<T>::bits;
    constexpr uint32_t STRIDE = (uint32_t)NTH << vb;
    const uint32_t lt = threadIdx.x << vb;
    const uint64_t gt = base | tile_offset(sp, lt);
    const uint32_t pt = lds_phys<T>(lt);
    for (uint32_t r0 = 0; r0 < tsize; r0 += U * STRIDE) {
        typename Amp16<T>::type w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t ru = r0 + u * STRIDE;
            if (ru + lt < tsize) w[u] = v[(gt | tile_offset(sp, ru)) >> vb];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t ru = r0 + u * STRIDE;
            if (ru + lt < tsize) {
                const uint32_t p = lds_phys<T>(ru) ^ pt;
                lds[p] = cpx<T>{w[u].x, w[u].y};
                if constexpr (vb == 1) lds[p ^ 1u] = cpx<T>{w[u].z, w[u].w};
            }
        }
    }
}

template <typename T, int NTH, int U>
__device__ __forceinline__ void tile_store(typename Amp16<T>::type *__restrict__ v, const cpx<T> *lds,
                                           const TileSpec &sp, uint64_t base, uint32_t tsize) {
    constexpr int vb = Amp16<T>::bits;
    constexpr uint32_t STRIDE = (uint32_t)NTH << vb;
    const uint32_t lt = threadIdx.x << vb;
    const uint64_t gt = base | tile_offset(sp, lt);
    const uint32_t pt = lds_phys<T>(lt);
    for (uint32_t r0 = 0; r0 < tsize; r0 += U * STRIDE) {
        typename Amp16<T>::type w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t ru = r0 + u * STRIDE;
            if (ru + lt < tsize) {
                const uint32_t p = lds_phys<T>(ru) ^ pt;
                const cpx<T> a = lds[p];
                if constexpr (vb == 1) {
                    const cpx<T> b = lds[p ^ 1u];
                    w[u] = typename Amp16<T>::type{a.re, a.im, b.re, b.im};
                } else {
                    w[u] = typename Amp16<T>::type{a.re, a.im};
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t ru = r0 + u * STRIDE;
            if (ru + lt < tsize) v[(gt | tile_offset(sp, ru)) >> vb] = w[u];
        }
    }
}

// Matrix entry i of a record, stored in the state's own precision.
template <typename T>
__device__ __forceinline__ cpx<T> gmat(const TileGate &G, int i) {
    const T *m = reinterpret_cast<const T *>(G.m);
    return cpx<T>{m[2 * i], m[2 * i + 1]};
}
template <typename T>
__device__ __forceinline__ T gre(const TileGate &G, int i) {
    return reinterpret_cast<const T *>(G.m)[2 * i];
}

// x *= d with each component's own term taken last (see sweep_1q).
template <typename T>
__device__ __forceinline__ void cmul_inplace(cpx<T> &x, cpx<T> d) {
    const T a = -d.im * x.im, b = d.im * x.re;
    x.re = fma(d.re, x.re, a);
    x.im = fma(d.re, x.im, b);
}

// Exchange two amplitudes held in registers without renaming registers
// (a renamed set cannot share registers with the paths that leave the
// group unchanged, and every gate then pays a copy of the whole group).
__device__ __forceinline__ void swap_words(uint32_t &a, uint32_t &b) {
    asm volatile("v_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}
__device__ __forceinline__ void swap_f(float &a, float &b) {
    uint32_t x = __builtin_bit_cast(uint32_t, a), y = __builtin_bit_cast(uint32_t, b);
    swap_words(x, y);
    a = __builtin_bit_cast(float, x);
    b = __builtin_bit_cast(float, y);
}
__device__ __forceinline__ void swap_f(double &a, double &b) {
    uint64_t x = __builtin_bit_cast(uint64_t, a), y = __builtin_bit_cast(uint64_t, b);
    uint32_t xl = (uint32_t)x, xh = (uint32_t)(x >> 32), yl = (uint32_t)y, yh = (uint32_t)(y >> 32);
    swap_words(xl, yl);
    swap_words(xh, yh);
    a = __builtin_bit_cast(double, ((uint64_t)xh << 32) | xl);
    b = __builtin_bit_cast(double, ((uint64_t)yh << 32) | yl);
}
template <typename T>
__device__ __forceinline__ void swap_regs(cpx<T> &a, cpx<T> &b) {
    swap_f(a.re, b.re);
    swap_f(a.im, b.im);
}
// The local index of amplitude j of a group is gb | F[j]: gb holds the
// group's own tile bits (per lane), F[j] the bits of register index j at the
// sweep's positions (wave-uniform).  Every test of tile bits therefore splits
// into one per-lane test of gb per gate and a uniform test of F[j] per
// amplitude; gates without controls inside the tile compile the tests out.
template <int W>
struct GroupBits {
    uint32_t gb;
    uint32_t F[1 << W];
    uint32_t fall; // all register position bits
};

// Per-lane part of a control test: the control bits outside the registers.
template <int W>
__device__ __forceinline__ bool lane_controls(const GroupBits<W> &g, uint32_t cin) {
    const uint32_t cg = cin & ~g.fall;
    return (g.gb & cg) == cg;
}

// Gate on register position P of a group of 2^W (pairs j, j | 2^P).
template <typename T, int W, int P, bool CHECK>
__device__ __forceinline__ void sweep_1q(cpx<T> (&v)[1 << W], const GroupBits<W> &g, const TileGate &G,
                                         int kind, uint32_t cin) {
    constexpr int D = 1 << W;
    const uint32_t cr = cin & g.fall;
    if (CHECK && !lane_controls(g, cin)) return;
    // Every output first collects the terms that do not read its own input
    // component, then takes that component in one final FMA: the input dies
    // at its last use and the result can stay in the same register.
    if (kind == SK_GEN) {
        const cpx<T> g0 = gmat<T>(G, 0), g1 = gmat<T>(G, 1), g2 = gmat<T>(G, 2), g3 = gmat<T>(G, 3);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (j & (1 << P)) continue;
            if (CHECK && (g.F[j] & cr) != cr) continue;
            const int c = j | (1 << P);
            const cpx<T> x0 = v[j], x1 = v[c];
            const T a_re = fma(g1.re, x1.re, fma(-g1.im, x1.im, -g0.im * x0.im));
            const T a_im = fma(g1.re, x1.im, fma(g1.im, x1.re, g0.im * x0.re));
            const T b_re = fma(g2.re, x0.re, fma(-g2.im, x0.im, -g3.im * x1.im));
            const T b_im = fma(g2.re, x0.im, fma(g2.im, x0.re, g3.im * x1.re));
            v[j] = cpx<T>{fma(g0.re, x0.re, a_re), fma(g0.re, x0.im, a_im)};
            v[c] = cpx<T>{fma(g3.re, x1.re, b_re), fma(g3.re, x1.im, b_im)};
        }
    } else if (kind == SK_REAL) {
        const T r0 = gre<T>(G, 0), r1 = gre<T>(G, 1), r2 = gre<T>(G, 2), r3 = gre<T>(G, 3);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (j & (1 << P)) continue;
            if (CHECK && (g.F[j] & cr) != cr) continue;
            const int c = j | (1 << P);
            const cpx<T> x0 = v[j], x1 = v[c];
            const T a_re = r1 * x1.re, a_im = r1 * x1.im, b_re = r2 * x0.re, b_im = r2 * x0.im;
            v[j] = cpx<T>{fma(r0, x0.re, a_re), fma(r0, x0.im, a_im)};
            v[c] = cpx<T>{fma(r3, x1.re, b_re), fma(r3, x1.im, b_im)};
        }
    } else { // SK_SWAP: exchanged in place, so no register is renamed
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (j & (1 << P)) continue;
            if (CHECK && (g.F[j] & cr) != cr) continue;
            swap_regs(v[j], v[j | (1 << P)]);
        }
    }
}

template <typename T, int W, int P, int Q, bool CHECK>
__device__ __forceinline__ void sweep_2q(cpx<T> (&v)[1 << W], const GroupBits<W> &g, const TileGate &G,
                                         uint32_t cin) {
    constexpr int D = 1 << W;
    const uint32_t cr = cin & g.fall;
    if (CHECK && !lane_controls(g, cin)) return;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        if (j & ((1 << P) | (1 << Q))) continue;
        if (CHECK && (g.F[j] & cr) != cr) continue;
        const int idx[4] = {j, j | (1 << P), j | (1 << Q), j | (1 << P) | (1 << Q)};
        cpx<T> x[4], a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = v[idx[q]];
        // partial sums without each output's own component (see sweep_1q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const cpx<T> d = gmat<T>(G, 5 * r);
            cpx<T> acc{-d.im * x[r].im, d.im * x[r].re};
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c != r) acc = cfma(gmat<T>(G, 4 * r + c), x[c], acc);
            a[r] = acc;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const T dr = gre<T>(G, 5 * r);
            v[idx[r]] = cpx<T>{fma(dr, x[r].re, a[r].re), fma(dr, x[r].im, a[r].im)};
        }
    }
}

// diag(d0, d1) on tile bit b0.  On a register position the factor of each
// amplitude is a uniform choice; on a group bit it is one choice per lane.
template <typename T, int W, bool CHECK>
__device__ __forceinline__ void sweep_diag(cpx<T> (&v)[1 << W], const GroupBits<W> &g, const TileGate &G,
                                           uint32_t cin) {
    constexpr int D = 1 << W;
    const cpx<T> d0 = gmat<T>(G, 0), d1 = gmat<T>(G, 1);
    const uint32_t bm = 1u << G.b0;
    const uint32_t cr = cin & g.fall;
    const bool d0_one = d0.re == T(1) && d0.im == T(0);
    if (CHECK && !lane_controls(g, cin)) return;
    if (bm & g.fall) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (CHECK && (g.F[j] & cr) != cr) continue;
            const bool up = (g.F[j] & bm) != 0;
            if (d0_one) {
                if (up) cmul_inplace(v[j], d1);
            } else {
                cmul_inplace(v[j], up ? d1 : d0);
            }
        }
    } else {
        const bool up = (g.gb & bm) != 0;
        if (d0_one && !up) return; // phase gate: only amplitudes with the bit set change
        const cpx<T> d{up ? d1.re : d0.re, up ? d1.im : d0.im}; // component-wise select
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (CHECK && (g.F[j] & cr) != cr) continue;
            cmul_inplace(v[j], d);
        }
    }
}

template <typename T, int W, bool CHECK>
__device__ __forceinline__ void sweep_gate_t(cpx<T> (&v)[1 << W], const GroupBits<W> &li, const TileGate &G) {
    const int kind = G.kind;
    const uint32_t cin = G.cin;
    if (kind == SK_DIAG) {
        sweep_diag<T, W, CHECK>(v, li, G, cin);
        return;
    }
    if (kind == SK_2Q) {
        if constexpr (W >= 2) {
            const int pq = G.b0 * 4 + G.b1;
            if (pq == 1) { sweep_2q<T, W, 0, 1, CHECK>(v, li, G, cin); return; }
            if constexpr (W >= 3) {
                if (pq == 2) { sweep_2q<T, W, 0, 2, CHECK>(v, li, G, cin); return; }
                if (pq == 6) { sweep_2q<T, W, 1, 2, CHECK>(v, li, G, cin); return; }
            }
            if constexpr (W >= 4) {
                if (pq == 3) { sweep_2q<T, W, 0, 3, CHECK>(v, li, G, cin); return; }
                if (pq == 7) { sweep_2q<T, W, 1, 3, CHECK>(v, li, G, cin); return; }
                if (pq == 11) { sweep_2q<T, W, 2, 3, CHECK>(v, li, G, cin); return; }
            }
        }
        return;
    }
    const int p = G.b0;
    if (p == 0) { sweep_1q<T, W, 0, CHECK>(v, li, G, kind, cin); return; }
    if constexpr (W >= 2) if (p == 1) { sweep_1q<T, W, 1, CHECK>(v, li, G, kind, cin); return; }
    if constexpr (W >= 3) if (p == 2) { sweep_1q<T, W, 2, CHECK>(v, li, G, kind, cin); return; }
    if constexpr (W >= 4) if (p == 3) { sweep_1q<T, W, 3, CHECK>(v, li, G, kind, cin); return; }
}

// Apply the sweeps of one pass to the tile in LDS.  'base' is the global
// index of the tile's local amplitude 0 (for controls outside the tile).
// Caller synchronises before (tile loaded); every sweep ends with a barrier.
// The LDS swizzle is linear over XOR and gb, F[j] have disjoint bits, so the
// address of amplitude j is lds_phys(gb) ^ lds_phys(F[j]).
template <typename T, int W>
__device__ void tile_run_sweeps(cpx<T> *lds, int m, uint64_t base, const TileSweep *__restrict__ sweeps,
                                int n_sweeps, const TileGate *__restrict__ gates) {
    constexpr int D = 1 << W;
    const uint32_t n_groups = (1u << m) >> W;
    int goff = 0;
    for (int si = 0; si < n_sweeps; ++si) {
        const TileSweep &S = sweeps[si];
        const int ng = S.n_gates;
        uint32_t F[D], PF[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            uint32_t f = 0;
#pragma unroll
            for (int b = 0; b < W; ++b)
                if ((j >> b) & 1) f |= 1u << S.qpos[b];
            F[j] = f;
            PF[j] = lds_phys<T>(f);
        }
        for (uint32_t g = threadIdx.x; g < n_groups; g += blockDim.x) {
            uint32_t gb = g;
#pragma unroll
            for (int b = 0; b < W; ++b) {
                const uint32_t low = (1u << S.qpos[b]) - 1u;
                gb = (gb & low) | ((gb & ~low) << 1);
            }
            const uint32_t pg = lds_phys<T>(gb);
            cpx<T> v[D];
            GroupBits<W> li;
            li.gb = gb;
            li.fall = F[D - 1];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                li.F[j] = F[j];
                v[j] = lds[pg ^ PF[j]];
            }
            for (int gi = 0; gi < ng; ++gi) {
                const TileGate &G = gates[goff + gi];
                if ((base & G.cout) != G.cout) continue; // uniform
                if (G.cin == 0) sweep_gate_t<T, W, false>(v, li, G);
                else sweep_gate_t<T, W, true>(v, li, G);
            }
#pragma unroll
            for (int j = 0; j < D; ++j) lds[pg ^ PF[j]] = v[j];
        }
        goff += ng;
        __syncthreads();
    }
}

} // namespace sv
