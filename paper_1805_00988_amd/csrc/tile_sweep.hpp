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
// LDS addresses are swizzled: the low bits of the index (one 128-byte LDS
// row: 16 complex64 or 8 complex128 amplitudes) are XOR-ed with a fold of the
// higher bits, so the lanes of a wave, whose groups differ in arbitrary tile
// bits, spread over the banks.
#pragma once

#include "sv_internal.hpp"

namespace sv {


template <typename T>
__device__ __forceinline__ uint32_t lds_phys(uint32_t l) {
    return lds_swizzle(l, lds_swizzle_bits(2 * sizeof(T)));
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

// The local index of amplitude j of a group is gb | F[j] (gb: the group's
// bits, F[j]: j's bits deposited at the sweep's register positions, uniform).
// Control tests are compiled out for gates without controls inside the tile.

// Gate on register position P of a group of 2^W (pairs j, j | 2^P).
template <typename T, int W, int P, bool CHECK>
__device__ __forceinline__ void sweep_1q(cpx<T> (&v)[1 << W], const uint32_t (&li)[1 << W],
                                         const TileGate &G, int kind, uint32_t cin) {
    constexpr int D = 1 << W;
    if (kind == SK_GEN) {
        const cpx<T> g0 = gmat<T>(G, 0), g1 = gmat<T>(G, 1), g2 = gmat<T>(G, 2), g3 = gmat<T>(G, 3);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (j & (1 << P)) continue;
            if (CHECK && (li[j] & cin) != cin) continue;
            const int c = j | (1 << P);
            const cpx<T> x0 = v[j], x1 = v[c];
            v[j] = cfma(g0, x0, cmul(g1, x1));
            v[c] = cfma(g2, x0, cmul(g3, x1));
        }
    } else if (kind == SK_REAL) {
        const T r0 = gre<T>(G, 0), r1 = gre<T>(G, 1), r2 = gre<T>(G, 2), r3 = gre<T>(G, 3);
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (j & (1 << P)) continue;
            if (CHECK && (li[j] & cin) != cin) continue;
            const int c = j | (1 << P);
            const cpx<T> x0 = v[j], x1 = v[c];
            v[j] = cpx<T>{fma(r0, x0.re, r1 * x1.re), fma(r0, x0.im, r1 * x1.im)};
            v[c] = cpx<T>{fma(r2, x0.re, r3 * x1.re), fma(r2, x0.im, r3 * x1.im)};
        }
    } else { // SK_SWAP
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (j & (1 << P)) continue;
            if (CHECK && (li[j] & cin) != cin) continue;
            const int c = j | (1 << P);
            const cpx<T> x0 = v[j];
            v[j] = v[c];
            v[c] = x0;
        }
    }
}

template <typename T, int W, int P, int Q, bool CHECK>
__device__ __forceinline__ void sweep_2q(cpx<T> (&v)[1 << W], const uint32_t (&li)[1 << W],
                                         const TileGate &G, uint32_t cin) {
    constexpr int D = 1 << W;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        if (j & ((1 << P) | (1 << Q))) continue;
        if (CHECK && (li[j] & cin) != cin) continue;
        const int idx[4] = {j, j | (1 << P), j | (1 << Q), j | (1 << P) | (1 << Q)};
        cpx<T> x[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = v[idx[q]];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            cpx<T> acc = cmul(gmat<T>(G, 4 * r), x[0]);
#pragma unroll
            for (int c = 1; c < 4; ++c) acc = cfma(gmat<T>(G, 4 * r + c), x[c], acc);
            v[idx[r]] = acc;
        }
    }
}

template <typename T, int W, bool CHECK>
__device__ __forceinline__ void sweep_diag(cpx<T> (&v)[1 << W], const uint32_t (&li)[1 << W],
                                           const TileGate &G, uint32_t cin) {
    constexpr int D = 1 << W;
    const cpx<T> d0 = gmat<T>(G, 0), d1 = gmat<T>(G, 1);
    const uint32_t bm = 1u << G.b0;
    const bool d0_one = d0.re == T(1) && d0.im == T(0);
    if (d0_one) { // phase gate: only amplitudes with the target bit set change
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const uint32_t l = li[j];
            if (CHECK && (l & cin) != cin) continue;
            if (l & bm) v[j] = cmul(d1, v[j]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const uint32_t l = li[j];
            if (CHECK && (l & cin) != cin) continue;
            const bool up = (l & bm) != 0; // component-wise select keeps d0, d1 in registers
            const cpx<T> d{up ? d1.re : d0.re, up ? d1.im : d0.im};
            v[j] = cmul(d, v[j]);
        }
    }
}

template <typename T, int W, bool CHECK>
__device__ __forceinline__ void sweep_gate_t(cpx<T> (&v)[1 << W], const uint32_t (&li)[1 << W],
                                             const TileGate &G) {
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
            uint32_t li[D];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                li[j] = gb | F[j];
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
