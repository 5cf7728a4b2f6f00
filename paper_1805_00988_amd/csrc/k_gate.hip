// Gate kernels: streamed pair/quad updates for gates on high qubits, a
// subspace-scaling kernel for phase-type diagonal gates, and the on-chip tile
// pass that applies a run of gates to tiles staged in LDS.
//
// Memory access: the state is read and written as 16-byte vectors (float4 =
// two complex64 amplitudes, double2 = one complex128 amplitude).  Consecutive
// lanes take consecutive vectors of the same half of the pair space, so every
// wavefront load is a contiguous run as long as the target qubit is above the
// vector width.
#include "sv_internal.hpp"
#include "tile_sweep.hpp"

#include <algorithm>

namespace sv {

template <typename T>
struct Vec;
template <>
struct Vec<float> {
    using type = float4;
    static constexpr int amps = 2;
    static constexpr int bits = 1;
    __device__ static cpx<float> get(const float4 &v, int k) {
        return k == 0 ? cpx<float>{v.x, v.y} : cpx<float>{v.z, v.w};
    }
    __device__ static void put(float4 &v, int k, cpx<float> c) {
        if (k == 0) { v.x = c.re; v.y = c.im; } else { v.z = c.re; v.w = c.im; }
    }
};
template <>
struct Vec<double> {
    using type = double2;
    static constexpr int amps = 1;
    static constexpr int bits = 0;
    __device__ static cpx<double> get(const double2 &v, int) { return {v.x, v.y}; }
    __device__ static void put(double2 &v, int, cpx<double> c) { v.x = c.re; v.y = c.im; }
};

constexpr int kStreamThreads = 256;

// 16-byte access, nontemporal when NT.  Launchers pick NT only when every
// wavefront access is a run of at least 128 contiguous bytes: nontemporal
// accesses to interleaved shorter runs (a gate on the lowest qubits) were
// measured much slower.
template <bool NT, typename V>
__device__ __forceinline__ V ld16(const V *p) {
    if constexpr (NT) return ld_nt(p);
    else return *p;
}
template <bool NT, typename V>
__device__ __forceinline__ void st16(V *p, V v) {
    if constexpr (NT) st_nt(p, v);
    else *p = v;
}
constexpr int kMinNtRunBits = 3; // 2^3 16-byte vectors = 128 bytes

static inline uint64_t grid_for(uint64_t work_items, uint64_t per_block, uint64_t cap) {
    uint64_t b = (work_items + per_block - 1) / per_block;
    return std::max<uint64_t>(1, std::min<uint64_t>(b, cap));
}

// ---------------------------------------------------------------- init
// UNROLL vectors per thread and round; a grid of up to 2^20 workgroups
// covers a 32 GiB state in one round (measured faster than fewer
// workgroups looping).
template <typename T, int UNROLL>
__global__ __launch_bounds__(kStreamThreads) void k_init_basis(typename Vec<T>::type *v,
                                                               uint64_t n_vec, uint64_t x) {
    using V = Vec<T>;
    const uint64_t per_block = (uint64_t)UNROLL * kStreamThreads;
    for (uint64_t base = (uint64_t)blockIdx.x * per_block; base < n_vec;
         base += (uint64_t)gridDim.x * per_block) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const uint64_t e = base + (uint64_t)u * kStreamThreads + threadIdx.x;
            if (e >= n_vec) break;
            typename V::type z;
            for (int k = 0; k < V::amps; ++k)
                V::put(z, k, cpx<T>{(((e << V::bits) | k) == x) ? T(1) : T(0), T(0)});
            v[e] = z;
        }
    }
}

hipError_t launch_init_basis(void *amps, int n, int dtype, uint64_t x, hipStream_t s) {
    const uint64_t N = 1ull << n;
    constexpr int U = 4;
    const uint64_t nv = dtype == SV_C64 ? N / 2 : N;
    const dim3 grid((unsigned)grid_for(nv, (uint64_t)U * kStreamThreads, 1ull << 20));
    if (dtype == SV_C64)
        k_init_basis<float, U><<<grid, dim3(kStreamThreads), 0, s>>>((float4 *)amps, nv, x);
    else
        k_init_basis<double, U><<<grid, dim3(kStreamThreads), 0, s>>>((double2 *)amps, nv, x);
    return hipGetLastError();
}

// ------------------------------------------------------- streamed 1q gate
// Element-pair j -> element a (bit te clear, control bits set) and a | 2^te.
// lane_ctrl holds control bits below the vector width (amplitude bits inside
// one 16-byte element): only amplitudes with all of them set are updated.
template <typename T, int UNROLL, bool NT>
__global__ __launch_bounds__(kStreamThreads) void k_gate1(typename Vec<T>::type *v, Enum e, int te,
                                                          uint64_t count, Mat2<T> g,
                                                          uint32_t lane_ctrl) {
    using V = Vec<T>;
    const uint64_t per_block = (uint64_t)UNROLL * kStreamThreads;
    const uint64_t bstep = 1ull << te;
    for (uint64_t base = (uint64_t)blockIdx.x * per_block; base < count;
         base += (uint64_t)gridDim.x * per_block) {
        typename V::type va[UNROLL], vb[UNROLL];
        uint64_t ia[UNROLL];
        bool ok[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const uint64_t j = base + (uint64_t)u * kStreamThreads + threadIdx.x;
            const uint64_t a = expand(e, j < count ? j : 0);
            ok[u] = (j < count) && ((a & e.check) == e.check);
            ia[u] = a;
            if (ok[u]) {
                va[u] = ld16<NT>(&v[a]);
                vb[u] = ld16<NT>(&v[a + bstep]);
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            if (!ok[u]) continue;
            typename V::type oa = va[u], ob = vb[u];
#pragma unroll
            for (int k = 0; k < V::amps; ++k) {
                if (((uint32_t)k & lane_ctrl) != lane_ctrl) continue;
                const cpx<T> x0 = V::get(va[u], k), x1 = V::get(vb[u], k);
                V::put(oa, k, cfma(g.m[0], x0, cmul(g.m[1], x1)));
                V::put(ob, k, cfma(g.m[2], x0, cmul(g.m[3], x1)));
            }
            st16<NT>(&v[ia[u]], oa);
            st16<NT>(&v[ia[u] + bstep], ob);
        }
    }
}

// complex64 gate on qubit 0: both amplitudes of a pair sit in one float4.
template <int UNROLL, bool NT>
__global__ __launch_bounds__(kStreamThreads) void k_gate1_q0(float4 *v, Enum e, uint64_t count,
                                                             Mat2<float> g) {
    const uint64_t per_block = (uint64_t)UNROLL * kStreamThreads;
    for (uint64_t base = (uint64_t)blockIdx.x * per_block; base < count;
         base += (uint64_t)gridDim.x * per_block) {
        float4 w[UNROLL];
        uint64_t ia[UNROLL];
        bool ok[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const uint64_t j = base + (uint64_t)u * kStreamThreads + threadIdx.x;
            const uint64_t a = expand(e, j < count ? j : 0);
            ok[u] = (j < count) && ((a & e.check) == e.check);
            ia[u] = a;
            if (ok[u]) w[u] = ld16<NT>(&v[a]);
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            if (!ok[u]) continue;
            const cpx<float> x0{w[u].x, w[u].y}, x1{w[u].z, w[u].w};
            const cpx<float> y0 = cfma(g.m[0], x0, cmul(g.m[1], x1));
            const cpx<float> y1 = cfma(g.m[2], x0, cmul(g.m[3], x1));
            st16<NT>(&v[ia[u]], float4{y0.re, y0.im, y1.re, y1.im});
        }
    }
}

// Build the element-level enumeration for a set of zero positions (element
// bit indices) plus control bits; controls beyond the insert capacity are
// checked instead of enumerated.
static Enum make_enum(int vbits, const int *zero_pos, int n_zero, uint64_t ctrl,
                      uint32_t *lane_ctrl, int *n_enumerated) {
    Enum e{};
    int pos[64];
    int np = 0;
    for (int i = 0; i < n_zero; ++i) pos[np++] = zero_pos[i];
    const uint64_t lane_mask = (1ull << vbits) - 1ull;
    *lane_ctrl = (uint32_t)(ctrl & lane_mask);
    uint64_t ec = ctrl >> vbits;
    e.set = 0;
    e.check = 0;
    while (ec) {
        const int b = __builtin_ctzll(ec);
        ec &= ec - 1;
        if (np < kMaxInsert) {
            pos[np++] = b;
            e.set |= 1ull << b;
        } else {
            e.check |= 1ull << b;
        }
    }
    std::sort(pos, pos + np);
    e.n_pos = np;
    for (int i = 0; i < np; ++i) e.pos[i] = pos[i];
    *n_enumerated = np;
    return e;
}

// Every enumerated element index lies in a run of 2^pos[0] consecutive
// vectors (the lowest inserted bit), and checked controls thin the runs out.
static bool nt_ok(const Enum &e) {
    return e.check == 0 && (e.n_pos == 0 || e.pos[0] >= kMinNtRunBits);
}

template <typename T>
static Mat2<T> to_mat2(const double *U) {
    Mat2<T> g;
    for (int i = 0; i < 4; ++i) g.m[i] = cpx<T>{(T)U[2 * i], (T)U[2 * i + 1]};
    return g;
}

constexpr int kUnroll = 4;
constexpr uint64_t kGridCap = 1ull << 20;
// The streamed one-qubit gate on pairs of 16-byte elements: one pair per
// thread and a grid covering the state in one round measured 5.5-6.0 TB/s
// on a 32 GiB state against 4.9-5.6 TB/s with four pairs per thread, except
// for element strides near 2^20 (5.44 against 5.59 TB/s).  The grid stops
// at 2^23 workgroups (a launch's threads must number fewer than 2^32): one
// round up to 33 qubits complex64 / 32 complex128, grid-stride beyond.
constexpr int kPairUnroll = 1;
constexpr uint64_t kPairGridCap = 1ull << 23;

hipError_t launch_gate1(void *amps, int n, int dtype, int t, uint64_t ctrl, const double *U,
                        hipStream_t s) {
    const int vbits = dtype == SV_C64 ? 1 : 0;
    const uint64_t n_el = (1ull << n) >> vbits;
    uint32_t lane_ctrl = 0;
    int np = 0;
    if (t < vbits) {
        // complex64, target qubit 0: enumerate elements restricted by controls
        Enum e = make_enum(vbits, nullptr, 0, ctrl, &lane_ctrl, &np);
        const uint64_t count = n_el >> np;
        const uint64_t per = (uint64_t)kUnroll * kStreamThreads;
        const dim3 grid((unsigned)grid_for(count, per, kGridCap));
        if (nt_ok(e))
            k_gate1_q0<kUnroll, true><<<grid, dim3(kStreamThreads), 0, s>>>((float4 *)amps, e, count, to_mat2<float>(U));
        else
            k_gate1_q0<kUnroll, false><<<grid, dim3(kStreamThreads), 0, s>>>((float4 *)amps, e, count, to_mat2<float>(U));
        return hipGetLastError();
    }
    const int te = t - vbits;
    Enum e = make_enum(vbits, &te, 1, ctrl, &lane_ctrl, &np);
    const uint64_t count = n_el >> np;
    const uint64_t per = (uint64_t)kPairUnroll * kStreamThreads;
    const dim3 grid((unsigned)grid_for(count, per, kPairGridCap));
    const bool nt = nt_ok(e);
    constexpr int PU = kPairUnroll;
    if (dtype == SV_C64 && nt)
        k_gate1<float, PU, true><<<grid, dim3(kStreamThreads), 0, s>>>((float4 *)amps, e, te, count, to_mat2<float>(U), lane_ctrl);
    else if (dtype == SV_C64)
        k_gate1<float, PU, false><<<grid, dim3(kStreamThreads), 0, s>>>((float4 *)amps, e, te, count, to_mat2<float>(U), lane_ctrl);
    else if (nt)
        k_gate1<double, PU, true><<<grid, dim3(kStreamThreads), 0, s>>>((double2 *)amps, e, te, count, to_mat2<double>(U), lane_ctrl);
    else
        k_gate1<double, PU, false><<<grid, dim3(kStreamThreads), 0, s>>>((double2 *)amps, e, te, count, to_mat2<double>(U), lane_ctrl);
    return hipGetLastError();
}

// ------------------------------------------------------- streamed 2q gate
// Quad index q = b0 + 2 b1 (bit j of q = value of targets[j]); both targets
// at or above the vector width.
template <typename T, int UNROLL, bool NT>
__global__ __launch_bounds__(kStreamThreads) void k_gate2(typename Vec<T>::type *v, Enum e, int te0,
                                                          int te1, uint64_t count, Mat4<T> g,
                                                          uint32_t lane_ctrl) {
    using V = Vec<T>;
    const uint64_t per_block = (uint64_t)UNROLL * kStreamThreads;
    const uint64_t s0 = 1ull << te0, s1 = 1ull << te1;
    for (uint64_t base = (uint64_t)blockIdx.x * per_block; base < count;
         base += (uint64_t)gridDim.x * per_block) {
        typename V::type w[UNROLL][4];
        uint64_t ia[UNROLL];
        bool ok[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const uint64_t j = base + (uint64_t)u * kStreamThreads + threadIdx.x;
            const uint64_t a = expand(e, j < count ? j : 0);
            ok[u] = (j < count) && ((a & e.check) == e.check);
            ia[u] = a;
            if (ok[u]) {
                w[u][0] = ld16<NT>(&v[a]);
                w[u][1] = ld16<NT>(&v[a + s0]);
                w[u][2] = ld16<NT>(&v[a + s1]);
                w[u][3] = ld16<NT>(&v[a + s0 + s1]);
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            if (!ok[u]) continue;
            typename V::type o[4] = {w[u][0], w[u][1], w[u][2], w[u][3]};
#pragma unroll
            for (int k = 0; k < V::amps; ++k) {
                if (((uint32_t)k & lane_ctrl) != lane_ctrl) continue;
                cpx<T> x[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) x[q] = V::get(w[u][q], k);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    cpx<T> acc = cmul(g.m[4 * r], x[0]);
#pragma unroll
                    for (int c = 1; c < 4; ++c) acc = cfma(g.m[4 * r + c], x[c], acc);
                    V::put(o[r], k, acc);
                }
            }
            st16<NT>(&v[ia[u]], o[0]);
            st16<NT>(&v[ia[u] + s0], o[1]);
            st16<NT>(&v[ia[u] + s1], o[2]);
            st16<NT>(&v[ia[u] + s0 + s1], o[3]);
        }
    }
}

template <typename T>
static Mat4<T> to_mat4(const double *U) {
    Mat4<T> g;
    for (int i = 0; i < 16; ++i) g.m[i] = cpx<T>{(T)U[2 * i], (T)U[2 * i + 1]};
    return g;
}

hipError_t launch_gate2(void *amps, int n, int dtype, int t0, int t1, uint64_t ctrl,
                        const double *U, hipStream_t s) {
    const int vbits = dtype == SV_C64 ? 1 : 0;
    if (t0 < vbits || t1 < vbits) return hipErrorInvalidValue; // routed to the tile pass
    const uint64_t n_el = (1ull << n) >> vbits;
    const int te[2] = {t0 - vbits, t1 - vbits};
    uint32_t lane_ctrl = 0;
    int np = 0;
    Enum e = make_enum(vbits, te, 2, ctrl, &lane_ctrl, &np);
    const uint64_t count = n_el >> np;
    constexpr int U2 = 2;
    const uint64_t per = (uint64_t)U2 * kStreamThreads;
    const dim3 grid((unsigned)grid_for(count, per, kGridCap));
    const bool nt = nt_ok(e);
    if (dtype == SV_C64 && nt)
        k_gate2<float, U2, true><<<grid, dim3(kStreamThreads), 0, s>>>((float4 *)amps, e, te[0], te[1], count, to_mat4<float>(U), lane_ctrl);
    else if (dtype == SV_C64)
        k_gate2<float, U2, false><<<grid, dim3(kStreamThreads), 0, s>>>((float4 *)amps, e, te[0], te[1], count, to_mat4<float>(U), lane_ctrl);
    else if (nt)
        k_gate2<double, U2, true><<<grid, dim3(kStreamThreads), 0, s>>>((double2 *)amps, e, te[0], te[1], count, to_mat4<double>(U), lane_ctrl);
    else
        k_gate2<double, U2, false><<<grid, dim3(kStreamThreads), 0, s>>>((double2 *)amps, e, te[0], te[1], count, to_mat4<double>(U), lane_ctrl);
    return hipGetLastError();
}

// ------------------------------------------------- subspace scaling
// Multiply every amplitude x with (x & mask) == mask by a complex factor:
// a phase-type diagonal gate (diag(1, f), optionally controlled) only changes
// the amplitudes whose target and control bits are all 1.
template <typename T, int UNROLL, bool NT>
__global__ __launch_bounds__(kStreamThreads) void k_scale(typename Vec<T>::type *v, Enum e,
                                                          uint64_t count, cpx<T> f,
                                                          uint32_t lane_set) {
    using V = Vec<T>;
    const uint64_t per_block = (uint64_t)UNROLL * kStreamThreads;
    for (uint64_t base = (uint64_t)blockIdx.x * per_block; base < count;
         base += (uint64_t)gridDim.x * per_block) {
        typename V::type w[UNROLL];
        uint64_t ia[UNROLL];
        bool ok[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const uint64_t j = base + (uint64_t)u * kStreamThreads + threadIdx.x;
            const uint64_t a = expand(e, j < count ? j : 0);
            ok[u] = (j < count) && ((a & e.check) == e.check);
            ia[u] = a;
            if (ok[u]) w[u] = ld16<NT>(&v[a]);
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            if (!ok[u]) continue;
#pragma unroll
            for (int k = 0; k < V::amps; ++k) {
                if (((uint32_t)k & lane_set) != lane_set) continue;
                V::put(w[u], k, cmul(f, V::get(w[u], k)));
            }
            st16<NT>(&v[ia[u]], w[u]);
        }
    }
}

hipError_t launch_scale(void *amps, int n, int dtype, uint64_t set_mask, const double *factor,
                        hipStream_t s) {
    const int vbits = dtype == SV_C64 ? 1 : 0;
    const uint64_t n_el = (1ull << n) >> vbits;
    uint32_t lane_set = 0;
    int np = 0;
    Enum e = make_enum(vbits, nullptr, 0, set_mask, &lane_set, &np);
    const uint64_t count = n_el >> np;
    const uint64_t per = (uint64_t)kUnroll * kStreamThreads;
    const dim3 grid((unsigned)grid_for(count, per, kGridCap));
    const cpx<float> f32{(float)factor[0], (float)factor[1]};
    const cpx<double> f64{factor[0], factor[1]};
    const bool nt = nt_ok(e);
    if (dtype == SV_C64 && nt)
        k_scale<float, kUnroll, true><<<grid, dim3(kStreamThreads), 0, s>>>((float4 *)amps, e, count, f32, lane_set);
    else if (dtype == SV_C64)
        k_scale<float, kUnroll, false><<<grid, dim3(kStreamThreads), 0, s>>>((float4 *)amps, e, count, f32, lane_set);
    else if (nt)
        k_scale<double, kUnroll, true><<<grid, dim3(kStreamThreads), 0, s>>>((double2 *)amps, e, count, f64, lane_set);
    else
        k_scale<double, kUnroll, false><<<grid, dim3(kStreamThreads), 0, s>>>((double2 *)amps, e, count, f64, lane_set);
    return hipGetLastError();
}

// ------------------------------------------------------------ tile pass
// A workgroup stages one tile of 2^m amplitudes in LDS: the low qubits
// 0..L-1 (contiguous runs of 2^L amplitudes in HBM) plus K further qubits.
// The pass's gates, grouped into register sweeps by the host, are applied
// to the tile (tile_sweep.hpp); controls outside the tile are constant over a
// tile and tested once on its base index.
constexpr int kTileThreads = 512;

// Tiles of 4096 amplitudes: 32 KiB of LDS for complex64 (five 256-thread
// workgroups per CU, the register file's limit too), 64 KiB for complex128.
// Measured on the 32-qubit headline circuits: complex64 tiles of 8192
// amplitudes need fewer passes (44 against 53) but hold only four waves
// per SIMD, and were slower overall; tiles of 16384 slower still.  The
// batch kernel keeps 8192-amplitude complex64 tiles (whole circuits of up
// to 13 qubits in one workgroup).
int tile_max_qubits(int dtype) { return dtype == SV_C64 ? 12 : 12; }
// Largest tile a tile pass accepts: the fused path's complex64 passes keep
// 8192-amplitude tiles (64 KiB of LDS, 512 threads) when they run as plain
// sweeps.
int tile_launch_qubits(int dtype) { return dtype == SV_C64 ? 13 : 12; }
int batch_tile_qubits(int dtype) { return dtype == SV_C64 ? 13 : 12; }

// Register qubits per sweep: 16 complex64 or 8 complex128 amplitudes per
// group (64 and 32 VGPRs); a 4096-amplitude tile then takes 256 or 512
// threads.
int sweep_width(int dtype) { return dtype == SV_C64 ? 4 : 3; }

__device__ __forceinline__ uint64_t tile_global(const TileSpec &sp, uint64_t base, uint32_t l) {
    uint64_t g = base | (l & ((1u << sp.L) - 1u));
    uint32_t hi = l >> sp.L;
#pragma unroll
    for (int i = 0; i < kMaxTileHigh; ++i) {
        if (i >= sp.K) break;
        if ((hi >> i) & 1u) g |= 1ull << sp.high[i];
    }
    return g;
}

// The pass's sweeps over one tile.  The first sweep reads its groups
// straight from the state and the last writes them straight back, so the
// tile crosses LDS only between sweeps (a pass of one sweep never touches
// it); each sweep ends with a barrier, which also keeps the next tile's
// first LDS writes behind this tile's last LDS reads.
template <typename T, int W, bool TWOQ, bool LPH>
__device__ void tile_pass_direct(cpx<T> *__restrict__ state, cpx<T> *lds, const TileSpec &sp, uint64_t base,
                                 int m, const TileSweep *__restrict__ sweeps, int n_sweeps,
                                 const char *__restrict__ recs, uint32_t direct) {
    constexpr int D = 1 << W;
    const uint32_t n_groups = (1u << m) >> W;
    using V = typename Vec<T>::type;
    if (!(direct & kDirectFirst)) {
        tile_load<T, kTileThreads, 8>(reinterpret_cast<const V *>(state), lds, sp, base, 1u << m);
        __syncthreads();
    }
    for (int si = 0; si < n_sweeps; ++si) {
        const TileSweep &S = sweeps[si];
        const int ng = S.n_gates;
        const bool first = si == 0 && (direct & kDirectFirst), last = si == n_sweeps - 1 && (direct & kDirectLast);
        // both offsets of register index j combine per-bit parts: the LDS
        // swizzle by XOR, the global offset by OR (disjoint bits)
        uint32_t pb[W];
        uint64_t gbit[W];
#pragma unroll
        for (int b = 0; b < W; ++b) {
            pb[b] = lds_phys<T>(1u << S.qpos[b]);
            gbit[b] = tile_offset(sp, 1u << S.qpos[b]);
        }
        auto goff_of = [&](int j) {
            uint64_t o = 0;
#pragma unroll
            for (int b = 0; b < W; ++b)
                if ((j >> b) & 1) o |= gbit[b];
            return o;
        };
        auto poff_of = [&](int j) {
            uint32_t o = 0;
#pragma unroll
            for (int b = 0; b < W; ++b)
                if ((j >> b) & 1) o ^= pb[b];
            return o;
        };
        for (uint32_t g = threadIdx.x; g < n_groups; g += blockDim.x) {
            const uint32_t gb = group_bits<W>(S, g);
            const uint32_t pg = lds_phys<T>(gb);
            cpx<T> *row = state + (base | tile_offset(sp, gb));
            cpx<T> v[D];
            if (first) {
#pragma unroll
                for (int j = 0; j < D; ++j) v[j] = row[goff_of(j)];
            } else {
#pragma unroll
                for (int j = 0; j < D; ++j) v[j] = lds[pg ^ poff_of(j)];
            }
            PhaseAcc<T, W> acc;
            acc.init();
            run_records<T, W, TWOQ, LPH>(v, acc, gb, recs + S.rec_off, ng, base);
            if (last) {
#pragma unroll
                for (int j = 0; j < D; ++j) row[goff_of(j)] = v[j];
            } else {
#pragma unroll
                for (int j = 0; j < D; ++j) lds[pg ^ poff_of(j)] = v[j];
            }
        }
        __syncthreads();
    }
    if (!(direct & kDirectLast)) {
        tile_store<T, kTileThreads, 8>(reinterpret_cast<V *>(state), lds, sp, base, 1u << m);
        __syncthreads();
    }
}

template <typename T, int W, bool TWOQ, bool LPH>
__global__ __launch_bounds__(kTileThreads) void k_tile(typename Vec<T>::type *v, TileSpec sp, int m,
                                                       const TileSweep *__restrict__ sweeps, int n_sweeps,
                                                       const char *__restrict__ recs,
                                                       uint64_t n_tiles, uint32_t direct) {
    extern __shared__ char lds_raw[];
    cpx<T> *lds = reinterpret_cast<cpx<T> *>(lds_raw);
    cpx<T> *state = reinterpret_cast<cpx<T> *>(v);
    // 32-bit tile counter (at most 2^27 tiles): the loop test stays on the
    // scalar unit
    const uint32_t nt = (uint32_t)n_tiles;
    for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
        uint64_t base = (uint64_t)tile << sp.L;
        for (int i = 0; i < sp.K; ++i) base = insert_zero(base, sp.high[i]);
        tile_pass_direct<T, W, TWOQ, LPH>(state, lds, sp, base, m, sweeps, n_sweeps, recs, direct);
    }
}

template <typename T, int W, bool TWOQ, bool LPH = std::is_same<T, double>::value>
static void launch_tile_t(typename Vec<T>::type *v, const TileSpec &spec, int m, const TileSweep *sw,
                          int n_sweeps, const char *g, uint64_t n_tiles, uint32_t direct, size_t lds,
                          hipStream_t s) {
    (void)hipFuncSetAttribute((const void *)k_tile<T, W, TWOQ, LPH>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    // one workgroup per tile (measured faster than a capped grid looping
    // over tiles), and one thread per register group
    const unsigned grid = (unsigned)std::min<uint64_t>(n_tiles, 1u << 30);
    const unsigned threads = (unsigned)std::max(64, std::min(kTileThreads, (1 << m) >> W));
    k_tile<T, W, TWOQ, LPH><<<grid, threads, lds, s>>>(v, spec, m, sw, n_sweeps, g, n_tiles, direct);
}

template <int W>
static bool tile_staging_ok(int m, uint32_t direct) {
    // staging the whole tile through LDS (a pass without direct first and
    // last sweeps) moves it with kTileThreads threads
    const int threads = std::max(64, std::min(kTileThreads, (1 << m) >> W));
    return direct == (kDirectFirst | kDirectLast) || threads == kTileThreads;
}

hipError_t launch_tile(void *amps, int n, int dtype, const TileSpec &spec, const TileSweep *dev_sweeps,
                       int n_sweeps, const char *dev_gates, bool two_qubit, bool lane_phases, uint32_t direct,
                       hipStream_t s) {
    const int m = spec.L + spec.K;
    const int vbits = dtype == SV_C64 ? 1 : 0;
    if (m > n || m > tile_launch_qubits(dtype) || spec.L < vbits || spec.K > kMaxTileHigh || m < 1)
        return hipErrorInvalidValue;
    const uint64_t n_tiles = 1ull << (n - m);
    const size_t lds = (size_t)(1u << m) * (dtype == SV_C64 ? 8 : 16);
    const int W = std::min(m, sweep_width(dtype));
    // complex64 lane-bit phase lists: only the full-width instances hold
    // them (the complex128 instances always do)
    if (lane_phases && dtype == SV_C64) {
        if (W != sweep_width(SV_C64) || !tile_staging_ok<4>(m, direct)) return hipErrorInvalidValue;
        if (two_qubit)
            launch_tile_t<float, 4, true, true>((float4 *)amps, spec, m, dev_sweeps, n_sweeps, dev_gates, n_tiles,
                                                direct, lds, s);
        else
            launch_tile_t<float, 4, false, true>((float4 *)amps, spec, m, dev_sweeps, n_sweeps, dev_gates,
                                                 n_tiles, direct, lds, s);
        return hipGetLastError();
    }
#define SV_TILE_CASE(WW, Q)                                                                        \
    if (W == WW && two_qubit == Q) {                                                               \
        if (!tile_staging_ok<WW>(m, direct)) return hipErrorInvalidValue;                          \
        if (dtype == SV_C64)                                                                       \
            launch_tile_t<float, WW, Q>((float4 *)amps, spec, m, dev_sweeps, n_sweeps, dev_gates,  \
                                        n_tiles, direct, lds, s);                                  \
        else                                                                                       \
            launch_tile_t<double, WW, Q>((double2 *)amps, spec, m, dev_sweeps, n_sweeps,           \
                                         dev_gates, n_tiles, direct, lds, s);                      \
        return hipGetLastError();                                                                  \
    }
    SV_TILE_CASE(4, false)
    SV_TILE_CASE(3, false)
    SV_TILE_CASE(2, false)
    SV_TILE_CASE(1, false)
    SV_TILE_CASE(4, true)
    SV_TILE_CASE(3, true)
    SV_TILE_CASE(2, true)
    SV_TILE_CASE(1, true)
#undef SV_TILE_CASE
    return hipErrorInvalidValue;
}

} // namespace sv
