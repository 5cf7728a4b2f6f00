// Adjoint-method gradient kernels.
//
// With psi the circuit output and lam = H psi for a diagonal observable H,
// the reverse sweep undoes one gate at a time on both vectors.  For a
// parametrised gate U(theta) whose derivative is U' = c M U (c a constant,
// M a 2x2 "probe": the Pauli of a rotation, or the projector |1><1| of the
// phase gate) the gradient term 2 Re <lam| U' |psi_before> equals a real
// multiple of Im <lam| M |psi_after>, evaluated on the vectors before the
// gate is undone.  One kernel does the probe and the undo in the same pass
// over both vectors; the probe's FP64 partial sums go to one slot per gate.
#include "sv_internal.hpp"

#include <algorithm>

namespace sv {

constexpr int kAdjThreads = 256;

template <typename T>
struct AV;
template <>
struct AV<float> {
    using type = float4;
    static constexpr int amps = 2, bits = 1;
    __device__ static cpx<float> get(const float4 &v, int k) {
        return k == 0 ? cpx<float>{v.x, v.y} : cpx<float>{v.z, v.w};
    }
    __device__ static void put(float4 &v, int k, cpx<float> c) {
        if (k == 0) { v.x = c.re; v.y = c.im; } else { v.z = c.re; v.w = c.im; }
    }
};
template <>
struct AV<double> {
    using type = double2;
    static constexpr int amps = 1, bits = 0;
    __device__ static cpx<double> get(const double2 &v, int) { return {v.x, v.y}; }
    __device__ static void put(double2 &v, int, cpx<double> c) { v.x = c.re; v.y = c.im; }
};

__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ double block_sum_d(double x) {
    __shared__ double sh[kAdjThreads / 64];
    x = wave_sum_d(x);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = x;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kAdjThreads / 64; ++w) r += sh[w];
    __syncthreads();
    return r;
}

// Im(conj(y) z) in FP64
template <typename T>
__device__ __forceinline__ double im_conj_mul(cpx<T> y, cpx<T> z) {
    return (double)y.re * (double)z.im - (double)y.im * (double)z.re;
}

// lam = h(x) psi, loss partial = sum h(x) |psi_x|^2, h(x) = sum_j c_j (-1)^popcount(x & m_j)
struct AdjTerms {
    int n;
    uint64_t mask[kMaxTerms];
    double coeff[kMaxTerms];
};

template <typename T>
__global__ __launch_bounds__(kAdjThreads) void k_adjoint_init(const typename AV<T>::type *__restrict__ psi,
                                                              typename AV<T>::type *__restrict__ lam,
                                                              uint64_t n_vec, AdjTerms t,
                                                              double *partials) {
    using V = AV<T>;
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kAdjThreads;
    for (uint64_t e = (uint64_t)blockIdx.x * kAdjThreads + threadIdx.x; e < n_vec; e += stride) {
        const typename V::type w = psi[e];
        typename V::type o;
#pragma unroll
        for (int k = 0; k < V::amps; ++k) {
            const uint64_t x = (e << V::bits) | (uint64_t)k;
            double h = 0.0;
            for (int j = 0; j < t.n; ++j) h += (__popcll(x & t.mask[j]) & 1) ? -t.coeff[j] : t.coeff[j];
            const cpx<T> a = V::get(w, k);
            V::put(o, k, cpx<T>{(T)(h * (double)a.re), (T)(h * (double)a.im)});
            acc += h * ((double)a.re * a.re + (double)a.im * a.im);
        }
        lam[e] = o;
    }
    acc = block_sum_d(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// Probe then undo one (controlled) one-qubit gate on psi and lam.
template <typename T>
__global__ __launch_bounds__(kAdjThreads) void k_adjoint_param(typename AV<T>::type *psi,
                                                               typename AV<T>::type *lam, Enum e, int te,
                                                               uint64_t count, Mat2<T> udag,
                                                               Mat2<T> probe, uint32_t lane_ctrl,
                                                               double *partials) {
    using V = AV<T>;
    double acc = 0.0;
    const uint64_t bstep = 1ull << te;
    const uint64_t stride = (uint64_t)gridDim.x * kAdjThreads;
    for (uint64_t j = (uint64_t)blockIdx.x * kAdjThreads + threadIdx.x; j < count; j += stride) {
        const uint64_t a = expand(e, j);
        if ((a & e.check) != e.check) continue;
        typename V::type pa = psi[a], pb = psi[a + bstep], la = lam[a], lb = lam[a + bstep];
#pragma unroll
        for (int k = 0; k < V::amps; ++k) {
            if (((uint32_t)k & lane_ctrl) != lane_ctrl) continue;
            const cpx<T> x0 = V::get(pa, k), x1 = V::get(pb, k);
            const cpx<T> y0 = V::get(la, k), y1 = V::get(lb, k);
            const cpx<T> z0 = cfma(probe.m[0], x0, cmul(probe.m[1], x1));
            const cpx<T> z1 = cfma(probe.m[2], x0, cmul(probe.m[3], x1));
            acc += im_conj_mul(y0, z0) + im_conj_mul(y1, z1);
            V::put(pa, k, cfma(udag.m[0], x0, cmul(udag.m[1], x1)));
            V::put(pb, k, cfma(udag.m[2], x0, cmul(udag.m[3], x1)));
            V::put(la, k, cfma(udag.m[0], y0, cmul(udag.m[1], y1)));
            V::put(lb, k, cfma(udag.m[2], y0, cmul(udag.m[3], y1)));
        }
        psi[a] = pa;
        psi[a + bstep] = pb;
        lam[a] = la;
        lam[a + bstep] = lb;
    }
    acc = block_sum_d(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// complex64 probe/undo on qubit 0 (pair inside one float4)
__global__ __launch_bounds__(kAdjThreads) void k_adjoint_param_q0(float4 *psi, float4 *lam, Enum e,
                                                                  uint64_t count, Mat2<float> udag,
                                                                  Mat2<float> probe,
                                                                  double *partials) {
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * kAdjThreads;
    for (uint64_t j = (uint64_t)blockIdx.x * kAdjThreads + threadIdx.x; j < count; j += stride) {
        const uint64_t a = expand(e, j);
        if ((a & e.check) != e.check) continue;
        const float4 p = psi[a], l = lam[a];
        const cpx<float> x0{p.x, p.y}, x1{p.z, p.w}, y0{l.x, l.y}, y1{l.z, l.w};
        const cpx<float> z0 = cfma(probe.m[0], x0, cmul(probe.m[1], x1));
        const cpx<float> z1 = cfma(probe.m[2], x0, cmul(probe.m[3], x1));
        acc += im_conj_mul(y0, z0) + im_conj_mul(y1, z1);
        const cpx<float> u0 = cfma(udag.m[0], x0, cmul(udag.m[1], x1));
        const cpx<float> u1 = cfma(udag.m[2], x0, cmul(udag.m[3], x1));
        const cpx<float> v0 = cfma(udag.m[0], y0, cmul(udag.m[1], y1));
        const cpx<float> v1 = cfma(udag.m[2], y0, cmul(udag.m[3], y1));
        psi[a] = float4{u0.re, u0.im, u1.re, u1.im};
        lam[a] = float4{v0.re, v0.im, v1.re, v1.im};
    }
    acc = block_sum_d(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// Sum each slot's partials: out[s] = sum_b partials[s * n_blocks + b].
__global__ __launch_bounds__(kAdjThreads) void k_sum_slots(const double *partials, int n_blocks,
                                                           double *out) {
    double acc = 0.0;
    const double *p = partials + (size_t)blockIdx.x * n_blocks;
    for (int i = threadIdx.x; i < n_blocks; i += kAdjThreads) acc += p[i];
    acc = block_sum_d(acc);
    if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

int adjoint_blocks() { return 512; }

hipError_t launch_adjoint_init(const void *psi, void *lam, int n, int dtype, int n_terms,
                               const uint64_t *masks, const double *coeffs, double *partials,
                               hipStream_t s) {
    if (n_terms < 1 || n_terms > kMaxTerms) return hipErrorInvalidValue;
    AdjTerms t{};
    t.n = n_terms;
    for (int j = 0; j < n_terms; ++j) {
        t.mask[j] = masks[j];
        t.coeff[j] = coeffs[j];
    }
    const uint64_t N = 1ull << n;
    const unsigned grid = (unsigned)adjoint_blocks();
    if (dtype == SV_C64)
        k_adjoint_init<float><<<grid, kAdjThreads, 0, s>>>((const float4 *)psi, (float4 *)lam, N / 2, t,
                                                            partials);
    else
        k_adjoint_init<double><<<grid, kAdjThreads, 0, s>>>((const double2 *)psi, (double2 *)lam, N, t,
                                                             partials);
    return hipGetLastError();
}

static Enum adj_enum(int vbits, int te, bool with_target, uint64_t ctrl, uint32_t *lane_ctrl, int *np) {
    Enum e{};
    int pos[64];
    int cnt = 0;
    if (with_target) pos[cnt++] = te;
    *lane_ctrl = (uint32_t)(ctrl & ((1ull << vbits) - 1ull));
    uint64_t ec = ctrl >> vbits;
    while (ec) {
        const int b = __builtin_ctzll(ec);
        ec &= ec - 1;
        if (cnt < kMaxInsert) {
            pos[cnt++] = b;
            e.set |= 1ull << b;
        } else {
            e.check |= 1ull << b;
        }
    }
    std::sort(pos, pos + cnt);
    e.n_pos = cnt;
    for (int i = 0; i < cnt; ++i) e.pos[i] = pos[i];
    *np = cnt;
    return e;
}

hipError_t launch_adjoint_param(void *psi, void *lam, int n, int dtype, int t, uint64_t ctrl,
                                const double *udag, const double *probe, double *partials,
                                hipStream_t s) {
    const int vbits = dtype == SV_C64 ? 1 : 0;
    const uint64_t n_el = (1ull << n) >> vbits;
    uint32_t lane_ctrl = 0;
    int np = 0;
    const unsigned grid = (unsigned)adjoint_blocks();
    if (t < vbits) {
        Enum e = adj_enum(vbits, 0, false, ctrl, &lane_ctrl, &np);
        Mat2<float> u, p;
        for (int i = 0; i < 4; ++i) {
            u.m[i] = {(float)udag[2 * i], (float)udag[2 * i + 1]};
            p.m[i] = {(float)probe[2 * i], (float)probe[2 * i + 1]};
        }
        k_adjoint_param_q0<<<grid, kAdjThreads, 0, s>>>((float4 *)psi, (float4 *)lam, e, n_el >> np, u, p,
                                                        partials);
        return hipGetLastError();
    }
    const int te = t - vbits;
    Enum e = adj_enum(vbits, te, true, ctrl, &lane_ctrl, &np);
    const uint64_t count = n_el >> np;
    if (dtype == SV_C64) {
        Mat2<float> u, p;
        for (int i = 0; i < 4; ++i) {
            u.m[i] = {(float)udag[2 * i], (float)udag[2 * i + 1]};
            p.m[i] = {(float)probe[2 * i], (float)probe[2 * i + 1]};
        }
        k_adjoint_param<float><<<grid, kAdjThreads, 0, s>>>((float4 *)psi, (float4 *)lam, e, te, count, u, p,
                                                            lane_ctrl, partials);
    } else {
        Mat2<double> u, p;
        for (int i = 0; i < 4; ++i) {
            u.m[i] = {udag[2 * i], udag[2 * i + 1]};
            p.m[i] = {probe[2 * i], probe[2 * i + 1]};
        }
        k_adjoint_param<double><<<grid, kAdjThreads, 0, s>>>((double2 *)psi, (double2 *)lam, e, te, count, u,
                                                             p, lane_ctrl, partials);
    }
    return hipGetLastError();
}

hipError_t launch_sum_slots(const double *partials, int n_slots, int n_blocks, double *out,
                            hipStream_t s) {
    if (n_slots <= 0) return hipSuccess;
    k_sum_slots<<<n_slots, kAdjThreads, 0, s>>>(partials, n_blocks, out);
    return hipGetLastError();
}

} // namespace sv
