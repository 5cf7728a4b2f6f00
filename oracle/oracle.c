/*
 * FP64 CPU oracle: plain, slow, obviously correct state-vector simulation.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing).  The
 * product library never includes, links or calls this file.  Every function
 * follows a definition of the paper (section cited at the function) or a
 * textbook identity; there is no blocking, fusion or reordering.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OC_MAXK 6 /* stride of the per-gate target array; largest k of an explicit matrix */

typedef double complex cplx;

int oc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Host threads of the calls that follow (the host baseline is timed on one
 * thread and on all of them); t < 1 restores the default. */
void oc_set_num_threads(int t) {
#ifdef _OPENMP
    static int dflt = 0;
    if (!dflt) dflt = omp_get_max_threads();
    omp_set_num_threads(t < 1 ? dflt : t);
#else
    (void)t;
#endif
}

/* Sec. 2.1: a register starts in a basis state; all amplitude on index x. */
void oc_init_basis(int n, uint64_t x, cplx *psi) {
    const uint64_t dim = 1ULL << n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)dim; ++i) psi[i] = 0.0;
    psi[x] = 1.0;
}

/* One-qubit gate table.  H X Y Z S T follow the gate table of Sec. 1.3.2;
 * the rotations are R_P(theta) = exp(-i theta P / 2) written out with
 * c = cos(theta/2), s = sin(theta/2); U1 is the phase gate diag(1, e^{i theta})
 * that the QFT benchmark applies in controlled form (App. A). */
int oc_gate_matrix(int kind, double theta, cplx m[4]) {
    const double c = cos(0.5 * theta), s = sin(0.5 * theta);
    const double r = 1.0 / sqrt(2.0);
    switch (kind) {
    case OC_H:  m[0] = r;   m[1] = r;    m[2] = r;   m[3] = -r;  return 0;
    case OC_X:  m[0] = 0;   m[1] = 1;    m[2] = 1;   m[3] = 0;   return 0;
    case OC_Y:  m[0] = 0;   m[1] = -I;   m[2] = I;   m[3] = 0;   return 0;
    case OC_Z:  m[0] = 1;   m[1] = 0;    m[2] = 0;   m[3] = -1;  return 0;
    case OC_S:  m[0] = 1;   m[1] = 0;    m[2] = 0;   m[3] = I;   return 0;
    case OC_T:  m[0] = 1;   m[1] = 0;    m[2] = 0;   m[3] = cexp(I * M_PI / 4.0); return 0;
    case OC_RX: m[0] = c;   m[1] = -I * s; m[2] = -I * s; m[3] = c; return 0;
    case OC_RY: m[0] = c;   m[1] = -s;   m[2] = s;   m[3] = c;   return 0;
    case OC_RZ: m[0] = cexp(-0.5 * I * theta); m[1] = 0; m[2] = 0; m[3] = cexp(0.5 * I * theta); return 0;
    case OC_U1: m[0] = 1;   m[1] = 0;    m[2] = 0;   m[3] = cexp(I * theta); return 0;
    default: return -1;
    }
}

/* Entry-wise theta-derivative of the parametrised matrices above. */
int oc_gate_dmatrix(int kind, double theta, cplx m[4]) {
    const double c = cos(0.5 * theta), s = sin(0.5 * theta);
    switch (kind) {
    case OC_RX: m[0] = -0.5 * s; m[1] = -0.5 * I * c; m[2] = -0.5 * I * c; m[3] = -0.5 * s; return 0;
    case OC_RY: m[0] = -0.5 * s; m[1] = -0.5 * c; m[2] = 0.5 * c; m[3] = -0.5 * s; return 0;
    case OC_RZ: m[0] = -0.5 * I * cexp(-0.5 * I * theta); m[1] = 0; m[2] = 0;
                m[3] = 0.5 * I * cexp(0.5 * I * theta); return 0;
    case OC_U1: m[0] = 0; m[1] = 0; m[2] = 0; m[3] = I * cexp(I * theta); return 0;
    default: return -1;
    }
}

/* The i-th integer whose bit t is 0: bits below t kept, bits from t upward
 * moved one place up (Alg. 1, first step of the loop body). */
static uint64_t ith_with_zero_bit(uint64_t i, int t) {
    const uint64_t below = i & ((1ULL << t) - 1);
    const uint64_t above = (i >> t) << (t + 1);
    return above | below;
}

/* Alg. 1 (Sec. 2.3) and its controlled adaptation: loop over the 2^{n-1}
 * pairs; a has bit t clear, b = a with bit t set; both new values are formed
 * from the old pair.  With controls, the pair is updated only where every
 * control bit is 1 (a and b agree on every bit except t). */
void oc_apply_1q(int n, cplx *psi, int t, uint64_t ctrl, const cplx m[4]) {
    const uint64_t pairs = 1ULL << (n - 1);
    const cplx g00 = m[0], g01 = m[1], g10 = m[2], g11 = m[3];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)pairs; ++i) {
        const uint64_t a = ith_with_zero_bit((uint64_t)i, t);
        const uint64_t b = a | (1ULL << t);
        if ((a & ctrl) != ctrl) continue;
        const cplx va = psi[a], vb = psi[b];
        psi[a] = g00 * va + g01 * vb;
        psi[b] = g10 * va + g11 * vb;
    }
}

/* k-qubit generalisation of Alg. 1: the 2^{n-k} groups of amplitudes that
 * differ only in the bits q[0..k-1]; each group is multiplied by the 2^k x 2^k
 * matrix, local index bit j <-> qubit q[j]. */
void oc_apply_kq(int n, cplx *psi, int k, const int *q, uint64_t ctrl, const cplx *m) {
    const int dim = 1 << k;
    int sorted[OC_MAXK];
    if (k < 1 || k > OC_MAXK) return;
    for (int j = 0; j < k; ++j) sorted[j] = q[j];
    for (int a = 1; a < k; ++a)
        for (int b = a; b > 0 && sorted[b - 1] > sorted[b]; --b) {
            int tmp = sorted[b]; sorted[b] = sorted[b - 1]; sorted[b - 1] = tmp;
        }
    const uint64_t groups = 1ULL << (n - k);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)groups; ++i) {
        uint64_t base = (uint64_t)i;
        for (int j = 0; j < k; ++j) base = ith_with_zero_bit(base, sorted[j]);
        if ((base & ctrl) != ctrl) continue;
        uint64_t idx[1 << OC_MAXK];
        cplx in[1 << OC_MAXK];
        for (int l = 0; l < dim; ++l) {
            uint64_t x = base;
            for (int j = 0; j < k; ++j)
                if ((l >> j) & 1) x |= 1ULL << q[j];
            idx[l] = x;
            in[l] = psi[x];
        }
        for (int r = 0; r < dim; ++r) {
            cplx acc = 0.0;
            for (int c = 0; c < dim; ++c) acc += m[(size_t)r * dim + c] * in[c];
            psi[idx[r]] = acc;
        }
    }
}

static int n_targets(const int *tq, int g) {
    int k = 0;
    while (k < OC_MAXK && tq[g * OC_MAXK + k] >= 0) ++k;
    return k;
}

static void dagger(int dim, const cplx *m, cplx *out) {
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c) out[(size_t)c * dim + r] = conj(m[(size_t)r * dim + c]);
}

/* Apply gate g with angle th (or its inverse). */
static void apply_gate(int n, cplx *psi, int g, const int *kind, const int *tq,
                       const uint64_t *ctrl, double th, const int64_t *mat_off,
                       const cplx *mats, int inverse) {
    const int k = n_targets(tq, g);
    if (kind[g] == OC_MAT) {
        const int dim = 1 << k;
        const cplx *m = mats + mat_off[g];
        if (inverse) {
            cplx *mi = (cplx *)malloc(sizeof(cplx) * dim * dim);
            dagger(dim, m, mi);
            oc_apply_kq(n, psi, k, tq + g * OC_MAXK, ctrl[g], mi);
            free(mi);
        } else {
            oc_apply_kq(n, psi, k, tq + g * OC_MAXK, ctrl[g], m);
        }
        return;
    }
    cplx m[4], mi[4];
    oc_gate_matrix(kind[g], th, m);
    if (inverse) dagger(2, m, mi);
    oc_apply_1q(n, psi, tq[g * OC_MAXK], ctrl[g], inverse ? mi : m);
}

void oc_run(int n, cplx *psi, int n_gates, const int *kind, const int *tq,
            const uint64_t *ctrl, const double *theta, const int64_t *mat_off,
            const cplx *mats, int inverse) {
    for (int s = 0; s < n_gates; ++s) {
        const int g = inverse ? n_gates - 1 - s : s;
        apply_gate(n, psi, g, kind, tq, ctrl, theta[g], mat_off, mats, inverse);
    }
}

/* Sec. 2.4: the probability of outcome x is |psi_x|^2 = re^2 + im^2. */
double oc_probabilities(int n, const cplx *psi, double *p) {
    const uint64_t dim = 1ULL << n;
    double total = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : total)
    for (int64_t x = 0; x < (int64_t)dim; ++x) {
        const double px = creal(psi[x]) * creal(psi[x]) + cimag(psi[x]) * cimag(psi[x]);
        if (p) p[x] = px;
        total += px;
    }
    return total;
}

/* Z-string observable: Z^m is diagonal with entry (-1)^popcount(x & m), so its
 * expectation is the probability-weighted sum of those signs (Sec. 1.3.3:
 * outcome probabilities in the computational basis). */
static double zsum_at(uint64_t x, int n_terms, const uint64_t *masks, const double *coeffs) {
    double h = 0.0;
    for (int j = 0; j < n_terms; ++j) {
        const int odd = __builtin_popcountll(x & masks[j]) & 1;
        h += odd ? -coeffs[j] : coeffs[j];
    }
    return h;
}

double oc_expectation_z(int n, const cplx *psi, int n_terms, const uint64_t *masks,
                        const double *coeffs) {
    const uint64_t dim = 1ULL << n;
    double total = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : total)
    for (int64_t x = 0; x < (int64_t)dim; ++x) {
        const double px = creal(psi[x]) * creal(psi[x]) + cimag(psi[x]) * cimag(psi[x]);
        total += px * zsum_at((uint64_t)x, n_terms, masks, coeffs);
    }
    return total;
}

static double gate_theta(int g, const double *theta, const int *param, const double *params) {
    return param[g] >= 0 ? params[param[g]] : theta[g];
}

/* Adjoint differentiation, step by step:
 *   forward   psi = U_G ... U_1 |0>;  lam = H psi;  L = <psi|lam>
 *   backward  for g = G..1:  psi <- U_g^dagger psi            (now psi_{g-1})
 *             if gate g carries parameter p:
 *                 mu = (dU_g/dtheta) psi_{g-1}   (zero outside the control subspace)
 *                 grad[p] += 2 Re <lam|mu>
 *             lam <- U_g^dagger lam
 * H is Hermitian, so dL/dtheta = 2 Re <psi|H dpsi/dtheta>, and lam carries
 * U_{g+1}^dagger ... U_G^dagger H psi at step g. */
double oc_adjoint_grad(int n, cplx *psi, cplx *lam, cplx *mu, int n_gates, const int *kind,
                       const int *tq, const uint64_t *ctrl, const double *theta,
                       const int *param, const int64_t *mat_off, const cplx *mats,
                       const double *params, int n_params, int n_terms, const uint64_t *masks,
                       const double *coeffs, double *grad) {
    const uint64_t dim = 1ULL << n;
    oc_init_basis(n, 0, psi);
    for (int g = 0; g < n_gates; ++g)
        apply_gate(n, psi, g, kind, tq, ctrl, gate_theta(g, theta, param, params), mat_off, mats, 0);

    double loss = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : loss)
    for (int64_t x = 0; x < (int64_t)dim; ++x) {
        lam[x] = zsum_at((uint64_t)x, n_terms, masks, coeffs) * psi[x];
        loss += creal(conj(psi[x]) * lam[x]);
    }
    for (int p = 0; p < n_params; ++p) grad[p] = 0.0;

    for (int g = n_gates - 1; g >= 0; --g) {
        const double th = gate_theta(g, theta, param, params);
        apply_gate(n, psi, g, kind, tq, ctrl, th, mat_off, mats, 1);
        if (param[g] >= 0) {
            cplx dm[4];
            if (kind[g] == OC_MAT || oc_gate_dmatrix(kind[g], th, dm) != 0) return NAN;
            memcpy(mu, psi, sizeof(cplx) * dim);
            oc_apply_1q(n, mu, tq[g * OC_MAXK], ctrl[g], dm);
            double acc = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : acc)
            for (int64_t x = 0; x < (int64_t)dim; ++x) {
                if (((uint64_t)x & ctrl[g]) != ctrl[g]) continue; /* derivative is 0 there */
                acc += creal(conj(lam[x]) * mu[x]);
            }
            grad[param[g]] += 2.0 * acc;
        }
        apply_gate(n, lam, g, kind, tq, ctrl, th, mat_off, mats, 1);
    }
    return loss;
}

/* ------------------------------------------------------------ measurement */
/* Outcome index of x for the qubits of mask: bit i = bit of the i-th lowest
 * qubit in mask. */
static uint64_t outcome_of(int n, uint64_t x, uint64_t mask) {
    uint64_t o = 0;
    int i = 0;
    for (int b = 0; b < n; ++b) {
        if (!((mask >> b) & 1ULL)) continue;
        if ((x >> b) & 1ULL) o |= 1ULL << i;
        ++i;
    }
    return o;
}

void oc_marginals(int n, const cplx *psi, uint64_t mask, double *out) {
    const uint64_t dim = 1ULL << n;
    const int k = __builtin_popcountll(mask);
    for (uint64_t o = 0; o < (1ULL << k); ++o) out[o] = 0.0;
    for (uint64_t x = 0; x < dim; ++x) {
        const double px = creal(psi[x]) * creal(psi[x]) + cimag(psi[x]) * cimag(psi[x]);
        out[outcome_of(n, x, mask)] += px;
    }
}

double oc_collapse(int n, cplx *psi, uint64_t mask, uint64_t value) {
    const uint64_t dim = 1ULL << n;
    const uint64_t want = value & mask;
    double p = 0.0;
    for (uint64_t x = 0; x < dim; ++x)
        if ((x & mask) == want) p += creal(psi[x]) * creal(psi[x]) + cimag(psi[x]) * cimag(psi[x]);
    if (p == 0.0) return 0.0;
    const double s = 1.0 / sqrt(p);
    for (uint64_t x = 0; x < dim; ++x) psi[x] = ((x & mask) == want) ? psi[x] * s : 0.0;
    return p;
}

uint64_t oc_select(uint64_t m, const double *p, double u) {
    double total = 0.0;
    for (uint64_t i = 0; i < m; ++i) total += p[i];
    const double t = u * total;
    double c = 0.0;
    uint64_t last = 0;
    for (uint64_t i = 0; i < m; ++i) {
        c += p[i];
        if (p[i] > 0.0) last = i;
        if (c > t) return i;
    }
    return last;
}

void oc_sample(int n, const cplx *psi, int n_samples, const double *uniforms, uint64_t *out) {
    const uint64_t dim = 1ULL << n;
    double *p = (double *)malloc(dim * sizeof(double));
    for (uint64_t x = 0; x < dim; ++x) p[x] = creal(psi[x]) * creal(psi[x]) + cimag(psi[x]) * cimag(psi[x]);
    for (int s = 0; s < n_samples; ++s) out[s] = oc_select(dim, p, uniforms[s]);
    free(p);
}

double oc_measure(int n, cplx *psi, uint64_t mask, double u, uint64_t *value) {
    const int k = __builtin_popcountll(mask);
    double *marg = (double *)malloc(((size_t)1 << k) * sizeof(double));
    oc_marginals(n, psi, mask, marg);
    const uint64_t o = oc_select(1ULL << k, marg, u);
    free(marg);
    uint64_t v = 0;
    int i = 0;
    for (int b = 0; b < n; ++b) {
        if (!((mask >> b) & 1ULL)) continue;
        if ((o >> i) & 1ULL) v |= 1ULL << b;
        ++i;
    }
    *value = v;
    return oc_collapse(n, psi, mask, v);
}
