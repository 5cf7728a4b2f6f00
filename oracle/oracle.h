/*
 * FP64 CPU oracle for the state-vector simulator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this code; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP library: gate matrices, index arithmetic and reductions are written
 * here independently from the paper's definitions.
 *
 * State layout: 2^n amplitudes, C99 double complex (re, im interleaved),
 * qubit q = bit q of the amplitude index.  All functions are plain loops in
 * the order the paper states them; OpenMP only splits the independent loop
 * iterations (the paper notes the body of the gate loop is independent).
 */
#ifndef SV_ORACLE_H
#define SV_ORACLE_H

#include <complex.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Gate kinds understood by the oracle (its own numbering). */
enum {
    OC_H = 1, OC_X = 2, OC_Y = 3, OC_Z = 4, OC_S = 5, OC_T = 6,
    OC_RX = 7, OC_RY = 8, OC_RZ = 9, OC_U1 = 10,
    OC_MAT = 11 /* explicit 2^k x 2^k matrix */
};

/* |x>: amplitude 1 at index x, 0 elsewhere (Sec. 2.1: a new register is |0...0>). */
void oc_init_basis(int n, uint64_t x, double complex *psi);

/* 2x2 matrix of a named one-qubit gate, row-major [[m0, m1], [m2, m3]]. */
int oc_gate_matrix(int kind, double theta, double complex m[4]);

/* d/dtheta of oc_gate_matrix for the parametrised kinds (RX RY RZ U1). */
int oc_gate_dmatrix(int kind, double theta, double complex m[4]);

/* Alg. 1 of Sec. 2.3 with the controlled variant: for every pair (a, b) that
 * differs only in bit t, apply [[m0,m1],[m2,m3]] to (v_a, v_b), but only where
 * every bit of ctrl is set. */
void oc_apply_1q(int n, double complex *psi, int t, uint64_t ctrl, const double complex m[4]);

/* Generic k-qubit unitary on qubits q[0..k-1] (local bit j <-> qubit q[j]),
 * applied where every bit of ctrl is set.  Used for two-qubit gates and for
 * checking fused blocks.  m is 2^k x 2^k row-major. */
void oc_apply_kq(int n, double complex *psi, int k, const int *q, uint64_t ctrl,
                 const double complex *m);

/* Run a gate list.  Gate g: kind[g]; targets tq[g*6 .. g*6+5], -1 padded
 * (at most 6 targets); ctrl[g]; theta[g]; for OC_MAT, mat_off[g] indexes the
 * first complex entry of its matrix in mats.  inverse != 0 applies the
 * conjugate-transposed gates in reverse order. */
void oc_run(int n, double complex *psi, int n_gates, const int *kind, const int *tq,
            const uint64_t *ctrl, const double *theta, const int64_t *mat_off,
            const double complex *mats, int inverse);

/* Sec. 2.4: p_x = |psi_x|^2 for every x; returns sum_x p_x. */
double oc_probabilities(int n, const double complex *psi, double *p);

/* <psi| sum_j c_j Z^{m_j} |psi> = sum_x p_x sum_j c_j (-1)^popcount(x & m_j). */
double oc_expectation_z(int n, const double complex *psi, int n_terms,
                        const uint64_t *masks, const double *coeffs);

/* Adjoint-method gradient of L(theta) = <psi(theta)| H |psi(theta)>, psi(theta)
 * = U_G ... U_1 |0>, H = sum_j c_j Z^{m_j}.  Gates as in oc_run plus param[g]
 * (-1 = fixed; else theta[g] is replaced by params[param[g]]).  Needs three
 * work vectors of 2^n amplitudes.  Writes dL/dparams into grad (n_params
 * entries) and returns L. */
double oc_adjoint_grad(int n, double complex *psi, double complex *lam, double complex *mu,
                       int n_gates, const int *kind, const int *tq, const uint64_t *ctrl,
                       const double *theta, const int *param, const int64_t *mat_off,
                       const double complex *mats, const double *params, int n_params,
                       int n_terms, const uint64_t *masks, const double *coeffs,
                       double *grad);

/* Sec. 1.3.3: measuring the k qubits of 'mask' in the computational basis
 * (projectors M_o = |o><o| on those qubits) has 2^k outcomes; outcome o
 * (bit i of o = value of the i-th lowest qubit of mask) has probability
 * p(o) = <psi|M_o|psi> = sum of |psi_x|^2 over the x whose mask bits spell o.
 * Writes the 2^k probabilities, summed in index order. */
void oc_marginals(int n, const double complex *psi, uint64_t mask, double *out);

/* Sec. 1.3.3 post-measurement state M psi / sqrt(p) for the projector M onto
 * the x with (x & mask) == (value & mask); returns p.  The state is left
 * unchanged when p == 0. */
double oc_collapse(int n, double complex *psi, uint64_t mask, uint64_t value);

/* Sec. 2.4 outcome selection from outcome probabilities p[0..m-1], by the
 * inverse cumulative distribution: with c_i = p_0 + ... + p_i summed in
 * index order and T = c_{m-1}, the outcome for u in [0, 1) is the smallest i
 * with c_i > u T (the last i with p_i > 0 if rounding leaves none). */
uint64_t oc_select(uint64_t m, const double *p, double u);

/* Full-register samples (the state is not changed): outcome s is oc_select
 * over p_x = |psi_x|^2 with u = uniforms[s]. */
void oc_sample(int n, const double complex *psi, int n_samples, const double *uniforms, uint64_t *out);

/* Measure the qubits of mask: select an outcome of oc_marginals with u,
 * collapse onto it, write it (as bits at the mask positions) to *value and
 * return its probability. */
double oc_measure(int n, double complex *psi, uint64_t mask, double u, uint64_t *value);

/* Number of OpenMP threads the oracle's loops use. */
int oc_num_threads(void);
void oc_set_num_threads(int t);

#ifdef __cplusplus
}
#endif
#endif
