/*
 * oracle.h -- plain FP64 CPU reference of the anisotropic Heisenberg
 * spin-glass Monte Carlo (Baity-Jesi, Fernandez, Martin-Mayor, Sanz,
 * arXiv:1309.1599).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header or table with the GPU
 * library; the two meet only through seeded inputs and through the
 * published Philox4x32-10 definition, which each side implements itself.
 *
 * Every routine is written for clarity, not speed: direct loops over sites,
 * neighbours recomputed from coordinates, FP64 throughout (FP32 inputs are
 * widened exactly before use).
 *
 * Conventions (shared by contract with the GPU library, not by code):
 *   site i = x + L*(y + L*z), periodic boundaries, L even, colour (x+y+z)&1;
 *   couplings M[mu][i][a][b], mu = 0,1,2 (x,y,z), bond (i, i+e_mu),
 *   bond energy  -sum_ab s_i[a] M[a][b] s_{i+e_mu}[b]   (Sec. II.A, Eq. (1)
 *   with the symmetric J*1 + D generalised to a full 3x3 matrix);
 *   spins s[i][3] of one chain.
 *
 * Parity status: every function here is pinned by the not-gpu tests
 * (tests/test_oracle_*.py); none is "parity unpinned".
 */
#ifndef PTSG_ORACLE_H
#define PTSG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Random-number tags (fourth counter word, bits 28..31). */
enum { OR_TAG_HB = 0, OR_TAG_PT = 1, OR_TAG_INIT = 2 };

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11). */
void or_philox4x32_10(const uint32_t key[2], const uint32_t ctr[4], uint32_t out[4]);

/* Periodic neighbour of site i along axis mu (0..2), dir = +1 or -1. */
int or_neighbour(int L, int i, int mu, int dir);

/* Local field h_i: the vector with dE/ds_i = -h_i (appendix A.1, Eq. for the
 * conditional density).  M is [3][N][3][3], s is [N][3]. */
void or_local_field(int L, const double *M, const double *s, int i, double h[3]);

/* Hamiltonian, Eq. (1): -sum over the 3N bonds of s_i^T M s_{i+e_mu}. */
double or_energy(int L, const double *M, const double *s);

/* Heat-bath draw of one spin from P(s) ~ exp(beta s.h) (appendix A.1), using
 * the two uniforms v, u2 in (0,1).  Writes the new spin into s. */
void or_heatbath_spin(const double h[3], double beta, double v, double u2, double s[3]);

/* Overrelaxation (appendix A.1): s <- 2 h (h.s)/h^2 - s, then |s| = 1.
 * Leaves s unchanged if h = 0. */
void or_overrelax_spin(const double h[3], double s[3]);

/* Uniforms from Philox words (exact in both FP32 and FP64). */
double or_u23(uint32_t w);            /* ((w>>9)+0.5) * 2^-23 */
double or_u52(uint32_t w0, uint32_t w1); /* (((w0>>6)<<26 | (w1>>6)) + 0.5) * 2^-52 */

/* Fourth counter word for (tag, temperature slot, replica). */
uint32_t or_ctr3(uint32_t tag, uint32_t tslot, uint32_t rep);

/* Row-ordered overrelaxation sweep: rows of 8 along x in two classes
 * ((x/8 + y + z) mod 2), sequential in x inside a row.  L must be 8 or a
 * multiple of 16 (returns -1 otherwise, leaving s unchanged). */
int or_row_sweep(int L, const double *M, double *s);

/* One checkerboard half-sweep of colour c over one chain.
 * kind 0 = overrelaxation, 1 = heat-bath at inverse temperature beta; the
 * heat-bath draws use counter (i, hb_sweep, sample, ctr3(HB, tslot, rep)). */
void or_half_sweep(int L, const double *M, double *s, int colour, int kind,
                   double beta, uint64_t seed, uint32_t hb_sweep,
                   uint32_t sample, uint32_t tslot, uint32_t rep);

/* Hot start: uniform spins on the sphere from counter
 * (i, 0, sample, ctr3(INIT, chain, rep)). */
void or_init_spins(int L, double *s, uint64_t seed, uint32_t sample,
                   uint32_t chain, uint32_t rep);

/* One parallel-tempering pass for one (sample, replica): pairs of slots
 * (k, k+1), k = 0..T-2 in ascending order, Metropolis acceptance.
 * beta[T] by slot; E[chain] by chain; perm[T]: chain at each slot (updated).
 * Uniform for pair k: counter (k, pass, sample, ctr3(PT, 0, rep)).
 * Returns the number of accepted swaps. */
int or_pt_pass(int T, const double *beta, const double *E, int32_t *perm,
               uint64_t seed, uint32_t pass, uint32_t sample, uint32_t rep);

/* Observables of Sec. II.B for replicas a, b of one sample at one
 * temperature (spins sa, sb [N][3]).  With k_d = (2 pi / L) e_d:
 *   q0[9]        Q^{ab}(0)[alpha*3+beta] = (1/N) sum_x sa_alpha sb_beta
 *   qk_re/im[27] same times exp(+i k_d . x), index d*9 + alpha*3 + beta
 *   cg0[3]       (1/N) sum_x zeta^a_{x,mu} zeta^b_{x,mu}
 *   cgk_re/im[9] same times exp(+i k_d . x), index d*3 + mu
 * zeta_{x,mu} = s_{x+e_mu} . (s_x cross s_{x-e_mu}). */
void or_overlaps(int L, const double *sa, const double *sb,
                 double q0[9], double qk_re[27], double qk_im[27],
                 double cg0[3], double cgk_re[9], double cgk_im[9]);

/* Schwinger-Dyson sums (appendix A.4): sd1 = sum_x s.h,
 * sd2 = sum_x (h^2 - (s.h)^2). */
void or_sd_sums(int L, const double *M, const double *s, double *sd1, double *sd2);

#ifdef __cplusplus
}
#endif
#endif
