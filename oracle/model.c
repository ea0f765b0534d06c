/*
 * model.c -- lattice, local field, energy and observables (FP64 oracle).
 *
 * Test infrastructure: see oracle.h.
 */
#include <math.h>
#include "oracle.h"

/* Coordinates of site i = x + L*(y + L*z). */
static void coords(int L, int i, int x[3])
{
    x[0] = i % L;
    x[1] = (i / L) % L;
    x[2] = i / (L * L);
}

static int site(int L, const int x[3])
{
    return x[0] + L * (x[1] + L * x[2]);
}

/* Periodic boundary conditions (Sec. II.A). */
int or_neighbour(int L, int i, int mu, int dir)
{
    int x[3];
    coords(L, i, x);
    x[mu] = (x[mu] + dir + L) % L;
    return site(L, x);
}

/* Element (a, b) of the bond matrix of bond (i, i + e_mu). */
static double bond(const double *M, int N, int mu, int i, int a, int b)
{
    return M[(((long)mu * N + i) * 3 + a) * 3 + b];
}

/* h_i = sum_mu [ M_{mu,i} s_{i+e_mu} + M_{mu,i-e_mu}^T s_{i-e_mu} ].
 * Each bond (i, j = i + e_mu) contributes -s_i^T M s_j to the Hamiltonian
 * Eq. (1); its derivative with respect to s_i is -M s_j and with respect to
 * s_j is -M^T s_i, so h_i = -dH/ds_i collects M s_{i+e_mu} from the bond
 * where i is the first end and M^T s_{i-e_mu} from the bond where it is the
 * second.  With the paper's symmetric D the transpose is immaterial. */
void or_local_field(int L, const double *M, const double *s, int i, double h[3])
{
    const int N = L * L * L;
    h[0] = h[1] = h[2] = 0.0;
    for (int mu = 0; mu < 3; ++mu) {
        int jp = or_neighbour(L, i, mu, +1);
        int jm = or_neighbour(L, i, mu, -1);
        for (int a = 0; a < 3; ++a) {
            for (int b = 0; b < 3; ++b) {
                h[a] += bond(M, N, mu, i, a, b) * s[3 * jp + b];
                h[a] += bond(M, N, mu, jm, b, a) * s[3 * jm + b];
            }
        }
    }
}

/* Eq. (1): H = - sum_<x,y> s_x^T M_xy s_y, one term per bond. */
double or_energy(int L, const double *M, const double *s)
{
    const int N = L * L * L;
    double E = 0.0;
    for (int i = 0; i < N; ++i) {
        for (int mu = 0; mu < 3; ++mu) {
            int j = or_neighbour(L, i, mu, +1);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    E -= s[3 * i + a] * bond(M, N, mu, i, a, b) * s[3 * j + b];
        }
    }
    return E;
}

/* Schwinger-Dyson sums of appendix A.4. */
void or_sd_sums(int L, const double *M, const double *s, double *sd1, double *sd2)
{
    const int N = L * L * L;
    double a1 = 0.0, a2 = 0.0;
    for (int i = 0; i < N; ++i) {
        double h[3];
        or_local_field(L, M, s, i, h);
        double sh = s[3 * i] * h[0] + s[3 * i + 1] * h[1] + s[3 * i + 2] * h[2];
        double hh = h[0] * h[0] + h[1] * h[1] + h[2] * h[2];
        a1 += sh;
        a2 += hh - sh * sh;
    }
    *sd1 = a1;
    *sd2 = a2;
}

/* Chirality of Sec. II.B: zeta_{x,mu} = s_{x+e_mu} . (s_x cross s_{x-e_mu}). */
static double chirality(int L, const double *s, int i, int mu)
{
    int jp = or_neighbour(L, i, mu, +1);
    int jm = or_neighbour(L, i, mu, -1);
    const double *u = s + 3 * i, *w = s + 3 * jm, *v = s + 3 * jp;
    double c0 = u[1] * w[2] - u[2] * w[1];
    double c1 = u[2] * w[0] - u[0] * w[2];
    double c2 = u[0] * w[1] - u[1] * w[0];
    return v[0] * c0 + v[1] * c1 + v[2] * c2;
}

/* Overlap tensor and chiral-glass overlap at k = 0 and k = (2 pi / L) e_d,
 * Fourier convention of Sec. II.B: (1/N) sum_x f(x) exp(+i k . x). */
void or_overlaps(int L, const double *sa, const double *sb,
                 double q0[9], double qk_re[27], double qk_im[27],
                 double cg0[3], double cgk_re[9], double cgk_im[9])
{
    const int N = L * L * L;
    const double two_pi = 6.283185307179586476925286766559;
    for (int n = 0; n < 9; ++n) q0[n] = 0.0;
    for (int n = 0; n < 27; ++n) qk_re[n] = qk_im[n] = 0.0;
    for (int n = 0; n < 3; ++n) cg0[n] = 0.0;
    for (int n = 0; n < 9; ++n) cgk_re[n] = cgk_im[n] = 0.0;

    for (int i = 0; i < N; ++i) {
        int x[3];
        coords(L, i, x);
        double q[9], kappa[3];
        for (int al = 0; al < 3; ++al)
            for (int be = 0; be < 3; ++be)
                q[al * 3 + be] = sa[3 * i + al] * sb[3 * i + be];
        for (int mu = 0; mu < 3; ++mu)
            kappa[mu] = chirality(L, sa, i, mu) * chirality(L, sb, i, mu);

        for (int n = 0; n < 9; ++n) q0[n] += q[n];
        for (int mu = 0; mu < 3; ++mu) cg0[mu] += kappa[mu];
        for (int d = 0; d < 3; ++d) {
            double ph = two_pi * (double)x[d] / (double)L;
            double c = cos(ph), sn = sin(ph);
            for (int n = 0; n < 9; ++n) {
                qk_re[d * 9 + n] += q[n] * c;
                qk_im[d * 9 + n] += q[n] * sn;
            }
            for (int mu = 0; mu < 3; ++mu) {
                cgk_re[d * 3 + mu] += kappa[mu] * c;
                cgk_im[d * 3 + mu] += kappa[mu] * sn;
            }
        }
    }
    for (int n = 0; n < 9; ++n) q0[n] /= N;
    for (int n = 0; n < 27; ++n) { qk_re[n] /= N; qk_im[n] /= N; }
    for (int n = 0; n < 3; ++n) cg0[n] /= N;
    for (int n = 0; n < 9; ++n) { cgk_re[n] /= N; cgk_im[n] /= N; }
}
