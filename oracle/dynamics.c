/*
 * dynamics.c -- heat-bath, overrelaxation, checkerboard sweeps, hot start
 * and parallel tempering (FP64 oracle, appendix A.1).
 *
 * Test infrastructure: see oracle.h.
 */
#include <math.h>
#include "oracle.h"

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static void normalise(double s[3])
{
    double n = sqrt(dot3(s, s));
    s[0] /= n; s[1] /= n; s[2] /= n;
}

/* Heat-bath.  The conditional density of one spin is proportional to
 * exp(beta s.h) on the unit sphere (appendix A.1).  With n = h/|h| and
 * X = beta |h|, c = cos(theta) = s.n has density ~ exp(X c) on [-1, 1] and
 * the azimuth phi about n is uniform.  Inverting the upper tail of the CDF,
 *   1 - F(c) = (e^X - e^{X c}) / (e^X - e^{-X}) = v,
 * gives t = 1 - c = -log1p(v * expm1(-2X)) / X, finite for every X > 0.
 * (This is the p = 3 case of A. T. A. Wood, "Simulation of the von
 * Mises-Fisher distribution", 1994.)  For X below 2^-60 the density is flat:
 * t = 2v, n = z-hat.  The frame (b1, b2) orthogonal to n is the branch-free
 * construction of Duff et al., "Building an Orthonormal Basis, Revisited",
 * JCGT 6(1), 2017. */
void or_heatbath_spin(const double h[3], double beta, double v, double u2, double s[3])
{
    const double two_pi = 6.283185307179586476925286766559;
    double hn = sqrt(dot3(h, h));
    double X = beta * hn;
    double n[3], t;
    if (X < 0x1p-60) {
        n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
        t = 2.0 * v;
    } else {
        n[0] = h[0] / hn; n[1] = h[1] / hn; n[2] = h[2] / hn;
        t = -log1p(v * expm1(-2.0 * X)) / X;
    }
    double cos_t = 1.0 - t;
    double sin2 = t * (2.0 - t);
    double sin_t = sin2 > 0.0 ? sqrt(sin2) : 0.0;
    double phi = two_pi * u2;

    double sign = copysign(1.0, n[2]);
    double a = -1.0 / (sign + n[2]);
    double b = n[0] * n[1] * a;
    double b1[3] = {1.0 + sign * n[0] * n[0] * a, sign * b, -sign * n[0]};
    double b2[3] = {b, sign + n[1] * n[1] * a, -n[1]};

    double cp = cos(phi), sp = sin(phi);
    for (int k = 0; k < 3; ++k)
        s[k] = cos_t * n[k] + sin_t * (cp * b1[k] + sp * b2[k]);
    normalise(s);
}

/* Overrelaxation (appendix A.1): reflect s about h, keeping s.h, hence the
 * energy, fixed; renormalise afterwards.  No move when h = 0. */
void or_overrelax_spin(const double h[3], double s[3])
{
    double hh = dot3(h, h);
    if (hh == 0.0) return;
    double f = 2.0 * dot3(h, s) / hh;
    for (int k = 0; k < 3; ++k) s[k] = f * h[k] - s[k];
    normalise(s);
}

/* Checkerboard half-sweep (appendix A.1: first one sublattice, then the
 * other).  Sites of one colour share no bond, so the in-place update in
 * site order gives the same result as any other order. */
void or_half_sweep(int L, const double *M, double *s, int colour, int kind,
                   double beta, uint64_t seed, uint32_t hb_sweep,
                   uint32_t sample, uint32_t tslot, uint32_t rep)
{
    const int N = L * L * L;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int i = 0; i < N; ++i) {
        int x = i % L, y = (i / L) % L, z = i / (L * L);
        if (((x + y + z) & 1) != colour) continue;
        double h[3];
        or_local_field(L, M, s, i, h);
        if (kind == 0) {
            or_overrelax_spin(h, s + 3 * i);
        } else {
            uint32_t ctr[4] = {(uint32_t)i, hb_sweep, sample,
                               or_ctr3(OR_TAG_HB, tslot, rep)};
            uint32_t w[4];
            or_philox4x32_10(key, ctr, w);
            or_heatbath_spin(h, beta, or_u23(w[0]), or_u23(w[1]), s + 3 * i);
        }
    }
}

/* Row-ordered overrelaxation sweep (the alternative deterministic order of
 * Sec. III and appendix A.3: rows of 8 spins along x, updated one after the
 * other inside a row, rows that share no bond updated together).  Reading
 * taken: row (b, y, z) holds x = 8b .. 8b+7; its class is (b + y + z) mod 2.
 * Two rows of one class share no bond when the number of rows along x,
 * B = L/8, is even (rows that touch differ by one in exactly one of b, y, z;
 * b = 0 and b = B-1 touch across the periodic boundary and then differ in
 * parity) or B = 1 (a row is a whole x line, its own neighbour along x).
 * For odd B >= 3 the rows b = 0 and b = B-1 of one (y, z) share a bond and
 * fall in the same class, so the class order would not be defined by the
 * classes alone: such L are refused (return -1).  The class-0 rows, then the
 * class-1 rows, in any order; inside a row the sites go in increasing x,
 * each seeing the spins already updated before it.  L must be a multiple
 * of 8. */
int or_row_sweep(int L, const double *M, double *s)
{
    const int B = L / 8;
    if (L % 8 != 0 || (B > 1 && B % 2 != 0)) return -1;
    for (int cls = 0; cls < 2; ++cls)
        for (int z = 0; z < L; ++z)
            for (int y = 0; y < L; ++y)
                for (int b = 0; b < B; ++b) {
                    if (((b + y + z) & 1) != cls) continue;
                    for (int x = 8 * b; x < 8 * b + 8; ++x) {
                        const int i = x + L * (y + L * z);
                        double h[3];
                        or_local_field(L, M, s, i, h);
                        or_overrelax_spin(h, s + 3 * i);
                    }
                }
    return 0;
}

/* Hot start: z = 1 - 2 u1 is uniform on [-1, 1] and the azimuth uniform,
 * which is the uniform law on the sphere (Archimedes). */
void or_init_spins(int L, double *s, uint64_t seed, uint32_t sample,
                   uint32_t chain, uint32_t rep)
{
    const int N = L * L * L;
    const double two_pi = 6.283185307179586476925286766559;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int i = 0; i < N; ++i) {
        uint32_t ctr[4] = {(uint32_t)i, 0u, sample, or_ctr3(OR_TAG_INIT, chain, rep)};
        uint32_t w[4];
        or_philox4x32_10(key, ctr, w);
        double z = 1.0 - 2.0 * or_u23(w[0]);
        double phi = two_pi * or_u23(w[1]);
        double r = sqrt(1.0 - z * z);
        s[3 * i] = r * cos(phi);
        s[3 * i + 1] = r * sin(phi);
        s[3 * i + 2] = z;
    }
}

/* Parallel tempering (appendix A.1): propose exchanging the configurations
 * at neighbouring temperatures, accept with the Metropolis probability
 * min(1, exp((beta_k - beta_{k+1}) (E_k - E_{k+1}))).  Exchanging the
 * configurations is done by exchanging the slot -> chain labels. */
int or_pt_pass(int T, const double *beta, const double *E, int32_t *perm,
               uint64_t seed, uint32_t pass, uint32_t sample, uint32_t rep)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int accepted = 0;
    for (int k = 0; k + 1 < T; ++k) {
        int32_t a = perm[k], b = perm[k + 1];
        double delta = (beta[k] - beta[k + 1]) * (E[a] - E[b]);
        uint32_t ctr[4] = {(uint32_t)k, pass, sample, or_ctr3(OR_TAG_PT, 0, rep)};
        uint32_t w[4];
        or_philox4x32_10(key, ctr, w);
        double u = or_u52(w[0], w[1]);
        if (delta >= 0.0 || u < exp(delta)) {
            perm[k] = b;
            perm[k + 1] = a;
            ++accepted;
        }
    }
    return accepted;
}
