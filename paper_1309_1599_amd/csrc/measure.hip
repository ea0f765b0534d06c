// measure.hip -- overlap-tensor, chiral-overlap and Schwinger-Dyson sums
// (Sec. II.B, appendix A.4) in FP64.
//
// Stage 1: one workgroup per (record, z plane) sums, over the plane's sites,
// the products f(x) and f(x) exp(i k x_d) for k along x and y (the twiddle
// of k along z is constant on a plane).  FP32 x FP32 products are exact in
// FP64.  Lane sums are reduced by wave shuffles and then across the four
// waves in a fixed order, so results are bit-reproducible.  (The chirality
// and Schwinger-Dyson sums of 3 or 4 replicas take one workgroup per
// (temperature slot, z plane) for all the slot's records, with the same
// per-record arithmetic.)
// Stage 2: one wave per record, lane q adding plane quantity q over the
// planes in order, applies the z twiddles and the 1/N normalisation, and
// writes the record.
#include "../../include/ptsg.h"
#include "kernels.hpp"

namespace ptsg {

namespace {

// Plane-quantity slots.
constexpr int kS0 = 0, kSxR = 9, kSxI = 18, kSyR = 27, kSyI = 36;       // overlap, 9 each
constexpr int kK0 = 45, kKxR = 48, kKxI = 51, kKyR = 54, kKyI = 57;     // chiral, 3 each
constexpr int kSD = 60;                                                  // sd1a sd2a sd1b sd2b

// One chain of a record: generic access to its spins in either layout.
struct Chain {
    const float *spins;
    int64_t base;
    int lanes, j, L, Lh, H;
    __device__ __forceinline__ int packed(int x, int y, int z) const
    {
        return (x >> 1) + Lh * (y + L * z);
    }
    __device__ __forceinline__ void get(int x, int y, int z, double v[3]) const
    {
        const int c = (x + y + z) & 1;
        const int p = packed(x, y, z);
#pragma unroll
        for (int k = 0; k < 3; ++k) v[k] = spins[spin_index(base, lanes, H, j, c, k, p)];
    }
};

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <int NQ>
__device__ __forceinline__ void block_store(double (&acc)[NQ], double *dst)
{
    __shared__ double red[kMeasBlock / 64][NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double v = wave_sum(acc[q]);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < NQ; q += kMeasBlock) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kMeasBlock / 64; ++w) v += red[w][q];
        dst[q] = v;
    }
}

struct RecordChains {
    Chain a, b;
    int s, L;
    const double *cw, *sw;
};

__device__ __forceinline__ RecordChains record_chains(const MeasParams &P, int rec)
{
    const int *rd = P.rec + 4 * rec;
    const int s = rd[0], k = rd[1], ra = rd[2], rb = rd[3];
    const int L = P.L[s], T = P.n_temps[s];
    const int H = L * L * L / 2;
    const int *perm = P.perm + P.perm_base[s];
    const int ja = ra * T + perm[ra * T + k];
    const int jb = rb * T + perm[rb * T + k];
    RecordChains rc;
    const bool staged = s == P.stage_sample;
    const float *src = staged ? P.stage : P.spins;
    const int64_t base = staged ? 0 : P.spin_base[s];
    const int lanes = staged ? 1 : P.lanes[s];
    rc.a = Chain{src, base, lanes, ja, L, L / 2, H};
    rc.b = Chain{src, base, lanes, jb, L, L / 2, H};
    rc.s = s;
    rc.L = L;
    rc.cw = P.twid + P.twid_base[s];
    rc.sw = rc.cw + L;
    return rc;
}

__global__ __launch_bounds__(kMeasBlock) void overlap_plane_kernel(MeasParams P)
{
    const int rec = P.rec0 + blockIdx.x, z = blockIdx.y;
    const RecordChains rc = record_chains(P, rec);
    const int L = rc.L;
    if (z >= L) return;
    double acc[45];
#pragma unroll
    for (int q = 0; q < 45; ++q) acc[q] = 0.0;
    for (int idx = threadIdx.x; idx < L * L; idx += kMeasBlock) {
        const int x = idx % L, y = idx / L;
        double va[3], vb[3];
        rc.a.get(x, y, z, va);
        rc.b.get(x, y, z, vb);
        const double cx = rc.cw[x], sx = rc.sw[x], cy = rc.cw[y], sy = rc.sw[y];
#pragma unroll
        for (int al = 0; al < 3; ++al) {
#pragma unroll
            for (int be = 0; be < 3; ++be) {
                const int n = al * 3 + be;
                const double q = va[al] * vb[be];
                acc[kS0 + n] += q;
                acc[kSxR + n] += q * cx;
                acc[kSxI + n] += q * sx;
                acc[kSyR + n] += q * cy;
                acc[kSyI + n] += q * sy;
            }
        }
    }
    block_store<45>(acc, P.part + (static_cast<int64_t>(rec - P.part_rec0) * P.Lmax + z) * kPlaneQ);
}

// u is the chain's spin at (x, y, z), read once for the three directions.
__device__ __forceinline__ double chirality(const Chain &c, const double (&u)[3], int x, int y, int z, int mu)
{
    const int L = c.L;
    int p[3] = {x, y, z}, m[3] = {x, y, z};
    p[mu] = (p[mu] + 1 == L) ? 0 : p[mu] + 1;
    m[mu] = (m[mu] == 0) ? L - 1 : m[mu] - 1;
    double v[3], w[3];
    c.get(p[0], p[1], p[2], v);
    c.get(m[0], m[1], m[2], w);
    // zeta = s_{x+e} . (s_x cross s_{x-e})
    return v[0] * (u[1] * w[2] - u[2] * w[1]) + v[1] * (u[2] * w[0] - u[0] * w[2]) +
           v[2] * (u[0] * w[1] - u[1] * w[0]);
}

// FP64 local field from the site-major couplings:
// h = sum_mu M_{mu,x} s_{x+e_mu} + M_{mu,x-e_mu}^T s_{x-e_mu}.
__device__ __forceinline__ void field64(const Chain &c, const float *cpls, int x, int y, int z,
                                        double h[3])
{
    const int L = c.L;
    const int xp = x + 1 == L ? 0 : x + 1, xm = x == 0 ? L - 1 : x - 1;
    const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
    const int zp = z + 1 == L ? 0 : z + 1, zm = z == 0 ? L - 1 : z - 1;
    const int pc[3][3] = {{xp, y, z}, {x, yp, z}, {x, y, zp}};
    const int mc[3][3] = {{xm, y, z}, {x, ym, z}, {x, y, zm}};
    const int64_t i = x + static_cast<int64_t>(L) * (y + L * z);
    h[0] = h[1] = h[2] = 0.0;
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
        double vp[3], vm[3];
        c.get(pc[mu][0], pc[mu][1], pc[mu][2], vp);
        c.get(mc[mu][0], mc[mu][1], mc[mu][2], vm);
        const int64_t im = mc[mu][0] + static_cast<int64_t>(L) * (mc[mu][1] + L * mc[mu][2]);
        const float *F = cpls + i * 27 + mu * 9;
        const float *B = cpls + im * 27 + mu * 9;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                h[a] += static_cast<double>(F[a * 3 + b]) * vp[b] +
                        static_cast<double>(B[b * 3 + a]) * vm[b];
    }
}

// Chiral-glass plane sums (slots kK0 .. kSD-1).
__global__ __launch_bounds__(kMeasBlock) void chiral_plane_kernel(MeasParams P)
{
    const int rec = P.rec0 + blockIdx.x, z = blockIdx.y;
    const RecordChains rc = record_chains(P, rec);
    const int L = rc.L;
    if (z >= L) return;
    double acc[15];
#pragma unroll
    for (int q = 0; q < 15; ++q) acc[q] = 0.0;
    for (int idx = threadIdx.x; idx < L * L; idx += kMeasBlock) {
        const int x = idx % L, y = idx / L;
        const double cx = rc.cw[x], sx = rc.sw[x], cy = rc.cw[y], sy = rc.sw[y];
        double ua[3], ub[3];
        rc.a.get(x, y, z, ua);
        rc.b.get(x, y, z, ub);
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
            const double kap = chirality(rc.a, ua, x, y, z, mu) * chirality(rc.b, ub, x, y, z, mu);
            acc[mu] += kap;
            acc[3 + mu] += kap * cx;
            acc[6 + mu] += kap * sx;
            acc[9 + mu] += kap * cy;
            acc[12 + mu] += kap * sy;
        }
    }
    block_store<15>(acc, P.part + (static_cast<int64_t>(rec - P.part_rec0) * P.Lmax + z) * kPlaneQ + kK0);
}

// The chirality sums of all R(R-1)/2 records of one temperature slot (one
// sample, replicas a < b in record order) in one workgroup: each chain's
// chirality at a site is computed once for the slot instead of once per
// record it belongs to.  Every record's sums are formed as in
// chiral_plane_kernel: the same products, in the same order over the sites,
// and the same reduction.
template <int R>
__global__ __launch_bounds__(kMeasBlock) void chiral_slot_kernel(MeasParams P)
{
    constexpr int NP = R * (R - 1) / 2, NQ = 15 * NP;
    const int rec_first = P.rec0 + static_cast<int>(blockIdx.x) * NP, z = blockIdx.y;
    const int *rd = P.rec + 4 * rec_first;
    const int s = rd[0], k = rd[1];
    const int L = P.L[s], T = P.n_temps[s];
    if (z >= L) return;
    const int H = L * L * L / 2;
    const int *perm = P.perm + P.perm_base[s];
    const bool staged = s == P.stage_sample;
    const float *src = staged ? P.stage : P.spins;
    const int64_t base = staged ? 0 : P.spin_base[s];
    const int lanes = staged ? 1 : P.lanes[s];
    Chain ch[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ch[r] = Chain{src, base, lanes, r * T + perm[r * T + k], L, L / 2, H};
    const double *cw = P.twid + P.twid_base[s], *sw = cw + L;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    for (int idx = threadIdx.x; idx < L * L; idx += kMeasBlock) {
        const int x = idx % L, y = idx / L;
        const double cx = cw[x], sx = sw[x], cy = cw[y], sy = sw[y];
        double zeta[R][3];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            double u[3];
            ch[r].get(x, y, z, u);
#pragma unroll
            for (int mu = 0; mu < 3; ++mu) zeta[r][mu] = chirality(ch[r], u, x, y, z, mu);
        }
        int p = 0;
#pragma unroll
        for (int a = 0; a < R; ++a)
#pragma unroll
            for (int b = a + 1; b < R; ++b, ++p)
#pragma unroll
                for (int mu = 0; mu < 3; ++mu) {
                    const double kap = zeta[a][mu] * zeta[b][mu];
                    double *q = acc + 15 * p;
                    q[mu] += kap;
                    q[3 + mu] += kap * cx;
                    q[6 + mu] += kap * sx;
                    q[9 + mu] += kap * cy;
                    q[12 + mu] += kap * sy;
                }
    }
    __shared__ double red[kMeasBlock / 64][NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double v = wave_sum(acc[q]);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < NQ; q += kMeasBlock) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kMeasBlock / 64; ++w) v += red[w][q];
        const int rec = rec_first + q / 15;
        P.part[(static_cast<int64_t>(rec - P.part_rec0) * P.Lmax + z) * kPlaneQ + kK0 + q % 15] = v;
    }
}

// Schwinger-Dyson plane sums (slots kSD .. kSD+3): s.h and |h|^2 - (s.h)^2
// of both chains with the FP64 field.
__global__ __launch_bounds__(kMeasBlock) void sd_plane_kernel(MeasParams P)
{
    const int rec = P.rec0 + blockIdx.x, z = blockIdx.y;
    const RecordChains rc = record_chains(P, rec);
    const int L = rc.L;
    if (z >= L) return;
    const float *cpl = P.cpls + P.cpls_base[rc.s];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int idx = threadIdx.x; idx < L * L; idx += kMeasBlock) {
        const int x = idx % L, y = idx / L;
        double h[3], v[3];
        field64(rc.a, cpl, x, y, z, h);
        rc.a.get(x, y, z, v);
        double sh = v[0] * h[0] + v[1] * h[1] + v[2] * h[2];
        acc[0] += sh;
        acc[1] += h[0] * h[0] + h[1] * h[1] + h[2] * h[2] - sh * sh;
        field64(rc.b, cpl, x, y, z, h);
        rc.b.get(x, y, z, v);
        sh = v[0] * h[0] + v[1] * h[1] + v[2] * h[2];
        acc[2] += sh;
        acc[3] += h[0] * h[0] + h[1] * h[1] + h[2] * h[2] - sh * sh;
    }
    block_store<4>(acc, P.part + (static_cast<int64_t>(rec - P.part_rec0) * P.Lmax + z) * kPlaneQ + kSD);
}

// The Schwinger-Dyson sums of the R chains of one temperature slot, each
// computed once and written into every record of the slot that holds the
// chain (as chain a or b); per chain the sums are formed as in
// sd_plane_kernel: the same terms, in the same order over the sites, and the
// same reduction.
template <int R>
__global__ __launch_bounds__(kMeasBlock) void sd_slot_kernel(MeasParams P)
{
    constexpr int NP = R * (R - 1) / 2, NQ = 2 * R;
    const int rec_first = P.rec0 + static_cast<int>(blockIdx.x) * NP, z = blockIdx.y;
    const int *rd = P.rec + 4 * rec_first;
    const int s = rd[0], k = rd[1];
    const int L = P.L[s], T = P.n_temps[s];
    if (z >= L) return;
    const int H = L * L * L / 2;
    const int *perm = P.perm + P.perm_base[s];
    const bool staged = s == P.stage_sample;
    const float *src = staged ? P.stage : P.spins;
    const int64_t base = staged ? 0 : P.spin_base[s];
    const int lanes = staged ? 1 : P.lanes[s];
    const float *cpl = P.cpls + P.cpls_base[s];
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    for (int idx = threadIdx.x; idx < L * L; idx += kMeasBlock) {
        const int x = idx % L, y = idx / L;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const Chain c{src, base, lanes, r * T + perm[r * T + k], L, L / 2, H};
            double h[3], v[3];
            field64(c, cpl, x, y, z, h);
            c.get(x, y, z, v);
            const double sh = v[0] * h[0] + v[1] * h[1] + v[2] * h[2];
            acc[2 * r] += sh;
            acc[2 * r + 1] += h[0] * h[0] + h[1] * h[1] + h[2] * h[2] - sh * sh;
        }
    }
    __shared__ double red[kMeasBlock / 64][NQ];
    __shared__ double chain_sum[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double v = wave_sum(acc[q]);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < NQ) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kMeasBlock / 64; ++w) v += red[w][threadIdx.x];
        chain_sum[threadIdx.x] = v;
    }
    __syncthreads();
    // record p = (a, b) gets sd1_a sd2_a sd1_b sd2_b
    if (threadIdx.x < 4 * NP) {
        const int p = threadIdx.x / 4, f = threadIdx.x % 4;
        int a = 0, b = 1, i = 0;
        for (int aa = 0; aa < R; ++aa)
            for (int bb = aa + 1; bb < R; ++bb, ++i)
                if (i == p) {
                    a = aa;
                    b = bb;
                }
        const int r = f < 2 ? a : b;
        P.part[(static_cast<int64_t>(rec_first + p - P.part_rec0) * P.Lmax + z) * kPlaneQ + kSD + f] =
            chain_sum[2 * r + (f & 1)];
    }
}

// One wave per record: lane q adds plane quantity q over z in order (and,
// for Q(0) and kappa(0), its z Fourier pair with the twiddles), then writes
// the record field(s) that quantity becomes; lane 0 writes the header.
__global__ __launch_bounds__(kPlaneQ) void finalize_kernel(MeasParams P)
{
    static_assert(kPlaneQ == 64, "one lane per plane quantity");
    const int rec = P.rec0 + static_cast<int>(blockIdx.x);
    if (rec >= P.n_records) return;
    const int q = static_cast<int>(threadIdx.x);
    const int *rd = P.rec + 4 * rec;
    const int s = rd[0], k = rd[1], ra = rd[2], rb = rd[3];
    const int L = P.L[s], T = P.n_temps[s];
    const double invN = 1.0 / (static_cast<double>(L) * L * L);
    const double *cw = P.twid + P.twid_base[s], *sw = cw + L;
    const double *part = P.part + static_cast<int64_t>(rec - P.part_rec0) * P.Lmax * kPlaneQ;
    pt_meas *out = P.cursor ? static_cast<pt_meas *>(P.cursor->base) + P.cursor->k * P.cursor->stride
                            : static_cast<pt_meas *>(P.out);
    pt_meas &m = out[rec];
    if (q == 0) {
        m.sample = s;
        m.tslot = k;
        m.rep_a = ra;
        m.rep_b = rb;
        m.beta = P.betas[P.beta_base[s] + k];
        const int *perm = P.perm + P.perm_base[s];
        m.E_a = P.E[P.chain_base[s] + ra * T + perm[ra * T + k]];
        m.E_b = P.E[P.chain_base[s] + rb * T + perm[rb * T + k]];
    }
    double sum = 0.0, re = 0.0, im = 0.0;
    for (int z = 0; z < L; ++z) {
        const double v = part[static_cast<int64_t>(z) * kPlaneQ + q];
        sum += v;
        re += v * cw[z];
        im += v * sw[z];
    }
    const bool ovl = P.what & PT_M_OVERLAP, chi = P.what & PT_M_CHIRAL, sd = P.what & PT_M_SD;
    if (q < kK0) {
        const int blk = q / 9, n = q - 9 * blk;      // Q(0), Q(kx) re, im, Q(ky) re, im
        const double v = ovl ? sum * invN : 0.0;
        if (blk == 0) {
            m.q0[n] = v;
            m.qk_re[2][n] = ovl ? re * invN : 0.0;   // k along z from the z planes
            m.qk_im[2][n] = ovl ? im * invN : 0.0;
        } else {
            double *dst = (blk & 1) ? m.qk_re[(blk - 1) / 2] : m.qk_im[(blk - 1) / 2];
            dst[n] = v;
        }
    } else if (q < kSD) {
        const int blk = (q - kK0) / 3, n = q - kK0 - 3 * blk;   // kappa(0), kappa(kx) re, im, ...
        const double v = chi ? sum * invN : 0.0;
        if (blk == 0) {
            m.cg0[n] = v;
            m.cgk_re[2][n] = chi ? re * invN : 0.0;
            m.cgk_im[2][n] = chi ? im * invN : 0.0;
        } else {
            double *dst = (blk & 1) ? m.cgk_re[(blk - 1) / 2] : m.cgk_im[(blk - 1) / 2];
            dst[n] = v;
        }
    } else {
        double *dst = q == kSD ? &m.sd1_a : q == kSD + 1 ? &m.sd2_a : q == kSD + 2 ? &m.sd1_b : &m.sd2_b;
        *dst = sd ? sum : 0.0;
    }
}

}  // namespace

namespace {

// 64 sites x 64 chains x 3 components per workgroup: rows of 64 chains are
// read coalesced, transposed in LDS (row pitch 65: no bank conflicts either
// way) and written as rows of 64 sites per (chain, component).
__global__ __launch_bounds__(256) void cl_to_sl_kernel(const float *spins, int64_t base, int H, int C,
                                                       float *stage)
{
    __shared__ float tile[3][64][65];
    const int p0 = blockIdx.x * 64, c = blockIdx.y, g = blockIdx.z;
    const int lane = threadIdx.x & 63;
    const float *src = spins + base + (static_cast<int64_t>(g) * 2 + c) * H * 192;
    // 48 rows per wave, 16 loads in flight at a time
#pragma unroll 16
    for (int row = threadIdx.x >> 6; row < 192; row += 4) {
        const int q = row / 3, k = row - 3 * q;
        if (p0 + q < H) tile[k][lane][q] = src[(static_cast<int64_t>(p0 + q) * 3 + k) * 64 + lane];
    }
    __syncthreads();
#pragma unroll 16
    for (int row = threadIdx.x >> 6; row < 192; row += 4) {
        const int l = row / 3, k = row - 3 * l;
        const int j = g * 64 + l;
        if (j < C && p0 + lane < H)
            stage[((static_cast<int64_t>(j) * 2 + c) * 3 + k) * H + p0 + lane] = tile[k][l][lane];
    }
}

__global__ void set_cursor_kernel(RecordCursor *cursor, void *base, uint64_t stride)
{
    if (threadIdx.x == 0) {
        cursor->base = base;
        cursor->k = 0;
        cursor->stride = stride;
    }
}

__global__ void advance_cursor_kernel(RecordCursor *cursor)
{
    if (threadIdx.x == 0) cursor->k += 1;
}

}  // namespace

hipError_t launch_set_cursor(RecordCursor *cursor, void *base, uint64_t stride, hipStream_t st)
{
    hipLaunchKernelGGL(set_cursor_kernel, dim3(1), dim3(64), 0, st, cursor, base, stride);
    return hipGetLastError();
}

hipError_t launch_advance_cursor(RecordCursor *cursor, hipStream_t st)
{
    hipLaunchKernelGGL(advance_cursor_kernel, dim3(1), dim3(64), 0, st, cursor);
    return hipGetLastError();
}

hipError_t launch_measure_records(const MeasParams &p, int n, int L, int R, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const dim3 grid(n, L);
    if (p.what & PT_M_OVERLAP)
        hipLaunchKernelGGL(overlap_plane_kernel, grid, dim3(kMeasBlock), 0, st, p);
    if (p.what & PT_M_CHIRAL) {
        // whole slots (R = 3 or 4 and a range of whole slots): one workgroup per
        // slot and plane; otherwise one per record and plane (same arithmetic)
        const int np = R * (R - 1) / 2;
        if ((R == 3 || R == 4) && n % np == 0) {
            const dim3 g(n / np, L);
            if (R == 3) hipLaunchKernelGGL(chiral_slot_kernel<3>, g, dim3(kMeasBlock), 0, st, p);
            else hipLaunchKernelGGL(chiral_slot_kernel<4>, g, dim3(kMeasBlock), 0, st, p);
        } else {
            hipLaunchKernelGGL(chiral_plane_kernel, grid, dim3(kMeasBlock), 0, st, p);
        }
    }
    if (p.what & PT_M_SD) {
        const int np = R * (R - 1) / 2;
        if ((R == 3 || R == 4) && n % np == 0) {
            const dim3 g(n / np, L);
            if (R == 3) hipLaunchKernelGGL(sd_slot_kernel<3>, g, dim3(kMeasBlock), 0, st, p);
            else hipLaunchKernelGGL(sd_slot_kernel<4>, g, dim3(kMeasBlock), 0, st, p);
        } else {
            hipLaunchKernelGGL(sd_plane_kernel, grid, dim3(kMeasBlock), 0, st, p);
        }
    }
    return hipGetLastError();
}

hipError_t launch_measure_finalize(const MeasParams &p, hipStream_t st)
{
    const int n = p.n_records - p.rec0;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3(n), dim3(kPlaneQ), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_cl_to_sl(const float *spins, int64_t base, int H, int C, float *stage, hipStream_t st)
{
    const dim3 grid((H + 63) / 64, 2, (C + 63) / 64);
    hipLaunchKernelGGL(cl_to_sl_kernel, grid, dim3(256), 0, st, spins, base, H, C, stage);
    return hipGetLastError();
}

}  // namespace ptsg
