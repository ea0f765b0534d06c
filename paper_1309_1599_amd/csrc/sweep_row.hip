// sweep_row.hip -- overrelaxation in the row order, chain-lane layout.
//
// The paper's alternative deterministic order (Sec. III, appendix A.3):
// rows of 8 spins along x, updated one after the other inside a row, and
// rows that share no bond updated together.  Row (b, y, z) holds
// x = 8b .. 8b+7 and belongs to class (b + y + z) mod 2; neighbouring rows
// differ by one in exactly one of b, y, z (b = 0 and b = L/8 - 1 touch
// across the periodic boundary, and differ in parity because the host
// accepts only L = 8 or L a multiple of 16), so a class is a set of
// independent rows and a sweep is class 0, then class 1.
//
// One wave = one row for 64 chains of a sample (lane = chain, as in the
// chain-lane half-sweep): the wave walks x upward, the spin it just
// updated is the -x neighbour of the next site (kept in registers), the
// next site's old spin is its +x neighbour, and the y/z neighbours lie in
// rows of the other class, which do not change during this class.  When
// L = 8 a row is a whole x line: its -x neighbour at x = 0 is the old spin
// at x = 7, and the +x neighbour at x = 7 is the spin updated at x = 0.
// Couplings come from the per-site packed blocks [colour][H][54] of the
// chain-lane mapping; the field and the update are those of the other
// kernels, so only the order differs.
#include "kernels.hpp"
#include "spin_update.hpp"

namespace ptsg {

namespace {

using CFloat = __attribute__((address_space(4))) const float;
typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
using CV16 = __attribute__((address_space(4))) const v16f;
using CV4 = __attribute__((address_space(4))) const v4f;
using CV2 = __attribute__((address_space(4))) const v2f;

constexpr unsigned kRow = 3u * 64u * 4u;  // bytes of one site of one group

__device__ __forceinline__ void load3(float (&v)[3], Rsrc r, unsigned voff, unsigned soff)
{
    v[0] = ld(r, voff + 0u, soff);
    v[1] = ld(r, voff + 256u, soff);
    v[2] = ld(r, voff + 512u, soff);
}

__global__ __launch_bounds__(kClBlock) void cl_row_or_kernel(ClParams P, int cls, int compact)
{
    const int s = P.items[2 * blockIdx.z];
    const int g = P.items[2 * blockIdx.z + 1];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const bool lane_on = g * 64 + lane < P.C;
    const int L = P.L, Lh = L >> 1, B = L >> 3;
    const unsigned H = static_cast<unsigned>(P.H);
    const float *grp = P.spins + P.spin_base[s] + static_cast<int64_t>(g) * 6 * H * 64;
    const Rsrc r = make_rsrc(grp, 2u * H * kRow);
    const unsigned voff = 4u * static_cast<unsigned>(lane);
    const CFloat *M = (const CFloat *)(P.cpl + P.cpl_base[s]);

    // this wave's row of class `cls`
    const int w = xcd_tile(blockIdx.x, P.per) * kClWaves + wave;
    int b, y, z;
    if (compact) {  // B even: B/2 rows of the class on every (y, z)
        const int half = B >> 1;
        const int yz = w / half;
        if (yz >= L * L) return;
        y = yz % L;
        z = yz / L;
        b = 2 * (w - yz * half) + ((cls + y + z) & 1);
    } else {        // B odd: one wave per row, those of the other class leave
        if (w >= B * L * L) return;
        b = w % B;
        const int yz = w / B;
        y = yz % L;
        z = yz / L;
        if (((b + y + z) & 1) != cls) return;
    }
    const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
    const int zp = z + 1 == L ? 0 : z + 1, zm = z == 0 ? L - 1 : z - 1;
    auto site = [&](int x, int yy, int zz) {   // byte offset of a site's 768-byte block
        const unsigned c = static_cast<unsigned>((x + yy + zz) & 1);
        const unsigned p = static_cast<unsigned>((x >> 1) + Lh * (yy + L * zz));
        return (c * H + p) * kRow;
    };
    auto cpl_block = [&](int x) {
        const unsigned c = static_cast<unsigned>((x + y + z) & 1);
        const unsigned p = static_cast<unsigned>((x >> 1) + Lh * (y + L * z));
        return (c * H + p) * 54u;
    };

    const int x0 = 8 * b;
    const int xl = x0 == 0 ? L - 1 : x0 - 1;          // -x neighbour of the first site
    const int xr = x0 + 8 == L ? 0 : x0 + 8;          // +x neighbour of the last site
    // Software pipeline: the loads of site k+1 (its +x, y and z neighbours,
    // none of which is written by site k) are issued before site k is
    // stored, so they are in flight while site k is updated.
    struct Gather {
        float n[6][3];  // n[1] (-x) is filled from registers
    };
    auto gather = [&](Gather &gt, int k) {
        const int x = x0 + k;
        if (k < 7) load3(gt.n[0], r, voff, site(x + 1, y, z));
        else if (B != 1) load3(gt.n[0], r, voff, site(xr, y, z));
        load3(gt.n[2], r, voff, site(x, yp, z));
        load3(gt.n[3], r, voff, site(x, ym, z));
        load3(gt.n[4], r, voff, site(x, y, zp));
        load3(gt.n[5], r, voff, site(x, y, zm));
    };
    float prev[3], cur[3], first[3];
    load3(prev, r, voff, site(xl, y, z));
    load3(cur, r, voff, site(x0, y, z));
    Gather ga, gb;
    gather(ga, 0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        Gather &g0 = (k & 1) ? gb : ga;
        Gather &g1 = (k & 1) ? ga : gb;
        if (k < 7) gather(g1, k + 1);
        const int x = x0 + k;
        if (k == 7 && B == 1) {   // the row is the whole x line: +x of x = 7 is the updated x = 0
            g0.n[0][0] = first[0]; g0.n[0][1] = first[1]; g0.n[0][2] = first[2];
        }
        g0.n[1][0] = prev[0]; g0.n[1][1] = prev[1]; g0.n[1][2] = prev[2];
        const CFloat *A = M + cpl_block(x);
        const v16f a0 = *(CV16 *)(A);
        const v16f a1 = *(CV16 *)(A + 16);
        const v16f a2 = *(CV16 *)(A + 32);
        const v4f a3 = *(CV4 *)(A + 48);
        const v2f a4 = *(CV2 *)(A + 52);
        asm volatile("" ::"s"(a0), "s"(a1), "s"(a2), "s"(a3), "s"(a4));
        float h[3];
        local_field(g0.n, [&](int n, int a, int bb) {
            const int q = n * 9 + a * 3 + bb;
            return q < 16 ? a0[q] : q < 32 ? a1[q - 16] : q < 48 ? a2[q - 32] : q < 52 ? a3[q - 48] : a4[q - 52];
        }, h);
        overrelax(cur[0], cur[1], cur[2], h[0], h[1], h[2]);
        if (lane_on) {
            const unsigned o = site(x, y, z);
            st(r, cur[0], voff + 0u, o);
            st(r, cur[1], voff + 256u, o);
            st(r, cur[2], voff + 512u, o);
        }
        if (k == 0) {
            first[0] = cur[0]; first[1] = cur[1]; first[2] = cur[2];
        }
        prev[0] = cur[0]; prev[1] = cur[1]; prev[2] = cur[2];
        cur[0] = g0.n[0][0]; cur[1] = g0.n[0][1]; cur[2] = g0.n[0][2];
    }
}

}  // namespace

int row_waves(int L)
{
    const int B = L / 8;
    return (B % 2 == 0) ? B / 2 * L * L : B * L * L;
}

hipError_t launch_cl_row_or(const ClParams &p, int cls, int n_items, hipStream_t st, const LaunchTiming &t)
{
    const int B = p.L / 8;
    const int compact = B % 2 == 0;
    const dim3 grid(kXcds * p.per, 1, n_items);
    return launch_kernel(cl_row_or_kernel, grid, dim3(kClBlock), 0, st, t, p, cls, compact);
}

}  // namespace ptsg
