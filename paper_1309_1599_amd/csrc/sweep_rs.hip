// sweep_rs.hip -- lattice-resident sweeps for small lattices.
//
// One workgroup owns one chain for a whole step: its spins (12 N bytes,
// 48 KB at L = 16) are loaded into LDS once, all heat-bath and
// overrelaxation sweeps of the step run there with a workgroup barrier
// between half-sweeps (same-colour sites never interact, appendix A.1),
// and the spins are written back once.  Small lattices are otherwise bound
// by launch latency: a half-sweep of one L = 16 chain is 2048 updates.
// Couplings come from the packed six-matrix layout (L2 resident at these
// sizes); when every thread owns at most one site of each colour (N/2 <=
// kRsRegSites, L <= 10) the 108 coefficients of its two sites are loaded
// into registers once per step instead of once per half-sweep.  The field
// order and the update rules are the ones of the other mappings, so the
// spins are bit-identical to theirs.
#include <algorithm>

#include "kernels.hpp"
#include "philox.hpp"
#include "spin_update.hpp"

namespace ptsg {

namespace {

__device__ __forceinline__ void rs_neighbours(int p, int L, int colour, int (&idx)[6], int &site)
{
    const int Lh = L >> 1;
    const int xh = p % Lh;
    const int row = p / Lh;
    const int y = row % L;
    const int z = row / L;
    const int par = (colour + y + z) & 1;
    const int rb = p - xh;
    idx[0] = rb + (par ? (xh + 1 == Lh ? 0 : xh + 1) : xh);
    idx[1] = rb + (par ? xh : (xh == 0 ? Lh - 1 : xh - 1));
    const int dy = Lh, dz = Lh * L;
    idx[2] = p + (y == L - 1 ? -(L - 1) * dy : dy);
    idx[3] = p + (y == 0 ? (L - 1) * dy : -dy);
    idx[4] = p + (z == L - 1 ? -(L - 1) * dz : dz);
    idx[5] = p + (z == 0 ? (L - 1) * dz : -dz);
    site = 2 * xh + par + L * row;
}

// Largest half-lattice whose coefficients stay in registers: one site of
// each colour per thread, 108 floats, in workgroups of at most 512 threads
// (two waves per SIMD leave 256 VGPRs to a lane).
constexpr int kRsRegSites = 512;

template <bool kRegCpl>
__global__ __launch_bounds__(kRegCpl ? kRsRegSites : kRsMaxBlock) void resident_step_kernel(RsParams P)
{
    extern __shared__ float lds[];  // [colour][component][H]
    const int item = blockIdx.x;    // chain of the class: sample P.samples[item / C], chain item % C
    const int s = P.samples[item / P.C];
    const int j = item % P.C;
    const int H = P.H;
    const int chain = P.chain_base[s] + j;
    float *g = P.spins + P.spin_base[s] + static_cast<int64_t>(j) * 6 * H;
    for (int q = threadIdx.x; q < 6 * H; q += blockDim.x) lds[q] = g[q];

    uint32_t ctr3 = 0;
    float beta = 0.0f;
    if (P.n_hb > 0) {
        ctr3 = ctr_word3(0u, static_cast<uint32_t>(P.slot_of[chain]), static_cast<uint32_t>(j / P.T));
        beta = P.beta_of[chain];
    }
    const float *cpl = P.cpl + P.cpl_base[s];
    // kRegCpl: the coefficients of site threadIdx.x of each colour
    float Areg[2][54];
    if constexpr (kRegCpl) {
        const int p = threadIdx.x < H ? threadIdx.x : 0;
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int m = 0; m < 54; ++m) Areg[c][m] = cpl[(static_cast<int64_t>(c) * 54 + m) * H + p];
    }
    const int total = P.n_hb + P.n_or;
    const uint32_t hb0 = P.counters[0];
    double e_acc = 0.0;
    __syncthreads();
    for (int n = 0; n < total; ++n) {
        const int kind = P.energy_only ? kEnergyOnly : (n < P.n_hb ? kHeatbath : kOverrelax);
        const uint32_t hb_sweep = hb0 + static_cast<uint32_t>(n);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const float *oth = lds + (1 - c) * 3 * H;
            float *own = lds + c * 3 * H;
            const float *A = cpl + static_cast<int64_t>(c) * 54 * H;
            const bool last = n == total - 1 && c == 1;
            for (int p = threadIdx.x; p < H; p += blockDim.x) {
                int idx[6], site;
                rs_neighbours(p, P.L, c, idx, site);
                float sn[6][3];
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    sn[q][0] = oth[idx[q]];
                    sn[q][1] = oth[H + idx[q]];
                    sn[q][2] = oth[2 * H + idx[q]];
                }
                float h[3];
                local_field(sn, [&](int q, int a, int b) {
                    if constexpr (kRegCpl) return Areg[c][q * 9 + a * 3 + b];
                    else return A[static_cast<int64_t>(q * 9 + a * 3 + b) * H + p];
                }, h);
                float sx, sy, sz;
                if (kind == kHeatbath) {
                    const uint4 w = philox10(make_uint4(static_cast<uint32_t>(site), hb_sweep,
                                                        static_cast<uint32_t>(s), ctr3),
                                             P.key0, P.key1);
                    heatbath(sx, sy, sz, h[0], h[1], h[2], beta, unit23(w.x), unit23(w.y));
                } else {
                    sx = own[p];
                    sy = own[H + p];
                    sz = own[2 * H + p];
                    if (kind == kOverrelax) overrelax(sx, sy, sz, h[0], h[1], h[2]);
                }
                if (kind != kEnergyOnly) {
                    own[p] = sx;
                    own[H + p] = sy;
                    own[2 * H + p] = sz;
                }
                if (last)
                    e_acc += static_cast<double>(sx) * h[0] + static_cast<double>(sy) * h[1] +
                             static_cast<double>(sz) * h[2];
            }
            __syncthreads();
        }
    }
    if (!P.energy_only)
        for (int q = threadIdx.x; q < 6 * H; q += blockDim.x) g[q] = lds[q];

    // E = -sum over colour-1 sites of s.h, reduced in a fixed order
    __shared__ double e_wave[kRsMaxBlock / 64];
    const double w = wave_sum(e_acc);
    if ((threadIdx.x & 63) == 0) e_wave[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        double e = 0.0;
        for (int q = 0; q < static_cast<int>(blockDim.x >> 6); ++q) e += e_wave[q];
        P.E[chain] = -e;
    }
}

}  // namespace

int rs_block(int L)
{
    const int H = L * L * L / 2;
    return std::min(kRsMaxBlock, (H + 63) / 64 * 64);
}

hipError_t launch_resident_step(const RsParams &p, int n_chains, hipStream_t st, const LaunchTiming &t)
{
    const uint32_t lds = static_cast<uint32_t>(sizeof(float) * 6 * static_cast<size_t>(p.H));
    if (p.H <= kRsRegSites)   // one site of each colour per thread: rs_block(L) >= H
        return launch_kernel(resident_step_kernel<true>, dim3(n_chains), dim3(rs_block(p.L)), lds, st, t, p);
    return launch_kernel(resident_step_kernel<false>, dim3(n_chains), dim3(rs_block(p.L)), lds, st, t, p);
}

}  // namespace ptsg
