// sweep.hip -- checkerboard half-sweep kernels (heat-bath, overrelaxation),
// fused energy partials, energy finalisation and the hot start.
//
// Mapping: one lane = one site of the active colour; a workgroup owns 256
// consecutive packed sites of one sample and a group of G chains of that
// sample.  The 54 coupling values of the lane's site (six 3x3 matrices, see
// kernels.hpp) are loaded once into registers and reused for every chain of
// the group, so coupling traffic is divided by G; spins stream through
// coalesced component rows.  Same-colour sites share no bond (appendix A.1),
// so all lanes update independently and the result does not depend on the
// schedule.
#include <hip/hip_cooperative_groups.h>

#include "kernels.hpp"
#include "philox.hpp"
#include "spin_update.hpp"

namespace ptsg {

namespace {

struct Nbr {
    int idx[6];  // packed indices in the other colour: +x, -x, +y, -y, +z, -z
    int site;    // canonical site index x + L*(y + L*z)
};

__device__ __forceinline__ Nbr neighbours(int p, int L, int colour)
{
    const int Lh = L >> 1;
    const int xh = p % Lh;
    const int row = p / Lh;         // y + L*z
    const int y = row % L;
    const int z = row / L;
    const int par = (colour + y + z) & 1;   // parity of x
    const int x = 2 * xh + par;
    const int rb = p - xh;
    Nbr n;
    // x +- 1 lands in the other colour at packed x index xh (+1 or -1)
    n.idx[0] = rb + (par ? (xh + 1 == Lh ? 0 : xh + 1) : xh);
    n.idx[1] = rb + (par ? xh : (xh == 0 ? Lh - 1 : xh - 1));
    const int dy = Lh, dz = Lh * L;
    n.idx[2] = p + (y == L - 1 ? -(L - 1) * dy : dy);
    n.idx[3] = p + (y == 0 ? (L - 1) * dy : -dy);
    n.idx[4] = p + (z == L - 1 ? -(L - 1) * dz : dz);
    n.idx[5] = p + (z == 0 ? (L - 1) * dz : -dz);
    n.site = x + L * row;
    return n;
}

// The 21 spin values one lane reads per chain: the three components of
// its own spin (overrelaxation only) and of its six other-colour neighbours.
struct Gather {
    float o[3];
    float n[6][3];
};

// Byte offsets of those values inside one chain's [2][3][H] block; the
// component k adds k*4H (scalar).
struct Offsets {
    unsigned own;    // 4 * (c*3H + p)
    unsigned n[6];   // 4 * ((1-c)*3H + neighbour index)
};

template <bool OWN>
__device__ __forceinline__ void gather(Gather &g, Rsrc r, const Offsets &off, unsigned H4)
{
#pragma unroll
    for (int n = 0; n < 6; ++n) {
        g.n[n][0] = ld(r, off.n[n], 0);
        g.n[n][1] = ld(r, off.n[n], H4);
        g.n[n][2] = ld(r, off.n[n], 2 * H4);
    }
    if constexpr (OWN) {
        g.o[0] = ld(r, off.own, 0);
        g.o[1] = ld(r, off.own, H4);
        g.o[2] = ld(r, off.own, 2 * H4);
    }
}

// h = sum_n A_n s_n, then the update; returns s.h of the new spin (FP64)
// for the energy partial.
template <int KIND>
__device__ __forceinline__ double update(const Gather &g, const float (&A)[54], Rsrc r,
                                         const Offsets &off, unsigned H4, bool active,
                                         uint32_t site, uint32_t sample, uint32_t ctr3,
                                         uint32_t hb_sweep, uint32_t key0, uint32_t key1, float beta)
{
    float h[3];
    local_field(g.n, [&](int n, int a, int b) { return A[n * 9 + a * 3 + b]; }, h);
    float sx, sy, sz;
    if constexpr (KIND == kHeatbath) {
        const uint4 w = philox10(make_uint4(site, hb_sweep, sample, ctr3), key0, key1);
        heatbath(sx, sy, sz, h[0], h[1], h[2], beta, unit23(w.x), unit23(w.y));
    } else {
        sx = g.o[0]; sy = g.o[1]; sz = g.o[2];
        if constexpr (KIND == kOverrelax) overrelax(sx, sy, sz, h[0], h[1], h[2]);
    }
    if (KIND != kEnergyOnly && active) {
        st(r, sx, off.own, 0);
        st(r, sy, off.own, H4);
        st(r, sz, off.own, 2 * H4);
    }
    return static_cast<double>(sx) * h[0] + static_cast<double>(sy) * h[1] +
           static_cast<double>(sz) * h[2];
}

// The six matrices of a site from its bond codes (PT_F_BIMODAL): code bit 0
// gives J = -1, bits 1..6 negative entries of D in the order 00, 11, 22,
// 01, 02, 12; the diagonal is the FP32 sum J + d, so the values are those
// of the matrices the codes were made from, bit for bit.  The family is
// symmetric, so a backward matrix needs no transpose.
__device__ __forceinline__ void decode_bonds(uint32_t lo, uint32_t hi, float D, float (&A)[54])
{
#pragma unroll
    for (int n = 0; n < 6; ++n) {
        const uint32_t code = ((n < 4 ? lo >> (8 * n) : hi >> (8 * (n - 4)))) & 0x7fu;
        const float J = (code & 1u) ? -1.0f : 1.0f;
        float d[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) d[k] = ((code >> (1 + k)) & 1u) ? -D : D;
        float *m = A + 9 * n;
        m[0] = J + d[0];
        m[4] = J + d[1];
        m[8] = J + d[2];
        m[1] = m[3] = d[3];
        m[2] = m[6] = d[4];
        m[5] = m[7] = d[5];
    }
}

using EWave = double[kSweepBlock / 64][kMaxGroup];

// One workgroup's share of a half-sweep: block (bx, by, bz) of the launch
// grid (8*per, ceil(C/G), samples).  `e_wave` is LDS for the energy
// partials (ENERGY only).
template <int KIND, bool ENERGY, bool BM, class Params>
__device__ __forceinline__ void half_sweep_block(Params &P, unsigned bx, unsigned by, unsigned bz, EWave *e_wave)
{
    constexpr bool kOwn = KIND != kHeatbath;  // heat-bath ignores the old spin
    const int s = P.samples[bz];
    const int tile = xcd_tile(bx, P.per, P.colour == 1);   // colour 1 backwards
    if (tile >= P.n_tiles) return;
    const int p = tile * kSweepBlock + threadIdx.x;
    const bool active = p < P.H;
    const int pc = active ? p : 0;
    const int c = P.colour;
    const unsigned H = static_cast<unsigned>(P.H);
    const unsigned H4 = 4u * H;
    const Nbr nb = neighbours(pc, P.L, c);
    Offsets off;
    off.own = 4u * (static_cast<unsigned>(c) * 3u * H + static_cast<unsigned>(pc));
#pragma unroll
    for (int n = 0; n < 6; ++n)
        off.n[n] = 4u * (static_cast<unsigned>(1 - c) * 3u * H + static_cast<unsigned>(nb.idx[n]));

    float A[54];
    if constexpr (BM) {
        const Rsrc rc = make_rsrc(P.cpl + P.cpl_base[s] + static_cast<int64_t>(c) * 2 * H, 2u * H4);
        const unsigned o = 8u * static_cast<unsigned>(pc);
        decode_bonds(__float_as_uint(ld(rc, o, 0)), __float_as_uint(ld(rc, o, 4)), P.bm_D[s], A);
    } else {
        const Rsrc rc = make_rsrc(P.cpl + P.cpl_base[s] + static_cast<int64_t>(c) * 54 * H, 54u * H4);
        const unsigned o = 4u * static_cast<unsigned>(pc);
#pragma unroll
        for (int m = 0; m < 54; ++m) A[m] = ld(rc, o, static_cast<unsigned>(m) * H4);
    }

    const int j0 = by * P.G;
    const int j1 = min(j0 + P.G, P.C);
    const int cb = P.chain_base[s];
    const int64_t stride = 6 * static_cast<int64_t>(H);
    const float *chain0 = P.spins + P.spin_base[s] + static_cast<int64_t>(j0) * stride;
    const unsigned chain_bytes = 6u * H4;

    auto rsrc_of = [&](int j) { return make_rsrc(chain0 + static_cast<int64_t>(j - j0) * stride, chain_bytes); };

    auto process = [&](const Gather &g, int j) {
        uint32_t ctr3 = 0;
        float beta = 0.0f;
        if constexpr (KIND == kHeatbath) {
            const int chain = cb + j;
            ctr3 = ctr_word3(0u, static_cast<uint32_t>(P.slot_of[chain]),
                             static_cast<uint32_t>(j / P.T));
            beta = P.beta_of[chain];
        }
        const double e = update<KIND>(g, A, rsrc_of(j), off, H4, active,
                                      static_cast<uint32_t>(nb.site), static_cast<uint32_t>(s),
                                      ctr3, P.counters[0] + P.hb_offset, P.key0, P.key1, beta);
        if constexpr (ENERGY) {
            // every bond has exactly one end of colour 1: E = -sum_{colour 1} s.h
            const double w = wave_sum(active ? e : 0.0);
            if ((threadIdx.x & 63) == 0) (*e_wave)[threadIdx.x >> 6][j - j0] = w;
        }
    };

    // Software pipeline over the chains: the loads of chain j+1 are in
    // flight while chain j is updated.
    Gather ga, gb;
    gather<kOwn>(ga, rsrc_of(j0), off, H4);
    for (int j = j0; j < j1; j += 2) {
        const bool has_b = j + 1 < j1;
        if (has_b) gather<kOwn>(gb, rsrc_of(j + 1), off, H4);
        process(ga, j);
        if (!has_b) break;
        if (j + 2 < j1) gather<kOwn>(ga, rsrc_of(j + 2), off, H4);
        process(gb, j + 1);
    }

    if constexpr (ENERGY) {
        __syncthreads();
        const int nj = j1 - j0;
        for (int t = threadIdx.x; t < nj; t += kSweepBlock) {
            double e = 0.0;
#pragma unroll
            for (int w = 0; w < kSweepBlock / 64; ++w) e += (*e_wave)[w][t];
            P.e_part[static_cast<int64_t>(cb + j0 + t) * P.e_stride + tile] = e;
        }
    }
}

template <int KIND, bool ENERGY, bool BM>
__global__ __launch_bounds__(kSweepBlock) void half_sweep_kernel(SweepParams P)
{
    if constexpr (ENERGY) {
        __shared__ EWave e_wave;
        half_sweep_block<KIND, ENERGY, BM>(P, blockIdx.x, blockIdx.y, blockIdx.z, &e_wave);
    } else {
        half_sweep_block<KIND, ENERGY, BM>(P, blockIdx.x, blockIdx.y, blockIdx.z, nullptr);
    }
}

// The persistent step in this mapping: the phases of a step's descriptors
// (site-lane half-sweeps and energy finalisations), a grid-wide barrier
// after each; the descriptors and phase tables are read-only for the
// launch, so they are read through the constant address space (scalar
// loads).
using CDesc = __attribute__((address_space(4))) const StepDesc;
using CInt = __attribute__((address_space(4))) const int;

template <bool BM, class Params>
__device__ __forceinline__ void site_dispatch(Params &p, int kind, int energy, unsigned bx, unsigned by,
                                              unsigned bz, EWave *ew)
{
    if (kind == kOverrelax) {
        if (energy) half_sweep_block<kOverrelax, true, BM>(p, bx, by, bz, ew);
        else half_sweep_block<kOverrelax, false, BM>(p, bx, by, bz, ew);
    } else if (kind == kHeatbath) {
        if (energy) half_sweep_block<kHeatbath, true, BM>(p, bx, by, bz, ew);
        else half_sweep_block<kHeatbath, false, BM>(p, bx, by, bz, ew);
    } else {
        half_sweep_block<kEnergyOnly, true, BM>(p, bx, by, bz, ew);
    }
}

__global__ __launch_bounds__(kSweepBlock) void site_step_kernel(PersistParams P)
{
    __shared__ EWave e_wave;
    const CDesc *desc = (const CDesc *)(P.desc);
    const CInt *first = (const CInt *)(P.phase_first);
    const CInt *blocks = (const CInt *)(P.phase_blocks);
    for (int ph = 0; ph < P.n_phases; ++ph) {
        const unsigned n = static_cast<unsigned>(blocks[ph]);
        for (unsigned v = blockIdx.x; v < n; v += gridDim.x) {
            int d = first[ph];
            unsigned off = v;
            while (off >= static_cast<unsigned>(desc[d].n_blocks)) off -= desc[d].n_blocks, ++d;
            const unsigned gx = desc[d].gx, gy = desc[d].gy;
            const unsigned bx = off % gx, r = off / gx, by = r % gy, bz = r / gy;
            if (desc[d].op == kOpFinalize) {
                energy_finalize_block(desc[d].ep, bx, by);
            } else {
                auto &p = desc[d].sp;
                const int kind = desc[d].kind, energy = desc[d].energy;
                if (p.bimodal) site_dispatch<true>(p, kind, energy, bx, by, bz, &e_wave);
                else site_dispatch<false>(p, kind, energy, bx, by, bz, &e_wave);
            }
            __syncthreads();   // e_wave is reused by the next block
        }
        cooperative_groups::this_grid().sync();
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && P.d_hb) P.counters[0] += P.d_hb;
}

// One wave per chain (energy_finalize_block).
__global__ __launch_bounds__(256) void energy_finalize_kernel(EnergyParams P)
{
    energy_finalize_block(P, blockIdx.x, blockIdx.y);
}

// Hot start: z = 1 - 2u1 uniform on [-1,1], azimuth 2 pi u2 (uniform law on
// the sphere), counter (site, 0, sample, tag 2 | start slot j | replica).
__global__ void init_spins_kernel(float *spins, int64_t base, int lanes, int L, int H, int T,
                                  int sample, uint32_t key0, uint32_t key1)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= H) return;
    const int colour = blockIdx.y;
    const int chain = blockIdx.z;  // rep*T + j
    const Nbr nb = neighbours(p, L, colour);
    const uint4 w = philox10(make_uint4(static_cast<uint32_t>(nb.site), 0u,
                                        static_cast<uint32_t>(sample),
                                        ctr_word3(2u, static_cast<uint32_t>(chain % T),
                                                  static_cast<uint32_t>(chain / T))),
                             key0, key1);
    const float z = 1.0f - 2.0f * unit23(w.x);
    float sp, cp;
    sincospif(2.0f * unit23(w.y), &sp, &cp);
    const float r = sqrtf(fmaxf(1.0f - z * z, 0.0f));
    spins[spin_index(base, lanes, H, chain, colour, 0, p)] = r * cp;
    spins[spin_index(base, lanes, H, chain, colour, 1, p)] = r * sp;
    spins[spin_index(base, lanes, H, chain, colour, 2, p)] = z;
}

// Copy one chain between the device layout and canonical [N][3] order.
__global__ void chain_io_kernel(float *spins, int64_t base, int lanes, int L, int j, float *canon,
                                int to_canon)
{
    const int N = L * L * L;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int x = i % L, y = (i / L) % L, z = i / (L * L);
    const int c = (x + y + z) & 1;
    const int p = (x >> 1) + (L >> 1) * (y + L * z);
    for (int k = 0; k < 3; ++k) {
        const int64_t q = spin_index(base, lanes, N / 2, j, c, k, p);
        if (to_canon) canon[3 * i + k] = spins[q];
        else spins[q] = canon[3 * i + k];
    }
}

__global__ void advance_counters_kernel(uint32_t *counters, uint32_t d_hb, uint32_t d_pt)
{
    if (threadIdx.x == 0) {
        counters[0] += d_hb;
        counters[1] += d_pt;
    }
}

}  // namespace

hipError_t launch_advance_counters(uint32_t *counters, uint32_t d_hb, uint32_t d_pt, hipStream_t st)
{
    hipLaunchKernelGGL(advance_counters_kernel, dim3(1), dim3(64), 0, st, counters, d_hb, d_pt);
    return hipGetLastError();
}

hipError_t launch_chain_io(float *spins, int64_t base, int lanes, int L, int j, float *canon,
                           bool to_canon, hipStream_t st)
{
    const int N = L * L * L;
    hipLaunchKernelGGL(chain_io_kernel, dim3((N + 255) / 256), dim3(256), 0, st, spins, base, lanes,
                       L, j, canon, to_canon ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_half_sweep(int kind, bool energy, const SweepParams &p, int n_samples,
                             hipStream_t st,
                             const LaunchTiming &t)
{
    const dim3 grid(kXcds * p.per, (p.C + p.G - 1) / p.G, n_samples);
    const dim3 block(kSweepBlock);
    auto go = [&](auto kernel) { return launch_kernel(kernel, grid, block, 0, st, t, p); };
    if (p.bimodal) {
        if (kind == kOverrelax)
            return energy ? go(half_sweep_kernel<kOverrelax, true, true>) : go(half_sweep_kernel<kOverrelax, false, true>);
        if (kind == kHeatbath)
            return energy ? go(half_sweep_kernel<kHeatbath, true, true>) : go(half_sweep_kernel<kHeatbath, false, true>);
        return go(half_sweep_kernel<kEnergyOnly, true, true>);
    }
    if (kind == kOverrelax)
        return energy ? go(half_sweep_kernel<kOverrelax, true, false>) : go(half_sweep_kernel<kOverrelax, false, false>);
    if (kind == kHeatbath)
        return energy ? go(half_sweep_kernel<kHeatbath, true, false>) : go(half_sweep_kernel<kHeatbath, false, false>);
    return go(half_sweep_kernel<kEnergyOnly, true, false>);
}

int site_step_blocks_per_cu()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, site_step_kernel, kSweepBlock, 0) != hipSuccess) return 0;
    return n;
}

hipError_t launch_site_step(const PersistParams &p, int grid, hipStream_t st)
{
    void *args[] = {const_cast<PersistParams *>(&p)};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(site_step_kernel), dim3(grid),
                                      dim3(kSweepBlock), args, 0, st);
}

hipError_t launch_energy_finalize(const EnergyParams &p, int n_samples, hipStream_t st)
{
    const dim3 grid((p.C + 3) / 4, n_samples);
    hipLaunchKernelGGL(energy_finalize_kernel, grid, dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_init_spins(float *spins, int64_t spin_base, int lanes, int L, int C, int T,
                             int sample, uint32_t key0, uint32_t key1, hipStream_t st)
{
    const int H = L * L * L / 2;
    const dim3 grid((H + 255) / 256, 2, C);
    hipLaunchKernelGGL(init_spins_kernel, grid, dim3(256), 0, st, spins, spin_base, lanes, L, H, T,
                       sample, key0, key1);
    return hipGetLastError();
}

}  // namespace ptsg
