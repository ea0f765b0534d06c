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
#include "kernels.hpp"
#include "philox.hpp"

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

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Overrelaxation (appendix A.1): reflect about h, keep s.h; renormalise.
__device__ __forceinline__ void overrelax(float &sx, float &sy, float &sz,
                                          float hx, float hy, float hz)
{
    const float q = hx * hx + hy * hy + hz * hz;
    if (q > 0.0f) {
        const float f = 2.0f * (hx * sx + hy * sy + hz * sz) * rcp(q);
        sx = f * hx - sx;
        sy = f * hy - sy;
        sz = f * hz - sz;
        const float r = rsq(sx * sx + sy * sy + sz * sz);
        sx *= r; sy *= r; sz *= r;
    }
}

// Heat-bath (appendix A.1): draw s from exp(beta s.h) on the sphere.
// c = cos(theta) about n = h/|h| has density ~ exp(X c), X = beta|h|;
// inverting the upper tail of its CDF with a uniform v gives
//   t = 1 - c = -log(1 + v expm1(-2X)) / X    (flat law t = 2v below 2^-60).
// FP32 evaluation: the argument 1 + v expm1(-2X) equals (1-v) + v e^{-2X},
// a sum of two positive terms (1-v is exact), which keeps its relative
// accuracy where it is small; log1p is used where it is not.  The
// complement p = 1 + c = log1p((1-v) expm1(2X)) / X is evaluated on its own
// so that sin(theta) = sqrt(t p) stays accurate near both poles.
// The azimuth 2 pi u2 is measured in the branch-free orthonormal frame of
// Duff et al. (JCGT 6(1), 2017) around n.
__device__ __forceinline__ void heatbath(float &sx, float &sy, float &sz,
                                         float hx, float hy, float hz,
                                         float beta, float v, float u2)
{
    const float hn = sqrtf(hx * hx + hy * hy + hz * hz);
    const float X = beta * hn;
    const float u = 1.0f - v;  // exact: v has 24 significant bits at most
    float nx, ny, nz, t, p;
    if (X < 0x1p-60f) {
        nx = 0.0f; ny = 0.0f; nz = 1.0f;
        t = 2.0f * v;
        p = 2.0f * u;
    } else {
        const float ih = 1.0f / hn;
        nx = hx * ih; ny = hy * ih; nz = hz * ih;
        const float w = v * expm1f(-2.0f * X);
        t = -(w > -0.5f ? log1pf(w) : logf(u + v * expf(-2.0f * X))) / X;
        p = X <= 40.0f ? log1pf(u * expm1f(2.0f * X)) / X : 2.0f - t;
    }
    const float ct = t <= 1.0f ? 1.0f - t : p - 1.0f;
    const float st = sqrtf(fmaxf(t * p, 0.0f));
    float sp, cp;
    sincospif(2.0f * u2, &sp, &cp);
    const float sg = copysignf(1.0f, nz);
    const float a = -1.0f / (sg + nz);
    const float b = nx * ny * a;
    const float b1x = 1.0f + sg * nx * nx * a, b1y = sg * b, b1z = -sg * nx;
    const float b2x = b, b2y = sg + ny * ny * a, b2z = -ny;
    sx = ct * nx + st * (cp * b1x + sp * b2x);
    sy = ct * ny + st * (cp * b1y + sp * b2y);
    sz = ct * nz + st * (cp * b1z + sp * b2z);
    const float r = rsq(sx * sx + sy * sy + sz * sz);
    sx *= r; sy *= r; sz *= r;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Buffer-resource access: the chain's base address and size live in
// SGPRs, each lane supplies a 32-bit byte offset, and the component stride
// goes in the scalar offset, so addressing costs no vector ALU work.
// Out-of-range offsets read as zero and drop stores (the size bound).
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit dwords (CDNA3/CDNA4)

__device__ __forceinline__ Rsrc make_rsrc(const float *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(base), 0, static_cast<int>(bytes),
                                             kRsrcWord3);
}

__device__ __forceinline__ float ld(Rsrc r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

__device__ __forceinline__ void st(Rsrc r, float v, unsigned voff, unsigned soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
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
    // 54 chained multiply-adds
    float h[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        h[a] = A[a * 3] * g.n[0][0];
        h[a] = fmaf(A[a * 3 + 1], g.n[0][1], h[a]);
        h[a] = fmaf(A[a * 3 + 2], g.n[0][2], h[a]);
    }
#pragma unroll
    for (int n = 1; n < 6; ++n)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) h[a] = fmaf(A[n * 9 + a * 3 + b], g.n[n][b], h[a]);
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

template <int KIND, bool ENERGY>
__global__ __launch_bounds__(kSweepBlock) void half_sweep_kernel(SweepParams P)
{
    constexpr bool kOwn = KIND != kHeatbath;  // heat-bath ignores the old spin
    const int s = P.samples[blockIdx.z];
    const int p = blockIdx.x * kSweepBlock + threadIdx.x;
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
    {
        const Rsrc rc = make_rsrc(P.cpl + P.cpl_base[s] + static_cast<int64_t>(c) * 54 * H, 54u * H4);
        const unsigned o = 4u * static_cast<unsigned>(pc);
#pragma unroll
        for (int m = 0; m < 54; ++m) A[m] = ld(rc, o, static_cast<unsigned>(m) * H4);
    }

    const int j0 = blockIdx.y * P.G;
    const int j1 = min(j0 + P.G, P.C);
    const int cb = P.chain_base[s];
    const int64_t stride = 6 * static_cast<int64_t>(H);
    const float *chain0 = P.spins + P.spin_base[s] + static_cast<int64_t>(j0) * stride;
    const unsigned chain_bytes = 6u * H4;
    __shared__ double e_wave[kSweepBlock / 64][kMaxGroup];

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
                                      ctr3, P.hb_sweep, P.key0, P.key1, beta);
        if constexpr (ENERGY) {
            // every bond has exactly one end of colour 1: E = -sum_{colour 1} s.h
            const double w = wave_sum(active ? e : 0.0);
            if ((threadIdx.x & 63) == 0) e_wave[threadIdx.x >> 6][j - j0] = w;
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
            for (int w = 0; w < kSweepBlock / 64; ++w) e += e_wave[w][t];
            P.e_part[static_cast<int64_t>(cb + j0 + t) * P.e_stride + blockIdx.x] = e;
        }
    }
}

// E[chain] = -(sum of its partials), summed in block order.
__global__ void energy_finalize_kernel(EnergyParams P)
{
    const int s = P.samples[blockIdx.y];
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P.C) return;
    const int chain = P.chain_base[s] + j;
    const double *e = P.e_part + static_cast<int64_t>(chain) * P.e_stride;
    double acc = 0.0;
    for (int b = 0; b < P.n_blocks; ++b) acc += e[b];
    P.E[chain] = -acc;
}

// Hot start: z = 1 - 2u1 uniform on [-1,1], azimuth 2 pi u2 (uniform law on
// the sphere), counter (site, 0, sample, tag 2 | start slot j | replica).
__global__ void init_spins_kernel(float *spins, int L, int H, int T, int sample,
                                  uint32_t key0, uint32_t key1)
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
    float *o = spins + static_cast<int64_t>(chain) * 6 * H + colour * 3 * H;
    o[p] = r * cp;
    o[H + p] = r * sp;
    o[2 * H + p] = z;
}

}  // namespace

hipError_t launch_half_sweep(int kind, bool energy, const SweepParams &p, int n_samples,
                             hipStream_t st)
{
    const dim3 grid((p.H + kSweepBlock - 1) / kSweepBlock, (p.C + p.G - 1) / p.G, n_samples);
    const dim3 block(kSweepBlock);
    if (kind == kOverrelax) {
        if (energy) hipLaunchKernelGGL((half_sweep_kernel<kOverrelax, true>), grid, block, 0, st, p);
        else hipLaunchKernelGGL((half_sweep_kernel<kOverrelax, false>), grid, block, 0, st, p);
    } else if (kind == kHeatbath) {
        if (energy) hipLaunchKernelGGL((half_sweep_kernel<kHeatbath, true>), grid, block, 0, st, p);
        else hipLaunchKernelGGL((half_sweep_kernel<kHeatbath, false>), grid, block, 0, st, p);
    } else {
        hipLaunchKernelGGL((half_sweep_kernel<kEnergyOnly, true>), grid, block, 0, st, p);
    }
    return hipGetLastError();
}

hipError_t launch_energy_finalize(const EnergyParams &p, int n_samples, hipStream_t st)
{
    const dim3 grid((p.C + 63) / 64, n_samples);
    hipLaunchKernelGGL(energy_finalize_kernel, grid, dim3(64), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_init_spins(float *spins, int64_t spin_base, int L, int C, int T, int sample,
                             uint32_t key0, uint32_t key1, hipStream_t st)
{
    const int H = L * L * L / 2;
    const dim3 grid((H + 255) / 256, 2, C);
    hipLaunchKernelGGL(init_spins_kernel, grid, dim3(256), 0, st, spins + spin_base, L, H, T,
                       sample, key0, key1);
    return hipGetLastError();
}

}  // namespace ptsg
