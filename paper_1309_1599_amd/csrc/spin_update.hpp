// spin_update.hpp -- device pieces shared by the two sweep mappings: the
// single-spin updates of appendix A.1, the local-field accumulation order,
// buffer-resource access and a wave reduction.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace ptsg {

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

// E[chain] = -(sum of its partials) for chain bx*4 + (wave) of sample
// samples[by]: lane l adds the partials l, l+64, ... in order, then the lanes
// are combined by the fixed shuffle tree of wave_sum (a fixed order:
// bit-reproducible).  Waves past the last chain return at once.
template <class Params>
__device__ __forceinline__ void energy_finalize_block(Params &P, unsigned bx, unsigned by)
{
    const int s = P.samples[by];
    const int j = static_cast<int>(bx * 4 + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (j >= P.C) return;   // wave-uniform
    const int chain = P.chain_base[s] + j;
    const double *e = P.e_part + static_cast<int64_t>(chain) * P.e_stride;
    double acc = 0.0;
    for (int b = lane; b < P.n_blocks; b += 64) acc += e[b];
    acc = wave_sum(acc);
    if (lane == 0) P.E[chain] = -acc;
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

// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each
// with its own L2: workgroup w runs on XCD w % 8.  Tile t = xcd_tile(w, per)
// gives XCD x the contiguous tiles [x*per, (x+1)*per), so that spatially
// neighbouring tiles (whose spins a half-sweep reads as halo) share an L2.
// The grid has 8*per (kXcds*per) workgroups; those mapped beyond the last
// tile exit.

// With `reverse` each XCD takes its range backwards: the colour-1
// half-sweeps do, so that a half-sweep begins where the one before it ended
// (measured: chain lanes at L64x8 1 % faster, site lanes at L32x64 0.3 %;
// the results do not change, since same-colour sites are independent).
__device__ __forceinline__ int xcd_tile(int w, int per, bool reverse = false)
{
    const int i = w / kXcds;
    return (w % kXcds) * per + (reverse ? per - 1 - i : i);
}

// h_a = sum over the six neighbours n (+x, -x, +y, -y, +z, -z) and b of
// A_n[a][b] s_n[b], accumulated in exactly this order (first term a product,
// then chained multiply-adds), so that both mappings produce bit-identical
// spins.  coef(n, a, b) returns A_n[a][b].
template <class Coef>
__device__ __forceinline__ void local_field(const float (&sn)[6][3], Coef coef, float (&h)[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        h[a] = coef(0, a, 0) * sn[0][0];
        h[a] = fmaf(coef(0, a, 1), sn[0][1], h[a]);
        h[a] = fmaf(coef(0, a, 2), sn[0][2], h[a]);
    }
#pragma unroll
    for (int n = 1; n < 6; ++n)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) h[a] = fmaf(coef(n, a, b), sn[n][b], h[a]);
}

}  // namespace ptsg
