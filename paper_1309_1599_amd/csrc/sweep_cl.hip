// sweep_cl.hip -- checkerboard half-sweeps in the chain-lane mapping.
//
// One wave = 64 chains of one sample at the same site: lane l owns chain
// 64*g + l of chain group g.  All lanes read the same site, so
//  * the site's six matrices are wave-uniform.  The overrelaxation and
//    energy half-sweeps read them from the canonical 27-float blocks (the
//    site's own block and the backward neighbours' bond matrices): one
//    16-byte load per lane leaves a copy of the 54 coefficients in each
//    16-lane row, and each multiply-add takes its coefficient by a DPP row
//    broadcast.  The heat-bath half-sweeps read the 216-byte block of the
//    per-site packed couplings [colour][H][54] with five scalar loads into
//    SGPRs (one memory round trip per site, no vector registers);
//  * every spin access is a 256-byte row: the layout of a group is
//    [colour][H][component][64 lanes], each lane uses the same vector offset
//    (4*lane), the site enters through the scalar offset and the component
//    through the instruction's immediate offset (0, 256, 512), so
//    addressing costs no vector ALU work.
// Each wave walks a segment of one packed row of the active colour (fixed
// y, z), so all its offsets advance by one site per step; the loads of the
// next site are in flight while the current one is updated.  Rows are
// visited in strips of `strip` y-rows, z-major within a strip, so that the
// y- and z-neighbour rows a wave reads were fetched into its XCD's L2 by
// the waves of the rows just before it.
// The host runs all sweeps of one chain group back to back so that the
// group stays in the 256 MB Infinity Cache between half-sweeps.  At L = 64
// a group is 201 MB of spins and its sample's canonical couplings 28 MB, so
// a whole sweep touches 229 MB, which fits (with the packed blocks, 216
// bytes a site, it would be 258 MB: slightly more than the cache).  Each
// XCD walks its tiles backwards in the colour-1 half-sweeps, so that a
// half-sweep starts where the previous one ended.
#include <hip/hip_cooperative_groups.h>

#include "kernels.hpp"
#include "philox.hpp"
#include "spin_update.hpp"

namespace ptsg {

namespace {

using CFloat = __attribute__((address_space(4))) const float;

constexpr unsigned kRow = 3u * 64u * 4u;  // bytes of one site of one group: 3 components x 64 lanes

typedef float v4f __attribute__((ext_vector_type(4)));

struct ClGather {
    float o[3];
    float n[6][3];
    v4f cv;   // canonical couplings: four coefficients of the site per lane (see canon_lane)
};

// Canonical-block couplings: in each 16-lane row, lanes 0-6 hold floats
// 0..27 of the site's own block (its three forward matrices), lanes 7-9,
// 10-12 and 13-15 floats of the x-, y- and z-bond matrix of the backward
// neighbour along x, y and z (four floats a lane, 9 of 12 used).  Lane k
// reads 16 bytes at float 27*site + off from the site of kind `kind`
// (0 own, 1..3 backward along x, y, z).
struct CanonLane {
    int kind;
    unsigned off;
};

__device__ __forceinline__ CanonLane canon_lane(int lane)
{
    const int k = lane & 15;
    if (k < 7) return CanonLane{0, 4u * static_cast<unsigned>(k)};
    const int mu = (k - 7) / 3, m = (k - 7) - 3 * mu;
    return CanonLane{1 + mu, static_cast<unsigned>(9 * mu + 4 * m)};
}

// The local field of spin_update.hpp's local_field, term for term in the
// same order per component, each coefficient taken by a DPP row broadcast
// inside the multiply-add from the lane that holds it (the layout above:
// A_{2mu}[a][b] is float 9mu + 3a + b of the own block, A_{2mu+1}[a][b]
// float 3b + a of the mu-bond matrix of the backward neighbour).  The three
// components are interleaved, so every instruction is at least two after
// the one that wrote the accumulator it reads (the DPP read-after-write
// distance); the leading s_nop covers VALU writes of the inputs before it.
__device__ __forceinline__ void local_field_rows(const float (&sn)[6][3], const v4f &cv, float (&h)[3])
{
    asm("s_nop 4\n"
        "v_mul_f32_dpp %0, %3, %7 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
        "v_mul_f32_dpp %1, %6, %7 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
        "v_mul_f32_dpp %2, %5, %7 row_newbcast:1 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %4, %8 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %3, %8 row_newbcast:1 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %6, %8 row_newbcast:1 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %5, %9 row_newbcast:0 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %4, %9 row_newbcast:1 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %3, %9 row_newbcast:2 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %3, %10 row_newbcast:7 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %4, %10 row_newbcast:7 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %5, %10 row_newbcast:7 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %6, %11 row_newbcast:7 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %3, %11 row_newbcast:8 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %4, %11 row_newbcast:8 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %5, %12 row_newbcast:8 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %6, %12 row_newbcast:8 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %3, %12 row_newbcast:9 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %4, %13 row_newbcast:2 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %3, %13 row_newbcast:3 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %6, %13 row_newbcast:3 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %5, %14 row_newbcast:2 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %4, %14 row_newbcast:3 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %3, %14 row_newbcast:4 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %6, %15 row_newbcast:2 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %5, %15 row_newbcast:3 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %4, %15 row_newbcast:4 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %3, %16 row_newbcast:10 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %4, %16 row_newbcast:10 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %5, %16 row_newbcast:10 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %6, %17 row_newbcast:10 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %3, %17 row_newbcast:11 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %4, %17 row_newbcast:11 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %5, %18 row_newbcast:11 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %6, %18 row_newbcast:11 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %3, %18 row_newbcast:12 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %5, %19 row_newbcast:4 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %4, %19 row_newbcast:5 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %3, %19 row_newbcast:6 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %6, %20 row_newbcast:4 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %5, %20 row_newbcast:5 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %4, %20 row_newbcast:6 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %3, %21 row_newbcast:5 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %6, %21 row_newbcast:5 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %5, %21 row_newbcast:6 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %3, %22 row_newbcast:13 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %4, %22 row_newbcast:13 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %5, %22 row_newbcast:13 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %6, %23 row_newbcast:13 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %3, %23 row_newbcast:14 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %4, %23 row_newbcast:14 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %0, %5, %24 row_newbcast:14 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %1, %6, %24 row_newbcast:14 row_mask:0xf bank_mask:0xf\n"
        "v_fmac_f32_dpp %2, %3, %24 row_newbcast:15 row_mask:0xf bank_mask:0xf\n"
        : "=&v"(h[0]), "=&v"(h[1]), "=&v"(h[2])
        : "v"(cv[0]), "v"(cv[1]), "v"(cv[2]), "v"(cv[3]),
          "v"(sn[0][0]), "v"(sn[0][1]), "v"(sn[0][2]), "v"(sn[1][0]), "v"(sn[1][1]), "v"(sn[1][2]),
          "v"(sn[2][0]), "v"(sn[2][1]), "v"(sn[2][2]), "v"(sn[3][0]), "v"(sn[3][1]), "v"(sn[3][2]),
          "v"(sn[4][0]), "v"(sn[4][1]), "v"(sn[4][2]), "v"(sn[5][0]), "v"(sn[5][1]), "v"(sn[5][2]));
}

__device__ __forceinline__ void load_site(float (&v)[3], Rsrc r, unsigned voff, unsigned soff)
{
    v[0] = ld(r, voff + 0u, soff);
    v[1] = ld(r, voff + 256u, soff);
    v[2] = ld(r, voff + 512u, soff);
}

// Byte offsets (scalar) of the 7 sites a lane reads for one update, and the
// float offset of the site's block in the packed couplings (or, with bond
// codes, the site's eight code bytes, read one site ahead).
struct ClSite {
    unsigned own, nb[6];
    unsigned cpl;        // first of the site's 54 coupling floats
    uint32_t lo, hi;     // bond codes of A_0..A_3 and A_4, A_5 (bimodal samples)
    int site;            // canonical index
    unsigned cvoff;      // canonical couplings: this lane's byte offset (canon_lane)
};

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v2f __attribute__((ext_vector_type(2)));
using CV16 = __attribute__((address_space(4))) const v16f;
using CV4 = __attribute__((address_space(4))) const v4f;
using CV2 = __attribute__((address_space(4))) const v2f;
typedef float v8f __attribute__((ext_vector_type(8)));
using CV8 = __attribute__((address_space(4))) const v8f;
using CU32 = __attribute__((address_space(4))) const uint32_t;

template <bool OWN, bool CANON>
__device__ __forceinline__ void cl_gather(ClGather &g, Rsrc r, unsigned voff, const ClSite &t, Rsrc rc)
{
#pragma unroll
    for (int n = 0; n < 6; ++n) load_site(g.n[n], r, voff, t.nb[n]);
    if constexpr (OWN) load_site(g.o, r, voff, t.own);
    if constexpr (CANON)
        g.cv = __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(rc, t.cvoff, 0, 0));
}

using ClEWave = double[kClWaves][64];

// One workgroup's share of a half-sweep: block (bx, bz) of the launch grid
// (8*per, 1, items).  `e_wave` is LDS for the energy partials (ENERGY only).
template <int KIND, bool ENERGY, int CM, class Params>
__device__ __forceinline__ void cl_half_sweep_block(Params &P, unsigned bx, unsigned bz, ClEWave *e_wave)
{
    constexpr bool BM = CM == 1;      // bond codes and the per-sample matrix table
    constexpr bool CANON = CM == 2;   // float couplings from the canonical blocks
    constexpr bool kOwn = KIND != kHeatbath;
    const int s = P.items[2 * bz];
    const int g = P.items[2 * bz + 1];
    const int lane = threadIdx.x & 63;
    // wave-uniform (the compiler cannot infer it from threadIdx.x)
    const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int j = g * 64 + lane;               // chain of the sample
    const bool lane_on = j < P.C;
    const int c = P.colour;
    const int L = P.L, Lh = L >> 1;
    const unsigned H = static_cast<unsigned>(P.H);
    const float *grp = P.spins + P.spin_base[s] + static_cast<int64_t>(g) * 6 * H * 64;
    const Rsrc r = make_rsrc(grp, 2u * H * kRow);
    const unsigned voff = 4u * static_cast<unsigned>(lane);
    // The couplings are read-only for the whole launch: reading them through
    // the constant address space lets wave-uniform loads become scalar loads.
    const CFloat *M = (const CFloat *)(P.cpl + P.cpl_base[s]);
    // bimodal samples: eight code bytes per site in place of the 54 floats,
    // and the sample's 128 decoded matrices (9 floats each), a table small
    // enough to stay in the scalar cache
    const CU32 *codes = (const CU32 *)(P.cpl + P.cpl_base[s]);
    const CFloat *table = BM ? (const CFloat *)(P.bm_table) + s * (128 * 9) : nullptr;
    // canonical blocks of the sample (27 floats a site) and this lane's part
    const Rsrc rc = make_rsrc(CANON ? P.cpls + P.cpls_base[s] : P.cpl, CANON ? 2u * H * 27u * 4u : 0u);
    const CanonLane cl = canon_lane(lane);

    uint32_t ctr3 = 0, hb_sweep = 0;
    float beta = 0.0f;
    if constexpr (KIND == kHeatbath) {
        hb_sweep = P.counters[0] + P.hb_offset;
        const int chain = P.chain_base[s] + (lane_on ? j : 0);
        ctr3 = ctr_word3(0u, static_cast<uint32_t>(P.slot_of[chain]), static_cast<uint32_t>(j / P.T));
        beta = P.beta_of[chain];
    }

    // This wave's segment: packed row `row` (= y + L*z), x-halves [x0, x0 + len).
    const int tile = xcd_tile(bx, P.per, P.colour == 1);   // colour 1 backwards
    if (tile >= P.n_tiles) return;
    const int seg = tile * kClWaves + wave;
    const int rl = seg / P.split;                 // row in visiting order
    const int len = Lh / P.split;
    const int x0 = (seg - rl * P.split) * len;
    int row = rl;                                 // packed row y + L*z
    if (P.strip > 0) {
        const int per_strip = L * P.strip;
        const int q = rl % per_strip;
        row = (q / P.strip) * L + (rl / per_strip) * P.strip + q % P.strip;
    }
    double e_acc = 0.0;
    if (rl < L * L) {  // strip order maps [0, L*L) onto itself
        const int y = row % L, z = row / L;
        const int par = (c + y + z) & 1;              // parity of x along this row
        const unsigned oth = static_cast<unsigned>(1 - c) * H;
        const unsigned rowp = static_cast<unsigned>(row * Lh);
        const unsigned yp = static_cast<unsigned>((y == L - 1 ? row - (L - 1) : row + 1) * Lh);
        const unsigned ym = static_cast<unsigned>((y == 0 ? row + (L - 1) : row - 1) * Lh);
        const unsigned zp = static_cast<unsigned>((z == L - 1 ? row - (L - 1) * L : row + L) * Lh);
        const unsigned zm = static_cast<unsigned>((z == 0 ? row + (L - 1) * L : row - L) * Lh);
        const int rowc = L * row;                      // canonical index of (0, y, z)
        // per-row bases; a site adds xh * kRow (spins) or xh * 54 (couplings)
        const unsigned b_own = (static_cast<unsigned>(c) * H + rowp) * kRow;
        const unsigned b_x = (oth + rowp) * kRow;
        const unsigned b_yp = (oth + yp) * kRow, b_ym = (oth + ym) * kRow;
        const unsigned b_zp = (oth + zp) * kRow, b_zm = (oth + zm) * kRow;
        const unsigned c_site = static_cast<unsigned>(c) * H + rowp;   // packed index of (0, y, z), colour c

        auto site_at = [&](int xh) {
            ClSite t;
            const int x = 2 * xh + par;
            const int xpp = par ? (xh + 1 == Lh ? 0 : xh + 1) : xh;   // packed x of x+1
            const int xmm = par ? xh : (xh == 0 ? Lh - 1 : xh - 1);   // packed x of x-1
            const unsigned o = static_cast<unsigned>(xh) * kRow;
            t.own = b_own + o;
            t.nb[0] = b_x + static_cast<unsigned>(xpp) * kRow;
            t.nb[1] = b_x + static_cast<unsigned>(xmm) * kRow;
            t.nb[2] = b_yp + o;
            t.nb[3] = b_ym + o;
            t.nb[4] = b_zp + o;
            t.nb[5] = b_zm + o;
            t.site = rowc + x;
            t.cpl = (c_site + static_cast<unsigned>(xh)) * 54u;
            if constexpr (CANON) {
                // canonical index of the site of this lane's kind: own, or the
                // backward neighbour along x, y or z
                const int xm = x == 0 ? L - 1 : x - 1;
                const int sx = rowc + xm;
                const int sy = (y == 0 ? t.site + (L - 1) * L : t.site - L);
                const int sz = (z == 0 ? t.site + (L - 1) * L * L : t.site - L * L);
                const int sel = cl.kind == 0 ? t.site : cl.kind == 1 ? sx : cl.kind == 2 ? sy : sz;
                t.cvoff = (27u * static_cast<unsigned>(sel) + cl.off) * 4u;
            }
            if constexpr (BM) {
                t.lo = codes[2 * (c_site + static_cast<unsigned>(xh))];
                t.hi = codes[2 * (c_site + static_cast<unsigned>(xh)) + 1];
            }
            return t;
        };

        auto process = [&](const ClGather &gt, const ClSite &t) {
            // The site's 54 coefficients in five scalar loads.  The empty asm
            // needs all of them at once, so the loads are issued together and
            // waited for once, instead of one round trip per load.
            float h[3];
            if constexpr (BM) {
                // the six matrices from the table, twelve scalar loads issued
                // together (the codes arrived with the previous site)
                v8f m8[6];
                float m1[6];
#pragma unroll
                for (int n = 0; n < 6; ++n) {
                    const uint32_t code = (n < 4 ? t.lo >> (8 * n) : t.hi >> (8 * (n - 4))) & 0x7fu;
                    const CFloat *q = table + 9u * code;
                    m8[n] = *(CV8 *)(q);
                    m1[n] = q[8];
                }
                asm volatile("" ::"s"(m8[0]), "s"(m8[1]), "s"(m8[2]), "s"(m8[3]), "s"(m8[4]), "s"(m8[5]),
                             "s"(m1[0]), "s"(m1[1]), "s"(m1[2]), "s"(m1[3]), "s"(m1[4]), "s"(m1[5]));
                local_field(gt.n, [&](int n, int a, int b) {
                    const int q = a * 3 + b;
                    return q < 8 ? m8[n][q] : m1[n];
                }, h);
            } else if constexpr (CANON) {
                local_field_rows(gt.n, gt.cv, h);
            } else {
                const CFloat *A = M + t.cpl;
                const v16f a0 = *(CV16 *)(A);
                const v16f a1 = *(CV16 *)(A + 16);
                const v16f a2 = *(CV16 *)(A + 32);
                const v4f a3 = *(CV4 *)(A + 48);
                const v2f a4 = *(CV2 *)(A + 52);
                asm volatile("" ::"s"(a0), "s"(a1), "s"(a2), "s"(a3), "s"(a4));
                local_field(gt.n, [&](int n, int a, int b) {
                    const int q = n * 9 + a * 3 + b;
                    return q < 16 ? a0[q] : q < 32 ? a1[q - 16] : q < 48 ? a2[q - 32] : q < 52 ? a3[q - 48] : a4[q - 52];
                }, h);
            }
            float sx, sy, sz;
            if constexpr (KIND == kHeatbath) {
                const uint4 w = philox10(make_uint4(static_cast<uint32_t>(t.site), hb_sweep,
                                                    static_cast<uint32_t>(s), ctr3),
                                         P.key0, P.key1);
                heatbath(sx, sy, sz, h[0], h[1], h[2], beta, unit23(w.x), unit23(w.y));
            } else {
                sx = gt.o[0]; sy = gt.o[1]; sz = gt.o[2];
                if constexpr (KIND == kOverrelax) overrelax(sx, sy, sz, h[0], h[1], h[2]);
            }
            if (KIND != kEnergyOnly && lane_on) {
                st(r, sx, voff + 0u, t.own);
                st(r, sy, voff + 256u, t.own);
                st(r, sz, voff + 512u, t.own);
            }
            if constexpr (ENERGY)
                e_acc += static_cast<double>(sx) * h[0] + static_cast<double>(sy) * h[1] +
                         static_cast<double>(sz) * h[2];
        };

        // software pipeline: the loads of the next site are issued before
        // the current site is updated
        ClGather ga, gb;
        ClSite ta = site_at(x0), tb;
        cl_gather<kOwn, CANON>(ga, r, voff, ta, rc);
        for (int xh = x0; xh < x0 + len; xh += 2) {
            const bool has_b = xh + 1 < x0 + len;
            if (has_b) {
                tb = site_at(xh + 1);
                cl_gather<kOwn, CANON>(gb, r, voff, tb, rc);
            }
            process(ga, ta);
            if (!has_b) break;
            if (xh + 2 < x0 + len) {
                ta = site_at(xh + 2);
                cl_gather<kOwn, CANON>(ga, r, voff, ta, rc);
            }
            process(gb, tb);
        }
    }

    if constexpr (ENERGY) {
        // the four waves hold the same 64 chains: reduce them in a fixed order
        (*e_wave)[wave][lane] = e_acc;
        __syncthreads();
        if (wave == 0 && lane_on) {
            double e = 0.0;
#pragma unroll
            for (int w = 0; w < kClWaves; ++w) e += (*e_wave)[w][lane];
            P.e_part[static_cast<int64_t>(P.chain_base[s] + j) * P.e_stride + tile] = e;
        }
    }
}

template <int KIND, bool ENERGY, int CM>
__global__ __launch_bounds__(kClBlock) void cl_half_sweep_kernel(ClParams P)
{
    if constexpr (ENERGY) {
        __shared__ ClEWave e_wave;
        cl_half_sweep_block<KIND, ENERGY, CM>(P, blockIdx.x, blockIdx.z, &e_wave);
    } else {
        cl_half_sweep_block<KIND, ENERGY, CM>(P, blockIdx.x, blockIdx.z, nullptr);
    }
}

// The persistent step in this mapping (see site_step_kernel).
using CDesc = __attribute__((address_space(4))) const StepDesc;
using CInt = __attribute__((address_space(4))) const int;

template <int BM, class Params>
__device__ __forceinline__ void cl_dispatch(Params &p, int kind, int energy, unsigned bx, unsigned bz, ClEWave *ew)
{
    if (kind == kOverrelax) {
        if (energy) cl_half_sweep_block<kOverrelax, true, BM>(p, bx, bz, ew);
        else cl_half_sweep_block<kOverrelax, false, BM>(p, bx, bz, ew);
    } else if (kind == kHeatbath) {
        if (energy) cl_half_sweep_block<kHeatbath, true, BM>(p, bx, bz, ew);
        else cl_half_sweep_block<kHeatbath, false, BM>(p, bx, bz, ew);
    } else {
        cl_half_sweep_block<kEnergyOnly, true, BM>(p, bx, bz, ew);
    }
}

__global__ __launch_bounds__(kClBlock) __attribute__((amdgpu_waves_per_eu(6))) void cl_step_kernel(PersistParams P)
{
    __shared__ ClEWave e_wave;
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
                auto &p = desc[d].cp;
                const int kind = desc[d].kind, energy = desc[d].energy;
                if (p.bimodal) cl_dispatch<true>(p, kind, energy, bx, bz, &e_wave);
                else cl_dispatch<false>(p, kind, energy, bx, bz, &e_wave);
            }
            __syncthreads();   // e_wave is reused by the next block
        }
        cooperative_groups::this_grid().sync();
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && P.d_hb) P.counters[0] += P.d_hb;
}

}  // namespace

int cl_step_blocks_per_cu()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, cl_step_kernel, kClBlock, 0) != hipSuccess) return 0;
    return n;
}

hipError_t launch_cl_step(const PersistParams &p, int grid, hipStream_t st)
{
    void *args[] = {const_cast<PersistParams *>(&p)};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(cl_step_kernel), dim3(grid),
                                      dim3(kClBlock), args, 0, st);
}

int cl_blocks(int L, int split) { return (L * L * split + kClWaves - 1) / kClWaves; }

hipError_t launch_cl_half_sweep(int kind, bool energy, const ClParams &p, int n_items, hipStream_t st,
                                const LaunchTiming &t)
{
    const dim3 grid(kXcds * p.per, 1, n_items);
    const dim3 block(kClBlock);
    auto go = [&](auto kernel) { return launch_kernel(kernel, grid, block, 0, st, t, p); };
    if (p.bimodal) {
        if (kind == kOverrelax)
            return energy ? go(cl_half_sweep_kernel<kOverrelax, true, 1>) : go(cl_half_sweep_kernel<kOverrelax, false, 1>);
        if (kind == kHeatbath)
            return energy ? go(cl_half_sweep_kernel<kHeatbath, true, 1>) : go(cl_half_sweep_kernel<kHeatbath, false, 1>);
        return go(cl_half_sweep_kernel<kEnergyOnly, true, 1>);
    }
    // Float couplings: the overrelaxation and energy half-sweeps read the
    // canonical blocks (27 floats a site: a group and its sample's couplings
    // then fit the Infinity Cache), the heat-bath ones the packed blocks (the
    // canonical form's extra registers cost that VALU-bound kernel more
    // than its bytes save).
    if (p.canon && kind != kHeatbath)
        return kind == kOverrelax
                   ? (energy ? go(cl_half_sweep_kernel<kOverrelax, true, 2>) : go(cl_half_sweep_kernel<kOverrelax, false, 2>))
                   : go(cl_half_sweep_kernel<kEnergyOnly, true, 2>);
    if (kind == kOverrelax)
        return energy ? go(cl_half_sweep_kernel<kOverrelax, true, 0>) : go(cl_half_sweep_kernel<kOverrelax, false, 0>);
    if (kind == kHeatbath)
        return energy ? go(cl_half_sweep_kernel<kHeatbath, true, 0>) : go(cl_half_sweep_kernel<kHeatbath, false, 0>);
    return go(cl_half_sweep_kernel<kEnergyOnly, true, 0>);
}

}  // namespace ptsg
