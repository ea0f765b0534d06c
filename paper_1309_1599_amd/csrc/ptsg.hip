// ptsg.hip -- the C ABI (include/ptsg.h): validation, device memory plan,
// host-side packing of couplings, and the launch sequence of a step.
#include "../../include/ptsg.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <mutex>
#include <tuple>
#include <new>
#include <string>
#include <vector>

#include "kernels.hpp"

using namespace ptsg;

namespace {

thread_local std::string g_err;

pt_status fail(pt_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

#define PT_HIP(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(PT_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

constexpr size_t kAlign = 256;


size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// One lattice class: samples sharing L, the number of temperatures and the
// kernel mapping, swept by the same launches.
enum Mapping { kSiteLanes = 0, kChainLanes = 1, kResident = 2 };

struct LatticeClass {
    int L = 0, T = 0, C = 0, lanes = 1, mapping = kSiteLanes;
    int G = 1;                       // site lanes: chains per workgroup
    int split = 1;                   // chain lanes: waves per packed row
    int strip = 0;                   // chain lanes: y-rows per strip of the row order
    int blocks = 0;                  // workgroups per (sample or item) and half-sweep
    int batch = 1;                   // chain lanes: items per launch; site lanes: samples per launch
                                     // (both sized to the Infinity Cache budget)
    std::vector<int> samples;
    int *d_samples = nullptr;
    std::vector<int> items;          // chain lanes: (sample, group) pairs
    int *d_items = nullptr;
};

// Device memory plan of a batch: byte offsets into one workspace.
struct Plan {
    int S = 0, R = 0, n_chains = 0, Lmax = 0, n_records = 0, e_stride = 1, twid_len = 0;
    std::vector<int> L, T, lanes, mapping, chain_base, perm_base, beta_base, twid_base;
    std::vector<char> codes;          // per sample: bond codes instead of packed floats (PT_F_BIMODAL, site and chain lanes)
    std::vector<int64_t> spin_base, cpls_base, cpl6_base;
    int64_t spin_floats = 0, cpls_floats = 0, cpl6_floats = 0;
    int total_perm = 0, n_items = 0;
    size_t off_spins = 0, off_cpls = 0, off_cpl6 = 0, off_slot = 0, off_beta_of = 0, off_E = 0,
           off_perm = 0, off_betas = 0, off_epart = 0, off_twid = 0, off_meta = 0, off_rec = 0,
           off_mpart = 0, off_meas = 0, off_classes = 0, off_items = 0, off_stage = 0, off_counters = 0,
           off_bmD = 0, off_bmtab = 0, off_cursor = 0,
           bytes = 0;
};

// Chain-lane launches keep the working set of one batch of (sample, group)
// items -- 64 chains of spins plus the sample's couplings -- inside this
// share of the 256 MB Infinity Cache.
constexpr int64_t kCacheBudget = 192ll << 20;

// Largest split of a packed row into wave segments (1, 2, 4 or 8 segments,
// at least 2 sites each).
int max_split(int L)
{
    const int Lh = L / 2;
    int best = 1;
    for (int s = 2; s <= 8; s *= 2)
        if (Lh % s == 0 && Lh / s >= 2) best = s;
    return best;
}

// Samples per site-lane launch within the cache budget (spins of all chains
// plus the packed couplings, or their byte codes).  Every sweep of a step
// runs on one batch before the next, so the half-sweeps after the first
// find the batch in the Infinity Cache instead of HBM.
int site_batch(int L, int C, bool codes, int n_samples)
{
    const int64_t N = static_cast<int64_t>(L) * L * L;
    const int64_t sample = static_cast<int64_t>(C) * 12 * N + (codes ? 8 : 216) * N;
    const int64_t budget = kCacheBudget;
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(n_samples, budget / sample)));
}

// Items (64-chain groups) per chain-lane launch within the cache budget.
int cl_batch(int L, int n_items)
{
    const int64_t N = static_cast<int64_t>(L) * L * L;
    const int64_t item = 64 * 3 * N * 4 + 54 * N * 4;
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(n_items, kCacheBudget / item)));
}

// Segments per packed row: the most segments (up to 8) that keep at least 4
// sites per wave (at L = 64 eight segments of 4 sites measured 6% faster
// than four of 8, and those 14% faster than whole rows: more waves in
// flight to cover the memory latency), then more while a launch would have
// fewer than 1024 workgroups.
int choose_split(int L, int batch)
{
    const int Lh = L / 2;
    int best = 1;
    for (int s = 2; s <= 8; s *= 2)
        if (Lh % s == 0 && Lh / s >= 4) best = s;
    while (static_cast<int64_t>(cl_blocks(L, best)) * batch < 1024 && best < 8 && Lh % (2 * best) == 0 &&
           Lh / (2 * best) >= 2)
        best *= 2;
    return best;
}

// Rows are visited in strips of this many y-rows (z-major inside a strip);
// 16 measured best at L = 64, against 8, 32 and plain y-major order.
int choose_strip(int L)
{
    for (int w : {16, 8, 4})
        if (L % w == 0) return w;
    return 0;
}

// Chain lanes where they are measured faster: 24 <= L <= 64 with the
// sample's chains filling its 64-lane waves to >= 90%.
bool chain_lanes_pay(int L, int C)
{
    const int waves = (C + 63) / 64;
    return L >= 24 && L <= 64 && 10 * C >= 9 * 64 * waves;
}

// A persistent step is one kernel, so one mapping serves the whole batch:
// chain lanes when forced (and every L <= 128) or when they pay for every
// sample, else site lanes.
int persistent_mapping(const pt_batch_desc *d)
{
    bool chain = !(d->flags & (PT_F_SITE_LANES | PT_F_PLAIN));
    for (int q = 0; q < d->n_samples && chain; ++q)
        chain = (d->flags & PT_F_CHAIN_LANES) ? d->L[q] <= 128
                                              : chain_lanes_pay(d->L[q], d->n_replicas * d->n_temps[q]);
    return chain ? kChainLanes : kSiteLanes;
}

int choose_mapping(const pt_batch_desc *d, int s)
{
    const int L = d->L[s], C = d->n_replicas * d->n_temps[s];
    if (d->flags & PT_F_ROW_OR) return kChainLanes;  // the row-order kernel is chain-lane
    if (d->flags & PT_F_PERSISTENT) return persistent_mapping(d);
    if (d->flags & (PT_F_SITE_LANES | PT_F_PLAIN)) return kSiteLanes;
    if (d->flags & PT_F_CHAIN_LANES) return L <= 128 ? kChainLanes : kSiteLanes;
    if (d->flags & PT_F_RESIDENT) return L <= kRsMaxL ? kResident : kSiteLanes;
    // Resident lattices (one workgroup per chain) need enough chains to fill
    // the chip: with 16 samples of L = 12 or 16 they beat both other mappings
    // (18.7 and 14.1 ps/SU), with the 32 chains of one L = 16 sample they
    // trail them (83 against 68 site lanes, 66 chain lanes).
    int class_chains = 0;
    for (int q = 0; q < d->n_samples; ++q)
        if (d->L[q] == L && d->n_temps[q] == d->n_temps[s]) class_chains += C;
    if (L <= 8 || (L <= kRsMaxL && class_chains >= 256)) return kResident;
    // Chain lanes only when the 64-lane waves are (nearly) full and L is in
    // the measured range where they win: site lanes are faster at L = 20
    // and at L = 96 and 128, chain lanes from L = 24 to 64 (up to there a
    // group of 64 chains, 201 MB at L = 64, stays in the 256 MB Infinity
    // Cache between the half-sweeps that the group-major order runs back to
    // back).
    return chain_lanes_pay(L, C) ? kChainLanes : kSiteLanes;
}

// The paper's coupling family (Sec. II.A): M = J*1 + D_sym with J = +-1 and
// the six independent entries of the symmetric D equal to +-D.  A bond is
// one byte: bit 0 set for J = -1, bits 1..6 set for a negative D entry, in
// the order 00, 11, 22, 01, 02, 12.  Decoding computes the diagonal as the
// FP32 sum J + d, exactly as the device decoder does.
void bimodal_matrix(unsigned code, float D, float m[9])
{
    const float J = (code & 1u) ? -1.0f : 1.0f;
    float d[6];
    for (int k = 0; k < 6; ++k) d[k] = ((code >> (1 + k)) & 1u) ? -D : D;
    m[0] = J + d[0];
    m[4] = J + d[1];
    m[8] = J + d[2];
    m[1] = m[3] = d[3];
    m[2] = m[6] = d[4];
    m[5] = m[7] = d[5];
}

// The code of bond matrix m (row-major), or -1 if m is not J*1 + D_sym of
// this D bit for bit.
int bimodal_code(const float m[9], float D)
{
    for (unsigned jbit = 0; jbit < 2; ++jbit) {
        const float J = jbit ? -1.0f : 1.0f;
        unsigned c = jbit;
        for (int a = 0; a < 3; ++a)
            if (m[4 * a] == J + (-D)) c |= 1u << (1 + a);
        if (m[1] == -D) c |= 1u << 4;
        if (m[2] == -D) c |= 1u << 5;
        if (m[5] == -D) c |= 1u << 6;
        float t[9];
        bimodal_matrix(c, D, t);
        if (std::memcmp(t, m, sizeof(t)) == 0) return static_cast<int>(c);
    }
    return -1;
}

// D of a sample in the family (> 0, from its first bond), or 0 if the sample
// is not in it.
float bimodal_D(int L, const float *M)
{
    const float D = std::fabs(M[1]);
    if (!(D > 0.0f) || !std::isfinite(D)) return 0.0f;
    const int64_t nb = 3 * static_cast<int64_t>(L) * L * L;
    for (int64_t b = 0; b < nb; ++b)
        if (bimodal_code(M + 9 * b, D) < 0) return 0.0f;
    return D;
}

std::string validate(const pt_batch_desc *d)
{
    if (!d) return "descriptor is NULL";
    if (d->n_samples < 1) return "n_samples must be >= 1";
    if (!d->L || !d->n_temps || !d->temps || !d->couplings) return "NULL array in descriptor";
    if ((d->flags & PT_F_ROW_OR) && (d->flags & (PT_F_SITE_LANES | PT_F_RESIDENT | PT_F_PLAIN)))
        return "PT_F_ROW_OR runs on the chain-lane mapping: it excludes PT_F_SITE_LANES, PT_F_RESIDENT and PT_F_PLAIN";
    if ((d->flags & PT_F_PERSISTENT) && (d->flags & (PT_F_ROW_OR | PT_F_RESIDENT)))
        return "PT_F_PERSISTENT runs the checkerboard site-lane or chain-lane sweeps: it excludes PT_F_ROW_OR "
               "and PT_F_RESIDENT";
    if (d->n_replicas < 1 || d->n_replicas > 256) return "n_replicas must be in [1, 256]";
    for (int s = 0; s < d->n_samples; ++s) {
        const int L = d->L[s];
        if (L < 4 || L > 256 || (L & 1))
            return "sample " + std::to_string(s) + ": L must be even and in [4, 256]";
        const int T = d->n_temps[s];
        if (T < 1 || T > 4096) return "sample " + std::to_string(s) + ": n_temps must be in [1, 4096]";
        if (!d->temps[s] || !d->couplings[s]) return "sample " + std::to_string(s) + ": NULL pointer";
        for (int k = 0; k < T; ++k) {
            const double t = d->temps[s][k];
            if (!(t > 0.0) || !std::isfinite(t))
                return "sample " + std::to_string(s) + ": temperatures must be finite and > 0";
            if (k > 0 && !(t > d->temps[s][k - 1]))
                return "sample " + std::to_string(s) + ": temperatures must be strictly ascending";
        }
        // Rows of 8 along x fall in classes (x/8 + y + z) mod 2; with an odd
        // number of rows along x above one, the first and last row of an x
        // line touch across the boundary in the same class.
        if ((d->flags & PT_F_ROW_OR) && ((L != 8 && L % 16 != 0) || L > 128))
            return "sample " + std::to_string(s) + ": PT_F_ROW_OR needs L = 8 or a multiple of 16, and L <= 128";
        if ((d->flags & PT_F_BIMODAL) && bimodal_D(L, d->couplings[s]) == 0.0f)
            return "sample " + std::to_string(s) +
                   ": PT_F_BIMODAL needs every bond to be J*1 + D_sym with J = +-1 and D_ab = +-D, D > 0";
    }
    return "";
}

// A tuned plan of one lattice class: the mapping and its tile shape (0 or
// -1: the heuristic's choice).
struct Tile {
    int mapping = -1;
    int G = 0;        // site lanes: chains per workgroup
    int split = 0;    // chain lanes: waves per packed row
    int strip = -1;   // chain lanes: y-rows per strip of the row order (0: y-major)
};

// `forced`, when given, holds one tuned plan per sample (from the autotuner).
Plan make_plan(const pt_batch_desc *d, const std::vector<Tile> *forced = nullptr)
{
    Plan p;
    p.S = d->n_samples;
    p.R = d->n_replicas;
    int chains = 0, perm = 0, betas = 0, twid = 0;
    int64_t spins = 0, cpls = 0, cpl6 = 0;
    int max_blocks = 1;
    for (int s = 0; s < p.S; ++s) {
        const int L = d->L[s], T = d->n_temps[s];
        const int64_t N = static_cast<int64_t>(L) * L * L;
        const int C = p.R * T;
        const int mapping = forced ? (*forced)[s].mapping : choose_mapping(d, s);
        const int lanes = mapping == kChainLanes ? 64 : 1;
        const int C_alloc = (C + lanes - 1) / lanes * lanes;
        p.L.push_back(L);
        p.T.push_back(T);
        p.lanes.push_back(lanes);
        p.mapping.push_back(mapping);
        p.chain_base.push_back(chains);
        p.perm_base.push_back(perm);
        p.beta_base.push_back(betas);
        p.twid_base.push_back(twid);
        p.spin_base.push_back(spins);
        p.cpls_base.push_back(cpls);
        p.cpl6_base.push_back(cpl6);  // [colour][54][H] (lanes = 1) or [colour][H][54] (chain lanes)
        chains += C;
        perm += C;
        betas += T;
        twid += 2 * L;
        spins += static_cast<int64_t>(C_alloc) * 3 * N;
        cpls += 27 * N;
        // the row-order kernel and the resident kernel read floats
        const bool codes = (d->flags & PT_F_BIMODAL) &&
                           (mapping == kSiteLanes || (mapping == kChainLanes && !(d->flags & PT_F_ROW_OR)));
        p.codes.push_back(codes);
        cpl6 += codes ? 2 * N : 54 * N;   // 8 bytes per site, or 54 floats
        if (lanes == 1) {
            max_blocks = std::max<int>(max_blocks, static_cast<int>((N / 2 + kSweepBlock - 1) / kSweepBlock));
        } else {
            max_blocks = std::max(max_blocks, cl_blocks(L, max_split(L)));
            p.n_items += (C + 63) / 64;
        }
        p.Lmax = std::max(p.Lmax, L);
        p.n_records += T * p.R * (p.R - 1) / 2;
    }
    p.n_chains = chains;
    p.total_perm = perm;
    p.spin_floats = spins;
    p.cpls_floats = cpls;
    p.cpl6_floats = cpl6;
    p.e_stride = max_blocks;
    p.twid_len = twid;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    p.off_spins = take(sizeof(float) * static_cast<size_t>(spins));
    p.off_cpls = take(sizeof(float) * static_cast<size_t>(cpls));
    p.off_cpl6 = take(sizeof(float) * static_cast<size_t>(std::max<int64_t>(cpl6, 1)));
    p.off_slot = take(sizeof(int) * chains);
    p.off_beta_of = take(sizeof(float) * chains);
    p.off_E = take(sizeof(double) * chains);
    p.off_perm = take(sizeof(int) * perm);
    p.off_betas = take(sizeof(double) * betas);
    p.off_epart = take(sizeof(double) * static_cast<size_t>(chains) * p.e_stride);
    p.off_twid = take(sizeof(double) * twid);
    // per-sample tables: spin_base, cpls_base, cpl6_base (int64); L, n_temps,
    // chain_base, perm_base, beta_base, twid_base, lanes (int)
    p.off_meta = take(3 * sizeof(int64_t) * p.S + 7 * sizeof(int) * p.S);
    p.off_rec = take(sizeof(int) * 4 * std::max(1, p.n_records));
    p.off_mpart = take(sizeof(double) * static_cast<size_t>(std::max(1, p.n_records)) * p.Lmax * kPlaneQ);
    p.off_meas = take(sizeof(pt_meas) * std::max(1, p.n_records));
    p.off_classes = take(sizeof(int) * p.S);
    p.off_items = take(sizeof(int) * 2 * std::max(1, p.n_items));
    // staging: one chain in canonical order, or all chains of the largest
    // chain-lane sample in the site-lane layout (measurement)
    size_t stage = 3 * static_cast<size_t>(p.Lmax) * p.Lmax * p.Lmax;
    for (int s = 0; s < p.S; ++s)
        if (p.lanes[s] != 1)
            stage = std::max(stage, 3 * static_cast<size_t>(p.L[s]) * p.L[s] * p.L[s] * p.R * p.T[s]);
    p.off_stage = take(sizeof(float) * stage);
    p.off_counters = take(2 * sizeof(uint32_t));
    p.off_bmD = take(sizeof(float) * p.S);
    // bimodal: per sample the matrix of each of the 128 codes (chain lanes)
    p.off_bmtab = take(sizeof(float) * ((d->flags & PT_F_BIMODAL) ? 128 * 9 * static_cast<size_t>(p.S) : 1));
    p.off_cursor = take(sizeof(RecordCursor));
    p.bytes = o;
    return p;
}

struct Event {
    hipEvent_t a = nullptr, b = nullptr;
};

// Measurement partials of pt_measure_noalloc: a fixed device array instead
// of the context's workspace (8 MB, every device the library runs on holds
// one until the process ends).  Host code never passes `scratch` itself to a
// kernel: its device address, per device, comes from hipGetSymbolAddress.
constexpr size_t kScratchDoubles = size_t(1) << 20;
__device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_ptr;   // device -> address of its `scratch`

// Address of `scratch` on `device` (which must be current); looked up once
// per device.
pt_status scratch_on(int device, double **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it == g_scratch_ptr.end()) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PT_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        it = g_scratch_ptr.emplace(device, static_cast<double *>(p)).first;
    }
    *out = it->second;
    return PT_OK;
}

}  // namespace

struct pt_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    uint64_t seed = 0, hb_sweeps = 0, pt_passes = 0;
    std::vector<uint64_t> cpl_hash;   // per sample: FNV-1a of the couplings given at init
    std::vector<double> betas_host;   // per sample, concatenated: 1/T of each slot
    Plan plan;
    std::vector<LatticeClass> classes;
    char *ws = nullptr;
    bool own_ws = false;
    // device views
    float *spins = nullptr, *cpls = nullptr, *cpl6 = nullptr, *beta_of = nullptr;
    int *slot_of = nullptr, *perm = nullptr, *rec = nullptr;
    double *E = nullptr, *betas = nullptr, *epart = nullptr, *twid = nullptr, *mpart = nullptr;
    pt_meas *meas = nullptr;
    float *stage = nullptr;           // one chain in canonical [N][3] order
    uint32_t *counters = nullptr;     // device: heat-bath sweeps, PT passes
    float *bm_D = nullptr;            // device, per sample: D of the bimodal family (PT_F_BIMODAL)
    float *bm_table = nullptr;        // device, per sample: [128][9] matrix of each bond code
    RecordCursor *cursor = nullptr;   // device: where pt_run's next measurement goes
    bool use_graphs = false;
    bool row_or = false;              // PT_F_ROW_OR: overrelaxation sweeps in the row order
    hipStream_t capture_stream = nullptr;
    std::map<std::pair<int, int>, hipGraphExec_t> step_graphs;
    // pt_run: (n_hb, n_or, measurement bits or ~0 for none) -> graphs of one
    // step without and with a measurement after it
    struct RunGraphs {
        hipGraphExec_t one[2] = {nullptr, nullptr};
    };
    std::map<std::tuple<int, int, unsigned>, RunGraphs> run_graphs;
    // PT_F_PERSISTENT: one program per (n_hb, n_or), in library-owned memory
    struct Program {
        std::vector<StepDesc> desc;
        std::vector<int> first, blocks;   // per phase
        char *mem = nullptr;              // device copies of desc, first, blocks
        const StepDesc *d_desc = nullptr;
        const int *d_first = nullptr, *d_blocks = nullptr;
        int grid = 0;
    };
    bool persistent = false;
    std::map<std::pair<int, int>, Program> programs;
    int *d_L = nullptr, *d_T = nullptr, *d_chain_base = nullptr, *d_perm_base = nullptr,
        *d_beta_base = nullptr, *d_twid_base = nullptr, *d_lanes = nullptr;
    int64_t *d_spin_base = nullptr, *d_cpls_base = nullptr, *d_cpl6_base = nullptr;
    // profiling
    bool profiling = false;
    std::vector<std::pair<int, Event>> pending;
    std::vector<Event> free_events;
    uint64_t prof_launches[4] = {0, 0, 0, 0};
    double prof_ms[4] = {0.0, 0.0, 0.0, 0.0};
};

namespace {

SweepParams sweep_params(pt_ctx *c, const LatticeClass &k, int colour, uint32_t hb_offset)
{
    SweepParams p{};
    p.spins = c->spins;
    p.cpl = c->cpl6;
    p.samples = k.d_samples;
    p.spin_base = c->d_spin_base;
    p.cpl_base = c->d_cpl6_base;
    p.bm_D = c->bm_D;
    p.bimodal = c->plan.codes[k.samples[0]];
    p.chain_base = c->d_chain_base;
    p.slot_of = c->slot_of;
    p.beta_of = c->beta_of;
    p.e_part = c->epart;
    p.e_stride = c->plan.e_stride;
    p.L = k.L;
    p.H = k.L * k.L * k.L / 2;
    p.C = k.C;
    p.G = k.G;
    p.T = k.T;
    p.n_tiles = k.blocks;
    p.per = (k.blocks + 7) / 8;
    p.colour = colour;
    p.counters = c->counters;
    p.hb_offset = hb_offset;
    p.key0 = static_cast<uint32_t>(c->seed);
    p.key1 = static_cast<uint32_t>(c->seed >> 32);
    return p;
}

ClParams cl_params(pt_ctx *c, const LatticeClass &k, int first_item, int colour, uint32_t hb_offset)
{
    ClParams p{};
    p.spins = c->spins;
    p.cpl = c->cpl6;
    p.items = k.d_items + 2 * first_item;
    p.spin_base = c->d_spin_base;
    p.cpl_base = c->d_cpl6_base;
    p.chain_base = c->d_chain_base;
    p.slot_of = c->slot_of;
    p.beta_of = c->beta_of;
    p.e_part = c->epart;
    p.e_stride = c->plan.e_stride;
    p.L = k.L;
    p.H = k.L * k.L * k.L / 2;
    p.C = k.C;
    p.T = k.T;
    p.bimodal = c->plan.codes[k.samples[0]];
    p.bm_table = c->bm_table;
    p.canon = !p.bimodal;   // overrelaxation and energy half-sweeps read the canonical blocks
    p.cpls = c->cpls;
    p.cpls_base = c->d_cpls_base;
    p.split = k.split;
    p.strip = k.strip;
    p.n_tiles = k.blocks;
    p.per = (k.blocks + 7) / 8;
    p.colour = colour;
    p.counters = c->counters;
    p.hb_offset = hb_offset;
    p.key0 = static_cast<uint32_t>(c->seed);
    p.key1 = static_cast<uint32_t>(c->seed >> 32);
    return p;
}

pt_status get_event(pt_ctx *c, Event &ev)
{
    if (!c->free_events.empty()) {
        ev = c->free_events.back();
        c->free_events.pop_back();
        return PT_OK;
    }
    PT_HIP(hipEventCreate(&ev.a));
    PT_HIP(hipEventCreate(&ev.b));
    return PT_OK;
}

pt_status drain_events(pt_ctx *c)
{
    if (c->pending.empty()) return PT_OK;
    PT_HIP(hipStreamSynchronize(c->stream));
    for (auto &pe : c->pending) {
        float ms = 0.0f;
        PT_HIP(hipEventElapsedTime(&ms, pe.second.a, pe.second.b));
        c->prof_ms[pe.first] += ms;
        c->prof_launches[pe.first] += 1;
        c->free_events.push_back(pe.second);
    }
    c->pending.clear();
    return PT_OK;
}

constexpr int kResidentKind = 3;  // profiling tag of whole-step resident launches

// Launch one sweep kernel; when profiling, the dispatch stamps a pair of
// events at the kernel's start and end.
template <class Launch>
pt_status timed_launch(pt_ctx *c, int kind, Launch launch)
{
    const bool timed = c->profiling && kind != kEnergyOnly;
    Event ev;
    LaunchTiming t;
    if (timed) {
        if (c->pending.size() >= 4096) {
            pt_status st = drain_events(c);
            if (st != PT_OK) return st;
        }
        pt_status st = get_event(c, ev);
        if (st != PT_OK) return st;
        t.start = ev.a;
        t.stop = ev.b;
    }
    PT_HIP(launch(t));
    if (timed)
        c->pending.push_back({kind == kOverrelax ? PT_K_OVERRELAX
                              : kind == kHeatbath ? PT_K_HEATBATH : PT_K_RESIDENT, ev});
    return PT_OK;
}

EnergyParams energy_params(pt_ctx *c, const LatticeClass &k)
{
    EnergyParams e{};
    e.e_part = c->epart;
    e.e_stride = c->plan.e_stride;
    e.n_blocks = k.blocks;
    e.samples = k.d_samples;
    e.chain_base = c->d_chain_base;
    e.C = k.C;
    e.E = c->E;
    return e;
}

pt_status finalize_energies(pt_ctx *c, const LatticeClass &k)
{
    PT_HIP(launch_energy_finalize(energy_params(c, k), static_cast<int>(k.samples.size()), c->stream));
    return PT_OK;
}

// The launches of one site-lane or chain-lane class's checkerboard sweeps,
// in order, as descriptors (the last one finalises the energies).  `kinds`
// lists the sweep kinds in order; the n-th heat-bath sweep of the list uses
// Philox counter (device heat-bath count) + n, and the energy partials are
// fused into the last half-sweep.  A descriptor may depend on the ones
// before it, never on a later one.
std::vector<StepDesc> class_sequence(pt_ctx *c, const LatticeClass &k, const std::vector<int> &kinds)
{
    std::vector<StepDesc> seq;
    const int total = static_cast<int>(kinds.size());
    const bool site = k.lanes == 1;
    // site lanes: sample-batch-major; chain lanes: chain-group-major -- every
    // sweep of one batch before the next
    const int n_units = site ? static_cast<int>(k.samples.size()) : static_cast<int>(k.items.size() / 2);
    for (int first = 0; first < n_units; first += k.batch) {
        const int cnt = std::min(k.batch, n_units - first);
        uint32_t hb = 0;
        for (int n = 0; n < total; ++n) {
            for (int colour = 0; colour < 2; ++colour) {
                StepDesc D{};
                D.kind = kinds[n];
                D.energy = n == total - 1 && colour == 1;
                if (site) {
                    D.op = kOpSite;
                    D.sp = sweep_params(c, k, colour, hb);
                    D.sp.samples = k.d_samples + first;
                    D.gx = kXcds * D.sp.per;
                    D.gy = (k.C + k.G - 1) / k.G;
                } else {
                    D.op = kOpChain;
                    D.cp = cl_params(c, k, first, colour, hb);
                    D.gx = kXcds * D.cp.per;
                    D.gy = 1;
                }
                D.gz = cnt;
                D.n_blocks = D.gx * D.gy * D.gz;
                seq.push_back(D);
            }
            if (kinds[n] == kHeatbath) ++hb;
        }
    }
    StepDesc F{};
    F.op = kOpFinalize;
    F.ep = energy_params(c, k);
    F.gx = ((k.C + 3) / 4 + kXcds - 1) / kXcds * kXcds;   // a multiple of 8; waves past C return
    F.gy = static_cast<int>(k.samples.size());
    F.gz = 1;
    F.n_blocks = F.gx * F.gy;
    seq.push_back(F);
    return seq;
}

// One descriptor as its own kernel launch.
pt_status launch_desc(pt_ctx *c, const StepDesc &D)
{
    if (D.op == kOpSite)
        return timed_launch(c, D.kind, [&](const LaunchTiming &t) {
            return launch_half_sweep(D.kind, D.energy, D.sp, D.gz, c->stream, t);
        });
    if (D.op == kOpChain)
        return timed_launch(c, D.kind, [&](const LaunchTiming &t) {
            return launch_cl_half_sweep(D.kind, D.energy, D.cp, D.gz, c->stream, t);
        });
    PT_HIP(launch_energy_finalize(D.ep, D.gy, c->stream));
    return PT_OK;
}

// The sweeps of one class: `kinds` lists the sweep kinds in order (see
// class_sequence).
pt_status sweep_class(pt_ctx *c, const LatticeClass &k, const std::vector<int> &kinds)
{
    const int total = static_cast<int>(kinds.size());
    if (total == 0) return PT_OK;
    pt_status st;
    if (k.mapping == kResident) {
        // one launch for the whole list: heat-bath sweeps first, then overrelaxation
        RsParams p{};
        p.spins = c->spins;
        p.cpl = c->cpl6;
        p.samples = k.d_samples;
        p.spin_base = c->d_spin_base;
        p.cpl_base = c->d_cpl6_base;
        p.chain_base = c->d_chain_base;
        p.slot_of = c->slot_of;
        p.beta_of = c->beta_of;
        p.E = c->E;
        p.L = k.L;
        p.H = k.L * k.L * k.L / 2;
        p.C = k.C;
        p.T = k.T;
        p.energy_only = kinds[0] == kEnergyOnly;
        p.n_hb = p.energy_only ? 0 : static_cast<int>(std::count(kinds.begin(), kinds.end(), kHeatbath));
        p.n_or = p.energy_only ? 1 : total - p.n_hb;
        p.counters = c->counters;
        p.key0 = static_cast<uint32_t>(c->seed);
        p.key1 = static_cast<uint32_t>(c->seed >> 32);
        const int n_chains = static_cast<int>(k.samples.size()) * k.C;
        return timed_launch(c, p.energy_only ? kEnergyOnly : kResidentKind,
                            [&](const LaunchTiming &t) { return launch_resident_step(p, n_chains, c->stream, t); });
    }
    if (k.lanes == 1 || !c->row_or) {
        for (const StepDesc &D : class_sequence(c, k, kinds))
            if ((st = launch_desc(c, D)) != PT_OK) return st;
        return PT_OK;
    }
    // chain lanes with the row-ordered overrelaxation: chain-group-major,
    // every sweep of one batch of items before the next
    const int n_items = static_cast<int>(k.items.size() / 2);
    for (int first = 0; first < n_items; first += k.batch) {
        const int cnt = std::min(k.batch, n_items - first);
        uint32_t hb = 0;
        for (int n = 0; n < total; ++n) {
            const int kind = kinds[n];
            if (kind == kOverrelax) {
                // class 0 rows, then class 1; energies after the last sweep
                ClParams p = cl_params(c, k, first, 0, hb);
                const int tiles = (row_waves(k.L) + kClWaves - 1) / kClWaves;
                p.per = (tiles + 7) / 8;   // grid = 8 XCDs x per
                for (int cls = 0; cls < 2; ++cls) {
                    st = timed_launch(c, kind, [&](const LaunchTiming &t) {
                        return launch_cl_row_or(p, cls, cnt, c->stream, t);
                    });
                    if (st != PT_OK) return st;
                }
                if (n == total - 1) {
                    const ClParams q = cl_params(c, k, first, 1, hb);
                    st = timed_launch(c, kEnergyOnly, [&](const LaunchTiming &t) {
                        return launch_cl_half_sweep(kEnergyOnly, true, q, cnt, c->stream, t);
                    });
                    if (st != PT_OK) return st;
                }
                continue;
            }
            for (int colour = 0; colour < 2; ++colour) {
                const bool energy = n == total - 1 && colour == 1;
                const ClParams p = cl_params(c, k, first, colour, hb);
                st = timed_launch(c, kind, [&](const LaunchTiming &t) {
                    return launch_cl_half_sweep(kind, energy, p, cnt, c->stream, t);
                });
                if (st != PT_OK) return st;
            }
            if (kind == kHeatbath) ++hb;
        }
    }
    return finalize_energies(c, k);
}

// Energies of every chain from the current spins (no update).
pt_status refresh_energies(pt_ctx *c)
{
    for (const auto &k : c->classes) {
        pt_status st = sweep_class(c, k, {kEnergyOnly});
        if (st != PT_OK) return st;
    }
    return PT_OK;
}

// Chains per workgroup: enough workgroups to cover the chip several times,
// as many chains as possible sharing one coupling load.
int choose_group(int H, int C, int n_samples)
{
    const int blocks = (H + kSweepBlock - 1) / kSweepBlock * n_samples;
    int G = std::min(C, kMaxGroup);
    while (G > 1 && static_cast<int64_t>(blocks) * ((C + G - 1) / G) < 2048) G = (G + 1) / 2;
    return G;
}

void pack_couplings(int L, const float *M, float *out)
{
    // out[colour][54][H]; see kernels.hpp.  M is [3][N][3][3].
    const int N = L * L * L, H = N / 2, Lh = L / 2;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                const int i = x + L * (y + L * z);
                const int col = (x + y + z) & 1;
                const int p = (x >> 1) + Lh * (y + L * z);
                const int back[3] = {((x + L - 1) % L) + L * (y + L * z),
                                     x + L * (((y + L - 1) % L) + L * z),
                                     x + L * (y + L * ((z + L - 1) % L))};
                float *o = out + static_cast<int64_t>(col) * 54 * H + p;
                for (int mu = 0; mu < 3; ++mu) {
                    const float *fw = M + (static_cast<int64_t>(mu) * N + i) * 9;
                    const float *bw = M + (static_cast<int64_t>(mu) * N + back[mu]) * 9;
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) {
                            o[static_cast<int64_t>((2 * mu) * 9 + a * 3 + b) * H] = fw[a * 3 + b];
                            o[static_cast<int64_t>((2 * mu + 1) * 9 + a * 3 + b) * H] = bw[b * 3 + a];
                        }
                }
            }
}

// Per-site packed couplings for the chain-lane mapping: out[colour][H][54],
// the same 54 numbers per site as pack_couplings, site by site.
void pack_couplings_site(int L, const float *M, float *out)
{
    const int N = L * L * L, H = N / 2;
    std::vector<float> soa(static_cast<size_t>(54) * N);
    pack_couplings(L, M, soa.data());
    for (int c = 0; c < 2; ++c)
        for (int p = 0; p < H; ++p)
            for (int q = 0; q < 54; ++q)
                out[(static_cast<int64_t>(c) * H + p) * 54 + q] = soa[(static_cast<int64_t>(c) * 54 + q) * H + p];
}

uint64_t fnv1a(const void *data, size_t n)
{
    const unsigned char *p = static_cast<const unsigned char *>(data);
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Bond codes of a bimodal sample for the site-lane and chain-lane kernels: out[colour][H][8],
// byte n of a site = code of its matrix A_n (n = 0..5: forward and backward
// bond along x, y, z; the family is symmetric, so A_{2mu+1} = M_{mu,x-e_mu}
// has the code of that bond), bytes 6 and 7 zero.
void pack_bond_codes(int L, const float *M, float D, uint8_t *out)
{
    const int N = L * L * L, H = N / 2, Lh = L / 2;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                const int i = x + L * (y + L * z);
                const int col = (x + y + z) & 1;
                const int p = (x >> 1) + Lh * (y + L * z);
                const int back[3] = {((x + L - 1) % L) + L * (y + L * z), x + L * (((y + L - 1) % L) + L * z),
                                     x + L * (y + L * ((z + L - 1) % L))};
                uint8_t *o = out + (static_cast<int64_t>(col) * H + p) * 8;
                for (int mu = 0; mu < 3; ++mu) {
                    o[2 * mu] = static_cast<uint8_t>(bimodal_code(M + (static_cast<int64_t>(mu) * N + i) * 9, D));
                    o[2 * mu + 1] =
                        static_cast<uint8_t>(bimodal_code(M + (static_cast<int64_t>(mu) * N + back[mu]) * 9, D));
                }
            }
}

pt_status check_ctx(pt_ctx *c)
{
    if (!c) return fail(PT_ESTATE, "context is NULL (call pt_init first)");
    PT_HIP(hipSetDevice(c->device));
    return PT_OK;
}

// Plan cache on disk.  The file that PTSG_PLAN_CACHE names holds one tuned
// plan per line:
//   ptsg-plan <version> <arch> <CUs> <L> <n_temps> <n_replicas> <samples timed>
//             <graphs 0|1> <bimodal 0|1> <site|chain|resident> <G> <split> <strip>
// Lines that do not parse, carry another version, or name a mapping the
// lattice cannot use are skipped; the last matching line wins.  The version
// changes whenever the kernels or the tuned parameters change enough to move
// the choice.
constexpr int kPlanVersion = 2;

struct PlanKey {
    std::string arch;
    int cus = 0, L = 0, T = 0, R = 0, n = 0, graphs = 0, bimodal = 0;
    std::string text() const
    {
        std::ostringstream o;
        o << "ptsg-plan " << kPlanVersion << ' ' << arch << ' ' << cus << ' ' << L << ' ' << T << ' ' << R << ' '
          << n << ' ' << graphs << ' ' << bimodal;
        return o.str();
    }
};

const char *const kMappingName[3] = {"site", "chain", "resident"};

bool mapping_fits(int m, int L)
{
    return m == kSiteLanes || (m == kChainLanes && L <= 128) || (m == kResident && L <= kRsMaxL);
}

bool plan_cache_lookup(const PlanKey &k, Tile &out)
{
    const char *path = std::getenv("PTSG_PLAN_CACHE");
    if (!path || !*path) return false;
    std::ifstream in(path);
    const std::string want = k.text() + ' ';
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {
        if (line.compare(0, want.size(), want) != 0) continue;
        std::istringstream rest(line.substr(want.size()));
        std::string name, extra;
        Tile t;
        if (!(rest >> name >> t.G >> t.split >> t.strip) || (rest >> extra)) continue;
        for (int m = 0; m < 3; ++m)
            if (name == kMappingName[m] && mapping_fits(m, k.L) && t.G >= 0 && t.G <= kMaxGroup && t.split >= 0 &&
                t.split <= 8 && t.strip >= -1 && t.strip <= k.L) {
                t.mapping = m;
                out = t;
                found = true;
            }
    }
    return found;
}

// Appends one line; a file that cannot be written leaves the tuning result
// in the process cache only.
void plan_cache_store(const PlanKey &k, const Tile &t)
{
    const char *path = std::getenv("PTSG_PLAN_CACHE");
    if (!path || !*path) return;
    const std::string line = k.text() + ' ' + kMappingName[t.mapping] + ' ' + std::to_string(t.G) + ' ' +
                             std::to_string(t.split) + ' ' + std::to_string(t.strip) + '\n';
    if (FILE *f = std::fopen(path, "a")) {
        std::fwrite(line.data(), 1, line.size(), f);
        std::fclose(f);
    }
}

}  // namespace

extern "C" {

const char *pt_last_error(void) { return g_err.c_str(); }

static pt_status init_batch(pt_ctx **out, const pt_batch_desc *d, const std::vector<Tile> *forced);
static pt_status autotuned_tiles(const pt_batch_desc *d, std::vector<Tile> &tiles);

// The autotuner runs only when no mapping is forced by a flag.
static bool wants_autotune(const pt_batch_desc *d)
{
    const unsigned forced = PT_F_SITE_LANES | PT_F_CHAIN_LANES | PT_F_RESIDENT | PT_F_PLAIN | PT_F_ROW_OR |
                            PT_F_PERSISTENT;
    return (d->flags & PT_F_AUTOTUNE) && !(d->flags & forced);
}

size_t pt_workspace_size(const pt_batch_desc *desc)
{
    const std::string why = validate(desc);
    if (!why.empty()) {
        fail(PT_EINVAL, why);
        return 0;
    }
    if (wants_autotune(desc)) {
        std::vector<Tile> tiles;
        if (autotuned_tiles(desc, tiles) != PT_OK) return 0;
        return make_plan(desc, &tiles).bytes;
    }
    return make_plan(desc).bytes;
}

pt_status pt_init_batch(pt_ctx **out, const pt_batch_desc *d)
{
    if (!out) return fail(PT_EINVAL, "ctx output pointer is NULL");
    *out = nullptr;
    const std::string why = validate(d);
    if (!why.empty()) return fail(PT_EINVAL, why);
    if (wants_autotune(d)) {
        std::vector<Tile> tiles;
        pt_status st = autotuned_tiles(d, tiles);
        if (st != PT_OK) return st;
        return init_batch(out, d, &tiles);
    }
    return init_batch(out, d, nullptr);
}

static pt_status init_batch(pt_ctx **out, const pt_batch_desc *d, const std::vector<Tile> *forced)
{
    *out = nullptr;
    const std::string why = validate(d);
    if (!why.empty()) return fail(PT_EINVAL, why);
    for (int s = 0; s < d->n_samples; ++s) {
        const int64_t n = 27ll * d->L[s] * d->L[s] * d->L[s];
        for (int64_t q = 0; q < n; ++q)
            if (!std::isfinite(d->couplings[s][q]))
                return fail(PT_EINVAL, "sample " + std::to_string(s) + ": non-finite coupling");
    }
    pt_ctx *c = new (std::nothrow) pt_ctx();
    if (!c) return fail(PT_ENOMEM, "host allocation failed");
    struct Guard {
        pt_ctx *&c;
        ~Guard() { if (c) pt_free(c); }
    } guard{c};

    if (hipGetDevice(&c->device) != hipSuccess) return fail(PT_EDEVICE, "no HIP device");
    {
        double *unused = nullptr;
        pt_status st_scratch = scratch_on(c->device, &unused);
        if (st_scratch != PT_OK) return st_scratch;
    }
    c->stream = static_cast<hipStream_t>(d->stream);
    c->seed = d->seed;
    c->plan = make_plan(d, forced);
    Plan &P = c->plan;
    if (d->workspace) {
        if (d->workspace_bytes < P.bytes)
            return fail(PT_ENOMEM, "workspace of " + std::to_string(d->workspace_bytes) +
                                       " bytes is smaller than the " + std::to_string(P.bytes) +
                                       " required");
        if (reinterpret_cast<uintptr_t>(d->workspace) % kAlign)
            return fail(PT_EINVAL, "workspace must be 256-byte aligned");
        c->ws = static_cast<char *>(d->workspace);
    } else {
        void *w = nullptr;
        if (hipMalloc(&w, P.bytes) != hipSuccess)
            return fail(PT_ENOMEM, "hipMalloc of " + std::to_string(P.bytes) + " bytes failed");
        c->ws = static_cast<char *>(w);
        c->own_ws = true;
    }
    char *w = c->ws;
    c->spins = reinterpret_cast<float *>(w + P.off_spins);
    c->cpls = reinterpret_cast<float *>(w + P.off_cpls);
    c->cpl6 = reinterpret_cast<float *>(w + P.off_cpl6);
    c->slot_of = reinterpret_cast<int *>(w + P.off_slot);
    c->beta_of = reinterpret_cast<float *>(w + P.off_beta_of);
    c->E = reinterpret_cast<double *>(w + P.off_E);
    c->perm = reinterpret_cast<int *>(w + P.off_perm);
    c->betas = reinterpret_cast<double *>(w + P.off_betas);
    c->epart = reinterpret_cast<double *>(w + P.off_epart);
    c->twid = reinterpret_cast<double *>(w + P.off_twid);
    c->rec = reinterpret_cast<int *>(w + P.off_rec);
    c->mpart = reinterpret_cast<double *>(w + P.off_mpart);
    c->meas = reinterpret_cast<pt_meas *>(w + P.off_meas);
    c->stage = reinterpret_cast<float *>(w + P.off_stage);
    c->counters = reinterpret_cast<uint32_t *>(w + P.off_counters);
    c->bm_D = reinterpret_cast<float *>(w + P.off_bmD);
    c->bm_table = reinterpret_cast<float *>(w + P.off_bmtab);
    c->cursor = reinterpret_cast<RecordCursor *>(w + P.off_cursor);
    c->use_graphs = (d->flags & PT_F_GRAPHS) != 0;
    c->row_or = (d->flags & PT_F_ROW_OR) != 0;
    c->persistent = (d->flags & PT_F_PERSISTENT) != 0;
    {
        const uint32_t zero[2] = {0u, 0u};
        PT_HIP(hipMemcpy(c->counters, zero, sizeof(zero), hipMemcpyHostToDevice));
    }
    {
        char *m = w + P.off_meta;
        c->d_spin_base = reinterpret_cast<int64_t *>(m);
        c->d_cpls_base = c->d_spin_base + P.S;
        c->d_cpl6_base = c->d_spin_base + 2 * P.S;
        int *ip = reinterpret_cast<int *>(c->d_spin_base + 3 * P.S);
        c->d_L = ip;
        c->d_T = ip + P.S;
        c->d_chain_base = ip + 2 * P.S;
        c->d_perm_base = ip + 3 * P.S;
        c->d_beta_base = ip + 4 * P.S;
        c->d_twid_base = ip + 5 * P.S;
        c->d_lanes = ip + 6 * P.S;
    }
    hipStream_t st = c->stream;
    // per-sample tables
    {
        std::vector<char> meta(3 * sizeof(int64_t) * P.S + 7 * sizeof(int) * P.S);
        int64_t *lp = reinterpret_cast<int64_t *>(meta.data());
        std::copy(P.spin_base.begin(), P.spin_base.end(), lp);
        std::copy(P.cpls_base.begin(), P.cpls_base.end(), lp + P.S);
        std::copy(P.cpl6_base.begin(), P.cpl6_base.end(), lp + 2 * P.S);
        int *ip = reinterpret_cast<int *>(lp + 3 * P.S);
        std::copy(P.L.begin(), P.L.end(), ip);
        std::copy(P.T.begin(), P.T.end(), ip + P.S);
        std::copy(P.chain_base.begin(), P.chain_base.end(), ip + 2 * P.S);
        std::copy(P.perm_base.begin(), P.perm_base.end(), ip + 3 * P.S);
        std::copy(P.beta_base.begin(), P.beta_base.end(), ip + 4 * P.S);
        std::copy(P.twid_base.begin(), P.twid_base.end(), ip + 5 * P.S);
        std::copy(P.lanes.begin(), P.lanes.end(), ip + 6 * P.S);
        PT_HIP(hipMemcpy(w + P.off_meta, meta.data(), meta.size(), hipMemcpyHostToDevice));
    }
    // temperatures, permutation, slots, twiddles, measurement records
    {
        std::vector<double> betas, twid;
        std::vector<int> perm, slot;
        std::vector<float> beta_of;
        std::vector<int> rec;
        for (int s = 0; s < P.S; ++s) {
            const int T = P.T[s], L = P.L[s];
            for (int k = 0; k < T; ++k) betas.push_back(1.0 / d->temps[s][k]);
            c->cpl_hash.push_back(fnv1a(d->couplings[s], sizeof(float) * 27 * static_cast<size_t>(L) * L * L));
            for (int r = 0; r < P.R; ++r)
                for (int j = 0; j < T; ++j) {
                    perm.push_back(j);
                    slot.push_back(j);
                    beta_of.push_back(static_cast<float>(1.0 / d->temps[s][j]));
                }
            const double two_pi = 6.283185307179586476925286766559;
            for (int n = 0; n < L; ++n) twid.push_back(std::cos(two_pi * n / L));
            for (int n = 0; n < L; ++n) twid.push_back(std::sin(two_pi * n / L));
            for (int k = 0; k < T; ++k)
                for (int a = 0; a < P.R; ++a)
                    for (int b = a + 1; b < P.R; ++b) {
                        rec.push_back(s);
                        rec.push_back(k);
                        rec.push_back(a);
                        rec.push_back(b);
                    }
        }
        PT_HIP(hipMemcpy(c->betas, betas.data(), betas.size() * sizeof(double), hipMemcpyHostToDevice));
        c->betas_host = betas;
        PT_HIP(hipMemcpy(c->perm, perm.data(), perm.size() * sizeof(int), hipMemcpyHostToDevice));
        PT_HIP(hipMemcpy(c->slot_of, slot.data(), slot.size() * sizeof(int), hipMemcpyHostToDevice));
        PT_HIP(hipMemcpy(c->beta_of, beta_of.data(), beta_of.size() * sizeof(float), hipMemcpyHostToDevice));
        PT_HIP(hipMemcpy(c->twid, twid.data(), twid.size() * sizeof(double), hipMemcpyHostToDevice));
        if (!rec.empty())
            PT_HIP(hipMemcpy(c->rec, rec.data(), rec.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    // couplings: site-major copy for every sample, the packed six-matrix
    // form for site-lane samples
    {
        std::vector<float> buf;
        for (int s = 0; s < P.S; ++s) {
            const int L = P.L[s];
            const int64_t N = static_cast<int64_t>(L) * L * L;
            buf.resize(static_cast<size_t>(27 * N));
            for (int64_t i = 0; i < N; ++i)
                for (int mu = 0; mu < 3; ++mu)
                    std::memcpy(&buf[(i * 3 + mu) * 9], d->couplings[s] + (mu * N + i) * 9, 9 * sizeof(float));
            PT_HIP(hipMemcpy(c->cpls + P.cpls_base[s], buf.data(), buf.size() * sizeof(float),
                             hipMemcpyHostToDevice));
            if (P.codes[s]) {
                const float D = bimodal_D(L, d->couplings[s]);
                std::vector<uint8_t> codes(8 * static_cast<size_t>(N), 0);
                pack_bond_codes(L, d->couplings[s], D, codes.data());
                PT_HIP(hipMemcpy(c->cpl6 + P.cpl6_base[s], codes.data(), codes.size(), hipMemcpyHostToDevice));
                PT_HIP(hipMemcpy(c->bm_D + s, &D, sizeof(float), hipMemcpyHostToDevice));
                std::vector<float> table(128 * 9);
                for (unsigned code = 0; code < 128; ++code) bimodal_matrix(code, D, &table[9 * code]);
                PT_HIP(hipMemcpy(c->bm_table + static_cast<size_t>(s) * 128 * 9, table.data(),
                                 table.size() * sizeof(float), hipMemcpyHostToDevice));
                continue;
            }
            buf.assign(static_cast<size_t>(54 * N), 0.0f);
            if (P.lanes[s] == 1)
                pack_couplings(L, d->couplings[s], buf.data());
            else
                pack_couplings_site(L, d->couplings[s], buf.data());
            PT_HIP(hipMemcpy(c->cpl6 + P.cpl6_base[s], buf.data(), buf.size() * sizeof(float),
                             hipMemcpyHostToDevice));
        }
    }
    // lattice classes (same L, T and mapping), swept by the same launches
    {
        std::map<std::tuple<int, int, int>, std::vector<int>> groups;
        for (int s = 0; s < P.S; ++s) groups[{P.L[s], P.T[s], P.mapping[s]}].push_back(s);
        int *dsamp = reinterpret_cast<int *>(w + P.off_classes);
        int *ditems = reinterpret_cast<int *>(w + P.off_items);
        int at = 0, at_items = 0;
        for (auto &g : groups) {
            LatticeClass k;
            k.L = std::get<0>(g.first);
            k.T = std::get<1>(g.first);
            k.mapping = std::get<2>(g.first);
            k.lanes = k.mapping == kChainLanes ? 64 : 1;
            k.C = P.R * k.T;
            const int H = k.L * k.L * k.L / 2;
            k.samples = g.second;
            k.d_samples = dsamp + at;
            PT_HIP(hipMemcpy(k.d_samples, g.second.data(), g.second.size() * sizeof(int),
                             hipMemcpyHostToDevice));
            at += static_cast<int>(g.second.size());
            if (k.mapping == kResident) {
                k.blocks = 1;
            } else if (k.mapping == kSiteLanes) {
                k.blocks = (H + kSweepBlock - 1) / kSweepBlock;
                const int ns = static_cast<int>(g.second.size());
                // the plain single-chain form stays one launch over every sample
                k.batch = (d->flags & PT_F_PLAIN) ? ns : site_batch(k.L, k.C, P.codes[g.second[0]], ns);
                k.G = (d->flags & PT_F_PLAIN) ? 1 : choose_group(H, k.C, k.batch);
                if (forced && (*forced)[g.second[0]].G > 0) k.G = std::min((*forced)[g.second[0]].G, k.C);
            } else {
                for (int s : g.second)
                    for (int grp = 0; grp < (k.C + 63) / 64; ++grp) {
                        k.items.push_back(s);
                        k.items.push_back(grp);
                    }
                const int n_items = static_cast<int>(k.items.size() / 2);
                k.batch = cl_batch(k.L, n_items);
                k.split = choose_split(k.L, k.batch);
                k.strip = choose_strip(k.L);
                if (forced) {
                    const Tile &t = (*forced)[g.second[0]];
                    if (t.split > 0 && (k.L / 2) % t.split == 0 && (k.L / 2) / t.split >= 2) k.split = t.split;
                    if (t.strip == 0 || (t.strip > 0 && k.L % t.strip == 0)) k.strip = t.strip;
                }
                k.blocks = cl_blocks(k.L, k.split);
                k.d_items = ditems + 2 * at_items;
                PT_HIP(hipMemcpy(k.d_items, k.items.data(), k.items.size() * sizeof(int),
                                 hipMemcpyHostToDevice));
                at_items += n_items;
            }
            c->classes.push_back(k);
        }
    }
    // hot start, then energies
    for (int s = 0; s < P.S; ++s)
        PT_HIP(launch_init_spins(c->spins, P.spin_base[s], P.lanes[s], P.L[s], P.R * P.T[s], P.T[s], s,
                                 static_cast<uint32_t>(c->seed),
                                 static_cast<uint32_t>(c->seed >> 32), st));
    {
        pt_status e = refresh_energies(c);
        if (e != PT_OK) return e;
    }
    PT_HIP(hipStreamSynchronize(st));
    *out = c;
    c = nullptr;  // disarm the guard
    return PT_OK;
}

// Autotuner: for each distinct (L, n_temps) of the batch, on a temporary
// context holding a representative share of those samples (enough for 4096
// chains, at least 4, at most 2 GB of spins), time a step of one heat-bath
// and min(L, 32) overrelaxation sweeps (best of two, after a warm-up step)
// of every applicable mapping with its heuristic tile shape, then of the
// fastest mapping with neighbouring tile shapes: site lanes with half and
// twice the chains per workgroup, chain lanes with half and twice the waves
// per packed row and the y-strips half and twice as tall.  The fastest plan
// is kept.  The step is long enough for the chain-lane order to pay for its
// first, cold pass through the cache.  Bimodal samples are timed in their
// byte coding.  Results are cached per (device, L, n_temps, n_replicas,
// samples timed, graphs, bimodal) for the process, and in the file
// PTSG_PLAN_CACHE names when it is set.
static pt_status autotuned_tiles(const pt_batch_desc *d, std::vector<Tile> &tiles)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int, bool, bool>, Tile> cache;
    const unsigned graphs = d->flags & PT_F_GRAPHS;
    const unsigned bimodal = d->flags & PT_F_BIMODAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(PT_EDEVICE, "no HIP device");
    hipDeviceProp_t prop{};
    PT_HIP(hipGetDeviceProperties(&prop, dev));
    std::string arch(prop.gcnArchName);
    std::replace(arch.begin(), arch.end(), ' ', '_');
    tiles.assign(d->n_samples, Tile{kSiteLanes, 0, 0, -1});
    std::map<std::pair<int, int>, std::vector<int>> classes;
    for (int s = 0; s < d->n_samples; ++s) classes[{d->L[s], d->n_temps[s]}].push_back(s);
    for (auto &cl : classes) {
        const int L = cl.first.first;
        // a representative batch: enough samples for >= 4096 chains (at least
        // 4), at most 2 GB of spins per candidate context
        const int64_t C = static_cast<int64_t>(d->n_replicas) * cl.first.second;
        const int64_t chain_bytes = 12 * static_cast<int64_t>(L) * L * L;
        int n = static_cast<int>(std::max<int64_t>(4, (4096 + C - 1) / C));
        while (n > 1 && n * C * chain_bytes > (2ll << 30)) --n;
        n = std::min<int>(n, static_cast<int>(cl.second.size()));
        const auto key = std::make_tuple(dev, L, cl.first.second, d->n_replicas, n, graphs != 0, bimodal != 0);
        const PlanKey pkey{arch, prop.multiProcessorCount, L, cl.first.second, d->n_replicas, n,
                           graphs != 0, bimodal != 0};
        Tile best;
        bool have = false;
        {
            std::lock_guard<std::mutex> lock(mu);
            auto it = cache.find(key);
            if (it != cache.end()) {
                best = it->second;
                have = true;
            } else if (plan_cache_lookup(pkey, best)) {
                cache[key] = best;
                have = true;
            }
        }
        if (!have) {
            std::vector<int> Ls(n, L), Ts(n, cl.first.second);
            std::vector<const double *> temps;
            std::vector<const float *> cpl;
            for (int q = 0; q < n; ++q) {
                temps.push_back(d->temps[cl.second[q]]);
                cpl.push_back(d->couplings[cl.second[q]]);
            }
            // time one plan; `used` receives the tile shape the context ran
            auto time_plan = [&](const Tile &plan, float &ms_out, Tile &used) -> pt_status {
                pt_batch_desc t{};
                t.n_samples = n;
                t.L = Ls.data();
                t.n_temps = Ts.data();
                t.temps = temps.data();
                t.couplings = cpl.data();
                t.n_replicas = d->n_replicas;
                t.seed = d->seed;
                t.flags = graphs | bimodal;
                const std::vector<Tile> forced(n, plan);
                pt_ctx *tc = nullptr;
                pt_status st = init_batch(&tc, &t, &forced);
                if (st != PT_OK) return st;
                const LatticeClass &k = tc->classes[0];
                used = Tile{k.mapping, k.mapping == kSiteLanes ? k.G : 0, k.mapping == kChainLanes ? k.split : 0,
                            k.mapping == kChainLanes ? k.strip : -1};
                hipEvent_t e0 = nullptr, e1 = nullptr;
                float ms = 0.0f, best_rep = 0.0f;
                hipError_t he = hipEventCreate(&e0);
                if (he == hipSuccess) he = hipEventCreate(&e1);
                const int n_or = std::min(L, 32);
                if (he == hipSuccess) st = pt_step(tc, 1, n_or);
                for (int rep = 0; rep < 2 && he == hipSuccess && st == PT_OK; ++rep) {
                    he = hipEventRecord(e0, tc->stream);
                    if (he == hipSuccess && (st = pt_step(tc, 1, n_or)) == PT_OK) {
                        he = hipEventRecord(e1, tc->stream);
                        if (he == hipSuccess) he = hipEventSynchronize(e1);
                        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
                        if (he == hipSuccess && (rep == 0 || ms < best_rep)) best_rep = ms;
                    }
                }
                if (e0) (void)hipEventDestroy(e0);
                if (e1) (void)hipEventDestroy(e1);
                pt_free(tc);
                if (st != PT_OK) return st;
                if (he != hipSuccess) return fail(PT_EDEVICE, std::string("autotune timing: ") + hipGetErrorString(he));
                ms_out = best_rep;
                return PT_OK;
            };
            double best_t = 0.0;
            std::vector<int> maps = {kSiteLanes};
            if (L <= 128) maps.push_back(kChainLanes);
            if (L <= kRsMaxL) maps.push_back(kResident);
            for (int m : maps) {
                float ms = 0.0f;
                Tile used;
                pt_status st = time_plan(Tile{m, 0, 0, -1}, ms, used);
                if (st != PT_OK) return st;
                if (!have || ms < best_t) {
                    best = used;
                    best_t = ms;
                    have = true;
                }
            }
            // neighbouring tile shapes of the fastest mapping
            std::vector<Tile> shapes;
            const int Cn = static_cast<int>(C);
            if (best.mapping == kSiteLanes) {
                for (int G : {best.G / 2, best.G * 2})
                    if (G >= 1 && G <= std::min(Cn, kMaxGroup) && G != best.G) shapes.push_back(Tile{kSiteLanes, G, 0, -1});
            } else if (best.mapping == kChainLanes) {
                const int Lh = L / 2;
                for (int sp : {best.split / 2, best.split * 2})
                    if (sp >= 1 && sp <= 8 && Lh % sp == 0 && Lh / sp >= 2)
                        shapes.push_back(Tile{kChainLanes, 0, sp, best.strip});
                for (int sr : {best.strip / 2, best.strip * 2})
                    if (best.strip > 0 && sr >= 2 && sr <= L && L % sr == 0 && sr != best.strip)
                        shapes.push_back(Tile{kChainLanes, 0, best.split, sr});
            }
            for (const Tile &shape : shapes) {
                float ms = 0.0f;
                Tile used;
                pt_status st = time_plan(shape, ms, used);
                if (st != PT_OK) return st;
                if (ms < best_t) {
                    best = used;
                    best_t = ms;
                }
            }
            std::lock_guard<std::mutex> lock(mu);
            cache[key] = best;
            plan_cache_store(pkey, best);
        }
        for (int s : cl.second) tiles[s] = best;
    }
    return PT_OK;
}

pt_status pt_get_tile(pt_ctx *c, int sample, int *chains_per_group, int *split, int *strip)
{
    if (!c) return fail(PT_ESTATE, "context is NULL (call pt_init first)");
    if (sample < 0 || sample >= c->plan.S) return fail(PT_EINVAL, "sample out of range");
    for (const auto &k : c->classes)
        if (std::find(k.samples.begin(), k.samples.end(), sample) != k.samples.end()) {
            if (chains_per_group) *chains_per_group = k.mapping == kSiteLanes ? k.G : k.mapping == kChainLanes ? 64 : 1;
            if (split) *split = k.mapping == kChainLanes ? k.split : 0;
            if (strip) *strip = k.mapping == kChainLanes ? k.strip : 0;
            return PT_OK;
        }
    return fail(PT_EINVAL, "sample has no class");
}

pt_status pt_get_mapping(pt_ctx *c, int sample, unsigned *flag)
{
    if (!c) return fail(PT_ESTATE, "context is NULL (call pt_init first)");
    if (sample < 0 || sample >= c->plan.S) return fail(PT_EINVAL, "sample out of range");
    if (!flag) return fail(PT_EINVAL, "output is NULL");
    const int m = c->plan.mapping[sample];
    *flag = m == kResident ? PT_F_RESIDENT : m == kChainLanes ? PT_F_CHAIN_LANES : PT_F_SITE_LANES;
    return PT_OK;
}

pt_status pt_init(pt_ctx **ctx, int L, const float *couplings, const double *temps, int n_temps,
                  int n_replicas, uint64_t seed)
{
    pt_batch_desc d{};
    d.n_samples = 1;
    d.L = &L;
    d.n_temps = &n_temps;
    d.temps = &temps;
    d.couplings = &couplings;
    d.n_replicas = n_replicas;
    d.seed = seed;
    return pt_init_batch(ctx, &d);
}

// Queue one step on `st`: every class's sweeps (n_or == PT_OR_L: L
// overrelaxation sweeps for a class of linear size L), then advance the
// device heat-bath counter.
static pt_status queue_step(pt_ctx *c, int n_hb, int n_or)
{
    pt_status st;
    for (const auto &k : c->classes) {
        std::vector<int> kinds(n_hb, kHeatbath);
        kinds.insert(kinds.end(), n_or == PT_OR_L ? k.L : n_or, kOverrelax);
        if ((st = sweep_class(c, k, kinds)) != PT_OK) return st;
    }
    if (n_hb > 0) PT_HIP(launch_advance_counters(c->counters, static_cast<uint32_t>(n_hb), 0u, c->stream));
    return PT_OK;
}

// Capture what `queue` enqueues on the context's stream as a graph, on a
// private default-priority stream, and instantiate it.  The random-number
// counters live in device memory and are advanced by kernels inside the
// work, so every replay draws fresh numbers; nothing captured is a memset.
extern "C++" template <class Queue>
static pt_status capture_graph(pt_ctx *c, Queue queue, hipGraphExec_t *out)
{
    if (!c->capture_stream) PT_HIP(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    const hipError_t eb = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal);
    if (eb != hipSuccess) return fail(PT_EDEVICE, std::string("stream capture: ") + hipGetErrorString(eb));
    hipStream_t user = c->stream;
    c->stream = c->capture_stream;
    const pt_status st = queue();
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(c->capture_stream, &graph);
    c->stream = user;
    if (st != PT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(PT_EDEVICE, std::string("stream capture: ") + hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(PT_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
    return PT_OK;
}

// PT_F_PERSISTENT: the step's descriptors, class by class, merged into
// phases: phase i holds the i-th descriptor of every class whose sequence
// is that long (classes share no data, and a descriptor depends at most on
// those before it in its own class).  The grid is what the device keeps
// resident, rounded down to whole XCD rounds (a multiple of 8, so that
// workgroup w and every virtual block it takes sit on the same XCD), and
// no larger than the widest phase.
static pt_status build_program(pt_ctx *c, int n_hb, int n_or, pt_ctx::Program &g)
{
    std::vector<std::vector<StepDesc>> seqs;
    size_t longest = 0;
    for (const auto &k : c->classes) {
        std::vector<int> kinds(n_hb, kHeatbath);
        kinds.insert(kinds.end(), n_or == PT_OR_L ? k.L : n_or, kOverrelax);
        seqs.push_back(class_sequence(c, k, kinds));
        longest = std::max(longest, seqs.back().size());
    }
    int64_t widest = 0;
    for (size_t ph = 0; ph < longest; ++ph) {
        g.first.push_back(static_cast<int>(g.desc.size()));
        int64_t blocks = 0;
        for (const auto &q : seqs)
            if (ph < q.size()) {
                g.desc.push_back(q[ph]);
                blocks += static_cast<int64_t>(q[ph].gx) * q[ph].gy * q[ph].gz;
            }
        if (blocks > (int64_t(1) << 30)) return fail(PT_EINVAL, "persistent step: a phase has too many workgroups");
        g.blocks.push_back(static_cast<int>(blocks));
        widest = std::max(widest, blocks);
    }
    const bool chain = c->classes[0].lanes != 1;   // one mapping serves the batch
    int cus = 0;
    PT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
    const int per_cu = chain ? cl_step_blocks_per_cu() : site_step_blocks_per_cu();
    const int cap = per_cu * cus / kXcds * kXcds;
    if (cap < kXcds) return fail(PT_EDEVICE, "persistent step: the kernel does not fit the device");
    g.grid = static_cast<int>(std::min<int64_t>(cap, (widest + kXcds - 1) / kXcds * kXcds));
    const size_t b_desc = align_up(sizeof(StepDesc) * g.desc.size());
    const size_t b_int = align_up(sizeof(int) * g.first.size());
    void *mem = nullptr;
    if (hipMalloc(&mem, b_desc + 2 * b_int) != hipSuccess)
        return fail(PT_ENOMEM, "hipMalloc of the persistent step program failed");
    g.mem = static_cast<char *>(mem);
    g.d_desc = reinterpret_cast<const StepDesc *>(g.mem);
    g.d_first = reinterpret_cast<const int *>(g.mem + b_desc);
    g.d_blocks = reinterpret_cast<const int *>(g.mem + b_desc + b_int);
    PT_HIP(hipMemcpy(g.mem, g.desc.data(), sizeof(StepDesc) * g.desc.size(), hipMemcpyHostToDevice));
    PT_HIP(hipMemcpy(g.mem + b_desc, g.first.data(), sizeof(int) * g.first.size(), hipMemcpyHostToDevice));
    PT_HIP(hipMemcpy(g.mem + b_desc + b_int, g.blocks.data(), sizeof(int) * g.blocks.size(),
                     hipMemcpyHostToDevice));
    return PT_OK;
}

// One persistent launch for the step (the heat-bath counter advances inside).
static pt_status persistent_step(pt_ctx *c, int n_hb, int n_or)
{
    pt_status st;
    auto it = c->programs.find({n_hb, n_or});
    if (it == c->programs.end()) {
        pt_ctx::Program g;
        if ((st = build_program(c, n_hb, n_or, g)) != PT_OK) {
            if (g.mem) (void)hipFree(g.mem);
            return st;
        }
        it = c->programs.emplace(std::make_pair(n_hb, n_or), std::move(g)).first;
    }
    const pt_ctx::Program &g = it->second;
    PersistParams p{};
    p.desc = g.d_desc;
    p.phase_first = g.d_first;
    p.phase_blocks = g.d_blocks;
    p.n_phases = static_cast<int>(g.first.size());
    p.counters = c->counters;
    p.d_hb = static_cast<uint32_t>(n_hb);
    Event ev;
    if (c->profiling) {
        if (c->pending.size() >= 4096 && (st = drain_events(c)) != PT_OK) return st;
        if ((st = get_event(c, ev)) != PT_OK) return st;
        PT_HIP(hipEventRecord(ev.a, c->stream));
    }
    PT_HIP(c->classes[0].lanes != 1 ? launch_cl_step(p, g.grid, c->stream) : launch_site_step(p, g.grid, c->stream));
    if (c->profiling) {
        PT_HIP(hipEventRecord(ev.b, c->stream));
        c->pending.push_back({PT_K_PERSISTENT, ev});
    }
    return PT_OK;
}

pt_status pt_step(pt_ctx *c, int n_hb, int n_or)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (n_hb < 0 || (n_or < 0 && n_or != PT_OR_L))
        return fail(PT_EINVAL, "n_hb must be >= 0 and n_or >= 0 or PT_OR_L");
    if (n_hb == 0 && n_or == 0) return PT_OK;
    if (c->persistent) {
        if ((st = persistent_step(c, n_hb, n_or)) != PT_OK) return st;
    } else if (!c->use_graphs || c->profiling) {
        if ((st = queue_step(c, n_hb, n_or)) != PT_OK) return st;
    } else {
        // A step's launch sequence depends only on (n_hb, n_or): capture it
        // once on a private stream, then replay it on the context's stream.
        auto it = c->step_graphs.find({n_hb, n_or});
        if (it == c->step_graphs.end()) {
            hipGraphExec_t exec = nullptr;
            if ((st = capture_graph(c, [&] { return queue_step(c, n_hb, n_or); }, &exec)) != PT_OK) return st;
            it = c->step_graphs.emplace(std::make_pair(n_hb, n_or), exec).first;
        }
        PT_HIP(hipGraphLaunch(it->second, c->stream));
    }
    c->hb_sweeps += n_hb;
    return PT_OK;
}

// Queue one tempering pass (its kernel advances the pass counter).
static pt_status queue_swap(pt_ctx *c)
{
    SwapParams p{};
    p.perm = c->perm;
    p.slot_of = c->slot_of;
    p.beta_of = c->beta_of;
    p.E = c->E;
    p.betas = c->betas;
    p.chain_base = c->d_chain_base;
    p.perm_base = c->d_perm_base;
    p.beta_base = c->d_beta_base;
    p.n_temps = c->d_T;
    p.n_samples = c->plan.S;
    p.R = c->plan.R;
    p.counters = c->counters;
    p.key0 = static_cast<uint32_t>(c->seed);
    p.key1 = static_cast<uint32_t>(c->seed >> 32);
    PT_HIP(launch_swap(p, c->stream));   // also advances the pass counter
    return PT_OK;
}

pt_status pt_swap(pt_ctx *c)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if ((st = queue_swap(c)) != PT_OK) return st;
    c->pt_passes += 1;
    return PT_OK;
}

// Queue the record kernels of every record into the context's device
// records (c->meas); no copy, no wait.
static pt_status queue_measure(pt_ctx *c, unsigned what, bool to_cursor = false)
{
    const Plan &P = c->plan;
    MeasParams m{};
    m.cursor = to_cursor ? c->cursor : nullptr;
    m.spins = c->spins;
    m.cpls = c->cpls;
    m.rec = c->rec;
    m.perm = c->perm;
    m.perm_base = c->d_perm_base;
    m.n_temps = c->d_T;
    m.L = c->d_L;
    m.chain_base = c->d_chain_base;
    m.twid_base = c->d_twid_base;
    m.spin_base = c->d_spin_base;
    m.cpls_base = c->d_cpls_base;
    m.lanes = c->d_lanes;
    m.twid = c->twid;
    m.E = c->E;
    m.betas = c->betas;
    m.beta_base = c->d_beta_base;
    m.part = c->mpart;
    m.Lmax = P.Lmax;
    m.n_records = P.n_records;
    m.what = what;
    m.out = c->meas;
    m.stage = c->stage;
    m.stage_sample = -1;
    // Records are ordered by sample.  Runs of site-lane samples are measured
    // in place; a chain-lane sample is first copied to the site-lane layout
    // (its lanes interleave 64 chains, which the per-site record kernels
    // would read one float per cache line).
    {
        int first = 0, run_start = 0, run_L = 0;
        auto flush = [&](int end) -> hipError_t {
            if (end <= run_start) return hipSuccess;
            MeasParams q = m;
            q.rec0 = run_start;
            return launch_measure_records(q, end - run_start, run_L, P.R, c->stream);
        };
        for (int s = 0; s < P.S; ++s) {
            const int n = P.T[s] * P.R * (P.R - 1) / 2;
            if (P.lanes[s] != 1 && (what & (PT_M_OVERLAP | PT_M_CHIRAL | PT_M_SD))) {
                PT_HIP(flush(first));
                const int L = P.L[s];
                PT_HIP(launch_cl_to_sl(c->spins, P.spin_base[s], L * L * L / 2, P.R * P.T[s], c->stage,
                                       c->stream));
                MeasParams q = m;
                q.stage_sample = s;
                q.rec0 = first;
                PT_HIP(launch_measure_records(q, n, L, P.R, c->stream));
                run_start = first + n;
                run_L = 0;
            } else {
                run_L = std::max(run_L, P.L[s]);
            }
            first += n;
        }
        PT_HIP(flush(first));
        PT_HIP(launch_measure_finalize(m, c->stream));
    }
    if (to_cursor) PT_HIP(launch_advance_cursor(c->cursor, c->stream));
    return PT_OK;
}

pt_status pt_measure(pt_ctx *c, unsigned what, pt_meas *out, size_t cap, size_t *n_out)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (what & ~static_cast<unsigned>(PT_M_ALL)) return fail(PT_EINVAL, "unknown measurement bits");
    const Plan &P = c->plan;
    if ((what & (PT_M_OVERLAP | PT_M_CHIRAL)) && P.R < 2)
        return fail(PT_ESTATE, "overlap and chirality need n_replicas >= 2");
    if (n_out) *n_out = static_cast<size_t>(P.n_records);
    if (P.n_records == 0) return PT_OK;
    if (!out && cap == 0) return PT_OK;   // size query
    if (!out) return fail(PT_EINVAL, "output buffer is NULL");
    if (cap < static_cast<size_t>(P.n_records))
        return fail(PT_ENOMEM, "output holds " + std::to_string(cap) + " records, " +
                                   std::to_string(P.n_records) + " needed");
    if ((st = queue_measure(c, what)) != PT_OK) return st;
    PT_HIP(hipMemcpyAsync(out, c->meas, sizeof(pt_meas) * P.n_records, hipMemcpyDeviceToHost,
                          c->stream));
    PT_HIP(hipStreamSynchronize(c->stream));
    return PT_OK;
}

// pt_measure's records written to a device buffer, with the plane partials
// in the fixed `scratch` array (records in chunks that fit it) and
// chain-lane samples staged in the context's own workspace: nothing is
// allocated, nothing is copied to the host, nothing waits.
pt_status pt_measure_noalloc(pt_ctx *c, unsigned what, pt_meas *d_out, size_t cap)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (what & ~static_cast<unsigned>(PT_M_ALL)) return fail(PT_EINVAL, "unknown measurement bits");
    const Plan &P = c->plan;
    if ((what & (PT_M_OVERLAP | PT_M_CHIRAL)) && P.R < 2)
        return fail(PT_ESTATE, "overlap and chirality need n_replicas >= 2");
    if (P.n_records == 0) return PT_OK;
    if (!d_out) return fail(PT_EINVAL, "output buffer is NULL");
    if (cap < static_cast<size_t>(P.n_records))
        return fail(PT_ENOMEM, "output holds " + std::to_string(cap) + " records, " +
                                   std::to_string(P.n_records) + " needed");
    const size_t per_record = static_cast<size_t>(P.Lmax) * kPlaneQ;
    if (per_record > kScratchDoubles)
        return fail(PT_EUNSUPPORTED, "one record's partials (" + std::to_string(per_record * 8) +
                                         " bytes) exceed the fixed scratch of " +
                                         std::to_string(kScratchDoubles * 8) + " bytes");
    double *part = nullptr;
    if ((st = scratch_on(c->device, &part)) != PT_OK) return st;
    // whole temperature slots per chunk (the R(R-1)/2 records of a slot are
    // measured together), as many as the scratch array holds
    const int np = P.R * (P.R - 1) / 2;
    int chunk = static_cast<int>(std::min<size_t>(kScratchDoubles / per_record, P.n_records));
    if (chunk >= np) chunk -= chunk % np;
    MeasParams m{};
    m.spins = c->spins;
    m.cpls = c->cpls;
    m.rec = c->rec;
    m.perm = c->perm;
    m.perm_base = c->d_perm_base;
    m.n_temps = c->d_T;
    m.L = c->d_L;
    m.chain_base = c->d_chain_base;
    m.twid_base = c->d_twid_base;
    m.spin_base = c->d_spin_base;
    m.cpls_base = c->d_cpls_base;
    m.lanes = c->d_lanes;
    m.twid = c->twid;
    m.E = c->E;
    m.betas = c->betas;
    m.beta_base = c->d_beta_base;
    m.part = part;
    m.Lmax = P.Lmax;
    m.what = what;
    m.out = d_out;
    m.stage = c->stage;
    // records [a, b) (lattices up to L), in chunks whose partials fit the
    // scratch array; `staged` names the chain-lane sample whose chains sit in
    // the context's staging buffer (-1: none)
    auto run_range = [&](int a, int b, int L, int staged) -> hipError_t {
        for (int r0 = a; r0 < b; r0 += chunk) {
            MeasParams q = m;
            q.stage_sample = staged;
            q.rec0 = r0;
            q.part_rec0 = r0;
            q.n_records = std::min(r0 + chunk, b);
            hipError_t e = launch_measure_records(q, q.n_records - r0, L, P.R, c->stream);
            if (e == hipSuccess) e = launch_measure_finalize(q, c->stream);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    // As in pt_measure: runs of site-lane samples in place; a chain-lane
    // sample (64 chains interleaved per site) first copied to the site-lane
    // layout in the context's staging buffer (part of its workspace: nothing
    // is allocated), so the record kernels read whole component rows.
    const bool planes = what & (PT_M_OVERLAP | PT_M_CHIRAL | PT_M_SD);
    int first = 0, run_start = 0, run_L = 0;
    for (int s = 0; s < P.S; ++s) {
        const int n = P.T[s] * P.R * (P.R - 1) / 2;
        if (P.lanes[s] != 1 && planes) {
            PT_HIP(run_range(run_start, first, run_L, -1));
            const int L = P.L[s];
            PT_HIP(launch_cl_to_sl(c->spins, P.spin_base[s], L * L * L / 2, P.R * P.T[s], c->stage, c->stream));
            PT_HIP(run_range(first, first + n, L, s));
            run_start = first + n;
            run_L = 0;
        } else {
            run_L = std::max(run_L, P.L[s]);
        }
        first += n;
    }
    PT_HIP(run_range(run_start, first, run_L, -1));
    return PT_OK;
}

pt_status pt_run(pt_ctx *c, int n_steps, int n_hb, int n_or, int every, unsigned what, pt_meas *d_out,
                 size_t cap)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (n_steps < 0 || every < 0) return fail(PT_EINVAL, "n_steps and every must be >= 0");
    if (n_hb < 0 || (n_or < 0 && n_or != PT_OR_L))
        return fail(PT_EINVAL, "n_hb must be >= 0 and n_or >= 0 or PT_OR_L");
    if (what & ~static_cast<unsigned>(PT_M_ALL)) return fail(PT_EINVAL, "unknown measurement bits");
    const Plan &P = c->plan;
    const int64_t n_meas = (every > 0 && P.n_records > 0) ? n_steps / every : 0;
    if (n_meas > 0) {
        if ((what & (PT_M_OVERLAP | PT_M_CHIRAL)) && P.R < 2)
            return fail(PT_ESTATE, "overlap and chirality need n_replicas >= 2");
        if (!d_out) return fail(PT_EINVAL, "output buffer is NULL");
        if (cap < static_cast<size_t>(n_meas) * P.n_records)
            return fail(PT_ENOMEM, "output holds " + std::to_string(cap) + " records, " +
                                       std::to_string(n_meas * P.n_records) + " needed");
    }
    const bool sweeps = n_hb > 0 || n_or != 0;
    // `n` Monte Carlo steps from step t0 on, each followed by a measurement
    // when it is a multiple of `every`; records go through the device cursor
    auto queue = [&](int t0, int n) -> pt_status {
        for (int t = t0; t < t0 + n; ++t) {
            pt_status q = PT_OK;
            if (sweeps) q = c->persistent ? persistent_step(c, n_hb, n_or) : queue_step(c, n_hb, n_or);
            if (q == PT_OK) q = queue_swap(c);
            if (q == PT_OK && n_meas > 0 && (t + 1) % every == 0) q = queue_measure(c, what, true);
            if (q != PT_OK) return q;
        }
        return PT_OK;
    };
    if (n_steps == 0) return PT_OK;
    if (n_meas > 0) PT_HIP(launch_set_cursor(c->cursor, d_out, static_cast<uint64_t>(P.n_records), c->stream));
    // the persistent step builds its work list on first use, and kernel
    // timing needs every launch on its own: both run the steps one by one
    const bool graphs = c->use_graphs && !c->profiling && !c->persistent;
    if (!graphs) {
        if ((st = queue(0, n_steps)) != PT_OK) return st;
    } else {
        // graphs of one step, without and with a measurement after it
        const unsigned mbits = n_meas > 0 ? what : ~0u;
        hipGraphExec_t *g = c->run_graphs[std::make_tuple(n_hb, n_or, mbits)].one;
        for (int t = 0; t < n_steps; ++t) {
            const int m = n_meas > 0 && (t + 1) % every == 0;
            if (!g[m] && (st = capture_graph(c, [&] { return queue(t, 1); }, &g[m])) != PT_OK) return st;
            PT_HIP(hipGraphLaunch(g[m], c->stream));
        }
    }
    c->hb_sweeps += static_cast<uint64_t>(n_hb) * n_steps;
    c->pt_passes += static_cast<uint64_t>(n_steps);
    return PT_OK;
}

static pt_status chain_of(pt_ctx *c, int sample, int rep, int tslot, int *chain_local)
{
    const Plan &P = c->plan;
    if (sample < 0 || sample >= P.S) return fail(PT_EINVAL, "sample out of range");
    if (rep < 0 || rep >= P.R) return fail(PT_EINVAL, "replica out of range");
    if (tslot < 0 || tslot >= P.T[sample]) return fail(PT_EINVAL, "slot out of range");
    int j = 0;
    PT_HIP(hipMemcpyAsync(&j, c->perm + P.perm_base[sample] + rep * P.T[sample] + tslot, sizeof(int),
                          hipMemcpyDeviceToHost, c->stream));
    PT_HIP(hipStreamSynchronize(c->stream));
    *chain_local = rep * P.T[sample] + j;
    return PT_OK;
}

pt_status pt_get_spins(pt_ctx *c, int sample, int rep, int tslot, float *out)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (!out) return fail(PT_EINVAL, "output is NULL");
    int j;
    if ((st = chain_of(c, sample, rep, tslot, &j)) != PT_OK) return st;
    const Plan &P = c->plan;
    const int L = P.L[sample];
    const size_t n = 3 * static_cast<size_t>(L) * L * L;
    PT_HIP(launch_chain_io(c->spins, P.spin_base[sample], P.lanes[sample], L, j, c->stage, true, c->stream));
    PT_HIP(hipMemcpyAsync(out, c->stage, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    PT_HIP(hipStreamSynchronize(c->stream));
    return PT_OK;
}

pt_status pt_set_spins(pt_ctx *c, int sample, int rep, int tslot, const float *in)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (!in) return fail(PT_EINVAL, "input is NULL");
    int j;
    if ((st = chain_of(c, sample, rep, tslot, &j)) != PT_OK) return st;
    const Plan &P = c->plan;
    const int L = P.L[sample];
    const size_t n = 3 * static_cast<size_t>(L) * L * L;
    PT_HIP(hipMemcpyAsync(c->stage, in, n * sizeof(float), hipMemcpyHostToDevice, c->stream));
    PT_HIP(launch_chain_io(c->spins, P.spin_base[sample], P.lanes[sample], L, j, c->stage, false, c->stream));
    if ((st = refresh_energies(c)) != PT_OK) return st;
    PT_HIP(hipStreamSynchronize(c->stream));
    return PT_OK;
}

pt_status pt_get_perm(pt_ctx *c, int sample, int rep, int32_t *out)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    const Plan &P = c->plan;
    if (!out) return fail(PT_EINVAL, "output is NULL");
    if (sample < 0 || sample >= P.S) return fail(PT_EINVAL, "sample out of range");
    if (rep < 0 || rep >= P.R) return fail(PT_EINVAL, "replica out of range");
    PT_HIP(hipMemcpyAsync(out, c->perm + P.perm_base[sample] + rep * P.T[sample], sizeof(int) * P.T[sample],
                          hipMemcpyDeviceToHost, c->stream));
    PT_HIP(hipStreamSynchronize(c->stream));
    return PT_OK;
}

pt_status pt_get_perms(pt_ctx *c, int32_t *out)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (!out) return fail(PT_EINVAL, "output is NULL");
    const Plan &P = c->plan;
    std::vector<int> perm(P.total_perm);
    PT_HIP(hipMemcpyAsync(perm.data(), c->perm, perm.size() * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    PT_HIP(hipStreamSynchronize(c->stream));
    size_t o = 0;
    for (int s = 0; s < P.S; ++s)
        for (int r = 0; r < P.R; ++r)
            for (int k = 0; k < P.T[s]; ++k) out[o++] = perm[P.perm_base[s] + r * P.T[s] + k];
    return PT_OK;
}

pt_status pt_get_energy(pt_ctx *c, double *out)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (!out) return fail(PT_EINVAL, "output is NULL");
    const Plan &P = c->plan;
    std::vector<double> E(P.n_chains);
    std::vector<int> perm(P.total_perm);
    PT_HIP(hipMemcpyAsync(E.data(), c->E, E.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    PT_HIP(hipMemcpyAsync(perm.data(), c->perm, perm.size() * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    PT_HIP(hipStreamSynchronize(c->stream));
    size_t o = 0;
    for (int s = 0; s < P.S; ++s)
        for (int r = 0; r < P.R; ++r)
            for (int k = 0; k < P.T[s]; ++k) {
                const int j = perm[P.perm_base[s] + r * P.T[s] + k];
                out[o++] = E[P.chain_base[s] + r * P.T[s] + j];
            }
    return PT_OK;
}

pt_status pt_get_counters(pt_ctx *c, uint64_t *hb, uint64_t *pt)
{
    if (!c) return fail(PT_ESTATE, "context is NULL (call pt_init first)");
    if (hb) *hb = c->hb_sweeps;
    if (pt) *pt = c->pt_passes;
    return PT_OK;
}

// Checkpoint blob: header, then per sample its shape and state.
//   "PTSGCKP1" | u32 version=1 | u32 S | u32 R | u32 0 | u64 seed | u64 hb | u64 pt
//   per sample: i32 L | i32 T | u64 coupling hash | f64 beta[T]
//   per sample: i32 perm[R][T] | f64 E[R*T] | f32 spins[R*T][N][3] (chain order)
//   u64 FNV-1a of everything before it
extern "C++" {
namespace {

constexpr char kCkpMagic[8] = {'P', 'T', 'S', 'G', 'C', 'K', 'P', '1'};

size_t checkpoint_bytes(const Plan &P)
{
    size_t n = 8 + 4 * 4 + 3 * 8;
    for (int s = 0; s < P.S; ++s) {
        const size_t T = P.T[s], C = static_cast<size_t>(P.R) * T;
        const size_t N = static_cast<size_t>(P.L[s]) * P.L[s] * P.L[s];
        n += 4 + 4 + 8 + 8 * T;
        n += 4 * C + 8 * C + 4 * 3 * N * C;
    }
    return n + 8;
}

struct Writer {
    unsigned char *p;
    template <class V> void put(const V &v) { std::memcpy(p, &v, sizeof(V)); p += sizeof(V); }
    void put(const void *src, size_t n) { std::memcpy(p, src, n); p += n; }
};

struct Reader {
    const unsigned char *p, *end;
    template <class V> bool get(V &v)
    {
        if (static_cast<size_t>(end - p) < sizeof(V)) return false;
        std::memcpy(&v, p, sizeof(V));
        p += sizeof(V);
        return true;
    }
};

}  // namespace
}  // extern "C++"

pt_status pt_save(pt_ctx *c, void *blob, size_t cap, size_t *n_bytes)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    const Plan &P = c->plan;
    const size_t need = checkpoint_bytes(P);
    if (n_bytes) *n_bytes = need;
    if (!blob) return PT_OK;
    if (cap < need) return fail(PT_EINVAL, "checkpoint buffer too small (" + std::to_string(need) + " bytes needed)");
    PT_HIP(hipStreamSynchronize(c->stream));
    Writer w{static_cast<unsigned char *>(blob)};
    w.put(kCkpMagic, 8);
    w.put(static_cast<uint32_t>(1));
    w.put(static_cast<uint32_t>(P.S));
    w.put(static_cast<uint32_t>(P.R));
    w.put(static_cast<uint32_t>(0));
    w.put(c->seed);
    w.put(c->hb_sweeps);
    w.put(c->pt_passes);
    for (int s = 0; s < P.S; ++s) {
        w.put(static_cast<int32_t>(P.L[s]));
        w.put(static_cast<int32_t>(P.T[s]));
        w.put(c->cpl_hash[s]);
        w.put(c->betas_host.data() + P.beta_base[s], sizeof(double) * P.T[s]);
    }
    for (int s = 0; s < P.S; ++s) {
        const int L = P.L[s], C = P.R * P.T[s];
        const size_t n = 3 * static_cast<size_t>(L) * L * L;
        PT_HIP(hipMemcpyAsync(w.p, c->perm + P.perm_base[s], sizeof(int) * C, hipMemcpyDeviceToHost, c->stream));
        w.p += sizeof(int) * C;
        PT_HIP(hipMemcpyAsync(w.p, c->E + P.chain_base[s], sizeof(double) * C, hipMemcpyDeviceToHost, c->stream));
        w.p += sizeof(double) * C;
        for (int j = 0; j < C; ++j) {
            PT_HIP(launch_chain_io(c->spins, P.spin_base[s], P.lanes[s], L, j, c->stage, true, c->stream));
            PT_HIP(hipMemcpyAsync(w.p, c->stage, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
            PT_HIP(hipStreamSynchronize(c->stream));
            w.p += n * sizeof(float);
        }
    }
    PT_HIP(hipStreamSynchronize(c->stream));
    const size_t body = static_cast<size_t>(w.p - static_cast<unsigned char *>(blob));
    w.put(fnv1a(blob, body));
    return PT_OK;
}

pt_status pt_load(pt_ctx *c, const void *blob, size_t n_bytes)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (!blob) return fail(PT_EINVAL, "checkpoint is NULL");
    const Plan &P = c->plan;
    const size_t need = checkpoint_bytes(P);
    if (n_bytes != need)
        return fail(PT_EINVAL, "checkpoint size " + std::to_string(n_bytes) + " does not match this context (" +
                                   std::to_string(need) + " bytes)");
    const unsigned char *b = static_cast<const unsigned char *>(blob);
    uint64_t sum = 0;
    std::memcpy(&sum, b + need - 8, 8);
    if (sum != fnv1a(b, need - 8)) return fail(PT_EINVAL, "checkpoint checksum mismatch (damaged blob)");
    Reader r{b, b + need - 8};
    char magic[8];
    for (char &ch : magic) r.get(ch);
    uint32_t version = 0, S = 0, R = 0, pad = 0;
    uint64_t seed = 0, hb = 0, pt = 0;
    r.get(version);
    r.get(S);
    r.get(R);
    r.get(pad);
    r.get(seed);
    r.get(hb);
    r.get(pt);
    if (std::memcmp(magic, kCkpMagic, 8) != 0 || version != 1) return fail(PT_EINVAL, "not a checkpoint of this library");
    if (static_cast<int>(S) != P.S || static_cast<int>(R) != P.R)
        return fail(PT_EINVAL, "checkpoint has another number of samples or replicas");
    if (seed != c->seed) return fail(PT_EINVAL, "checkpoint was made with another seed");
    for (int s = 0; s < P.S; ++s) {
        int32_t L = 0, T = 0;
        uint64_t h = 0;
        r.get(L);
        r.get(T);
        r.get(h);
        if (L != P.L[s] || T != P.T[s])
            return fail(PT_EINVAL, "checkpoint sample " + std::to_string(s) + " has another L or n_temps");
        if (h != c->cpl_hash[s])
            return fail(PT_EINVAL, "checkpoint sample " + std::to_string(s) + " has other couplings");
        for (int k = 0; k < T; ++k) {
            double beta = 0.0;
            r.get(beta);
            if (beta != c->betas_host[P.beta_base[s] + k])
                return fail(PT_EINVAL, "checkpoint sample " + std::to_string(s) + " has other temperatures");
        }
    }
    {
        // every permutation row must be a permutation of the slots
        const unsigned char *q = r.p;
        for (int s = 0; s < P.S; ++s) {
            const int L = P.L[s], T = P.T[s], C = P.R * T;
            std::vector<int> perm(C);
            std::memcpy(perm.data(), q, sizeof(int) * C);
            for (int rep = 0; rep < P.R; ++rep) {
                std::vector<char> seen(T, 0);
                for (int k = 0; k < T; ++k) {
                    const int j = perm[rep * T + k];
                    if (j < 0 || j >= T || seen[j]) return fail(PT_EINVAL, "checkpoint holds an invalid permutation");
                    seen[j] = 1;
                }
            }
            q += (sizeof(int) + sizeof(double)) * C + sizeof(float) * 3 * static_cast<size_t>(L) * L * L * C;
        }
    }
    // validated: restore
    PT_HIP(hipStreamSynchronize(c->stream));
    std::vector<int> slot(P.n_chains);
    std::vector<float> beta_of(P.n_chains);
    for (int s = 0; s < P.S; ++s) {
        const int L = P.L[s], T = P.T[s], C = P.R * T;
        const size_t n = 3 * static_cast<size_t>(L) * L * L;
        std::vector<int> perm(C);
        std::memcpy(perm.data(), r.p, sizeof(int) * C);
        r.p += sizeof(int) * C;
        for (int rep = 0; rep < P.R; ++rep)
            for (int k = 0; k < T; ++k) {
                const int j = perm[rep * T + k];
                slot[P.chain_base[s] + rep * T + j] = k;
                beta_of[P.chain_base[s] + rep * T + j] = static_cast<float>(c->betas_host[P.beta_base[s] + k]);
            }
        PT_HIP(hipMemcpy(c->perm + P.perm_base[s], perm.data(), sizeof(int) * C, hipMemcpyHostToDevice));
        PT_HIP(hipMemcpy(c->E + P.chain_base[s], r.p, sizeof(double) * C, hipMemcpyHostToDevice));
        r.p += sizeof(double) * C;
        for (int j = 0; j < C; ++j) {
            PT_HIP(hipMemcpy(c->stage, r.p, n * sizeof(float), hipMemcpyHostToDevice));
            PT_HIP(launch_chain_io(c->spins, P.spin_base[s], P.lanes[s], L, j, c->stage, false, c->stream));
            PT_HIP(hipStreamSynchronize(c->stream));
            r.p += n * sizeof(float);
        }
    }
    PT_HIP(hipMemcpy(c->slot_of, slot.data(), sizeof(int) * slot.size(), hipMemcpyHostToDevice));
    PT_HIP(hipMemcpy(c->beta_of, beta_of.data(), sizeof(float) * beta_of.size(), hipMemcpyHostToDevice));
    const uint32_t ctr[2] = {static_cast<uint32_t>(hb), static_cast<uint32_t>(pt)};
    PT_HIP(hipMemcpy(c->counters, ctr, sizeof(ctr), hipMemcpyHostToDevice));
    c->hb_sweeps = hb;
    c->pt_passes = pt;
    return PT_OK;
}

pt_status pt_set_stream(pt_ctx *c, void *stream)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if ((st = drain_events(c)) != PT_OK) return st;
    c->stream = static_cast<hipStream_t>(stream);
    return PT_OK;
}

pt_status pt_sync(pt_ctx *c)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    PT_HIP(hipStreamSynchronize(c->stream));
    return PT_OK;
}

pt_status pt_profile(pt_ctx *c, int enable)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if ((st = drain_events(c)) != PT_OK) return st;
    c->profiling = enable != 0;
    for (int q = 0; q < 4; ++q) {
        c->prof_launches[q] = 0;
        c->prof_ms[q] = 0.0;
    }
    return PT_OK;
}

pt_status pt_kernel_time(pt_ctx *c, int kind, uint64_t *launches, double *ms)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (kind != PT_K_OVERRELAX && kind != PT_K_HEATBATH && kind != PT_K_RESIDENT && kind != PT_K_PERSISTENT)
        return fail(PT_EINVAL, "unknown kernel kind");
    if ((st = drain_events(c)) != PT_OK) return st;
    if (launches) *launches = c->prof_launches[kind];
    if (ms) *ms = c->prof_ms[kind];
    return PT_OK;
}

void pt_free(pt_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (auto &pe : c->pending) c->free_events.push_back(pe.second);
    for (auto &e : c->free_events) {
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    for (auto &g : c->step_graphs) (void)hipGraphExecDestroy(g.second);
    for (auto &g : c->run_graphs)
        for (hipGraphExec_t e : g.second.one)
            if (e) (void)hipGraphExecDestroy(e);
    for (auto &g : c->programs) (void)hipFree(g.second.mem);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    delete c;
}

}  // extern "C"
