// kernels.hpp -- parameter blocks and launchers of the gfx950 kernels.
//
// Device layouts (all chosen for coalesced 64-lane access on CDNA):
//
//  spins   per chain: [colour 2][component 3][H] FP32, H = N/2.  A site
//          (x,y,z) of colour c = (x+y+z)&1 sits at packed index
//          p = (x>>1) + (L/2)*(y + L*z) of its colour plane, so a
//          half-sweep reads its own colour and the other colour as dense
//          component rows.  Chains of a sample are contiguous.
//  cpl     per sample: [colour 2][54][H] FP32.  For the site at packed
//          index p of colour c, element n*9 + a*3 + b is A_n[a][b], where
//          A_0, A_2, A_4 are the bond matrices M_{mu,x} towards x+e_mu and
//          A_1, A_3, A_5 are the transposes M_{mu,x-e_mu}^T of the bonds
//          from x-e_mu, so that  h_x = sum_n A_n s_{nbr_n(x)}.  The
//          duplication (each bond stored twice) buys fully coalesced,
//          gather-free coupling loads.
//          (This is the site-lane layout, lanes = 1.  The chain-lane layout,
//          lanes = 64, stores group g = j/64 of a sample as
//          [colour][H][component][64], lane = j%64; see spin_index.)
//          Chain-lane samples keep the same 54 numbers per site site-major,
//          [colour 2][H][54]: one 216-byte block per site, which a
//          heat-bath wave reads with five back-to-back scalar loads (the
//          overrelaxation and energy waves read the canonical blocks).
//  cpls    per sample, site-major canonical couplings [N][3][3][3]: the
//          three forward bond matrices of site i are floats 27i .. 27i+26.
//  chains  global chain id = chain_base[sample] + rep*T + j, j = start slot.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptsg {

constexpr int kXcds = 8;           // XCDs of the chip, each with its own L2
constexpr int kSweepBlock = 256;   // threads per sweep workgroup (4 waves)
constexpr int kMaxGroup = 128;     // chains per sweep workgroup (upper bound)
constexpr int kMeasBlock = 256;
constexpr int kClWaves = 4;        // chain-lane mapping: waves per workgroup
constexpr int kClBlock = 64 * kClWaves;
constexpr int kRsMaxBlock = 1024;  // lattice-resident mapping: threads per workgroup (max)
constexpr int kRsMaxL = 16;        // largest L whose chain (12 N bytes) is kept in LDS
constexpr int kOverlapQ = 45;      // plane partials: Q(0), Q(kx), Q(ky) re/im, 9 each
constexpr int kChiralQ = 19;       // kappa(0), kappa(kx), kappa(ky) re/im, 3 each; 4 SD sums
constexpr int kPlaneQ = kOverlapQ + kChiralQ;

enum SweepKind { kOverrelax = 0, kHeatbath = 1, kEnergyOnly = 2 };

// Float index of component k of the site with packed index p (colour c) of
// chain j of a sample whose spins start at `base`, in either layout.
__host__ __device__ inline int64_t spin_index(int64_t base, int lanes, int64_t H, int j, int c, int k,
                                             int64_t p)
{
    if (lanes == 1) return base + ((static_cast<int64_t>(j) * 2 + c) * 3 + k) * H + p;
    const int g = j >> 6, l = j & 63;
    return base + (((static_cast<int64_t>(g) * 2 + c) * H + p) * 3 + k) * 64 + l;
}

struct SweepParams {
    float *spins;
    const float *cpl;
    const int *samples;          // sample ids of this launch (one lattice class)
    const int64_t *spin_base;    // per sample: float offset of its chain 0
    const int64_t *cpl_base;     // per sample: float offset of its couplings
    const float *bm_D;           // per sample: D of the bimodal family
    int bimodal;                 // cpl holds 8 bytes of bond codes per site ([colour][H][8])
    const int *chain_base;       // per sample: global id of its chain 0
    const int *slot_of;          // per global chain: current temperature slot
    const float *beta_of;        // per global chain: 1/T of its slot
    double *e_part;              // [global chain][e_stride] energy partials
    int e_stride;
    int L, H, C, G, T;           // lattice, N/2, chains/sample, chains/workgroup, slots
    int n_tiles, per;            // site blocks per sample; blocks per XCD (grid = 8*per)
    int colour;
    const uint32_t *counters;    // device [0]: heat-bath sweeps done, [1]: PT passes done
    uint32_t hb_offset;          // this sweep's index within the step
    uint32_t key0, key1;
};

// Chain-lane mapping (one wave = 64 chains of one sample at one site).
struct ClParams {
    float *spins;
    const float *cpl;            // per-site packed couplings [colour][H][54] per sample
                                 // (bimodal: 8 code bytes per site, [colour][H][8])
    const int *items;            // [n_items][2]: (sample, chain group)
    const int64_t *spin_base;
    const int64_t *cpl_base;
    const int *chain_base;
    const int *slot_of;
    const float *beta_of;
    double *e_part;
    int e_stride;
    int L, H, C, T;
    int bimodal;                 // cpl holds bond codes; bm_table their matrices
    const float *bm_table;       // [sample][128][9]: the matrix of each code (bimodal samples)
    int canon;                   // float couplings read from the canonical blocks below
    const float *cpls;           // site-major canonical couplings [N][27] per sample
    const int64_t *cpls_base;
    int split;                   // waves per packed row (divides L/2)
    int strip;                   // row order: strips of `strip` y-rows, z-major within a strip (0: y-major)
    int n_tiles, per;            // workgroups of rows per item; per XCD (grid = 8*per)
    int colour;
    const uint32_t *counters;    // device [0]: heat-bath sweeps done, [1]: PT passes done
    uint32_t hb_offset;          // this sweep's index within the step
    uint32_t key0, key1;
};

// Lattice-resident mapping: one workgroup per chain, spins in LDS for a step.
struct RsParams {
    float *spins;
    const float *cpl;            // packed six-matrix couplings (site-lane layout)
    const int *samples;
    const int64_t *spin_base, *cpl_base;
    const int *chain_base, *slot_of;
    const float *beta_of;
    double *E;
    int L, H, C, T;
    int n_hb, n_or, energy_only;
    const uint32_t *counters;    // device [0]: heat-bath sweeps done before this step
    uint32_t key0, key1;
};

struct SwapParams {
    int *perm;                   // [sample][rep][T]: chain j at each slot
    int *slot_of;
    float *beta_of;
    const double *E;             // per global chain
    const double *betas;         // [sample][T] by slot
    const int *chain_base, *perm_base, *beta_base, *n_temps;
    int n_samples, R;
    uint32_t *counters;          // device [1]: PT passes done (read, then advanced by the kernel)
    uint32_t key0, key1;
};

struct EnergyParams {
    const double *e_part;
    int e_stride, n_blocks;      // partial blocks per chain for this class
    const int *samples, *chain_base;
    int C;
    double *E;
};

// Where the records of the next measurement go when a run of whole steps is
// replayed as graphs: base + k * stride, k advanced on the device after
// every measurement (so the captured kernels need no new arguments).
struct RecordCursor {
    void *base;                  // device pt_meas array of the caller
    uint64_t k;                  // measurements written so far
    uint64_t stride;             // records per measurement
};

struct MeasParams {
    const float *spins;
    const float *cpls;           // site-major couplings
    const int *rec;              // [n_records][4]: sample, slot, rep_a, rep_b
    const int *perm, *perm_base, *n_temps, *L, *chain_base, *twid_base;
    const int64_t *spin_base, *cpls_base;
    const int *lanes;            // per sample: 1 (site lanes) or 64 (chain lanes)
    const double *twid;          // per lattice: cos(2 pi n/L), then sin, n < L
    const double *E, *betas;
    const int *beta_base;
    double *part;                // [record - part_rec0][Lmax][kPlaneQ]
    int Lmax, n_records;         // finalisation covers records [rec0, n_records)
    int part_rec0;               // record whose partials sit at the start of `part`
    unsigned what;
    void *out;                   // device pt_meas[n_records]
    RecordCursor *cursor;        // non-null: write to cursor->base + cursor->k * stride instead
    // Sample `stage_sample` (-1: none) is read from `stage`, a site-lane
    // copy of its chains ([chain][colour][component][H]) instead of `spins`.
    const float *stage;
    int stage_sample;
    int rec0;                    // first record of a launch (blockIdx.x is relative)
};

// Persistent step: one cooperative launch runs the half-sweeps (and energy
// finalisations) of a whole step.  Every launch the multi-launch path would
// make becomes a descriptor of the same parameters and grid; descriptors
// whose launches may run concurrently form a phase, and the workgroups of
// the persistent grid meet at a grid-wide barrier after each phase.  Within
// a phase, virtual block v of the concatenated grids is taken by workgroup
// v mod gridDim.x; its (x, y, z) in the descriptor's grid is x fastest.
enum StepOp { kOpSite = 0, kOpChain = 1, kOpFinalize = 2 };

struct StepDesc {
    int op, kind, energy;        // body (StepOp), sweep kind, fused energy partials
    int gx, gy, gz, n_blocks;    // grid of the launch it stands for (gx a multiple of 8)
    union {
        SweepParams sp;
        ClParams cp;
        EnergyParams ep;
    };
};

struct PersistParams {
    const StepDesc *desc;        // every descriptor, phase by phase
    const int *phase_first;      // [n_phases]: first descriptor of each phase
    const int *phase_blocks;     // [n_phases]: virtual blocks of each phase
    int n_phases;
    uint32_t *counters;          // [0] += d_hb by one lane once every phase is done
    uint32_t d_hb;
};

// Optional kernel timing: when `start` is set, the dispatch itself stamps the
// two events at the kernel's start and end (the time a profiler reports).
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};

template <typename Kernel, typename... Args>
hipError_t launch_kernel(Kernel kernel, dim3 grid, dim3 block, uint32_t shm, hipStream_t st,
                         const LaunchTiming &t, Args... args)
{
    if (t.start)
        hipExtLaunchKernelGGL(kernel, grid, block, shm, st, t.start, t.stop, 0u, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, shm, st, args...);
    return hipGetLastError();
}

hipError_t launch_half_sweep(int kind, bool energy, const SweepParams &p, int n_samples,
                             hipStream_t st, const LaunchTiming &t = {});
hipError_t launch_cl_half_sweep(int kind, bool energy, const ClParams &p, int n_items,
                                hipStream_t st, const LaunchTiming &t = {});
// Row-ordered overrelaxation (chain-lane layout): one launch per row class.
int row_waves(int L);
hipError_t launch_cl_row_or(const ClParams &p, int cls, int n_items, hipStream_t st,
                            const LaunchTiming &t = {});
hipError_t launch_resident_step(const RsParams &p, int n_chains, hipStream_t st,
                                const LaunchTiming &t = {});
int rs_block(int L);
hipError_t launch_energy_finalize(const EnergyParams &p, int n_samples, hipStream_t st);
hipError_t launch_swap(const SwapParams &p, hipStream_t st);
// counters[0] += d_hb, counters[1] += d_pt (one lane; keeps replays of a
// captured step on fresh Philox counters)
hipError_t launch_advance_counters(uint32_t *counters, uint32_t d_hb, uint32_t d_pt, hipStream_t st);
hipError_t launch_init_spins(float *spins, int64_t spin_base, int lanes, int L, int C, int T,
                             int sample, uint32_t key0, uint32_t key1, hipStream_t st);
int cl_blocks(int L, int split);
// Persistent step launches (cooperative: every workgroup of the grid is
// resident at once, or the launch fails).  `grid` must be a multiple of 8
// and at most the CU count times the *_step_blocks_per_cu() figure.
int site_step_blocks_per_cu();
int cl_step_blocks_per_cu();
hipError_t launch_site_step(const PersistParams &p, int grid, hipStream_t st);
hipError_t launch_cl_step(const PersistParams &p, int grid, hipStream_t st);
hipError_t launch_chain_io(float *spins, int64_t base, int lanes, int L, int j, float *canon,
                           bool to_canon, hipStream_t st);
// Plane kernels for records [rec0, rec0 + n) (lattices up to L), then, once
// all records are done, the per-record finalisation of records
// [rec0, n_records).
hipError_t launch_measure_records(const MeasParams &p, int n, int L, int R, hipStream_t st);
hipError_t launch_measure_finalize(const MeasParams &p, hipStream_t st);
// One lane: cursor = {base, 0, stride}; cursor->k += 1.
hipError_t launch_set_cursor(RecordCursor *cursor, void *base, uint64_t stride, hipStream_t st);
hipError_t launch_advance_cursor(RecordCursor *cursor, hipStream_t st);
// Copy the chains of a chain-lane sample into the site-lane layout (the
// measurement kernels then read each component plane coalesced).
hipError_t launch_cl_to_sl(const float *spins, int64_t base, int H, int C, float *stage, hipStream_t st);

}  // namespace ptsg
