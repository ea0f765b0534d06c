/*
 * ptsg.h -- C ABI of the MI355X (gfx950) library for equilibrium Monte Carlo
 * of the 3d Heisenberg spin glass with random anisotropic couplings
 * (Baity-Jesi, Fernandez, Martin-Mayor, Sanz, arXiv:1309.1599).
 *
 * One Monte Carlo step of the paper (Sec. III and appendix A.1) is
 *     pt_step(ctx, 1, L);   pt_swap(ctx);
 * i.e. one heat-bath sweep, L overrelaxation sweeps, one parallel-tempering
 * pass.  Measurements (Sec. II.B) are taken with pt_measure; pt_run runs many
 * such steps, with a measurement every few, as replayed graphs.
 *
 * Model (Sec. II.A, Eq. (1)).  N = L^3 unit 3-vectors on a periodic cubic
 * lattice, site i = x + L*(y + L*z).  Each of the 3N bonds (i, i+e_mu),
 * mu = 0,1,2 for x,y,z, carries a real 3x3 matrix M, and
 *     H = - sum_i sum_mu  s_i^T M_{mu,i} s_{i+e_mu}.
 * The paper's bond J*1 + D (D symmetric) is the special case M = J*1 + D;
 * general matrices are accepted.  L must be even (checkerboard), 4 <= L <= 256.
 *
 * Ensemble.  A sample is one set of couplings; it is simulated at n_temps
 * temperatures T_0 < T_1 < ... (the temperature slots) with n_replicas
 * replicas each.  Chain (r, j) of a sample starts at slot j; parallel
 * tempering permutes which chain sits at which slot and never moves spins
 * (appendix A.1).
 *
 * Random numbers.  Philox4x32-10 (Salmon et al., SC'11) with key
 * (seed lo32, seed hi32).  Counters (fourth word: tag<<28 | slot<<16 | rep<<8):
 *   heat-bath at site i:      (i, hb_sweep, sample, 0<<28 | slot<<16 | rep<<8)
 *   hot start at site i:      (i, 0, sample, 2<<28 | j<<16 | rep<<8)
 *   PT pair (k, k+1):         (k, pt_pass, sample, 1<<28 | rep<<8)
 * where hb_sweep counts the heat-bath sweeps done so far by the context and
 * pt_pass the PT passes.  Uniforms: u = ((w >> 9) + 0.5) * 2^-23 from one
 * word (heat-bath, hot start), u = ((w0>>6)*2^26 + (w1>>6) + 0.5) * 2^-52
 * from two (PT).  So n_temps <= 4096 and n_replicas <= 256.
 *
 * Precision.  Spins and couplings are FP32 in device memory; energies,
 * the PT acceptance and all measurement sums are FP64.
 *
 * Memory and streams.  Host arrays passed in are copied before the call
 * returns.  Device memory is either one caller-owned workspace (see
 * pt_workspace_size) or allocated by the library and released by pt_free.
 * Work is queued on the context's stream (pt_set_stream); pt_step, pt_swap,
 * pt_run and pt_measure_noalloc are asynchronous, every call that returns
 * data to the host synchronises the stream.  A context is not thread-safe; distinct contexts
 * are independent.
 *
 * Errors.  Every call returns a pt_status; no C++ exception crosses the ABI.
 * pt_last_error() returns a message for the last failure on the calling
 * thread.
 */
#ifndef PTSG_H
#define PTSG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pt_ctx pt_ctx;

typedef enum {
    PT_OK = 0,
    PT_EINVAL = -1,       /* invalid argument (message says which) */
    PT_ENOMEM = -2,       /* workspace too small or allocation failed */
    PT_EDEVICE = -3,      /* HIP runtime error (message holds its string) */
    PT_ESTATE = -4,       /* call not valid in the context's state */
    PT_EUNSUPPORTED = -5  /* valid but not supported by this library */
} pt_status;

/* Measurement selection bits for pt_measure. */
enum {
    PT_M_OVERLAP = 1u, /* overlap tensor Q^{ab}(k), Sec. II.B */
    PT_M_CHIRAL = 2u,  /* chiral-glass overlap q_CG^mu(k), Sec. II.B */
    PT_M_SD = 4u,      /* Schwinger-Dyson sums, appendix A.4 */
    PT_M_ENERGY = 8u,  /* energies E_a, E_b and beta (Eq. (1); every record carries them,
                        * so this bit alone asks for nothing else and launches no
                        * lattice reduction) */
    PT_M_ALL = 15u
};

/* One measurement record: replicas a < b of one sample at one temperature
 * slot.  Fourier sums use (1/N) sum_x f(x) exp(+i k.x) with k = 0 or
 * k = (2 pi / L) e_d, d = 0,1,2 (Sec. II.B):
 *   q0[al*3+be]        = (1/N) sum_x s^a_al(x) s^b_be(x); q(0) = trace
 *   qk_re/im[d][al*3+be] the same at k = (2 pi/L) e_d
 *   cg0[mu]            = (1/N) sum_x zeta^a_{x,mu} zeta^b_{x,mu},
 *                        zeta_{x,mu} = s_{x+e_mu} . (s_x cross s_{x-e_mu})
 *   cgk_re/im[d][mu]   the same at k = (2 pi/L) e_d
 *   sd1 = sum_x s.h, sd2 = sum_x (h^2 - (s.h)^2) for chains a and b;
 *   E_a, E_b: energies (Eq. (1)) from the last pt_step / pt_set_spins.
 * Fields not selected by `what` are zero. */
typedef struct {
    int32_t sample, tslot, rep_a, rep_b;
    double beta, E_a, E_b;
    double q0[9];
    double qk_re[3][9], qk_im[3][9];
    double cg0[3];
    double cgk_re[3][3], cgk_im[3][3];
    double sd1_a, sd2_a, sd1_b, sd2_b;
} pt_meas;

/* A batch of samples in one context.  Samples may differ in L and in their
 * temperature grids; all share n_replicas and seed. */
typedef struct {
    int n_samples;
    const int *L;                  /* [n_samples] linear sizes */
    const int *n_temps;            /* [n_samples] */
    const double *const *temps;    /* [n_samples] -> host [n_temps[s]], ascending, > 0 */
    const float *const *couplings; /* [n_samples] -> host [3][L^3][3][3], finite */
    int n_replicas;
    uint64_t seed;
    void *stream;                  /* hipStream_t for all work; NULL = null stream */
    void *workspace;               /* caller device memory, or NULL: library allocates */
    size_t workspace_bytes;        /* size of `workspace` (>= pt_workspace_size) */
    unsigned flags;                /* PT_F_* below; 0 = automatic choices */
} pt_batch_desc;

/* Kernel mapping of the sweeps (the spins are bit-identical in all three):
 * site lanes: one lane per site, a workgroup loops over the chains of a
 *   sample with the site's couplings held in registers;
 * chain lanes: one wave = 64 chains of a sample at one site, couplings in
 *   scalar registers; each 64-chain group runs all sweeps of a step back to
 *   back so that its working set stays in the 256 MB Infinity Cache;
 * resident: one workgroup per chain keeps the whole lattice in LDS for all
 *   sweeps of a step (L <= 16).
 * Automatic: resident for L <= 8, and for L <= 16 when the lattice class
 * (the samples of one L and number of temperatures) holds at least 256
 * chains, enough workgroups for the chip; chain lanes for 24 <= L <= 64 (the
 * measured range where they are faster) when the sample's chains fill its
 * 64-lane waves to >= 90%; else site lanes.  A forced mapping that does not
 * apply to a sample (resident with L > 16, chain lanes with L > 128) falls
 * back to site lanes for it. */
enum {
    PT_F_SITE_LANES = 1u,
    PT_F_CHAIN_LANES = 2u,
    PT_F_RESIDENT = 4u,
    /* Capture the launch sequence of pt_step(n_hb, n_or) in a hipGraph the
     * first time each (n_hb, n_or) is used and replay it afterwards (the
     * Philox counters live in device memory, so replays are exact).  Steps
     * taken while kernel timing is enabled run without the graph. */
    PT_F_GRAPHS = 8u,
    /* The plain single-chain form, kept as a reference point: site lanes with
     * one chain per workgroup, so every chain re-reads its couplings. */
    PT_F_PLAIN = 16u,
    /* Autotuner: for each distinct (L, n_temps) in the batch, time a step of
     * 1 heat-bath + min(L, 32) overrelaxation sweeps of every applicable
     * mapping on a temporary context (enough of those samples for 4096
     * chains, at least 4, at most 2 GB of spins), then of the fastest
     * mapping with neighbouring tile shapes (site lanes: half and twice the
     * chains per workgroup; chain lanes: half and twice the waves per packed
     * row and the y-strips of the row order half and twice as tall), and use
     * the fastest plan (pt_get_mapping, pt_get_tile); results are cached for
     * the process.  Ignored when a mapping flag or PT_F_PLAIN is set.
     * Runs kernels on the current device, so pt_workspace_size needs the
     * device too when this flag is set.  When the environment variable
     * PTSG_PLAN_CACHE names a file, results are also looked up there before
     * timing and appended after it, one text line per (device architecture,
     * CU count, L, n_temps, n_replicas, samples timed, PT_F_GRAPHS,
     * PT_F_BIMODAL) holding the mapping and the tile shape; lines that do not
     * parse or name a plan the lattice cannot use are skipped, and an
     * unwritable file is not an error. */
    PT_F_AUTOTUNE = 32u,
    /* The paper's coupling family (Sec. II.A): every bond is
     * M = J*1 + D_sym, J = +-1, the six entries D_ab (a <= b) of the
     * symmetric D equal to +-D, one D > 0 per sample (checked bit for bit;
     * PT_EINVAL otherwise).  Site-lane and chain-lane samples then keep one
     * byte per bond (8 bytes per site instead of 216): site lanes decode it
     * in the sweep kernel, chain lanes read each code's matrix from a
     * per-sample table of the 128 codes; results are bit-identical to
     * passing the same matrices without the flag.  Resident samples and the
     * row order (PT_F_ROW_OR) keep the float layouts. */
    PT_F_BIMODAL = 64u,
    /* Overrelaxation sweeps in the row order (Sec. III, appendix A.3) instead
     * of the checkerboard: rows of 8 spins along x, row (b, y, z) holding
     * x = 8b .. 8b+7 in class (b + y + z) mod 2; a sweep updates every
     * class-0 row, then every class-1 row, each row in increasing x with
     * each spin seeing those updated before it.  Heat-bath sweeps stay
     * checkerboard.  Needs L = 8 or a multiple of 16 (an odd number of rows
     * along x above one would put the first and last row of an x line, which
     * touch across the boundary, in one class), L <= 128, and runs on the
     * chain-lane mapping (excludes PT_F_SITE_LANES, PT_F_RESIDENT,
     * PT_F_PLAIN). */
    PT_F_ROW_OR = 128u,
    /* Persistent step (App. A.3: all lattices of the batch updated by one
     * program): pt_step runs as ONE cooperative kernel launch that performs
     * every half-sweep of every sample and L class, then the energies, with a
     * grid-wide barrier between dependent half-sweeps (the launches the
     * multi-launch path makes become descriptors of a device work list; the
     * half-sweeps of different classes share a phase).  The grid is what the
     * device keeps resident (the launch fails with PT_EDEVICE otherwise).
     * Results are bit-identical to the multi-launch path with the same
     * mapping and tile shape.  One mapping serves the whole batch: chain
     * lanes when PT_F_CHAIN_LANES is set (and every L <= 128) or, with no
     * mapping flag, when they pay for every sample (24 <= L <= 64 and
     * >= 90% wave fill); else site lanes.  Excludes PT_F_RESIDENT and
     * PT_F_ROW_OR; PT_F_GRAPHS and PT_F_AUTOTUNE are ignored.  The work list
     * of each (n_hb, n_or) is built on its first use, in device memory the
     * library allocates even when the caller provides the workspace. */
    PT_F_PERSISTENT = 256u
};

/* The mapping used for a sample: PT_F_SITE_LANES, PT_F_CHAIN_LANES or
 * PT_F_RESIDENT. */
pt_status pt_get_mapping(pt_ctx *ctx, int sample, unsigned *flag);

/* The tile shape of a sample's sweeps (App. A.3: how the batch is laid on
 * the GPU), from the heuristics or the autotuner: chains per workgroup
 * (site lanes: G, chain lanes: 64, resident: 1); waves per packed row and
 * y-rows per strip of the row visiting order (chain lanes; 0 otherwise). */
pt_status pt_get_tile(pt_ctx *ctx, int sample, int *chains_per_group, int *split, int *strip);

/* One sample (the single-lattice form of the API).  Equivalent to
 * pt_init_batch with n_samples = 1, the null stream and library-owned
 * memory.  Spins start hot (uniform on the sphere, Philox tag 2). */
pt_status pt_init(pt_ctx **ctx, int L, const float *couplings, const double *temps,
                  int n_temps, int n_replicas, uint64_t seed);

/* Bytes of device workspace a batch needs (0 if the descriptor is invalid;
 * pt_last_error then says why). */
size_t pt_workspace_size(const pt_batch_desc *desc);

/* Create a context for a batch of samples (see pt_batch_desc). */
pt_status pt_init_batch(pt_ctx **ctx, const pt_batch_desc *desc);

/* n_or value for the paper's Monte Carlo step in a batch of several L
 * (Sec. III): every sample runs L overrelaxation sweeps, L its own linear
 * size. */
#define PT_OR_L (-1)

/* n_hb heat-bath sweeps then n_or overrelaxation sweeps of every chain
 * (appendix A.1); n_or = PT_OR_L gives each sample L of them.  A sweep is the checkerboard half-sweep of colour 0
 * ((x+y+z) even) then of colour 1.  Heat-bath draws s from
 * P(s) ~ exp(s.h / T); overrelaxation maps s -> 2 h (h.s)/h^2 - s; both
 * renormalise the spin.  The local field is
 *   h_i = sum_mu [ M_{mu,i} s_{i+e_mu} + M_{mu,i-e_mu}^T s_{i-e_mu} ],
 * i.e. -dH/ds_i.  Energies are refreshed at the end.  Asynchronous. */
pt_status pt_step(pt_ctx *ctx, int n_hb, int n_or);

/* One parallel-tempering pass per (sample, replica) (appendix A.1): for
 * k = 0 .. n_temps-2 in order, exchange the chains at slots k and k+1 with
 * probability min(1, exp((beta_k - beta_{k+1}) (E_k - E_{k+1}))).
 * Asynchronous. */
pt_status pt_swap(pt_ctx *ctx);

/* Measure every (sample, slot, replica pair a < b) and copy the records,
 * ordered by sample, slot, then pair, into out[cap].  *n_out receives the
 * record count (sum over samples of n_temps * R(R-1)/2); PT_ENOMEM if cap is
 * smaller; out == NULL with cap == 0 only stores the count.  PT_M_OVERLAP /
 * PT_M_CHIRAL need n_replicas >= 2 (PT_ESTATE).  Synchronous. */
pt_status pt_measure(pt_ctx *ctx, unsigned what, pt_meas *out, size_t cap, size_t *n_out);

/* Whole Monte Carlo steps (Sec. III: the sweeps of one step, then one
 * tempering pass, and every `every` steps a measurement): n_steps times
 * pt_step(n_hb, n_or) + pt_swap, and after steps every, 2*every, ... the
 * records of pt_measure(what), measurement k written to
 * d_out[k * n_records ...], d_out a DEVICE array of cap pt_meas the caller
 * owns (cap >= (n_steps / every) * n_records; every = 0: no measurement,
 * d_out may be NULL).  With PT_F_GRAPHS each kind of step (with and without
 * a measurement) is captured once as one hipGraph -- sweeps, tempering and
 * measurement kernels together -- and replayed, so a step costs one graph
 * launch on the host; the results equal those of the separate calls.
 * Asynchronous.  Errors as pt_step, pt_measure; PT_ENOMEM if cap is short. */
pt_status pt_run(pt_ctx *ctx, int n_steps, int n_hb, int n_or, int every, unsigned what, pt_meas *d_out,
                 size_t cap);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the records of
 * pt_measure, written to d_out, a DEVICE array of cap pt_meas the caller
 * owns, asynchronously on the context's stream.  No allocation, no host copy,
 * no synchronisation.  The plane partials go to a fixed 8 MB device array of
 * the library (one per device, held until the process ends; records are
 * processed in chunks that fit it, so any batch pt_init_batch accepts fits);
 * chain-lane samples are copied to the site-lane layout in the context's own
 * staging buffer first, as pt_measure does.  Every call on one device shares
 * that array: calls that overlap on one device (different streams, threads
 * or contexts) race.  PT_ENOMEM if cap is below the record count; the other
 * errors as pt_measure's.  The records equal pt_measure's. */
pt_status pt_measure_noalloc(pt_ctx *ctx, unsigned what, pt_meas *d_out, size_t cap);

/* Spins of the chain at (sample, replica, slot), host [N][3] FP32.
 * pt_set_spins copies them in (no normalisation) and refreshes that
 * sample's energies.  Synchronous. */
pt_status pt_get_spins(pt_ctx *ctx, int sample, int rep, int tslot, float *out);
pt_status pt_set_spins(pt_ctx *ctx, int sample, int rep, int tslot, const float *in);

/* out[k] = index j of the chain now at slot k, for one (sample, replica). */
pt_status pt_get_perm(pt_ctx *ctx, int sample, int rep, int32_t *out);

/* The same for every (sample, replica) at once, ordered by sample, replica,
 * slot (sum over samples of n_replicas * n_temps entries, the order of
 * pt_get_energy): one copy for following the temperature random walk of
 * every chain (Sec. III).  Synchronous. */
pt_status pt_get_perms(pt_ctx *ctx, int32_t *out);

/* Energies (Eq. (1)) of all chains, ordered by sample, replica, slot. */
pt_status pt_get_energy(pt_ctx *ctx, double *out);

/* Heat-bath sweeps and PT passes done so far (the Philox counters). */
pt_status pt_get_counters(pt_ctx *ctx, uint64_t *hb_sweeps, uint64_t *pt_passes);

/* Checkpoint and resume.  pt_save writes the whole Monte Carlo state of a
 * context into blob[cap]: every chain's spins (host [N][3] FP32, chains in
 * (sample, replica, start slot) order), the slot permutations, the chain
 * energies and the two Philox counters, behind a header that records the
 * batch shape (L, n_temps, inverse temperatures, n_replicas, seed) and a
 * 64-bit FNV-1a hash of each sample's couplings.  With blob == NULL it only
 * stores the size it needs in *n_bytes; a smaller cap is PT_EINVAL.
 * pt_load restores such a blob into a context created from the same
 * descriptor (the kernel mapping and the graph flag may differ); a blob of
 * another shape, seed or coupling set, or a damaged one, is PT_EINVAL and
 * leaves the context unchanged.  Continuing after pt_load gives the spins,
 * permutations and energies the saved run would have given.  Both are
 * synchronous. */
pt_status pt_save(pt_ctx *ctx, void *blob, size_t cap, size_t *n_bytes);
pt_status pt_load(pt_ctx *ctx, const void *blob, size_t n_bytes);

/* Queue all further work on `stream` (hipStream_t, NULL = null stream). */
pt_status pt_set_stream(pt_ctx *ctx, void *stream);

/* Wait for all work queued by the context. */
pt_status pt_sync(pt_ctx *ctx);

/* Kernel timing.  When enabled, each sweep-kernel launch is bracketed by
 * HIP events on the context's stream; pt_kernel_time synchronises and
 * returns, for one kernel kind, the number of launches and their summed
 * device time since profiling was (re-)enabled. */
enum { PT_K_OVERRELAX = 0, PT_K_HEATBATH = 1, PT_K_RESIDENT = 2 /* whole-step launches */,
       PT_K_PERSISTENT = 3 /* PT_F_PERSISTENT step launches (timed by events around the launch) */ };
pt_status pt_profile(pt_ctx *ctx, int enable);
pt_status pt_kernel_time(pt_ctx *ctx, int kind, uint64_t *launches, double *ms);

/* Release the context and any memory the library allocated. NULL is a no-op. */
void pt_free(pt_ctx *ctx);

/* Message of the last failed call on this thread ("" if none). */
const char *pt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PTSG_H */
