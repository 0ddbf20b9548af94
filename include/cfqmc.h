/* cfqmc.h - C ABI of the MI355X continuous-field DQMC sweep.
 *
 * Method: Liao, Chen, Rong, Assaad, Janssen, Meng, "Numerical evidence of a
 * critical point in the (2+1)D SO(5) nonlinear sigma model with
 * Wess-Zumino-Witten term" (arXiv 2605.03700), Methods section:
 *   - torus density operator (eq. torus density operator) and momentum cutoff,
 *   - Fierz-transformed Hamiltonian H = sum_i g_i H_i (eq. newmodel),
 *   - continuous Hubbard-Stratonovich transform (eq. HS transform),
 *   - Z = int Dphi exp(-S_0) det[1 + B(beta,0)] and the equal-time Green's
 *     function G(tau) = (1 + B(tau,0) B(beta,tau))^{-1} (eq. green function),
 *   - Langevin (MALA) proposal of all fields of a time slice (eq. Langevin
 *     proposal) with the Metropolis-Hastings test and the adaptive step size.
 *
 * Conventions
 *   N = n_phi orbitals per flavour, n = 2N spin-block dimension (the Fierz
 *   channels act as identity on spin, so G_4N = 1_spin (x) G_2N).
 *   Spin-block index v*N + k (valley v, orbital k = 0..N-1); 4N index
 *   s*2N + v*N + k. G_ij = <c_i c_j^dagger>, complex128, row major.
 *   Fields phi are real, laid out [chain][l_tau][4][n_q]: channel i = 0..3
 *   (O^i = 1, tau_x, tau_y, tau_z) and component c = 0..n_q-1, where c = 0 is
 *   sqrt(2) n_0 and the remaining components follow the half set of momenta
 *   {q_y > 0} U {q_y = 0, q_x > 0} sorted by (q_y, q_x), each contributing
 *   n_q + n_{-q} then i (n_q - n_{-q}) (self-conjugate momenta of the
 *   Brillouin-zone mode contribute one component sqrt(2) n_q).
 *
 * Ownership: the caller owns every host buffer it passes; the library owns
 * all device state it allocates. Device output buffers (measure_G with
 * on_device = 1) belong to the caller. Calls enqueue on the stream given at
 * creation; calls that return host data synchronise that stream.
 * Errors: every call returns 0 on success or a negative CFQMC_E* code; the
 * message is available from cfqmc_last_error. An error other than
 * CFQMC_ENUMERIC leaves the context unchanged. CFQMC_ENUMERIC (non-finite
 * values, exponential range exceeded) marks the chain state invalid until
 * cfqmc_init_fields is called again.
 * Threading: one context per host thread at a time; no global state.
 * Debugging: with CFQMC_DEBUG_SYNC=1 in the environment every kernel launch
 * is followed by a device synchronisation, and a failing launch prints the
 * kernel's name to stderr (slow; for locating a fault). CFQMC_LU_NP_LMAX
 * (read at cfqmc_create, default 8) is the largest multiplier the
 * non-pivoted LU of the Woodbury matrix M accepts before a chain is
 * refactorised with partial pivoting; 0 sends every chain to the pivoted
 * path (for testing that path). CFQMC_GUARD_PAIR=1 (read at cfqmc_create)
 * runs each precision-guarded channel application as two launches, one per
 * precision class, instead of one launch whose workgroups take their chain's
 * path (for testing that the two give identical results).
 */
#ifndef CFQMC_H
#define CFQMC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  CFQMC_OK = 0,
  CFQMC_EINVAL = -1,   /* invalid argument */
  CFQMC_ENOMEM = -2,   /* device allocation failed */
  CFQMC_EHIP = -3,     /* HIP runtime error */
  CFQMC_ENUMERIC = -4, /* non-finite result or exponential range exceeded */
  CFQMC_ESTATE = -5,   /* call not valid in the current state */
  CFQMC_ENOTIMPL = -6
};

/* Momentum sets. The first four are torus geometries (Methods, toric
 * regularization). CFQMC_Q_SPHERE is the spherical regularization (Methods):
 * N_phi = 2s + 1 orbitals m_k = k - 1 - s, density operators n_{l,m} from
 * Wigner 3j symbols for every 0 <= l <= 2s, |m| <= l (N_phi^2 per channel);
 * components per channel sqrt(2) n_{l,0} (l = 0..2s), then for m = 1..2s and
 * l = m..2s the pair n_{l,m} + n_{l,m}^+ and i (n_{l,m} - n_{l,m}^+). */
enum { CFQMC_Q_PAPER = 0, CFQMC_Q_RADIUS = 1, CFQMC_Q_BZ = 2, CFQMC_Q_LIST = 3, CFQMC_Q_SPHERE = 4 };
/* Precision of the slice work. FP64: everything in FP64. MIXED: the wraps and
 * the drift frames in complex FP32 on MFMA with FP64 accumulation (FP64 master
 * G), the Woodbury product M in FP64. MIXED_ALL: M and the rank-k update
 * G' = G M^-1 in FP32 as well (the solve's block products in FP32, an FP64
 * accumulation point per 16-deep step). The LU of M, the exponentials,
 * stabilisation and recomputation stay FP64. With the precision guard on, a
 * chain it moves to FP64 runs all of these in FP64. */
enum { CFQMC_FP64 = 0, CFQMC_MIXED = 1, CFQMC_MIXED_ALL = 2 };

typedef struct cfqmc_ctx cfqmc_ctx;

typedef struct {
  int32_t n_phi;         /* LLL degeneracy N_phi (Methods, toric regularization), 1..140 */
  int32_t l_tau;         /* imaginary-time slices N_tau = beta / dtau */
  double dtau;           /* Trotter step (eq. Trotter decomposition) */
  double u0, uk, un;     /* couplings U_0, U_K, U_N (Results: U_0 = 1, SO(5) line U_K = U_N = u) */
  int32_t q_mode;        /* CFQMC_Q_*: paper cutoff exp(-2 pi |q|^2/(4N)) > 0.01, |q| l_B <= q_max,
                            the N^2 Brillouin-zone momenta, an explicit list, or the sphere */
  double q_max;          /* CFQMC_Q_RADIUS only */
  const int32_t* q_list; /* CFQMC_Q_LIST: pairs (qx, qy), closed under q -> -q; host, read at create */
  int32_t n_q_list;
  int32_t n_stab;        /* slices between FP64 recomputations of G (UDT stabilisation) */
  int32_t precision;     /* CFQMC_FP64, CFQMC_MIXED or CFQMC_MIXED_ALL (see above) */
  double eps0;           /* initial Langevin step size epsilon */
  double r0, deps;       /* acceptance set point and gain of eps <- eps + (r_a - r0) deps (0.574, 0.1) */
  double eps_min, eps_max;
  int32_t adapt_eps;     /* 1: adapt after every sweep; 0: frozen */
  uint64_t seed;         /* Philox4x32-10 key of the proposal noise; seeds the host draw of initial fields */
  int32_t n_chains;      /* independent chains of this shape, run together in every launch */
  const double* chain_u; /* optional host [n_chains][3] = (u0, uk, un) per chain; NULL: all equal */
  int32_t exp_squarings; /* max scaling-and-squaring steps of the Taylor exponential, 0..16 (default 2) */
  int32_t tile_cfg;      /* -1: autotune tile shapes at create; 0..19 fixed channel-application
                            configuration (GEMMs use min(tile_cfg, 3)). In the FP32 applications
                            0..7 and 14..16 add each 16-deep k slab into FP64 registers (14 with
                            three real products per complex step), 8..13, 17 and 18 accumulate in
                            FP32 over the whole k range (12, 13, 17, 18 with three products); the
                            autotuner picks among the former there unless the precision guard is
                            on. 15..18 use 8- or 16-wave workgroups of 16 x 16 wave tiles; 19 splits
                            the two valley products of a 32 x 32 tile over eight waves in FP64 (1 in
                            the FP32 applications) */
  int32_t dense4n;       /* 0 (only value): the spin-block form n = 2 N_phi. The Fierz channels act as
                            the identity on spin (eq. newmodel), so G_4N = 1_spin (x) G_2N exactly and
                            every output is expanded to 4N; 1 (the un-Fierzed dense 4N coupling, which
                            has a sign problem) returns CFQMC_ENOTIMPL from cfqmc_create */
  int32_t exact_drift;   /* 0 (only value): the Langevin drift differentiates each channel exponential to
                            first order, D = -phi + 2 Re alpha_i Tr[(1 - G_i)(o_i (x) q_c)] with G_i the
                            frame of channel i. 1 (the exact Frechet gradient of the printed gradient
                            equation) returns CFQMC_ENOTIMPL: any deterministic drift leaves the
                            Metropolis-Hastings chain exact, only its acceptance differs */
  int32_t precision_guard; /* mixed modes: 1 (default) runs the FP32 applications of a chain in FP64 for
                            the next block of n_stab slices when, at the last FP64 recomputation, its
                            max|G_FP64| exceeded guard_gmax or its max|G_updated - G_FP64| exceeded
                            guard_err, and from the next slice to the end of the block once its
                            updated G has an entry above guard_gmax (the FP32 rounding error of G
                            scales with |G|); 0: FP32 for every chain. Ignored in CFQMC_FP64 */
  double guard_gmax;     /* default 0.8 */
  double guard_err;      /* default 2.5e-7 */
  int32_t sweep_graph;   /* 1 (default): the launches of one whole sweep are recorded once as HIP graphs
                            (one per chunk of whole stabilisation blocks, at most about 64 slices) and
                            each later sweep is those graph launches, when the context has a stream of
                            its own (the groups of a batch; not the null stream); the device-side sweep
                            counter and series index make every replay the next sweep. With kernel
                            timing on, a second recorded form is cut at the timed launches, which run
                            as ordinary launches between the HIP events. 0: launch by launch. Results
                            are identical either way; a recording that fails is reported once on
                            stderr and the context launches one by one */
} cfqmc_params;

typedef struct {
  int64_t proposed, accepted; /* slice proposals and acceptances over the call */
  double eps;                 /* step size after the call */
  double max_stab_err;        /* max |G_updated - G_recomputed_fp64| at recomputation points */
  double max_phase_err;       /* max |Im ln R| (mod 2 pi) of the weight ratio, sign-free check */
  int32_t exp_range_flag;     /* 1 if an exponential needed more squarings than allowed */
  int32_t pad;
  double max_stab_rel;        /* max over recomputation points of max|G_updated - G_FP64| / max|G_FP64| */
  double max_abs_g;           /* max over recomputation points of max|G_FP64| */
  double fp64_guard_frac;     /* fraction of the chain's stabilisation blocks run with FP64 applications
                                 (from some slice on) by the precision guard (mixed modes) */
  double graph_sweep_frac;    /* fraction of the call's sweeps of the chain's context run as one launch of
                                 the recorded sweep graph (see sweep_graph) */
} cfqmc_stats;

/* Fill *p with the defaults (N=6, L=40, dtau=0.1, u0=1, uk=un=1, paper cutoff,
 * n_stab=10, FP64, eps0=0.5, r0=0.574, deps=0.1, eps in [1e-3, 5], adapt on,
 * one chain, exp_squarings=2, tile_cfg=-1, dense4n=0, exact_drift=0,
 * precision_guard=1, guard_gmax=0.8, guard_err=2.5e-7, sweep_graph=1). */
void cfqmc_default_params(cfqmc_params* p);

/* Create a context: builds the model tables on the host, allocates device
 * state. hip_stream: a hipStream_t (NULL = default stream). No fields yet.
 * CFQMC_EINVAL for invalid parameters, CFQMC_ENOTIMPL for dense4n or
 * exact_drift other than 0 (*out stays NULL in both cases). */
int cfqmc_create(const cfqmc_params* p, void* hip_stream, cfqmc_ctx** out);
int cfqmc_destroy(cfqmc_ctx* c);

/* Sizes: number of HS components per channel, chains, 4N. Any pointer may be NULL. */
int cfqmc_sizes(const cfqmc_ctx* c, int32_t* n_q, int32_t* n_chains, int32_t* dim_g4n);

/* Set the fields (host [n_chains][l_tau][4][n_q]) or, with phi == NULL, draw
 * them N(0,1) on the host (Box-Muller on a splitmix64 stream of the seed) and
 * upload them; rebuilds every slice propagator, both UDT stacks and G(0) in
 * FP64; resets eps and statistics. */
int cfqmc_init_fields(cfqmc_ctx* c, const double* phi);
int cfqmc_get_fields(cfqmc_ctx* c, double* phi_out);

/* Checkpoint / resume of a Markov chain set. cfqmc_checkpoint writes to the
 * file `path` (created or truncated) the fields, each chain's step size eps,
 * the couplings, the device-RNG position (seed and sweep count) and the m^2
 * series; it needs initialised fields (else CFQMC_ESTATE). cfqmc_restore reads
 * such a file into a context of the same shape and couplings (else
 * CFQMC_EINVAL, context unchanged), rebuilds every slice propagator, both UDT
 * stacks and G(0) in FP64 from the fields (as cfqmc_init_fields) and then
 * continues eps, the RNG stream and the series: later sweeps with device noise
 * draw the same noise as the uninterrupted run. Synchronise. */
int cfqmc_checkpoint(cfqmc_ctx* c, const char* path);
int cfqmc_restore(cfqmc_ctx* c, const char* path);

/* Run n_sweeps sweeps (slices tau = 1..L each) on all chains.
 * replay: NULL (device Philox noise) or host [n_chains][n_sweeps][l_tau][4 n_q + 1]
 * holding per slice the 4 n_q proposal normals (channel-major) and the
 * acceptance uniform u. stats: NULL or [n_chains]. Synchronises. */
int cfqmc_sweep(cfqmc_ctx* c, int32_t n_sweeps, const double* replay, cfqmc_stats* stats);

/* Equal-time Green's function G(tau) of one chain, 0 <= tau <= l_tau, expanded
 * to 4N (1_spin (x) G). g_out: [4N][4N] complex128, host (on_device = 0) or
 * device memory owned by the caller (on_device = 1). Computed in FP64 from the
 * UDT stacks. */
int cfqmc_measure_G(cfqmc_ctx* c, int32_t chain, int32_t tau, void* g_out, int32_t on_device);

/* Time-displaced Green's functions of one chain (Supplementary Note 2 needs
 * them for the imaginary-time correlator), on the spin block n = 2 N_phi, for
 * the current configuration, 0 <= tau <= l_tau (slice units):
 *   gt0 = G(tau,0) = <c(tau) c^dagger(0)> = B(tau,0) G(0),
 *   g0t = G(0,tau), element [i][j] = -<c_j^dagger(tau) c_i(0)> = -(1 - G(0)) B(tau,0)^-1,
 *   gtt = G(tau,tau).
 * Each output is NULL or a host [n][n] complex128 buffer (row-major, re/im
 * interleaved) owned by the caller. FP64 in every precision mode: recomputed
 * from the UDT stacks at block boundaries, carried through the slices of a
 * block by the slice propagators. Call between sweeps. Synchronises. */
int cfqmc_green_displaced(cfqmc_ctx* c, int32_t chain, int32_t tau, double* gt0, double* g0t, double* gtt);

/* Imaginary-time correlator of the SO(5) order parameter at q = 0
 * (Supplementary Note 2), C^i(tau) = <n^{Gamma^i}_{q=0}(tau) n^{Gamma^i}_{q=0}(0)>
 * for i = 1..5 and tau = 0..l_tau, of the current configuration of every chain
 * by Wick's theorem from G(tau,0), G(0,tau), G(tau,tau) and G(0) (one pass
 * over the slices, FP64). m^2_SO(5)(tau, q=0) is the mean over i; C^i(0) is the
 * equal-time S^i_{q=0}, C^i(l_tau) = C^i(0). Per configuration the values are
 * complex; their Monte Carlo average is real. out: host
 * [n_chains][l_tau + 1][5] complex128 (re/im interleaved), owned by the caller.
 * stab_rel: NULL or host [n_chains][3]: for G(tau,0), G(0,tau), G(tau,tau), the
 * largest max|carried - recomputed| / max|recomputed| over the block
 * boundaries (the FP64 accuracy of carrying them through a block).
 * Call between sweeps. Synchronises. */
int cfqmc_measure_tau(cfqmc_ctx* c, double* out, double* stab_rel);

/* Allocation-free variant of cfqmc_measure_tau, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same pass and kernels, with the
 * correlator's per-chain partial results (traces of G(0), running maxima of
 * the carried-vs-recomputed check) in a fixed device array of the library
 * (64 KiB per GPU: at most 512 chains, else CFQMC_EINVAL with a message) and
 * the outputs in caller-owned device memory:
 *   out_dev       device [n_chains][l_tau + 1][5] complex128 (re/im interleaved),
 *   stab_rel_dev  NULL or device [n_chains][3] doubles (as stab_rel above).
 * Calls no hipMalloc/hipFree and does not synchronise: the results are ready
 * when the context's stream reaches them. Every call on one GPU shares that
 * array, so calls that overlap on one GPU (different streams or threads) race;
 * the array keeps the last call's contents and each call clears what must
 * start at zero. Call between sweeps. */
int cfqmc_measure_tau_noalloc(cfqmc_ctx* c, void* out_dev, void* stab_rel_dev);

/* Orbital weights of the sphere's density operators (Methods, eq. sphere
 * density operator), the table behind CFQMC_Q_SPHERE: out[(l N + m) N + r] =
 * n_{l,m}[r, r + m] for 0 <= m <= l <= N - 1 and rows r of the orbitals
 * m_r = r - s (zero where r + m >= N). out: host buffer of N^3 doubles owned by
 * the caller; 1 <= n_phi <= 288. Host computation only (no device use). */
int cfqmc_sphere_weights(int32_t n_phi, double* out);

/* Equal-time structure factors S^i_q = <n^{Gamma^i}_q n^{Gamma^i}_{-q}>,
 * i = 1..5, at the given momenta (Results: S^i_q; the correlation ratio
 * R = 1 - S(Q + dq) / S(Q) and the VBS (i = 1, 2) and AFM (i = 3, 4, 5) order
 * parameters off the SO(5) line use them) for the current configuration of
 * every chain, by Wick's theorem from G(0), FP64. q_xy: host [n_q][2] integers:
 * on the torus momenta (qx, qy) in units of the grid, used as given (the form
 * factor depends on q itself, the orbital shift on qy mod N_phi); on the
 * sphere (l, m) with 0 <= m <= l <= N_phi - 1 and n_{-q} read as
 * n_{l,m}^dagger; 1 <= n_q <= 4096. out: host [n_chains][n_q][5] complex128
 * (re/im interleaved), owned by the caller. Per configuration the values are
 * complex; their average is real. Call between sweeps. Allocates small
 * temporaries. Synchronises. */
int cfqmc_structure_factors(cfqmc_ctx* c, const int32_t* q_xy, int32_t n_q, double* out);

/* ln of the fermion weight exp(sum_tau c_tau) det(1 + B(beta,0))^2 of one chain
 * (complex; the imaginary part is 0 mod 2 pi for the sign-free model), FP64. */
int cfqmc_logdet(cfqmc_ctx* c, int32_t chain, double* re, double* im);

/* Equal-time observables of the current configuration of one chain:
 * s_q0[5] = Re S^i_{q=0}, i = 1..5, and m2 = Re m^2_SO(5) (Results, eq. for
 * m^2_SO(5)), from G(l_tau) by Wick's theorem. */
int cfqmc_observables(cfqmc_ctx* c, int32_t chain, double* s_q0, double* m2);

/* Per-sweep series recorded at the end of every sweep since the last init (or
 * continued by cfqmc_restore), for autocorrelation times: writes up to max_len
 * values, returns the count in *len. which = 0: m^2_SO(5) (Results, order
 * parameter); 1: the action S = |phi|^2/2 - ln w_F, ln w_F = sum_tau Re c_tau +
 * 2 ln|det(1 + B(beta, 0))| (FP64 from the UDT stack); 2: the power of the q = 0
 * fields, sum_i (sum_tau phi^i_{tau,0})^2 / L. cfqmc_series is which = 0. */
int cfqmc_series_of(cfqmc_ctx* c, int32_t chain, int32_t which, double* out, int32_t max_len, int32_t* len);
int cfqmc_series(cfqmc_ctx* c, int32_t chain, double* out, int32_t max_len, int32_t* len);

/* Accept flags and ln A of every slice of the last sweep of one chain. */
int cfqmc_last_sweep(cfqmc_ctx* c, int32_t chain, int32_t* accepted, double* ln_a);

int cfqmc_get_eps(cfqmc_ctx* c, double* eps /* [n_chains] */);
int cfqmc_set_eps(cfqmc_ctx* c, const double* eps /* [n_chains] */);

/* Tile configuration chosen for (channel application, n x n GEMM). */
int cfqmc_tile_config(const cfqmc_ctx* c, int32_t* chan_cfg, int32_t* gemm_cfg);
/* The whole launch configuration chosen at create (autotuned or fixed), out
 * [5] host: channel-application configuration of the context's precision (the
 * FP32 one in mixed contexts), that of a mixed context's FP64 applications,
 * the n x n GEMM configuration, the exponential's N x N GEMM configuration,
 * and the launch form of precision-guarded applications (0: one launch per
 * precision class; 1, 2: one launch for both, three or four waves per SIMD). */
int cfqmc_launch_config(const cfqmc_ctx* c, int32_t* out);

/* Sampled HIP-event timing of the dominant kernel, the channel-exponential
 * application (two N x N x n complex products per chain on MFMA): when enabled,
 * one launch per slice is bracketed by events on the context's stream (up to
 * 4096 launches per sample set). enable = 1 starts a new sample set. */
int cfqmc_kernel_timing(cfqmc_ctx* c, int32_t enable);
/* Mean duration (ms) and count of the sampled launches, and the real flops one
 * launch performs: two N x N x n complex products per chain, 8 flops per complex
 * multiply-add, 16 N^2 n = 4 n^3 per chain (n = 2N). One application carries an
 * eighth of the wrap G -> B G B^-1, whose algorithmic work counted as two dense
 * n x n x n complex products is 16 n^3: 2 n^3 per application. Synchronises. */
int cfqmc_kernel_timing_read(cfqmc_ctx* c, double* avg_ms, int64_t* count, double* flops_per_launch);
/* The same for one channel application per slice of the Woodbury product
 * M = G + B'B^-1 (1 - G) (the left application of channel 2's inverse,
 * FP64 except in CFQMC_MIXED_ALL): the FP64 application's rate in a mixed run. */
int cfqmc_kernel_timing_read_woodbury(cfqmc_ctx* c, double* avg_ms, int64_t* count, double* flops_per_launch);

/* Heterogeneous batch: groups of chains with different shapes (N_phi, L_tau,
 * q-set, couplings), one context per group on its own HIP stream (default
 * priority). A batch sweep interleaves the slice steps of all groups on the
 * host so the groups' kernels run concurrently on the GPU. Contexts stay
 * owned by the batch; cfqmc_batch_context gives a view for measure_G,
 * logdet, init_fields and the other per-context calls. */
typedef struct cfqmc_batch cfqmc_batch;
int cfqmc_batch_create(const cfqmc_params* groups, int32_t n_groups, cfqmc_batch** out);
int cfqmc_batch_context(cfqmc_batch* b, int32_t group, cfqmc_ctx** ctx);
/* n_sweeps per group (equal_time = 0), or scaled by L_max / L_group so every
 * group runs the same number of slice steps (equal_time = 1). stats: NULL or
 * [total chains], group-major. Synchronises. */
int cfqmc_batch_sweep(cfqmc_batch* b, int32_t n_sweeps, int32_t equal_time, cfqmc_stats* stats);
/* The same interleaved sweep (n_sweeps per group) with replayed noise: replay
 * NULL (device noise for every group) or an array of n_groups host pointers,
 * entry g NULL or the group's buffer [n_chains_g][n_sweeps][l_tau_g][4 n_q_g + 1]
 * in the layout of cfqmc_sweep. stats as cfqmc_batch_sweep. Synchronises. */
int cfqmc_batch_sweep_replay(cfqmc_batch* b, int32_t n_sweeps, const double* const* replay, cfqmc_stats* stats);
/* The context holding chain `chain` of the batch (chains numbered group-major,
 * as the stats of cfqmc_batch_sweep) and the chain's index inside it
 * (local_chain may be NULL): a view for cfqmc_measure_G, cfqmc_logdet and the
 * other per-context calls, owned by the batch. CFQMC_EINVAL if chain is out of
 * range. */
int cfqmc_batch_get(cfqmc_batch* b, int32_t chain, cfqmc_ctx** view, int32_t* local_chain);
int cfqmc_batch_destroy(cfqmc_batch* b);

/* ---- Learned global proposal (self-learning Monte Carlo).
 * The paper samples with whole-slice Langevin moves (Methods, eq. Langevin
 * proposal); these calls add global moves proposed by a Markov chain on a
 * learned effective action S_eff(phi) = |phi|^2/2 + S_NN(phi) and accepted by
 * the exact weight: ln A = ln w_F(phi') - ln w_F(phi) + S_NN(phi') - S_NN(phi),
 * with ln w_F = sum_tau c_tau + 2 ln det(1 + B(beta,0)) computed from scratch in
 * FP64 (eq. green function / HS transform). The local sweep stays unchanged.
 *
 * S_NN: three-layer perceptron tanh(W1 x + b1) -> tanh(W2 . + b2) -> w3 . + b3,
 * output s_y * out + y_bar, on standardised features x = (f - mu) / sigma of:
 *   f[i][s][w]: mean over components c of |q|^2 shell s (s = floor(n_qbins r2 /
 *     (r2_max + 1)), r2 = qx^2 + qy^2) and frequencies of bin w (floor(n_wbins w /
 *     (L/2 + 1))) of |sum_tau phi^i_{tau,c} e^{-2 pi i w tau / L}|^2 / L;
 *   f[4 n_qbins n_wbins + i] = sum_tau phi^i_{tau,0} / sqrt(L).
 * n_feat = 4 n_qbins n_wbins + 4. Weights BF16 in every product (FP32 master
 * copy, Adam), FP32 accumulation, biases and activations. Parameters flat, FP32:
 * W1 [H][n_feat], b1 [H], W2 [H][H], b2 [H], w3 [H], b3 [1].
 * An SLMC object belongs to one context and uses its stream; it must be
 * destroyed before the context. */
typedef struct cfqmc_slmc cfqmc_slmc;
typedef struct {
  int32_t hidden;            /* H, default 256 */
  int32_t n_qbins, n_wbins;  /* feature bins, default 16 x 16 (n_wbins capped at L/2 + 1) */
  int32_t capacity;          /* stored training configurations, default 10000 */
  int32_t max_batch;         /* largest minibatch, default 256 */
  uint64_t seed;             /* initial weights, minibatch order, host uniforms */
} cfqmc_slmc_params;
typedef struct {
  int32_t accepted;          /* global move accepted */
  int32_t inner_accepted;    /* accepted HMC trajectories of the inner chain */
  double ln_a;               /* ln A of the global test */
  double d_lnw, d_snn;       /* ln w_F(phi') - ln w_F(phi), S_NN(phi') - S_NN(phi) */
  double max_abs_dh;         /* largest |Delta H| of the inner trajectories */
} cfqmc_slmc_move;

void cfqmc_slmc_default_params(cfqmc_slmc_params* p);
int cfqmc_slmc_create(cfqmc_ctx* c, const cfqmc_slmc_params* p, cfqmc_slmc** out);
int cfqmc_slmc_destroy(cfqmc_slmc* s);
int cfqmc_slmc_sizes(const cfqmc_slmc* s, int32_t* n_feat, int64_t* n_params, int32_t* n_data);
int cfqmc_slmc_set_params(cfqmc_slmc* s, const float* w);   /* host [n_params]; resets Adam */
int cfqmc_slmc_get_params(cfqmc_slmc* s, float* w);
int cfqmc_slmc_set_norm(cfqmc_slmc* s, const float* mu, const float* sigma, double y_bar, double s_y);
int cfqmc_slmc_get_norm(cfqmc_slmc* s, float* mu, float* sigma, double* y_bar, double* s_y);
/* Raw features of n host configurations phi [n][l_tau][4][n_q] -> feat [n][n_feat]. */
int cfqmc_slmc_features(cfqmc_slmc* s, const double* phi, int32_t n, float* feat);
/* S_NN of n host configurations, and dS_NN/dphi [n][l_tau][4][n_q] if grad_phi != NULL. */
int cfqmc_slmc_action(cfqmc_slmc* s, const double* phi, int32_t n, double* s_nn, double* grad_phi);
/* Gradient check of the learned action against a CPU reference: for n >= 1 host
 * configurations phi [n][l_tau][4][n_q], the GPU forward value fwd_out[n] =
 * S_NN(phi) and its field gradient grad_out [n][l_tau][4][n_q] = dS_NN/dphi
 * (features, BF16 network and the backward pass through the binning and the
 * DFT run in the library's kernels; outputs FP64, host, owned by the caller).
 * Both outputs are required (else CFQMC_EINVAL). Synchronises. */
int cfqmc_slmc_grad_check(cfqmc_slmc* s, const double* phi, int32_t n, double* fwd_out, double* grad_out);
/* Mean squared error of the network on n <= max_batch standardised inputs x [n][n_feat]
 * against standardised targets y [n], its parameter gradient [n_params] and the outputs
 * [n] (any output may be NULL). No parameter update. */
int cfqmc_slmc_loss_grad(cfqmc_slmc* s, const float* x, const double* y, int32_t n, double* loss, float* grad,
                         float* out);
/* Append the current configuration of every chain (features and -ln w_F). */
int cfqmc_slmc_collect(cfqmc_slmc* s);
int cfqmc_slmc_clear_data(cfqmc_slmc* s);
/* Adam training on the stored configurations (MSE on standardised targets).
 * refit_norm = 1 (or the first call) sets mu, sigma, y_bar, s_y from the data.
 * loss_out: mean minibatch loss of the last epoch. */
int cfqmc_slmc_train(cfqmc_slmc* s, int32_t epochs, int32_t batch, double lr, int32_t refit_norm, double* loss_out);
/* Adam training with a held-out set and early stopping: the last n_val stored
 * configurations (collected last, e.g. the final sweeps of every chain) are
 * never trained on; after each epoch over the others (shuffled minibatches)
 * the validation MSE on them is evaluated, and training stops once it has not
 * improved for `patience` epochs (or after max_epochs). The parameters of the
 * best validation epoch are kept. refit_norm = 1 (or the first call) sets mu,
 * sigma, y_bar, s_y from the training configurations only. Outputs (any may be
 * NULL): the last epoch's mean minibatch training loss, the best validation
 * loss (standardised targets) and its epoch (0-based). CFQMC_ESTATE with fewer
 * than two training configurations. Synchronises. */
int cfqmc_slmc_train_heldout(cfqmc_slmc* s, int32_t max_epochs, int32_t batch, double lr, int32_t refit_norm,
                             int32_t n_val, int32_t patience, double* train_loss, double* val_loss,
                             int32_t* best_epoch);
/* Subspace of the learned global move. mode 0 moves every field (the
 * default); 1 moves only component 0 of every channel and slice (q = 0 on the
 * torus, (l, m) = (0, 0) on the sphere); 2 moves only the four slice-uniform
 * amplitudes A_i = sum_tau phi^i_{tau,0} / sqrt(L) per chain (every slice's
 * component 0 shifted together), the field modes local whole-slice moves relax
 * most slowly. The HMC on the effective action runs in that subspace (its
 * momenta alone are nonzero); the exact Metropolis test is unchanged.
 * EINVAL for another mode. */
int cfqmc_slmc_set_subspace(cfqmc_slmc* s, int32_t mode);

/* One global move of every chain: n_traj HMC trajectories of n_leap leapfrog steps
 * of size step on S_eff, each with its own Metropolis test, then the exact test.
 * Accepted chains keep phi', rejected chains return to phi; the chain state (UDT
 * stacks, G) is rebuilt from scratch. replay: NULL (Philox momenta, host uniforms)
 * or host [n_chains][n_traj * l_tau * 4 * n_q + n_traj + 1]: the momenta of every
 * trajectory, the inner uniforms, then the uniform of the global test.
 * out: NULL or [n_chains]. Synchronises. */
int cfqmc_slmc_global_move(cfqmc_slmc* s, int32_t n_traj, int32_t n_leap, double step, const double* replay,
                           cfqmc_slmc_move* out);
/* Proposal phi' of the last global move of one chain (host [l_tau][4][n_q]). */
int cfqmc_slmc_last_proposal(cfqmc_slmc* s, int32_t chain, double* phi_out);

/* The stabilisation check the sweep applies at every FP64 recomputation, on
 * caller data: for count pairs of n x n complex128 matrices X_z, Y_z (device,
 * contiguous, row-major, stride n*n, owned by the caller), out[2z] =
 * max|X_z - Y_z| and out[2z + 1] = max|X_z - Y_z| / max|Y_z| (host [count][2]).
 * A non-finite entry of X_z or Y_z gives +inf in both and the call returns
 * CFQMC_ENUMERIC, as a sweep does for such a state. hip_stream: a hipStream_t
 * (NULL = default). Allocates a small temporary. Synchronises. */
int cfqmc_green_maxdiff(const void* x_dev, const void* y_dev, int32_t n, int32_t count, void* hip_stream,
                        double* out);

/* Message of the last error of a context; with c == NULL, the message of the
 * last cfqmc_create that failed on the calling thread. */
const char* cfqmc_last_error(const cfqmc_ctx* c);

#ifdef __cplusplus
}
#endif
#endif
