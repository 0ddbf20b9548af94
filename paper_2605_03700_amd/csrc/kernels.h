// Host-side launch interface of the device kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

// GEMM_PQ: D = C + alpha A B, D2 = C - alpha A B.
// GEMM_SQUARE: one step of repeated squaring, step number pred_thresh, of the
// matrices whose squaring count pred[...] exceeds it (the others return at once).
enum { GEMM_NORMAL = 0, GEMM_PQ = 1, GEMM_SQUARE = 2 };

// Launch checking: with CFQMC_DEBUG_SYNC=1 in the environment every launch is
// followed by a device synchronisation and an error check naming the kernel.
int cfqmc_debug_sync();
void cfqmc_post_launch(const char* name);

struct GemmArgs {
  int M, N, K;
  int opA, opB;             // 0: as stored, 1: conjugate transpose
  MatRef A, B, C, D, D2;    // C may have p == nullptr (beta ignored)
  MatRef E, E2;             // with pred: final destinations of matrices that need no further squaring
  int nz2;                  // inner batch count (z = z1 * nz2 + z2)
  double2 alpha, beta;
  const double2* alpha_dev; // optional per-batch factor, index z1*ad_s1 + z2*ad_s2
  int ad_s1, ad_s2;
  int mode;
  const int* pred;          // squaring count per matrix (GEMM_PQ, GEMM_SQUARE), index z1*pred_s1 + z2*pred_s2
  int bandA, bandB;         // >= 0: A (resp. B) vanishes outside the wrap-around band
                            // |(col - row) mod K| <= band; k slabs that meet no band entry of
                            // the tile's rows (columns) are skipped (their terms are exact zeros)
  int herm;                 // GEMM_NORMAL with a Hermitian result (M == N; alpha, beta real): only the
                            // tiles on and above the diagonal are computed, each strictly upper tile
                            // also writes its conjugate transpose
  int pred_s1, pred_s2, pred_thresh;
};

struct ChanArgs {
  int N;                    // orbital block size
  int n_other;              // columns of M (LEFT) or rows of M (RIGHT)
  const double2* M; int ldM; long long sM;
  const double2* X0; const double2* X1; int ldX; long long sX;   // orbital blocks e^{+-alpha h}
  int one_minus;            // use (1 - M) instead of M (left, non-rotating channel)
  const double2* Cadd; int ldC; long long sC;   // optional addend
  double2* Y; int ldY; long long sY;
  double2* Y2;              // optional second copy of the output (same layout as Y)
  const int* chain_sel;     // optional [chain]: only chains with chain_sel[z] == sel_want are computed
  int sel_want;
};

// Tile configurations: zgemm 0..3; chan_apply 0..19 (a fixed tile_cfg applies to both;
// 8..13, 17 and 18 accumulate the FP32 path in FP32 over the whole k range, 12,
// 13, 17 and 18 with three real products per complex step; 14 has three-product
// slabs with an FP64 accumulation point per slab, as 0..7, 15, 16 and 19; 15..18
// are 8- and 16-wave workgroups of 16 x 16 wave tiles; 19 splits the two valley
// products of a 32 x 32 tile over eight waves in FP64 and is 1 in FP32).
#define CFQMC_GEMM_CFGS 4
#define CFQMC_CHAN_CFGS 20
// FP32 path: does configuration cfg keep an FP64 accumulation point per slab?
inline bool chan_cfg_acc64(int cfg) { return cfg < 8 || cfg == 14 || cfg == 15 || cfg == 16 || cfg == 19; }
void launch_zgemm(const GemmArgs& g, int nbatch, int mixed, int cfg, hipStream_t s);
// One launch for both precision classes of a guarded mixed context
// (c.chain_sel[z] = 1: FP64, else the FP32 correction form of configuration
// cfg32). variant 1: registers as allocated (three waves per SIMD); 2: held to
// four waves per SIMD. false (nothing launched) unless cfg32 is 1 or 12 and
// cfg64 one of 1, 8, 12, 14 (the same 32 x 32 single-stage tile).
bool launch_chan_apply_dual(const ChanArgs& c, int left, int rot, int nbatch, int cfg32, int cfg64, int variant,
                            hipStream_t s);
// rot: 0 none (channels 0, 3), 1 tau_x (channel 1), 2 tau_y (channel 2)
void launch_chan_apply(const ChanArgs& c, int left, int rot, int nbatch, int mixed, int cfg, hipStream_t s);

// ---- dense linear algebra (linalg.hip), one matrix per batch entry
// LU with partial pivoting (pivot=1) or without (pivot=0), in place; ipiv
// [batch][n]; logdet[batch] = ln det A (complex, principal imaginary part).
// only_if: optional [batch] predicate (run only where nonzero); restore: optional
// source copied into A before factorising (fallback after launch_lu_np).
void launch_lu(double2* A, int n, int lda, long long sA, int* ipiv, int sP, double2* logdet, int pivot,
               int nbatch, hipStream_t s, const int* only_if = nullptr, const double2* restore = nullptr);
// LU without pivoting (ipiv = identity); flag[batch] = 1 if a multiplier exceeds lmax_allowed.
void launch_lu_np(double2* A, int n, int lda, long long sA, int* ipiv, int sP, double2* logdet, int* flag,
                  double lmax_allowed, int nbatch, hipStream_t s);
// X <- X * A^{-1} with A = P^T L U from launch_lu. upper_only: X <- X U^{-1}.
// mixed: the block products in FP32 with an FP64 accumulation point per
// 16-deep step, for every chain or, with sel64, for the chains with
// sel64[z] == 0 (the others in FP64).
void launch_rsolve(const double2* X, int ldx, long long sX, double2* Y, int ldy, long long sY,
                   const double2* LU, int ldlu, long long sLU, const int* ipiv, int sP, int n, int upper_only,
                   int nbatch, hipStream_t s, double2* work, int mixed = 0, const int* sel64 = nullptr);
// Workspace of launch_rsolve (inverted diagonal blocks), in double2 per batch entry.
inline long long rsolve_work_size(int n) { return (long long)((n + 15) / 16) * 512; }
void launch_set_identity(double2* A, int n, int lda, long long sA, int nbatch, hipStream_t s);
void launch_copy(const double2* X, double2* Y, long long count, long long sX, long long sY, int nbatch,
                 hipStream_t s);
// p[0..count) = v (a kernel, so that callers under stream capture record no memset node)
void launch_fill(double* p, long long count, double v, hipStream_t s);
// Y[:, k] = X[:, k] * d[k]   (d real, per batch stride sd) ; inv: divide instead
void launch_colscale(const double2* X, int ldx, long long sX, double2* Y, int ldy, long long sY,
                     const double* d, long long sd, int n_rows, int n_cols, int inv, int nbatch, hipStream_t s);
// running max |X - Y| (out[so z]) and max |X - Y| / max |Y| (out[so z + 1]) per batch
// entry; out[so z + 2], out[so z + 3] are scratch that must start at zero. A
// non-finite entry of X or Y makes both maxima +inf. last: optional [batch][2],
// receives max |X - Y| and max |Y| of this call.
void launch_maxdiff(const double2* X, const double2* Y, int n, long long sX, double* out, int nbatch,
                    hipStream_t s, int so = 4, double* last = nullptr);
// Precision guard of the mixed path, after a recomputation: count[z] += sel[z]
// (the block that ended ran in FP64 from some slice on), then from last [batch][2]
// (max |G_updated - G_FP64|, max |G_FP64| of the block just ended) set
// sel[z] = 1 (FP64 applications for the next block) if max |G_FP64| > gmax or the
// error > err, else 0; gmax_run[z] = max(gmax_run[z], max |G_FP64|).
void launch_precision_guard(const double* last, int* sel, int* count, double* gmax_run, double gmax, double err,
                            int nbatch, hipStream_t s);

// ---- UDT stabilisation helpers (linalg.hip)
// Column norms of W (n x n) -> nrm; descending-order permutation perm.
void launch_colnorm_sort(const double2* W, int n, long long sW, double* nrm, int* perm, int nbatch,
                         hipStream_t s);
// A[:, k] = W[:, perm[k]] / nrm[perm[k]]
void launch_permute_normalize(const double2* W, int n, long long sW, const double* nrm, const int* perm,
                              double2* A, int nbatch, hipStream_t s);
// Cholesky factor from an unpivoted LU of a Hermitian PD Gram matrix:
// R = diag(1/sqrt(u_kk)) U (upper triangle of LU), sqrtd[k] = sqrt(u_kk).
// A pivot that is not positive and finite sets bit 2 of *err (when err != nullptr).
void launch_chol_from_lu(const double2* LU, int n, long long sLU, double2* R, double* sqrtd, int nbatch,
                         hipStream_t s, int* err);
// From Rt (upper, n x n), norms and permutation: D' = |diag(Rt) * nrm|,
// T'[i][perm[k]] = Rt[i][k] * nrm[perm[k]] / D'[i].
void launch_udt_finish(const double2* Rt, int n, long long sR, const double* nrm, const int* perm,
                       double* Dout, long long sD, double2* Tp, int nbatch, hipStream_t s);
// Y = Dlmax^-1 K Drmax^-1 + Dlmin M Drmin (Loh split), n x n
void launch_loh_combine(const double2* K, const double2* Mm, const double* Dl, long long sDl, const double* Dr,
                        long long sDr, double2* Y, int n, int nbatch, hipStream_t s);
// d -> 1/max(d,1) (mode 0) ; used for column scalings of the Loh formula
void launch_dmax_inv(const double* d, long long sd, double* out, int n, int nbatch, hipStream_t s);
// sum ln max(D,1) per batch
void launch_sum_log_dmax(const double* d, long long sd, int n, double* out, int nbatch, hipStream_t s);
// d -> min(d, 1), the small part of the same split (out stride n)
void launch_dmin1(const double* d, long long sd, double* out, int n, int nbatch, hipStream_t s);
// A = scale * diag(d), n x n
void launch_diag_set(double2* A, int n, long long sA, const double* d, long long sd, double scale, int nbatch,
                     hipStream_t s);

// ---- model kernels (qmc.hip)
struct ModelDev {
  int N, n, nq, L;
  // h-building table: per shift d (0..N-1) terms [hoff[d], hoff[d+1]); hdiag the
  // nhdiag shifts that carry a term (h is zero on every other diagonal)
  const int* hoff;
  const int* hdiag;
  int nhdiag;
  const int* h_cre; const int* h_cim; const int* h_qx; const int* h_qy; const int* h_dag;
  const double* h_sgn; const double* h_scale; const double* h_F;
  // trace table: per row r (0..nrow-1) components [toff[r], toff[r+1])
  int nrow, maxrow;   // rows and the largest component count of one row
  const int* toff; const int* t_qy; const int* t_qx; const int* t_kind; const int* t_comp;
  const double* t_F;
  const double* beta;       // background c-number per component [nq]
  const double2* phase;     // exp(i pi m / N), m = 0..2N-1
  const double* cw;         // sphere: orbital weights [nq][N] replacing F e^{i phase} (nullptr on the torus)
  const double* tw;         // sphere: the same per trace-table entry t, orbital-major [N][ntw]
  int ntw;
};

struct ChainDev {
  int nchain;
  const double2* alpha;     // [chain][4]
  const double2* U;         // [4][2][2] valley rotations
};

// h_i = sum_c phi^i_c q_c for all batch entries; phi [batch][4][nq] (stride sphi), h [batch][4][N][N].
// Writes the diagonals listed in m.hdiag only: the others must hold zeros
// (the caller clears h once).
void launch_build_h(const ModelDev& m, const double* phi, long long sphi, double2* h, long long sh, int nbatch,
                    hipStream_t s);
// exponential helper: norm estimate and Taylor coefficients per (batch, channel)
void launch_exp_coef(const double2* X2, const double2* X3, int N, const double2* alpha, int alpha_per_batch,
                     double* coef, int* sq, int smax, double theta, int* err, int nbatch4, hipStream_t s);
// Coefficients of the exponential per (entry, channel) matrix: e_0..e_6 (even part),
// o_0..o_6 (odd part), then the complex scale of h (alpha / 2^s).
#define EXP_NC 16
// E and O of the exponential's even/odd split from x = h^2, x^2, x^3 and the
// coefficients of exp_coef (one fused pass; Hermitian tiles only)
void launch_exp_eo(const double2* H2, const double2* X2, const double2* X3, const double* coef, int N, double2* Eo,
                   double2* Oo, int nmat, hipStream_t s);

struct StepArgs {
  int N, n, nq, L, tau;      // tau 0-based slice index
  int nchain;                // chains in the launch (set by the launchers)
  const double2* G[4];       // frames G_0..G_3 (batch stride sG)
  long long sG;
  const double* phi; long long sphi;     // phi of slice tau (batch stride = chain stride)
  double* phip; long long sphip;
  const double2* alpha;      // [chain][4]
  const double* eps;         // [chain]
  const double* noise; long long snoise; // replay slice: [4 nq + 1] per chain, or null
  uint64_t seed; long long counter;      // RNG counter (sweep * L + slice) when counter_dev is null
  const long long* counter_dev;          // sweep counter in device memory: counter = *counter_dev * L + tau
  double* part;              // partial sums [chain][nblk][4]
  int nblk;
  const double2* lndetM;     // [chain]
  double* lnA;               // [chain]
  int* accept;               // [chain]
  double* stat;              // [chain][8] running stats
  double* u_out;             // [chain] uniform used (diagnostics)
};
void launch_drift_propose(const ModelDev& m, const StepArgs& a, int nchain, hipStream_t s);
void launch_drift_mh(const ModelDev& m, const StepArgs& a, int nchain, hipStream_t s);

// Metropolis-Hastings decision from the drift kernels' partial sums, then
// commit of the accepted slice move. sel (precision guard, or null): set to 1
// for a chain whose new G has an entry of modulus above gmax (never cleared
// here).
void launch_commit(const StepArgs& a, int nchain, const double2* Gp, const double2* G0, double2* G, long long nn,
                   long long sG, const double* phip, long long sphip, double* phi_tau, long long sphi, int nphi,
                   const double2* PQp, long long sPQp, double2* PQ_tau, long long sPQ, long long npq,
                   int* acc_count, hipStream_t s, int* sel = nullptr, double gmax = 0.0);
void launch_eps_update(double* eps, const int* acc_count, int L, double r0, double deps, double emin,
                       double emax, int adapt, int nchain, hipStream_t s);
// S^i_{q=0} (i=1..5) and m^2 from the spin-block G; out [chain][8]
void launch_observables(const double2* G, long long sG, int N, double F0, double* out, long long sout,
                        int nchain, hipStream_t s);
// imaginary-time correlator <n^i_{q=0}(tau) n^i_{q=0}(0)>, i = 1..5, of every chain for
// one tau from X = G(tau,0), Y = G(0,tau), W = G(tau,tau) (spin block); tr0 [chain][2]
// traces of G(0), written when first != 0; out[chain * sout + i] complex
void launch_disp_corr(const double2* X, const double2* Y, const double2* W, long long sG, int N, double F0,
                      double2* tr0, int first, double2* out, long long sout, int nchain, hipStream_t s);
// S^i_q (i = 1..5) at the momenta qxy[2 iq], qxy[2 iq + 1] (device) of every chain from
// the spin-block G; on the sphere the pairs are (l, m) and qw [nql][N] holds the rows'
// weights n_{l,m}[k, k + m] (nullptr on the torus); out[(chain * nql + iq) * 5 + i] complex
void launch_structure_factors(const double2* G, long long sG, int N, const int* qxy, int nql, const double* qw,
                              double2* out, int nchain, hipStream_t s);
// background sum over slices: c[chain] = sum_tau alpha0 * phi0 . beta
void launch_background(const ModelDev& m, const double* phi, long long sphi_chain, const double2* alpha,
                       double2* out, int nchain, hipStream_t s);
// per chain |phi|^2 and the q = 0 power sum_i (sum_tau phi^i_{tau,0})^2 / L
void launch_field_sums(const double* phi, long long sphi, int L, int nq, double* sq, double* q0, int nchain,
                       hipStream_t s);
// series entry k: S = |phi|^2/2 - ln w_F from the UDT pieces, and the q = 0 power
void launch_action_series(const double2* ldY, const double2* ldU, const double* sdm, const double2* bg,
                          const double* sq, const double* q0, const double* m2, int m2_stride, double* ser_m,
                          double* ser_s, double* ser_p, long long cap, const int* k_dev, int nchain, hipStream_t s);
// sweep counter += 1 and series length += 1 (up to cap), on the device
void launch_sweep_advance(long long* counter, int* series_len, int cap, hipStream_t s);
// 4N expansion of the spin block
void launch_expand4n(const double2* G, int n, double2* G4, hipStream_t s);

// ---- learned global proposal (slmc.hip)
void launch_slmc_dft(const double* phi, long long sphi, int L, int nq, int nw, const float* twc, const float* tws,
                     float* Xre, float* Xim, long long sX, int nb, hipStream_t s);
void launch_slmc_bin(const float* Xre, const float* Xim, long long sX, int nq, int nw, int L, int nqb, int nwb,
                     const int* shell_off, const int* shell_comp, const int* w_off, float* feat, int F, int nb,
                     hipStream_t s);
void launch_slmc_standardize(const float* feat, int F, int Fp, const float* mu, const float* sig, uint16_t* xb,
                             int nb, hipStream_t s);
void launch_slmc_gemm(int at, int bt, int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb,
                      float* C, int ldc, const float* bias, int act, uint16_t* Cb, int ldcb, hipStream_t s);
void launch_slmc_head(const uint16_t* a2b, int H, const uint16_t* w3b, const float* b3, float* out, int nb,
                      hipStream_t s);
void launch_slmc_dout(const float* out, const float* y, int nb, int mode, float const_d, float* dout, double* loss_acc,
                      hipStream_t s);
void launch_slmc_dz2(const float* dout, const uint16_t* w3b, const float* a2, int H, float* dz2, uint16_t* dz2b, int nb,
                     hipStream_t s);
void launch_slmc_tanh_bwd(const float* dA, const float* a, long long n, float* dz, uint16_t* dzb, hipStream_t s);
void launch_slmc_colsum(const float* X, int nb, int H, float* out, hipStream_t s);
void launch_slmc_head_grad(const float* dout, const uint16_t* a2b, int nb, int H, float* gw3, float* gb3,
                           hipStream_t s);
void launch_slmc_adam(float* p, const float* g, float* m, float* v, long long n, double lr, int t, hipStream_t s);
void launch_slmc_to_bf16(const float* src, int rows, int cols, uint16_t* dst, int ldd, hipStream_t s);
void launch_slmc_gather(const uint16_t* xall, const float* yall, int Fp, const int* idx, int nb, uint16_t* xb, float* yb,
                        hipStream_t s);
void launch_slmc_dx_to_gf(const float* dX, int Fp, const float* sig, int F, float scale, float* gf, int nb,
                          hipStream_t s);
void launch_slmc_vjp(const float* Xre, const float* Xim, long long sX, const float* gf, int F, int nq, int nw, int L,
                     int nqb, int nwb, const int* shell, const int* wbin, const float* inv_cnt, const float* twc,
                     const float* tws, double* grad, long long sg, int nb, hipStream_t s);
void launch_slmc_momenta(double* p, long long n, int nb, uint64_t key, long long counter, const double* replay,
                         long long s_replay, int mode, int nq, hipStream_t s);
// subspace mode: 0 every field, 1 component 0 of every channel and slice, 2 the four
// slice-uniform component-0 amplitudes per chain (momenta at slice 0)
void launch_slmc_kick(double* p, const double* phi, const double* g, double h, long long n, int mode, int nq, int L,
                      int nb, hipStream_t s);
void launch_slmc_drift(double* phi, const double* p, double h, long long n, int mode, int nq, int L, int nb,
                       hipStream_t s);
void launch_slmc_sumsq(const double* x, long long n, double* out, int nb, hipStream_t s);
void launch_slmc_select(const int* flag, int want, const double* src, double* dst, long long n, int nb, hipStream_t s);
