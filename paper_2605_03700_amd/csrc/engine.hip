// Chain state, sweep orchestration and the C ABI (include/cfqmc.h).
//
// Per slice tau of a sweep (all chains of the context advance together, every
// step is one launch over all chains, no host synchronisation):
//   1. wrap  G_i = E_i G_{i+1} E_i^{-1}, i = 3..0, G_4 = G(tau-1), G_0 = G(tau)
//   2. drift from the frames G_i, Langevin proposal phi' (eq. Langevin proposal)
//   3. h'_i and the channel exponentials P' = e^{alpha h'}, Q' = e^{-alpha h'}
//   4. M = G_0 + B' B^{-1} (1 - G_0) = 1 + Delta (1 - G_0), Delta = B' B^{-1} - 1
//   5. LU(M): the determinant ratio det(1 + B'...)/det(1 + B...) = det M
//   6. G' = G_0 M^{-1} (Woodbury update, rank n for a whole-slice move)
//   7. drift at phi' from the frames of G', Metropolis-Hastings decision
//   8. commit G, phi, P/Q of the slice on acceptance
// Every n_stab slices the block product C_b is formed in FP64, the left UDT
// stack is advanced, and G is recomputed from the stacks (Loh et al. split)
// in FP64; the difference to the updated G is recorded. After the sweep the
// right stack is rebuilt from the final slices for the next sweep.
#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cfqmc.h"
#include "kernels.h"


namespace {

struct HostTables {
  std::vector<int> comp_kind, comp_qx, comp_qy;   // kind 0 S, 1 A, 2 C
  std::vector<double> comp_F, beta;
  std::vector<long long> comp_r2;   // |q|^2 (torus) or l (l + 1) (sphere): shells of the learned features
  // sphere: per component the orbital weights w[c * N + r] = n_{l,m}[r, r + m]
  // (q_x = 0, q_y = -m and F = 1 in the tables, so phases are 1 and the
  // weights carry the density operator); t_w the same per trace-table entry,
  // orbital-major (t_w[k * n_t + t]) so the drift's threads read it coalesced
  std::vector<double> comp_w, t_w;
  // h table
  std::vector<int> hoff, h_cre, h_cim, h_qx, h_qy, h_dag;
  std::vector<int> hdiag;   // shifts d that carry a term
  std::vector<double> h_sgn, h_scale, h_F;
  // trace table
  std::vector<int> toff, t_qy, t_qx, t_kind, t_comp;
  std::vector<double> t_F;
  std::vector<double2> phase;
};

double form_factor(int qx, int qy, int N) {
  return std::exp(-2.0 * M_PI * (double)(qx * qx + qy * qy) / (4.0 * N)) / (4.0 * M_PI * std::sqrt((double)N));
}

int wrap_bz(int v, int N) {
  int r = ((v % N) + N) % N;
  return r > N / 2 ? r - N : r;
}

// Orbital weights of the sphere's density operators (Methods, spherical
// regularization): n_{l,m}[r, r + m] for 0 <= m <= l <= 2s = N - 1, rows r of
// the LLL orbitals m_r = r - s, in W[(l * N + m) * N + r] (zero where r + m >= N),
// from the printed 3j form
//   n_{l,m}[r, r+m] = (-1)^(r+m) (2s+1) sqrt(2l+1)/2 3j(s l s; -m_r, -m, m_r+m) 3j(s l s; -s, 0, s).
// Each 3j family f(l) = 3j(s l s; a, b, c) over l = |b|..2s (cyclically
// 3j(l s s; b, c, a)) follows from the Schulten-Gordon three-term recursion
//   l A(l+1) f(l+1) + B(l) f(l) + (l+1) A(l) f(l-1) = 0,
//   A(l) = sqrt(l^2 ((2s+1)^2 - l^2)(l^2 - b^2)), B(l) = -(2l+1) l(l+1)(c - a),
// run downwards from l = 2s (A(2s+1) = 0) in extended precision, normalised by
// sum_l (2l+1) f(l)^2 = 1, with sign f(2s) = (-1)^(b) (the closed form at the
// largest l).
std::vector<double> sphere_weights(int N) {
  typedef long double R;
  const int ts = N - 1;
  std::vector<double> W((size_t)N * N * N, 0.0);
  // family of 3j(s l s; a, b, c) with doubled a, c and integer b = -m
  auto family = [&](int ta, int m, std::vector<R>& f) {
    const int b = -m, lmin = std::abs(b);
    f.assign(N + 1, 0.0L);
    const R a = ta / 2.0L, c = -(a + b);
    auto A = [&](int l) { return std::sqrt((R)l * l * ((R)(ts + 1) * (ts + 1) - (R)l * l) * ((R)l * l - (R)b * b)); };
    auto Bc = [&](int l) { return -(2.0L * l + 1) * l * (l + 1.0L) * (c - a); };
    f[ts] = 1.0L;
    for (int l = ts; l > lmin; --l) f[l - 1] = -(l * A(l + 1) * f[l + 1] + Bc(l) * f[l]) / ((l + 1) * A(l));
    R nrm = 0.0L;
    for (int l = lmin; l <= ts; ++l) nrm += (2.0L * l + 1) * f[l] * f[l];
    const R sc = ((std::abs(b) % 2) ? -1.0L : 1.0L) / std::sqrt(nrm);
    for (int l = lmin; l <= ts; ++l) f[l] *= sc;
  };
  std::vector<R> g, f;
  family(-ts, 0, g);   // 3j(s l s; -s, 0, s)
  for (int m = 0; m < N; ++m)
    for (int r = 0; r + m < N; ++r) {
      const int tmr = 2 * r - ts;   // 2 m_r
      family(-tmr, m, f);           // 3j(s l s; -m_r, -m, m_r + m)
      for (int l = m; l <= ts; ++l) {
        const R v = (((r + m) % 2) ? -1.0L : 1.0L) * (R)(ts + 1) * std::sqrt(2.0L * l + 1) / 2.0L * f[l] * g[l];
        W[((size_t)l * N + m) * N + r] = (double)v;
      }
    }
  return W;
}

// Components on the sphere, per channel: sqrt(2) n_{l,0} for l = 0..2s, then
// for m = 1..2s and l = m..2s the pair n_{l,m} + n_{l,m}^+ (A) and
// i (n_{l,m} - n_{l,m}^+) (C). Background -2 tr of each m = 0 component.
void sphere_components(int N, HostTables& T) {
  const std::vector<double> W = sphere_weights(N);
  auto add = [&](int kind, int l, int m) {
    T.comp_kind.push_back(kind); T.comp_qx.push_back(0); T.comp_qy.push_back(-m);
    T.comp_F.push_back(1.0);
    T.comp_r2.push_back((long long)l * (l + 1));
    double tr = 0.0;
    for (int r = 0; r < N; ++r) {
      const double w = W[((size_t)l * N + m) * N + r];
      T.comp_w.push_back(w);
      if (m == 0) tr += w;
    }
    T.beta.push_back(kind == 0 ? -2.0 * std::sqrt(2.0) * tr : 0.0);
  };
  for (int l = 0; l < N; ++l) add(0, l, 0);
  for (int m = 1; m < N; ++m)
    for (int l = m; l < N; ++l) { add(1, l, m); add(2, l, m); }
}

// Momentum set and components (see cfqmc.h for the ordering).
bool build_components(const cfqmc_params& p, HostTables& T, std::string& err) {
  const int N = p.n_phi;
  if (p.q_mode == CFQMC_Q_SPHERE) {
    sphere_components(N, T);
  } else {
    std::vector<std::pair<int, int>> qs;
    if (p.q_mode == CFQMC_Q_PAPER || p.q_mode == CFQMC_Q_RADIUS) {
      int R;
      if (p.q_mode == CFQMC_Q_PAPER) R = (int)std::ceil(std::sqrt(4.0 * N * std::log(100.0) / (2.0 * M_PI))) + 1;
      else R = (int)std::ceil(p.q_max * std::sqrt(N / (2.0 * M_PI))) + 1;
      for (int qy = -R; qy <= R; ++qy)
        for (int qx = -R; qx <= R; ++qx) {
          const double q2 = (double)(qx * qx + qy * qy);
          bool keep;
          if (p.q_mode == CFQMC_Q_PAPER) keep = std::exp(-2.0 * M_PI * q2 / (4.0 * N)) > 0.01;
          else keep = (2.0 * M_PI / N) * q2 <= p.q_max * p.q_max * (1 + 1e-12);
          if (keep) qs.push_back({qx, qy});
        }
    } else if (p.q_mode == CFQMC_Q_BZ) {
      const int lo = -(N / 2) + (N % 2 == 0 ? 1 : 0), hi = N / 2;
      for (int qy = lo; qy <= hi; ++qy)
        for (int qx = lo; qx <= hi; ++qx) qs.push_back({qx, qy});
    } else if (p.q_mode == CFQMC_Q_LIST) {
      if (!p.q_list || p.n_q_list <= 0) { err = "q_list missing"; return false; }
      for (int i = 0; i < p.n_q_list; ++i) qs.push_back({p.q_list[2 * i], p.q_list[2 * i + 1]});
      for (auto& q : qs) {
        if (std::count(qs.begin(), qs.end(), q) != 1) { err = "q_list has duplicates"; return false; }
        if (std::find(qs.begin(), qs.end(), std::make_pair(-q.first, -q.second)) == qs.end()) {
          err = "q_list not closed under q -> -q";
          return false;
        }
      }
    } else {
      err = "unknown q_mode";
      return false;
    }
    // (kind 'P' pair or 'S' self) items, q = 0 first
    struct Item { int self, qx, qy; };
    std::vector<Item> items;
    bool has0 = false;
    for (auto& q : qs) {
      if (q.first == 0 && q.second == 0) { has0 = true; continue; }
      if (p.q_mode == CFQMC_Q_BZ) {
        const int px = wrap_bz(-q.first, N), py = wrap_bz(-q.second, N);
        if (px == q.first && py == q.second) items.push_back({1, q.first, q.second});
        else if (std::make_pair(q.second, q.first) > std::make_pair(py, px)) items.push_back({0, q.first, q.second});
      } else if (q.second > 0 || (q.second == 0 && q.first > 0)) {
        items.push_back({0, q.first, q.second});
      }
    }
    std::sort(items.begin(), items.end(), [](const Item& a, const Item& b) {
      return std::make_pair(a.qy, a.qx) < std::make_pair(b.qy, b.qx);
    });
    if (has0) { T.comp_kind.push_back(0); T.comp_qx.push_back(0); T.comp_qy.push_back(0); }
    for (auto& it : items) {
      if (it.self) { T.comp_kind.push_back(0); T.comp_qx.push_back(it.qx); T.comp_qy.push_back(it.qy); }
      else {
        for (int k = 1; k <= 2; ++k) { T.comp_kind.push_back(k); T.comp_qx.push_back(it.qx); T.comp_qy.push_back(it.qy); }
      }
    }
    const int nq = (int)T.comp_kind.size();
    if (nq == 0) { err = "empty momentum set"; return false; }
    T.comp_F.resize(nq);
    T.beta.resize(nq);
    T.comp_r2.resize(nq);
    for (int c = 0; c < nq; ++c) {
      T.comp_r2[c] = (long long)T.comp_qx[c] * T.comp_qx[c] + (long long)T.comp_qy[c] * T.comp_qy[c];
      const int qx = T.comp_qx[c], qy = T.comp_qy[c];
      const double F = form_factor(qx, qy, N);
      T.comp_F[c] = F;
      // background c-number -2 tr(q_c): only shifts q_y = 0 (mod N) have a diagonal
      double tr_re = 0.0, tr_im = 0.0;
      if (((qy % N) + N) % N == 0) {
        for (int k = 1; k <= N; ++k) {
          const double a = M_PI * (double)((2 * k - qy) * qx) / N;
          tr_re += F * std::cos(a);
          tr_im += F * std::sin(a);
        }
      }
      const int kind = T.comp_kind[c];
      T.beta[c] = kind == 0 ? -2.0 * std::sqrt(2.0) * tr_re : (kind == 1 ? -4.0 * tr_re : 4.0 * tr_im);
    }
  }
  const int nq = (int)T.comp_kind.size();
  // h table grouped by shift d = (row - col) mod N
  std::vector<std::vector<int>> by_shift(N);
  struct HT { int cre, cim, qx, qy, dag; double sgn, scale, F; };
  std::vector<HT> terms;
  for (int c = 0; c < nq; ++c) {
    const int kind = T.comp_kind[c], qx = T.comp_qx[c], qy = T.comp_qy[c];
    const double F = T.comp_F[c];
    if (kind == 0) {
      terms.push_back({c, -1, qx, qy, 0, 0.0, std::sqrt(2.0), F});
      by_shift[((qy % N) + N) % N].push_back((int)terms.size() - 1);
    } else if (kind == 1) {
      // (phi_A + i phi_C) m_q + (phi_A - i phi_C) m_q^dagger
      terms.push_back({c, c + 1, qx, qy, 0, 1.0, 1.0, F});
      by_shift[((qy % N) + N) % N].push_back((int)terms.size() - 1);
      terms.push_back({c, c + 1, qx, qy, 1, -1.0, 1.0, F});
      by_shift[((-qy % N) + N) % N].push_back((int)terms.size() - 1);
    }
  }
  T.hoff.assign(N + 1, 0);
  for (int d = 0; d < N; ++d) {
    T.hoff[d + 1] = T.hoff[d] + (int)by_shift[d].size();
    for (int t : by_shift[d]) {
      const HT& h = terms[t];
      T.h_cre.push_back(h.cre); T.h_cim.push_back(h.cim); T.h_qx.push_back(h.qx); T.h_qy.push_back(h.qy);
      T.h_dag.push_back(h.dag); T.h_sgn.push_back(h.sgn); T.h_scale.push_back(h.scale); T.h_F.push_back(h.F);
    }
  }
  // trace table grouped by q_y of the component
  std::vector<int> rows;
  for (int c = 0; c < nq; ++c) rows.push_back(T.comp_qy[c]);
  std::sort(rows.begin(), rows.end());
  rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
  T.toff.assign(1, 0);
  for (int qy : rows) {
    for (int c = 0; c < nq; ++c)
      if (T.comp_qy[c] == qy) {
        T.t_qx.push_back(T.comp_qx[c]); T.t_kind.push_back(T.comp_kind[c]); T.t_comp.push_back(c);
        T.t_F.push_back(T.comp_F[c]);
      }
    T.t_qy.push_back(qy);
    T.toff.push_back((int)T.t_qx.size());
    if (T.toff.back() - T.toff[T.toff.size() - 2] > 1024) { err = "too many components in one momentum row"; return false; }
  }
  if (!T.comp_w.empty()) {
    const size_t nt = T.t_comp.size();
    T.t_w.assign((size_t)N * nt, 0.0);
    for (size_t t = 0; t < nt; ++t)
      for (int k = 0; k < N; ++k) T.t_w[(size_t)k * nt + t] = T.comp_w[(size_t)T.t_comp[t] * N + k];
  }
  T.phase.resize(2 * N);
  for (int m = 0; m < 2 * N; ++m) T.phase[m] = make_double2(std::cos(M_PI * m / N), std::sin(M_PI * m / N));
  return true;
}

}  // namespace

// Device scratch of the allocation-free correlator entry point
// (cfqmc_measure_tau_noalloc): per chain the two traces of G(0) the correlator
// kernel keeps (2 x 16 B) and the twelve running maxima of the carried-vs-
// recomputed check (12 x 8 B), 128 B per chain, at most 512 chains. Each GPU
// holds its own copy until the process ends. Host code never passes the
// symbol itself to a kernel: it uses the device address from
// hipGetSymbolAddress, resolved once per device.
constexpr size_t kScratchBytes = 64 * 1024;
constexpr size_t kScratchPerChain = 2 * sizeof(double2) + 12 * sizeof(double);
__device__ __align__(256) unsigned char scratch[kScratchBytes];

struct Udt {
  double2* U;   // [chain][nb+1][n][n]
  double2* T;
  double* D;    // [chain][nb+1][n]
};

struct cfqmc_ctx {
  cfqmc_params p;
  hipStream_t s;
  int N, n, nq, L, nch, nstab, nblk_stab, mixed, mixed_m, smax;
  int hband;   // h = sum_c phi_c q_c vanishes outside |(col - row) mod N| <= hband (-1: dense)
  long long nn, NN;
  HostTables ht;
  ModelDev md;
  std::vector<void*> allocs;
  // chain state
  double* phi;
  double2* PQ;
  double2* G;
  double2* F[4];
  double2* Fp[4];
  double2* S1;
  double2* S2;
  double2* Mw;
  double2* Mb;
  int* lu_flag;
  int* ipiv;
  double2* lndet;
  double* phip;
  double2* PQp;
  double2* h;
  // exp work
  int exp_cap;        // capacity in (entry) units of 4 channels
  double2 *H2, *X2, *X3, *Eo, *Oo, *Wa, *Wb;
  double* coef;
  int* sq;
  int* d_err;
  // stabilisation
  double2* Cb;
  Udt Ls, Rs;
  double2 *W1, *A1, *Gr, *Q1, *Q2, *R1, *R2, *Rt, *Tp, *K1, *M1, *Yl, *Wm, *X1, *Gs;
  double2* rs_ws;   // inverted diagonal blocks for the right solves
  double *nrm, *sqd1, *sqd2, *dinvL, *dinvR, *tmpd, *dminL, *dminR;
  // imaginary-time correlator: [chain][L+1][5] values and the traces of G(0)
  double2* corr;
  double2* tr0;
  double* disp_err;   // [chain][3][4] carried vs recomputed at the block boundaries
  int* perm;
  // scalars per chain
  double2* alpha;
  double2 Urot[4][2][2];
  double* eps;
  int* acc_count;
  double* lnA;
  int* accept;
  double* stat;
  double* part;
  double* obs;
  double* stab_err;
  double* series;     // [chain][series_cap] m^2_SO(5) per sweep
  double* series_s;   // action S = |phi|^2/2 - ln w_F per sweep
  double* series_p;   // power of the q = 0 fields per sweep
  double *fsq, *fq0;  // per-chain field sums of the current sweep
  double2* ldY2;      // ln det Y of the sweep-end weight
  int series_cap, series_len;
  int* hist_acc;
  double* hist_lnA;
  double* noise;
  double2* bg;
  double2* ldtmp;
  long long sweep_counter;
  int cfg_chan, cfg_chan64, cfg_gemm, cfg_small;   // cfg_chan64: FP64 applications in a mixed context
  // sampled HIP-event timing of the channel application (one launch per slice)
  bool timing;
  std::vector<hipEvent_t> ev;
  size_t ev_used;
  std::vector<hipEvent_t> ev2;   // the same for one application of the Woodbury product per slice
  size_t ev2_used;
  bool ready;
  int guard;            // precision guard active (mixed context with precision_guard = 1)
  int* sel64;           // [chain] 1: the chain's FP32 applications run in FP64 in the current block
  int* guard_cnt;       // [chain] blocks run under the guard since the last stats reset
  double* gmax_run;     // [chain] running max |G_FP64| since the last stats reset
  double* blk_last;     // [chain][2] max |G_updated - G_FP64|, max |G_FP64| of the last block
  long long blocks_in_call;
  double lu_lmax;   // largest multiplier the non-pivoted LU of M accepts before the pivoted refactorisation
  int dev;   // device current at creation (owner of the stream's memory)
  // the sweep counter (random-number stream) and the series length in device
  // memory, so that the recorded graph of a sweep replays unchanged
  long long* d_counter;
  int* d_series_len;
  // recorded graphs of one sweep, [0] device noise, [1] replayed noise: one
  // graph per chunk of whole stabilisation blocks (the last chunk also holds
  // the end of the sweep); state 0 not recorded yet, 1 recorded, -1 recording
  // failed (launches one by one)
  std::vector<hipGraphExec_t> gexec[2];
  int graph_state[2];
  long long blocks_per_sweep;
  long long sweeps_in_call, graph_sweeps_in_call;
  int guard_launch;     // guarded applications: 0 one launch per precision class, 1 / 2 one launch
                        // for both (launch_chan_apply_dual variant)
  bool guard_pair_only; // testing knob CFQMC_GUARD_PAIR=1: always one launch per class
  bool graph_noted;     // a failed recording or launch has been reported on stderr
  bool launch_failed;   // a recorded chunk failed to launch: the sweep is incomplete
  // timing variant of the recorded sweep (kernel timing on): the capture is cut
  // at the timed launches, each of which becomes a graph of its own, so that
  // the host records HIP events around it on the stream. Items in launch
  // order; kind -1 untimed launches, 0 the wrap's timed application, 1 the
  // Woodbury product's.
  struct TimedItem {
    hipGraphExec_t x;              // untimed launches (kind -1)
    int kind;
    std::function<void()> launch;  // the timed application, launched as such (kind 0, 1)
  };
  std::vector<TimedItem> titems[2];
  int tstate[2];
  bool seg_rec;              // recording the timing variant
  int seg_m;                 // of mode seg_m (0 device noise, 1 replayed noise)
  const char* seg_fail;      // first failing step while recording it
  hipError_t seg_fail_err;
  bool seg_broken;           // a capture could not be restarted: launches ran for real
  std::string err;
};

namespace {

#define HIPCHK(x)                                                        \
  do {                                                                   \
    hipError_t e_ = (x);                                                 \
    if (e_ != hipSuccess) {                                              \
      c->err = std::string("HIP error: ") + hipGetErrorString(e_) + " at " #x; \
      return CFQMC_EHIP;                                                 \
    }                                                                    \
  } while (0)

// Message of the last cfqmc_create that failed on this thread (no context to hold it).
thread_local std::string g_create_err;

template <typename T>
int dalloc(cfqmc_ctx* c, T** p, size_t count) {
  void* q = nullptr;
  if (count == 0) count = 1;
  const hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    size_t fr = 0, tot = 0;
    (void)hipMemGetInfo(&fr, &tot);
    c->err = "device allocation of " + std::to_string(count * sizeof(T)) + " B failed (" + hipGetErrorString(e) +
             "; " + std::to_string(fr >> 20) + " MiB of " + std::to_string(tot >> 20) + " MiB free)";
    return CFQMC_ENOMEM;
  }
  hipMemsetAsync(q, 0, count * sizeof(T), c->s);
  c->allocs.push_back(q);
  *p = (T*)q;
  return CFQMC_OK;
}

template <typename T>
int upload(cfqmc_ctx* c, T** p, const std::vector<T>& v) {
  int r = dalloc(c, p, v.size());
  if (r) return r;
  if (!v.empty()) HIPCHK(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->s));
  return CFQMC_OK;
}

// ---------------------------------------------------------------- launch helpers

GemmArgs gemm0(int M, int N, int K) {
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.M = M; g.N = N; g.K = K;
  g.nz2 = 1;
  g.alpha = make_double2(1.0, 0.0);
  g.beta = make_double2(0.0, 0.0);
  g.mode = GEMM_NORMAL;
  g.bandA = g.bandB = -1;
  return g;
}
MatRef mref(const double2* p, int ld, long long s1, long long s2 = 0) {
  MatRef m;
  m.p = (double2*)p; m.ld = ld; m.s1 = s1; m.s2 = s2;
  return m;
}

// Y = E X (left) or X E (right) for channel ch of the P/Q block at PQch (chain stride sPQ).
void chan(cfqmc_ctx* c, int left, int ch, bool inverse, const double2* PQch, long long sPQ, const double2* X,
          double2* Y, bool one_minus, const double2* add, int mixed, long long sY = -1, double2* Y2 = nullptr) {
  ChanArgs a;
  memset(&a, 0, sizeof(a));
  const int N = c->N;
  a.N = N;
  a.n_other = c->n;
  a.M = X; a.ldM = c->n; a.sM = c->nn;
  const double2* P = PQch;
  const double2* Q = PQch + c->NN;
  if (ch == 0) { a.X0 = a.X1 = inverse ? Q : P; }
  else { a.X0 = inverse ? Q : P; a.X1 = inverse ? P : Q; }
  a.ldX = N; a.sX = sPQ;
  a.one_minus = one_minus ? 1 : 0;
  a.Cadd = add; a.ldC = c->n; a.sC = c->nn;
  a.Y = Y; a.ldY = c->n; a.sY = sY < 0 ? c->nn : sY;
  a.Y2 = Y2;
  const int rot = ch == 1 ? 1 : ch == 2 ? 2 : 0;   // tau_x, tau_y valley rotations
  if (one_minus && (!left || rot)) {                // 1 - M exists only for the left, non-rotating application
    std::fprintf(stderr, "cfqmc: internal error: 1 - M requested for a rotating or right channel\n");
    std::abort();
  }
  if (mixed && c->guard) {
    // FP32 for the chains the guard leaves in FP32, FP64 for the others: one
    // launch where both tile configurations allow it, else one per class
    a.chain_sel = c->sel64;
    if (c->guard_launch &&
        launch_chan_apply_dual(a, left, rot, c->nch, c->cfg_chan, c->cfg_chan64, c->guard_launch, c->s))
      return;
    a.sel_want = 0;
    launch_chan_apply(a, left, rot, c->nch, 1, c->cfg_chan, c->s);
    a.sel_want = 1;
    launch_chan_apply(a, left, rot, c->nch, 0, c->cfg_chan64, c->s);
    return;
  }
  launch_chan_apply(a, left, rot, c->nch, mixed, mixed ? c->cfg_chan : c->cfg_chan64, c->s);
}

// C = op(A) op(B) on n x n per chain (FP64)
void gemm_nn(cfqmc_ctx* c, const double2* A, int opA, long long sA, const double2* B, int opB, long long sB,
             double2* D, long long sD, int nbatch, bool herm = false) {
  GemmArgs g = gemm0(c->n, c->n, c->n);
  g.opA = opA; g.opB = opB;
  g.herm = herm ? 1 : 0;
  g.A = mref(A, c->n, sA); g.B = mref(B, c->n, sB); g.D = mref(D, c->n, sD);
  launch_zgemm(g, nbatch, 0, c->cfg_gemm, c->s);
}

// Taylor exponentials of nent entries x 4 channels; h at hb [entry][4][N][N];
// outputs P/Q at out + entry*sOut + ch*2N^2 (+N^2 for Q). alpha index = entry/alpha_div.
void exps(cfqmc_ctx* c, const double2* hb, int nent, const double2* alpha, int alpha_div, double2* out,
          long long sOut) {
  const int N = c->N;
  const long long NN = c->NN, s4 = 4 * NN;
  // h is Hermitian, so are its powers and the even / odd polynomials in h^2
  // (real coefficients): those products compute the upper tile triangle only
  // h has band b = hband, h^2 band 2b: slabs of exact zeros are skipped
  const int b1 = c->hband, b2 = (b1 >= 0 && 4 * b1 < N) ? 2 * b1 : -1;
  auto sq = [&](const double2* A, const double2* B, double2* D, int bandA, int bandB) {
    GemmArgs g = gemm0(N, N, N);
    g.A = mref(A, N, s4, NN); g.B = mref(B, N, s4, NN); g.D = mref(D, N, s4, NN);
    g.nz2 = 4;
    g.herm = 1;
    g.bandA = bandA; g.bandB = bandB;
    launch_zgemm(g, nent * 4, 0, c->cfg_small, c->s);
  };
  sq(hb, hb, c->H2, b1, b1);
  sq(c->H2, c->H2, c->X2, b2, b2);
  sq(c->X2, c->H2, c->X3, -1, b2);
  launch_exp_coef(c->X2, c->X3, N, alpha, alpha_div, c->coef, c->sq, c->smax, 0.4, c->d_err, nent * 4, c->s);
  launch_exp_eo(c->H2, c->X2, c->X3, c->coef, N, c->Eo, c->Oo, nent * 4, c->s);
  {
    // P, Q = E +- alpha h O; matrices with squaring count 0 go straight to out
    GemmArgs g = gemm0(N, N, N);
    g.mode = GEMM_PQ;
    g.A = mref(hb, N, s4, NN); g.B = mref(c->Oo, N, s4, NN); g.C = mref(c->Eo, N, s4, NN);
    g.bandA = b1;
    g.alpha_dev = (const double2*)(c->coef + 14);
    g.ad_s1 = 4 * EXP_NC / 2; g.ad_s2 = EXP_NC / 2;
    g.nz2 = 4;
    g.E = mref(out, N, sOut, 2 * NN);
    g.E2 = mref(out + NN, N, sOut, 2 * NN);
    if (c->smax > 0) {
      g.D = mref(c->Wa, N, 8 * NN, 2 * NN);
      g.D2 = mref(c->Wa + NN, N, 8 * NN, 2 * NN);
      g.pred = c->sq; g.pred_s1 = 8; g.pred_s2 = 2;
    } else {
      g.D = g.E;
      g.D2 = g.E2;
    }
    launch_zgemm(g, nent * 4, 0, c->cfg_small, c->s);
  }
  // squaring step j on the matrices that need more than j squarings; the last
  // step of each matrix writes it to out
  for (int j = 0; j < c->smax; ++j) {
    double2* src = (j % 2 == 0) ? c->Wa : c->Wb;
    double2* dst = (j % 2 == 0) ? c->Wb : c->Wa;
    GemmArgs g = gemm0(N, N, N);
    g.mode = GEMM_SQUARE;
    g.A = mref(src, N, 8 * NN, NN); g.B = mref(src, N, 8 * NN, NN);
    g.D = mref(dst, N, 8 * NN, NN);
    g.E = mref(out, N, sOut, NN);
    g.nz2 = 8;
    g.pred = c->sq; g.pred_s1 = 8; g.pred_s2 = 1; g.pred_thresh = j;
    launch_zgemm(g, nent * 8, 0, c->cfg_small, c->s);
  }
}

// The q = 0 density operator is a multiple of the identity on the orbitals:
// F(0) = 1 / (4 pi sqrt N) on the torus, the l = m = 0 weight on the sphere.
double q0_weight(const cfqmc_ctx* c) {
  return c->ht.comp_w.empty() ? 1.0 / (4.0 * M_PI * std::sqrt((double)c->N)) : c->ht.comp_w[0];
}

// UDT accumulation: (Uo, Do, To) <- decomposition of op(C) * (Ui Di Ti), all [chain] batched.
void udt_acc(cfqmc_ctx* c, const double2* C, long long sC, int opC, const double2* Ui, const double* Di,
             const double2* Ti, double2* Uo, double* Do, double2* To, long long sU, long long sD) {
  const int n = c->n, B = c->nch;
  const long long nn = c->nn;
  gemm_nn(c, C, opC, sC, Ui, 0, sU, c->W1, nn, B);
  launch_colscale(c->W1, n, nn, c->W1, n, nn, Di, sD, n, n, 0, B, c->s);
  launch_colnorm_sort(c->W1, n, nn, c->nrm, c->perm, B, c->s);
  launch_permute_normalize(c->W1, n, nn, c->nrm, c->perm, c->A1, B, c->s);
  // Cholesky-QR, twice
  gemm_nn(c, c->A1, 1, nn, c->A1, 0, nn, c->Gr, nn, B, true);   // Gram matrix: Hermitian
  launch_lu_np(c->Gr, n, n, nn, c->ipiv, n, nullptr, nullptr, 1e300, B, c->s);
  launch_chol_from_lu(c->Gr, n, nn, c->R1, c->sqd1, B, c->s, c->d_err);
  launch_rsolve(c->A1, n, nn, c->Q1, n, nn, c->Gr, n, nn, c->ipiv, n, n, 1, B, c->s, c->rs_ws);
  launch_colscale(c->Q1, n, nn, c->Q1, n, nn, c->sqd1, n, n, n, 0, B, c->s);
  gemm_nn(c, c->Q1, 1, nn, c->Q1, 0, nn, c->Gr, nn, B, true);
  launch_lu_np(c->Gr, n, n, nn, c->ipiv, n, nullptr, nullptr, 1e300, B, c->s);
  launch_chol_from_lu(c->Gr, n, nn, c->R2, c->sqd2, B, c->s, c->d_err);
  launch_rsolve(c->Q1, n, nn, Uo, n, sU, c->Gr, n, nn, c->ipiv, n, n, 1, B, c->s, c->rs_ws);
  launch_colscale(Uo, n, sU, Uo, n, sU, c->sqd2, n, n, n, 0, B, c->s);
  gemm_nn(c, c->R2, 0, nn, c->R1, 0, nn, c->Rt, nn, B);
  launch_udt_finish(c->Rt, n, nn, c->nrm, c->perm, Do, sD, c->Tp, B, c->s);
  gemm_nn(c, c->Tp, 0, nn, Ti, 0, sU, To, sU, B);
}

// G = (1 + U_L D_L T_L T_R^dagger D_R U_R^dagger)^{-1} into Gout (all chains).
void green_udt(cfqmc_ctx* c, int bl, int br, double2* Gout) {
  const int n = c->n, B = c->nch;
  const long long nn = c->nn, sU = (long long)(c->nblk_stab + 1) * nn, sD = (long long)(c->nblk_stab + 1) * n;
  const double2 *UL = c->Ls.U + bl * nn, *TL = c->Ls.T + bl * nn, *UR = c->Rs.U + br * nn, *TR = c->Rs.T + br * nn;
  const double *DL = c->Ls.D + bl * n, *DR = c->Rs.D + br * n;
  gemm_nn(c, UL, 1, sU, UR, 0, sU, c->K1, nn, B);
  gemm_nn(c, TL, 0, sU, TR, 1, sU, c->M1, nn, B);
  launch_loh_combine(c->K1, c->M1, DL, sD, DR, sD, c->Yl, n, B, c->s);
  launch_lu(c->Yl, n, n, nn, c->ipiv, n, c->ldtmp, 1, B, c->s);
  launch_dmax_inv(DR, sD, c->dinvR, n, B, c->s);
  launch_dmax_inv(DL, sD, c->dinvL, n, B, c->s);
  launch_colscale(UR, n, sU, c->Wm, n, nn, c->dinvR, n, n, n, 0, B, c->s);
  launch_rsolve(c->Wm, n, nn, c->X1, n, nn, c->Yl, n, nn, c->ipiv, n, n, 0, B, c->s, c->rs_ws);
  launch_colscale(c->X1, n, nn, c->X1, n, nn, c->dinvL, n, n, n, 0, B, c->s);
  gemm_nn(c, c->X1, 0, nn, UL, 1, sU, Gout, nn, B);
}

// The three Green's functions at the block boundary tau_b from the same
// stacks and the same Loh matrix Y (B(tau,0) = U_L D_L T_L, B(beta,tau) =
// T_R^+ D_R U_R^+, D = D^max D^min with D^max = max(D, 1)):
//   G(tau,tau) = U_R D_R^max^-1 Y^-1 D_L^max^-1 U_L^+     (as green_udt)
//   G(tau,0)   = G(tau,tau) B(tau,0)  = U_R D_R^max^-1 Y^-1 D_L^min T_L
//   G(0,tau)   = -B(beta,tau) G(tau,tau) = -T_R^+ D_R^min Y^-1 D_L^max^-1 U_L^+
// Every diagonal factor is at most one, so no scale is amplified.
void green_udt3(cfqmc_ctx* c, int b, double2* Gtt, double2* Gt0, double2* G0t) {
  const int n = c->n, B = c->nch;
  const long long nn = c->nn, sU = (long long)(c->nblk_stab + 1) * nn, sD = (long long)(c->nblk_stab + 1) * n;
  const double2 *UL = c->Ls.U + b * nn, *TL = c->Ls.T + b * nn, *UR = c->Rs.U + b * nn, *TR = c->Rs.T + b * nn;
  const double *DL = c->Ls.D + b * n, *DR = c->Rs.D + b * n;
  gemm_nn(c, UL, 1, sU, UR, 0, sU, c->K1, nn, B);
  gemm_nn(c, TL, 0, sU, TR, 1, sU, c->M1, nn, B);
  launch_loh_combine(c->K1, c->M1, DL, sD, DR, sD, c->Yl, n, B, c->s);
  launch_lu(c->Yl, n, n, nn, c->ipiv, n, c->ldtmp, 1, B, c->s);
  launch_dmax_inv(DR, sD, c->dinvR, n, B, c->s);
  launch_dmax_inv(DL, sD, c->dinvL, n, B, c->s);
  launch_dmin1(DL, sD, c->dminL, n, B, c->s);
  launch_dmin1(DR, sD, c->dminR, n, B, c->s);
  // W = U_R D_R^max^-1 Y^-1
  launch_colscale(UR, n, sU, c->Wm, n, nn, c->dinvR, n, n, n, 0, B, c->s);
  launch_rsolve(c->Wm, n, nn, c->X1, n, nn, c->Yl, n, nn, c->ipiv, n, n, 0, B, c->s, c->rs_ws);
  launch_colscale(c->X1, n, nn, c->Wm, n, nn, c->dminL, n, n, n, 0, B, c->s);
  gemm_nn(c, c->Wm, 0, nn, TL, 0, sU, Gt0, nn, B);
  launch_colscale(c->X1, n, nn, c->X1, n, nn, c->dinvL, n, n, n, 0, B, c->s);
  gemm_nn(c, c->X1, 0, nn, UL, 1, sU, Gtt, nn, B);
  // Z = -D_R^min Y^-1 D_L^max^-1 U_L^+, then G(0,tau) = T_R^+ Z
  launch_diag_set(c->Wm, n, nn, c->dminR, n, -1.0, B, c->s);
  launch_rsolve(c->Wm, n, nn, c->X1, n, nn, c->Yl, n, nn, c->ipiv, n, n, 0, B, c->s, c->rs_ws);
  launch_colscale(c->X1, n, nn, c->X1, n, nn, c->dinvL, n, n, n, 0, B, c->s);
  gemm_nn(c, c->X1, 0, nn, UL, 1, sU, c->Wm, nn, B);
  gemm_nn(c, TR, 1, sU, c->Wm, 0, nn, G0t, nn, B);
}

// Imaginary-time pass over tau = 0..L of the current configuration (between
// sweeps: both stacks and the slice exponentials are current). G(tau,0),
// G(0,tau) and G(tau,tau) are recomputed from the stacks at every block
// boundary and carried through the slices of a block by channel applications
// in FP64: G(tau,0) <- B_tau G(tau-1,0), G(0,tau) <- G(0,tau-1) B_tau^-1,
// G(tau,tau) <- B_tau G(tau-1,tau-1) B_tau^-1. At each boundary after the
// first the carried matrices are compared with the recomputed ones (running
// max |carried - recomputed| and its ratio to max |recomputed| per chain and
// matrix in err[chain][3][4], when err != nullptr; entries 2, 3 of each
// quadruple are scratch and must start at zero). With corr != nullptr the
// correlator of every tau goes to corr[chain][tau][5]; the pass stops after
// tau_stop (-1: all). out[0..2] receive the buffers holding the final
// G(tau,0), G(0,tau), G(tau,tau) (two of F / Fp each). tr0 [chain][2]: the
// correlator's traces of G(0) (needed when corr != nullptr).
void displaced_pass(cfqmc_ctx* c, int tau_stop, double2* corr, double* err, double2** out, double2* tr0) {
  const long long nn = c->nn, NN = c->NN, sPQ = (long long)c->L * 8 * NN;
  double2* cur[3] = {c->Fp[0], c->Fp[1], c->Fp[2]};
  double2* alt[3] = {c->F[0], c->F[1], c->F[2]};
  const double F0 = q0_weight(c);
  const int last = tau_stop < 0 ? c->L : tau_stop;
  for (int tau = 0; tau <= last; ++tau) {
    const bool boundary = tau % c->nstab == 0 || tau == c->L;
    if (tau > 0) {
      const int t = tau - 1;   // 0-based slice
      // B_tau X, X B_tau^-1 and B_tau X B_tau^-1 with B_tau = E_0 E_1 E_2 E_3;
      // each chain of four applications ends in the buffer it started from
      const double2* in = cur[0];
      for (int ch = 3; ch >= 0; --ch) {
        const double2* pq = c->PQ + (long long)t * 8 * NN + ch * 2 * NN;
        double2* dst = ch == 0 ? cur[0] : (ch % 2 ? c->S1 : c->S2);
        chan(c, 1, ch, false, pq, sPQ, in, dst, false, nullptr, 0);
        in = dst;
      }
      in = cur[1];
      for (int ch = 3; ch >= 0; --ch) {
        const double2* pq = c->PQ + (long long)t * 8 * NN + ch * 2 * NN;
        double2* dst = ch == 0 ? cur[1] : (ch % 2 ? c->S1 : c->S2);
        chan(c, 0, ch, true, pq, sPQ, in, dst, false, nullptr, 0);
        in = dst;
      }
      in = cur[2];
      for (int ch = 3; ch >= 0; --ch) {
        const double2* pq = c->PQ + (long long)t * 8 * NN + ch * 2 * NN;
        chan(c, 1, ch, false, pq, sPQ, in, c->S1, false, nullptr, 0);
        double2* dst = ch == 0 ? cur[2] : (in == c->S2 ? c->Fp[3] : c->S2);
        chan(c, 0, ch, true, pq, sPQ, c->S1, dst, false, nullptr, 0);
        in = dst;
      }
    }
    if (boundary) {
      const int b = tau == c->L ? c->nblk_stab : tau / c->nstab;
      if (tau == 0) {
        green_udt3(c, b, cur[2], cur[0], cur[1]);
      } else {
        green_udt3(c, b, alt[2], alt[0], alt[1]);
        for (int k = 0; k < 3; ++k) {
          if (err) launch_maxdiff(cur[k], alt[k], c->n, nn, err + 4 * k, c->nch, c->s, 12);
          std::swap(cur[k], alt[k]);
        }
      }
    }
    if (corr)
      launch_disp_corr(cur[0], cur[1], cur[2], nn, c->N, F0, tr0, tau == 0, corr + (long long)tau * 5,
                       (long long)(c->L + 1) * 5, c->nch, c->s);
  }
  if (out)
    for (int k = 0; k < 3; ++k) out[k] = cur[k];
}

// C_b = B_{tau_{b+1}} ... B_{tau_b + 1} of block b (FP64), all chains.
void block_product(cfqmc_ctx* c, int b) {
  const long long nn = c->nn, sPQ = (long long)c->L * 8 * c->NN;
  const int t0 = b * c->nstab, t1 = std::min(c->L, t0 + c->nstab);
  double2* cur = c->S1;
  double2* nxt = c->S2;
  launch_set_identity(cur, c->n, c->n, nn, c->nch, c->s);
  for (int t = t0; t < t1; ++t)
    for (int ch = 3; ch >= 0; --ch) {
      const double2* pq = c->PQ + (long long)t * 8 * c->NN + ch * 2 * c->NN;
      const bool last = (t == t1 - 1 && ch == 0);
      double2* dst = last ? c->Cb + (long long)b * nn : nxt;
      chan(c, 1, ch, false, pq, sPQ, cur, dst, false, nullptr, 0, last ? (long long)c->nblk_stab * nn : -1);
      if (!last) std::swap(cur, nxt);
    }
}

long long sU_(cfqmc_ctx* c) { return (long long)(c->nblk_stab + 1) * c->nn; }
long long sD_(cfqmc_ctx* c) { return (long long)(c->nblk_stab + 1) * c->n; }

void set_udt_identity(cfqmc_ctx* c, Udt& u, int b) {
  const long long sU = sU_(c), sD = sD_(c);
  launch_set_identity(u.U + b * c->nn, c->n, c->n, sU, c->nch, c->s);
  launch_set_identity(u.T + b * c->nn, c->n, c->n, sU, c->nch, c->s);
  std::vector<double> ones(c->n, 1.0);
  for (int z = 0; z < c->nch; ++z)
    hipMemcpyAsync(u.D + z * sD + b * c->n, ones.data(), c->n * sizeof(double), hipMemcpyHostToDevice, c->s);
  hipStreamSynchronize(c->s);
}

void restack_right(cfqmc_ctx* c) {
  const long long sU = sU_(c), sD = sD_(c), nn = c->nn;
  const long long sC = (long long)c->nblk_stab * nn;
  for (int b = c->nblk_stab - 1; b >= 0; --b)
    udt_acc(c, c->Cb + b * nn, sC, 1, c->Rs.U + (b + 1) * nn, c->Rs.D + (b + 1) * c->n, c->Rs.T + (b + 1) * nn,
            c->Rs.U + b * nn, c->Rs.D + b * c->n, c->Rs.T + b * nn, sU, sD);
}

void left_acc(cfqmc_ctx* c, int b) {
  const long long sU = sU_(c), sD = sD_(c), nn = c->nn;
  const long long sC = (long long)c->nblk_stab * nn;
  udt_acc(c, c->Cb + b * nn, sC, 0, c->Ls.U + b * nn, c->Ls.D + b * c->n, c->Ls.T + b * nn, c->Ls.U + (b + 1) * nn,
          c->Ls.D + (b + 1) * c->n, c->Ls.T + (b + 1) * nn, sU, sD);
}

int build_model_dev(cfqmc_ctx* c) {
  HostTables& T = c->ht;
  ModelDev& m = c->md;
  m.N = c->N; m.n = c->n; m.nq = c->nq; m.L = c->L;
  int r = 0;
  int *p_hoff, *p_cre, *p_cim, *p_qx, *p_qy, *p_dag, *p_toff, *p_tqy, *p_tqx, *p_tk, *p_tc;
  double *p_sgn, *p_sc, *p_F, *p_tF, *p_beta;
  double2* p_ph;
  r |= upload(c, &p_hoff, T.hoff); r |= upload(c, &p_cre, T.h_cre); r |= upload(c, &p_cim, T.h_cim);
  r |= upload(c, &p_qx, T.h_qx); r |= upload(c, &p_qy, T.h_qy); r |= upload(c, &p_dag, T.h_dag);
  r |= upload(c, &p_sgn, T.h_sgn); r |= upload(c, &p_sc, T.h_scale); r |= upload(c, &p_F, T.h_F);
  r |= upload(c, &p_toff, T.toff); r |= upload(c, &p_tqy, T.t_qy); r |= upload(c, &p_tqx, T.t_qx);
  r |= upload(c, &p_tk, T.t_kind); r |= upload(c, &p_tc, T.t_comp); r |= upload(c, &p_tF, T.t_F);
  r |= upload(c, &p_beta, T.beta); r |= upload(c, &p_ph, T.phase);
  T.hdiag.clear();
  for (int d = 0; d < c->N; ++d)
    if (T.hoff[d + 1] > T.hoff[d]) T.hdiag.push_back(d);
  int* p_hdiag = nullptr;
  if (!T.hdiag.empty()) r |= upload(c, &p_hdiag, T.hdiag);
  if (r) return CFQMC_ENOMEM;
  m.hoff = p_hoff; m.h_cre = p_cre; m.h_cim = p_cim; m.h_qx = p_qx; m.h_qy = p_qy; m.h_dag = p_dag;
  m.hdiag = p_hdiag;
  m.nhdiag = (int)T.hdiag.size();
  m.h_sgn = p_sgn; m.h_scale = p_sc; m.h_F = p_F;
  m.nrow = (int)T.t_qy.size();
  m.maxrow = 1;
  for (size_t r = 0; r + 1 < T.toff.size(); ++r) m.maxrow = std::max(m.maxrow, T.toff[r + 1] - T.toff[r]);
  m.toff = p_toff; m.t_qy = p_tqy; m.t_qx = p_tqx; m.t_kind = p_tk; m.t_comp = p_tc; m.t_F = p_tF;
  m.beta = p_beta; m.phase = p_ph;
  m.cw = nullptr;
  m.tw = nullptr;
  m.ntw = (int)T.t_comp.size();
  if (!T.comp_w.empty()) {
    double *p_cw, *p_tw;
    if (upload(c, &p_cw, T.comp_w) || upload(c, &p_tw, T.t_w)) return CFQMC_ENOMEM;
    m.cw = p_cw;
    m.tw = p_tw;
  }
  return CFQMC_OK;
}

// Message of the device error flags: bit 1 an exponential needed more
// squarings than allowed, bit 2 a Cholesky-QR of the stabilisation broke down.
std::string dev_err_msg(int ef) {
  std::string m;
  if (ef & 1) m = "exponential range exceeded";
  if (ef & 2) m += std::string(m.empty() ? "" : "; ") + "Cholesky-QR breakdown in the stabilisation (Gram pivot not positive)";
  return m;
}

// Device copies of the host's sweep counter and series length (synchronous).
hipError_t upload_counters(cfqmc_ctx* c) {
  const int sl = c->series_len;
  hipError_t e = hipMemcpy(c->d_counter, &c->sweep_counter, sizeof(long long), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_series_len, &sl, sizeof(int), hipMemcpyHostToDevice);
  return e;
}

void drop_graphs(cfqmc_ctx* c) {
  for (int m = 0; m < 2; ++m) {
    for (hipGraphExec_t x : c->gexec[m]) hipGraphExecDestroy(x);
    c->gexec[m].clear();
    c->graph_state[m] = 0;
    for (auto& it : c->titems[m])
      if (it.x) hipGraphExecDestroy(it.x);
    c->titems[m].clear();
    c->tstate[m] = 0;
  }
}

int check_finite_host(cfqmc_ctx* c, const double* dptr, long long count) {
  std::vector<double> h(count);
  HIPCHK(hipMemcpy(h.data(), dptr, count * sizeof(double), hipMemcpyDeviceToHost));
  for (double v : h)
    if (!std::isfinite(v)) return CFQMC_ENUMERIC;
  return CFQMC_OK;
}

// Ends the capture of the current piece of untimed launches of the timing
// variant, keeps it as a graph unless it is empty, and starts capturing the
// next piece.
void cut_piece(cfqmc_ctx* c) {
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->s, &g);
  if (e != hipSuccess || !g) {
    if (g) hipGraphDestroy(g);
    if (!c->seg_fail) { c->seg_fail = "end capture"; c->seg_fail_err = e; }
  } else {
    size_t nodes = 0;
    (void)hipGraphGetNodes(g, nullptr, &nodes);
    if (nodes > 0) {
      hipGraphExec_t x = nullptr;
      e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      if (e == hipSuccess) c->titems[c->seg_m].push_back({x, -1, nullptr});
      else if (!c->seg_fail) { c->seg_fail = "instantiate"; c->seg_fail_err = e; }
    }
    hipGraphDestroy(g);
  }
  e = hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    // the launches that follow would run for real: the recording pass is no
    // longer side-effect free
    c->seg_broken = true;
    if (!c->seg_fail) { c->seg_fail = "begin capture"; c->seg_fail_err = e; }
  }
}

// A timed launch (kind 0: the wrap's application of channel 2; 1: the
// Woodbury product's): launch by launch it runs between two HIP events on the
// stream. While the timing variant of the sweep graph is recorded it is not
// captured: the capture is cut there and the launch kept as a call, which each
// replay issues between the events as it would be issued launch by launch.
void timed_launch(cfqmc_ctx* c, int kind, std::function<void()> fn) {
  if (c->seg_rec) {
    if (!c->seg_broken) {
      cut_piece(c);
      c->titems[c->seg_m].push_back({nullptr, kind, std::move(fn)});
    }
    return;
  }
  std::vector<hipEvent_t>& ev = kind ? c->ev2 : c->ev;
  size_t& used = kind ? c->ev2_used : c->ev_used;
  hipEventRecord(ev[used], c->s);
  fn();
  hipEventRecord(ev[used + 1], c->s);
  used += 2;
}

// One slice move of all chains; t is the 0-based slice.
void slice_step(cfqmc_ctx* c, int t, const double* noise_dev) {
  const int N = c->N, mixed = c->mixed, mixed_m = c->mixed_m;
  const long long nn = c->nn, NN = c->NN;
  const long long sPQ = (long long)c->L * 8 * NN, sPQp = 8 * NN;
  const double2* pq = c->PQ + (long long)t * 8 * NN;   // chain 0 of slice t
  // 1. wrap through the channels of slice t, keeping the frames
  const double2* cur = c->G;
  const bool tm = c->timing && (c->seg_rec || c->ev_used + 2 <= c->ev.size());
  for (int ch = 3; ch >= 0; --ch) {
    const double2* pqc = pq + ch * 2 * NN;
    if (tm && ch == 2)
      timed_launch(c, 0, [c, ch, pqc, sPQ, cur, mixed]() {
        chan(c, 1, ch, false, pqc, sPQ, cur, c->S1, false, nullptr, mixed);
      });
    else
      chan(c, 1, ch, false, pqc, sPQ, cur, c->S1, false, nullptr, mixed);
    chan(c, 0, ch, true, pq + ch * 2 * NN, sPQ, c->S1, c->F[ch], false, nullptr, mixed);
    cur = c->F[ch];
  }
  // 2. drift and proposal
  StepArgs a;
  memset(&a, 0, sizeof(a));
  a.N = N; a.n = c->n; a.nq = c->nq; a.L = c->L; a.tau = t;
  for (int i = 0; i < 4; ++i) a.G[i] = c->F[i];
  a.sG = nn;
  a.phi = c->phi + (long long)t * 4 * c->nq;
  a.sphi = (long long)c->L * 4 * c->nq;
  a.phip = c->phip; a.sphip = 4 * c->nq;
  a.alpha = c->alpha; a.eps = c->eps;
  a.noise = noise_dev ? noise_dev + (long long)t * (4 * c->nq + 1) : nullptr;
  a.snoise = (long long)c->L * (4 * c->nq + 1);
  a.seed = c->p.seed;
  a.counter = c->sweep_counter * c->L + t;
  a.counter_dev = c->d_counter;
  a.part = c->part; a.nblk = 4 * c->md.nrow;
  a.lndetM = c->lndet; a.lnA = c->lnA; a.accept = c->accept; a.stat = c->stat;
  launch_drift_propose(c->md, a, c->nch, c->s);
  // 3. exponentials of the proposed fields
  launch_build_h(c->md, c->phip, 4 * c->nq, c->h, 4 * NN, c->nch, c->s);
  exps(c, c->h, c->nch, c->alpha, 1, c->PQp, sPQp);
  // 4. M = G_0 + B' B^{-1} (1 - G_0)
  double2* y = c->S1;
  double2* y2 = c->S2;
  chan(c, 1, 0, true, pq + 0 * 2 * NN, sPQ, c->F[0], y, true, nullptr, mixed_m);
  const bool tm2 = c->timing && (c->seg_rec || c->ev2_used + 2 <= c->ev2.size());
  for (int ch = 1; ch <= 3; ++ch) {
    const double2* pqc = pq + ch * 2 * NN;
    if (tm2 && ch == 2)
      timed_launch(c, 1, [c, ch, pqc, sPQ, y, y2, mixed_m]() {
        chan(c, 1, ch, true, pqc, sPQ, y, y2, false, nullptr, mixed_m);
      });
    else
      chan(c, 1, ch, true, pqc, sPQ, y, y2, false, nullptr, mixed_m);
    std::swap(y, y2);
  }
  for (int ch = 3; ch >= 1; --ch) {
    chan(c, 1, ch, false, c->PQp + ch * 2 * NN, sPQp, y, y2, false, nullptr, mixed_m);
    std::swap(y, y2);
  }
  chan(c, 1, 0, false, c->PQp, sPQp, y, c->Mw, false, c->F[0], mixed_m, -1, c->Mb);
  // 5. LU of M: ln det M. M is close to the identity, so the blocked LU without
  //    pivoting is tried first; chains whose multipliers exceed the threshold
  //    are refactorised with partial pivoting from the saved copy.
  launch_lu_np(c->Mw, c->n, c->n, nn, c->ipiv, c->n, c->lndet, c->lu_flag, c->lu_lmax, c->nch, c->s);
  launch_lu(c->Mw, c->n, c->n, nn, c->ipiv, c->n, c->lndet, 1, c->nch, c->s, c->lu_flag, c->Mb);
  // 6. G' = G_0 M^{-1} (MIXED_ALL: FP32 block products for the chains the
  //    guard leaves in FP32)
  launch_rsolve(c->F[0], c->n, nn, c->Fp[0], c->n, nn, c->Mw, c->n, nn, c->ipiv, c->n, c->n, 0, c->nch, c->s,
                c->rs_ws, mixed_m, c->guard ? c->sel64 : nullptr);
  // 7. frames of G' for the drift at phi'
  for (int ch = 0; ch < 3; ++ch) {
    chan(c, 1, ch, true, c->PQp + ch * 2 * NN, sPQp, c->Fp[ch], c->S1, false, nullptr, mixed);
    chan(c, 0, ch, false, c->PQp + ch * 2 * NN, sPQp, c->S1, c->Fp[ch + 1], false, nullptr, mixed);
  }
  for (int i = 0; i < 4; ++i) a.G[i] = c->Fp[i];
  launch_drift_mh(c->md, a, c->nch, c->s);
  // 8. commit
  launch_commit(a, c->nch, c->Fp[0], c->F[0], c->G, nn, nn, c->phip, 4 * c->nq,
                c->phi + (long long)t * 4 * c->nq, (long long)c->L * 4 * c->nq, 4 * c->nq, c->PQp, sPQp,
                c->PQ + (long long)t * 8 * NN, sPQ, 8 * NN, c->acc_count, c->s,
                // precision guard: a chain whose G grew past the threshold finishes the block in FP64
                c->guard ? c->sel64 : nullptr, c->p.guard_gmax);
  // history of this slice
  hipMemcpy2DAsync(c->hist_acc + t, c->L * sizeof(int), c->accept, sizeof(int), sizeof(int), c->nch,
                   hipMemcpyDeviceToDevice, c->s);
  hipMemcpy2DAsync(c->hist_lnA + t, c->L * sizeof(double), c->lnA, sizeof(double), sizeof(double), c->nch,
                   hipMemcpyDeviceToDevice, c->s);
}

// FP64 recomputation of G at the end of block b (left stack advanced first).
void block_end(cfqmc_ctx* c, int b) {
  block_product(c, b);
  left_acc(c, b);
  green_udt(c, b + 1, b + 1, c->Gs);
  launch_maxdiff(c->G, c->Gs, c->n, c->nn, c->stab_err, c->nch, c->s, 4, c->blk_last);
  launch_copy(c->Gs, c->G, c->nn, c->nn, c->nn, c->nch, c->s);
  if (c->guard)
    launch_precision_guard(c->blk_last, c->sel64, c->guard_cnt, c->gmax_run, c->p.guard_gmax, c->p.guard_err, c->nch,
                           c->s);
  else
    launch_precision_guard(c->blk_last, c->sel64, c->guard_cnt, c->gmax_run, INFINITY, INFINITY, c->nch, c->s);
  c->blocks_in_call++;
}

int build_all_exps(cfqmc_ctx* c) {
  // per chain, in chunks of slices
  const long long NN = c->NN;
  const int chunk = c->exp_cap;
  for (int z = 0; z < c->nch; ++z)
    for (int t0 = 0; t0 < c->L; t0 += chunk) {
      const int cnt = std::min(chunk, c->L - t0);
      const double* ph = c->phi + (long long)z * c->L * 4 * c->nq + (long long)t0 * 4 * c->nq;
      launch_build_h(c->md, ph, 4 * c->nq, c->h, 4 * NN, cnt, c->s);
      exps(c, c->h, cnt, c->alpha + z * 4, 1 << 30, c->PQ + (long long)z * c->L * 8 * NN + (long long)t0 * 8 * NN,
           8 * NN);
    }
  return CFQMC_OK;
}

// Everything that depends on the fields, from scratch in FP64: slice
// exponentials, block products, both UDT stacks and G(0). The identity slots
// Rs[nb] and Ls[0] are set once at initialisation.
void rebuild_state(cfqmc_ctx* c) {
  build_all_exps(c);
  for (int b = 0; b < c->nblk_stab; ++b) block_product(c, b);
  restack_right(c);
  for (int b = 0; b < c->nblk_stab; ++b) left_acc(c, b);
  green_udt(c, 0, 0, c->G);
}

// ln w_F = sum_tau c_tau + 2 ln det(1 + B(beta,0)) of every chain from the right
// stack at tau = 0 (left factor = 1): 1 + T_R^+ D_R U_R^+ = Y D_R^max U_R^+ with
// Y = U_R D_R^max^-1 + T_R^+ D_R^min (Loh split). Imaginary part wrapped to (-pi, pi].
int lnw_all(cfqmc_ctx* c, std::vector<double>& re, std::vector<double>& im) {
  const int n = c->n, B = c->nch;
  const long long nn = c->nn, sU = sU_(c), sD = sD_(c);
  green_udt(c, 0, 0, c->Gs);   // leaves LU(Y) in Yl and ln det Y in ldtmp
  std::vector<double2> ldY(B);
  HIPCHK(hipStreamSynchronize(c->s));
  HIPCHK(hipMemcpy(ldY.data(), c->ldtmp, B * sizeof(double2), hipMemcpyDeviceToHost));
  // ln det U_R (unitary: phase only)
  launch_copy(c->Rs.U, c->Q2, nn, sU, nn, B, c->s);
  launch_lu(c->Q2, n, n, nn, c->ipiv, n, c->ldtmp, 1, B, c->s);
  launch_sum_log_dmax(c->Rs.D, sD, n, c->tmpd, B, c->s);
  launch_background(c->md, c->phi, (long long)c->L * 4 * c->nq, c->alpha, c->bg, B, c->s);
  std::vector<double2> ldU(B), bg(B);
  std::vector<double> sdm(B);
  HIPCHK(hipStreamSynchronize(c->s));
  HIPCHK(hipMemcpy(ldU.data(), c->ldtmp, B * sizeof(double2), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(sdm.data(), c->tmpd, B * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(bg.data(), c->bg, B * sizeof(double2), hipMemcpyDeviceToHost));
  re.assign(B, 0.0);
  im.assign(B, 0.0);
  for (int z = 0; z < B; ++z) {
    // ln det(1+B) = ln det Y + sum ln D_R^max + ln det U_R^dagger
    const double lr = ldY[z].x + sdm[z] - ldU[z].x;
    const double li = ldY[z].y - ldU[z].y;
    double r_ = 2.0 * lr + bg[z].x, i_ = 2.0 * li + bg[z].y;
    i_ = std::fmod(i_, 2.0 * M_PI);
    if (i_ > M_PI) i_ -= 2.0 * M_PI;
    if (i_ <= -M_PI) i_ += 2.0 * M_PI;
    if (!std::isfinite(r_)) { c->err = "non-finite weight"; return CFQMC_ENUMERIC; }
    re[z] = r_;
    im[z] = i_;
  }
  return CFQMC_OK;
}

int autotune(cfqmc_ctx* c) {
  // time the channel application, the n x n GEMM and the batched N x N GEMM of
  // the exponential for each tile configuration; keep the fastest of each
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  float best_c = 1e30f, best_g = 1e30f, best_s = 1e30f;
  int bc = 1, bg = 1, bs = 0;
  const long long NN = c->NN, s4 = 4 * NN;
  // the best of three timings of four calls each after a warm-up call: a
  // single timing is too noisy to separate configurations a few percent apart
  auto timeit = [&](auto&& fn) {
    float best = 1e30f;
    fn();   // warm-up
    for (int r = 0; r < 3; ++r) {
      float ms = 0.f;
      hipEventRecord(e0, c->s);
      for (int k = 0; k < 4; ++k) fn();
      hipEventRecord(e1, c->s);
      hipEventSynchronize(e1);
      hipEventElapsedTime(&ms, e0, e1);
      best = std::min(best, ms);
    }
    return best;
  };
  // the FP32 applications keep their FP64 accumulation points (configurations
  // 0..7) unless the precision guard watches every chain's error (then the
  // FP32-accumulating configurations compete as well) or a configuration is
  // fixed by the caller; guarded applications are timed as separate launches
  // here (every chain in FP32), their launch form is chosen below
  const int gl0 = c->guard_launch;
  c->guard_launch = 0;
  for (int cfg = 0; cfg < CFQMC_CHAN_CFGS; ++cfg) {
    if (c->mixed && !c->guard && !chan_cfg_acc64(cfg)) continue;
    c->cfg_chan = cfg;
    if (!c->mixed) c->cfg_chan64 = cfg;   // an FP64 context's applications use cfg_chan64
    const float tc = timeit([&]() {
      chan(c, 1, 1, false, c->PQ, (long long)c->L * 8 * c->NN, c->F[0], c->S1, false, nullptr, c->mixed);
      chan(c, 0, 2, false, c->PQ, (long long)c->L * 8 * c->NN, c->S1, c->S2, false, nullptr, c->mixed);
      if (!c->mixed) {
        // an FP64 sweep's applications are mostly left ones (the Woodbury
        // product, the block products): weight them as in a slice move
        chan(c, 1, 0, false, c->PQ, (long long)c->L * 8 * c->NN, c->S2, c->S1, false, nullptr, 0);
        chan(c, 1, 2, false, c->PQ, (long long)c->L * 8 * c->NN, c->S1, c->S2, false, nullptr, 0);
      }
    });
    if (tc < best_c) { best_c = tc; bc = cfg; }
  }
  // a mixed context also runs FP64 applications (Woodbury product, block
  // products): their tiles are tuned on their own
  int bc64 = bc;
  if (c->mixed) {
    float best = 1e30f;
    for (int cfg = 0; cfg < CFQMC_CHAN_CFGS; ++cfg) {
      c->cfg_chan64 = cfg;
      const float tc = timeit([&]() {
        chan(c, 1, 1, false, c->PQ, (long long)c->L * 8 * c->NN, c->F[0], c->S1, false, nullptr, 0);
        chan(c, 1, 0, false, c->PQ, (long long)c->L * 8 * c->NN, c->S1, c->S2, false, nullptr, 0);
      });
      if (tc < best) { best = tc; bc64 = cfg; }
    }
  }
  for (int cfg = 0; cfg < CFQMC_GEMM_CFGS; ++cfg) {
    c->cfg_gemm = cfg;
    const float tg = timeit([&]() { gemm_nn(c, c->F[0], 0, c->nn, c->F[1], 0, c->nn, c->S1, c->nn, c->nch); });
    if (tg < best_g) { best_g = tg; bg = cfg; }
    // the exponential's products as the sweep runs them: Hermitian tiles with
    // the band of h (h^2) and of h^2 (x^3), and the banded h O
    const int b1 = c->hband, b2 = (b1 >= 0 && 4 * b1 < c->N) ? 2 * b1 : -1;
    const float ts = timeit([&]() {
      GemmArgs g = gemm0(c->N, c->N, c->N);
      g.A = mref(c->H2, c->N, s4, NN); g.B = mref(c->X2, c->N, s4, NN); g.D = mref(c->X3, c->N, s4, NN);
      g.nz2 = 4;
      g.herm = 1;
      g.bandA = g.bandB = b1;
      launch_zgemm(g, c->nch * 4, 0, cfg, c->s);
      g.bandA = -1; g.bandB = b2;
      launch_zgemm(g, c->nch * 4, 0, cfg, c->s);
      g.herm = 0; g.bandA = b1; g.bandB = -1;
      launch_zgemm(g, c->nch * 4, 0, cfg, c->s);
    });
    if (ts < best_s) { best_s = ts; bs = cfg; }
  }
  c->cfg_chan = bc;
  c->cfg_chan64 = bc64;
  c->cfg_gemm = bg;
  c->cfg_small = bs;
  c->guard_launch = gl0;
  if (c->guard && !c->guard_pair_only) {
    // guarded applications: one launch per precision class, or one launch for
    // both in its two register budgets; timed with every other chain in FP64
    std::vector<int> sel(c->nch);
    for (int z = 0; z < c->nch; ++z) sel[z] = z & 1;
    hipMemcpy(c->sel64, sel.data(), c->nch * sizeof(int), hipMemcpyHostToDevice);
    float best = 1e30f;
    int bl = 0;
    for (int v = 0; v < 3; ++v) {
      c->guard_launch = v;
      const float t = timeit([&]() {
        chan(c, 1, 1, false, c->PQ, (long long)c->L * 8 * c->NN, c->F[0], c->S1, false, nullptr, c->mixed);
        chan(c, 0, 2, false, c->PQ, (long long)c->L * 8 * c->NN, c->S1, c->S2, false, nullptr, c->mixed);
      });
      if (t < best) { best = t; bl = v; }
    }
    c->guard_launch = bl;
    hipMemsetAsync(c->sel64, 0, c->nch * sizeof(int), c->s);
    hipStreamSynchronize(c->s);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return CFQMC_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

void cfqmc_default_params(cfqmc_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->n_phi = 6; p->l_tau = 40; p->dtau = 0.1;
  p->u0 = 1.0; p->uk = 1.0; p->un = 1.0;
  p->q_mode = CFQMC_Q_PAPER; p->q_max = 3.0;
  p->n_stab = 10; p->precision = CFQMC_FP64;
  p->eps0 = 0.5; p->r0 = 0.574; p->deps = 0.1; p->eps_min = 1e-3; p->eps_max = 5.0;
  p->adapt_eps = 1; p->seed = 1; p->n_chains = 1;
  p->exp_squarings = 2; p->tile_cfg = -1;
  p->dense4n = 0; p->exact_drift = 0;
  p->precision_guard = 1; p->guard_gmax = 0.8; p->guard_err = 2.5e-7;
  p->sweep_graph = 1;
}

int cfqmc_create(const cfqmc_params* pin, void* hip_stream, cfqmc_ctx** out) {
  if (!pin || !out) return CFQMC_EINVAL;
  *out = nullptr;
  const cfqmc_params& p = *pin;
  if (p.n_phi < 1 || p.n_phi > 140 || p.l_tau < 1 || !(p.dtau > 0) || p.n_chains < 1 || p.n_stab < 1 ||
      !(p.eps0 > 0) || p.eps_min <= 0 || p.eps_max < p.eps_min || p.exp_squarings < 0 || p.exp_squarings > 16 ||
      (p.precision < CFQMC_FP64 || p.precision > CFQMC_MIXED_ALL) || p.tile_cfg < -1 || p.tile_cfg >= CFQMC_CHAN_CFGS)
    return CFQMC_EINVAL;
  if (p.dense4n < 0 || p.dense4n > 1 || p.exact_drift < 0 || p.exact_drift > 1) return CFQMC_EINVAL;
  if (p.precision_guard < 0 || p.precision_guard > 1 || !(p.guard_gmax > 0) || !(p.guard_err > 0)) return CFQMC_EINVAL;
  if (p.sweep_graph < 0 || p.sweep_graph > 1) return CFQMC_EINVAL;
  if (p.dense4n || p.exact_drift) return CFQMC_ENOTIMPL;
  cfqmc_ctx* c = new cfqmc_ctx();
  c->p = p;
  c->p.q_list = nullptr;
  c->p.chain_u = nullptr;
  c->s = (hipStream_t)hip_stream;
  c->N = p.n_phi; c->n = 2 * p.n_phi; c->L = p.l_tau; c->nch = p.n_chains; c->nstab = p.n_stab;
  c->nblk_stab = (p.l_tau + p.n_stab - 1) / p.n_stab;
  c->mixed = p.precision != CFQMC_FP64;
  c->mixed_m = p.precision == CFQMC_MIXED_ALL;
  c->guard = c->mixed && p.precision_guard;
  c->blocks_in_call = 0;
  c->smax = p.exp_squarings;
  c->nn = (long long)c->n * c->n;
  c->NN = (long long)c->N * c->N;
  c->ready = false;
  c->dev = 0;
  hipGetDevice(&c->dev);
  c->lu_lmax = 8.0;
  if (const char* e = std::getenv("CFQMC_LU_NP_LMAX")) c->lu_lmax = std::atof(e);
  // testing knob: CFQMC_GUARD_PAIR=1 keeps one launch per precision class
  c->guard_pair_only = false;
  if (const char* e = std::getenv("CFQMC_GUARD_PAIR")) c->guard_pair_only = e[0] == '1';
  c->guard_launch = c->guard_pair_only ? 0 : 1;
  c->timing = false;
  c->ev_used = 0;
  c->sweep_counter = 0;
  if (!build_components(p, c->ht, c->err)) { g_create_err = c->err; delete c; return CFQMC_EINVAL; }
  c->nq = (int)c->ht.comp_kind.size();
  // band of h: the largest circular shift that carries a term
  c->hband = 0;
  for (int d = 0; d < c->N; ++d)
    if (c->ht.hoff[d + 1] > c->ht.hoff[d]) c->hband = std::max(c->hband, std::min(d, c->N - d));
  if (4 * c->hband >= c->N) c->hband = -1;
  // valley rotations: columns are the +1 / -1 eigenvectors of o_i
  const double r = 1.0 / std::sqrt(2.0);
  for (int ch = 0; ch < 4; ++ch) {
    for (int i = 0; i < 2; ++i) for (int j = 0; j < 2; ++j) c->Urot[ch][i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  c->Urot[1][0][0] = make_double2(r, 0); c->Urot[1][0][1] = make_double2(r, 0);
  c->Urot[1][1][0] = make_double2(r, 0); c->Urot[1][1][1] = make_double2(-r, 0);
  c->Urot[2][0][0] = make_double2(r, 0); c->Urot[2][0][1] = make_double2(r, 0);
  c->Urot[2][1][0] = make_double2(0, r); c->Urot[2][1][1] = make_double2(0, -r);

  const int B = c->nch, n = c->n, nq = c->nq, L = c->L, nb = c->nblk_stab;
  const long long nn = c->nn, NN = c->NN;
  c->exp_cap = std::max(1, std::min(L, 32));
  const long long ecap = (long long)std::max(B, c->exp_cap) * 4 * NN;
  int rc = 0;
  rc |= dalloc(c, &c->phi, (size_t)B * L * 4 * nq);
  rc |= dalloc(c, &c->PQ, (size_t)B * L * 8 * NN);
  rc |= dalloc(c, &c->G, (size_t)B * nn);
  for (int i = 0; i < 4; ++i) { rc |= dalloc(c, &c->F[i], (size_t)B * nn); rc |= dalloc(c, &c->Fp[i], (size_t)B * nn); }
  rc |= dalloc(c, &c->S1, (size_t)B * nn);
  rc |= dalloc(c, &c->S2, (size_t)B * nn);
  rc |= dalloc(c, &c->Mw, (size_t)B * nn);
  rc |= dalloc(c, &c->Mb, (size_t)B * nn);
  rc |= dalloc(c, &c->lu_flag, (size_t)B);
  rc |= dalloc(c, &c->ipiv, (size_t)B * n);
  rc |= dalloc(c, &c->lndet, (size_t)B);
  rc |= dalloc(c, &c->ldtmp, (size_t)B);
  rc |= dalloc(c, &c->phip, (size_t)B * 4 * nq);
  rc |= dalloc(c, &c->PQp, (size_t)B * 8 * NN);
  rc |= dalloc(c, &c->h, (size_t)ecap);
  double2** ebufs[] = {&c->H2, &c->X2, &c->X3, &c->Eo, &c->Oo};
  for (auto bp : ebufs) rc |= dalloc(c, bp, (size_t)ecap);
  rc |= dalloc(c, &c->Wa, (size_t)2 * ecap);
  rc |= dalloc(c, &c->Wb, (size_t)2 * ecap);
  rc |= dalloc(c, &c->coef, (size_t)(ecap / NN) * EXP_NC);
  rc |= dalloc(c, &c->sq, (size_t)(ecap / NN) * 2);
  rc |= dalloc(c, &c->d_err, 1);
  rc |= dalloc(c, &c->Cb, (size_t)B * nb * nn);
  rc |= dalloc(c, &c->Ls.U, (size_t)B * (nb + 1) * nn);
  rc |= dalloc(c, &c->Ls.T, (size_t)B * (nb + 1) * nn);
  rc |= dalloc(c, &c->Ls.D, (size_t)B * (nb + 1) * n);
  rc |= dalloc(c, &c->Rs.U, (size_t)B * (nb + 1) * nn);
  rc |= dalloc(c, &c->Rs.T, (size_t)B * (nb + 1) * nn);
  rc |= dalloc(c, &c->Rs.D, (size_t)B * (nb + 1) * n);
  double2** sbufs[] = {&c->W1, &c->A1, &c->Gr, &c->Q1, &c->Q2, &c->R1, &c->R2, &c->Rt, &c->Tp, &c->K1, &c->M1, &c->Yl, &c->Wm, &c->X1, &c->Gs};
  for (auto bp : sbufs) rc |= dalloc(c, bp, (size_t)B * nn);
  rc |= dalloc(c, &c->rs_ws, (size_t)B * rsolve_work_size(n));
  double** dbufs[] = {&c->nrm, &c->sqd1, &c->sqd2, &c->dinvL, &c->dinvR, &c->tmpd, &c->dminL, &c->dminR};
  for (auto bp : dbufs) rc |= dalloc(c, bp, (size_t)B * n);
  rc |= dalloc(c, &c->perm, (size_t)B * n);
  rc |= dalloc(c, &c->alpha, (size_t)B * 4);
  rc |= dalloc(c, &c->eps, (size_t)B);
  rc |= dalloc(c, &c->acc_count, (size_t)B);
  rc |= dalloc(c, &c->lnA, (size_t)B);
  rc |= dalloc(c, &c->accept, (size_t)B);
  rc |= dalloc(c, &c->stat, (size_t)B * 8);
  rc |= dalloc(c, &c->part, (size_t)B * 4 * 4 * 1024);
  rc |= dalloc(c, &c->obs, (size_t)B * 8);
  rc |= dalloc(c, &c->stab_err, (size_t)B * 4);
  c->series_cap = 1 << 16;
  rc |= dalloc(c, &c->series, (size_t)B * c->series_cap);
  rc |= dalloc(c, &c->series_s, (size_t)B * c->series_cap);
  rc |= dalloc(c, &c->series_p, (size_t)B * c->series_cap);
  rc |= dalloc(c, &c->fsq, (size_t)B);
  rc |= dalloc(c, &c->fq0, (size_t)B);
  rc |= dalloc(c, &c->ldY2, (size_t)B);
  rc |= dalloc(c, &c->hist_acc, (size_t)B * L);
  rc |= dalloc(c, &c->hist_lnA, (size_t)B * L);
  rc |= dalloc(c, &c->noise, (size_t)B * L * (4 * nq + 1));
  rc |= dalloc(c, &c->bg, (size_t)B);
  rc |= dalloc(c, &c->sel64, (size_t)B);
  rc |= dalloc(c, &c->guard_cnt, (size_t)B);
  rc |= dalloc(c, &c->d_counter, (size_t)1);
  rc |= dalloc(c, &c->d_series_len, (size_t)1);
  rc |= dalloc(c, &c->gmax_run, (size_t)B);
  rc |= dalloc(c, &c->blk_last, (size_t)B * 2);
  if (rc) { g_create_err = c->err; cfqmc_destroy(c); return CFQMC_ENOMEM; }
  // h is zero on the diagonals without terms, which build_h never writes
  if (hipMemsetAsync(c->h, 0, (size_t)ecap * sizeof(double2), c->s) != hipSuccess) {
    (void)hipGetLastError();
    g_create_err = "clearing the h buffer failed";
    cfqmc_destroy(c);
    return CFQMC_EHIP;
  }
  if (build_model_dev(c)) {
    g_create_err = "model tables: " + c->err;
    cfqmc_destroy(c);
    return CFQMC_ENOMEM;
  }
  if (c->md.nrow * 4 > 4 * 1024) { g_create_err = "too many momentum rows"; cfqmc_destroy(c); return CFQMC_EINVAL; }
  // couplings per chain: g = (U0+UN, -(UK+UN), -(UK+UN), 2 UN), alpha = sqrt(-dtau g)
  std::vector<double2> al(B * 4);
  for (int z = 0; z < B; ++z) {
    double u0 = p.u0, uk = p.uk, un = p.un;
    if (pin->chain_u) { u0 = pin->chain_u[3 * z]; uk = pin->chain_u[3 * z + 1]; un = pin->chain_u[3 * z + 2]; }
    const double g[4] = {u0 + un, -(uk + un), -(uk + un), 2.0 * un};
    for (int i = 0; i < 4; ++i) {
      const double x = -p.dtau * g[i];
      al[z * 4 + i] = x >= 0 ? make_double2(std::sqrt(x), 0.0) : make_double2(0.0, std::sqrt(-x));
    }
  }
  if (hipMemcpyAsync(c->alpha, al.data(), al.size() * sizeof(double2), hipMemcpyHostToDevice, c->s) != hipSuccess) {
    cfqmc_destroy(c);
    return CFQMC_EHIP;
  }
  c->cfg_chan = p.tile_cfg >= 0 ? p.tile_cfg : 1;
  c->cfg_chan64 = c->cfg_chan;
  c->cfg_gemm = p.tile_cfg >= 0 ? std::min(p.tile_cfg, CFQMC_GEMM_CFGS - 1) : 1;
  c->cfg_small = 0;
  if (hipStreamSynchronize(c->s) != hipSuccess) { cfqmc_destroy(c); return CFQMC_EHIP; }
  if (p.tile_cfg < 0) autotune(c);
  *out = c;
  return CFQMC_OK;
}

int cfqmc_destroy(cfqmc_ctx* c) {
  if (!c) return CFQMC_EINVAL;
  hipStreamSynchronize(c->s);
  for (int m = 0; m < 2; ++m) {
    for (hipGraphExec_t x : c->gexec[m]) hipGraphExecDestroy(x);
    for (auto& it : c->titems[m])
      if (it.x) hipGraphExecDestroy(it.x);
  }
  for (hipEvent_t e : c->ev) hipEventDestroy(e);
  for (hipEvent_t e : c->ev2) hipEventDestroy(e);
  for (void* q : c->allocs) hipFree(q);
  delete c;
  return CFQMC_OK;
}

int cfqmc_sizes(const cfqmc_ctx* c, int32_t* n_q, int32_t* n_chains, int32_t* dim_g4n) {
  if (!c) return CFQMC_EINVAL;
  if (n_q) *n_q = c->nq;
  if (n_chains) *n_chains = c->nch;
  if (dim_g4n) *dim_g4n = 4 * c->N;
  return CFQMC_OK;
}

int cfqmc_init_fields(cfqmc_ctx* c, const double* phi) {
  if (!c) return CFQMC_EINVAL;
  const int B = c->nch, L = c->L, nq = c->nq;
  const long long cnt = (long long)B * L * 4 * nq;
  std::vector<double> h(cnt);
  if (phi) {
    memcpy(h.data(), phi, cnt * sizeof(double));
    for (double v : h)
      if (!std::isfinite(v)) { c->err = "non-finite field"; return CFQMC_EINVAL; }
  } else {
    // N(0,1) by Box-Muller on a host Philox-independent splitmix stream of the seed
    uint64_t st = c->p.seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    auto next = [&]() {
      st += 0x9E3779B97F4A7C15ull;
      uint64_t z = st;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      return z ^ (z >> 31);
    };
    for (long long i = 0; i < cnt; i += 2) {
      const double u1 = ((next() >> 11) + 1.0) * (1.0 / 9007199254740993.0);
      const double u2 = (next() >> 11) * (1.0 / 9007199254740992.0);
      const double rr = std::sqrt(-2.0 * std::log(u1));
      h[i] = rr * std::cos(2.0 * M_PI * u2);
      if (i + 1 < cnt) h[i + 1] = rr * std::sin(2.0 * M_PI * u2);
    }
  }
  HIPCHK(hipMemcpyAsync(c->phi, h.data(), cnt * sizeof(double), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipMemsetAsync(c->d_err, 0, sizeof(int), c->s));
  HIPCHK(hipMemsetAsync(c->sel64, 0, c->nch * sizeof(int), c->s));   // every chain starts in FP32
  HIPCHK(hipGetLastError());
  set_udt_identity(c, c->Rs, c->nblk_stab);
  set_udt_identity(c, c->Ls, 0);
  rebuild_state(c);
  std::vector<double> e(B, c->p.eps0);
  HIPCHK(hipMemcpyAsync(c->eps, e.data(), B * sizeof(double), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipMemsetAsync(c->acc_count, 0, B * sizeof(int), c->s));
  HIPCHK(hipMemsetAsync(c->stat, 0, B * 8 * sizeof(double), c->s));
  HIPCHK(hipMemsetAsync(c->stab_err, 0, B * 4 * sizeof(double), c->s));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->s));
  int ef = 0;
  HIPCHK(hipMemcpy(&ef, c->d_err, sizeof(int), hipMemcpyDeviceToHost));
  c->series_len = 0;
  c->sweep_counter = 0;
  HIPCHK(upload_counters(c));
  if (ef) { c->err = dev_err_msg(ef) + " at init"; c->ready = false; return CFQMC_ENUMERIC; }
  std::vector<double2> g(c->nn);
  HIPCHK(hipMemcpy(g.data(), c->G, c->nn * sizeof(double2), hipMemcpyDeviceToHost));
  for (auto& v : g)
    if (!std::isfinite(v.x) || !std::isfinite(v.y)) { c->err = "non-finite G at init"; c->ready = false; return CFQMC_ENUMERIC; }
  c->ready = true;
  return CFQMC_OK;
}

int cfqmc_get_fields(cfqmc_ctx* c, double* phi_out) {
  if (!c || !phi_out) return CFQMC_EINVAL;
  HIPCHK(hipStreamSynchronize(c->s));
  HIPCHK(hipMemcpy(phi_out, c->phi, (size_t)c->nch * c->L * 4 * c->nq * sizeof(double), hipMemcpyDeviceToHost));
  return CFQMC_OK;
}

// Checkpoint file: header, then fields [B][L][4][n_q], eps [B], couplings
// alpha [B][4] (complex), the three series (m^2, action, q = 0 power) each
// [B][series_len]; all FP64, native byte order.
struct CkptHeader {
  char magic[8];
  int32_t version, n_phi, l_tau, n_q, n_chains, n_stab;
  uint64_t seed;
  int64_t sweep_counter;
  int32_t series_len, pad;
};
static const char kCkptMagic[8] = {'C', 'F', 'Q', 'M', 'C', 'C', 'K', '1'};

int cfqmc_checkpoint(cfqmc_ctx* c, const char* path) {
  if (!c || !path) return CFQMC_EINVAL;
  if (!c->ready) { c->err = "checkpoint: no fields initialised"; return CFQMC_ESTATE; }
  const int B = c->nch;
  const long long cnt = (long long)B * c->L * 4 * c->nq;
  const size_t ns = (size_t)B * std::max(c->series_len, 0);
  std::vector<double> phi(cnt), eps(B), ser(3 * ns);
  std::vector<double2> al((size_t)B * 4);
  const double* srcs[3] = {c->series, c->series_s, c->series_p};
  HIPCHK(hipStreamSynchronize(c->s));
  HIPCHK(hipMemcpy(phi.data(), c->phi, cnt * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(eps.data(), c->eps, B * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(al.data(), c->alpha, al.size() * sizeof(double2), hipMemcpyDeviceToHost));
  for (int w = 0; w < 3; ++w)
    for (int z = 0; z < B && c->series_len > 0; ++z)
      HIPCHK(hipMemcpy(ser.data() + w * ns + (size_t)z * c->series_len, srcs[w] + (long long)z * c->series_cap,
                       c->series_len * sizeof(double), hipMemcpyDeviceToHost));
  CkptHeader h;
  memset(&h, 0, sizeof(h));
  memcpy(h.magic, kCkptMagic, 8);
  h.version = 2; h.n_phi = c->N; h.l_tau = c->L; h.n_q = c->nq; h.n_chains = B; h.n_stab = c->nstab;
  h.seed = c->p.seed; h.sweep_counter = c->sweep_counter; h.series_len = c->series_len;
  FILE* f = std::fopen(path, "wb");
  if (!f) { c->err = std::string("checkpoint: cannot open ") + path; return CFQMC_EINVAL; }
  bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 &&
            std::fwrite(phi.data(), sizeof(double), cnt, f) == (size_t)cnt &&
            std::fwrite(eps.data(), sizeof(double), B, f) == (size_t)B &&
            std::fwrite(al.data(), sizeof(double2), al.size(), f) == al.size() &&
            std::fwrite(ser.data(), sizeof(double), ser.size(), f) == ser.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) { c->err = std::string("checkpoint: write failed on ") + path; return CFQMC_EINVAL; }
  return CFQMC_OK;
}

int cfqmc_restore(cfqmc_ctx* c, const char* path) {
  if (!c || !path) return CFQMC_EINVAL;
  FILE* f = std::fopen(path, "rb");
  if (!f) { c->err = std::string("restore: cannot open ") + path; return CFQMC_EINVAL; }
  CkptHeader h;
  const int B = c->nch;
  const long long cnt = (long long)B * c->L * 4 * c->nq;
  bool ok = std::fread(&h, sizeof(h), 1, f) == 1 && memcmp(h.magic, kCkptMagic, 8) == 0 && h.version == 2;
  if (ok && (h.n_phi != c->N || h.l_tau != c->L || h.n_q != c->nq || h.n_chains != B || h.series_len < 0 ||
             h.series_len > c->series_cap)) {
    std::fclose(f);
    c->err = "restore: checkpoint shape differs from the context";
    return CFQMC_EINVAL;
  }
  const size_t ns = ok ? (size_t)B * h.series_len : 0;
  std::vector<double> phi(ok ? cnt : 0), eps(ok ? B : 0), ser(3 * ns);
  std::vector<double2> al(ok ? (size_t)B * 4 : 0), al_ctx((size_t)B * 4);
  ok = ok && std::fread(phi.data(), sizeof(double), cnt, f) == (size_t)cnt &&
       std::fread(eps.data(), sizeof(double), B, f) == (size_t)B &&
       std::fread(al.data(), sizeof(double2), al.size(), f) == al.size() &&
       std::fread(ser.data(), sizeof(double), ser.size(), f) == ser.size();
  std::fclose(f);
  if (!ok) { c->err = std::string("restore: not a readable checkpoint: ") + path; return CFQMC_EINVAL; }
  HIPCHK(hipStreamSynchronize(c->s));
  HIPCHK(hipMemcpy(al_ctx.data(), c->alpha, al_ctx.size() * sizeof(double2), hipMemcpyDeviceToHost));
  for (size_t i = 0; i < al.size(); ++i)
    if (al[i].x != al_ctx[i].x || al[i].y != al_ctx[i].y) {
      c->err = "restore: checkpoint couplings differ from the context";
      return CFQMC_EINVAL;
    }
  for (long long i = 0; i < cnt; ++i)
    if (!std::isfinite(phi[i])) { c->err = "restore: non-finite field"; return CFQMC_EINVAL; }
  // the state is rebuilt from the fields (all slice propagators, UDT stacks,
  // G(0) in FP64); eps, the RNG position and the series continue
  const int rc = cfqmc_init_fields(c, phi.data());
  if (rc != CFQMC_OK) return rc;
  HIPCHK(hipMemcpy(c->eps, eps.data(), B * sizeof(double), hipMemcpyHostToDevice));
  double* dsts[3] = {c->series, c->series_s, c->series_p};
  for (int w = 0; w < 3; ++w)
    for (int z = 0; z < B && h.series_len > 0; ++z)
      HIPCHK(hipMemcpy(dsts[w] + (long long)z * c->series_cap, ser.data() + w * ns + (size_t)z * h.series_len,
                       h.series_len * sizeof(double), hipMemcpyHostToDevice));
  c->series_len = h.series_len;
  c->sweep_counter = h.sweep_counter;
  HIPCHK(upload_counters(c));
  // the seed is an argument of the recorded sweeps' kernels: record them again
  if (c->p.seed != h.seed) drop_graphs(c);
  c->p.seed = h.seed;
  return CFQMC_OK;
}

}  // extern "C"

namespace {

// Sweep pieces shared by cfqmc_sweep and the heterogeneous batch.
void sweep_reset_stats(cfqmc_ctx* c) {
  hipMemsetAsync(c->stat, 0, c->nch * 8 * sizeof(double), c->s);
  hipMemsetAsync(c->stab_err, 0, c->nch * 4 * sizeof(double), c->s);
  hipMemsetAsync(c->guard_cnt, 0, c->nch * sizeof(int), c->s);
  hipMemsetAsync(c->gmax_run, 0, c->nch * sizeof(double), c->s);
  c->blocks_in_call = 0;
  c->sweeps_in_call = 0;
  c->graph_sweeps_in_call = 0;
}

void sweep_slice(cfqmc_ctx* c, int t, const double* noise_dev) {
  slice_step(c, t, noise_dev);
  if ((t + 1) % c->nstab == 0 || t == c->L - 1) block_end(c, t / c->nstab);
}

// Launches of the end of a sweep (step size, observables, right stack, the
// series entry, counters advanced on the device).
void sweep_end_dev(cfqmc_ctx* c) {
  const int B = c->nch;
  launch_eps_update(c->eps, c->acc_count, c->L, c->p.r0, c->p.deps, c->p.eps_min, c->p.eps_max, c->p.adapt_eps, B,
                    c->s);
  launch_observables(c->G, c->nn, c->N, q0_weight(c), c->obs, 8, B, c->s);
  restack_right(c);
  // per-sweep series for the autocorrelation: m^2_SO(5), the action and the
  // q = 0 field power (ln w_F from the fresh right stack, as cfqmc_logdet);
  // entry *d_series_len, skipped on the device once the series is full
  const long long nn = c->nn, sU = sU_(c), sD = sD_(c);
  green_udt(c, 0, 0, c->Gs);   // ln det Y in ldtmp
  launch_copy((const double2*)c->ldtmp, c->ldY2, 1, 1, 1, B, c->s);
  launch_copy(c->Rs.U, c->Q2, nn, sU, nn, B, c->s);
  launch_lu(c->Q2, c->n, c->n, nn, c->ipiv, c->n, c->ldtmp, 1, B, c->s);
  launch_sum_log_dmax(c->Rs.D, sD, c->n, c->tmpd, B, c->s);
  launch_background(c->md, c->phi, (long long)c->L * 4 * c->nq, c->alpha, c->bg, B, c->s);
  launch_field_sums(c->phi, (long long)c->L * 4 * c->nq, c->L, c->nq, c->fsq, c->fq0, B, c->s);
  launch_action_series(c->ldY2, c->ldtmp, c->tmpd, c->bg, c->fsq, c->fq0, c->obs + 5, 8, c->series, c->series_s,
                       c->series_p, c->series_cap, c->d_series_len, B, c->s);
  launch_sweep_advance(c->d_counter, c->d_series_len, c->series_cap, c->s);
}

// Host copies of the device counters after a sweep.
void sweep_end_host(cfqmc_ctx* c) {
  if (c->series_len < c->series_cap) c->series_len++;
  c->sweep_counter++;
  c->sweeps_in_call++;
}

// Reports (once per context) why sweeps run launch by launch.
void graph_note(cfqmc_ctx* c, const char* step, hipError_t e) {
  if (c->graph_noted) return;
  c->graph_noted = true;
  std::fprintf(stderr, "[cfqmc] recorded sweep graph not used (%s: %s); sweeps run launch by launch\n", step,
               hipGetErrorString(e));
}

void sweep_end(cfqmc_ctx* c) {
  sweep_end_dev(c);
  sweep_end_host(c);
}

// With kernel timing on, the timing variant runs: the timing events must be
// recorded by the runtime on the stream (events recorded inside a graph are
// not timed by this runtime).
bool graph_usable(const cfqmc_ctx* c) {
  return c->p.sweep_graph && c->s != nullptr && !cfqmc_debug_sync();
}

// Slices per recorded chunk: whole stabilisation blocks, at most about 64
// slices (a few thousand launches per graph).
int chunk_slices(const cfqmc_ctx* c) {
  return std::max(1, 64 / c->nstab) * c->nstab;
}

// Records the launches of one whole sweep (m = 0: device noise, 1: replayed
// noise from c->noise) on the context's stream as graphs, one per chunk of
// slices. Recording runs no kernel; a failure leaves the context on launches
// one by one.
void record_sweep(cfqmc_ctx* c, int m) {
  c->graph_state[m] = -1;
  const long long blocks0 = c->blocks_in_call;
  const int S = chunk_slices(c);
  std::vector<hipGraphExec_t> execs;
  const char* step = nullptr;
  hipError_t err = hipSuccess;
  size_t nodes = 0;
  for (int t0 = 0; t0 < c->L && !step; t0 += S) {
    err = hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal);
    if (err != hipSuccess) { step = "begin capture"; break; }
    const int t1 = std::min(c->L, t0 + S);
    for (int t = t0; t < t1; ++t) sweep_slice(c, t, m ? c->noise : nullptr);
    if (t1 == c->L) sweep_end_dev(c);
    hipGraph_t g = nullptr;
    err = hipStreamEndCapture(c->s, &g);
    if (err != hipSuccess || !g) {
      if (g) hipGraphDestroy(g);
      step = "end capture";
      break;
    }
    (void)hipGraphGetNodes(g, nullptr, &nodes);
    hipGraphExec_t x = nullptr;
    err = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (err != hipSuccess) { step = "instantiate"; break; }
    execs.push_back(x);
  }
  c->blocks_per_sweep = c->blocks_in_call - blocks0;
  c->blocks_in_call = blocks0;
  if (step) {
    (void)hipGetLastError();
    for (hipGraphExec_t x : execs) hipGraphExecDestroy(x);
    std::fprintf(stderr, "[cfqmc] sweep graph chunk of %d slices, %zu nodes\n", S, nodes);
    graph_note(c, step, err);
    return;
  }
  c->gexec[m] = execs;
  c->graph_state[m] = 1;
}

// Records the timing variant of one sweep (see titems). Recording runs no
// kernel unless a capture cannot be restarted (then the context needs new
// fields: the call fails).
void record_timed_sweep(cfqmc_ctx* c, int m) {
  c->tstate[m] = -1;
  const long long blocks0 = c->blocks_in_call;
  c->seg_fail = nullptr;
  c->seg_broken = false;
  c->seg_m = m;
  hipError_t e = hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    graph_note(c, "begin capture (timed sweep)", e);
    return;
  }
  c->seg_rec = true;
  for (int t = 0; t < c->L; ++t) sweep_slice(c, t, m ? c->noise : nullptr);
  sweep_end_dev(c);
  c->seg_rec = false;
  if (!c->seg_broken) {
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->s, &g);
    if (e == hipSuccess && g) {
      size_t nodes = 0;
      (void)hipGraphGetNodes(g, nullptr, &nodes);
      hipGraphExec_t x = nullptr;
      if (nodes > 0) {
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e == hipSuccess) c->titems[m].push_back({x, -1, nullptr});
        else if (!c->seg_fail) { c->seg_fail = "instantiate"; c->seg_fail_err = e; }
      }
      hipGraphDestroy(g);
    } else {
      if (g) hipGraphDestroy(g);
      if (!c->seg_fail) { c->seg_fail = "end capture"; c->seg_fail_err = e; }
    }
  }
  c->blocks_per_sweep = c->blocks_in_call - blocks0;
  c->blocks_in_call = blocks0;
  if (c->seg_broken) {
    c->err = "recording the timed sweep graph ran launches: fields must be initialised again";
    c->launch_failed = true;
  }
  if (c->seg_fail) {
    (void)hipGetLastError();
    for (auto& it : c->titems[m])
      if (it.x) hipGraphExecDestroy(it.x);
    c->titems[m].clear();
    graph_note(c, c->seg_fail, c->seg_fail_err);
    return;
  }
  c->tstate[m] = 1;
}

// Queues one sweep of all chains: as launches of the recorded graphs where the
// context allows it (with kernel timing on: the timing variant, HIP events
// around its timed pieces), else launch by launch. replay: noise from c->noise.
void run_sweep(cfqmc_ctx* c, bool replay) {
  const int m = replay ? 1 : 0;
  if (graph_usable(c) && c->timing) {
    if (c->tstate[m] == 0) record_timed_sweep(c, m);
    if (c->launch_failed) return;
    if (c->tstate[m] == 1) {
      hipError_t e = hipSuccess;
      for (auto& it : c->titems[m]) {
        if (e != hipSuccess) break;
        if (it.kind < 0) {
          e = hipGraphLaunch(it.x, c->s);
          continue;
        }
        std::vector<hipEvent_t>& ev = it.kind ? c->ev2 : c->ev;
        size_t& used = it.kind ? c->ev2_used : c->ev_used;
        const bool rec = used + 2 <= ev.size();
        if (rec) hipEventRecord(ev[used], c->s);
        it.launch();
        if (rec) {
          hipEventRecord(ev[used + 1], c->s);
          used += 2;
        }
      }
      if (e == hipSuccess) {
        c->blocks_in_call += c->blocks_per_sweep;
        c->graph_sweeps_in_call++;
        sweep_end_host(c);
        return;
      }
      c->err = std::string("timed sweep graph launch failed: ") + hipGetErrorString(e);
      graph_note(c, "launch (timed sweep)", e);
      c->launch_failed = true;
      sweep_end_host(c);
      return;
    }
  }
  if (graph_usable(c) && !c->timing) {
    if (c->graph_state[m] == 0) record_sweep(c, m);
    if (c->graph_state[m] == 1) {
      hipError_t e = hipSuccess;
      for (hipGraphExec_t x : c->gexec[m])
        if (e == hipSuccess) e = hipGraphLaunch(x, c->s);
      if (e == hipSuccess) {
        c->blocks_in_call += c->blocks_per_sweep;
        c->graph_sweeps_in_call++;
        sweep_end_host(c);
        return;
      }
      // a chunk that failed to launch leaves the sweep incomplete: an error the
      // caller sees at the end of the call
      c->err = std::string("sweep graph launch failed: ") + hipGetErrorString(e);
      graph_note(c, "launch", e);
      for (hipGraphExec_t x : c->gexec[m]) hipGraphExecDestroy(x);
      c->gexec[m].clear();
      c->graph_state[m] = -1;
      c->launch_failed = true;
      sweep_end_host(c);
      return;
    }
  }
  for (int t = 0; t < c->L; ++t) sweep_slice(c, t, replay ? c->noise : nullptr);
  sweep_end(c);
}

int sweep_collect(cfqmc_ctx* c, cfqmc_stats* stats) {
  const int B = c->nch;
  if (c->launch_failed) {
    // the fields and G are no longer a consistent Markov-chain state
    c->launch_failed = false;
    c->ready = false;
    (void)hipStreamSynchronize(c->s);
    return CFQMC_EHIP;
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->s));
  int ef = 0;
  HIPCHK(hipMemcpy(&ef, c->d_err, sizeof(int), hipMemcpyDeviceToHost));
  std::vector<double> st(B * 8), se(B * 4), ep(B), gm(B);
  std::vector<int> gc(B);
  HIPCHK(hipMemcpy(st.data(), c->stat, B * 8 * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(se.data(), c->stab_err, B * 4 * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(ep.data(), c->eps, B * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(gm.data(), c->gmax_run, B * sizeof(double), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(gc.data(), c->guard_cnt, B * sizeof(int), hipMemcpyDeviceToHost));
  bool bad = ef != 0;
  for (int z = 0; z < B; ++z) {
    if (!std::isfinite(se[4 * z]) || !std::isfinite(ep[z])) bad = true;
    if (stats) {
      stats[z].proposed = (int64_t)st[z * 8 + 1];
      stats[z].accepted = (int64_t)st[z * 8 + 2];
      stats[z].eps = ep[z];
      stats[z].max_stab_err = se[4 * z];
      stats[z].max_stab_rel = se[4 * z + 1];
      stats[z].max_phase_err = st[z * 8 + 0];
      stats[z].exp_range_flag = ef;
      stats[z].pad = 0;
      stats[z].max_abs_g = gm[z];
      // the guard's choice at the last block end of a sweep applies to the next sweep
      stats[z].fp64_guard_frac = c->blocks_in_call ? (double)gc[z] / (double)c->blocks_in_call : 0.0;
      stats[z].graph_sweep_frac =
          c->sweeps_in_call ? (double)c->graph_sweeps_in_call / (double)c->sweeps_in_call : 0.0;
    }
  }
  if (bad) {
    c->ready = false;
    c->err = ef ? dev_err_msg(ef) : "non-finite state (G, its FP64 recomputation or the step size)";
    return CFQMC_ENUMERIC;
  }
  return CFQMC_OK;
}

}  // namespace

struct cfqmc_batch {
  std::vector<cfqmc_ctx*> g;
  std::vector<hipStream_t> streams;
  std::string err;
};

// Average duration of the event pairs [0, used) of ev (one timed channel
// application each) and the flops of one such application: two N x N x n
// complex products per chain, 8 * 2 N^2 n real flops.
static int timing_average(cfqmc_ctx* c, const std::vector<hipEvent_t>& ev, size_t used, double* avg_ms,
                          int64_t* count, double* flops_per_launch) {
  HIPCHK(hipStreamSynchronize(c->s));
  double tot = 0.0;
  const int64_t k = (int64_t)(used / 2);
  for (int64_t i = 0; i < k; ++i) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
    tot += ms;
  }
  if (avg_ms) *avg_ms = k ? tot / k : 0.0;
  if (count) *count = k;
  if (flops_per_launch) *flops_per_launch = 8.0 * 2.0 * (double)c->N * c->N * c->n * c->nch;
  return CFQMC_OK;
}

extern "C" {

int cfqmc_sweep(cfqmc_ctx* c, int32_t n_sweeps, const double* replay, cfqmc_stats* stats) {
  if (!c || n_sweeps < 0) return CFQMC_EINVAL;
  if (!c->ready) { c->err = "fields not initialised"; return CFQMC_ESTATE; }
  const int B = c->nch, L = c->L, W = 4 * c->nq + 1;
  sweep_reset_stats(c);
  for (int sw = 0; sw < n_sweeps; ++sw) {
    if (replay) {
      HIPCHK(hipMemcpy2DAsync(c->noise, (size_t)L * W * sizeof(double), replay + (size_t)sw * L * W,
                              (size_t)n_sweeps * L * W * sizeof(double), (size_t)L * W * sizeof(double), B,
                              hipMemcpyHostToDevice, c->s));
    }
    run_sweep(c, replay != nullptr);
  }
  return sweep_collect(c, stats);
}

int cfqmc_batch_create(const cfqmc_params* groups, int32_t n_groups, cfqmc_batch** out) {
  if (!groups || n_groups < 1 || !out) return CFQMC_EINVAL;
  *out = nullptr;
  cfqmc_batch* b = new cfqmc_batch();
  for (int k = 0; k < n_groups; ++k) {
    hipStream_t st = nullptr;
    if (hipStreamCreate(&st) != hipSuccess) { cfqmc_batch_destroy(b); return CFQMC_EHIP; }
    b->streams.push_back(st);
    cfqmc_ctx* c = nullptr;
    const int rc = cfqmc_create(&groups[k], (void*)st, &c);
    if (rc) { cfqmc_batch_destroy(b); return rc; }
    b->g.push_back(c);
  }
  *out = b;
  return CFQMC_OK;
}

int cfqmc_batch_destroy(cfqmc_batch* b) {
  if (!b) return CFQMC_EINVAL;
  for (auto c : b->g) cfqmc_destroy(c);
  for (auto st : b->streams) hipStreamDestroy(st);
  delete b;
  return CFQMC_OK;
}

int cfqmc_batch_context(cfqmc_batch* b, int32_t group, cfqmc_ctx** ctx) {
  if (!b || !ctx || group < 0 || group >= (int)b->g.size()) return CFQMC_EINVAL;
  *ctx = b->g[group];
  return CFQMC_OK;
}

int cfqmc_batch_get(cfqmc_batch* b, int32_t chain, cfqmc_ctx** view, int32_t* local_chain) {
  if (!b || !view || chain < 0) return CFQMC_EINVAL;
  int off = 0;
  for (cfqmc_ctx* c : b->g) {
    if (chain < off + c->nch) {
      *view = c;
      if (local_chain) *local_chain = chain - off;
      return CFQMC_OK;
    }
    off += c->nch;
  }
  return CFQMC_EINVAL;
}

int cfqmc_batch_sweep_replay(cfqmc_batch* b, int32_t n_sweeps, const double* const* replay, cfqmc_stats* stats) {
  if (!b || n_sweeps < 0) return CFQMC_EINVAL;
  const int G = (int)b->g.size();
  int Lmax = 0;
  for (auto c : b->g) {
    if (!c->ready) { b->err = "fields not initialised"; return CFQMC_ESTATE; }
    Lmax = std::max(Lmax, c->L);
    sweep_reset_stats(c);
  }
  bool graphs = true;
  for (auto c : b->g) graphs = graphs && graph_usable(c);
  if (graphs) {
    // one recorded sweep per group and sweep, each group on its own stream
    for (int sw = 0; sw < n_sweeps; ++sw)
      for (int q = 0; q < G; ++q) {
        cfqmc_ctx* c = b->g[q];
        const double* rp = replay ? replay[q] : nullptr;
        if (rp) {
          const int W = 4 * c->nq + 1;
          if (hipMemcpy2DAsync(c->noise, (size_t)c->L * W * sizeof(double), rp + (size_t)sw * c->L * W,
                               (size_t)n_sweeps * c->L * W * sizeof(double), (size_t)c->L * W * sizeof(double),
                               c->nch, hipMemcpyHostToDevice, c->s) != hipSuccess) {
            b->err = "replay upload failed";
            return CFQMC_EHIP;
          }
        }
        run_sweep(c, rp != nullptr);
      }
    Lmax = 0;   // nothing left for the interleaved loop below
  }
  // every group runs n_sweeps sweeps; slice steps interleaved as in cfqmc_batch_sweep
  const long long kmax = (long long)n_sweeps * Lmax;
  for (long long k = 0; k < kmax; ++k)
    for (int q = 0; q < G; ++q) {
      cfqmc_ctx* c = b->g[q];
      if (k >= (long long)n_sweeps * c->L) continue;
      const int t = (int)(k % c->L);
      const double* rp = replay ? replay[q] : nullptr;
      if (rp && t == 0) {
        const int W = 4 * c->nq + 1, sw = (int)(k / c->L);
        if (hipMemcpy2DAsync(c->noise, (size_t)c->L * W * sizeof(double), rp + (size_t)sw * c->L * W,
                             (size_t)n_sweeps * c->L * W * sizeof(double), (size_t)c->L * W * sizeof(double), c->nch,
                             hipMemcpyHostToDevice, c->s) != hipSuccess) {
          b->err = "replay upload failed";
          return CFQMC_EHIP;
        }
      }
      sweep_slice(c, t, rp ? c->noise : nullptr);
      if (t == c->L - 1) sweep_end(c);
    }
  int rc = CFQMC_OK, off = 0;
  for (int q = 0; q < G; ++q) {
    const int r = sweep_collect(b->g[q], stats ? stats + off : nullptr);
    if (r && !rc) rc = r;
    off += b->g[q]->nch;
  }
  return rc;
}

int cfqmc_batch_sweep(cfqmc_batch* b, int32_t n_sweeps, int32_t equal_time, cfqmc_stats* stats) {
  if (!b || n_sweeps < 0) return CFQMC_EINVAL;
  const int G = (int)b->g.size();
  int Lmax = 0;
  for (auto c : b->g) {
    if (!c->ready) { b->err = "fields not initialised"; return CFQMC_ESTATE; }
    Lmax = std::max(Lmax, c->L);
  }
  // sweeps per group: equal count, or scaled so every group runs for the same number of slice steps
  std::vector<long long> steps(G);
  long long kmax = 0;
  for (int k = 0; k < G; ++k) {
    const cfqmc_ctx* c = b->g[k];
    const long long ns = equal_time ? std::max(1LL, (long long)std::llround((double)n_sweeps * Lmax / c->L)) : n_sweeps;
    steps[k] = ns * c->L;
    kmax = std::max(kmax, steps[k]);
    sweep_reset_stats(b->g[k]);
  }
  bool graphs = true;
  for (auto c : b->g) graphs = graphs && graph_usable(c);
  if (graphs) {
    // one recorded sweep per group and sweep, each group on its own stream
    long long smax = 0;
    for (int q = 0; q < G; ++q) smax = std::max(smax, steps[q] / b->g[q]->L);
    for (long long sw = 0; sw < smax; ++sw)
      for (int q = 0; q < G; ++q)
        if (sw < steps[q] / b->g[q]->L) run_sweep(b->g[q], false);
    kmax = 0;
  }
  // interleave slice steps of all groups; each group's kernels go to its own stream
  for (long long k = 0; k < kmax; ++k)
    for (int q = 0; q < G; ++q) {
      if (k >= steps[q]) continue;
      cfqmc_ctx* c = b->g[q];
      const int t = (int)(k % c->L);
      sweep_slice(c, t, nullptr);
      if (t == c->L - 1) sweep_end(c);
    }
  int rc = CFQMC_OK, off = 0;
  for (int q = 0; q < G; ++q) {
    const int r = sweep_collect(b->g[q], stats ? stats + off : nullptr);
    if (r && !rc) rc = r;
    off += b->g[q]->nch;
  }
  return rc;
}

int cfqmc_measure_G(cfqmc_ctx* c, int32_t chain, int32_t tau, void* g_out, int32_t on_device) {
  if (!c || !g_out || chain < 0 || chain >= c->nch || tau < 0 || tau > c->L) return CFQMC_EINVAL;
  if (!c->ready) { c->err = "fields not initialised"; return CFQMC_ESTATE; }
  const long long nn = c->nn, NN = c->NN, sPQ = (long long)c->L * 8 * NN;
  const double2* src;
  if (tau == 0 || tau == c->L) {
    src = c->G;
  } else {
    const int b = tau / c->nstab;
    green_udt(c, b, b, c->Gs);
    const double2* cur = c->Gs;
    for (int t = b * c->nstab; t < tau; ++t)
      for (int ch = 3; ch >= 0; --ch) {
        const double2* pq = c->PQ + (long long)t * 8 * NN + ch * 2 * NN;
        chan(c, 1, ch, false, pq, sPQ, cur, c->S1, false, nullptr, 0);
        chan(c, 0, ch, true, pq, sPQ, c->S1, c->S2, false, nullptr, 0);
        launch_copy(c->S2, c->Gs, nn, nn, nn, c->nch, c->s);
        cur = c->Gs;
      }
    src = c->Gs;
  }
  if (on_device) {
    launch_expand4n(src + chain * nn, c->n, (double2*)g_out, c->s);
    HIPCHK(hipStreamSynchronize(c->s));
    return CFQMC_OK;
  }
  std::vector<double2> tmp(nn);
  HIPCHK(hipStreamSynchronize(c->s));
  HIPCHK(hipMemcpy(tmp.data(), src + chain * nn, nn * sizeof(double2), hipMemcpyDeviceToHost));
  double2* o = (double2*)g_out;
  const int n = c->n;
  for (int i = 0; i < 2 * n; ++i)
    for (int j = 0; j < 2 * n; ++j)
      o[(long long)i * 2 * n + j] = (i / n == j / n) ? tmp[(long long)(i % n) * n + (j % n)] : make_double2(0.0, 0.0);
  return CFQMC_OK;
}

int cfqmc_measure_tau(cfqmc_ctx* c, double* out, double* stab_rel) {
  if (!c || !out) return CFQMC_EINVAL;
  if (!c->ready) { c->err = "fields not initialised"; return CFQMC_ESTATE; }
  const long long cnt = (long long)c->nch * (c->L + 1) * 5;
  if (!c->corr) {
    int rc = dalloc(c, &c->corr, (size_t)cnt);
    rc |= dalloc(c, &c->tr0, (size_t)c->nch * 2);
    rc |= dalloc(c, &c->disp_err, (size_t)c->nch * 12);
    if (rc) { c->corr = nullptr; return CFQMC_ENOMEM; }
  }
  hipMemsetAsync(c->disp_err, 0, (size_t)c->nch * 12 * sizeof(double), c->s);
  displaced_pass(c, -1, c->corr, c->disp_err, nullptr, c->tr0);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->s));
  HIPCHK(hipMemcpy(out, c->corr, cnt * sizeof(double2), hipMemcpyDeviceToHost));
  if (stab_rel) {
    std::vector<double> e((size_t)c->nch * 12);
    HIPCHK(hipMemcpy(e.data(), c->disp_err, e.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int z = 0; z < c->nch; ++z)
      for (int k = 0; k < 3; ++k) stab_rel[3 * z + k] = e[12 * z + 4 * k + 1];
  }
  for (long long i = 0; i < 2 * cnt; ++i)
    if (!std::isfinite(out[i])) { c->err = "non-finite correlator"; return CFQMC_ENUMERIC; }
  return CFQMC_OK;
}

namespace {
// Device address of `scratch` on device dev, from hipGetSymbolAddress with that
// device current (each GPU holds its own copy of the array); resolved once per
// device and kept.
std::mutex g_scratch_mu;
void* g_scratch_addr[64] = {};

int scratch_address(cfqmc_ctx* c, void** out) {
  if (c->dev < 0 || c->dev >= 64) { c->err = "scratch: device index out of range"; return CFQMC_EINVAL; }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[c->dev]) {
    int cur = 0;
    HIPCHK(hipGetDevice(&cur));
    if (cur != c->dev) HIPCHK(hipSetDevice(c->dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != c->dev) HIPCHK(hipSetDevice(cur));
    if (e != hipSuccess || !p) {
      c->err = std::string("scratch: hipGetSymbolAddress failed: ") + hipGetErrorString(e);
      return CFQMC_EHIP;
    }
    g_scratch_addr[c->dev] = p;
  }
  *out = g_scratch_addr[c->dev];
  return CFQMC_OK;
}
}  // namespace

int cfqmc_measure_tau_noalloc(cfqmc_ctx* c, void* out_dev, void* stab_rel_dev) {
  if (!c || !out_dev) return CFQMC_EINVAL;
  if (!c->ready) { c->err = "fields not initialised"; return CFQMC_ESTATE; }
  if ((size_t)c->nch * kScratchPerChain > kScratchBytes) {
    c->err = "measure_tau_noalloc: " + std::to_string(c->nch) + " chains exceed the " +
             std::to_string(kScratchBytes / kScratchPerChain) + " chains its fixed scratch holds";
    return CFQMC_EINVAL;
  }
  void* base = nullptr;
  const int rc = scratch_address(c, &base);
  if (rc) return rc;
  double2* tr0 = (double2*)base;
  double* derr = (double*)(tr0 + 2 * c->nch);
  // the running maxima start at zero (a fill kernel: no memset node under capture)
  launch_fill(derr, 12LL * c->nch, 0.0, c->s);
  displaced_pass(c, -1, (double2*)out_dev, derr, nullptr, tr0);
  if (stab_rel_dev)
    HIPCHK(hipMemcpy2DAsync(stab_rel_dev, sizeof(double), derr + 1, 4 * sizeof(double), sizeof(double), 3 * c->nch,
                            hipMemcpyDeviceToDevice, c->s));
  HIPCHK(hipGetLastError());
  return CFQMC_OK;
}

int cfqmc_green_displaced(cfqmc_ctx* c, int32_t chain, int32_t tau, double* gt0, double* g0t, double* gtt) {
  if (!c || chain < 0 || chain >= c->nch || tau < 0 || tau > c->L) return CFQMC_EINVAL;
  if (!c->ready) { c->err = "fields not initialised"; return CFQMC_ESTATE; }
  double2* res[3];
  displaced_pass(c, tau, nullptr, nullptr, res, nullptr);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->s));
  double* outs[3] = {gt0, g0t, gtt};
  for (int k = 0; k < 3; ++k)
    if (outs[k])
      HIPCHK(hipMemcpy(outs[k], res[k] + chain * c->nn, c->nn * sizeof(double2), hipMemcpyDeviceToHost));
  return CFQMC_OK;
}

int cfqmc_sphere_weights(int32_t n_phi, double* out) {
  if (n_phi < 1 || n_phi > 288 || !out) return CFQMC_EINVAL;
  const std::vector<double> W = sphere_weights(n_phi);
  std::memcpy(out, W.data(), W.size() * sizeof(double));
  return CFQMC_OK;
}

int cfqmc_structure_factors(cfqmc_ctx* c, const int32_t* q_xy, int32_t n_q, double* out) {
  if (!c || !q_xy || !out || n_q <= 0 || n_q > 4096) return CFQMC_EINVAL;
  if (!c->ready) { c->err = "fields not initialised"; return CFQMC_ESTATE; }
  const bool sphere = !c->ht.comp_w.empty();
  const int N = c->N;
  std::vector<double> qw;
  if (sphere) {
    // rows' weights n_{l,m}[k, k + m] of the requested (l, m), 0 <= m <= l <= N - 1
    const std::vector<double> W = sphere_weights(N);
    qw.assign((size_t)n_q * N, 0.0);
    for (int i = 0; i < n_q; ++i) {
      const int l = q_xy[2 * i], m = q_xy[2 * i + 1];
      if (l < 0 || l >= N || m < 0 || m > l) { c->err = "sphere momenta need 0 <= m <= l <= N_phi - 1"; return CFQMC_EINVAL; }
      for (int r = 0; r < N; ++r) qw[(size_t)i * N + r] = W[((size_t)l * N + m) * N + r];
    }
  }
  int* dq = nullptr;
  double* dw = nullptr;
  double2* dout = nullptr;
  const long long cnt = (long long)c->nch * n_q * 5;
  int rc = CFQMC_OK;
  if (hipMalloc(&dq, 2 * n_q * sizeof(int)) != hipSuccess || hipMalloc(&dout, cnt * sizeof(double2)) != hipSuccess ||
      (sphere && hipMalloc(&dw, qw.size() * sizeof(double)) != hipSuccess))
    rc = CFQMC_ENOMEM;
  if (!rc && (hipMemcpyAsync(dq, q_xy, 2 * n_q * sizeof(int), hipMemcpyHostToDevice, c->s) != hipSuccess ||
              (sphere && hipMemcpyAsync(dw, qw.data(), qw.size() * sizeof(double), hipMemcpyHostToDevice, c->s) !=
                             hipSuccess)))
    rc = CFQMC_EHIP;
  if (!rc) {
    launch_structure_factors(c->G, c->nn, N, dq, n_q, dw, dout, c->nch, c->s);
    if (hipStreamSynchronize(c->s) != hipSuccess ||
        hipMemcpy(out, dout, cnt * sizeof(double2), hipMemcpyDeviceToHost) != hipSuccess)
      rc = CFQMC_EHIP;
  }
  hipFree(dq);
  hipFree(dw);
  hipFree(dout);
  return rc;
}

int cfqmc_logdet(cfqmc_ctx* c, int32_t chain, double* re, double* im) {
  if (!c || chain < 0 || chain >= c->nch) return CFQMC_EINVAL;
  if (!c->ready) { c->err = "fields not initialised"; return CFQMC_ESTATE; }
  std::vector<double> r, i;
  const int rc = lnw_all(c, r, i);
  if (rc) return rc;
  if (re) *re = r[chain];
  if (im) *im = i[chain];
  return CFQMC_OK;
}

int cfqmc_observables(cfqmc_ctx* c, int32_t chain, double* s_q0, double* m2) {
  if (!c || chain < 0 || chain >= c->nch) return CFQMC_EINVAL;
  if (!c->ready) { c->err = "fields not initialised"; return CFQMC_ESTATE; }
  launch_observables(c->G, c->nn, c->N, q0_weight(c), c->obs, 8, c->nch, c->s);
  std::vector<double> o(8);
  HIPCHK(hipStreamSynchronize(c->s));
  HIPCHK(hipMemcpy(o.data(), c->obs + chain * 8, 8 * sizeof(double), hipMemcpyDeviceToHost));
  if (s_q0) for (int i = 0; i < 5; ++i) s_q0[i] = o[i];
  if (m2) *m2 = o[5];
  return CFQMC_OK;
}

int cfqmc_series_of(cfqmc_ctx* c, int32_t chain, int32_t which, double* out, int32_t max_len, int32_t* len) {
  if (!c || chain < 0 || chain >= c->nch || !out || max_len < 0 || which < 0 || which > 2) return CFQMC_EINVAL;
  const double* src = which == 0 ? c->series : which == 1 ? c->series_s : c->series_p;
  const int k = std::min(max_len, c->series_len);
  HIPCHK(hipStreamSynchronize(c->s));
  if (k > 0) HIPCHK(hipMemcpy(out, src + (long long)chain * c->series_cap, k * sizeof(double), hipMemcpyDeviceToHost));
  if (len) *len = k;
  return CFQMC_OK;
}

int cfqmc_series(cfqmc_ctx* c, int32_t chain, double* out, int32_t max_len, int32_t* len) {
  return cfqmc_series_of(c, chain, 0, out, max_len, len);
}

int cfqmc_last_sweep(cfqmc_ctx* c, int32_t chain, int32_t* accepted, double* ln_a) {
  if (!c || chain < 0 || chain >= c->nch) return CFQMC_EINVAL;
  HIPCHK(hipStreamSynchronize(c->s));
  if (accepted) HIPCHK(hipMemcpy(accepted, c->hist_acc + (long long)chain * c->L, c->L * sizeof(int), hipMemcpyDeviceToHost));
  if (ln_a) HIPCHK(hipMemcpy(ln_a, c->hist_lnA + (long long)chain * c->L, c->L * sizeof(double), hipMemcpyDeviceToHost));
  return CFQMC_OK;
}

int cfqmc_get_eps(cfqmc_ctx* c, double* eps) {
  if (!c || !eps) return CFQMC_EINVAL;
  HIPCHK(hipStreamSynchronize(c->s));
  HIPCHK(hipMemcpy(eps, c->eps, c->nch * sizeof(double), hipMemcpyDeviceToHost));
  return CFQMC_OK;
}

int cfqmc_set_eps(cfqmc_ctx* c, const double* eps) {
  if (!c || !eps) return CFQMC_EINVAL;
  for (int z = 0; z < c->nch; ++z)
    if (!(eps[z] > 0)) return CFQMC_EINVAL;
  HIPCHK(hipMemcpyAsync(c->eps, eps, c->nch * sizeof(double), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  return CFQMC_OK;
}

int cfqmc_tile_config(const cfqmc_ctx* c, int32_t* chan_cfg, int32_t* gemm_cfg) {
  if (!c) return CFQMC_EINVAL;
  if (chan_cfg) *chan_cfg = c->cfg_chan;
  if (gemm_cfg) *gemm_cfg = c->cfg_gemm;
  return CFQMC_OK;
}

int cfqmc_launch_config(const cfqmc_ctx* c, int32_t* out) {
  if (!c || !out) return CFQMC_EINVAL;
  out[0] = c->cfg_chan;
  out[1] = c->cfg_chan64;
  out[2] = c->cfg_gemm;
  out[3] = c->cfg_small;
  out[4] = c->guard ? c->guard_launch : 0;
  return CFQMC_OK;
}

int cfqmc_kernel_timing(cfqmc_ctx* c, int32_t enable) {
  if (!c) return CFQMC_EINVAL;
  HIPCHK(hipStreamSynchronize(c->s));
  if (enable && c->ev.empty()) {
    c->ev.resize(2 * 4096);
    for (auto& e : c->ev) HIPCHK(hipEventCreate(&e));
    c->ev2.resize(2 * 4096);
    for (auto& e : c->ev2) HIPCHK(hipEventCreate(&e));
  }
  c->timing = enable != 0;
  c->ev_used = 0;
  c->ev2_used = 0;
  // record the timing variant of the sweep now (recording runs no kernel), so
  // that the first timed sweep does not pay for it
  if (c->timing && c->ready && graph_usable(c) && c->tstate[0] == 0) {
    record_timed_sweep(c, 0);
    if (c->launch_failed) {
      c->launch_failed = false;
      c->ready = false;
      return CFQMC_EHIP;
    }
  }
  return CFQMC_OK;
}

int cfqmc_kernel_timing_read(cfqmc_ctx* c, double* avg_ms, int64_t* count, double* flops_per_launch) {
  if (!c) return CFQMC_EINVAL;
  return timing_average(c, c->ev, c->ev_used, avg_ms, count, flops_per_launch);
}

int cfqmc_kernel_timing_read_woodbury(cfqmc_ctx* c, double* avg_ms, int64_t* count, double* flops_per_launch) {
  if (!c) return CFQMC_EINVAL;
  return timing_average(c, c->ev2, c->ev2_used, avg_ms, count, flops_per_launch);
}

}  // extern "C"

// ---------------------------------------------------------------- learned global proposal

struct cfqmc_slmc {
  cfqmc_ctx* c;
  cfqmc_slmc_params p;
  int L, nq, nw, nqb, nwb, F, Fp, H, NX, Bmax, nch;
  long long nf, P, oW1, ob1, oW2, ob2, ow3, ob3;
  std::vector<void*> allocs;
  int *shell, *wbin, *shell_off, *shell_comp, *w_off;
  float *inv_cnt, *twc, *tws;
  float *w, *g, *m, *v, *mu, *sig;
  uint16_t *W1b, *W2b, *w3b;
  int t_adam;
  double ybar, sy;
  bool norm_set;
  int cap, n_data;
  float* dx_raw;
  std::vector<double> hy;
  uint16_t* xall;
  float* yall;
  float *Xre, *Xim, *feat, *yb, *a1, *a2, *out, *dout, *dz2, *dA1, *dz1, *dX, *gf;
  uint16_t *xb, *a1b, *a2b, *dz2b, *dz1b;
  double* loss_acc;
  double *phi_cur, *phi_save, *mom, *grad, *prop, *sumsq, *rp;
  int* flag;
  long long move_counter;
  uint64_t rng;
  int sub;   // subspace of the global moves: 0 all fields, 1 q = 0 components, 2 slice-uniform q = 0 amplitudes
};

namespace {

template <typename T>
int salloc(cfqmc_slmc* s, T** p, size_t count) {
  void* q = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) {
    s->c->err = "device allocation failed";
    return CFQMC_ENOMEM;
  }
  hipMemsetAsync(q, 0, count * sizeof(T), s->c->s);
  s->allocs.push_back(q);
  *p = (T*)q;
  return CFQMC_OK;
}

uint64_t splitmix(uint64_t& st) {
  st += 0x9E3779B97F4A7C15ull;
  uint64_t z = st;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double host_uniform(uint64_t& st) { return ((splitmix(st) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
double host_normal(uint64_t& st) {
  const double u1 = host_uniform(st), u2 = host_uniform(st);
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
}

void slmc_refresh_bf16(cfqmc_slmc* s) {
  hipStream_t st = s->c->s;
  launch_slmc_to_bf16(s->w + s->oW1, s->H, s->F, s->W1b, s->Fp, st);
  launch_slmc_to_bf16(s->w + s->oW2, s->H, s->H, s->W2b, s->H, st);
  launch_slmc_to_bf16(s->w + s->ow3, 1, s->H, s->w3b, s->H, st);
}

// Raw features of nb configurations (device fields, stride sphi) into s->feat.
void slmc_features_dev(cfqmc_slmc* s, const double* phi, long long sphi, int nb) {
  hipStream_t st = s->c->s;
  const long long sX = 4LL * s->nq * s->nw;
  launch_slmc_dft(phi, sphi, s->L, s->nq, s->nw, s->twc, s->tws, s->Xre, s->Xim, sX, nb, st);
  launch_slmc_bin(s->Xre, s->Xim, sX, s->nq, s->nw, s->L, s->nqb, s->nwb, s->shell_off, s->shell_comp, s->w_off,
                  s->feat, s->F, nb, st);
}

void slmc_forward(cfqmc_slmc* s, const uint16_t* xb, int nb) {
  hipStream_t st = s->c->s;
  const int H = s->H;
  launch_slmc_gemm(0, 0, nb, H, s->Fp, xb, s->Fp, s->W1b, s->Fp, s->a1, H, s->w + s->ob1, 1, s->a1b, H, st);
  launch_slmc_gemm(0, 0, nb, H, H, s->a1b, H, s->W2b, H, s->a2, H, s->w + s->ob2, 1, s->a2b, H, st);
  launch_slmc_head(s->a2b, H, s->w3b, s->w + s->ob3, s->out, nb, st);
}

// Back-propagation of sum_b dout[b] out[b]: parameter gradients into s->g
// (weights) and/or the gradient w.r.t. the standardised inputs into s->dX.
void slmc_backward(cfqmc_slmc* s, const uint16_t* xb, int nb, bool weights, bool input) {
  hipStream_t st = s->c->s;
  const int H = s->H, F = s->F, Fp = s->Fp;
  launch_slmc_dz2(s->dout, s->w3b, s->a2, H, s->dz2, s->dz2b, nb, st);
  if (weights) {
    launch_slmc_head_grad(s->dout, s->a2b, nb, H, s->g + s->ow3, s->g + s->ob3, st);
    launch_slmc_colsum(s->dz2, nb, H, s->g + s->ob2, st);
    launch_slmc_gemm(1, 1, H, H, nb, s->dz2b, H, s->a1b, H, s->g + s->oW2, H, nullptr, 0, nullptr, 0, st);
  }
  launch_slmc_gemm(0, 1, nb, H, H, s->dz2b, H, s->W2b, H, s->dA1, H, nullptr, 0, nullptr, 0, st);
  launch_slmc_tanh_bwd(s->dA1, s->a1, (long long)nb * H, s->dz1, s->dz1b, st);
  if (weights) {
    launch_slmc_colsum(s->dz1, nb, H, s->g + s->ob1, st);
    launch_slmc_gemm(1, 1, H, F, nb, s->dz1b, H, xb, Fp, s->g + s->oW1, F, nullptr, 0, nullptr, 0, st);
  }
  if (input) launch_slmc_gemm(0, 1, nb, F, H, s->dz1b, H, s->W1b, Fp, s->dX, Fp, nullptr, 0, nullptr, 0, st);
}

// S_NN and optionally dS_NN/dphi (into s->grad, stride nf) of nb <= NX device
// configurations. snn: host [nb].
int slmc_action_dev(cfqmc_slmc* s, const double* phi, int nb, std::vector<double>& snn, bool want_grad) {
  cfqmc_ctx* c = s->c;
  hipStream_t st = c->s;
  slmc_features_dev(s, phi, s->nf, nb);
  launch_slmc_standardize(s->feat, s->F, s->Fp, s->mu, s->sig, s->xb, nb, st);
  slmc_forward(s, s->xb, nb);
  if (want_grad) {
    launch_slmc_dout(s->out, nullptr, nb, 1, (float)s->sy, s->dout, nullptr, st);
    slmc_backward(s, s->xb, nb, false, true);
    launch_slmc_dx_to_gf(s->dX, s->Fp, s->sig, s->F, 1.f, s->gf, nb, st);
    launch_slmc_vjp(s->Xre, s->Xim, 4LL * s->nq * s->nw, s->gf, s->F, s->nq, s->nw, s->L, s->nqb, s->nwb, s->shell,
                    s->wbin, s->inv_cnt, s->twc, s->tws, s->grad, s->nf, nb, st);
  }
  std::vector<float> o(nb);
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipMemcpy(o.data(), s->out, nb * sizeof(float), hipMemcpyDeviceToHost));
  snn.resize(nb);
  for (int b = 0; b < nb; ++b) snn[b] = s->sy * (double)o[b] + s->ybar;
  return CFQMC_OK;
}

}  // namespace

extern "C" {

void cfqmc_slmc_default_params(cfqmc_slmc_params* p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->hidden = 256;
  p->n_qbins = 16;
  p->n_wbins = 16;
  p->capacity = 10000;
  p->max_batch = 256;
  p->seed = 1;
}

int cfqmc_slmc_destroy(cfqmc_slmc* s) {
  if (!s) return CFQMC_EINVAL;
  hipStreamSynchronize(s->c->s);
  for (void* q : s->allocs) hipFree(q);
  delete s;
  return CFQMC_OK;
}

int cfqmc_slmc_create(cfqmc_ctx* c, const cfqmc_slmc_params* pp, cfqmc_slmc** out) {
  if (!c || !pp || !out) return CFQMC_EINVAL;
  *out = nullptr;
  const cfqmc_slmc_params p = *pp;
  if (p.hidden < 16 || p.hidden > 4096 || p.n_qbins < 1 || p.n_wbins < 1 || p.capacity < 1 || p.max_batch < 1 ||
      p.max_batch > 65536) {
    c->err = "invalid SLMC parameters";
    return CFQMC_EINVAL;
  }
  if (c->L > 2000) { c->err = "SLMC features support L_tau <= 2000"; return CFQMC_EINVAL; }
  cfqmc_slmc* s = new cfqmc_slmc();
  s->c = c;
  s->p = p;
  s->L = c->L; s->nq = c->nq; s->nw = c->L / 2 + 1;
  s->nqb = p.n_qbins; s->nwb = std::min(p.n_wbins, s->nw);
  s->F = 4 * s->nqb * s->nwb + 4;
  s->Fp = (s->F + 31) / 32 * 32;
  s->H = p.hidden;
  s->nch = c->nch;
  s->NX = std::max(c->nch, 4);
  s->Bmax = std::max(s->NX, p.max_batch);
  s->nf = (long long)c->L * 4 * c->nq;
  const long long F = s->F, H = s->H;
  s->oW1 = 0; s->ob1 = H * F; s->oW2 = s->ob1 + H; s->ob2 = s->oW2 + H * H; s->ow3 = s->ob2 + H; s->ob3 = s->ow3 + H;
  s->P = s->ob3 + 1;
  s->cap = p.capacity;
  s->rng = p.seed * 0xD1B54A32D192ED03ull + 0x8CB92BA72F3D8DD7ull;
  // tables: shells by |q|^2, frequency bins, member lists
  const HostTables& T = c->ht;
  std::vector<int> sh(s->nq), wb(s->nw);
  long long r2max = 0;
  for (int q = 0; q < s->nq; ++q) r2max = std::max(r2max, T.comp_r2[q]);
  for (int q = 0; q < s->nq; ++q) {
    const long long r2 = T.comp_r2[q];
    sh[q] = (int)((s->nqb * r2) / (r2max + 1));
  }
  for (int w = 0; w < s->nw; ++w) wb[w] = (int)(((long long)s->nwb * w) / s->nw);
  std::vector<int> soff(s->nqb + 1, 0), scomp, woff(s->nwb + 1, 0);
  for (int b = 0; b < s->nqb; ++b) {
    for (int q = 0; q < s->nq; ++q)
      if (sh[q] == b) scomp.push_back(q);
    soff[b + 1] = (int)scomp.size();
  }
  for (int w = 0; w < s->nw; ++w) woff[wb[w] + 1] = w + 1;
  for (int b = 1; b <= s->nwb; ++b) woff[b] = std::max(woff[b], woff[b - 1]);
  std::vector<float> icnt(s->nqb * s->nwb), twc(s->L), tws(s->L);
  for (int a = 0; a < s->nqb; ++a)
    for (int b = 0; b < s->nwb; ++b) {
      const long long cnt = (long long)(soff[a + 1] - soff[a]) * (woff[b + 1] - woff[b]);
      icnt[a * s->nwb + b] = cnt > 0 ? (float)(1.0 / (double)cnt) : 0.f;
    }
  for (int k = 0; k < s->L; ++k) {
    twc[k] = (float)std::cos(2.0 * M_PI * k / s->L);
    tws[k] = (float)std::sin(2.0 * M_PI * k / s->L);
  }
  // initial parameters: N(0, 1/fan_in) weights, zero biases
  std::vector<float> w0(s->P, 0.f);
  for (long long e = 0; e < H * F; ++e) w0[s->oW1 + e] = (float)(host_normal(s->rng) / std::sqrt((double)F));
  for (long long e = 0; e < H * H; ++e) w0[s->oW2 + e] = (float)(host_normal(s->rng) / std::sqrt((double)H));
  for (long long e = 0; e < H; ++e) w0[s->ow3 + e] = (float)(host_normal(s->rng) / std::sqrt((double)H));
  std::vector<float> ones(F, 1.f);
  int r = 0;
  const long long NX = s->NX, Bm = s->Bmax, nf = s->nf;
  r |= salloc(s, &s->shell, s->nq); r |= salloc(s, &s->wbin, s->nw); r |= salloc(s, &s->shell_off, s->nqb + 1);
  r |= salloc(s, &s->shell_comp, s->nq); r |= salloc(s, &s->w_off, s->nwb + 1);
  r |= salloc(s, &s->inv_cnt, s->nqb * s->nwb); r |= salloc(s, &s->twc, s->L); r |= salloc(s, &s->tws, s->L);
  r |= salloc(s, &s->w, s->P); r |= salloc(s, &s->g, s->P); r |= salloc(s, &s->m, s->P); r |= salloc(s, &s->v, s->P);
  r |= salloc(s, &s->mu, F); r |= salloc(s, &s->sig, F);
  r |= salloc(s, &s->W1b, H * s->Fp); r |= salloc(s, &s->W2b, H * H); r |= salloc(s, &s->w3b, H);
  r |= salloc(s, &s->dx_raw, (long long)s->cap * F); r |= salloc(s, &s->xall, (long long)s->cap * s->Fp);
  r |= salloc(s, &s->yall, s->cap);
  r |= salloc(s, &s->Xre, NX * 4 * s->nq * s->nw); r |= salloc(s, &s->Xim, NX * 4 * s->nq * s->nw);
  r |= salloc(s, &s->feat, Bm * F); r |= salloc(s, &s->xb, Bm * s->Fp); r |= salloc(s, &s->yb, Bm);
  r |= salloc(s, &s->a1, Bm * H); r |= salloc(s, &s->a2, Bm * H); r |= salloc(s, &s->out, Bm);
  r |= salloc(s, &s->dout, Bm); r |= salloc(s, &s->dz2, Bm * H); r |= salloc(s, &s->dA1, Bm * H);
  r |= salloc(s, &s->dz1, Bm * H); r |= salloc(s, &s->dX, Bm * s->Fp); r |= salloc(s, &s->gf, Bm * F);
  r |= salloc(s, &s->a1b, Bm * H); r |= salloc(s, &s->a2b, Bm * H); r |= salloc(s, &s->dz2b, Bm * H);
  r |= salloc(s, &s->dz1b, Bm * H); r |= salloc(s, &s->loss_acc, 4096);
  r |= salloc(s, &s->phi_cur, NX * nf); r |= salloc(s, &s->phi_save, NX * nf); r |= salloc(s, &s->mom, NX * nf);
  r |= salloc(s, &s->grad, NX * nf); r |= salloc(s, &s->prop, NX * nf); r |= salloc(s, &s->rp, NX * nf);
  r |= salloc(s, &s->sumsq, NX); r |= salloc(s, &s->flag, NX);
  if (r) { cfqmc_slmc_destroy(s); return CFQMC_ENOMEM; }
  hipStream_t st = c->s;
  bool ok = true;
  ok &= hipMemcpyAsync(s->shell, sh.data(), sh.size() * 4, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(s->wbin, wb.data(), wb.size() * 4, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(s->shell_off, soff.data(), soff.size() * 4, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(s->shell_comp, scomp.data(), scomp.size() * 4, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(s->w_off, woff.data(), woff.size() * 4, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(s->inv_cnt, icnt.data(), icnt.size() * 4, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(s->twc, twc.data(), twc.size() * 4, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(s->tws, tws.data(), tws.size() * 4, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(s->w, w0.data(), w0.size() * 4, hipMemcpyHostToDevice, st) == hipSuccess;
  ok &= hipMemcpyAsync(s->sig, ones.data(), ones.size() * 4, hipMemcpyHostToDevice, st) == hipSuccess;
  s->ybar = 0.0;
  s->sy = 1.0;
  slmc_refresh_bf16(s);
  ok &= hipStreamSynchronize(st) == hipSuccess;
  if (!ok || hipGetLastError() != hipSuccess) { c->err = "SLMC set-up failed"; cfqmc_slmc_destroy(s); return CFQMC_EHIP; }
  *out = s;
  return CFQMC_OK;
}

int cfqmc_slmc_sizes(const cfqmc_slmc* s, int32_t* n_feat, int64_t* n_params, int32_t* n_data) {
  if (!s) return CFQMC_EINVAL;
  if (n_feat) *n_feat = s->F;
  if (n_params) *n_params = s->P;
  if (n_data) *n_data = s->n_data;
  return CFQMC_OK;
}

int cfqmc_slmc_set_params(cfqmc_slmc* s, const float* w) {
  if (!s || !w) return CFQMC_EINVAL;
  cfqmc_ctx* c = s->c;
  for (long long e = 0; e < s->P; ++e)
    if (!std::isfinite(w[e])) { c->err = "non-finite parameter"; return CFQMC_EINVAL; }
  HIPCHK(hipMemcpyAsync(s->w, w, s->P * sizeof(float), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipMemsetAsync(s->m, 0, s->P * sizeof(float), c->s));
  HIPCHK(hipMemsetAsync(s->v, 0, s->P * sizeof(float), c->s));
  s->t_adam = 0;
  slmc_refresh_bf16(s);
  HIPCHK(hipStreamSynchronize(c->s));
  return CFQMC_OK;
}

int cfqmc_slmc_get_params(cfqmc_slmc* s, float* w) {
  if (!s || !w) return CFQMC_EINVAL;
  cfqmc_ctx* c = s->c;
  HIPCHK(hipStreamSynchronize(c->s));
  HIPCHK(hipMemcpy(w, s->w, s->P * sizeof(float), hipMemcpyDeviceToHost));
  return CFQMC_OK;
}

int cfqmc_slmc_set_norm(cfqmc_slmc* s, const float* mu, const float* sigma, double y_bar, double s_y) {
  if (!s || !mu || !sigma || !(s_y > 0)) return CFQMC_EINVAL;
  cfqmc_ctx* c = s->c;
  for (int j = 0; j < s->F; ++j)
    if (!(sigma[j] > 0) || !std::isfinite(mu[j])) { c->err = "invalid standardisation"; return CFQMC_EINVAL; }
  HIPCHK(hipMemcpyAsync(s->mu, mu, s->F * sizeof(float), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipMemcpyAsync(s->sig, sigma, s->F * sizeof(float), hipMemcpyHostToDevice, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  s->ybar = y_bar;
  s->sy = s_y;
  s->norm_set = true;
  return CFQMC_OK;
}

int cfqmc_slmc_get_norm(cfqmc_slmc* s, float* mu, float* sigma, double* y_bar, double* s_y) {
  if (!s) return CFQMC_EINVAL;
  cfqmc_ctx* c = s->c;
  HIPCHK(hipStreamSynchronize(c->s));
  if (mu) HIPCHK(hipMemcpy(mu, s->mu, s->F * sizeof(float), hipMemcpyDeviceToHost));
  if (sigma) HIPCHK(hipMemcpy(sigma, s->sig, s->F * sizeof(float), hipMemcpyDeviceToHost));
  if (y_bar) *y_bar = s->ybar;
  if (s_y) *s_y = s->sy;
  return CFQMC_OK;
}

int cfqmc_slmc_features(cfqmc_slmc* s, const double* phi, int32_t n, float* feat) {
  if (!s || !phi || !feat || n < 0) return CFQMC_EINVAL;
  cfqmc_ctx* c = s->c;
  for (int b0 = 0; b0 < n; b0 += s->NX) {
    const int nb = std::min(s->NX, n - b0);
    HIPCHK(hipMemcpyAsync(s->prop, phi + (long long)b0 * s->nf, nb * s->nf * sizeof(double), hipMemcpyHostToDevice,
                          c->s));
    slmc_features_dev(s, s->prop, s->nf, nb);
    HIPCHK(hipStreamSynchronize(c->s));
    HIPCHK(hipMemcpy(feat + (long long)b0 * s->F, s->feat, (long long)nb * s->F * sizeof(float),
                     hipMemcpyDeviceToHost));
  }
  return CFQMC_OK;
}

int cfqmc_slmc_action(cfqmc_slmc* s, const double* phi, int32_t n, double* s_nn, double* grad_phi) {
  if (!s || !phi || !s_nn || n < 0) return CFQMC_EINVAL;
  cfqmc_ctx* c = s->c;
  std::vector<double> v;
  for (int b0 = 0; b0 < n; b0 += s->NX) {
    const int nb = std::min(s->NX, n - b0);
    HIPCHK(hipMemcpyAsync(s->prop, phi + (long long)b0 * s->nf, nb * s->nf * sizeof(double), hipMemcpyHostToDevice,
                          c->s));
    const int rc = slmc_action_dev(s, s->prop, nb, v, grad_phi != nullptr);
    if (rc) return rc;
    for (int b = 0; b < nb; ++b) s_nn[b0 + b] = v[b];
    if (grad_phi)
      HIPCHK(hipMemcpy(grad_phi + (long long)b0 * s->nf, s->grad, nb * s->nf * sizeof(double), hipMemcpyDeviceToHost));
  }
  return CFQMC_OK;
}

int cfqmc_slmc_grad_check(cfqmc_slmc* s, const double* phi, int32_t n, double* fwd_out, double* grad_out) {
  if (!s || !phi || !fwd_out || !grad_out || n < 1) return CFQMC_EINVAL;
  return cfqmc_slmc_action(s, phi, n, fwd_out, grad_out);
}

int cfqmc_slmc_loss_grad(cfqmc_slmc* s, const float* x, const double* y, int32_t n, double* loss, float* grad,
                         float* out) {
  if (!s || !x || !y || n < 1 || n > s->Bmax) return CFQMC_EINVAL;
  cfqmc_ctx* c = s->c;
  hipStream_t st = c->s;
  // standardised inputs as given (mu = 0, sigma = 1 path), rounded to BF16 by the kernel
  std::vector<float> zero(s->F, 0.f), one(s->F, 1.f), yf(n);
  for (int b = 0; b < n; ++b) yf[b] = (float)y[b];
  float *mu0 = nullptr, *sg1 = nullptr;
  // feat buffer holds x; temporary unit standardisation in gf scratch
  HIPCHK(hipMemcpyAsync(s->feat, x, (long long)n * s->F * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(s->yb, yf.data(), n * sizeof(float), hipMemcpyHostToDevice, st));
  mu0 = s->gf;
  sg1 = s->gf + s->F;
  HIPCHK(hipMemcpyAsync(mu0, zero.data(), s->F * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(sg1, one.data(), s->F * sizeof(float), hipMemcpyHostToDevice, st));
  launch_slmc_standardize(s->feat, s->F, s->Fp, mu0, sg1, s->xb, n, st);
  HIPCHK(hipMemsetAsync(s->loss_acc, 0, sizeof(double), st));
  slmc_forward(s, s->xb, n);
  launch_slmc_dout(s->out, s->yb, n, 0, 0.f, s->dout, s->loss_acc, st);
  slmc_backward(s, s->xb, n, true, false);
  HIPCHK(hipStreamSynchronize(st));
  if (loss) HIPCHK(hipMemcpy(loss, s->loss_acc, sizeof(double), hipMemcpyDeviceToHost));
  if (grad) HIPCHK(hipMemcpy(grad, s->g, s->P * sizeof(float), hipMemcpyDeviceToHost));
  if (out) HIPCHK(hipMemcpy(out, s->out, n * sizeof(float), hipMemcpyDeviceToHost));
  return CFQMC_OK;
}

int cfqmc_slmc_collect(cfqmc_slmc* s) {
  if (!s) return CFQMC_EINVAL;
  cfqmc_ctx* c = s->c;
  if (!c->ready) { c->err = "fields not initialised"; return CFQMC_ESTATE; }
  if (s->n_data + s->nch > s->cap) { c->err = "SLMC data set full"; return CFQMC_ESTATE; }
  std::vector<double> re, im;
  const int rc = lnw_all(c, re, im);
  if (rc) return rc;
  slmc_features_dev(s, c->phi, s->nf, s->nch);
  HIPCHK(hipMemcpyAsync(s->dx_raw + (long long)s->n_data * s->F, s->feat, (long long)s->nch * s->F * sizeof(float),
                        hipMemcpyDeviceToDevice, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  for (int z = 0; z < s->nch; ++z) s->hy.push_back(-re[z]);
  s->n_data += s->nch;
  return CFQMC_OK;
}

int cfqmc_slmc_clear_data(cfqmc_slmc* s) {
  if (!s) return CFQMC_EINVAL;
  s->n_data = 0;
  s->hy.clear();
  return CFQMC_OK;
}

int cfqmc_slmc_train(cfqmc_slmc* s, int32_t epochs, int32_t batch, double lr, int32_t refit_norm, double* loss_out) {
  if (!s || epochs < 1 || epochs > 4096 || batch < 1 || batch > s->Bmax || !(lr > 0)) return CFQMC_EINVAL;
  cfqmc_ctx* c = s->c;
  hipStream_t st = c->s;
  const int n = s->n_data, F = s->F;
  if (n < 2) { c->err = "SLMC data set needs at least two configurations"; return CFQMC_ESTATE; }
  if (!s->norm_set || refit_norm) {
    std::vector<float> fx((long long)n * F);
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(fx.data(), s->dx_raw, fx.size() * sizeof(float), hipMemcpyDeviceToHost));
    std::vector<float> mu(F), sg(F);
    for (int j = 0; j < F; ++j) {
      double a = 0.0, q = 0.0;
      for (int b = 0; b < n; ++b) a += fx[(long long)b * F + j];
      a /= n;
      for (int b = 0; b < n; ++b) {
        const double d = fx[(long long)b * F + j] - a;
        q += d * d;
      }
      const double sd = std::sqrt(q / n);
      mu[j] = (float)a;
      sg[j] = sd > 1e-12 ? (float)sd : 1.f;
    }
    double a = 0.0, q = 0.0;
    for (double v : s->hy) a += v;
    a /= n;
    for (double v : s->hy) q += (v - a) * (v - a);
    const double sy = std::sqrt(q / n);
    const int rc = cfqmc_slmc_set_norm(s, mu.data(), sg.data(), a, sy > 1e-12 ? sy : 1.0);
    if (rc) return rc;
  }
  std::vector<float> ys(n);
  for (int b = 0; b < n; ++b) ys[b] = (float)((s->hy[b] - s->ybar) / s->sy);
  HIPCHK(hipMemcpyAsync(s->yall, ys.data(), n * sizeof(float), hipMemcpyHostToDevice, st));
  launch_slmc_standardize(s->dx_raw, F, s->Fp, s->mu, s->sig, s->xall, n, st);
  // minibatch order of every epoch (Fisher-Yates on the SLMC generator)
  std::vector<int> order((long long)epochs * n);
  for (int e = 0; e < epochs; ++e) {
    int* o = order.data() + (long long)e * n;
    for (int b = 0; b < n; ++b) o[b] = b;
    for (int b = n - 1; b > 0; --b) std::swap(o[b], o[splitmix(s->rng) % (uint64_t)(b + 1)]);
  }
  int* idx = nullptr;
  if (hipMalloc(&idx, order.size() * sizeof(int)) != hipSuccess) { c->err = "device allocation failed"; return CFQMC_ENOMEM; }
  hipError_t e0 = hipMemcpyAsync(idx, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice, st);
  const int nbatches = (n + batch - 1) / batch;
  const int nl = std::min(epochs, 4096);
  hipMemsetAsync(s->loss_acc, 0, nl * sizeof(double), st);
  for (int e = 0; e < epochs && e0 == hipSuccess; ++e)
    for (int b0 = 0; b0 < n; b0 += batch) {
      const int nb = std::min(batch, n - b0);
      launch_slmc_gather(s->xall, s->yall, s->Fp, idx + (long long)e * n + b0, nb, s->xb, s->yb, st);
      slmc_forward(s, s->xb, nb);
      launch_slmc_dout(s->out, s->yb, nb, 0, 0.f, s->dout, s->loss_acc + e, st);
      slmc_backward(s, s->xb, nb, true, false);
      launch_slmc_adam(s->w, s->g, s->m, s->v, s->P, lr, ++s->t_adam, st);
      slmc_refresh_bf16(s);
    }
  std::vector<double> la(nl);
  const hipError_t e1 = hipStreamSynchronize(st);
  hipFree(idx);
  HIPCHK(e0);
  HIPCHK(e1);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpy(la.data(), s->loss_acc, nl * sizeof(double), hipMemcpyDeviceToHost));
  if (loss_out) *loss_out = la[nl - 1] / nbatches;
  if (!std::isfinite(la[nl - 1])) { c->err = "training diverged"; return CFQMC_ENUMERIC; }
  return CFQMC_OK;
}

int cfqmc_slmc_train_heldout(cfqmc_slmc* s, int32_t max_epochs, int32_t batch, double lr, int32_t refit_norm,
                             int32_t n_val, int32_t patience, double* train_loss, double* val_loss,
                             int32_t* best_epoch) {
  if (!s || max_epochs < 1 || max_epochs > 4096 || batch < 1 || batch > s->Bmax || !(lr > 0) || n_val < 1 ||
      patience < 1)
    return CFQMC_EINVAL;
  cfqmc_ctx* c = s->c;
  hipStream_t st = c->s;
  const int n = s->n_data, F = s->F, nt = n - n_val;
  if (nt < 2) { c->err = "SLMC held-out training needs at least two training configurations"; return CFQMC_ESTATE; }
  if (!s->norm_set || refit_norm) {
    // standardisation from the training configurations only
    std::vector<float> fx((long long)nt * F);
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(fx.data(), s->dx_raw, fx.size() * sizeof(float), hipMemcpyDeviceToHost));
    std::vector<float> mu(F), sg(F);
    for (int j = 0; j < F; ++j) {
      double a = 0.0, q = 0.0;
      for (int b = 0; b < nt; ++b) a += fx[(long long)b * F + j];
      a /= nt;
      for (int b = 0; b < nt; ++b) {
        const double d = fx[(long long)b * F + j] - a;
        q += d * d;
      }
      const double sd = std::sqrt(q / nt);
      mu[j] = (float)a;
      sg[j] = sd > 1e-12 ? (float)sd : 1.f;
    }
    double a = 0.0, q = 0.0;
    for (int b = 0; b < nt; ++b) a += s->hy[b];
    a /= nt;
    for (int b = 0; b < nt; ++b) q += (s->hy[b] - a) * (s->hy[b] - a);
    const double sy = std::sqrt(q / nt);
    const int rc = cfqmc_slmc_set_norm(s, mu.data(), sg.data(), a, sy > 1e-12 ? sy : 1.0);
    if (rc) return rc;
  }
  std::vector<float> ys(n);
  for (int b = 0; b < n; ++b) ys[b] = (float)((s->hy[b] - s->ybar) / s->sy);
  HIPCHK(hipMemcpyAsync(s->yall, ys.data(), n * sizeof(float), hipMemcpyHostToDevice, st));
  launch_slmc_standardize(s->dx_raw, F, s->Fp, s->mu, s->sig, s->xall, n, st);
  int* idx = nullptr;
  float* wbest = nullptr;
  if (hipMalloc(&idx, (size_t)n * sizeof(int)) != hipSuccess ||
      hipMalloc(&wbest, (size_t)s->P * sizeof(float)) != hipSuccess) {
    hipFree(idx);
    c->err = "device allocation failed";
    return CFQMC_ENOMEM;
  }
  // validation rows (the last n_val stored) after the training rows of each epoch's order
  std::vector<int> order(n);
  for (int b = 0; b < n; ++b) order[b] = b;
  std::vector<float> vout(n_val);
  double best = INFINITY, last_train = 0.0;
  int best_e = -1, since = 0, rc = CFQMC_OK;
  const int nbatches = (nt + batch - 1) / batch;
  for (int e = 0; e < max_epochs && !rc; ++e) {
    for (int b = nt - 1; b > 0; --b) std::swap(order[b], order[splitmix(s->rng) % (uint64_t)(b + 1)]);
    if (hipMemcpyAsync(idx, order.data(), n * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess) {
      rc = CFQMC_EHIP;
      break;
    }
    hipMemsetAsync(s->loss_acc, 0, sizeof(double), st);
    for (int b0 = 0; b0 < nt; b0 += batch) {
      const int nb = std::min(batch, nt - b0);
      launch_slmc_gather(s->xall, s->yall, s->Fp, idx + b0, nb, s->xb, s->yb, st);
      slmc_forward(s, s->xb, nb);
      launch_slmc_dout(s->out, s->yb, nb, 0, 0.f, s->dout, s->loss_acc, st);
      slmc_backward(s, s->xb, nb, true, false);
      launch_slmc_adam(s->w, s->g, s->m, s->v, s->P, lr, ++s->t_adam, st);
      slmc_refresh_bf16(s);
    }
    // validation loss: forward only, on the held-out rows
    double vl = 0.0;
    for (int v0 = 0; v0 < n_val && !rc; v0 += s->Bmax) {
      const int nb = std::min(s->Bmax, n_val - v0);
      launch_slmc_gather(s->xall, s->yall, s->Fp, idx + nt + v0, nb, s->xb, s->yb, st);
      slmc_forward(s, s->xb, nb);
      if (hipStreamSynchronize(st) != hipSuccess ||
          hipMemcpy(vout.data(), s->out, nb * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess) {
        rc = CFQMC_EHIP;
        break;
      }
      for (int b = 0; b < nb; ++b) {
        const double r = (double)vout[b] - ys[nt + v0 + b];
        vl += r * r;
      }
    }
    if (rc) break;
    vl /= n_val;
    double tl = 0.0;
    if (hipMemcpy(&tl, s->loss_acc, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) { rc = CFQMC_EHIP; break; }
    last_train = tl / nbatches;
    if (!std::isfinite(vl) || !std::isfinite(last_train)) { c->err = "training diverged"; rc = CFQMC_ENUMERIC; break; }
    if (vl < best) {
      best = vl;
      best_e = e;
      since = 0;
      if (hipMemcpyAsync(wbest, s->w, (size_t)s->P * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
        rc = CFQMC_EHIP;
    } else if (++since >= patience) {
      break;
    }
  }
  if (!rc && best_e >= 0) {
    // keep the parameters of the best validation epoch
    if (hipMemcpyAsync(s->w, wbest, (size_t)s->P * sizeof(float), hipMemcpyDeviceToDevice, st) != hipSuccess)
      rc = CFQMC_EHIP;
    else
      slmc_refresh_bf16(s);
  }
  const hipError_t e1 = hipStreamSynchronize(st);
  hipFree(idx);
  hipFree(wbest);
  if (rc) return rc;
  HIPCHK(e1);
  HIPCHK(hipGetLastError());
  if (train_loss) *train_loss = last_train;
  if (val_loss) *val_loss = best;
  if (best_epoch) *best_epoch = best_e;
  return CFQMC_OK;
}

int cfqmc_slmc_set_subspace(cfqmc_slmc* s, int32_t mode) {
  if (!s || mode < 0 || mode > 2) return CFQMC_EINVAL;
  s->sub = mode;
  return CFQMC_OK;
}

int cfqmc_slmc_global_move(cfqmc_slmc* s, int32_t n_traj, int32_t n_leap, double step, const double* replay,
                           cfqmc_slmc_move* out) {
  if (!s || n_traj < 1 || n_traj > 1024 || n_leap < 1 || n_leap > 100000 || !(step > 0)) return CFQMC_EINVAL;
  cfqmc_ctx* c = s->c;
  hipStream_t st = c->s;
  if (!c->ready) { c->err = "fields not initialised"; return CFQMC_ESTATE; }
  const int B = s->nch;
  const long long nf = s->nf, rs = (long long)n_traj * nf + n_traj + 1;
  std::vector<double> lw0, li, lw1, snn0, snn_cur, snn_new, q0(B), p0(B), q1(B), p1(B);
  int rc = lnw_all(c, lw0, li);
  if (rc) return rc;
  rc = slmc_action_dev(s, c->phi, B, snn0, false);
  if (rc) return rc;
  snn_cur = snn0;
  HIPCHK(hipMemcpyAsync(s->phi_cur, c->phi, B * nf * sizeof(double), hipMemcpyDeviceToDevice, st));
  std::vector<int> inner(B, 0), flag(B, 0);
  std::vector<double> maxdh(B, 0.0);
  const uint64_t key = c->p.seed ^ 0x5851F42D4C957F2Dull;
  for (int k = 0; k < n_traj; ++k) {
    if (replay) {
      HIPCHK(hipMemcpy2DAsync(s->rp, nf * sizeof(double), replay + (long long)k * nf, rs * sizeof(double),
                              nf * sizeof(double), B, hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));
    }
    launch_slmc_momenta(s->mom, nf, B, key, s->move_counter * 1024 + k, replay ? s->rp : nullptr, nf, s->sub, s->nq,
                        st);
    launch_slmc_sumsq(s->phi_cur, nf, s->sumsq, B, st);
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(q0.data(), s->sumsq, B * sizeof(double), hipMemcpyDeviceToHost));
    launch_slmc_sumsq(s->mom, nf, s->sumsq, B, st);
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(p0.data(), s->sumsq, B * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpyAsync(s->prop, s->phi_cur, B * nf * sizeof(double), hipMemcpyDeviceToDevice, st));
    rc = slmc_action_dev(s, s->prop, B, snn_new, true);
    if (rc) return rc;
    launch_slmc_kick(s->mom, s->prop, s->grad, 0.5 * step, B * nf, s->sub, s->nq, s->L, B, st);
    for (int l = 1; l <= n_leap; ++l) {
      launch_slmc_drift(s->prop, s->mom, step, B * nf, s->sub, s->nq, s->L, B, st);
      rc = slmc_action_dev(s, s->prop, B, snn_new, true);
      if (rc) return rc;
      launch_slmc_kick(s->mom, s->prop, s->grad, l < n_leap ? step : 0.5 * step, B * nf, s->sub, s->nq, s->L, B,
                       st);
    }
    launch_slmc_sumsq(s->prop, nf, s->sumsq, B, st);
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(q1.data(), s->sumsq, B * sizeof(double), hipMemcpyDeviceToHost));
    launch_slmc_sumsq(s->mom, nf, s->sumsq, B, st);
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpy(p1.data(), s->sumsq, B * sizeof(double), hipMemcpyDeviceToHost));
    for (int z = 0; z < B; ++z) {
      const double h0 = 0.5 * q0[z] + snn_cur[z] + 0.5 * p0[z];
      const double h1 = 0.5 * q1[z] + snn_new[z] + 0.5 * p1[z];
      const double dh = h1 - h0;
      const double u = replay ? replay[(long long)z * rs + (long long)n_traj * nf + k] : host_uniform(s->rng);
      flag[z] = std::isfinite(dh) && std::log(u) < -dh;
      if (std::isfinite(dh)) maxdh[z] = std::max(maxdh[z], std::fabs(dh));
      if (flag[z]) { snn_cur[z] = snn_new[z]; inner[z]++; }
    }
    HIPCHK(hipMemcpy(s->flag, flag.data(), B * sizeof(int), hipMemcpyHostToDevice));
    launch_slmc_select(s->flag, 1, s->prop, s->phi_cur, nf, B, st);
  }
  // exact weight of the proposal from scratch (FP64), then the global test
  HIPCHK(hipMemcpyAsync(s->phi_save, c->phi, B * nf * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(c->phi, s->phi_cur, B * nf * sizeof(double), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemsetAsync(c->d_err, 0, sizeof(int), st));
  rebuild_state(c);
  int ef = 0;
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipMemcpy(&ef, c->d_err, sizeof(int), hipMemcpyDeviceToHost));
  rc = ef ? CFQMC_ENUMERIC : lnw_all(c, lw1, li);
  if (rc == CFQMC_ENUMERIC) lw1.assign(B, -INFINITY);
  else if (rc) return rc;
  bool any_rej = false;
  for (int z = 0; z < B; ++z) {
    const double d_lnw = lw1[z] - lw0[z], d_snn = snn_cur[z] - snn0[z];
    const double lnA = d_lnw + d_snn;
    const double u = replay ? replay[(long long)z * rs + (long long)n_traj * nf + n_traj] : host_uniform(s->rng);
    flag[z] = std::isfinite(lnA) && std::log(u) < lnA;
    any_rej |= !flag[z];
    if (out) {
      out[z].accepted = flag[z];
      out[z].inner_accepted = inner[z];
      out[z].ln_a = lnA;
      out[z].d_lnw = d_lnw;
      out[z].d_snn = d_snn;
      out[z].max_abs_dh = maxdh[z];
    }
  }
  if (any_rej) {
    HIPCHK(hipMemcpy(s->flag, flag.data(), B * sizeof(int), hipMemcpyHostToDevice));
    launch_slmc_select(s->flag, 0, s->phi_save, c->phi, nf, B, st);
    HIPCHK(hipMemsetAsync(c->d_err, 0, sizeof(int), st));
    rebuild_state(c);
  }
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  s->move_counter++;
  return CFQMC_OK;
}

int cfqmc_slmc_last_proposal(cfqmc_slmc* s, int32_t chain, double* phi_out) {
  if (!s || !phi_out || chain < 0 || chain >= s->nch) return CFQMC_EINVAL;
  cfqmc_ctx* c = s->c;
  HIPCHK(hipStreamSynchronize(c->s));
  HIPCHK(hipMemcpy(phi_out, s->phi_cur + (long long)chain * s->nf, s->nf * sizeof(double), hipMemcpyDeviceToHost));
  return CFQMC_OK;
}

int cfqmc_green_maxdiff(const void* x_dev, const void* y_dev, int32_t n, int32_t count, void* hip_stream,
                        double* out) {
  if (!x_dev || !y_dev || !out || n < 1 || count < 1) return CFQMC_EINVAL;
  hipStream_t st = (hipStream_t)hip_stream;
  double* d = nullptr;
  if (hipMalloc(&d, (size_t)4 * count * sizeof(double)) != hipSuccess) return CFQMC_ENOMEM;
  std::vector<double> h((size_t)4 * count, 0.0);
  int rc = CFQMC_OK;
  if (hipMemcpyAsync(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess) rc = CFQMC_EHIP;
  if (!rc) {
    launch_maxdiff((const double2*)x_dev, (const double2*)y_dev, n, (long long)n * n, d, count, st, 4);
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(h.data(), d, h.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
      rc = CFQMC_EHIP;
  }
  hipFree(d);
  if (rc) return rc;
  for (int z = 0; z < count; ++z) {
    out[2 * z] = h[4 * z];
    out[2 * z + 1] = h[4 * z + 1];
    if (!std::isfinite(h[4 * z]) || !std::isfinite(h[4 * z + 1])) rc = CFQMC_ENUMERIC;
  }
  return rc;
}

const char* cfqmc_last_error(const cfqmc_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

}  // extern "C"
