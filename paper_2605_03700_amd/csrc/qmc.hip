// Model-specific kernels of the CF-DQMC sweep (arXiv 2605.03700, Methods).
//
//  build_h       h_i = sum_c phi^i_c q_c from the sparse shift-phase structure
//                of the torus density operator (eq. torus density operator):
//                each m_q has one entry per row, at column k - q_y (mod N), with
//                phase exp(i pi (2k - q_y) q_x / N) (k 1-based).
//  exp_coef /    Taylor exponential of alpha_i h_i in even/odd form:
//  exp_poly      e^{+-A} = E(A^2) +- A O(A^2), degree 13, with a norm check
//                (Al-Mohy & Higham style bound on ||A^4||^(1/4), ||A^6||^(1/6))
//                and scaling by 2^-s followed by s squarings.
//  drift_*       Langevin drift (eq. Langevin proposal, gradient equation with
//                first-order channel derivative), proposal, and the
//                Metropolis-Hastings test with the proposal density.
//  commit, eps   accept/reject bookkeeping and the adaptive step size
//                eps <- eps + (r_a - r_0) d_eps after each sweep.
//  observables   S^i_{q=0} and m^2_SO(5) by Wick's theorem from G.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include "common.h"
#include "kernels.h"

// Random-number counter of a slice move: sweep index * L + slice, the sweep
// index read from device memory when the context keeps it there.
CF_DEV long long step_counter(const StepArgs& a) {
  return a.counter_dev ? a.counter_dev[0] * (long long)a.L + a.tau : a.counter;
}

// ------------------------------------------------------------------ build_h
// h = sum_c phi_c q_c: the terms whose matrix has its nonzeros on the diagonal
// col = row - d (mod N) are grouped by the shift d.
#define BH_CPB 4     // chains per workgroup
#define BH_TC 64     // terms per LDS chunk
#define BH_MAXN 288
// One workgroup per (diagonal d carrying terms, group of BH_CPB entries), one
// thread per row; the diagonals without terms are never written (zero).
// The terms of a diagonal and their phases do not depend on the channel or the
// entry, so each thread computes a term's phase once (table in LDS) and adds
// it into the 4 x BH_CPB (channel, entry) accumulators with weights staged in
// LDS (read by all lanes at the same address).
__global__ void __launch_bounds__(256) build_h_kernel(ModelDev m, const double* phi_all, long long sphi,
                                                      double2* h_all, long long sh, int nbatch) {
  __shared__ double2 s_w[BH_TC][4 * BH_CPB];
  __shared__ int s_qx[BH_TC], s_qy[BH_TC], s_dag[BH_TC], s_cmp[BH_TC];
  __shared__ double2 s_ph[2 * BH_MAXN];
  // all diagonals of one group of entries on one XCD (consecutive workgroups go
  // to the eight XCDs in turn): the rows they write in 16-byte pieces merge in
  // that XCD's L2
  const int ngrp = (nbatch + BH_CPB - 1) / BH_CPB, T = m.nhdiag * ngrp, per = (T + 7) / 8;
  const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= T) return;
  const int d = m.hdiag[t % m.nhdiag], z0 = (t / m.nhdiag) * BH_CPB, N = m.N, N2 = 2 * N;
  const int r = threadIdx.x;
  const int col = ((r - d) % N + N) % N;
  for (int i = threadIdx.x; i < N2; i += blockDim.x) s_ph[i] = m.phase[i];
  double2 acc[4 * BH_CPB];
#pragma unroll
  for (int j = 0; j < 4 * BH_CPB; ++j) acc[j] = make_double2(0.0, 0.0);
  const int tb = m.hoff[d], te = m.hoff[d + 1];
  for (int c0 = tb; c0 < te; c0 += BH_TC) {
    const int cnt = min(BH_TC, te - c0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < cnt * 4 * BH_CPB; idx += blockDim.x) {
      const int k = idx / (4 * BH_CPB), j = idx % (4 * BH_CPB), ch = j / BH_CPB, z = z0 + j % BH_CPB;
      const int t = c0 + k;
      double2 w = make_double2(0.0, 0.0);
      if (z < nbatch) {
        const double* phi = phi_all + z * sphi + ch * m.nq;
        const double f = m.h_F[t] * m.h_scale[t];
        w.x = f * phi[m.h_cre[t]];
        w.y = m.h_cim[t] >= 0 ? f * m.h_sgn[t] * phi[m.h_cim[t]] : 0.0;
      }
      s_w[k][j] = w;
    }
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
      s_qx[k] = m.h_qx[c0 + k];
      s_qy[k] = m.h_qy[c0 + k];
      s_dag[k] = m.h_dag[c0 + k];
      s_cmp[k] = m.h_cre[c0 + k];
    }
    __syncthreads();
    if (r < N) {
      for (int k = 0; k < cnt; ++k) {
        const int qx = s_qx[k], qy = s_qy[k];
        const int row = s_dag[k] ? col : r;        // orbital whose phase enters
        double2 ph;
        if (m.cw) {
          ph = make_double2(m.cw[(long long)s_cmp[k] * N + row], 0.0);   // real sphere weight
        } else {
          int mm = ((2 * (row + 1) - qy) * qx) % N2;
          if (mm < 0) mm += N2;
          ph = s_ph[mm];
          if (s_dag[k]) ph.y = -ph.y;
        }
#pragma unroll
        for (int j = 0; j < 4 * BH_CPB; ++j) {
          const double2 w = s_w[k][j];
          acc[j].x += w.x * ph.x - w.y * ph.y;
          acc[j].y += w.x * ph.y + w.y * ph.x;
        }
      }
    }
  }
  if (r < N) {
#pragma unroll
    for (int j = 0; j < 4 * BH_CPB; ++j) {
      const int ch = j / BH_CPB, z = z0 + j % BH_CPB;
      if (z < nbatch) h_all[z * sh + (long long)ch * N * N + (long long)r * N + col] = acc[j];
    }
  }
}
void launch_build_h(const ModelDev& m, const double* phi, long long sphi, double2* h, long long sh, int nbatch,
                    hipStream_t s) {
  if (m.N > BH_MAXN || m.N > 256) { std::fprintf(stderr, "build_h: N = %d too large\n", m.N); std::abort(); }
  if (m.nhdiag <= 0 || nbatch <= 0) return;
  const int nt = (m.N + 63) / 64 * 64;
  const long long T = (long long)m.nhdiag * ((nbatch + BH_CPB - 1) / BH_CPB);
  dim3 grid((unsigned)((T + 7) / 8 * 8));
  hipLaunchKernelGGL(build_h_kernel, grid, dim3(nt), 0, s, m, phi, sphi, h, sh, nbatch); cfqmc_post_launch("build_h_kernel");
}

// ------------------------------------------------------------------ exponential helpers

__global__ void exp_coef_kernel(const double2* X2all, const double2* X3all, int N, const double2* alpha,
                                int alpha_div, double* coef, int* sq, int smax, double theta, int* err) {
  __shared__ double red[4];
  __shared__ double cs2[256], cs3[256];
  const int b4 = blockIdx.x;   // batch * 4 + channel
  const double2* X2 = X2all + (long long)b4 * N * N;
  const double2* X3 = X3all + (long long)b4 * N * N;
  // 1-norms (max column sums of |x|), N <= 256 (n_phi <= 140): R = 256 / N
  // row groups of threads per column, partial sums combined in LDS
  const int R = 256 / N;
  const int t = threadIdx.x, c = t % N, r0 = t / N;
  double s2 = 0.0, s3 = 0.0;
  if (r0 < R) {
#pragma unroll 4
    for (int i = r0; i < N; i += R) {
      s2 += sqrt(cabs2(X2[(long long)i * N + c]));
      s3 += sqrt(cabs2(X3[(long long)i * N + c]));
    }
  }
  cs2[t] = s2;
  cs3[t] = s3;
  __syncthreads();
  double n2 = 0.0, n3 = 0.0;
  if (r0 == 0) {
    for (int r = 1; r < R; ++r) { s2 += cs2[t + r * N]; s3 += cs3[t + r * N]; }
    n2 = s2;
    n3 = s3;
  }
  for (int o = 32; o > 0; o >>= 1) { n2 = fmax(n2, __shfl_xor(n2, o, 64)); n3 = fmax(n3, __shfl_xor(n3, o, 64)); }
  __shared__ double r3[4];
  if ((threadIdx.x & 63) == 0) { red[threadIdx.x >> 6] = n2; r3[threadIdx.x >> 6] = n3; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) { red[0] = fmax(red[0], red[w]); r3[0] = fmax(r3[0], r3[w]); }
    const int chain_ch = (b4 / 4 / alpha_div) * 4 + (b4 % 4);
    const double2 al = alpha[chain_ch];
    const double aa = sqrt(cabs2(al));
    const double a2 = al.x * al.x - al.y * al.y;   // alpha^2 is real
    const double d = aa * fmax(pow(red[0], 0.25), pow(r3[0], 1.0 / 6.0));
    int s = 0;
    if (d > theta) s = (int)ceil(log2(d / theta));
    if (s > smax) { s = smax; atomicOr(err, 1); }
    sq[2 * b4] = s;        // one predicate per P and Q matrix
    sq[2 * b4 + 1] = s;
    const double w = a2 / pow(4.0, (double)s);
    double* cf = coef + (long long)b4 * EXP_NC;
    double p = 1.0, fe = 1.0, fo = 1.0;   // w^k, (2k)!, (2k+1)!
    for (int k = 0; k < 7; ++k) {
      if (k > 0) { p *= w; fe *= (2.0 * k - 1.0) * (2.0 * k); fo *= (2.0 * k) * (2.0 * k + 1.0); }
      cf[k] = p / fe;
      cf[7 + k] = p / fo;
    }
    const double sc = 1.0 / pow(2.0, (double)s);
    cf[14] = al.x * sc;
    cf[15] = al.y * sc;
  }
}
void launch_exp_coef(const double2* X2, const double2* X3, int N, const double2* alpha, int alpha_div,
                     double* coef, int* sq, int smax, double theta, int* err, int nbatch4, hipStream_t s) {
  if (N > 256) { std::fprintf(stderr, "exp_coef: N = %d exceeds 256\n", N); std::abort(); }
  hipLaunchKernelGGL(exp_coef_kernel, dim3(nbatch4), dim3(256), 0, s, X2, X3, N, alpha, alpha_div, coef, sq, smax,
                     theta, err); cfqmc_post_launch("exp_coef_kernel");
}

// ------------------------------------------------------------------ drift, proposal, MH test

// Diagonals of Y = sum_{v,v'} o_{v'v} (1 - G)^{v v'} needed for Tr[Y m_q] (D1) and Tr[Y m_q^dagger] (D2).
CF_DEV double2 ytilde(const double2* G, int N, int n, int ch, int a, int b) {
  auto z = [&](int v, int vp) -> double2 {
    double2 g = G[(long long)(v * N + a) * n + vp * N + b];
    double2 r = make_double2(-g.x, -g.y);
    if (v == vp && a == b) r.x += 1.0;
    return r;
  };
  switch (ch) {
    case 0: return cadd(z(0, 0), z(1, 1));
    case 1: return cadd(z(0, 1), z(1, 0));
    case 2: { double2 d = csub(z(0, 1), z(1, 0)); return make_double2(-d.y, d.x); }   // i (Z01 - Z10)
    default: return csub(z(0, 0), z(1, 1));
  }
}

#define DR_NT 256
#define DR_MAXN 288
// drift workgroups: one (chain, channel, momentum row) each, a thread per
// component of the row (at most about 2 N / 3 of them at the paper's cut), so
// two waves; LDS sized from N and the widest row (drift_lds_bytes)
#define DRIFT_NT 128

// Drift D = -phi + 2 Re[alpha Tr((1 - G_i)(o_i kron q_c))] of all components in
// trace row `row` of channel `ch`, written to Dl[t - toff[row]]. One thread per
// component: the trace is a length-N phase sum over the two shifted diagonals
// d1, d2 held in LDS (all lanes of a wave read the same k: broadcast), with the
// phase table in LDS and its index advanced by 2 q_x (mod 2N) per k.
CF_DEV void row_drift(const ModelDev& m, const double2* G, const double* phi, double2 alpha, int ch, int row,
                      double* Dl, double2* d1, double2* d2, double2* ph) {
  const int N = m.N, n = m.n, qy = m.t_qy[row], N2 = 2 * N;
  const int c_lo = m.toff[row], c_hi = m.toff[row + 1];
  for (int k = threadIdx.x; k < N; k += DRIFT_NT) {
    d1[k] = ytilde(G, N, n, ch, ((k - qy) % N + N) % N, k);
    d2[k] = ytilde(G, N, n, ch, k, ((k - qy) % N + N) % N);
  }
  for (int i = threadIdx.x; i < N2; i += DRIFT_NT) ph[i] = m.phase[i];
  __syncthreads();
  for (int t = c_lo + threadIdx.x; t < c_hi; t += DRIFT_NT) {
    const int qx = m.t_qx[t];
    // phase index ((2 (k + 1) - q_y) q_x) mod 2N at k = 0, and its step
    int mm = ((2 - qy) * qx) % N2;
    if (mm < 0) mm += N2;
    int st = (2 * qx) % N2;
    if (st < 0) st += N2;
    double tpx = 0.0, tpy = 0.0, tmx = 0.0, tmy = 0.0;
    if (m.tw) {
      // sphere: real weights from global memory, eight loads issued ahead of
      // their products (a load per step would expose its latency N times)
      const double* tw = m.tw + t;
      for (int k0 = 0; k0 < N; k0 += 8) {
        double w[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) w[j] = k0 + j < N ? tw[(long long)(k0 + j) * m.ntw] : 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if (k0 + j >= N) break;
          const double2 a1 = d1[k0 + j], a2 = d2[k0 + j];
          tpx += a1.x * w[j];
          tpy += a1.y * w[j];
          tmx += a2.x * w[j];
          tmy += a2.y * w[j];
        }
      }
    } else {
      for (int k = 0; k < N; ++k) {
        const double2 p = ph[mm], a1 = d1[k], a2 = d2[k];
        tpx += a1.x * p.x - a1.y * p.y;
        tpy += a1.x * p.y + a1.y * p.x;
        tmx += a2.x * p.x + a2.y * p.y;     // d2 conj(p)
        tmy += a2.y * p.x - a2.x * p.y;
        mm += st;
        if (mm >= N2) mm -= N2;
      }
    }
    const double f = m.t_F[t];
    const double2 tp = make_double2(tpx * f, tpy * f), tm = make_double2(tmx * f, tmy * f);
    double2 v;
    const int kind = m.t_kind[t];
    if (kind == 0) v = cscale(tp, sqrt(2.0));                                  // sqrt(2) m_q
    else if (kind == 1) v = cadd(tp, tm);                                      // m_q + m_q^dagger
    else { const double2 d = csub(tp, tm); v = make_double2(-d.y, d.x); }      // i (m_q - m_q^dagger)
    const double2 av = cmul(alpha, v);
    Dl[t - c_lo] = -phi[m.t_comp[t]] + 2.0 * av.x;
  }
  __syncthreads();
}


// (row, channel, chain) of this workgroup: all workgroups of a chain on one XCD
// (consecutive workgroups go to the eight XCDs in turn), so its frames share an L2.
CF_DEV bool drift_block(int nrow, int nchain, int& row, int& ch, int& z) {
  const int per_chain = 4 * nrow, T = per_chain * nchain, per = (T + 7) / 8;
  const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= T) return false;
  z = t / per_chain;
  ch = (t % per_chain) / nrow;
  row = t % nrow;
  return true;
}

// LDS of a drift workgroup: the two gathered diagonals (N each), the phase
// table (2 N) and the row's drifts (widest row)
static size_t drift_lds_bytes(const ModelDev& m) {
  return (size_t)4 * m.N * sizeof(double2) + (size_t)m.maxrow * sizeof(double);
}

__global__ void __launch_bounds__(DRIFT_NT) drift_propose_kernel(ModelDev m, StepArgs a) {
  extern __shared__ double2 drift_lds[];
  double2 *d1 = drift_lds, *d2 = d1 + m.N, *ph = d2 + m.N;
  double* Dl = (double*)(ph + 2 * m.N);
  __shared__ double red[DRIFT_NT / 64];
  int row, ch, z;
  if (!drift_block(m.nrow, a.nchain, row, ch, z)) return;
  const int nq = m.nq;
  const double2* G = a.G[ch] + z * a.sG;
  const double* phi = a.phi + z * a.sphi + ch * nq;
  double* phip = a.phip + z * a.sphip + ch * nq;
  const int c_lo = m.toff[row], c_hi = m.toff[row + 1];
  row_drift(m, G, phi, a.alpha[z * 4 + ch], ch, row, Dl, d1, d2, ph);
  const double eps = a.eps[z];
  double s_norm = 0.0, s_eta = 0.0, s_bg = 0.0;
  for (int t = c_lo + threadIdx.x; t < c_hi; t += DRIFT_NT) {
    const int c = m.t_comp[t];
    const int j = ch * nq + c;
    const double eta = a.noise ? a.noise[z * a.snoise + j] : rng_normal(a.seed, z, step_counter(a), j);
    const double p0 = phi[c];
    const double p1 = p0 + 0.5 * eps * eps * Dl[t - c_lo] + eps * eta;
    phip[c] = p1;
    s_norm += p1 * p1 - p0 * p0;
    s_eta += eta * eta;
    if (ch == 0) s_bg += (p1 - p0) * m.beta[c];
  }
  s_norm = block_sum<DRIFT_NT>(s_norm, red);
  s_eta = block_sum<DRIFT_NT>(s_eta, red);
  s_bg = block_sum<DRIFT_NT>(s_bg, red);
  if (threadIdx.x == 0) {
    double* p = a.part + ((long long)z * a.nblk + ch * m.nrow + row) * 4;
    p[0] = s_norm;
    p[1] = s_eta;
    p[2] = s_bg;
  }
}

__global__ void __launch_bounds__(DRIFT_NT) drift_mh_kernel(ModelDev m, StepArgs a) {
  extern __shared__ double2 drift_lds[];
  double2 *d1 = drift_lds, *d2 = d1 + m.N, *ph = d2 + m.N;
  double* Dl = (double*)(ph + 2 * m.N);
  __shared__ double red[DRIFT_NT / 64];
  int row, ch, z;
  if (!drift_block(m.nrow, a.nchain, row, ch, z)) return;
  const int nq = m.nq;
  const double2* G = a.G[ch] + z * a.sG;
  const double* phi = a.phi + z * a.sphi + ch * nq;
  const double* phip = a.phip + z * a.sphip + ch * nq;
  const int c_lo = m.toff[row], c_hi = m.toff[row + 1];
  row_drift(m, G, phip, a.alpha[z * 4 + ch], ch, row, Dl, d1, d2, ph);   // drift at the proposed fields
  const double eps = a.eps[z];
  double s_rev = 0.0;
  for (int t = c_lo + threadIdx.x; t < c_hi; t += DRIFT_NT) {
    const int c = m.t_comp[t];
    const double r = phi[c] - phip[c] - 0.5 * eps * eps * Dl[t - c_lo];
    s_rev += r * r;
  }
  s_rev = block_sum<DRIFT_NT>(s_rev, red);
  if (threadIdx.x == 0) a.part[((long long)z * a.nblk + ch * m.nrow + row) * 4 + 3] = s_rev;
}

// Metropolis-Hastings decision of chain z from the partial sums the two drift
// kernels left per workgroup (read after the kernel boundary, so no fence or
// arrival counter is needed). Every workgroup that calls it gets the same
// result (same data, same reduction order); only the one with `write` stores
// ln A, the decision and the running statistics. Block size DR_NT.
CF_DEV int mh_decide(const StepArgs& a, int z, bool write, double* red, int* acc_s) {
  double s_norm = 0.0, s_eta = 0.0, s_bg = 0.0, s_r = 0.0;
  const double* pp = a.part + (long long)z * a.nblk * 4;
  for (int b = threadIdx.x; b < a.nblk; b += DR_NT) {
    s_norm += pp[b * 4 + 0];
    s_eta += pp[b * 4 + 1];
    s_bg += pp[b * 4 + 2];
    s_r += pp[b * 4 + 3];
  }
  s_norm = block_sum<DR_NT>(s_norm, red);
  s_eta = block_sum<DR_NT>(s_eta, red);
  s_bg = block_sum<DR_NT>(s_bg, red);
  s_r = block_sum<DR_NT>(s_r, red);
  if (threadIdx.x == 0) {
    const double eps = a.eps[z];
    const double2 ldm = a.lndetM[z];
    const double2 al0 = a.alpha[z * 4 + 0];
    // ln R = 2 ln det M + (c' - c); real for the sign-free model, the phase is monitored
    const double lnR = 2.0 * ldm.x + al0.x * s_bg;
    double ph = fmod(2.0 * ldm.y + al0.y * s_bg, 2.0 * M_PI);
    if (ph > M_PI) ph -= 2.0 * M_PI;
    if (ph < -M_PI) ph += 2.0 * M_PI;
    const double lnA = -0.5 * s_norm + lnR - s_r / (2.0 * eps * eps) + 0.5 * s_eta;
    const double u = a.noise ? a.noise[z * a.snoise + 4 * a.nq] : rng_uniform(a.seed, z, step_counter(a));
    const int acc = (u <= 0.0) ? 1 : (log(u) < lnA ? 1 : 0);
    *acc_s = acc;
    if (write) {
      a.lnA[z] = lnA;
      a.accept[z] = acc;
      if (a.u_out) a.u_out[z] = u;
      double* st = a.stat + z * 8;
      st[0] = fmax(st[0], fabs(ph));
      st[1] += 1.0;
      st[2] += acc;
    }
  }
  __syncthreads();
  return *acc_s;
}

void launch_drift_propose(const ModelDev& m, const StepArgs& a, int nchain, hipStream_t s) {
  StepArgs b = a;
  b.nchain = nchain;
  const int nblk = (int)(((long long)m.nrow * 4 * nchain + 7) / 8 * 8);
  hipLaunchKernelGGL(drift_propose_kernel, dim3(nblk), dim3(DRIFT_NT), drift_lds_bytes(m), s, m, b); cfqmc_post_launch("drift_propose_kernel");
}
void launch_drift_mh(const ModelDev& m, const StepArgs& a, int nchain, hipStream_t s) {
  StepArgs b = a;
  b.nchain = nchain;
  const int nblk = (int)(((long long)m.nrow * 4 * nchain + 7) / 8 * 8);
  hipLaunchKernelGGL(drift_mh_kernel, dim3(nblk), dim3(DRIFT_NT), drift_lds_bytes(m), s, m, b); cfqmc_post_launch("drift_mh_kernel");
}

// ------------------------------------------------------------------ commit
// Takes the Metropolis-Hastings decision of the slice move (every workgroup of
// a chain recomputes it; workgroup 0 records it) and commits the accepted move:
// G <- G', the slice exponentials and fields <- the proposed ones.
// sel (precision guard, may be null): a workgroup whose part of the new G has
// an entry with |G|^2 above gmax2 (or not finite) flags its chain for FP64
// applications; every flagging workgroup writes the same 1.
__global__ void __launch_bounds__(DR_NT) commit_kernel(StepArgs a, const double2* Gp, const double2* G0, double2* G,
                                                       long long nn, long long sG, const double* phip,
                                                       long long sphip, double* phi_tau, long long sphi, int nphi,
                                                       const double2* PQp, long long sPQp, double2* PQ_tau,
                                                       long long sPQ, long long npq, int* acc_count, int* sel,
                                                       double gmax2) {
  __shared__ double red[DR_NT / 64];
  __shared__ double redm[DR_NT / 64];
  __shared__ int acc_s;
  const int z = blockIdx.y;
  const int acc = mh_decide(a, z, blockIdx.x == 0, red, &acc_s);
  const long long tot = nn + npq + nphi;
  double m2 = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < tot; i += (long long)gridDim.x * blockDim.x) {
    if (i < nn) {
      const double2 v = acc ? Gp[z * sG + i] : G0[z * sG + i];
      G[z * sG + i] = v;
      const double a2 = cabs2(v);
      m2 = (a2 > m2 || a2 != a2) ? a2 : m2;   // a NaN stays (it fails the threshold test below)
    } else if (i < nn + npq) {
      if (acc) PQ_tau[z * sPQ + (i - nn)] = PQp[z * sPQp + (i - nn)];
    } else {
      if (acc) phi_tau[z * sphi + (i - nn - npq)] = phip[z * sphip + (i - nn - npq)];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) acc_count[z] += acc;
  if (sel) {
    for (int o = 32; o > 0; o >>= 1) {
      const double other = __shfl_xor(m2, o, 64);
      m2 = (other > m2 || other != other) ? other : m2;
    }
    if ((threadIdx.x & 63) == 0) redm[threadIdx.x >> 6] = m2;
    __syncthreads();
    if (threadIdx.x == 0) {
      bool big = false;
      for (int w = 0; w < DR_NT / 64; ++w) big = big || !(redm[w] <= gmax2);
      if (big) sel[z] = 1;
    }
  }
}
void launch_commit(const StepArgs& a, int nchain, const double2* Gp, const double2* G0, double2* G, long long nn,
                   long long sG, const double* phip, long long sphip, double* phi_tau, long long sphi, int nphi,
                   const double2* PQp, long long sPQp, double2* PQ_tau, long long sPQ, long long npq,
                   int* acc_count, hipStream_t s, int* sel, double gmax) {
  StepArgs b = a;
  b.nchain = nchain;
  const long long tot = nn + npq + nphi;
  dim3 grid((unsigned)std::min<long long>((tot + DR_NT - 1) / DR_NT, 64), nchain);
  hipLaunchKernelGGL(commit_kernel, grid, dim3(DR_NT), 0, s, b, Gp, G0, G, nn, sG, phip, sphip, phi_tau, sphi,
                     nphi, PQp, sPQp, PQ_tau, sPQ, npq, acc_count, sel, gmax * gmax); cfqmc_post_launch("commit_kernel");
}

__global__ void eps_update_kernel(double* eps, int* acc_count, int L, double r0, double deps, double emin,
                                  double emax, int adapt, int nchain) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= nchain) return;
  if (adapt) {
    const double ra = (double)acc_count[z] / (double)L;
    eps[z] = fmin(fmax(eps[z] + (ra - r0) * deps, emin), emax);
  }
  acc_count[z] = 0;
}
void launch_eps_update(double* eps, const int* acc_count, int L, double r0, double deps, double emin, double emax,
                       int adapt, int nchain, hipStream_t s) {
  hipLaunchKernelGGL(eps_update_kernel, dim3((nchain + 63) / 64), dim3(64), 0, s, eps, (int*)acc_count, L, r0, deps,
                     emin, emax, adapt, nchain); cfqmc_post_launch("eps_update_kernel");
}

// ------------------------------------------------------------------ observables
// With G_4N = 1_spin kron G and T_o = o kron 1_N on the spin block:
//   S^{1,2} = F0^2 [ (2 Tr T(1-G))^2 + 2 Tr(T G T (1-G)) ]   (o = tau_x, tau_y)
//   S^{3,4,5} = 2 F0^2 Tr(T G T (1-G))                        (o = tau_z)
// Tr(T G T (1-G)) = Tr G - sum_{a,b} tr_2(o g_ab o g_ba), g_ab the 2x2 valley block.
__global__ void observables_kernel(const double2* Gall, long long sG, int N, double F0, double* out, long long sout) {
  __shared__ double red[4];
  const int z = blockIdx.x, n = 2 * N;
  const double2* G = Gall + z * sG;
  double trG = 0.0, q[3] = {0.0, 0.0, 0.0}, txr = 0.0, txi = 0.0, tyr = 0.0, tyi = 0.0;
  for (int idx = threadIdx.x; idx < N * N; idx += 256) {
    const int a = idx / N, b = idx % N;
    double2 g[2][2], h[2][2];
    for (int v = 0; v < 2; ++v)
      for (int w = 0; w < 2; ++w) {
        g[v][w] = G[(long long)(v * N + a) * n + w * N + b];
        h[v][w] = G[(long long)(v * N + b) * n + w * N + a];
      }
    // tau_x: (o g o)_{vw} = g_{1-v,1-w} ; tau_z: (o g o)_{vw} = s_v s_w g_vw ; tau_y: s_v s_w g_{1-v,1-w} with s = (1,-1) after i*(-i) factors
    double2 sx = make_double2(0, 0), sy = sx, sz = sx;
    for (int v = 0; v < 2; ++v)
      for (int w = 0; w < 2; ++w) {
        const double2 hw = h[w][v];
        const double sgn = (v == w) ? 1.0 : -1.0;
        sx = cadd(sx, cmul(g[1 - v][1 - w], hw));
        sz = cadd(sz, cscale(cmul(g[v][w], hw), sgn));
        sy = cadd(sy, cscale(cmul(g[1 - v][1 - w], hw), sgn));
      }
    q[0] += sx.x; q[1] += sy.x; q[2] += sz.x;
    if (a == b) {
      trG += g[0][0].x + g[1][1].x;
      // tr(tau_x g_aa) = g10 + g01 ; tr(tau_y g_aa) = i (g01 - g10)
      txr += g[1][0].x + g[0][1].x;
      txi += g[1][0].y + g[0][1].y;
      tyr += -(g[0][1].y - g[1][0].y);
      tyi += g[0][1].x - g[1][0].x;
    }
  }
  trG = block_sum<256>(trG, red);
  q[0] = block_sum<256>(q[0], red);
  q[1] = block_sum<256>(q[1], red);
  q[2] = block_sum<256>(q[2], red);
  txr = block_sum<256>(txr, red);
  txi = block_sum<256>(txi, red);
  tyr = block_sum<256>(tyr, red);
  tyi = block_sum<256>(tyi, red);
  if (threadIdx.x == 0) {
    const double f2 = F0 * F0;
    const double cx = trG - q[0], cy = trG - q[1], cz = trG - q[2];
    double* o = out + z * sout;
    // Re[(2 tr T(1-G))^2] = 4 (re^2 - im^2) of tr(T G)
    o[0] = f2 * (4.0 * (txr * txr - txi * txi) + 2.0 * cx);
    o[1] = f2 * (4.0 * (tyr * tyr - tyi * tyi) + 2.0 * cy);
    o[2] = o[3] = o[4] = 2.0 * f2 * cz;
    o[5] = (o[0] + o[1] + o[2] + o[3] + o[4]) / (5.0 * N * N);
    o[6] = trG;
  }
}
void launch_observables(const double2* G, long long sG, int N, double F0, double* out, long long sout, int nchain,
                        hipStream_t s) {
  hipLaunchKernelGGL(observables_kernel, dim3(nchain), dim3(256), 0, s, G, sG, N, F0, out, sout); cfqmc_post_launch("observables_kernel");
}

__global__ void background_kernel(ModelDev m, const double* phi_all, long long sphi_chain, const double2* alpha,
                                  double2* out) {
  __shared__ double red[4];
  const int z = blockIdx.x;
  const double* phi = phi_all + z * sphi_chain;
  double s = 0.0;
  for (int idx = threadIdx.x; idx < m.L * m.nq; idx += 256) {
    const int t = idx / m.nq, c = idx % m.nq;
    s += phi[(long long)t * 4 * m.nq + c] * m.beta[c];
  }
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) out[z] = cscale(alpha[z * 4], s);
}
void launch_background(const ModelDev& m, const double* phi, long long sphi_chain, const double2* alpha,
                       double2* out, int nchain, hipStream_t s) {
  hipLaunchKernelGGL(background_kernel, dim3(nchain), dim3(256), 0, s, m, phi, sphi_chain, alpha, out); cfqmc_post_launch("background_kernel");
}

// Per chain: |phi|^2 (all fields) and the power of the q = 0 components,
// sum_i (sum_tau phi^i_{tau,0})^2 / L. One workgroup per chain.
__global__ void __launch_bounds__(256) field_sums_kernel(const double* phi_all, long long sphi, int L, int nq,
                                                         double* sq, double* q0) {
  __shared__ double red[4];
  const int z = blockIdx.x;
  const double* phi = phi_all + z * sphi;
  const long long cnt = (long long)L * 4 * nq;
  double s = 0.0;
  for (long long i = threadIdx.x; i < cnt; i += 256) s += phi[i] * phi[i];
  s = block_sum<256>(s, red);
  double p = 0.0;
  for (int i = 0; i < 4; ++i) {
    double m = 0.0;
    for (int t = threadIdx.x; t < L; t += 256) m += phi[(long long)t * 4 * nq + (long long)i * nq];
    m = block_sum<256>(m, red);
    p += m * m;
  }
  if (threadIdx.x == 0) {
    sq[z] = s;
    q0[z] = p / L;
  }
}
void launch_field_sums(const double* phi, long long sphi, int L, int nq, double* sq, double* q0, int nchain,
                       hipStream_t s) {
  hipLaunchKernelGGL(field_sums_kernel, dim3(nchain), dim3(256), 0, s, phi, sphi, L, nq, sq, q0);
  cfqmc_post_launch("field_sums_kernel");
}

// Action S = |phi|^2 / 2 - ln w_F with ln w_F = 2 ln|det(1 + B)| + Re sum_tau c_tau,
// ln|det(1 + B)| = ln|det Y| + sum ln D_R^max - ln|det U_R| (UDT form); written
// with the q = 0 power to entry k of the per-chain series.
__global__ void action_series_kernel(const double2* ldY, const double2* ldU, const double* sdm, const double2* bg,
                                     const double* sq, const double* q0, const double* m2, int m2_stride,
                                     double* ser_m, double* ser_s, double* ser_p, long long cap, const int* k_dev,
                                     int nchain) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = *k_dev;
  if (z >= nchain || k >= cap) return;
  const double lnw = 2.0 * (ldY[z].x + sdm[z] - ldU[z].x) + bg[z].x;
  ser_m[z * cap + k] = m2[(long long)z * m2_stride];
  ser_s[z * cap + k] = 0.5 * sq[z] - lnw;
  ser_p[z * cap + k] = q0[z];
}
void launch_action_series(const double2* ldY, const double2* ldU, const double* sdm, const double2* bg,
                          const double* sq, const double* q0, const double* m2, int m2_stride, double* ser_m,
                          double* ser_s, double* ser_p, long long cap, const int* k_dev, int nchain, hipStream_t s) {
  hipLaunchKernelGGL(action_series_kernel, dim3((nchain + 63) / 64), dim3(64), 0, s, ldY, ldU, sdm, bg, sq, q0, m2,
                     m2_stride, ser_m, ser_s, ser_p, cap, k_dev, nchain);
  cfqmc_post_launch("action_series_kernel");
}

// End of a sweep on the device: the sweep counter (random-number stream) and
// the series length advance; both live in device memory so that a captured
// sweep replays unchanged.
__global__ void sweep_advance_kernel(long long* counter, int* series_len, int cap) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    counter[0] += 1;
    if (series_len[0] < cap) series_len[0] += 1;
  }
}
void launch_sweep_advance(long long* counter, int* series_len, int cap, hipStream_t s) {
  hipLaunchKernelGGL(sweep_advance_kernel, dim3(1), dim3(64), 0, s, counter, series_len, cap);
  cfqmc_post_launch("sweep_advance_kernel");
}

__global__ void expand4n_kernel(const double2* G, int n, double2* G4) {
  const int n4 = 2 * n;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n4 * n4; idx += gridDim.x * blockDim.x) {
    const int i = idx / n4, j = idx % n4;
    const int si = i / n, sj = j / n;
    G4[idx] = si == sj ? G[(long long)(i % n) * n + (j % n)] : make_double2(0.0, 0.0);
  }
}
void launch_expand4n(const double2* G, int n, double2* G4, hipStream_t s) {
  hipLaunchKernelGGL(expand4n_kernel, dim3(min((4 * n * n + 255) / 256, 1024)), dim3(256), 0, s, G, n, G4); cfqmc_post_launch("expand4n_kernel");
}

// ------------------------------------------------------------------ imaginary-time correlator
// <n^{Gamma^i}_{q=0}(tau) n^{Gamma^i}_{q=0}(0)> (Supplementary Note 2) of every
// chain for one tau, by Wick's theorem. With T_o = o kron 1_N on the spin block,
// G_4N = 1_spin kron G, X = G(tau,0), Y = G(0,tau), W = G(tau,tau):
//   C^{1,2}   = F0^2 [4 Tr(T W) Tr(T G(0)) - 2 Tr(T X T Y)]   (o = tau_x, tau_y)
//   C^{3,4,5} = -2 F0^2 Tr(T X T Y)                          (o = tau_z; its spin trace
//                                                              removes the disconnected part)
// Tr(T X T Y) = sum o_ab o_cd Tr(X_bc Y_da) over the N x N valley blocks, built
// from eight block products P(a,b,c,d) = Tr(X_ab Y_cd). tr0[chain] holds
// Tr(T_x G(0)), Tr(T_y G(0)) and is written from W when first != 0 (tau = 0).
// One workgroup per chain; out[chain * sout + i], i = 0..4.
__global__ void __launch_bounds__(256) disp_corr_kernel(const double2* Xall, const double2* Yall,
                                                        const double2* Wall, long long sG, int N, double F0,
                                                        double2* tr0, int first, double2* out, long long sout) {
  constexpr int NV = 20;   // 8 block products + 2 block traces, complex
  __shared__ double red[4][NV];
  const int z = blockIdx.x, n = 2 * N;
  const double2* X = Xall + z * sG;
  const double2* Y = Yall + z * sG;
  const double2* W = Wall + z * sG;
  double2 p[8], t[2];
  for (int i = 0; i < 8; ++i) p[i] = make_double2(0.0, 0.0);
  for (int i = 0; i < 2; ++i) t[i] = make_double2(0.0, 0.0);
  for (int idx = threadIdx.x; idx < N * N; idx += 256) {
    const int k = idx / N, kp = idx % N;
    double2 x[2][2], y[2][2];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        x[a][b] = X[(long long)(a * N + k) * n + b * N + kp];
        y[a][b] = Y[(long long)(a * N + kp) * n + b * N + k];
      }
    p[0] = cadd(p[0], cmul(x[1][0], y[1][0]));
    p[1] = cadd(p[1], cmul(x[1][1], y[0][0]));
    p[2] = cadd(p[2], cmul(x[0][0], y[1][1]));
    p[3] = cadd(p[3], cmul(x[0][1], y[0][1]));
    p[4] = cadd(p[4], cmul(x[0][0], y[0][0]));
    p[5] = cadd(p[5], cmul(x[0][1], y[1][0]));
    p[6] = cadd(p[6], cmul(x[1][0], y[0][1]));
    p[7] = cadd(p[7], cmul(x[1][1], y[1][1]));
    if (k == kp) {
      t[0] = cadd(t[0], W[(long long)k * n + N + k]);         // Tr W_01
      t[1] = cadd(t[1], W[(long long)(N + k) * n + k]);       // Tr W_10
    }
  }
  double v[NV];
  for (int i = 0; i < 8; ++i) { v[2 * i] = p[i].x; v[2 * i + 1] = p[i].y; }
  v[16] = t[0].x; v[17] = t[0].y; v[18] = t[1].x; v[19] = t[1].y;
  for (int i = 0; i < NV; ++i) {
    double s = v[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][i] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[NV];
    for (int i = 0; i < NV; ++i) r[i] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
    double2 P[8];
    for (int i = 0; i < 8; ++i) P[i] = make_double2(r[2 * i], r[2 * i + 1]);
    const double2 w01 = make_double2(r[16], r[17]), w10 = make_double2(r[18], r[19]);
    // Tr(tau_x W) = Tr W_10 + Tr W_01 ; Tr(tau_y W) = -i Tr W_10 + i Tr W_01
    const double2 tx = cadd(w10, w01);
    const double2 d = csub(w01, w10);
    const double2 ty = make_double2(-d.y, d.x);
    if (first) {
      tr0[2 * z] = tx;
      tr0[2 * z + 1] = ty;
    }
    const double2 tx0 = first ? tx : tr0[2 * z], ty0 = first ? ty : tr0[2 * z + 1];
    const double2 qx = cadd(cadd(P[0], P[1]), cadd(P[2], P[3]));
    const double2 qy = cadd(csub(P[1], P[0]), csub(P[2], P[3]));
    const double2 qz = cadd(csub(P[4], P[5]), csub(P[7], P[6]));
    const double f2 = F0 * F0;
    double2* o = out + z * sout;
    o[0] = cscale(csub(cscale(cmul(tx, tx0), 4.0), cscale(qx, 2.0)), f2);
    o[1] = cscale(csub(cscale(cmul(ty, ty0), 4.0), cscale(qy, 2.0)), f2);
    o[2] = o[3] = o[4] = cscale(qz, -2.0 * f2);
  }
}
void launch_disp_corr(const double2* X, const double2* Y, const double2* W, long long sG, int N, double F0,
                      double2* tr0, int first, double2* out, long long sout, int nchain, hipStream_t s) {
  hipLaunchKernelGGL(disp_corr_kernel, dim3(nchain), dim3(256), 0, s, X, Y, W, sG, N, F0, tr0, first, out, sout);
  cfqmc_post_launch("disp_corr_kernel");
}

// ------------------------------------------------------------------ structure factors at any q
// S^i_q = <n^{Gamma^i}_q n^{Gamma^i}_{-q}> (Results; the correlation ratio uses
// q = Q + dq) of every chain from the spin-block G by Wick's theorem, with the
// torus density operator (m_q)[k, k - qy] = F(q) exp(i pi (2k - qy) qx / N)
// (k = 1..N) and n_{-q} = n_q^dagger. With T = o kron m_q, G_4N = 1_spin kron G:
//   S^{1,2}_q   = 4 Tr(T_q G) Tr(T_-q G) + 2 [F(q)^2 Tr G - Tr(T_q G T_-q G)]
//   S^{3,4,5}_q = 2 [F(q)^2 Tr G - Tr(T_q G T_-q G)]        (o = tau_z)
// using T_-q T_q = F(q)^2 (o^2 = 1, m_q^dagger m_q = F^2). On the sphere (qw
// non-null) q = (l, m) and the orbital matrix is n_{l,m}[k, k + m] = qw[iq][k]
// (no wrap: zero where k + m >= N), n_{-q} = n_{l,m}^dagger, and F^2 Tr G
// becomes Tr((n^+ n kron 1) G) = sum_j qw[j - m]^2 (G_00 + G_11)[j, j].
// One workgroup per (momentum, chain); out[(chain * nql + iq) * 5 + i].
__global__ void __launch_bounds__(256) sq_kernel(const double2* Gall, long long sG, int N, const int* qxy, int nql,
                                                 const double* qw, double2* out) {
  constexpr int NV = 16;
  __shared__ double red[4][NV];
  const int iq = blockIdx.x, z = blockIdx.y, n = 2 * N;
  const double2* G = Gall + z * sG;
  const double* w = qw ? qw + (long long)iq * N : nullptr;
  // sphere: (l, m) -> shift as q_y = -m, phases 1, weights from the table
  const int qx = w ? 0 : qxy[2 * iq], qy = w ? -qxy[2 * iq + 1] : qxy[2 * iq + 1];
  const int sy = ((qy % N) + N) % N;
  const double F = w ? 1.0 : exp(-2.0 * M_PI * (double)(qx * qx + qy * qy) / (4.0 * N)) / (4.0 * M_PI * sqrt((double)N));
  const int msph = -qy;   // sphere: m
  // row a of m_q: column (a - qy) mod N, phase exp(i pi (2(a+1) - qy) qx / N);
  // row b of m_-q: column (b + qy) mod N, phase exp(-i pi (2(b+1) + qy) qx / N)
  auto ph = [&](long long num) {   // exp(i pi num / N), num reduced mod 2N
    long long r = num % (2LL * N);
    if (r < 0) r += 2LL * N;
    double s, c;
    sincospi((double)r / (double)N, &s, &c);
    return make_double2(c, s);
  };
  double2 qo[3], tq[2], tm[2];
  for (int i = 0; i < 3; ++i) qo[i] = make_double2(0.0, 0.0);
  for (int i = 0; i < 2; ++i) tq[i] = tm[i] = make_double2(0.0, 0.0);
  double2 trg = make_double2(0.0, 0.0);
  for (int idx = threadIdx.x; idx < N * N; idx += 256) {
    const int a = idx / N, b = idx % N;
    const int a2 = (a - sy + N) % N, b4 = (b + sy) % N;
    // m_q[a, a2] m_-q[b, b4]; sphere: w(a) (a + m < N) and w(b - m) (b >= m)
    const double2 c = w ? make_double2((a + msph < N ? w[a] : 0.0) * (b >= msph ? w[b - msph] : 0.0), 0.0)
                        : cscale(cmul(ph((long long)(2 * (a + 1) - qy) * qx), ph(-(long long)(2 * (b + 1) + qy) * qx)),
                                 F * F);
    double2 g1[2][2], g2[2][2];
    for (int v = 0; v < 2; ++v)
      for (int w = 0; w < 2; ++w) {
        g1[v][w] = G[(long long)(v * N + a2) * n + w * N + b];    // G[(v, a2), (w, b)]
        g2[v][w] = G[(long long)(v * N + b4) * n + w * N + a];    // G[(v, b4), (w, a)]
      }
    double2 sx = make_double2(0.0, 0.0), syy = sx, sz = sx;
    for (int v1 = 0; v1 < 2; ++v1)
      for (int v3 = 0; v3 < 2; ++v3) {
        const double s = (v1 == v3) ? 1.0 : -1.0;
        const double2 px = cmul(g1[1 - v1][v3], g2[1 - v3][v1]);
        sx = cadd(sx, px);
        syy = cadd(syy, cscale(px, -s));
        sz = cadd(sz, cscale(cmul(g1[v1][v3], g2[v3][v1]), s));
      }
    qo[0] = cadd(qo[0], cmul(c, sx));
    qo[1] = cadd(qo[1], cmul(c, syy));
    qo[2] = cadd(qo[2], cmul(c, sz));
    if (b == 0) {
      // disconnected parts: Tr(T_q G) and Tr(T_-q G) for o = tau_x, tau_y (row a)
      const double2 mq = w ? make_double2(a + msph < N ? w[a] : 0.0, 0.0) : cscale(ph((long long)(2 * (a + 1) - qy) * qx), F);
      const double2 mm = w ? make_double2(a >= msph ? w[a - msph] : 0.0, 0.0)
                           : cscale(ph(-(long long)(2 * (a + 1) + qy) * qx), F);
      const int am = (a + sy) % N;
      // sum_{v,w} o_vw m[a, col] G[(w, col), (v, a)]
      const double2 x10 = G[(long long)(N + a2) * n + a], x01 = G[(long long)a2 * n + N + a];
      const double2 y10 = G[(long long)(N + am) * n + a], y01 = G[(long long)am * n + N + a];
      // tau_x: G[(1,c),(0,a)] + G[(0,c),(1,a)] ; tau_y: -i G[(1,c),(0,a)] + i G[(0,c),(1,a)]
      const double2 dx = csub(x01, x10), dy = csub(y01, y10);
      tq[0] = cadd(tq[0], cmul(mq, cadd(x10, x01)));
      tq[1] = cadd(tq[1], cmul(mq, make_double2(-dx.y, dx.x)));
      tm[0] = cadd(tm[0], cmul(mm, cadd(y10, y01)));
      tm[1] = cadd(tm[1], cmul(mm, make_double2(-dy.y, dy.x)));
      // F^2 Tr G (torus) or sum_j w(j - m)^2 (G_00 + G_11)[j, j] (sphere), F^2 applied later
      const double dj = w ? (a >= msph ? w[a - msph] * w[a - msph] : 0.0) : 1.0;
      trg = cadd(trg, cscale(cadd(G[(long long)a * n + a], G[(long long)(N + a) * n + N + a]), dj));
    }
  }
  double v[NV];
  for (int i = 0; i < 3; ++i) { v[2 * i] = qo[i].x; v[2 * i + 1] = qo[i].y; }
  for (int i = 0; i < 2; ++i) {
    v[6 + 2 * i] = tq[i].x; v[7 + 2 * i] = tq[i].y;
    v[10 + 2 * i] = tm[i].x; v[11 + 2 * i] = tm[i].y;
  }
  v[14] = trg.x;
  v[15] = trg.y;
  for (int i = 0; i < NV; ++i) {
    double s = v[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][i] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[NV];
    for (int i = 0; i < NV; ++i) r[i] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
    const double2 Qx = make_double2(r[0], r[1]), Qy = make_double2(r[2], r[3]), Qz = make_double2(r[4], r[5]);
    const double2 txq = make_double2(r[6], r[7]), tyq = make_double2(r[8], r[9]);
    const double2 txm = make_double2(r[10], r[11]), tym = make_double2(r[12], r[13]);
    const double2 f2tr = make_double2(F * F * r[14], F * F * r[15]);
    double2* o = out + ((long long)z * nql + iq) * 5;
    o[0] = cadd(cscale(cmul(txq, txm), 4.0), cscale(csub(f2tr, Qx), 2.0));
    o[1] = cadd(cscale(cmul(tyq, tym), 4.0), cscale(csub(f2tr, Qy), 2.0));
    o[2] = o[3] = o[4] = cscale(csub(f2tr, Qz), 2.0);
  }
}
void launch_structure_factors(const double2* G, long long sG, int N, const int* qxy, int nql, const double* qw,
                              double2* out, int nchain, hipStream_t s) {
  hipLaunchKernelGGL(sq_kernel, dim3(nql, nchain), dim3(256), 0, s, G, sG, N, qxy, nql, qw, out);
  cfqmc_post_launch("sq_kernel");
}
