// Dense linear algebra for the sweep: LU with partial pivoting (the Woodbury
// determinant ratio and the recomputation of G), right triangular solves
// (G' = G M^{-1}), and the helpers of the FP64 UDT stabilisation.
//
// LU: one workgroup per matrix. Right-looking blocked factorisation with a
// 16-wide panel held in LDS; the trailing update A22 -= L21 U12 runs on FP64
// MFMA with the A22 tile as the accumulator input. Pivot choice follows the
// LAPACK convention (largest |re|+|im|, first index on ties) and the row
// interchanges are recorded in the LAPACK order, so A = P_0 ... P_{n-1} L U.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <utility>
#include <vector>
#include "common.h"
#include "kernels.h"

#define LU_NB 16
#define LU_NT 512
#define LU_MAXN 288

// One workgroup per matrix, implicit pivoting: rows are never moved in memory;
// perm[i] is the physical row holding logical row i, so P A = L U with
// (P A)[i] = A[perm[i]]. Each thread keeps one row of the current 16-wide panel
// in registers (two barriers per column step: pivot choice and pivot-row
// broadcast); U12 = L11^{-1} A12 is one load/solve/store per column; the
// trailing update A22 -= L21 U12 runs on FP64 MFMA with L21 staged in LDS.
// On exit ipiv[i] = perm[i] and logdet = ln det A.
__global__ void __launch_bounds__(LU_NT) lu_kernel(double2* Aall, int n, int lda, long long sA, int* ipiv_all,
                                                   int sP, double2* logdet, int pivot, const int* only_if,
                                                   const double2* restore) {
  extern __shared__ double2 Ls[];          // panel rows x LU_NB (L11 / L21)
  __shared__ unsigned long long rk[LU_NT / 64];
  __shared__ double2 prow[LU_NB], jrow[LU_NB];
  __shared__ int perm[LU_MAXN];
  __shared__ double2 diag[LU_MAXN];
  __shared__ double2 Linv[LU_NB][LU_NB];
  __shared__ double red2[LU_NT / 64][2];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (only_if && only_if[blockIdx.x] == 0) return;   // fallback launch: nothing to do
  double2* A = Aall + blockIdx.x * sA;
  int* ipiv = ipiv_all + blockIdx.x * sP;
  if (restore) {
    const double2* Rm = restore + blockIdx.x * sA;
    for (int idx = tid; idx < n * n; idx += LU_NT) A[(long long)(idx / n) * lda + idx % n] = Rm[(long long)(idx / n) * lda + idx % n];
    __syncthreads();
  }
  int nswap = 0;                     // thread 0
  for (int i = tid; i < n; i += LU_NT) perm[i] = i;
  __syncthreads();
  for (int k0 = 0; k0 < n; k0 += LU_NB) {
    const int nb = min(LU_NB, n - k0), rows = n - k0;
    const int r = tid;                 // logical panel row owned by this thread
    double2 row[LU_NB];
    {
      const int ph = r < rows ? perm[k0 + r] : 0;
#pragma unroll
      for (int c = 0; c < LU_NB; ++c)
        row[c] = (r < rows && c < nb) ? A[(long long)ph * lda + k0 + c] : make_double2(0.0, 0.0);
    }
    for (int j = 0; j < nb; ++j) {
      double2 rj = row[0];
#pragma unroll
      for (int c = 1; c < LU_NB; ++c)
        if (c == j) rj = row[c];
      int p = j;
      if (pivot) {
        // pivot key: |re|+|im| with its low 12 mantissa bits replaced by the
        // complemented row index, so one unsigned max picks the largest
        // magnitude and the first row among (near) ties
        unsigned long long key = 0ull;
        if (r >= j && r < rows) {
          const double a = fabs(rj.x) + fabs(rj.y);
          key = ((unsigned long long)__double_as_longlong(a) & ~0xFFFull) | (unsigned long long)(0xFFF - r);
        }
        for (int o = 32; o > 0; o >>= 1) {
          const unsigned long long ok = __shfl_xor(key, o, 64);
          key = ok > key ? ok : key;
        }
        if (lane == 0) rk[wid] = key;
      }
      __syncthreads();
      if (pivot) {
        unsigned long long kv[LU_NT / 64];
#pragma unroll
        for (int w = 0; w < LU_NT / 64; ++w) kv[w] = rk[w];
        unsigned long long best = kv[0];
#pragma unroll
        for (int w = 1; w < LU_NT / 64; ++w) best = kv[w] > best ? kv[w] : best;
        p = 0xFFF - (int)(best & 0xFFFull);
      }
      if (r == p) {
#pragma unroll
        for (int c = 0; c < LU_NB; ++c) prow[c] = row[c];
      }
      if (r == j && p != j) {
#pragma unroll
        for (int c = 0; c < LU_NB; ++c) jrow[c] = row[c];
      }
      if (tid == 0) {
        if (p != j) {
          const int t = perm[k0 + j];
          perm[k0 + j] = perm[k0 + p];
          perm[k0 + p] = t;
        }
        nswap += (p != j);
      }
      __syncthreads();
      if (p != j) {
        if (r == p) {
#pragma unroll
          for (int c = 0; c < LU_NB; ++c) row[c] = jrow[c];
        } else if (r == j) {
#pragma unroll
          for (int c = 0; c < LU_NB; ++c) row[c] = prow[c];
        }
      }
      const double2 d = prow[j];
      if (r > j && r < rows) {
        double2 x = row[0];
#pragma unroll
        for (int c = 1; c < LU_NB; ++c)
          if (c == j) x = row[c];
        const double2 l = cdiv(x, d);
#pragma unroll
        for (int c = 0; c < LU_NB; ++c) {
          if (c == j) row[c] = l;
          else if (c > j) row[c] = csub(row[c], cmul(l, prow[c]));
        }
      }
      if (tid == 0) diag[k0 + j] = d;
    }
    __syncthreads();
    if (r < rows) {
      const int ph = perm[k0 + r];
#pragma unroll
      for (int c = 0; c < LU_NB; ++c) {
        if (c < nb) A[(long long)ph * lda + k0 + c] = row[c];
        Ls[r * LU_NB + c] = c < nb ? row[c] : make_double2(0.0, 0.0);
      }
    }
    __syncthreads();
    // U12 = L11^{-1} A12: invert the unit lower 16 x 16 block once (16 lanes,
    // one column each), then one MFMA product per 16-column tile
    if (wid == 0 && lane < LU_NB) {
      for (int i = 0; i < LU_NB; ++i) {
        double2 x = make_double2(i == lane ? 1.0 : 0.0, 0.0);
        if (i < nb)
          for (int l = 0; l < i; ++l) x = csub(x, cmul(Ls[i * LU_NB + l], Linv[l][lane]));
        Linv[i][lane] = x;
      }
    }
    __syncthreads();
    {
      const int c_lo = k0 + nb, ncol = n - c_lo;
      const int ntc = (ncol + 15) / 16;
      const int il = lane & 15, kl = lane >> 4;
      for (int tt = wid; tt < ntc; tt += LU_NT / 64) {
        const int c0 = c_lo + tt * 16;
        double2 b[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int k = kk * 4 + kl;
          b[kk] = (k < nb && c0 + il < n) ? A[(long long)perm[k0 + k] * lda + c0 + il] : make_double2(0.0, 0.0);
        }
        d4v ure = Mfma<double>::zero(), uim = Mfma<double>::zero();
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const double2 a = Linv[il][kk * 4 + kl];
          ure = Mfma<double>::mma(a.x, b[kk].x, ure);
          ure = Mfma<double>::mma(-a.y, b[kk].y, ure);
          uim = Mfma<double>::mma(a.x, b[kk].y, uim);
          uim = Mfma<double>::mma(a.y, b[kk].x, uim);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = Mfma<double>::row(lane, q), jc = c0 + il;
          if (i < nb && jc < n) A[(long long)perm[k0 + i] * lda + jc] = make_double2(ure[q], uim[q]);
        }
      }
    }
    __syncthreads();
    // trailing update on MFMA, tiles of 16 x 16, K = nb zero-padded to 16; 2 tiles per wave per pass
    const int t0 = k0 + nb, rem = n - t0;
    if (rem > 0) {
      const int nt = (rem + 15) / 16, ntt = nt * nt;
      const int il = lane & 15, kl = lane >> 4;
      for (int tb = wid * 2; tb < ntt; tb += (LU_NT / 64) * 2) {
        d4v cre[2], cim[2];
        double2 bu[2][4];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int t = tb + q;
          const int r0 = t0 + (t / nt) * 16, c0 = t0 + (t % nt) * 16;
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int i = r0 + Mfma<double>::row(lane, rr), jc = c0 + il;
            double2 v = make_double2(0.0, 0.0);
            if (t < ntt && i < n && jc < n) v = A[(long long)perm[i] * lda + jc];
            cre[q][rr] = v.x;
            cim[q][rr] = v.y;
          }
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int k = kk * 4 + kl;
            bu[q][kk] = (t < ntt && k < nb && c0 + il < n) ? A[(long long)perm[k0 + k] * lda + c0 + il]
                                                          : make_double2(0.0, 0.0);
          }
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int t = tb + q;
          const int r0 = t0 + (t / nt) * 16;
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int k = kk * 4 + kl;
            const int ar = r0 + il - k0;
            const double2 a = (t < ntt && k < nb && r0 + il < n) ? Ls[ar * LU_NB + k] : make_double2(0.0, 0.0);
            const double2 b = bu[q][kk];
            cre[q] = Mfma<double>::mma(-a.x, b.x, cre[q]);
            cre[q] = Mfma<double>::mma(a.y, b.y, cre[q]);
            cim[q] = Mfma<double>::mma(-a.x, b.y, cim[q]);
            cim[q] = Mfma<double>::mma(-a.y, b.x, cim[q]);
          }
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int t = tb + q;
          if (t >= ntt) continue;
          const int r0 = t0 + (t / nt) * 16, c0 = t0 + (t % nt) * 16;
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int i = r0 + Mfma<double>::row(lane, rr), jc = c0 + il;
            if (i < n && jc < n) A[(long long)perm[i] * lda + jc] = make_double2(cre[q][rr], cim[q][rr]);
          }
        }
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += LU_NT) ipiv[i] = perm[i];
  if (logdet) {
    // ln det = sum ln u_kk + i pi (number of interchanges), summed in parallel
    double lr = 0.0, li = 0.0;
    for (int i = tid; i < n; i += LU_NT) {
      const double2 d = diag[i];
      lr += 0.5 * log(cabs2(d));
      li += atan2(d.y, d.x);
    }
    for (int o = 32; o > 0; o >>= 1) { lr += __shfl_xor(lr, o, 64); li += __shfl_xor(li, o, 64); }
    if (lane == 0) { red2[wid][0] = lr; red2[wid][1] = li; }
    __syncthreads();
    if (tid == 0) {
      lr = 0.0; li = nswap * M_PI;
      for (int w = 0; w < LU_NT / 64; ++w) { lr += red2[w][0]; li += red2[w][1]; }
      double im = fmod(li, 2.0 * M_PI);
      if (im > M_PI) im -= 2.0 * M_PI;
      if (im <= -M_PI) im += 2.0 * M_PI;
      logdet[blockIdx.x] = make_double2(lr, im);
    }
  }
}

// ------------------------------------------------------------------ LU without pivoting
// Blocked LU for matrices close to the identity (the Woodbury matrix
// M = 1 + Delta (1 - G)) and Hermitian positive definite Gram matrices. The
// 16 x 16 diagonal block is factored by one wave in LDS; L11^{-1} and U11^{-1}
// turn the panel solves into MFMA products (U12 = L11^{-1} A12,
// L21 = A21 U11^{-1}), followed by the MFMA trailing update. Threshold test:
// if a multiplier exceeds lmax_allowed (or a value is not finite) flag[z] = 1
// and the caller runs the pivoted factorisation on the saved matrix.
#define NP_NT 256
#define NP_NB 16

CF_DEV void lds_order() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

__global__ void __launch_bounds__(NP_NT) lu_np_global_kernel(double2* Aall, int n, int lda, long long sA, int* ipiv_all,
                                                      int sP, double2* logdet, int* flag_all, double lmax_allowed) {
  __shared__ double2 D[NP_NB][NP_NB];
  __shared__ double2 Li[NP_NB][NP_NB], Ui[NP_NB][NP_NB];
  __shared__ double2 diag[LU_MAXN];
  __shared__ double red[NP_NT / 64][3];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int il = lane & 15, kl = lane >> 4;
  double2* A = Aall + blockIdx.x * sA;
  double lmax = 0.0;
  for (int k0 = 0; k0 < n; k0 += NP_NB) {
    const int nb = min(NP_NB, n - k0);
    {
      const int r = tid / NP_NB, c = tid % NP_NB;
      D[r][c] = (r < nb && c < nb) ? A[(long long)(k0 + r) * lda + k0 + c] : make_double2(r == c ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    if (wid == 0) {
      for (int j = 0; j < nb; ++j) {
        const double2 inv = cdiv(make_double2(1.0, 0.0), D[j][j]);
        double2 nv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = lane + 64 * q, r = e / NP_NB, c = e % NP_NB;
          nv[q] = D[r][c];
          if (r > j) {
            const double2 l = cmul(D[r][j], inv);
            if (c == j) nv[q] = l;
            else if (c > j) nv[q] = csub(nv[q], cmul(l, D[j][c]));
          }
        }
        lds_order();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = lane + 64 * q;
          D[e / NP_NB][e % NP_NB] = nv[q];
        }
        lds_order();
      }
    }
    __syncthreads();
    // inverses of the unit lower and the upper triangle (one column per lane)
    if (wid == 0 && lane < NP_NB) {
      const int t = lane;
      for (int i = 0; i < NP_NB; ++i) {
        double2 x = make_double2(i == t ? 1.0 : 0.0, 0.0);
        if (i < nb)
          for (int l = 0; l < i; ++l) x = csub(x, cmul(D[i][l], Li[l][t]));
        Li[i][t] = x;
      }
    } else if (wid == 1 && lane < NP_NB) {
      const int t = lane;
      for (int i = NP_NB - 1; i >= 0; --i) {
        double2 x = make_double2(i == t ? 1.0 : 0.0, 0.0);
        if (i < nb) {
          for (int l = i + 1; l < NP_NB; ++l) x = csub(x, cmul(D[i][l], Ui[l][t]));
          x = cdiv(x, D[i][i]);
        }
        Ui[i][t] = x;
      }
    } else if (wid == 2) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = lane + 64 * q, r = e / NP_NB, c = e % NP_NB;
        if (r < nb && c < nb) {
          const double2 v = D[r][c];
          A[(long long)(k0 + r) * lda + k0 + c] = v;
          if (r > c) lmax = fmax(lmax, sqrt(cabs2(v)));
          if (r == c) diag[k0 + r] = v;
        }
      }
    }
    __syncthreads();
    // panel solves on MFMA: U12 tiles (columns) and L21 tiles (rows)
    const int t0 = k0 + nb, rem = n - t0;
    if (rem > 0) {
      const int nt = (rem + 15) / 16;
      for (int task = wid; task < 2 * nt; task += NP_NT / 64) {
        d4v cre = Mfma<double>::zero(), cim = Mfma<double>::zero();
        const int tt = task % nt, o0 = t0 + tt * 16;
        if (task < nt) {
          // U12[:, o0..] = L11^{-1} A12
          double2 b[4];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int k = kk * 4 + kl;
            b[kk] = (k < nb && o0 + il < n) ? A[(long long)(k0 + k) * lda + o0 + il] : make_double2(0.0, 0.0);
          }
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const double2 a = Li[il][kk * 4 + kl];
            cre = Mfma<double>::mma(a.x, b[kk].x, cre);
            cre = Mfma<double>::mma(-a.y, b[kk].y, cre);
            cim = Mfma<double>::mma(a.x, b[kk].y, cim);
            cim = Mfma<double>::mma(a.y, b[kk].x, cim);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = Mfma<double>::row(lane, q), jc = o0 + il;
            if (i < nb && jc < n) A[(long long)(k0 + i) * lda + jc] = make_double2(cre[q], cim[q]);
          }
        } else {
          // L21[o0.., :] = A21 U11^{-1}
          double2 a[4];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int k = kk * 4 + kl;
            a[kk] = (k < nb && o0 + il < n) ? A[(long long)(o0 + il) * lda + k0 + k] : make_double2(0.0, 0.0);
          }
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const double2 b = Ui[kk * 4 + kl][il];
            cre = Mfma<double>::mma(a[kk].x, b.x, cre);
            cre = Mfma<double>::mma(-a[kk].y, b.y, cre);
            cim = Mfma<double>::mma(a[kk].x, b.y, cim);
            cim = Mfma<double>::mma(a[kk].y, b.x, cim);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = o0 + Mfma<double>::row(lane, q), jc = il;
            if (i < n && jc < nb) {
              const double2 v = make_double2(cre[q], cim[q]);
              A[(long long)i * lda + k0 + jc] = v;
              lmax = fmax(lmax, sqrt(cabs2(v)));
            }
          }
        }
      }
    }
    __syncthreads();
    // trailing update A22 -= L21 U12 on MFMA, 2 tiles per wave per pass
    if (rem > 0) {
      const int nt = (rem + 15) / 16, ntt = nt * nt;
      for (int tb = wid * 2; tb < ntt; tb += (NP_NT / 64) * 2) {
        d4v cre[2], cim[2];
        double2 au[2][4], bu[2][4];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int t = tb + q;
          const int r0 = t0 + (t / nt) * 16, c0 = t0 + (t % nt) * 16;
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int i = r0 + Mfma<double>::row(lane, rr), jc = c0 + il;
            double2 v = make_double2(0.0, 0.0);
            if (t < ntt && i < n && jc < n) v = A[(long long)i * lda + jc];
            cre[q][rr] = v.x;
            cim[q][rr] = v.y;
          }
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int k = kk * 4 + kl;
            const bool ok = t < ntt && k < nb;
            au[q][kk] = (ok && r0 + il < n) ? A[(long long)(r0 + il) * lda + k0 + k] : make_double2(0.0, 0.0);
            bu[q][kk] = (ok && c0 + il < n) ? A[(long long)(k0 + k) * lda + c0 + il] : make_double2(0.0, 0.0);
          }
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const double2 a = au[q][kk], b = bu[q][kk];
            cre[q] = Mfma<double>::mma(-a.x, b.x, cre[q]);
            cre[q] = Mfma<double>::mma(a.y, b.y, cre[q]);
            cim[q] = Mfma<double>::mma(-a.x, b.y, cim[q]);
            cim[q] = Mfma<double>::mma(-a.y, b.x, cim[q]);
          }
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int t = tb + q;
          if (t >= ntt) continue;
          const int r0 = t0 + (t / nt) * 16, c0 = t0 + (t % nt) * 16;
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int i = r0 + Mfma<double>::row(lane, rr), jc = c0 + il;
            if (i < n && jc < n) A[(long long)i * lda + jc] = make_double2(cre[q][rr], cim[q][rr]);
          }
        }
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += NP_NT) ipiv_all[blockIdx.x * sP + i] = i;
  // ln det and the threshold test
  double lr = 0.0, li = 0.0;
  for (int i = tid; i < n; i += NP_NT) {
    const double2 d = diag[i];
    lr += 0.5 * log(cabs2(d));
    li += atan2(d.y, d.x);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lr += __shfl_xor(lr, o, 64);
    li += __shfl_xor(li, o, 64);
    lmax = fmax(lmax, __shfl_xor(lmax, o, 64));
  }
  if (lane == 0) { red[wid][0] = lr; red[wid][1] = li; red[wid][2] = lmax; }
  __syncthreads();
  if (tid == 0) {
    lr = 0.0; li = 0.0; lmax = 0.0;
    for (int w = 0; w < NP_NT / 64; ++w) { lr += red[w][0]; li += red[w][1]; lmax = fmax(lmax, red[w][2]); }
    const bool bad = !(lmax <= lmax_allowed) || !isfinite(lr);
    if (flag_all) flag_all[blockIdx.x] = bad ? 1 : 0;
    if (logdet) {
      double im = fmod(li, 2.0 * M_PI);
      if (im > M_PI) im -= 2.0 * M_PI;
      if (im <= -M_PI) im += 2.0 * M_PI;
      logdet[blockIdx.x] = make_double2(lr, im);
    }
  }
}



// Same factorisation with the panel in LDS: the solved L21 (rows x 16, rows
// padded to 17 entries against bank conflicts) and U12 (16 x columns) of each
// panel are kept in LDS, so every trailing tile reads only its own A tile from
// memory; 8 waves share the tiles, each loading the A tile of its next pass
// while it multiplies the current one. L11^{-1} and U11^{-1} are formed by
// column elimination in one wave each, four entries per lane.
#define NP2_NT 512
#define NP2_LD 17
__global__ void __launch_bounds__(NP2_NT) lu_np_kernel(double2* Aall, int n, int lda, long long sA, int* ipiv_all,
                                                       int sP, double2* logdet, int* flag_all, double lmax_allowed) {
  extern __shared__ double2 pan[];
  __shared__ double2 D[NP_NB][NP_NB];
  __shared__ double2 Li[NP_NB][NP_NB], Ui[NP_NB][NP_NB];
  __shared__ double2 diag[LU_MAXN];
  __shared__ double red[NP2_NT / 64][3];
  const int capr = n > NP_NB ? n - NP_NB : 1;   // rows of L21 / columns of U12 held
  double2* L21s = pan;                          // [capr][NP2_LD]
  double2* U12s = pan + (long long)capr * NP2_LD;   // [NP_NB][capr]
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int il = lane & 15, kl = lane >> 4;
  constexpr int NW = NP2_NT / 64;
  double2* A = Aall + blockIdx.x * sA;
  double lmax = 0.0;
  for (int k0 = 0; k0 < n; k0 += NP_NB) {
    const int nb = min(NP_NB, n - k0);
    if (wid == 0) {
      // the diagonal block in registers, entries (r, c) = (lane/16 + 4q, lane%16)
      // (identity padding past nb, on which the remaining steps act as the
      // identity); step j takes the pivot row and the multipliers' column from
      // the lanes that hold them
      const int r0 = lane >> 4, c = lane & 15;
      double2 x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = r0 + 4 * q;
        x[q] = (r < nb && c < nb) ? A[(long long)(k0 + r) * lda + k0 + c] : make_double2(r == c ? 1.0 : 0.0, 0.0);
      }
#pragma unroll
      for (int j = 0; j < NP_NB - 1; ++j) {
        const int sj = (j & 3) * 16;
        const double2 djj = make_double2(__shfl(x[j >> 2].x, sj + j, 64), __shfl(x[j >> 2].y, sj + j, 64));
        const double2 djc = make_double2(__shfl(x[j >> 2].x, sj + c, 64), __shfl(x[j >> 2].y, sj + c, 64));
        const double2 inv = crcp(djj);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double2 drj = make_double2(__shfl(x[q].x, r0 * 16 + j, 64), __shfl(x[q].y, r0 * 16 + j, 64));
          if (r0 + 4 * q > j) {
            const double2 l = cmul(drj, inv);
            if (c == j) x[q] = l;
            else if (c > j) x[q] = csub(x[q], cmul(l, djc));
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) D[r0 + 4 * q][c] = x[q];
    }
    __syncthreads();
    if (wid < 2) {
      // L11^{-1} (wave 0, forward) and U11^{-1} (wave 1, backward) by column
      // elimination from the identity: lane holds entries (r, c) = (lane/16 +
      // 4q, lane%16), q < 4; step j takes row j, final at that step, from the
      // lanes that hold it (for U scaled by 1/U_jj) and subtracts its multiples
      // from the rows still open. Rows and columns past nb are identity padding.
      const int r0 = lane >> 4, c = lane & 15;
      double2 x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = make_double2(r0 + 4 * q == c ? 1.0 : 0.0, 0.0);
      if (wid == 0) {
#pragma unroll
        for (int j = 0; j < NP_NB - 1; ++j) {
          const int src = (j & 3) * 16 + c;
          const double2 xj = make_double2(__shfl(x[j >> 2].x, src, 64), __shfl(x[j >> 2].y, src, 64));
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (r0 + 4 * q > j) x[q] = csub(x[q], cmul(D[r0 + 4 * q][j], xj));
          asm volatile("" ::: "memory");   // one step's loads at a time (register budget)
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Li[r0 + 4 * q][c] = x[q];
      } else {
#pragma unroll
        for (int j = NP_NB - 1; j >= 0; --j) {
          const int src = (j & 3) * 16 + c;
          const double2 xj = cmul(make_double2(__shfl(x[j >> 2].x, src, 64), __shfl(x[j >> 2].y, src, 64)),
                                  crcp(D[j][j]));
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = r0 + 4 * q;
            if (r == j) x[q] = xj;
            else if (r < j) x[q] = csub(x[q], cmul(D[r][j], xj));
          }
          asm volatile("" ::: "memory");
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Ui[r0 + 4 * q][c] = x[q];
      }
    } else if (wid == 2) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = lane + 64 * q, r = e / NP_NB, c = e % NP_NB;
        if (r < nb && c < nb) {
          const double2 v = D[r][c];
          A[(long long)(k0 + r) * lda + k0 + c] = v;
          if (r > c) lmax = fmax(lmax, sqrt(cabs2(v)));
          if (r == c) diag[k0 + r] = v;
        }
      }
    }
    __syncthreads();
    const int t0 = k0 + nb, rem = n - t0;
    if (rem > 0) {
      // panel solves: U12 = L11^{-1} A12 (column tiles), L21 = A21 U11^{-1} (row tiles)
      const int nt = (rem + 15) / 16;
      for (int task = wid; task < 2 * nt; task += NW) {
        d4v cre = Mfma<double>::zero(), cim = Mfma<double>::zero();
        const int tt = task % nt, o0 = t0 + tt * 16;
        if (task < nt) {
          double2 b[4];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int k = kk * 4 + kl;
            b[kk] = (k < nb && o0 + il < n) ? A[(long long)(k0 + k) * lda + o0 + il] : make_double2(0.0, 0.0);
          }
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const double2 a = Li[il][kk * 4 + kl];
            cre = Mfma<double>::mma(a.x, b[kk].x, cre);
            cre = Mfma<double>::mma(-a.y, b[kk].y, cre);
            cim = Mfma<double>::mma(a.x, b[kk].y, cim);
            cim = Mfma<double>::mma(a.y, b[kk].x, cim);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = Mfma<double>::row(lane, q), jc = o0 + il;
            if (jc < n) {
              const double2 v = i < nb ? make_double2(cre[q], cim[q]) : make_double2(0.0, 0.0);
              if (i < nb) A[(long long)(k0 + i) * lda + jc] = v;
              U12s[(long long)i * capr + (jc - t0)] = v;
            }
          }
        } else {
          double2 a[4];
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const int k = kk * 4 + kl;
            a[kk] = (k < nb && o0 + il < n) ? A[(long long)(o0 + il) * lda + k0 + k] : make_double2(0.0, 0.0);
          }
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) {
            const double2 b = Ui[kk * 4 + kl][il];
            cre = Mfma<double>::mma(a[kk].x, b.x, cre);
            cre = Mfma<double>::mma(-a[kk].y, b.y, cre);
            cim = Mfma<double>::mma(a[kk].x, b.y, cim);
            cim = Mfma<double>::mma(a[kk].y, b.x, cim);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = o0 + Mfma<double>::row(lane, q), jc = il;
            if (i < n) {
              const double2 v = jc < nb ? make_double2(cre[q], cim[q]) : make_double2(0.0, 0.0);
              if (jc < nb) {
                A[(long long)i * lda + k0 + jc] = v;
                lmax = fmax(lmax, sqrt(cabs2(v)));
              }
              L21s[(long long)(i - t0) * NP2_LD + jc] = v;
            }
          }
        }
      }
      __syncthreads();
      // trailing update A22 -= L21 U12, one 16 x 16 tile per wave per pass; the
      // A tile of the wave's next pass is loaded while this one is multiplied
      const int ntt = nt * nt;
      double2 cur[4], nxt[4];
      auto load_tile = [&](int t, double2 (&r)[4]) {
        const int r0 = (t / nt) * 16, c0 = (t % nt) * 16;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int i = t0 + r0 + Mfma<double>::row(lane, rr), jc = t0 + c0 + il;
          const bool ok = t < ntt && i < n && jc < n;
          r[rr] = A[ok ? (long long)i * lda + jc : 0];
        }
      };
      if (wid < ntt) load_tile(wid, cur);
      for (int t = wid; t < ntt; t += NW) {
        if (t + NW < ntt) load_tile(t + NW, nxt);
        const int r0 = (t / nt) * 16, c0 = (t % nt) * 16;
        d4v cre, cim;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          cre[rr] = cur[rr].x;
          cim[rr] = cur[rr].y;
        }
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int k = kk * 4 + kl;
          const double2 a = r0 + il < rem ? L21s[(long long)(r0 + il) * NP2_LD + k] : make_double2(0.0, 0.0);
          const double2 b = c0 + il < rem ? U12s[(long long)k * capr + c0 + il] : make_double2(0.0, 0.0);
          cre = Mfma<double>::mma(-a.x, b.x, cre);
          cre = Mfma<double>::mma(a.y, b.y, cre);
          cim = Mfma<double>::mma(-a.x, b.y, cim);
          cim = Mfma<double>::mma(-a.y, b.x, cim);
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int i = t0 + r0 + Mfma<double>::row(lane, rr), jc = t0 + c0 + il;
          if (i < n && jc < n) A[(long long)i * lda + jc] = make_double2(cre[rr], cim[rr]);
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) cur[rr] = nxt[rr];
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += NP2_NT) ipiv_all[blockIdx.x * sP + i] = i;
  double lr = 0.0, li = 0.0;
  for (int i = tid; i < n; i += NP2_NT) {
    const double2 d = diag[i];
    lr += 0.5 * log(cabs2(d));
    li += atan2(d.y, d.x);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lr += __shfl_xor(lr, o, 64);
    li += __shfl_xor(li, o, 64);
    lmax = fmax(lmax, __shfl_xor(lmax, o, 64));
  }
  if (lane == 0) { red[wid][0] = lr; red[wid][1] = li; red[wid][2] = lmax; }
  __syncthreads();
  if (tid == 0) {
    lr = 0.0; li = 0.0; lmax = 0.0;
    for (int w = 0; w < NW; ++w) { lr += red[w][0]; li += red[w][1]; lmax = fmax(lmax, red[w][2]); }
    const bool bad = !(lmax <= lmax_allowed) || !isfinite(lr);
    if (flag_all) flag_all[blockIdx.x] = bad ? 1 : 0;
    if (logdet) {
      double im = fmod(li, 2.0 * M_PI);
      if (im > M_PI) im -= 2.0 * M_PI;
      if (im <= -M_PI) im += 2.0 * M_PI;
      logdet[blockIdx.x] = make_double2(lr, im);
    }
  }
}

static bool set_lds_limit(const void* fn, size_t shm);


void launch_lu_np(double2* A, int n, int lda, long long sA, int* ipiv, int sP, double2* logdet, int* flag,
                  double lmax_allowed, int nbatch, hipStream_t s) {
  const int capr = n > NP_NB ? n - NP_NB : 1;
  const size_t shm = (size_t)capr * (NP2_LD + NP_NB) * sizeof(double2);
  if (n <= LU_MAXN && set_lds_limit((const void*)lu_np_kernel, shm)) {
    hipLaunchKernelGGL(lu_np_kernel, dim3(nbatch), dim3(NP2_NT), shm, s, A, n, lda, sA, ipiv, sP, logdet, flag,
                       lmax_allowed); cfqmc_post_launch("lu_np_kernel");
  } else {
    hipLaunchKernelGGL(lu_np_global_kernel, dim3(nbatch), dim3(NP_NT), 0, s, A, n, lda, sA, ipiv, sP, logdet, flag,
                       lmax_allowed); cfqmc_post_launch("lu_np_global_kernel");
  }
}

// Allow more than 64 KB of dynamic LDS (gfx950 has 160 KB per workgroup); returns false if refused.
// A limit once granted is remembered per kernel, so that later launches (also
// those recorded into a sweep graph) make no runtime call for it.
static bool set_lds_limit(const void* fn, size_t shm) {
  if (shm <= 65536 - 24 * 1024) return true;
  static std::mutex mu;
  static std::vector<std::pair<const void*, size_t>> granted;
  std::lock_guard<std::mutex> lock(mu);
  for (const auto& g : granted)
    if (g.first == fn && g.second >= shm) return true;
  const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  (void)hipGetLastError();
  if (e != hipSuccess) return false;
  for (auto& g : granted)
    if (g.first == fn) { g.second = shm; return true; }
  granted.emplace_back(fn, shm);
  return true;
}

void launch_lu(double2* A, int n, int lda, long long sA, int* ipiv, int sP, double2* logdet, int pivot,
               int nbatch, hipStream_t s, const int* only_if, const double2* restore) {
  const size_t shm = (size_t)n * LU_NB * sizeof(double2);
  if (!set_lds_limit((const void*)lu_kernel, shm)) fprintf(stderr, "[cfqmc] LU: %zu B of LDS refused\n", shm);
  hipLaunchKernelGGL(lu_kernel, dim3(nbatch), dim3(LU_NT), shm, s, A, n, lda, sA, ipiv, sP, logdet, pivot, only_if,
                     restore); cfqmc_post_launch("lu_kernel");
}

// ------------------------------------------------------------------ right solve
// Y = X A^{-1} with P A = L U, (P A)[i] = A[perm[i]] (lu_kernel): Y = X U^{-1} L^{-1} P,
// i.e. W = X U^{-1} L^{-1} and Y[:, perm[i]] = W[:, i]. Row k of the factors is
// physical row perm[k]. A workgroup owns 16 rows of X.
#define RS_ROWS 16

// Inverses of the 16 x 16 diagonal blocks of U and of the unit-lower L of a
// factorisation from launch_lu / launch_lu_np (rows addressed through ipiv):
// Ui_J = U_JJ^{-1}, Li_J = L_JJ^{-1}, padded with the identity past n. Row r of
// an inverse solves z T = e_r, by the same substitution as the blocked solve.
// inv layout: [batch][nJ][2][16][16] (U then L).
__global__ void __launch_bounds__(256) tri_inv_kernel(const double2* LUall, int ldlu, long long sLU,
                                                      const int* ipiv_all, int sP, int n, int upper_only,
                                                      double2* inv_all) {
  __shared__ double2 Db[16][17];
  __shared__ double2 Dr[16];
  const int J = blockIdx.x, z = blockIdx.y, nJ = gridDim.x;
  const double2* LU = LUall + z * sLU;
  const int* ipiv = ipiv_all + z * sP;
  double2* inv = inv_all + ((long long)z * nJ + J) * 512;
  const int tid = threadIdx.x, lane = tid & 63, rr = tid >> 4, cc = tid & 15;
  const int c0 = 16 * J, bw = min(16, n - c0);
  const bool okd = rr < bw && cc < bw;
  const double2 dd = okd ? LU[(long long)(upper_only ? c0 + rr : ipiv[c0 + rr]) * ldlu + c0 + cc]
                         : make_double2(rr == cc ? 1.0 : 0.0, 0.0);
  Db[rr][cc] = dd;
  if (rr == cc) Dr[cc] = crcp(dd);
  __syncthreads();
  double2 y = make_double2(rr == cc ? 1.0 : 0.0, 0.0);
  for (int cp = 0; cp < 16; ++cp) {
    double2 zv = cmul(y, Dr[cp]);
    zv.x = __shfl(zv.x, (lane & ~15) + cp, 64);
    zv.y = __shfl(zv.y, (lane & ~15) + cp, 64);
    if (cc == cp) y = zv;
    else if (cc > cp) y = csub(y, cmul(zv, Db[cp][cc]));
  }
  inv[rr * 16 + cc] = y;
  if (upper_only) return;
  y = make_double2(rr == cc ? 1.0 : 0.0, 0.0);
  for (int cp = 15; cp >= 0; --cp) {
    double2 wv;
    wv.x = __shfl(y.x, (lane & ~15) + cp, 64);
    wv.y = __shfl(y.y, (lane & ~15) + cp, 64);
    if (cc < cp) y = csub(y, cmul(wv, Db[cp][cc]));
  }
  inv[256 + rr * 16 + cc] = y;
}

// Right-looking form of the same solve with the inverted diagonal blocks. The
// 16-row block of the right-hand side lives in MFMA accumulators: column tile t
// belongs to wave t % NW. At step J the owner wave multiplies its tile by the
// inverse diagonal block (one 16 x 16 x 16 product instead of a 16-step
// substitution) and publishes the solved block in LDS; after one barrier every
// wave subtracts it times row block J of U (phase 0) or L (phase 1) from the
// tiles it owns that are not solved yet. The published block is double-buffered;
// the owner's layout change goes through one LDS tile (one owner per step, and
// the barrier separates consecutive owners).
// CT = float (the rank-k update in FP32): the operands are rounded to FP32 as
// they enter the MFMAs, each 16-deep step's product is formed in FP32 and
// subtracted from the FP64 right-hand-side tile (an FP64 accumulation point per
// step); the tile then follows the FP32 instruction's result layout. sel: only
// the chains with sel[z] == want (the precision guard's classes), else all.
template <int NW, int MAXT, typename CT>
__global__ void __launch_bounds__(NW * 64) rsolve_rl_kernel(const double2* Xall, int ldx, long long sX,
                                                            double2* Yall, int ldy, long long sY,
                                                            const double2* LUall, int ldlu, long long sLU,
                                                            const int* ipiv_all, int sP, int n, int upper_only,
                                                            const double2* inv_all, int nbatch, const int* sel,
                                                            int want) {
  typedef Mfma<CT> MF;
  constexpr int NT = NW * 64;
  __shared__ double2 Tb[2][16][17];        // solved block of the step
  __shared__ double2 Tw[16][17];           // owner's layout change
  __shared__ int perm[LU_MAXN];
  const int nrb = (n + RS_ROWS - 1) / RS_ROWS, T = nrb * nbatch, per = (T + 7) / 8;
  const int t = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (t >= T) return;
  const int z = t / nrb;
  if (sel && sel[z] != want) return;
  const int nJ = (n + 15) / 16;
  const double2* X = Xall + z * sX;
  double2* Yo = Yall + z * sY;
  const double2* LU = LUall + z * sLU;
  const int* ipiv = ipiv_all + z * sP;
  const double2* inv = inv_all + (long long)z * nJ * 512;
  const int r0 = (t % nrb) * RS_ROWS;
  const int nr = min(RS_ROWS, n - r0);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int il = lane & 15, kl = lane >> 4;
  for (int i = tid; i < n; i += NT) perm[i] = upper_only ? i : ipiv[i];
  const double2 zero2 = make_double2(0.0, 0.0);
  d4v are[MAXT], aim[MAXT];
#pragma unroll
  for (int i = 0; i < MAXT; ++i) {
    const int tc = wid + NW * i;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = MF::row(lane, q), c = 16 * tc + il;
      const bool ok = tc < nJ && r < nr && c < n;
      const double2 v = X[ok ? (long long)(r0 + r) * ldx + c : 0];
      are[i][q] = ok ? v.x : 0.0;
      aim[i][q] = ok ? v.y : 0.0;
    }
  }
  __syncthreads();
  const int last_phase = upper_only ? 0 : 1;
  int step = 0;
  for (int phase = 0; phase <= last_phase; ++phase) {
    for (int jj = 0; jj < nJ; ++jj, ++step) {
      const int J = phase == 0 ? jj : nJ - 1 - jj;
      const int c0 = 16 * J, bw = min(16, n - c0), buf = step & 1;
      const bool owner = (J % NW) == wid;
      // loads of this step: row block J for the tiles still to update, and
      // (owner) the inverse diagonal block
      double2 bb[MAXT][4];
#pragma unroll
      for (int i = 0; i < MAXT; ++i) {
        const int tc = wid + NW * i;
        const bool upd = phase == 0 ? (tc > J && tc < nJ) : (tc < J);
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int k = 4 * s4 + kl, c = 16 * tc + il;
          const bool ok = upd && k < bw && c < n;
          bb[i][s4] = LU[ok ? (long long)perm[c0 + k] * ldlu + c : 0];
          if (!ok) bb[i][s4] = zero2;
        }
      }
      if (owner) {
        const double2* ib = inv + (long long)J * 512 + phase * 256;
        double2 bi[4];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) bi[s4] = ib[(4 * s4 + kl) * 16 + il];
        // the owner's tile J: accumulator layout -> A-operand layout through LDS
        const int io = J / NW;
#pragma unroll
        for (int i = 0; i < MAXT; ++i)
          if (i == io)
#pragma unroll
            for (int q = 0; q < 4; ++q) Tw[MF::row(lane, q)][il] = make_double2(are[i][q], aim[i][q]);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        d4v zr, zi;
        if constexpr (sizeof(CT) == 8) {
          zr = Mfma<double>::zero();
          zi = Mfma<double>::zero();
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const double2 a = Tw[il][4 * s4 + kl], b = bi[s4];
            zr = Mfma<double>::mma(a.x, b.x, zr);
            zr = Mfma<double>::mma(-a.y, b.y, zr);
            zi = Mfma<double>::mma(a.x, b.y, zi);
            zi = Mfma<double>::mma(a.y, b.x, zi);
          }
        } else {
          f4v zr32 = Mfma<float>::zero(), zi32 = Mfma<float>::zero();
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const float2 a = to_ct<float>(Tw[il][4 * s4 + kl]), b = to_ct<float>(bi[s4]);
            zr32 = Mfma<float>::mma(a.x, b.x, zr32);
            zr32 = Mfma<float>::mma(-a.y, b.y, zr32);
            zi32 = Mfma<float>::mma(a.x, b.y, zi32);
            zi32 = Mfma<float>::mma(a.y, b.x, zi32);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            zr[q] = zr32[q];
            zi[q] = zi32[q];
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = MF::row(lane, q);
          const double2 v = make_double2(zr[q], zi[q]);
          Tb[buf][r][il] = v;
          // the last phase's solved block is final: columns perm[c0 + il] of the output
          if (phase == last_phase && r < nr && il < bw) Yo[(long long)(r0 + r) * ldy + perm[c0 + il]] = v;
        }
        // tile J after phase 0 is the input of phase 1
        if (phase == 0) {
#pragma unroll
          for (int i = 0; i < MAXT; ++i)
            if (i == io) { are[i] = zr; aim[i] = zi; }
        }
      }
      __syncthreads();
      // A operand: the solved block (m = il, k = 4 s4 + kl)
      double2 av[4];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) av[s4] = Tb[buf][il][4 * s4 + kl];
      // tile -= solved block x row block (four real products per k step: a
      // three-product form needs registers that cost a wave per SIMD here)
#pragma unroll
      for (int i = 0; i < MAXT; ++i) {
        const int tc = wid + NW * i;
        const bool upd = phase == 0 ? (tc > J && tc < nJ) : (tc < J);
        if (upd) {
          if constexpr (sizeof(CT) == 8) {
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
              const double2 a = av[s4], b = bb[i][s4];
              are[i] = Mfma<double>::mma(-a.x, b.x, are[i]);
              are[i] = Mfma<double>::mma(a.y, b.y, are[i]);
              aim[i] = Mfma<double>::mma(-a.x, b.y, aim[i]);
              aim[i] = Mfma<double>::mma(-a.y, b.x, aim[i]);
            }
          } else {
            f4v pr = Mfma<float>::zero(), pi = Mfma<float>::zero();
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
              const float2 a = to_ct<float>(av[s4]), b = to_ct<float>(bb[i][s4]);
              pr = Mfma<float>::mma(a.x, b.x, pr);
              pr = Mfma<float>::mma(-a.y, b.y, pr);
              pi = Mfma<float>::mma(a.x, b.y, pi);
              pi = Mfma<float>::mma(a.y, b.x, pi);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              are[i][q] -= pr[q];
              aim[i][q] -= pi[q];
            }
          }
        }
      }
    }
  }
}

template <typename CT>
static void run_rsolve(const double2* X, int ldx, long long sX, double2* Y, int ldy, long long sY, const double2* LU,
                       int ldlu, long long sLU, const int* ipiv, int sP, int n, int upper_only, int nbatch,
                       hipStream_t s, const double2* inv, const int* sel, int want) {
  const int nrb = (n + RS_ROWS - 1) / RS_ROWS;
  const int nblk = (int)(((long long)nrb * nbatch + 7) / 8 * 8);
  // eight waves, each owning at most ceil(nJ / 8) column tiles (2 for n <= 256)
  if (n <= 256)
    hipLaunchKernelGGL((rsolve_rl_kernel<8, 2, CT>), dim3(nblk), dim3(512), 0, s, X, ldx, sX, Y, ldy, sY, LU, ldlu,
                       sLU, ipiv, sP, n, upper_only, inv, nbatch, sel, want);
  else
    hipLaunchKernelGGL((rsolve_rl_kernel<8, 3, CT>), dim3(nblk), dim3(512), 0, s, X, ldx, sX, Y, ldy, sY, LU, ldlu,
                       sLU, ipiv, sP, n, upper_only, inv, nbatch, sel, want);
  cfqmc_post_launch("rsolve_rl_kernel");
}

void launch_rsolve(const double2* X, int ldx, long long sX, double2* Y, int ldy, long long sY, const double2* LU,
                   int ldlu, long long sLU, const int* ipiv, int sP, int n, int upper_only, int nbatch,
                   hipStream_t s, double2* work, int mixed, const int* sel64) {
  if (!work || n > LU_MAXN) {
    std::fprintf(stderr, "rsolve: workspace missing or n = %d above %d\n", n, LU_MAXN);
    std::abort();
  }
  const int nJ = (n + 15) / 16;
  hipLaunchKernelGGL(tri_inv_kernel, dim3(nJ, nbatch), dim3(256), 0, s, LU, ldlu, sLU, ipiv, sP, n, upper_only, work);
  cfqmc_post_launch("tri_inv_kernel");
  const double2* inv = work;
  if (!mixed) {
    run_rsolve<double>(X, ldx, sX, Y, ldy, sY, LU, ldlu, sLU, ipiv, sP, n, upper_only, nbatch, s, inv, nullptr, 0);
    return;
  }
  // FP32 products for every chain, or with sel64 for the chains it leaves at 0
  // (the FP64 ones in a launch of their own)
  run_rsolve<float>(X, ldx, sX, Y, ldy, sY, LU, ldlu, sLU, ipiv, sP, n, upper_only, nbatch, s, inv, sel64, 0);
  if (sel64)
    run_rsolve<double>(X, ldx, sX, Y, ldy, sY, LU, ldlu, sLU, ipiv, sP, n, upper_only, nbatch, s, inv, sel64, 1);
}

// ------------------------------------------------------------------ elementwise helpers

__global__ void set_identity_kernel(double2* A, int n, int lda, long long sA) {
  double2* M = A + blockIdx.y * sA;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * n; idx += gridDim.x * blockDim.x) {
    const int i = idx / n, j = idx % n;
    M[(long long)i * lda + j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
}
void launch_set_identity(double2* A, int n, int lda, long long sA, int nbatch, hipStream_t s) {
  dim3 grid(min((n * n + 255) / 256, 1024), nbatch);
  hipLaunchKernelGGL(set_identity_kernel, grid, dim3(256), 0, s, A, n, lda, sA); cfqmc_post_launch("set_identity_kernel");
}

__global__ void fill_kernel(double* p, long long count, double v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}
void launch_fill(double* p, long long count, double v, hipStream_t s) {
  if (count <= 0) return;
  const int nblk = (int)std::min<long long>((count + 255) / 256, 1024);
  hipLaunchKernelGGL(fill_kernel, dim3(nblk), dim3(256), 0, s, p, count, v); cfqmc_post_launch("fill_kernel");
}

__global__ void copy_kernel(const double2* X, double2* Y, long long count, long long sX, long long sY) {
  const double2* x = X + blockIdx.y * sX;
  double2* y = Y + blockIdx.y * sY;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    y[i] = x[i];
}
void launch_copy(const double2* X, double2* Y, long long count, long long sX, long long sY, int nbatch,
                 hipStream_t s) {
  if (count <= 0 || nbatch <= 0) return;
  dim3 grid((unsigned)std::min<long long>((count + 255) / 256, 2048), nbatch);
  hipLaunchKernelGGL(copy_kernel, grid, dim3(256), 0, s, X, Y, count, sX, sY); cfqmc_post_launch("copy_kernel");
}

__global__ void colscale_kernel(const double2* X, int ldx, long long sX, double2* Y, int ldy, long long sY,
                                const double* d, long long sd, int nr, int nc, int inv) {
  const int z = blockIdx.y;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < nr * nc; idx += gridDim.x * blockDim.x) {
    const int i = idx / nc, j = idx % nc;
    const double f = inv ? 1.0 / d[z * sd + j] : d[z * sd + j];
    Y[z * sY + (long long)i * ldy + j] = cscale(X[z * sX + (long long)i * ldx + j], f);
  }
}
void launch_colscale(const double2* X, int ldx, long long sX, double2* Y, int ldy, long long sY, const double* d,
                     long long sd, int n_rows, int n_cols, int inv, int nbatch, hipStream_t s) {
  dim3 grid(min((n_rows * n_cols + 255) / 256, 1024), nbatch);
  hipLaunchKernelGGL(colscale_kernel, grid, dim3(256), 0, s, X, ldx, sX, Y, ldy, sY, d, sd, n_rows, n_cols, inv); cfqmc_post_launch("colscale_kernel");
}

// Per chain: out[4z+2] = max |X - Y| and out[4z+3] = max |Y| (atomic max over
// blocks), then maxdiff_fold folds them into the running maxima out[4z+0]
// (absolute) and out[4z+1] (relative to max |Y|) and clears the temporaries.
__global__ void maxdiff_kernel(const double2* X, const double2* Y, int n, long long sX, double* out, int so) {
  __shared__ double red[4], redy[4];
  const int z = blockIdx.y;
  double m = 0.0, my = 0.0;
  for (int idx = blockIdx.x * 256 + threadIdx.x; idx < n * n; idx += gridDim.x * 256) {
    const double2 a = X[z * sX + idx], b = Y[z * sX + idx];
    // fmax drops a NaN operand: a non-finite difference or entry counts as +inf
    double d = sqrt(cabs2(csub(a, b))), y = sqrt(cabs2(b));
    if (!(d <= 1.7976931348623157e308)) d = INFINITY;
    if (!(y <= 1.7976931348623157e308)) y = INFINITY;
    m = fmax(m, d);
    my = fmax(my, y);
  }
  for (int o = 32; o > 0; o >>= 1) {
    m = fmax(m, __shfl_xor(m, o, 64));
    my = fmax(my, __shfl_xor(my, o, 64));
  }
  if ((threadIdx.x & 63) == 0) { red[threadIdx.x >> 6] = m; redy[threadIdx.x >> 6] = my; }
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    my = fmax(fmax(redy[0], redy[1]), fmax(redy[2], redy[3]));
    // non-negative doubles order like their bit patterns
    atomicMax((unsigned long long*)&out[so * z + 2], (unsigned long long)__double_as_longlong(m));
    atomicMax((unsigned long long*)&out[so * z + 3], (unsigned long long)__double_as_longlong(my));
  }
}
__global__ void maxdiff_fold_kernel(double* out, int nbatch, int so, double* last) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= nbatch) return;
  const double d = out[so * z + 2], gm = out[so * z + 3];
  if (last) {
    last[2 * z] = d;
    last[2 * z + 1] = gm;
  }
  // +inf (a non-finite entry on either side) stays +inf in both maxima
  const double r = (isinf(d) || isinf(gm)) ? INFINITY : (gm > 0.0 ? d / gm : d);
  out[so * z + 0] = fmax(out[so * z + 0], d);
  out[so * z + 1] = fmax(out[so * z + 1], r);
  out[so * z + 2] = 0.0;
  out[so * z + 3] = 0.0;
}
void launch_maxdiff(const double2* X, const double2* Y, int n, long long sX, double* out, int nbatch,
                    hipStream_t s, int so, double* last) {
  dim3 grid(min((n * n + 1023) / 1024, 64), nbatch);
  hipLaunchKernelGGL(maxdiff_kernel, grid, dim3(256), 0, s, X, Y, n, sX, out, so); cfqmc_post_launch("maxdiff_kernel");
  hipLaunchKernelGGL(maxdiff_fold_kernel, dim3((nbatch + 63) / 64), dim3(64), 0, s, out, nbatch, so, last);
  cfqmc_post_launch("maxdiff_fold_kernel");
}

__global__ void precision_guard_kernel(const double* last, int* sel, int* count, double* gmax_run, double gmax,
                                       double err, int nbatch) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= nbatch) return;
  const double d = last[2 * z], gm = last[2 * z + 1];
  // the block that just ended ran (at least from some slice on) in FP64
  count[z] += sel[z];
  // a non-finite state (inf) selects FP64 as well
  sel[z] = (gm > gmax || d > err) ? 1 : 0;
  gmax_run[z] = fmax(gmax_run[z], gm);
}

void launch_precision_guard(const double* last, int* sel, int* count, double* gmax_run, double gmax, double err,
                            int nbatch, hipStream_t s) {
  hipLaunchKernelGGL(precision_guard_kernel, dim3((nbatch + 63) / 64), dim3(64), 0, s, last, sel, count, gmax_run,
                     gmax, err, nbatch);
  cfqmc_post_launch("precision_guard_kernel");
}

// ------------------------------------------------------------------ UDT helpers

__global__ void colnorm_sort_kernel(const double2* Wall, int n, long long sW, double* nrm_all, int* perm_all) {
  extern __shared__ double nr[];
  const int z = blockIdx.x;
  const double2* W = Wall + z * sW;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += cabs2(W[(long long)i * n + c]);
    nr[c] = sqrt(s);
    nrm_all[z * n + c] = nr[c];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    int rank = 0;
    const double v = nr[c];
    for (int c2 = 0; c2 < n; ++c2) rank += (nr[c2] > v) || (nr[c2] == v && c2 < c);
    perm_all[z * n + rank] = c;
  }
}
void launch_colnorm_sort(const double2* W, int n, long long sW, double* nrm, int* perm, int nbatch, hipStream_t s) {
  hipLaunchKernelGGL(colnorm_sort_kernel, dim3(nbatch), dim3(256), n * sizeof(double), s, W, n, sW, nrm, perm); cfqmc_post_launch("colnorm_sort_kernel");
}

__global__ void permute_normalize_kernel(const double2* W, int n, long long sW, const double* nrm, const int* perm,
                                         double2* A) {
  const int z = blockIdx.y;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * n; idx += gridDim.x * blockDim.x) {
    const int i = idx / n, k = idx % n;
    const int c = perm[z * n + k];
    A[z * sW + idx] = cscale(W[z * sW + (long long)i * n + c], 1.0 / nrm[z * n + c]);
  }
}
void launch_permute_normalize(const double2* W, int n, long long sW, const double* nrm, const int* perm, double2* A,
                              int nbatch, hipStream_t s) {
  dim3 grid(min((n * n + 255) / 256, 1024), nbatch);
  hipLaunchKernelGGL(permute_normalize_kernel, grid, dim3(256), 0, s, W, n, sW, nrm, perm, A); cfqmc_post_launch("permute_normalize_kernel");
}

__global__ void chol_from_lu_kernel(const double2* LU, int n, long long sLU, double2* R, double* sqrtd, int* err) {
  const int z = blockIdx.y;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * n; idx += gridDim.x * blockDim.x) {
    const int i = idx / n, j = idx % n;
    const double u = LU[z * sLU + (long long)i * n + i].x;
    // a Gram pivot that is not positive and finite: the Cholesky-QR broke down
    if (j == i && err && !(u > 0.0 && u <= 1.7976931348623157e308)) atomicOr(err, 2);
    const double sq = sqrt(u);
    R[z * sLU + idx] = j >= i ? cscale(LU[z * sLU + idx], 1.0 / sq) : make_double2(0.0, 0.0);
    if (j == i) sqrtd[z * n + i] = sq;
  }
}
void launch_chol_from_lu(const double2* LU, int n, long long sLU, double2* R, double* sqrtd, int nbatch,
                         hipStream_t s, int* err) {
  dim3 grid(min((n * n + 255) / 256, 1024), nbatch);
  hipLaunchKernelGGL(chol_from_lu_kernel, grid, dim3(256), 0, s, LU, n, sLU, R, sqrtd, err); cfqmc_post_launch("chol_from_lu_kernel");
}

__global__ void udt_finish_kernel(const double2* Rt, int n, long long sR, const double* nrm, const int* perm,
                                  double* Dout, long long sD, double2* Tp) {
  const int z = blockIdx.y;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * n; idx += gridDim.x * blockDim.x) {
    const int i = idx / n, k = idx % n;
    const double di = sqrt(cabs2(Rt[z * sR + (long long)i * n + i])) * nrm[z * n + perm[z * n + i]];
    const int c = perm[z * n + k];
    double2 v = make_double2(0.0, 0.0);
    if (k >= i) v = cscale(Rt[z * sR + (long long)i * n + k], nrm[z * n + c] / di);
    Tp[z * sR + (long long)i * n + c] = v;
    if (k == i) Dout[z * sD + i] = di;
  }
}
void launch_udt_finish(const double2* Rt, int n, long long sR, const double* nrm, const int* perm, double* Dout,
                       long long sD, double2* Tp, int nbatch, hipStream_t s) {
  dim3 grid(min((n * n + 255) / 256, 1024), nbatch);
  hipLaunchKernelGGL(udt_finish_kernel, grid, dim3(256), 0, s, Rt, n, sR, nrm, perm, Dout, sD, Tp); cfqmc_post_launch("udt_finish_kernel");
}

__global__ void loh_combine_kernel(const double2* K, const double2* Mm, const double* Dl, long long sDl,
                                   const double* Dr, long long sDr, double2* Y, int n) {
  const int z = blockIdx.y;
  const long long off = (long long)z * n * n;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * n; idx += gridDim.x * blockDim.x) {
    const int i = idx / n, j = idx % n;
    const double dl = Dl[z * sDl + i], dr = Dr[z * sDr + j];
    const double lmax = fmax(dl, 1.0), lmin = fmin(dl, 1.0), rmax = fmax(dr, 1.0), rmin = fmin(dr, 1.0);
    Y[off + idx] = cadd(cscale(K[off + idx], 1.0 / (lmax * rmax)), cscale(Mm[off + idx], lmin * rmin));
  }
}
void launch_loh_combine(const double2* K, const double2* Mm, const double* Dl, long long sDl, const double* Dr,
                        long long sDr, double2* Y, int n, int nbatch, hipStream_t s) {
  dim3 grid(min((n * n + 255) / 256, 1024), nbatch);
  hipLaunchKernelGGL(loh_combine_kernel, grid, dim3(256), 0, s, K, Mm, Dl, sDl, Dr, sDr, Y, n); cfqmc_post_launch("loh_combine_kernel");
}

__global__ void dmax_inv_kernel(const double* d, long long sd, double* out, int n) {
  const int z = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += blockDim.x) out[z * n + i] = 1.0 / fmax(d[z * sd + i], 1.0);
}
void launch_dmax_inv(const double* d, long long sd, double* out, int n, int nbatch, hipStream_t s) {
  hipLaunchKernelGGL(dmax_inv_kernel, dim3(nbatch), dim3(256), 0, s, d, sd, out, n); cfqmc_post_launch("dmax_inv_kernel");
}

__global__ void sum_log_dmax_kernel(const double* d, long long sd, int n, double* out) {
  __shared__ double red[4];
  const int z = blockIdx.x;
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += log(fmax(d[z * sd + i], 1.0));
  v = block_sum<256>(v, red);
  if (threadIdx.x == 0) out[z] = v;
}
void launch_sum_log_dmax(const double* d, long long sd, int n, double* out, int nbatch, hipStream_t s) {
  hipLaunchKernelGGL(sum_log_dmax_kernel, dim3(nbatch), dim3(256), 0, s, d, sd, n, out); cfqmc_post_launch("sum_log_dmax_kernel");
}

int cfqmc_debug_sync() {
  static int v = -1;
  if (v < 0) {
    const char* e = getenv("CFQMC_DEBUG_SYNC");
    v = (e && e[0] == '1') ? 1 : 0;
  }
  return v;
}

void cfqmc_post_launch(const char* name) {
  if (!cfqmc_debug_sync()) return;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    fprintf(stderr, "[cfqmc] kernel %s failed: %s\n", name, hipGetErrorString(e));
    fflush(stderr);
  }
}

__global__ void dmin1_kernel(const double* d, long long sd, double* out, int n) {
  const int z = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += blockDim.x) out[z * n + i] = fmin(d[z * sd + i], 1.0);
}
void launch_dmin1(const double* d, long long sd, double* out, int n, int nbatch, hipStream_t s) {
  hipLaunchKernelGGL(dmin1_kernel, dim3(nbatch), dim3(256), 0, s, d, sd, out, n); cfqmc_post_launch("dmin1_kernel");
}

__global__ void diag_set_kernel(double2* A, int n, long long sA, const double* d, long long sd, double scale) {
  const int z = blockIdx.y;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * n; idx += gridDim.x * blockDim.x) {
    const int i = idx / n, j = idx % n;
    A[z * sA + idx] = make_double2(i == j ? scale * d[z * sd + i] : 0.0, 0.0);
  }
}
void launch_diag_set(double2* A, int n, long long sA, const double* d, long long sd, double scale, int nbatch,
                     hipStream_t s) {
  dim3 grid(min((n * n + 255) / 256, 1024), nbatch);
  hipLaunchKernelGGL(diag_set_kernel, grid, dim3(256), 0, s, A, n, sA, d, sd, scale); cfqmc_post_launch("diag_set_kernel");
}
