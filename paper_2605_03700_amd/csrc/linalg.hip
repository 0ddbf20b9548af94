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
#include "common.h"
#include "kernels.h"

#define LU_NB 16
#define LU_NT 512

__global__ void __launch_bounds__(LU_NT) lu_kernel(double2* Aall, int n, int lda, long long sA, int* ipiv_all,
                                                   int sP, double2* logdet, int pivot) {
  extern __shared__ double2 P[];          // panel: rows x LU_NB
  __shared__ double rv[LU_NT / 64];
  __shared__ int ri[LU_NT / 64];
  __shared__ int piv_s;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  double2* A = Aall + blockIdx.x * sA;
  int* ipiv = ipiv_all + blockIdx.x * sP;
  double ld_re = 0.0, ld_im = 0.0;   // accumulated in thread 0
  for (int k0 = 0; k0 < n; k0 += LU_NB) {
    const int nb = min(LU_NB, n - k0), rows = n - k0;
    for (int idx = tid; idx < rows * LU_NB; idx += LU_NT) {
      const int r = idx / LU_NB, c = idx % LU_NB;
      P[idx] = c < nb ? A[(long long)(k0 + r) * lda + k0 + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
      if (pivot) {
        double best = -1.0;
        int bi = j;
        for (int r = j + tid; r < rows; r += LU_NT) {
          const double2 v = P[r * LU_NB + j];
          const double a = fabs(v.x) + fabs(v.y);
          if (a > best) { best = a; bi = r; }
        }
        for (int o = 32; o > 0; o >>= 1) {
          const double ob = __shfl_xor(best, o, 64);
          const int oi = __shfl_xor(bi, o, 64);
          if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if (lane == 0) { rv[wid] = best; ri[wid] = bi; }
        __syncthreads();
        if (tid == 0) {
          double b = rv[0];
          int i = ri[0];
          for (int w = 1; w < LU_NT / 64; ++w)
            if (rv[w] > b || (rv[w] == b && ri[w] < i)) { b = rv[w]; i = ri[w]; }
          piv_s = i;
          ipiv[k0 + j] = k0 + i;
        }
        __syncthreads();
        const int p = piv_s;
        if (p != j && tid < LU_NB) {
          const double2 t = P[j * LU_NB + tid];
          P[j * LU_NB + tid] = P[p * LU_NB + tid];
          P[p * LU_NB + tid] = t;
        }
        if (tid == 0 && p != j) ld_im += M_PI;
      } else if (tid == 0) {
        ipiv[k0 + j] = k0 + j;
      }
      __syncthreads();
      const double2 d = P[j * LU_NB + j];
      if (tid == 0) {
        ld_re += 0.5 * log(cabs2(d));
        ld_im += atan2(d.y, d.x);
      }
      for (int r = j + 1 + tid; r < rows; r += LU_NT) {
        const double2 l = cdiv(P[r * LU_NB + j], d);
        P[r * LU_NB + j] = l;
        for (int c = j + 1; c < nb; ++c) P[r * LU_NB + c] = csub(P[r * LU_NB + c], cmul(l, P[j * LU_NB + c]));
      }
      __syncthreads();
    }
    for (int idx = tid; idx < rows * nb; idx += LU_NT) {
      const int r = idx / nb, c = idx % nb;
      A[(long long)(k0 + r) * lda + k0 + c] = P[r * LU_NB + c];
    }
    // row interchanges outside the panel, then U12 = L11^{-1} A12 (one column per thread)
    for (int col = tid; col < n; col += LU_NT) {
      if (col >= k0 && col < k0 + nb) continue;
      for (int j = 0; j < nb; ++j) {
        const int p = ipiv[k0 + j];
        if (p != k0 + j) {
          const double2 t = A[(long long)(k0 + j) * lda + col];
          A[(long long)(k0 + j) * lda + col] = A[(long long)p * lda + col];
          A[(long long)p * lda + col] = t;
        }
      }
      if (col >= k0 + nb) {
        double2 u[LU_NB];
#pragma unroll
        for (int i = 0; i < LU_NB; ++i) {
          if (i < nb) {
            double2 v = A[(long long)(k0 + i) * lda + col];
            for (int l = 0; l < i; ++l) v = csub(v, cmul(P[i * LU_NB + l], u[l]));
            u[i] = v;
            A[(long long)(k0 + i) * lda + col] = v;
          }
        }
      }
    }
    __syncthreads();
    // trailing update on MFMA: tiles of 16 x 16, K = nb (zero padded to 16)
    const int t0 = k0 + nb, rem = n - t0;
    if (rem > 0) {
      const int nt = (rem + 15) / 16;
      const int il = lane & 15, kl = lane >> 4;
      for (int t = wid; t < nt * nt; t += LU_NT / 64) {
        const int r0 = t0 + (t / nt) * 16, c0 = t0 + (t % nt) * 16;
        d4v cre, cim;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = r0 + Mfma<double>::row(lane, r), j = c0 + il;
          double2 v = make_double2(0.0, 0.0);
          if (i < n && j < n) v = A[(long long)i * lda + j];
          cre[r] = v.x;
          cim[r] = v.y;
        }
#pragma unroll
        for (int kk = 0; kk < LU_NB; kk += 4) {
          const int k = kk + kl;
          const int ar = r0 + il - k0;           // panel row of L21
          double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
          if (k < nb && r0 + il < n) a = P[ar * LU_NB + k];
          if (k < nb && c0 + il < n) b = A[(long long)(k0 + k) * lda + c0 + il];
          cre = Mfma<double>::mma(-a.x, b.x, cre);
          cre = Mfma<double>::mma(a.y, b.y, cre);
          cim = Mfma<double>::mma(-a.x, b.y, cim);
          cim = Mfma<double>::mma(-a.y, b.x, cim);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = r0 + Mfma<double>::row(lane, r), j = c0 + il;
          if (i < n && j < n) A[(long long)i * lda + j] = make_double2(cre[r], cim[r]);
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0 && logdet) {
    double im = fmod(ld_im, 2.0 * M_PI);
    if (im > M_PI) im -= 2.0 * M_PI;
    if (im <= -M_PI) im += 2.0 * M_PI;
    logdet[blockIdx.x] = make_double2(ld_re, im);
  }
}

void launch_lu(double2* A, int n, int lda, long long sA, int* ipiv, int sP, double2* logdet, int pivot,
               int nbatch, hipStream_t s) {
  const size_t shm = (size_t)n * LU_NB * sizeof(double2);
  if (shm > 65536) {
    (void)hipFuncSetAttribute((const void*)lu_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    (void)hipGetLastError();
  }
  hipLaunchKernelGGL(lu_kernel, dim3(nbatch), dim3(LU_NT), shm, s, A, n, lda, sA, ipiv, sP, logdet, pivot); cfqmc_post_launch("lu_kernel");
}

// ------------------------------------------------------------------ right solve
// Y = X A^{-1}, A = P_0..P_{n-1} L U: Y = ((X U^{-1}) L^{-1}) P_{n-1} ... P_0.
// A workgroup owns RS_ROWS rows of X in LDS; columns are eliminated one at a
// time with a right-looking row update (rows of U and L are read contiguously).
#define RS_ROWS 8
#define RS_NT 256

__global__ void __launch_bounds__(RS_NT) rsolve_kernel(const double2* Xall, int ldx, long long sX, double2* Yall,
                                                       int ldy, long long sY, const double2* LUall, int ldlu,
                                                       long long sLU, const int* ipiv_all, int sP, int n,
                                                       int upper_only) {
  extern __shared__ double2 Ys[];          // RS_ROWS x n
  const int z = blockIdx.y;
  const double2* X = Xall + z * sX;
  double2* Yo = Yall + z * sY;
  const double2* LU = LUall + z * sLU;
  const int* ipiv = ipiv_all + z * sP;
  const int r0 = blockIdx.x * RS_ROWS;
  const int nr = min(RS_ROWS, n - r0);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < RS_ROWS * n; idx += RS_NT) {
    const int r = idx / n, c = idx % n;
    Ys[idx] = r < nr ? X[(long long)(r0 + r) * ldx + c] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  // z U = x, columns ascending
  for (int j = 0; j < n; ++j) {
    const double2 d = LU[(long long)j * ldlu + j];
    if (tid < RS_ROWS) Ys[tid * n + j] = cdiv(Ys[tid * n + j], d);
    __syncthreads();
    const int w = n - j - 1;
    for (int idx = tid; idx < RS_ROWS * w; idx += RS_NT) {
      const int r = idx / w, c = j + 1 + idx % w;
      Ys[r * n + c] = csub(Ys[r * n + c], cmul(Ys[r * n + j], LU[(long long)j * ldlu + c]));
    }
    __syncthreads();
  }
  if (!upper_only) {
    // w L = z (unit lower), columns descending
    for (int j = n - 1; j > 0; --j) {
      for (int idx = tid; idx < RS_ROWS * j; idx += RS_NT) {
        const int r = idx / j, c = idx % j;
        Ys[r * n + c] = csub(Ys[r * n + c], cmul(Ys[r * n + j], LU[(long long)j * ldlu + c]));
      }
      __syncthreads();
    }
    if (tid < RS_ROWS) {
      for (int k = n - 1; k >= 0; --k) {
        const int p = ipiv[k];
        if (p != k) {
          const double2 t = Ys[tid * n + k];
          Ys[tid * n + k] = Ys[tid * n + p];
          Ys[tid * n + p] = t;
        }
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < nr * n; idx += RS_NT) {
    const int r = idx / n, c = idx % n;
    Yo[(long long)(r0 + r) * ldy + c] = Ys[r * n + c];
  }
}

void launch_rsolve(const double2* X, int ldx, long long sX, double2* Y, int ldy, long long sY, const double2* LU,
                   int ldlu, long long sLU, const int* ipiv, int sP, int n, int upper_only, int nbatch,
                   hipStream_t s) {
  dim3 grid((n + RS_ROWS - 1) / RS_ROWS, nbatch);
  const size_t shm = (size_t)RS_ROWS * n * sizeof(double2);
  hipLaunchKernelGGL(rsolve_kernel, grid, dim3(RS_NT), shm, s, X, ldx, sX, Y, ldy, sY, LU, ldlu, sLU, ipiv, sP, n,
                     upper_only); cfqmc_post_launch("rsolve_kernel");
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

__global__ void maxdiff_kernel(const double2* X, const double2* Y, int n, long long sX, double* out) {
  __shared__ double red[4];
  const int z = blockIdx.x;
  double m = 0.0;
  for (int idx = threadIdx.x; idx < n * n; idx += 256) {
    const double2 a = X[z * sX + idx], b = Y[z * sX + idx];
    m = fmax(m, sqrt(cabs2(csub(a, b))));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) out[z] = fmax(out[z], fmax(fmax(red[0], red[1]), fmax(red[2], red[3])));
}
void launch_maxdiff(const double2* X, const double2* Y, int n, long long sX, double* out, int nbatch,
                    hipStream_t s) {
  hipLaunchKernelGGL(maxdiff_kernel, dim3(nbatch), dim3(256), 0, s, X, Y, n, sX, out); cfqmc_post_launch("maxdiff_kernel");
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

__global__ void chol_from_lu_kernel(const double2* LU, int n, long long sLU, double2* R, double* sqrtd) {
  const int z = blockIdx.y;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * n; idx += gridDim.x * blockDim.x) {
    const int i = idx / n, j = idx % n;
    const double u = LU[z * sLU + (long long)i * n + i].x;
    const double sq = sqrt(u);
    R[z * sLU + idx] = j >= i ? cscale(LU[z * sLU + idx], 1.0 / sq) : make_double2(0.0, 0.0);
    if (j == i) sqrtd[z * n + i] = sq;
  }
}
void launch_chol_from_lu(const double2* LU, int n, long long sLU, double2* R, double* sqrtd, int nbatch,
                         hipStream_t s) {
  dim3 grid(min((n * n + 255) / 256, 1024), nbatch);
  hipLaunchKernelGGL(chol_from_lu_kernel, grid, dim3(256), 0, s, LU, n, sLU, R, sqrtd); cfqmc_post_launch("chol_from_lu_kernel");
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
