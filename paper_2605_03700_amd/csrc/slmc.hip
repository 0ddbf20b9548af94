// Kernels of the learned global proposal (self-learning Monte Carlo).
//
// The effective action is S_eff(phi) = |phi|^2 / 2 + S_NN(phi) with S_NN a
// three-layer perceptron on translation-invariant features of the fields:
//   periodogram  P^i_c(w) = |sum_tau phi^i_{tau,c} e^{-2 pi i w tau / L}|^2 / L,
//                w = 0..L/2, averaged over bins of (channel, |q|^2 shell, w range),
//   mean         sum_tau phi^i_{tau,0} / sqrt(L) of the q = 0 component.
// Features are computed in FP32 by direct summation (one workgroup per
// channel and 16 components, the L x 16 field panel in LDS); the network runs
// on BF16 MFMA (16x16x16, FP32 accumulation) with every product operand in
// BF16 (round to nearest even) and FP32 biases, activations and gradients.
// All reductions have a fixed order, so S_NN is a deterministic function of
// phi: the inner HMC chain and the outer test see the same action.
#include <cmath>
#include <cstdio>

#include "common.h"
#include "kernels.h"

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

CF_DEV uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
CF_DEV float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

CF_DEV float wave_sum_f(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
CF_DEV double wave_sum_d(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

static bool lds_ok(const void* fn, size_t shm) {
  if (shm <= 48 * 1024) return true;
  const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  (void)hipGetLastError();
  return e == hipSuccess;
}

// ------------------------------------------------------------------ periodogram
// grid (ceil(nq/16), 4, nb), 256 threads = 16 components x 16 frequency lanes.
__global__ void __launch_bounds__(256) slmc_dft_kernel(const double* phi, long long sphi, int L, int nq, int nw,
                                                       const float* twc, const float* tws, float* Xre, float* Xim,
                                                       long long sX) {
  extern __shared__ float sh[];
  float* ph = sh;              // [L][16]
  float* cs = sh + L * 16;     // cos(2 pi k / L)
  float* sn = cs + L;          // sin(2 pi k / L)
  const int b = blockIdx.z, i = blockIdx.y, c0 = blockIdx.x * 16, tid = threadIdx.x;
  const double* P = phi + b * sphi;
  for (int e = tid; e < L * 16; e += 256) {
    const int t = e >> 4, cl = e & 15;
    ph[e] = c0 + cl < nq ? (float)P[(long long)t * 4 * nq + i * nq + c0 + cl] : 0.f;
  }
  for (int e = tid; e < L; e += 256) { cs[e] = twc[e]; sn[e] = tws[e]; }
  __syncthreads();
  const int cl = tid & 15, wl = tid >> 4, c = c0 + cl;
  for (int w = wl; w < nw; w += 16) {
    float re = 0.f, im = 0.f;
    int k = 0;
    for (int t = 0; t < L; ++t) {
      const float v = ph[t * 16 + cl];
      re += v * cs[k];
      im -= v * sn[k];
      k += w;
      if (k >= L) k -= L;
    }
    if (c < nq) {
      const long long o = b * sX + ((long long)i * nq + c) * nw + w;
      Xre[o] = re;
      Xim[o] = im;
    }
  }
}

void launch_slmc_dft(const double* phi, long long sphi, int L, int nq, int nw, const float* twc, const float* tws,
                     float* Xre, float* Xim, long long sX, int nb, hipStream_t s) {
  const size_t shm = (size_t)(16 * L + 2 * L) * sizeof(float);
  if (!lds_ok((const void*)slmc_dft_kernel, shm)) fprintf(stderr, "[cfqmc] SLMC: %zu B of LDS refused\n", shm);
  hipLaunchKernelGGL(slmc_dft_kernel, dim3((nq + 15) / 16, 4, nb), dim3(256), shm, s, phi, sphi, L, nq, nw, twc, tws,
                     Xre, Xim, sX); cfqmc_post_launch("slmc_dft_kernel");
}

// One wave per (feature, batch entry): bin average of the periodogram (members
// c in the shell's component list, w in the bin's range), or the q = 0 mean.
__global__ void __launch_bounds__(64) slmc_bin_kernel(const float* Xre, const float* Xim, long long sX, int nq, int nw,
                                                      int L, int nqb, int nwb, const int* shell_off,
                                                      const int* shell_comp, const int* w_off, float* feat, int F) {
  const int b = blockIdx.y, f = blockIdx.x, lane = threadIdx.x;
  float r;
  if (f < 4 * nqb * nwb) {
    const int i = f / (nqb * nwb), sb = (f / nwb) % nqb, wb = f % nwb;
    const int c_lo = shell_off[sb], nc = shell_off[sb + 1] - c_lo;
    const int w_lo = w_off[wb], nwr = w_off[wb + 1] - w_lo;
    const int cnt = nc * nwr;
    float acc = 0.f;
    for (int e = lane; e < cnt; e += 64) {
      const int c = shell_comp[c_lo + e / nwr], w = w_lo + e % nwr;
      const long long o = b * sX + ((long long)i * nq + c) * nw + w;
      acc += Xre[o] * Xre[o] + Xim[o] * Xim[o];
    }
    acc = wave_sum_f(acc);
    r = cnt > 0 ? acc / (float)L / (float)cnt : 0.f;
  } else {
    const int i = f - 4 * nqb * nwb;
    r = Xre[b * sX + (long long)i * nq * nw] / sqrtf((float)L);
  }
  if (lane == 0) feat[(long long)b * F + f] = r;
}

void launch_slmc_bin(const float* Xre, const float* Xim, long long sX, int nq, int nw, int L, int nqb, int nwb,
                     const int* shell_off, const int* shell_comp, const int* w_off, float* feat, int F, int nb,
                     hipStream_t s) {
  hipLaunchKernelGGL(slmc_bin_kernel, dim3(F, nb), dim3(64), 0, s, Xre, Xim, sX, nq, nw, L, nqb, nwb, shell_off,
                     shell_comp, w_off, feat, F); cfqmc_post_launch("slmc_bin_kernel");
}

// x = (f - mu) / sigma in BF16, zero padded to Fp columns.
__global__ void slmc_standardize_kernel(const float* feat, int F, int Fp, const float* mu, const float* sig,
                                        uint16_t* xb, int nb) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nb * Fp) return;
  const int b = (int)(e / Fp), j = (int)(e % Fp);
  xb[e] = j < F ? f2bf((feat[(long long)b * F + j] - mu[j]) / sig[j]) : (uint16_t)0;
}

void launch_slmc_standardize(const float* feat, int F, int Fp, const float* mu, const float* sig, uint16_t* xb,
                             int nb, hipStream_t s) {
  const long long n = (long long)nb * Fp;
  if (n == 0) return;
  hipLaunchKernelGGL(slmc_standardize_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, feat, F, Fp, mu, sig,
                     xb, nb); cfqmc_post_launch("slmc_standardize_kernel");
}

// ------------------------------------------------------------------ BF16 GEMM
// C[M][N] = sum_k A(m, k) B(k, n) (+ bias[n], optional tanh), FP32 accumulation.
// A(m, k) = A[m * lda + k] (AT = false) or A[k * lda + m] (AT = true);
// B(k, n) = B[n * ldb + k] (BT = false) or B[k * ldb + n] (BT = true).
// 64 x 64 tile per workgroup, four waves of 32 x 32, K slabs of 32 in LDS as
// [row][k] so each lane reads its eight consecutive k values in one load.
#define SG_BK 32
#define SG_LD (SG_BK + 8)
template <bool AT, bool BT>
__global__ void __launch_bounds__(256) slmc_gemm_kernel(int M, int N, int K, const uint16_t* A, int lda,
                                                        const uint16_t* B, int ldb, float* C, int ldc,
                                                        const float* bias, int act, uint16_t* Cb, int ldcb) {
  __shared__ __align__(16) uint16_t As[64 * SG_LD];
  __shared__ __align__(16) uint16_t Bs[64 * SG_LD];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = (wid >> 1) * 32, wn = (wid & 1) * 32;
  f4v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += SG_BK) {
    for (int e = tid; e < 64 * SG_BK; e += 256) {
      int r, k;
      if (AT) { r = e & 63; k = e >> 6; } else { k = e % SG_BK; r = e / SG_BK; }
      const int gm = m0 + r, gk = k0 + k;
      uint16_t v = 0;
      if (gm < M && gk < K) v = AT ? A[(long long)gk * lda + gm] : A[(long long)gm * lda + gk];
      As[r * SG_LD + k] = v;
    }
    for (int e = tid; e < 64 * SG_BK; e += 256) {
      int r, k;
      if (BT) { r = e & 63; k = e >> 6; } else { k = e % SG_BK; r = e / SG_BK; }
      const int gn = n0 + r, gk = k0 + k;
      uint16_t v = 0;
      if (gn < N && gk < K) v = BT ? B[(long long)gk * ldb + gn] : B[(long long)gn * ldb + gk];
      Bs[r * SG_LD + k] = v;
    }
    __syncthreads();
    // gfx950 BF16 MFMA 16x16x32: lane l supplies A[l % 16][8 (l / 16) + 0..7] and
    // B[8 (l / 16) + 0..7][l % 16] (16-byte LDS reads: rows are 80 B apart)
#pragma unroll
    for (int kk = 0; kk < SG_BK; kk += 32) {
      bf8v a[2], b[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const uint16_t* pa = As + (wm + s * 16 + (lane & 15)) * SG_LD + kk + 8 * (lane >> 4);
        const uint16_t* pb = Bs + (wn + s * 16 + (lane & 15)) * SG_LD + kk + 8 * (lane >> 4);
        a[s] = *(const bf8v*)pa;
        b[s] = *(const bf8v*)pb;
      }
#pragma unroll
      for (int si = 0; si < 2; ++si)
#pragma unroll
        for (int sj = 0; sj < 2; ++sj)
          acc[si][sj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[si], b[sj], acc[si][sj], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int si = 0; si < 2; ++si)
#pragma unroll
    for (int sj = 0; sj < 2; ++sj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + si * 16 + 4 * (lane >> 4) + r;
        const int n = n0 + wn + sj * 16 + (lane & 15);
        if (m >= M || n >= N) continue;
        float v = acc[si][sj][r];
        if (bias) v += bias[n];
        if (act) v = tanhf(v);
        if (C) C[(long long)m * ldc + n] = v;
        if (Cb) Cb[(long long)m * ldcb + n] = f2bf(v);
      }
}

void launch_slmc_gemm(int at, int bt, int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb,
                      float* C, int ldc, const float* bias, int act, uint16_t* Cb, int ldcb, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  const dim3 grid((N + 63) / 64, (M + 63) / 64);
  if (!at && !bt)
    hipLaunchKernelGGL((slmc_gemm_kernel<false, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias,
                       act, Cb, ldcb);
  else if (!at && bt)
    hipLaunchKernelGGL((slmc_gemm_kernel<false, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias,
                       act, Cb, ldcb);
  else if (at && bt)
    hipLaunchKernelGGL((slmc_gemm_kernel<true, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias,
                       act, Cb, ldcb);
  else
    hipLaunchKernelGGL((slmc_gemm_kernel<true, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, bias,
                       act, Cb, ldcb);
  cfqmc_post_launch("slmc_gemm_kernel");
}

// ------------------------------------------------------------------ head, loss, deltas
// out[b] = sum_h a2b[b][h] w3b[h] + b3 (one wave per b).
__global__ void __launch_bounds__(64) slmc_head_kernel(const uint16_t* a2b, int H, const uint16_t* w3b, const float* b3,
                                                       float* out) {
  const int b = blockIdx.x, lane = threadIdx.x;
  float acc = 0.f;
  for (int h = lane; h < H; h += 64) acc += bf2f(a2b[(long long)b * H + h]) * bf2f(w3b[h]);
  acc = wave_sum_f(acc);
  if (lane == 0) out[b] = acc + b3[0];
}

void launch_slmc_head(const uint16_t* a2b, int H, const uint16_t* w3b, const float* b3, float* out, int nb,
                      hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(slmc_head_kernel, dim3(nb), dim3(64), 0, s, a2b, H, w3b, b3, out); cfqmc_post_launch("slmc_head_kernel");
}

// dout[b]: mode 0 -> 2 (out - y) / nb and loss_acc += sum (out - y)^2 / nb;
// mode 1 -> const_d (gradient of const_d * out). One workgroup.
__global__ void __launch_bounds__(256) slmc_dout_kernel(const float* out, const float* y, int nb, int mode,
                                                        float const_d, float* dout, double* loss_acc) {
  __shared__ double red[4];
  double part = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    if (mode == 0) {
      const float r = out[b] - y[b];
      dout[b] = 2.f * r / (float)nb;
      part += (double)r * (double)r;
    } else {
      dout[b] = const_d;
    }
  }
  if (mode == 0) {
    const double t = block_sum<256>(part, red);
    if (threadIdx.x == 0 && loss_acc) *loss_acc += t / nb;
  }
}

void launch_slmc_dout(const float* out, const float* y, int nb, int mode, float const_d, float* dout, double* loss_acc,
                      hipStream_t s) {
  hipLaunchKernelGGL(slmc_dout_kernel, dim3(1), dim3(256), 0, s, out, y, nb, mode, const_d, dout, loss_acc);
  cfqmc_post_launch("slmc_dout_kernel");
}

// dz2[b][h] = dout[b] w3b[h] (1 - a2^2) (FP32 and BF16 copies); thread per (b, h).
__global__ void slmc_dz2_kernel(const float* dout, const uint16_t* w3b, const float* a2, int H, float* dz2,
                                uint16_t* dz2b, int nb) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nb * H) return;
  const int b = (int)(e / H), h = (int)(e % H);
  const float a = a2[e];
  const float v = dout[b] * bf2f(w3b[h]) * (1.f - a * a);
  dz2[e] = v;
  dz2b[e] = f2bf(v);
}

// dz[b][h] = dA[b][h] (1 - a^2)
__global__ void slmc_tanh_bwd_kernel(const float* dA, const float* a, long long n, float* dz, uint16_t* dzb) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float v = dA[e] * (1.f - a[e] * a[e]);
  dz[e] = v;
  dzb[e] = f2bf(v);
}

// Column sums over the batch: out[h] = sum_b X[b][h] (bias gradients), and
// for the head: gw3[h] = sum_b dout[b] a2b[b][h], gb3 = sum_b dout[b].
__global__ void slmc_colsum_kernel(const float* X, int nb, int H, float* out) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= H) return;
  float acc = 0.f;
  for (int b = 0; b < nb; ++b) acc += X[(long long)b * H + h];
  out[h] = acc;
}
__global__ void slmc_head_grad_kernel(const float* dout, const uint16_t* a2b, int nb, int H, float* gw3, float* gb3) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h < H) {
    float acc = 0.f;
    for (int b = 0; b < nb; ++b) acc += dout[b] * bf2f(a2b[(long long)b * H + h]);
    gw3[h] = acc;
  }
  if (h == 0) {
    float acc = 0.f;
    for (int b = 0; b < nb; ++b) acc += dout[b];
    gb3[0] = acc;
  }
}

void launch_slmc_dz2(const float* dout, const uint16_t* w3b, const float* a2, int H, float* dz2, uint16_t* dz2b, int nb,
                     hipStream_t s) {
  const long long n = (long long)nb * H;
  hipLaunchKernelGGL(slmc_dz2_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dout, w3b, a2, H, dz2, dz2b,
                     nb); cfqmc_post_launch("slmc_dz2_kernel");
}
void launch_slmc_tanh_bwd(const float* dA, const float* a, long long n, float* dz, uint16_t* dzb, hipStream_t s) {
  hipLaunchKernelGGL(slmc_tanh_bwd_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dA, a, n, dz, dzb);
  cfqmc_post_launch("slmc_tanh_bwd_kernel");
}
void launch_slmc_colsum(const float* X, int nb, int H, float* out, hipStream_t s) {
  hipLaunchKernelGGL(slmc_colsum_kernel, dim3((H + 255) / 256), dim3(256), 0, s, X, nb, H, out);
  cfqmc_post_launch("slmc_colsum_kernel");
}
void launch_slmc_head_grad(const float* dout, const uint16_t* a2b, int nb, int H, float* gw3, float* gb3,
                           hipStream_t s) {
  hipLaunchKernelGGL(slmc_head_grad_kernel, dim3((H + 255) / 256), dim3(256), 0, s, dout, a2b, nb, H, gw3, gb3);
  cfqmc_post_launch("slmc_head_grad_kernel");
}

// ------------------------------------------------------------------ optimiser
// Adam (Kingma and Ba) on the FP32 master parameters, t = step number >= 1.
__global__ void slmc_adam_kernel(float* p, const float* g, float* m, float* v, long long n, float lr, float b1,
                                 float b2, float eps, float c1, float c2) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.f - b1) * gg;
  const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

void launch_slmc_adam(float* p, const float* g, float* m, float* v, long long n, double lr, int t, hipStream_t s) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - std::pow(b1, t)), c2 = (float)(1.0 - std::pow(b2, t));
  hipLaunchKernelGGL(slmc_adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, (float)lr,
                     (float)b1, (float)b2, 1e-8f, c1, c2); cfqmc_post_launch("slmc_adam_kernel");
}

// BF16 copy of rows x cols of src (ld cols) into dst (ld ldd, zero padding).
__global__ void slmc_to_bf16_kernel(const float* src, int rows, int cols, uint16_t* dst, int ldd) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)rows * ldd) return;
  const int r = (int)(e / ldd), k = (int)(e % ldd);
  dst[e] = k < cols ? f2bf(src[(long long)r * cols + k]) : (uint16_t)0;
}

void launch_slmc_to_bf16(const float* src, int rows, int cols, uint16_t* dst, int ldd, hipStream_t s) {
  const long long n = (long long)rows * ldd;
  hipLaunchKernelGGL(slmc_to_bf16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, rows, cols, dst, ldd);
  cfqmc_post_launch("slmc_to_bf16_kernel");
}

// Row gather of BF16 inputs and FP32 targets for a minibatch.
__global__ void slmc_gather_kernel(const uint16_t* xall, const float* yall, int Fp, const int* idx, int nb,
                                   uint16_t* xb, float* yb) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nb * Fp) return;
  const int b = (int)(e / Fp), j = (int)(e % Fp);
  const int r = idx[b];
  xb[e] = xall[(long long)r * Fp + j];
  if (j == 0) yb[b] = yall[r];
}

void launch_slmc_gather(const uint16_t* xall, const float* yall, int Fp, const int* idx, int nb, uint16_t* xb, float* yb,
                        hipStream_t s) {
  const long long n = (long long)nb * Fp;
  hipLaunchKernelGGL(slmc_gather_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xall, yall, Fp, idx, nb,
                     xb, yb); cfqmc_post_launch("slmc_gather_kernel");
}

// ------------------------------------------------------------------ gradient to the fields
// gf[b][j] = scale * dX[b][j] / sigma[j]: cotangent of the raw features.
__global__ void slmc_dx_to_gf_kernel(const float* dX, int Fp, const float* sig, int F, float scale, float* gf, int nb) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nb * F) return;
  const int b = (int)(e / F), j = (int)(e % F);
  gf[e] = scale * dX[(long long)b * Fp + j] / sig[j];
}

void launch_slmc_dx_to_gf(const float* dX, int Fp, const float* sig, int F, float scale, float* gf, int nb,
                          hipStream_t s) {
  const long long n = (long long)nb * F;
  hipLaunchKernelGGL(slmc_dx_to_gf_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dX, Fp, sig, F, scale, gf,
                     nb); cfqmc_post_launch("slmc_dx_to_gf_kernel");
}

// d(gf . f)/d phi^i_{tau,c} = (2/L) sum_w gamma^i_c(w) [Xr cos - Xi sin](2 pi w tau / L)
//                            + delta_{c0} gf_lin[i] / sqrt(L),
// gamma^i_c(w) = gf[i][s(c)][bin(w)] / count. grid (ceil(nq/16), 4, nb), 256
// threads = 16 components x 16 slice lanes; writes grad in FP64 [b][L][4][nq].
__global__ void __launch_bounds__(256) slmc_vjp_kernel(const float* Xre, const float* Xim, long long sX, const float* gf,
                                                       int F, int nq, int nw, int L, int nqb, int nwb, const int* shell,
                                                       const int* wbin, const float* inv_cnt, const float* twc,
                                                       const float* tws, double* grad, long long sg) {
  extern __shared__ float sh[];
  float* Ar = sh;               // [16][nw]
  float* Ai = sh + 16 * nw;     // [16][nw]
  float* cs = Ai + 16 * nw;     // [L]
  float* sn = cs + L;
  const int b = blockIdx.z, i = blockIdx.y, c0 = blockIdx.x * 16, tid = threadIdx.x;
  const float* g = gf + (long long)b * F;
  const float two_l = 2.f / (float)L;
  for (int e = tid; e < 16 * nw; e += 256) {
    const int cl = e / nw, w = e % nw, c = c0 + cl;
    float ar = 0.f, ai = 0.f;
    if (c < nq) {
      const int bin = shell[c] * nwb + wbin[w];
      const float gm = g[i * nqb * nwb + bin] * inv_cnt[bin] * two_l;
      const long long o = b * sX + ((long long)i * nq + c) * nw + w;
      ar = gm * Xre[o];
      ai = gm * Xim[o];
    }
    Ar[e] = ar;
    Ai[e] = ai;
  }
  for (int e = tid; e < L; e += 256) { cs[e] = twc[e]; sn[e] = tws[e]; }
  __syncthreads();
  const int cl = tid & 15, tl = tid >> 4, c = c0 + cl;
  if (c >= nq) return;
  const float lin = c == 0 ? g[4 * nqb * nwb + i] / sqrtf((float)L) : 0.f;
  for (int t = tl; t < L; t += 16) {
    float acc = 0.f;
    int k = 0;
    for (int w = 0; w < nw; ++w) {
      acc += Ar[cl * nw + w] * cs[k] - Ai[cl * nw + w] * sn[k];
      k += t;
      if (k >= L) k -= L;
    }
    grad[b * sg + (long long)t * 4 * nq + i * nq + c] = (double)(acc + lin);
  }
}

void launch_slmc_vjp(const float* Xre, const float* Xim, long long sX, const float* gf, int F, int nq, int nw, int L,
                     int nqb, int nwb, const int* shell, const int* wbin, const float* inv_cnt, const float* twc,
                     const float* tws, double* grad, long long sg, int nb, hipStream_t s) {
  const size_t shm = (size_t)(32 * nw + 2 * L) * sizeof(float);
  if (!lds_ok((const void*)slmc_vjp_kernel, shm)) fprintf(stderr, "[cfqmc] SLMC: %zu B of LDS refused\n", shm);
  hipLaunchKernelGGL(slmc_vjp_kernel, dim3((nq + 15) / 16, 4, nb), dim3(256), shm, s, Xre, Xim, sX, gf, F, nq, nw, L,
                     nqb, nwb, shell, wbin, inv_cnt, twc, tws, grad, sg); cfqmc_post_launch("slmc_vjp_kernel");
}

// ------------------------------------------------------------------ HMC
// Momenta: replay [b][n] or N(0,1) from Philox (own key), counter per trajectory.
// Subspace (mode, nq): 0 every coordinate; 1 only component 0 (q = 0) of every
// channel and slice; 2 the four slice-uniform q = 0 amplitudes
// A_i = sum_tau phi^i_{tau,0} / sqrt(L), whose momenta sit at slice 0.
__global__ void slmc_momenta_kernel(double* p, long long n, int nb, uint64_t key, long long counter,
                                    const double* replay, long long s_replay, int mode, int nq) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nb * n) return;
  const int b = (int)(e / n);
  const long long j = e % n;
  const double v = replay ? replay[b * s_replay + j] : rng_normal(key, b, counter, (int)j);
  const bool keep = mode == 0 || (j % nq == 0 && (mode == 1 || j < 4LL * nq));
  p[e] = keep ? v : 0.0;
}
// p <- p - h (phi + g)   (gradient of S_eff = |phi|^2/2 + S_NN), on the moving
// coordinates only (modes 0 and 1 above; the field length per chain is a
// multiple of nq)
__global__ void slmc_kick_kernel(double* p, const double* phi, const double* g, double h, long long n, int mode,
                                 int nq) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  if (mode == 1 && e % nq != 0) return;
  p[e] -= h * (phi[e] + g[e]);
}
// Mode 2: p_i <- p_i - h sum_tau (phi + g)^i_{tau,0} / sqrt(L), one workgroup
// per (chain, channel), fixed summation order
__global__ void __launch_bounds__(256) slmc_kick_uniform_kernel(double* p, const double* phi, const double* g,
                                                                double h, int L, int nq) {
  __shared__ double red[4];
  const int z = blockIdx.x / 4, i = blockIdx.x % 4;
  const long long base = (long long)z * L * 4 * nq + (long long)i * nq;
  double acc = 0.0;
  for (int t = threadIdx.x; t < L; t += 256) {
    const long long e = base + (long long)t * 4 * nq;
    acc += phi[e] + g[e];
  }
  const double sum = block_sum<256>(acc, red);
  if (threadIdx.x == 0) p[base] -= h * sum / sqrt((double)L);
}
// Mode 2: phi^i_{tau,0} <- phi^i_{tau,0} + h p_i / sqrt(L) for every tau
__global__ void slmc_drift_uniform_kernel(double* phi, const double* p, double h, int L, int nq, int nb) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nb * L * 4) return;
  const int z = (int)(e / (4LL * L)), r = (int)(e % (4LL * L)), t = r / 4, i = r % 4;
  const long long chain = (long long)z * L * 4 * nq;
  phi[chain + (long long)t * 4 * nq + (long long)i * nq] += h * p[chain + (long long)i * nq] / sqrt((double)L);
}
// phi <- phi + h p
__global__ void slmc_drift_kernel(double* phi, const double* p, double h, long long n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  phi[e] += h * p[e];
}
// out[b] = sum_j x[b][j]^2 (one workgroup per b, fixed order)
__global__ void __launch_bounds__(256) slmc_sumsq_kernel(const double* x, long long n, double* out) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  double acc = 0.0;
  for (long long j = threadIdx.x; j < n; j += 256) {
    const double v = x[b * n + j];
    acc += v * v;
  }
  const double t = block_sum<256>(acc, red);
  if (threadIdx.x == 0) out[b] = t;
}
// dst[b] = src[b] where flag[b] == want
__global__ void slmc_select_kernel(const int* flag, int want, const double* src, double* dst, long long n, int nb) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nb * n) return;
  if (flag[e / n] == want) dst[e] = src[e];
}

void launch_slmc_momenta(double* p, long long n, int nb, uint64_t key, long long counter, const double* replay,
                         long long s_replay, int mode, int nq, hipStream_t s) {
  const long long t = (long long)nb * n;
  hipLaunchKernelGGL(slmc_momenta_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, p, n, nb, key, counter,
                     replay, s_replay, mode, nq); cfqmc_post_launch("slmc_momenta_kernel");
}
void launch_slmc_kick(double* p, const double* phi, const double* g, double h, long long n, int mode, int nq, int L,
                      int nb, hipStream_t s) {
  if (mode == 2) {
    hipLaunchKernelGGL(slmc_kick_uniform_kernel, dim3(nb * 4), dim3(256), 0, s, p, phi, g, h, L, nq);
    cfqmc_post_launch("slmc_kick_uniform_kernel");
    return;
  }
  hipLaunchKernelGGL(slmc_kick_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, phi, g, h, n, mode, nq);
  cfqmc_post_launch("slmc_kick_kernel");
}
void launch_slmc_drift(double* phi, const double* p, double h, long long n, int mode, int nq, int L, int nb,
                       hipStream_t s) {
  if (mode == 2) {
    const long long t = (long long)nb * L * 4;
    hipLaunchKernelGGL(slmc_drift_uniform_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, phi, p, h, L,
                       nq, nb);
    cfqmc_post_launch("slmc_drift_uniform_kernel");
    return;
  }
  hipLaunchKernelGGL(slmc_drift_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, phi, p, h, n);
  cfqmc_post_launch("slmc_drift_kernel");
}
void launch_slmc_sumsq(const double* x, long long n, double* out, int nb, hipStream_t s) {
  hipLaunchKernelGGL(slmc_sumsq_kernel, dim3(nb), dim3(256), 0, s, x, n, out); cfqmc_post_launch("slmc_sumsq_kernel");
}
void launch_slmc_select(const int* flag, int want, const double* src, double* dst, long long n, int nb, hipStream_t s) {
  const long long t = (long long)nb * n;
  hipLaunchKernelGGL(slmc_select_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, flag, want, src, dst, n,
                     nb); cfqmc_post_launch("slmc_select_kernel");
}
