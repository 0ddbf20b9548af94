// Kernel microbenchmark of the sweep's hot kernels at a given shape, for
// per-kernel timing and hardware-counter runs (rocprofv3) outside a sweep.
//
//   kbench <kernel> [n_phi] [chains] [iters] [cfg] [variant] [fp64_percent]
//   kernel: chan32 | chan64   channel application Y = E X (left, tau_y rotation,
//                             the wrap's timed launch), FP32 correction form or FP64
//           chan32r | chan64r the right application X E^-1 (tau_x rotation)
//           chandual          the precision-guarded form of chan32: one launch in
//                             which the chains flagged FP64 (fp64_percent of them,
//                             spread evenly) take the FP64 path; cfg the FP32
//                             configuration (1 or 12), variant 1 or 2 the register
//                             budget (launch_chan_apply_dual)
//           lu_np             LU of M = 1 + small (non-pivoted, in place)
//           lu                the same matrices by the partially pivoted LU
//           rsolve            G' = G M^-1 from that LU
//           rsolve32          the same with FP32 block products (FP64 accumulation)
//           copy              a plain device-to-device copy of 1 GiB (the reference
//                             for scaling the FETCH_SIZE / WRITE_SIZE counters)
//           mfma              the sustained rate of the 16 x 16 x 4 MFMA in FP64 and
//                             FP32 and of the FP64 4 x 4 x 4 four-block MFMA: waves
//                             of six independent accumulator chains and no memory
//                             traffic but one store per lane (the ceiling the
//                             MFMA-bound kernels can approach on this chip)
//
// Inputs are seeded random matrices of the sweep's shapes: M (n x n, n =
// 2 n_phi, entries O(1)), the orbital blocks X = 1 + A with ||A|| ~ 0.3 (the
// channel exponentials of typical fields). Every launch covers all chains, as
// in the sweep. The driver times `iters` launches after half a second of
// warm-up launches, with a device synchronisation on each side (no HIP
// events), and prints the
// mean duration and the launch's algorithmic work: for the channel
// application 2 n^3 real flops per chain (one of the eight applications that
// make up the two n x n x n complex products of the wrap) next to the 4 n^3
// the kernel issues (two N x N x n complex products).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "kernels.h"

namespace {

void fill_random(std::vector<double2>& v, uint64_t seed, double scale) {
  uint64_t s = seed * 0x9E3779B97F4A7C15ull + 1;
  for (auto& x : v) {
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    const double a = ((s >> 11) * (1.0 / 9007199254740992.0)) - 0.5;
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    const double b = ((s >> 11) * (1.0 / 9007199254740992.0)) - 0.5;
    x = make_double2(scale * a, scale * b);
  }
}

#define CK(x)                                                                      \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess) {                                                        \
      std::fprintf(stderr, "kbench: %s at %s\n", hipGetErrorString(e_), #x);     \
      std::exit(1);                                                                \
    }                                                                              \
  } while (0)

double2* upload(const std::vector<double2>& h) {
  double2* d = nullptr;
  CK(hipMalloc(&d, h.size() * sizeof(double2)));
  CK(hipMemcpy(d, h.data(), h.size() * sizeof(double2), hipMemcpyHostToDevice));
  return d;
}

// Six independent accumulator chains per wave, `iters` rounds; the operands
// stay in registers. One store per lane keeps the chains live.
typedef double mf64x4 __attribute__((ext_vector_type(4)));
typedef float mf32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) mfma_rate64(double* out, int iters, double x) {
  mf64x4 acc[6];
  for (int i = 0; i < 6; ++i) acc[i] = mf64x4{0.0, 0.0, 0.0, 0.0};
  const double a = x + threadIdx.x * 1e-9, b = x - threadIdx.x * 1e-9;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
  }
  double s = 0.0;
  for (int i = 0; i < 6; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ void __launch_bounds__(256) mfma_rate64q(double* out, int iters, double x) {
  double acc[6];
  for (int i = 0; i < 6; ++i) acc[i] = 0.0;
  const double a = x + threadIdx.x * 1e-9, b = x - threadIdx.x * 1e-9;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[i] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, acc[i], 0, 0, 0);
  }
  double s = 0.0;
  for (int i = 0; i < 6; ++i) s += acc[i];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}
__global__ void __launch_bounds__(256) mfma_rate32(float* out, int iters, float x) {
  mf32x4 acc[6];
  for (int i = 0; i < 6; ++i) acc[i] = mf32x4{0.0f, 0.0f, 0.0f, 0.0f};
  const float a = x + threadIdx.x * 1e-6f, b = x - threadIdx.x * 1e-6f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i], 0, 0, 0);
  }
  float s = 0.0f;
  for (int i = 0; i < 6; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

// 4 and 8 four-wave workgroups per CU (4 and 8 waves per SIMD): FP64 16x16x4,
// FP32 16x16x4, FP64 4x4x4 (four blocks); five timed launches each between HIP
// events after one untimed launch.
int mfma_rates() {
  int cus = 0;
  CK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
  const int iters = 4000, maxb = cus * 8;
  void* out = nullptr;
  CK(hipMalloc(&out, (size_t)maxb * 256 * sizeof(double)));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  for (int prec = 0; prec < 3; ++prec) {
    for (int per_cu : {4, 8}) {
      const int nb = cus * per_cu;
      auto run = [&]() {
        if (prec == 0) hipLaunchKernelGGL(mfma_rate64, dim3(nb), dim3(256), 0, nullptr, (double*)out, iters, 1.0);
        else if (prec == 1) hipLaunchKernelGGL(mfma_rate32, dim3(nb), dim3(256), 0, nullptr, (float*)out, iters, 1.0f);
        else hipLaunchKernelGGL(mfma_rate64q, dim3(nb), dim3(256), 0, nullptr, (double*)out, iters, 1.0);
      };
      run();
      CK(hipDeviceSynchronize());
      CK(hipEventRecord(e0, nullptr));
      for (int r = 0; r < 5; ++r) run();
      CK(hipEventRecord(e1, nullptr));
      CK(hipEventSynchronize(e1));
      CK(hipGetLastError());
      float ms = 0.0f;
      CK(hipEventElapsedTime(&ms, e0, e1));
      const double per_instr = prec == 2 ? 4.0 * 4.0 * 4.0 * 4.0 * 2.0 : 16.0 * 16.0 * 4.0 * 2.0;
      const double flops = 5.0 * nb * 4.0 * iters * 6.0 * per_instr;
      std::printf("{\"kernel\": \"mfma\", \"what\": \"%s, 6 chains per wave\", \"cus\": %d, "
                  "\"waves_per_simd\": %d, \"us_per_launch\": %.1f, \"tflops\": %.2f}\n",
                  prec == 0 ? "f64 16x16x4" : prec == 1 ? "f32 16x16x4" : "f64 4x4x4 4 blocks", cus, per_cu,
                  ms * 1e3 / 5, flops / (ms * 1e-3) * 1e-12);
    }
  }
  CK(hipEventDestroy(e0));
  CK(hipEventDestroy(e1));
  CK(hipFree(out));
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: kbench chan32|chan64|chan32r|chan64r|chandual|lu_np|lu|rsolve|rsolve32|copy|mfma [n_phi] [chains] "
                         "[iters] [cfg] [variant] [fp64_percent]\n");
    return 2;
  }
  const std::string k = argv[1];
  if (k == "mfma") return mfma_rates();
  if (k == "copy") {
    const size_t bytes = (size_t)1 << 30;
    void *a = nullptr, *b = nullptr;
    CK(hipMalloc(&a, bytes));
    CK(hipMalloc(&b, bytes));
    CK(hipMemset(a, 1, bytes));
    CK(hipDeviceSynchronize());
    for (int i = 0; i < 3; ++i) CK(hipMemcpyAsync(b, a, bytes, hipMemcpyDeviceToDevice, nullptr));
    CK(hipDeviceSynchronize());
    std::printf("{\"kernel\": \"copy\", \"bytes\": %zu, \"copies\": 3}\n", bytes);
    hipFree(a);
    hipFree(b);
    return 0;
  }
  const int N = argc > 2 ? std::atoi(argv[2]) : 100;
  const int B = argc > 3 ? std::atoi(argv[3]) : 256;
  const int iters = argc > 4 ? std::atoi(argv[4]) : 20;
  const int cfg = argc > 5 ? std::atoi(argv[5]) : 1;
  const int variant = argc > 6 ? std::atoi(argv[6]) : 2;
  const int pct64 = argc > 7 ? std::atoi(argv[7]) : 50;
  if (N < 1 || N > 140 || B < 1 || B > 512 || iters < 1 || cfg < 0 || cfg >= CFQMC_CHAN_CFGS || variant < 1 ||
      variant > 2 || pct64 < 0 || pct64 > 100) {
    std::fprintf(stderr, "kbench: n_phi 1..140, chains 1..512, iters >= 1, cfg 0..%d, variant 1..2, "
                 "fp64_percent 0..100\n", CFQMC_CHAN_CFGS - 1);
    return 2;
  }
  if (k == "chandual" && cfg != 1 && cfg != 12) {
    std::fprintf(stderr, "kbench: chandual needs cfg 1 or 12\n");
    return 2;
  }
  const int n = 2 * N;
  const long long nn = (long long)n * n, NN = (long long)N * N;
  hipStream_t s = nullptr;
  std::vector<double2> hM((size_t)B * nn);
  fill_random(hM, 1, 1.0);
  std::function<void()> run;
  double algo = 0.0, issued = 0.0;
  const char* what = "";
  std::vector<void*> bufs;
  if (k.rfind("chan", 0) == 0) {
    const bool dual = k == "chandual";
    const bool mixed = dual || k.find("32") != std::string::npos;
    const bool right = k.back() == 'r';
    std::vector<double2> hX((size_t)B * 2 * NN);
    fill_random(hX, 2, 0.3 / N);   // entries ~ 0.3 / N: a matrix norm ~ 0.3
    for (int z = 0; z < 2 * B; ++z)
      for (int i = 0; i < N; ++i) hX[(size_t)z * NN + (size_t)i * N + i].x += 1.0;
    double2* dM = upload(hM);
    double2* dX = upload(hX);
    double2* dY = nullptr;
    CK(hipMalloc(&dY, (size_t)B * nn * sizeof(double2)));
    bufs = {dM, dX, dY};
    ChanArgs a;
    std::memset(&a, 0, sizeof(a));
    a.N = N; a.n_other = n;
    a.M = dM; a.ldM = n; a.sM = nn;
    a.X0 = dX; a.X1 = dX + NN; a.ldX = N; a.sX = 2 * NN;
    a.Y = dY; a.ldY = n; a.sY = nn;
    const int left = right ? 0 : 1, rot = right ? 1 : 2;
    if (dual) {
      // FP64 flags for fp64_percent of the chains, spread evenly over the batch
      std::vector<int> sel(B);
      for (int z = 0; z < B; ++z) sel[z] = ((z + 1) * pct64) / 100 - (z * pct64) / 100;
      int* dsel = nullptr;
      CK(hipMalloc(&dsel, B * sizeof(int)));
      CK(hipMemcpy(dsel, sel.data(), B * sizeof(int), hipMemcpyHostToDevice));
      bufs.push_back(dsel);
      a.chain_sel = dsel;
      run = [=]() { launch_chan_apply_dual(a, left, rot, B, cfg, 1, variant, s); };
    } else {
      run = [=]() { launch_chan_apply(a, left, rot, B, mixed ? 1 : 0, cfg, s); };
    }
    algo = 2.0 * (double)n * n * n * B;
    issued = 16.0 * (double)N * N * n * B;
    what = dual ? "channel application, guarded (FP32 / FP64 chains in one launch)"
                : mixed ? "channel application, FP32 correction form" : "channel application, FP64 (3-product MFMA)";
  } else if (k == "lu_np" || k == "lu" || k == "rsolve" || k == "rsolve32") {
    // M = 1 + 0.05 R: close to the identity, as the Woodbury matrix of a slice move
    std::vector<double2> hA((size_t)B * nn);
    fill_random(hA, 3, 0.05 / std::sqrt((double)n));
    for (int z = 0; z < B; ++z)
      for (int i = 0; i < n; ++i) hA[(size_t)z * nn + (size_t)i * n + i].x += 1.0;
    double2* dA0 = upload(hA);
    double2* dA = nullptr;
    double2* dld = nullptr;
    int *dpiv = nullptr, *dflag = nullptr;
    CK(hipMalloc(&dA, (size_t)B * nn * sizeof(double2)));
    CK(hipMalloc(&dld, (size_t)B * sizeof(double2)));
    CK(hipMalloc(&dpiv, (size_t)B * n * sizeof(int)));
    CK(hipMalloc(&dflag, (size_t)B * sizeof(int)));
    CK(hipMemcpy(dA, dA0, (size_t)B * nn * sizeof(double2), hipMemcpyDeviceToDevice));
    bufs = {dA0, dA, dld, dpiv, dflag};
    if (k == "lu_np") {
      // the factorisation works in place: restore A before every launch (a copy kernel, timed apart)
      run = [=]() {
        launch_copy(dA0, dA, nn, nn, nn, B, s);
        launch_lu_np(dA, n, n, nn, dpiv, n, dld, dflag, 8.0, B, s);
      };
      algo = 8.0 / 3.0 * (double)n * n * n * B;
      issued = algo;
      what = "non-pivoted LU (plus the restoring copy)";
    } else if (k == "lu") {
      run = [=]() {
        launch_copy(dA0, dA, nn, nn, nn, B, s);
        launch_lu(dA, n, n, nn, dpiv, n, dld, 1, B, s, nullptr, nullptr);
      };
      algo = 8.0 / 3.0 * (double)n * n * n * B;
      issued = algo;
      what = "partially pivoted LU (plus the restoring copy)";
    } else {
      launch_lu_np(dA, n, n, nn, dpiv, n, dld, dflag, 8.0, B, s);
      double2* dG = upload(hM);
      double2 *dY = nullptr, *ws = nullptr;
      CK(hipMalloc(&dY, (size_t)B * nn * sizeof(double2)));
      CK(hipMalloc(&ws, (size_t)B * rsolve_work_size(n) * sizeof(double2)));
      bufs.push_back(dG);
      bufs.push_back(dY);
      bufs.push_back(ws);
      const int m32 = k == "rsolve32" ? 1 : 0;
      run = [=]() { launch_rsolve(dG, n, nn, dY, n, nn, dA, n, nn, dpiv, n, n, 0, B, s, ws, m32, nullptr); };
      algo = 8.0 * (double)n * n * n * B;
      issued = algo;
      what = m32 ? "right solve G M^-1, FP32 block products" : "right solve G M^-1 (two triangular solves)";
    }
  } else {
    std::fprintf(stderr, "kbench: unknown kernel %s\n", k.c_str());
    return 2;
  }
  // warm-up: half a second of launches, so that the clocks have ramped
  {
    const auto tw = std::chrono::steady_clock::now();
    do {
      for (int w = 0; w < 4; ++w) run();
      CK(hipDeviceSynchronize());
    } while (std::chrono::duration<double>(std::chrono::steady_clock::now() - tw).count() < 0.5);
  }
  const auto t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < iters; ++i) run();
  CK(hipDeviceSynchronize());
  const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count() / iters;
  CK(hipGetLastError());
  std::printf("{\"kernel\": \"%s\", \"what\": \"%s\", \"n_phi\": %d, \"chains\": %d, \"cfg\": %d, \"iters\": %d, "
              "\"variant\": %d, \"fp64_percent\": %d, "
              "\"us_per_launch\": %.2f, \"algorithmic_tflops\": %.3f, \"issued_tflops\": %.3f}\n",
              k.c_str(), what, N, B, cfg, iters, k == "chandual" ? variant : 0, k == "chandual" ? pct64 : 0, us,
              algo / us * 1e-6, issued / us * 1e-6);
  for (void* p : bufs) hipFree(p);
  return 0;
}
