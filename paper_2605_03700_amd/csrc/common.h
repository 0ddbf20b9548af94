// Shared device helpers for the CF-DQMC sweep kernels (gfx950 / CDNA4).
//
// Complex numbers are stored interleaved (re, im) as double2 (complex128
// layout); the mixed-precision path computes in float2 with FP64
// accumulation. All matrices are row-major with an explicit leading
// dimension; batches are addressed by base pointer + index * stride.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

#define CF_DEV __device__ __forceinline__

CF_DEV double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
CF_DEV double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
CF_DEV double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
CF_DEV double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
CF_DEV double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
CF_DEV double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
// 1/b = conj(b) / |b|^2 with a single real division (|b| is O(1) where used:
// pivots and diagonals of factors of well-scaled matrices)
CF_DEV double2 crcp(double2 b) {
  const double r = 1.0 / (b.x * b.x + b.y * b.y);
  return make_double2(b.x * r, -b.y * r);
}
CF_DEV double2 cdiv(double2 a, double2 b) {
  // Smith's algorithm for a/b
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  } else {
    double r = b.x / b.y, d = b.y + b.x * r;
    return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
  }
}

// MFMA 16x16x4 wrappers. Operand lane layout (both precisions, measured on
// gfx950): lane l supplies A[l%16][l/16] and B[l/16][l%16]. Result layout
// differs: FP64 holds D[4r + l/16][l%16] in item r, FP32 holds
// D[4(l/16) + r][l%16].
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4v acc_t;
  static CF_DEV acc_t zero() { acc_t z = {0.0, 0.0, 0.0, 0.0}; return z; }
  static CF_DEV acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static CF_DEV int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <> struct Mfma<float> {
  typedef f4v acc_t;
  static CF_DEV acc_t zero() { acc_t z = {0.f, 0.f, 0.f, 0.f}; return z; }
  static CF_DEV acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static CF_DEV int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T> struct cplx_t;
template <> struct cplx_t<double> { typedef double2 type; };
template <> struct cplx_t<float> { typedef float2 type; };

template <typename T> CF_DEV typename cplx_t<T>::type to_ct(double2 v);
template <> CF_DEV double2 to_ct<double>(double2 v) { return v; }
template <> CF_DEV float2 to_ct<float>(double2 v) { return make_float2((float)v.x, (float)v.y); }

// Batched matrix view: element (i, j) of batch z at p + z1*s1 + z2*s2 + i*ld + j
// with z = z1 * nz2 + z2.
struct MatRef {
  double2* p;
  int ld;
  long long s1, s2;
};
CF_DEV double2* mat_at(const MatRef& m, int z1, int z2) { return m.p + z1 * m.s1 + z2 * m.s2; }

// Block-wide sum for up to 1024 threads (result valid in all threads).
template <int NT>
CF_DEV double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

// ------------------------------------------------------------------ Philox4x32-10
// Counter-based generator of Salmon, Moraes, Dror & Shaw (SC'11), 10 rounds.
CF_DEV void philox_round(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
  c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}
CF_DEV void philox(uint32_t (&c)[4], uint64_t seed) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k0, k1);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}
CF_DEV double u53(uint32_t a, uint32_t b) { return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0); }
// Normal number j of stream (chain, counter) by Box-Muller on one Philox block.
CF_DEV double rng_normal(uint64_t seed, int chain, long long counter, int j) {
  uint32_t c[4] = {(uint32_t)(j >> 1), (uint32_t)counter, (uint32_t)(counter >> 32), (uint32_t)chain};
  philox(c, seed);
  const double u1 = 1.0 - u53(c[0], c[1]), u2 = u53(c[2], c[3]);
  const double r = sqrt(-2.0 * log(u1));
  return (j & 1) ? r * sin(2.0 * M_PI * u2) : r * cos(2.0 * M_PI * u2);
}
CF_DEV double rng_uniform(uint64_t seed, int chain, long long counter) {
  uint32_t c[4] = {0x7fffffffu, (uint32_t)counter, (uint32_t)(counter >> 32), (uint32_t)chain};
  philox(c, seed);
  return u53(c[0], c[1]);
}
