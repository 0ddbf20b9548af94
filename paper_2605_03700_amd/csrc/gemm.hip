// Complex GEMM and channel-exponential application on MFMA (gfx950).
//
// zgemm:      D = alpha * op(A) op(B) + beta * C, batched, with two extra
//             epilogues used by the Taylor exponential (P/Q split and the
//             predicated squaring).
// chan_apply: Y = E X or Y = X E for a channel exponential
//             E = (U kron 1) diag(X0, X1) (U^dagger kron 1), U a 2x2 unitary
//             acting on the valley index, X0/X1 the N x N orbital blocks
//             (Methods, HS transform: exp(alpha h kron o) splits into the +1 and
//             -1 eigenspaces of o). The valley rotation is applied while tiles
//             are staged into LDS, so one pass costs two N x N x n products
//             instead of one n x n x n product.
//
// FP64 complex products take three real 16x16x4 MFMAs per k step (Gauss:
// re = P - Q, im = S - P - Q); a tile whose last 16 rows or columns are only
// partly valid takes the FP64 4x4x4 four-block MFMA for its valid 4-row or
// 4-column groups instead (mma_slab3_rows / mma_slab3_cols). In the mixed path
// (CT = float) operands are rounded to FP32 when staged and multiplied on the
// FP32 MFMA (four real products per complex one, or three in the three-product
// configurations), each 16-deep k slab added into FP64 registers or, in the
// FP32-accumulating configurations, the whole k range. chan_apply
// additionally works in correction form there: it stages X_a - 1 (formed in
// FP64 before rounding; ||X_a - 1|| is the small channel exponent) and adds
// the FP64 input back in the epilogue, E M = M + (E - 1) M, so the FP32
// rounding only touches the increment.
#include <cstdio>
#include <cstdlib>

#include "common.h"
#include "kernels.h"

#define BK 16

template <typename CT, int WTM, int WTN>
struct Acc {
  typedef typename Mfma<CT>::acc_t acc_t;
  acc_t re[WTM][WTN], im[WTM][WTN];
  CF_DEV void zero() {
#pragma unroll
    for (int a = 0; a < WTM; ++a)
#pragma unroll
      for (int b = 0; b < WTN; ++b) { re[a][b] = Mfma<CT>::zero(); im[a][b] = Mfma<CT>::zero(); }
  }
};

// One BK-deep slab of wave-tile products from LDS (As[k][m], Bs[k][n]).
// mrem / nrem: valid rows / columns from the wave tile's origin, krem: valid k
// in the slab. 16 x 16 subtiles and k steps lying entirely in the zero padding
// are skipped (wave-uniform branches), which changes no valid output.
template <typename CT, int WTM, int WTN, int KD = BK>
CF_DEV void mma_slab(const typename cplx_t<CT>::type* As, int lda, const typename cplx_t<CT>::type* Bs, int ldb,
                     int wm0, int wn0, int lane, Acc<CT, WTM, WTN>& acc, int mrem = 1 << 30, int nrem = 1 << 30,
                     int krem = 1 << 30) {
  typedef typename cplx_t<CT>::type C2;
  const int il = lane & 15, kl = lane >> 4;
  mrem = __builtin_amdgcn_readfirstlane(mrem);
  nrem = __builtin_amdgcn_readfirstlane(nrem);
  krem = __builtin_amdgcn_readfirstlane(krem);
#pragma unroll
  for (int kk = 0; kk < KD; kk += 4) {
    if (kk >= krem) break;
    C2 a[WTM], b[WTN];
#pragma unroll
    for (int s = 0; s < WTM; ++s) a[s] = As[(kk + kl) * lda + wm0 + s * 16 + il];
#pragma unroll
    for (int s = 0; s < WTN; ++s) b[s] = Bs[(kk + kl) * ldb + wn0 + s * 16 + il];
#pragma unroll
    for (int si = 0; si < WTM; ++si)
#pragma unroll
      for (int sj = 0; sj < WTN; ++sj) {
        if (si * 16 >= mrem || sj * 16 >= nrem) continue;
        acc.re[si][sj] = Mfma<CT>::mma(a[si].x, b[sj].x, acc.re[si][sj]);
        acc.re[si][sj] = Mfma<CT>::mma(-a[si].y, b[sj].y, acc.re[si][sj]);
        acc.im[si][sj] = Mfma<CT>::mma(a[si].x, b[sj].y, acc.im[si][sj]);
        acc.im[si][sj] = Mfma<CT>::mma(a[si].y, b[sj].x, acc.im[si][sj]);
      }
  }
}

// FP64 complex products with three real MFMAs per k step (Gauss): with
// a = ar + i ai, b = br + i bi the sums P = sum ar br, Q = sum ai bi and
// S = sum (ar + ai)(br + bi) give re = P - Q, im = S - P - Q. The operand sums
// are two VALU adds per k step; the MFMA work drops by a quarter. Used for the
// FP64 products only (the FP32 path keeps four products: its rounding budget
// is set by the correction form).
template <int WTM, int WTN>
struct Acc3 {
  d4v p[WTM][WTN], q[WTM][WTN], t[WTM][WTN];
  CF_DEV void zero() {
#pragma unroll
    for (int a = 0; a < WTM; ++a)
#pragma unroll
      for (int b = 0; b < WTN; ++b) { p[a][b] = Mfma<double>::zero(); q[a][b] = p[a][b]; t[a][b] = p[a][b]; }
  }
  CF_DEV void to(Acc<double, WTM, WTN>& o) const {
#pragma unroll
    for (int a = 0; a < WTM; ++a)
#pragma unroll
      for (int b = 0; b < WTN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          o.re[a][b][r] = p[a][b][r] - q[a][b][r];
          o.im[a][b][r] = t[a][b][r] - p[a][b][r] - q[a][b][r];
        }
  }
};

template <int WTM, int WTN, int KD = BK>
CF_DEV void mma_slab3(const double2* As, int lda, const double2* Bs, int ldb, int wm0, int wn0, int lane,
                      Acc3<WTM, WTN>& acc, int mrem = 1 << 30, int nrem = 1 << 30, int krem = 1 << 30) {
  const int il = lane & 15, kl = lane >> 4;
  mrem = __builtin_amdgcn_readfirstlane(mrem);
  nrem = __builtin_amdgcn_readfirstlane(nrem);
  krem = __builtin_amdgcn_readfirstlane(krem);
#pragma unroll
  for (int kk = 0; kk < KD; kk += 4) {
    if (kk >= krem) break;
    double2 a[WTM], b[WTN];
    double sa[WTM], sb[WTN];
#pragma unroll
    for (int s = 0; s < WTM; ++s) {
      a[s] = As[(kk + kl) * lda + wm0 + s * 16 + il];
      sa[s] = a[s].x + a[s].y;
    }
#pragma unroll
    for (int s = 0; s < WTN; ++s) {
      b[s] = Bs[(kk + kl) * ldb + wn0 + s * 16 + il];
      sb[s] = b[s].x + b[s].y;
    }
#pragma unroll
    for (int si = 0; si < WTM; ++si)
#pragma unroll
      for (int sj = 0; sj < WTN; ++sj) {
        if (si * 16 >= mrem || sj * 16 >= nrem) continue;
        acc.p[si][sj] = Mfma<double>::mma(a[si].x, b[sj].x, acc.p[si][sj]);
        acc.q[si][sj] = Mfma<double>::mma(a[si].y, b[sj].y, acc.q[si][sj]);
        acc.t[si][sj] = Mfma<double>::mma(sa[si], sb[sj], acc.t[si][sj]);
      }
  }
}

// The same products for a wave tile with 0 < mrem < 16 valid rows: one FP64
// 4x4x4 four-block MFMA per 4-row group that holds valid rows (the blocks are
// the four 4-column groups and share the B operand) instead of the 16x16x4
// instruction over all 16 rows. Group r lands in accumulator element r, where
// the 16x16x4 instruction puts rows 4r .. 4r + 3.
template <int KD = BK>
CF_DEV void mma_slab3_rows(const double2* As, int lda, const double2* Bs, int ldb, int wm0, int wn0, int lane,
                           Acc3<1, 1>& acc, int mrem, int krem) {
  const int il = lane & 15, kl = lane >> 4, i4 = lane & 3;
  mrem = __builtin_amdgcn_readfirstlane(mrem);
  krem = __builtin_amdgcn_readfirstlane(krem);
#pragma unroll
  for (int kk = 0; kk < KD; kk += 4) {
    if (kk >= krem) break;
    const double2 b = Bs[(kk + kl) * ldb + wn0 + il];
    const double sb = b.x + b.y;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (4 * r >= mrem) break;
      const double2 a = As[(kk + kl) * lda + wm0 + 4 * r + i4];
      acc.p[0][0][r] = __builtin_amdgcn_mfma_f64_4x4x4f64(a.x, b.x, acc.p[0][0][r], 0, 0, 0);
      acc.q[0][0][r] = __builtin_amdgcn_mfma_f64_4x4x4f64(a.y, b.y, acc.q[0][0][r], 0, 0, 0);
      acc.t[0][0][r] = __builtin_amdgcn_mfma_f64_4x4x4f64(a.x + a.y, sb, acc.t[0][0][r], 0, 0, 0);
    }
  }
}

// The same products for a wave tile with 0 < nrem < 16 valid columns: the
// four blocks of the 4x4x4 MFMA lie along the rows (block b = rows 4b .. 4b+3,
// whose A operand is the 16x16x4 instruction's), one instruction per 4-column
// group c that holds valid columns, into accumulator element c. Element c of
// lane l then holds row 4 ((l >> 2) & 3) + (l >> 4), column 4c + (l & 3).
template <int KD = BK>
CF_DEV void mma_slab3_cols(const double2* As, int lda, const double2* Bs, int ldb, int wm0, int wn0, int lane,
                           Acc3<1, 1>& acc, int nrem, int krem) {
  const int il = lane & 15, kl = lane >> 4, j4 = lane & 3;
  nrem = __builtin_amdgcn_readfirstlane(nrem);
  krem = __builtin_amdgcn_readfirstlane(krem);
#pragma unroll
  for (int kk = 0; kk < KD; kk += 4) {
    if (kk >= krem) break;
    const double2 a = As[(kk + kl) * lda + wm0 + il];
    const double sa = a.x + a.y;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (4 * c >= nrem) break;
      const double2 b = Bs[(kk + kl) * ldb + wn0 + 4 * c + j4];
      acc.p[0][0][c] = __builtin_amdgcn_mfma_f64_4x4x4f64(a.x, b.x, acc.p[0][0][c], 0, 0, 0);
      acc.q[0][0][c] = __builtin_amdgcn_mfma_f64_4x4x4f64(a.y, b.y, acc.q[0][0][c], 0, 0, 0);
      acc.t[0][0][c] = __builtin_amdgcn_mfma_f64_4x4x4f64(sa, b.x + b.y, acc.t[0][0][c], 0, 0, 0);
    }
  }
}

// Which body a workgroup of an FP64 application with 16 x 16 wave tiles runs:
// 0 the 16x16x4 form; 1 the last row tile with fewer than 16 valid rows
// (mma_slab3_rows); 2 the last column tile with fewer than 16 valid columns
// (mma_slab3_cols). At a tile that is both, the form with fewer instructions.
CF_DEV int partial_mode(int rows, int cols, int ty, int tx, int tiles_y, int tiles_x, int BMv, int BNv) {
  const int rr = ty == tiles_y - 1 ? rows - ty * BMv : 16, rc = tx == tiles_x - 1 ? cols - tx * BNv : 16;
  const bool pr = rr < 16, pc = rc < 16;
  if (pr && pc) return (rc + 3) / 4 < (rr + 3) / 4 ? 2 : 1;
  return pr ? 1 : pc ? 2 : 0;
}

// The same three-product form with FP32 operands and accumulators (the FP32
// channel application without accumulation points: P, Q, S stay FP32 over the
// whole k range and are combined in FP64 in the epilogue).
template <int WTM, int WTN>
struct Acc3F {
  f4v p[WTM][WTN], q[WTM][WTN], t[WTM][WTN];
  CF_DEV void zero() {
#pragma unroll
    for (int a = 0; a < WTM; ++a)
#pragma unroll
      for (int b = 0; b < WTN; ++b) { p[a][b] = Mfma<float>::zero(); q[a][b] = p[a][b]; t[a][b] = p[a][b]; }
  }
  CF_DEV void to(Acc<double, WTM, WTN>& o) const {
#pragma unroll
    for (int a = 0; a < WTM; ++a)
#pragma unroll
      for (int b = 0; b < WTN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double P = p[a][b][r], Q = q[a][b][r], T = t[a][b][r];
          o.re[a][b][r] = P - Q;
          o.im[a][b][r] = T - P - Q;
        }
  }
};

template <int WTM, int WTN, int KD = BK>
CF_DEV void mma_slab3f(const float2* As, int lda, const float2* Bs, int ldb, int wm0, int wn0, int lane,
                       Acc3F<WTM, WTN>& acc, int mrem = 1 << 30, int nrem = 1 << 30, int krem = 1 << 30) {
  const int il = lane & 15, kl = lane >> 4;
  mrem = __builtin_amdgcn_readfirstlane(mrem);
  nrem = __builtin_amdgcn_readfirstlane(nrem);
  krem = __builtin_amdgcn_readfirstlane(krem);
#pragma unroll
  for (int kk = 0; kk < KD; kk += 4) {
    if (kk >= krem) break;
    float2 a[WTM], b[WTN];
    float sa[WTM], sb[WTN];
#pragma unroll
    for (int s = 0; s < WTM; ++s) {
      a[s] = As[(kk + kl) * lda + wm0 + s * 16 + il];
      sa[s] = a[s].x + a[s].y;
    }
#pragma unroll
    for (int s = 0; s < WTN; ++s) {
      b[s] = Bs[(kk + kl) * ldb + wn0 + s * 16 + il];
      sb[s] = b[s].x + b[s].y;
    }
#pragma unroll
    for (int si = 0; si < WTM; ++si)
#pragma unroll
      for (int sj = 0; sj < WTN; ++sj) {
        if (si * 16 >= mrem || sj * 16 >= nrem) continue;
        acc.p[si][sj] = Mfma<float>::mma(a[si].x, b[sj].x, acc.p[si][sj]);
        acc.q[si][sj] = Mfma<float>::mma(a[si].y, b[sj].y, acc.q[si][sj]);
        acc.t[si][sj] = Mfma<float>::mma(sa[si], sb[sj], acc.t[si][sj]);
      }
  }
}

// FP64 accumulation point: add an FP32 slab accumulator into FP64 registers.
template <int WTM, int WTN>
CF_DEV void flush(Acc<float, WTM, WTN>& a32, Acc<double, WTM, WTN>& a64) {
#pragma unroll
  for (int si = 0; si < WTM; ++si)
#pragma unroll
    for (int sj = 0; sj < WTN; ++sj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        a64.re[si][sj][r] += (double)a32.re[si][sj][r];
        a64.im[si][sj][r] += (double)a32.im[si][sj][r];
      }
}

// Output row of accumulator item r for lane (precision-dependent layout).
template <typename CT> CF_DEV int out_row(int lane, int r) { return Mfma<CT>::row(lane, r); }

// Tile order: the hardware hands consecutive workgroups to the eight XCDs in
// turn, so logical tile t = (b % 8) * ceil(T/8) + b / 8 gives every XCD a
// contiguous range of (chain, row tile, column tile): the tiles of one chain
// share that XCD's L2.
CF_DEV bool xcd_tile(int tiles_x, int tiles_y, int nbatch, int& z, int& ty, int& tx) {
  const int T = tiles_x * tiles_y * nbatch;
  const int per = (T + 7) / 8;
  const int b = blockIdx.x;
  const int t = (b % 8) * per + b / 8;
  if (t >= T) return false;
  z = t / (tiles_x * tiles_y);
  const int r = t % (tiles_x * tiles_y);
  ty = r / tiles_x;
  tx = r % tiles_x;
  return true;
}

// Does the block rows [r0, r0 + nr) x cols [c0, c0 + nc) meet the wrap-around
// band |(col - row) mod K| <= b? The differences col - row fill [dlo, dhi]; the
// band is the union of [mK - b, mK + b] over integers m.
CF_DEV bool band_meets(int r0, int nr, int c0, int nc, int b, int K) {
  if (b < 0) return true;
  const int dlo = c0 - (r0 + nr - 1), dhi = c0 + nc - 1 - r0;
  // smallest m with mK + b >= dlo, then check mK - b <= dhi
  int m = (dlo - b) >= 0 ? (dlo - b + K - 1) / K : -((b - dlo) / K);
  return m * K - b <= dhi;
}

// ------------------------------------------------------------------ zgemm

// The product of tile (ty, tx) of matrix z; As / Bs the workgroup's LDS
// operand tiles. RM (FP64, one 16 x 16 wave tile per wave; partial_mode): 1 a
// last row tile with fewer than 16 valid rows, 2 a last column tile with fewer
// than 16 valid columns, on the FP64 4x4x4 MFMA.
template <typename CT, int BM, int BN, int WTM, int WTN, int RM>
CF_DEV void zgemm_body(const GemmArgs& g, int z, int ty, int tx, typename cplx_t<CT>::type* As,
                       typename cplx_t<CT>::type* Bs) {
  typedef typename cplx_t<CT>::type C2;
  constexpr int WX = BN / (16 * WTN), WY = BM / (16 * WTM);
  constexpr int NT = WX * WY * 64;
  constexpr int LDA = BM + (sizeof(C2) == 16 ? 2 : 4), LDB = BN + (sizeof(C2) == 16 ? 2 : 4);
  const int z1 = z / g.nz2, z2 = z % g.nz2;
  const int m0 = ty * BM, n0 = tx * BN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm0 = (wid / WX) * 16 * WTM, wn0 = (wid % WX) * 16 * WTN;
  const double2* A = mat_at(g.A, z1, z2);
  const double2* B = mat_at(g.B, z1, z2);

  // squaring count of this matrix: a squaring step past it has nothing to do
  const int nsq = g.pred ? g.pred[z1 * g.pred_s1 + z2 * g.pred_s2] : 0;
  if (g.mode == GEMM_SQUARE && nsq <= g.pred_thresh) return;

  constexpr int EA = BM * BK / NT, EB = BN * BK / NT;
  double2 ra[EA], rb[EB];
  const double2 zero2 = make_double2(0.0, 0.0);
  // bare loads here (out-of-range elements read offset 0 and are zeroed at
  // staging time, like the conjugation), so the loads stay in flight
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * NT;
      int m, k;
      if (g.opA == 0) { k = idx % BK; m = idx / BK; } else { m = idx % BM; k = idx / BM; }
      const bool ok = m0 + m < g.M && k0 + k < g.K;
      const long long off = !ok ? 0 : g.opA == 0 ? (long long)(m0 + m) * g.A.ld + k0 + k
                                                  : (long long)(k0 + k) * g.A.ld + m0 + m;
      ra[e] = A[off];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + e * NT;
      int n, k;
      if (g.opB == 0) { n = idx % BN; k = idx / BN; } else { k = idx % BK; n = idx / BK; }
      const bool ok = n0 + n < g.N && k0 + k < g.K;
      const long long off = !ok ? 0 : g.opB == 0 ? (long long)(k0 + k) * g.B.ld + n0 + n
                                                  : (long long)(n0 + n) * g.B.ld + k0 + k;
      rb[e] = B[off];
    }
  };
  auto stage = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * NT;
      int m, k;
      if (g.opA == 0) { k = idx % BK; m = idx / BK; } else { m = idx % BM; k = idx / BM; }
      double2 v = ra[e];
      if (g.opA != 0) v.y = -v.y;
      if (!(m0 + m < g.M && k0 + k < g.K)) v = zero2;
      As[k * LDA + m] = to_ct<CT>(v);
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const int idx = tid + e * NT;
      int n, k;
      if (g.opB == 0) { n = idx % BN; k = idx / BN; } else { k = idx % BK; n = idx / BK; }
      double2 v = rb[e];
      if (g.opB != 0) v.y = -v.y;
      if (!(n0 + n < g.N && k0 + k < g.K)) v = zero2;
      Bs[k * LDB + n] = to_ct<CT>(v);
    }
  };
  Acc<double, WTM, WTN> acc;
  acc.zero();
  Acc3<WTM, WTN> acc3;
  acc3.zero();
  {
    // k slabs whose A block (tile rows) and B block (tile columns) can be
    // nonzero; the test is uniform over the workgroup
    auto live = [&](int k0) {
      const int kw = min(BK, g.K - k0);
      return band_meets(m0, min(BM, g.M - m0), k0, kw, g.bandA, g.K) &&
             band_meets(k0, kw, n0, min(BN, g.N - n0), g.bandB, g.K);
    };
    auto next_live = [&](int k0) {
      while (k0 < g.K && !live(k0)) k0 += BK;
      return k0;
    };
    int k0 = next_live(0);
    if (k0 < g.K) fetch(k0);
    for (; k0 < g.K;) {
      stage(k0);
      __syncthreads();
      const int k1 = next_live(k0 + BK);
      if (k1 < g.K) fetch(k1);
      const int mr = g.M - m0 - wm0, nr = g.N - n0 - wn0, kr = g.K - k0;
      if constexpr (sizeof(CT) == 8 && RM == 1) {
        if (mr > 0 && nr > 0)
          mma_slab3_rows<BK>((const double2*)As, LDA, (const double2*)Bs, LDB, wm0, wn0, lane, acc3, mr, kr);
      } else if constexpr (sizeof(CT) == 8 && RM == 2) {
        if (mr > 0 && nr > 0)
          mma_slab3_cols<BK>((const double2*)As, LDA, (const double2*)Bs, LDB, wm0, wn0, lane, acc3, nr, kr);
      } else if constexpr (sizeof(CT) == 8) {
        mma_slab3<WTM, WTN>((const double2*)As, LDA, (const double2*)Bs, LDB, wm0, wn0, lane, acc3, mr, nr, kr);
      } else {
        Acc<float, WTM, WTN> a32;
        a32.zero();
        mma_slab<float, WTM, WTN>((const float2*)As, LDA, (const float2*)Bs, LDB, wm0, wn0, lane, a32, mr, nr, kr);
        flush(a32, acc);
      }
      __syncthreads();
      k0 = k1;
    }
  }
  if constexpr (sizeof(CT) == 8) acc3.to(acc);
  double2 alpha = g.alpha;
  if (g.alpha_dev) alpha = cmul(alpha, g.alpha_dev[z1 * g.ad_s1 + z2 * g.ad_s2]);
  // with squaring counts: a matrix whose last step this is goes to its final place
  const bool fin = g.pred && (g.mode == GEMM_SQUARE ? nsq == g.pred_thresh + 1 : nsq == 0);
  double2* D = fin ? mat_at(g.E, z1, z2) : mat_at(g.D, z1, z2);
  const double2* Cm = g.C.p ? mat_at(g.C, z1, z2) : nullptr;
  double2* D2 = fin ? (g.E2.p ? mat_at(g.E2, z1, z2) : nullptr) : (g.D2.p ? mat_at(g.D2, z1, z2) : nullptr);
  const int ldd = fin ? g.E.ld : g.D.ld, ldd2 = fin ? g.E2.ld : g.D2.ld;
#pragma unroll
  for (int si = 0; si < WTM; ++si)
#pragma unroll
    for (int sj = 0; sj < WTN; ++sj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm0 + si * 16 + (RM == 2 ? 4 * ((lane >> 2) & 3) + (lane >> 4) : out_row<CT>(lane, r));
        const int j = n0 + wn0 + sj * 16 + (RM == 2 ? 4 * r + (lane & 3) : (lane & 15));
        if (i >= g.M || j >= g.N) continue;
        double2 p = make_double2(acc.re[si][sj][r], acc.im[si][sj][r]);
        if (g.mode == GEMM_SQUARE) {
          D[(long long)i * ldd + j] = p;
        } else if (g.mode == GEMM_PQ) {
          double2 x = cmul(alpha, p);
          double2 c = Cm[(long long)i * g.C.ld + j];
          D[(long long)i * ldd + j] = cadd(c, x);
          D2[(long long)i * ldd2 + j] = csub(c, x);
        } else {
          double2 v = cmul(alpha, p);
          if (Cm) v = cadd(v, cmul(g.beta, Cm[(long long)i * g.C.ld + j]));
          D[(long long)i * ldd + j] = v;
          if (g.herm && ty < tx) D[(long long)j * ldd + i] = make_double2(v.x, -v.y);
        }
      }
}

template <typename CT, int BM, int BN, int WTM, int WTN>
__global__ void __launch_bounds__((BM / (16 * WTM)) * (BN / (16 * WTN)) * 64)
__attribute__((amdgpu_waves_per_eu(sizeof(CT) == 8 && WTM == 1 && WTN == 1 ? (BM == 16 ? 4 : 5) : 1)))
zgemm_kernel(GemmArgs g, int tiles_x, int tiles_y, int nbatch) {
  typedef typename cplx_t<CT>::type C2;
  // padded rows: the k-fastest staging stores of a quarter wave hit distinct banks
  constexpr int LDA = BM + (sizeof(C2) == 16 ? 2 : 4), LDB = BN + (sizeof(C2) == 16 ? 2 : 4);
  __shared__ C2 As[BK * LDA];
  __shared__ C2 Bs[BK * LDB];
  int z, ty, tx;
  if (!xcd_tile(tiles_x, tiles_y, nbatch, z, ty, tx)) return;
  if (g.herm) {
    // tiles_x counts the upper triangle (row-major) of a herm x herm tile grid
    int r = tx, a = 0;
    while (r >= g.herm - a) { r -= g.herm - a; ++a; }
    ty = a;
    tx = a + r;
  }
  if constexpr (sizeof(CT) == 8 && WTM == 1 && WTN == 1) {
    const int pm = partial_mode(g.M, g.N, ty, tx, g.herm ? g.herm : tiles_y, g.herm ? g.herm : tiles_x, BM, BN);
    if (pm == 1) {
      zgemm_body<CT, BM, BN, WTM, WTN, 1>(g, z, ty, tx, As, Bs);
      return;
    }
    if (pm == 2) {
      zgemm_body<CT, BM, BN, WTM, WTN, 2>(g, z, ty, tx, As, Bs);
      return;
    }
  }
  zgemm_body<CT, BM, BN, WTM, WTN, 0>(g, z, ty, tx, As, Bs);
}

// ------------------------------------------------------------------ exp_eo
// Even and odd Taylor parts of the exponential in one pass (x = h^2, X2 = x^2,
// X3 = x^3, coefficients e_k = w^k/(2k)!, o_k = w^k/(2k+1)! per matrix):
//   E = (e0 + e1 x + e2 X2) + X3 (e3 + e4 x + e5 X2 + e6 X3)
//   O = (o0 + o1 x + o2 X2) + X3 (o3 + o4 x + o5 X2 + o6 X3)
// X3 is the shared A operand; the two polynomial B operands are formed from
// x, X2, X3 while staging, the low-order parts in the epilogue. Both results are
// Hermitian (h Hermitian, real coefficients): only tiles on and above the
// diagonal are computed, each strictly upper tile also writing its conjugate
// transpose. FP64, three-MFMA complex products.
// Tile (ty, tx) of matrix z; RM as for chan_apply_body (partial_mode: 1 / 2 a
// last row / column tile with fewer than 16 valid rows / columns, on the FP64
// 4x4x4 MFMA).
template <int BT, int RM>
CF_DEV void exp_eo_body(const double2* H2, const double2* X2, const double2* X3, const double* coef, int N,
                        double2* Eo, double2* Oo, int z, int ty, int tx, double2* As, double2* Be, double2* Bo) {
  constexpr int WX = BT / 16, NT = WX * WX * 64;
  constexpr int LD = BT + 2;
  const long long NN = (long long)N * N, off = z * NN;
  const double* cf = coef + (long long)z * EXP_NC;
  const double e3 = cf[3], e4 = cf[4], e5 = cf[5], e6 = cf[6];
  const double o3 = cf[10], o4 = cf[11], o5 = cf[12], o6 = cf[13];
  const int m0 = ty * BT, n0 = tx * BT;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm0 = (wid / WX) * 16, wn0 = (wid % WX) * 16;
  constexpr int EA = BT * BK / NT;
  static_assert(EA * NT == BT * BK, "tile / thread mismatch");
  double2 ra[EA], rh[EA], rx[EA], ry[EA];
  // bare loads from clamped offsets (out-of-range elements read element 0 of
  // the matrix and are zeroed when staged)
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * NT;
      {
        const int k = idx % BK, m = idx / BK;   // A: X3 (m, k)
        const bool ok = m0 + m < N && k0 + k < N;
        ra[e] = X3[off + (ok ? (long long)(m0 + m) * N + k0 + k : 0)];
      }
      {
        const int n = idx % BT, k = idx / BT;   // B sources (k, n)
        const bool ok = n0 + n < N && k0 + k < N;
        const long long o = off + (ok ? (long long)(k0 + k) * N + n0 + n : 0);
        rh[e] = H2[o];
        rx[e] = X2[o];
        ry[e] = X3[o];
      }
    }
  };
  auto stage = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const int idx = tid + e * NT;
      {
        const int k = idx % BK, m = idx / BK;
        const bool ok = m0 + m < N && k0 + k < N;
        As[k * LD + m] = make_double2(ok ? ra[e].x : 0.0, ok ? ra[e].y : 0.0);
      }
      {
        const int n = idx % BT, k = idx / BT;
        const bool ok = n0 + n < N && k0 + k < N;
        const double d = (k0 + k == n0 + n) ? 1.0 : 0.0;
        // the padding (whose loads read element 0) is zeroed component-wise
        const double ber = e3 * d + e4 * rh[e].x + e5 * rx[e].x + e6 * ry[e].x;
        const double bei = e4 * rh[e].y + e5 * rx[e].y + e6 * ry[e].y;
        const double bor = o3 * d + o4 * rh[e].x + o5 * rx[e].x + o6 * ry[e].x;
        const double boi = o4 * rh[e].y + o5 * rx[e].y + o6 * ry[e].y;
        Be[k * LD + n] = make_double2(ok ? ber : 0.0, ok ? bei : 0.0);
        Bo[k * LD + n] = make_double2(ok ? bor : 0.0, ok ? boi : 0.0);
      }
    }
  };
  Acc3<1, 1> ae, ao;
  ae.zero();
  ao.zero();
  const int mr = N - m0 - wm0, nr = N - n0 - wn0;
  fetch(0);
  for (int k0 = 0; k0 < N; k0 += BK) {
    stage(k0);
    __syncthreads();
    if (k0 + BK < N) fetch(k0 + BK);
    if constexpr (RM == 1) {
      if (mr > 0 && nr > 0) {
        mma_slab3_rows<BK>(As, LD, Be, LD, wm0, wn0, lane, ae, mr, N - k0);
        mma_slab3_rows<BK>(As, LD, Bo, LD, wm0, wn0, lane, ao, mr, N - k0);
      }
    } else if constexpr (RM == 2) {
      if (mr > 0 && nr > 0) {
        mma_slab3_cols<BK>(As, LD, Be, LD, wm0, wn0, lane, ae, nr, N - k0);
        mma_slab3_cols<BK>(As, LD, Bo, LD, wm0, wn0, lane, ao, nr, N - k0);
      }
    } else {
      mma_slab3<1, 1>(As, LD, Be, LD, wm0, wn0, lane, ae, mr, nr, N - k0);
      mma_slab3<1, 1>(As, LD, Bo, LD, wm0, wn0, lane, ao, mr, nr, N - k0);
    }
    __syncthreads();
  }
  const double e0 = cf[0], e1 = cf[1], e2 = cf[2], o0 = cf[7], o1 = cf[8], o2 = cf[9];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double er = ae.p[0][0][r] - ae.q[0][0][r], ei = ae.t[0][0][r] - ae.p[0][0][r] - ae.q[0][0][r];
    const double or_ = ao.p[0][0][r] - ao.q[0][0][r], oi = ao.t[0][0][r] - ao.p[0][0][r] - ao.q[0][0][r];
    const int i = m0 + wm0 + (RM == 2 ? 4 * ((lane >> 2) & 3) + (lane >> 4) : Mfma<double>::row(lane, r));
    const int j = n0 + wn0 + (RM == 2 ? 4 * r + (lane & 3) : (lane & 15));
    if (i >= N || j >= N) continue;
    const long long o = off + (long long)i * N + j;
    const double2 h = H2[o], x = X2[o];
    const double d = (i == j) ? 1.0 : 0.0;
    const double2 ve = make_double2(er + e0 * d + e1 * h.x + e2 * x.x, ei + e1 * h.y + e2 * x.y);
    const double2 vo = make_double2(or_ + o0 * d + o1 * h.x + o2 * x.x, oi + o1 * h.y + o2 * x.y);
    Eo[o] = ve;
    Oo[o] = vo;
    if (ty < tx) {
      const long long ot = off + (long long)j * N + i;
      Eo[ot] = make_double2(ve.x, -ve.y);
      Oo[ot] = make_double2(vo.x, -vo.y);
    }
  }
}

template <int BT>
__global__ void __launch_bounds__((BT / 16) * (BT / 16) * 64) __attribute__((amdgpu_waves_per_eu(3)))
exp_eo_kernel(const double2* H2, const double2* X2, const double2* X3, const double* coef, int N, double2* Eo,
              double2* Oo, int ntri, int tiles, int nbatch) {
  constexpr int LD = BT + 2;
  __shared__ double2 As[BK * LD];
  __shared__ double2 Be[BK * LD], Bo[BK * LD];
  int z, ty, tx;
  if (!xcd_tile(ntri, 1, nbatch, z, ty, tx)) return;
  {
    int r = tx, a = 0;
    while (r >= tiles - a) { r -= tiles - a; ++a; }
    ty = a;
    tx = a + r;
  }
  const int pm = partial_mode(N, N, ty, tx, tiles, tiles, BT, BT);
  if (pm == 1)
    exp_eo_body<BT, 1>(H2, X2, X3, coef, N, Eo, Oo, z, ty, tx, As, Be, Bo);
  else if (pm == 2)
    exp_eo_body<BT, 2>(H2, X2, X3, coef, N, Eo, Oo, z, ty, tx, As, Be, Bo);
  else
    exp_eo_body<BT, 0>(H2, X2, X3, coef, N, Eo, Oo, z, ty, tx, As, Be, Bo);
}

void launch_exp_eo(const double2* H2, const double2* X2, const double2* X3, const double* coef, int N, double2* Eo,
                   double2* Oo, int nmat, hipStream_t s) {
  constexpr int BT = 32;
  const int tiles = (N + BT - 1) / BT, ntri = tiles * (tiles + 1) / 2;
  const long long T = (long long)ntri * nmat;
  const int nblk = (int)((T + 7) / 8 * 8);
  hipLaunchKernelGGL((exp_eo_kernel<BT>), dim3(nblk), dim3((BT / 16) * (BT / 16) * 64), 0, s, H2, X2, X3, coef, N, Eo,
                     Oo, ntri, tiles, nmat);
  cfqmc_post_launch("exp_eo_kernel");
}

// ------------------------------------------------------------------ chan_apply

// Valley rotation of a channel: none (O^0 = 1, O^3 = tau_z are diagonal in the
// valley index), tau_x or tau_y. With U the matrix of eigenvectors of o_i
// (columns (1, 1)/sqrt2 and (1, -1)/sqrt2 for tau_x, (1, i)/sqrt2 and
// (1, -i)/sqrt2 for tau_y) the staged operand is S_a = sum_b w_ab M_b with
// w = sqrt2 conj(U) (left) or sqrt2 U (right), i.e. M_0 +- w M_1 with w = 1 or
// -+i, and the output is Y_0 = (T_0 + T_1)/2, Y_1 = z (T_0 - T_1)/2 with z = 1
// (tau_x), i (tau_y, left) or -i (tau_y, right): additions and swaps only.
enum { ROT_NONE = 0, ROT_X = 1, ROT_Y = 2 };

template <bool LEFT, int ROTK>
CF_DEV void rot_stage(double2 m0, double2 m1, double2& s0, double2& s1) {
  if (ROTK == ROT_X) {
    s0 = cadd(m0, m1);
    s1 = csub(m0, m1);
  } else {
    // w M_1 with w = -i (left) or +i (right): (-i)(x+iy) = y - ix ; (i)(x+iy) = -y + ix
    const double2 wm = LEFT ? make_double2(m1.y, -m1.x) : make_double2(-m1.y, m1.x);
    s0 = cadd(m0, wm);
    s1 = csub(m0, wm);
  }
}
template <bool LEFT, int ROTK>
CF_DEV double2 rot_out(double2 t0, double2 t1, int v) {
  if (v == 0) return make_double2(0.5 * (t0.x + t1.x), 0.5 * (t0.y + t1.y));
  const double2 d = make_double2(0.5 * (t0.x - t1.x), 0.5 * (t0.y - t1.y));
  if (ROTK == ROT_X) return d;
  return LEFT ? make_double2(-d.y, d.x) : make_double2(d.y, -d.x);   // i d or -i d
}

// BKC: k slab depth. DB: two LDS stages and one barrier per slab (the global
// loads of slab k+1 and the LDS stores into the other stage overlap the MFMAs
// of slab k); otherwise one stage with register prefetch and two barriers.
// OM: the input is 1 - M instead of M (left, non-rotating channel only).
// AM (FP32 path): 0 adds each slab's FP32 MFMA sum into FP64 registers (an
// FP64 accumulation point per slab); 1 runs the FP32 accumulators over the
// whole k range and converts them once in the epilogue, where the FP64 input
// is added back (correction form); 2 is 1 with three real products per
// complex k step (Gauss, as the FP64 path), combined in FP64 in the epilogue;
// 3 is 0 with the three-product slabs (combined in FP64 at each slab).
// Each thread keeps base pointers to its staging elements; a slab advances
// them by a constant.
// LDS bytes of one workgroup's operand tiles.
template <typename CT, int BM, int BN, int BKC, bool DB>
constexpr int chan_lds_bytes() {
  return (int)sizeof(typename cplx_t<CT>::type) * (DB ? 2 : 1) * 2 * BKC *
         (BM + (sizeof(CT) == 8 ? 2 : 4) + BN + (sizeof(CT) == 8 ? 2 : 4));
}

// The application for tile (ty, tx) of chain z; smem holds the workgroup's
// operand tiles (chan_lds_bytes).
// AM = 4 (FP64 only): the two valley products of a tile are split over twice
// the waves (one valley each, half the accumulator registers per wave); the
// rotating channels exchange the two halves through LDS in the epilogue.
// RM (FP64, 16 x 16 wave tiles; partial_mode): 1, the workgroup lies in the
// last row tile, which holds fewer than 16 valid rows, so that its waves either
// have no valid row or take mma_slab3_rows; 2, the same for the last column
// tile and mma_slab3_cols (whose accumulator layout the epilogue follows).
// Separate instantiations holding only that form, so that the register
// allocation of the other workgroups stays that of the 16x16x4 form.
template <typename CT, bool LEFT, int ROTK, bool OM, int BM, int BN, int WTM, int WTN, int BKC, bool DB, int AM,
          int RM = 0>
CF_DEV void chan_apply_body(const ChanArgs& c, int z, int ty, int tx, unsigned char* smem) {
  typedef typename cplx_t<CT>::type C2;
  constexpr bool VS = AM == 4;
  static_assert(!VS || sizeof(CT) == 8, "valley split: FP64 only");
  constexpr int WX = BN / (16 * WTN), WY = BM / (16 * WTM);
  constexpr int NT = WX * WY * 64 * (VS ? 2 : 1);
  constexpr int NS = DB ? 2 : 1;
  constexpr int LDA = BM + (sizeof(C2) == 16 ? 2 : 4), LDB = BN + (sizeof(C2) == 16 ? 2 : 4);
  C2 (*As)[2][BKC * LDA] = reinterpret_cast<C2 (*)[2][BKC * LDA]>(smem);
  C2 (*Bs)[2][BKC * LDB] = reinterpret_cast<C2 (*)[2][BKC * LDB]>(smem + sizeof(C2) * NS * 2 * BKC * LDA);
  const int m0 = ty * BM, n0 = tx * BN;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wt = VS ? wid % (WX * WY) : wid;   // wave tile
  const int va = VS ? wid / (WX * WY) : 0;     // valley of this wave (split form)
  const int wm0 = (wt / WX) * 16 * WTM, wn0 = (wt % WX) * 16 * WTN;
  constexpr bool CORR = sizeof(CT) == 4;   // correction form in the mixed path
  const int N = c.N;
  const double2* M = c.M + z * c.sM;
  const double2* X0 = c.X0 + z * c.sX;
  const double2* X1 = c.X1 + z * c.sX;
  const int rows = LEFT ? N : c.n_other;   // output rows of T
  const int cols = LEFT ? c.n_other : N;   // output cols of T

  auto mload = [&](int i, int j) -> double2 {
    double2 v = M[(long long)i * c.ldM + j];
    if (OM) { v.x = -v.x; v.y = -v.y; if (i == j) v.x += 1.0; }
    return v;
  };

  constexpr int EA = BM * BKC / NT, EB = BN * BKC / NT;
  static_assert(EA * NT == BM * BKC && EB * NT == BN * BKC, "tile / thread mismatch");
  // staging elements of this thread: A tile (m, k) with k fastest, B tile (k, n) with n fastest
  int am[EA], ak[EA], bn_[EB], bk[EB];
  const double2 *pa0[EA], *pb0[EB];
  bool arow[EA], bcol[EB];
  // the second valley's operand is the first one's plus a uniform offset
  const long long da = LEFT ? (long long)(X1 - X0) : (long long)N;
  const long long db = LEFT ? (long long)N * c.ldM : (long long)(X1 - X0);
#pragma unroll
  for (int e = 0; e < EA; ++e) {
    const int idx = tid + e * NT;
    ak[e] = idx % BKC;
    am[e] = idx / BKC;
    arow[e] = m0 + am[e] < rows;
    const int mr = arow[e] ? m0 + am[e] : 0;
    pa0[e] = LEFT ? X0 + (long long)mr * c.ldX + ak[e] : M + (long long)mr * c.ldM + ak[e];
  }
#pragma unroll
  for (int e = 0; e < EB; ++e) {
    const int idx = tid + e * NT;
    bn_[e] = idx % BN;
    bk[e] = idx / BN;
    bcol[e] = n0 + bn_[e] < cols;
    const int nc = bcol[e] ? n0 + bn_[e] : 0;
    pb0[e] = LEFT ? M + (long long)bk[e] * c.ldM + nc : X0 + (long long)bk[e] * c.ldX + nc;
  }
  // k advances along a row of A and down a column of B
  const long long bstep = LEFT ? (long long)c.ldM : (long long)c.ldX;

  double2 ra[EA][2], rb[EB][2];
  // bare loads; an out-of-range element reads k = 0 of its own row (A) or
  // column (B), which is inside the operand (the base pointers already carry
  // the thread's offset within the slab, which can exceed N when N < BKC), and
  // is zeroed when staged
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const bool ok = arow[e] && k0 + ak[e] < N;
      const long long o = ok ? k0 : -ak[e];
      ra[e][0] = pa0[e][o];
      ra[e][1] = pa0[e][o + da];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const bool ok = bcol[e] && k0 + bk[e] < N;
      const long long o = (long long)(ok ? k0 : -bk[e]) * bstep;
      rb[e][0] = pb0[e][o];
      rb[e][1] = pb0[e][o + db];
    }
  };
  const double2 zero2 = make_double2(0.0, 0.0);
  // fix up, rotate and store to LDS stage st
  auto stage = [&](int st, int k0) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      const bool ok = arow[e] && k0 + ak[e] < N;
      double2 v0 = ok ? ra[e][0] : zero2, v1 = ok ? ra[e][1] : zero2;
      const int m = am[e], k = ak[e];
      if (LEFT) {
        // X_a; correction form stages X_a - 1
        if (CORR && ok && m0 + m == k0 + k) { v0.x -= 1.0; v1.x -= 1.0; }
        As[st][0][k * LDA + m] = to_ct<CT>(v0);
        As[st][1][k * LDA + m] = to_ct<CT>(v1);
      } else {
        if (ROTK != ROT_NONE) {
          double2 s0, s1;
          rot_stage<false, ROTK>(v0, v1, s0, s1);
          As[st][0][k * LDA + m] = to_ct<CT>(s0);
          As[st][1][k * LDA + m] = to_ct<CT>(s1);
        } else {
          As[st][0][k * LDA + m] = to_ct<CT>(v0);
          As[st][1][k * LDA + m] = to_ct<CT>(v1);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      const bool ok = bcol[e] && k0 + bk[e] < N;
      double2 v0 = ok ? rb[e][0] : zero2, v1 = ok ? rb[e][1] : zero2;
      const int n = bn_[e], k = bk[e];
      if (LEFT) {
        if (OM && ok) {
          v0 = make_double2(-v0.x, -v0.y);
          v1 = make_double2(-v1.x, -v1.y);
          if (k0 + k == n0 + n) v0.x += 1.0;
          if (N + k0 + k == n0 + n) v1.x += 1.0;
        }
        if (ROTK != ROT_NONE) {
          double2 s0, s1;
          rot_stage<true, ROTK>(v0, v1, s0, s1);
          Bs[st][0][k * LDB + n] = to_ct<CT>(s0);
          Bs[st][1][k * LDB + n] = to_ct<CT>(s1);
        } else {
          Bs[st][0][k * LDB + n] = to_ct<CT>(v0);
          Bs[st][1][k * LDB + n] = to_ct<CT>(v1);
        }
      } else {
        if (CORR && ok && k0 + k == n0 + n) { v0.x -= 1.0; v1.x -= 1.0; }
        Bs[st][0][k * LDB + n] = to_ct<CT>(v0);
        Bs[st][1][k * LDB + n] = to_ct<CT>(v1);
      }
    }
  };
  Acc<double, WTM, WTN> acc[2];
  acc[0].zero();
  acc[1].zero();
  Acc3<WTM, WTN> acc3[2];
  acc3[0].zero();
  acc3[1].zero();
  Acc<float, WTM, WTN> acc32[2];
  acc32[0].zero();
  acc32[1].zero();
  Acc3F<WTM, WTN> acc3f[2];
  acc3f[0].zero();
  acc3f[1].zero();
  Acc3<WTM, WTN> accv;   // split form: this wave's valley
  accv.zero();
  const int mr = rows - m0 - wm0, nr = cols - n0 - wn0;
  auto mma = [&](int st, int k0) {
    if constexpr (VS) {
      mma_slab3<WTM, WTN, BKC>((const double2*)As[st][va], LDA, (const double2*)Bs[st][va], LDB, wm0, wn0, lane,
                               accv, mr, nr, N - k0);
      return;
    }
    if constexpr (RM != 0 && sizeof(CT) == 8 && WTM == 1 && WTN == 1) {
      if (mr > 0 && nr > 0) {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          if constexpr (RM == 1)
            mma_slab3_rows<BKC>((const double2*)As[st][a], LDA, (const double2*)Bs[st][a], LDB, wm0, wn0, lane,
                                acc3[a], mr, N - k0);
          else
            mma_slab3_cols<BKC>((const double2*)As[st][a], LDA, (const double2*)Bs[st][a], LDB, wm0, wn0, lane,
                                acc3[a], nr, N - k0);
        }
      }
      return;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      if constexpr (sizeof(CT) == 8) {
        mma_slab3<WTM, WTN, BKC>((const double2*)As[st][a], LDA, (const double2*)Bs[st][a], LDB, wm0, wn0, lane,
                                 acc3[a], mr, nr, N - k0);
      } else if constexpr (AM == 0) {
        Acc<float, WTM, WTN> a32;
        a32.zero();
        mma_slab<float, WTM, WTN, BKC>((const float2*)As[st][a], LDA, (const float2*)Bs[st][a], LDB, wm0, wn0, lane, a32,
                                       mr, nr, N - k0);
        flush(a32, acc[a]);
      } else if constexpr (AM == 1) {
        mma_slab<float, WTM, WTN, BKC>((const float2*)As[st][a], LDA, (const float2*)Bs[st][a], LDB, wm0, wn0, lane,
                                       acc32[a], mr, nr, N - k0);
      } else if constexpr (AM == 3) {
        // three-product slab, combined and added into FP64 registers per slab
        Acc3F<WTM, WTN> a3;
        a3.zero();
        mma_slab3f<WTM, WTN, BKC>((const float2*)As[st][a], LDA, (const float2*)Bs[st][a], LDB, wm0, wn0, lane, a3,
                                  mr, nr, N - k0);
        Acc<double, WTM, WTN> d;
        a3.to(d);
#pragma unroll
        for (int si = 0; si < WTM; ++si)
#pragma unroll
          for (int sj = 0; sj < WTN; ++sj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              acc[a].re[si][sj][r] += d.re[si][sj][r];
              acc[a].im[si][sj][r] += d.im[si][sj][r];
            }
      } else {
        mma_slab3f<WTM, WTN, BKC>((const float2*)As[st][a], LDA, (const float2*)Bs[st][a], LDB, wm0, wn0, lane,
                                  acc3f[a], mr, nr, N - k0);
      }
    }
  };
  fetch(0);
  if (DB) {
    stage(0, 0);
    __syncthreads();
    int cur = 0;
    for (int k0 = 0; k0 < N; k0 += BKC) {
      const bool more = k0 + BKC < N;
      if (more) fetch(k0 + BKC);
      mma(cur, k0);
      if (more) stage(cur ^ (NS - 1), k0 + BKC);
      __syncthreads();
      cur ^= (NS - 1);
    }
  } else {
    for (int k0 = 0; k0 < N; k0 += BKC) {
      stage(0, k0);
      __syncthreads();
      if (k0 + BKC < N) fetch(k0 + BKC);
      mma(0, k0);
      __syncthreads();
    }
  }
  if constexpr (VS) {
    Acc<double, WTM, WTN> av;
    accv.to(av);
    double2* Y = c.Y + z * c.sY;
    const double2* Cadd = c.Cadd ? c.Cadd + z * c.sC : nullptr;
    // rotating channels need both valleys' products for every output element:
    // exchange through the (no longer needed) operand tiles
    constexpr int PER = WX * WY * WTM * WTN * 4 * 64;
    static_assert(4 * PER * (int)sizeof(double) <= chan_lds_bytes<CT, BM, BN, BKC, DB>(), "exchange buffer");
    double* xr = reinterpret_cast<double*>(smem);
    double* xi = xr + 2 * PER;
    if constexpr (ROTK != ROT_NONE) {
      __syncthreads();
#pragma unroll
      for (int si = 0; si < WTM; ++si)
#pragma unroll
        for (int sj = 0; sj < WTN; ++sj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = (((wt * WTM + si) * WTN + sj) * 4 + r) * 64 + lane;
            xr[va * PER + e] = av.re[si][sj][r];
            xi[va * PER + e] = av.im[si][sj][r];
          }
      __syncthreads();
    }
#pragma unroll
    for (int si = 0; si < WTM; ++si)
#pragma unroll
      for (int sj = 0; sj < WTN; ++sj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = m0 + wm0 + si * 16 + out_row<CT>(lane, r);
          const int j = n0 + wn0 + sj * 16 + (lane & 15);
          if (i >= rows || j >= cols) continue;
          const double2 mine = make_double2(av.re[si][sj][r], av.im[si][sj][r]);
          double2 y = mine;
          if constexpr (ROTK != ROT_NONE) {
            const int e = (((wt * WTM + si) * WTN + sj) * 4 + r) * 64 + lane;
            const double2 other = make_double2(xr[(1 - va) * PER + e], xi[(1 - va) * PER + e]);
            y = rot_out<LEFT, ROTK>(va == 0 ? mine : other, va == 0 ? other : mine, va);
          }
          const int v = va;
          const long long off = LEFT ? (long long)(v * N + i) * c.ldY + j : (long long)i * c.ldY + v * N + j;
          if (Cadd) {
            const long long offc = LEFT ? (long long)(v * N + i) * c.ldC + j : (long long)i * c.ldC + v * N + j;
            y = cadd(y, Cadd[offc]);
          }
          Y[off] = y;
          if (c.Y2) c.Y2[z * c.sY + off] = y;
        }
    return;
  }
  if constexpr (sizeof(CT) == 8) {
    acc3[0].to(acc[0]);
    acc3[1].to(acc[1]);
  } else if constexpr (AM == 1) {
    flush(acc32[0], acc[0]);
    flush(acc32[1], acc[1]);
  } else if constexpr (AM == 2) {
    acc3f[0].to(acc[0]);
    acc3f[1].to(acc[1]);
  }
  // combine T_0, T_1 into the two valley blocks of the output
  double2* Y = c.Y + z * c.sY;
  const double2* Cadd = c.Cadd ? c.Cadd + z * c.sC : nullptr;
#pragma unroll
  for (int si = 0; si < WTM; ++si)
#pragma unroll
    for (int sj = 0; sj < WTN; ++sj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm0 + si * 16 + (RM == 2 ? 4 * ((lane >> 2) & 3) + (lane >> 4) : out_row<CT>(lane, r));
        const int j = n0 + wn0 + sj * 16 + (RM == 2 ? 4 * r + (lane & 3) : (lane & 15));
        if (i >= rows || j >= cols) continue;
        const double2 t0 = make_double2(acc[0].re[si][sj][r], acc[0].im[si][sj][r]);
        const double2 t1 = make_double2(acc[1].re[si][sj][r], acc[1].im[si][sj][r]);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          double2 y = ROTK != ROT_NONE ? rot_out<LEFT, ROTK>(t0, t1, v) : (v == 0 ? t0 : t1);
          const long long off = LEFT ? (long long)(v * N + i) * c.ldY + j : (long long)i * c.ldY + v * N + j;
          if (CORR) y = cadd(y, LEFT ? mload(v * N + i, j) : mload(i, v * N + j));
          if (Cadd) {
            const long long offc = LEFT ? (long long)(v * N + i) * c.ldC + j : (long long)i * c.ldC + v * N + j;
            y = cadd(y, Cadd[offc]);
          }
          Y[off] = y;
          if (c.Y2) c.Y2[z * c.sY + off] = y;
        }
      }
}

template <typename CT, bool LEFT, int ROTK, bool OM, int BM, int BN, int WTM, int WTN, int BKC, bool DB, int AM>
__global__ void __launch_bounds__((BM / (16 * WTM)) * (BN / (16 * WTN)) * 64 * (AM == 4 ? 2 : 1))
__attribute__((amdgpu_waves_per_eu(sizeof(CT) == 8 && AM != 4 && WTM == 1 && WTN == 1 ? 4 : 1)))
chan_apply_kernel(ChanArgs c, int tiles_x, int tiles_y, int nbatch) {
  __shared__ __align__(16) unsigned char smem[chan_lds_bytes<CT, BM, BN, BKC, DB>()];
  int z, ty, tx;
  if (!xcd_tile(tiles_x, tiles_y, nbatch, z, ty, tx)) return;
  // chains of the other precision class are computed by the companion launch
  if (c.chain_sel && c.chain_sel[z] != c.sel_want) return;
  if constexpr (sizeof(CT) == 8 && AM != 4 && WTM == 1 && WTN == 1) {
    const int pm = partial_mode(LEFT ? c.N : c.n_other, LEFT ? c.n_other : c.N, ty, tx, tiles_y, tiles_x, BM, BN);
    if (pm == 1) {
      chan_apply_body<CT, LEFT, ROTK, OM, BM, BN, WTM, WTN, BKC, DB, AM, 1>(c, z, ty, tx, smem);
      return;
    }
    if (pm == 2) {
      chan_apply_body<CT, LEFT, ROTK, OM, BM, BN, WTM, WTN, BKC, DB, AM, 2>(c, z, ty, tx, smem);
      return;
    }
  }
  chan_apply_body<CT, LEFT, ROTK, OM, BM, BN, WTM, WTN, BKC, DB, AM>(c, z, ty, tx, smem);
}

// Both precision classes of a precision-guarded context in one launch: the
// workgroups of a chain the guard runs in FP64 (chain_sel[z] = 1) take the FP64
// path, the others the FP32 correction form; same tile geometry, one LDS
// buffer sized for the larger of the two.
// RR: FP64 workgroups of a partial last row or column tile take the 4x4x4
// forms (partial_mode; the four-wave register budget only: they cost the
// compiler-allocated form a wave per SIMD).
template <bool LEFT, int ROTK, bool OM, int BM, int BN, int WTM, int WTN, int BKC, bool DB, int AM, bool RR>
CF_DEV void chan_apply_dual(const ChanArgs& c, int tiles_x, int tiles_y, int nbatch, unsigned char* smem) {
  int z, ty, tx;
  if (!xcd_tile(tiles_x, tiles_y, nbatch, z, ty, tx)) return;
  if (c.chain_sel[z]) {
    const int pm = RR && WTM == 1 && WTN == 1
                       ? partial_mode(LEFT ? c.N : c.n_other, LEFT ? c.n_other : c.N, ty, tx, tiles_y, tiles_x, BM, BN)
                       : 0;
    if (pm == 1)
      chan_apply_body<double, LEFT, ROTK, OM, BM, BN, WTM, WTN, BKC, DB, 0, 1>(c, z, ty, tx, smem);
    else if (pm == 2)
      chan_apply_body<double, LEFT, ROTK, OM, BM, BN, WTM, WTN, BKC, DB, 0, 2>(c, z, ty, tx, smem);
    else
      chan_apply_body<double, LEFT, ROTK, OM, BM, BN, WTM, WTN, BKC, DB, 0>(c, z, ty, tx, smem);
  } else
    chan_apply_body<float, LEFT, ROTK, OM, BM, BN, WTM, WTN, BKC, DB, AM>(c, z, ty, tx, smem);
}
template <int BM, int BN, int BKC, bool DB>
constexpr int dual_lds_bytes() {
  return chan_lds_bytes<double, BM, BN, BKC, DB>() > chan_lds_bytes<float, BM, BN, BKC, DB>()
             ? chan_lds_bytes<double, BM, BN, BKC, DB>()
             : chan_lds_bytes<float, BM, BN, BKC, DB>();
}
// registers as the compiler allocates them (both paths: three waves per SIMD)
template <bool LEFT, int ROTK, bool OM, int BM, int BN, int WTM, int WTN, int BKC, bool DB, int AM>
__global__ void __launch_bounds__((BM / (16 * WTM)) * (BN / (16 * WTN)) * 64)
chan_apply_dual_kernel(ChanArgs c, int tiles_x, int tiles_y, int nbatch) {
  __shared__ __align__(16) unsigned char smem[dual_lds_bytes<BM, BN, BKC, DB>()];
  chan_apply_dual<LEFT, ROTK, OM, BM, BN, WTM, WTN, BKC, DB, AM, false>(c, tiles_x, tiles_y, nbatch, smem);
}
// held to four waves per SIMD (128 registers; the compiler spills a few)
template <bool LEFT, int ROTK, bool OM, int BM, int BN, int WTM, int WTN, int BKC, bool DB, int AM>
__global__ void __launch_bounds__((BM / (16 * WTM)) * (BN / (16 * WTN)) * 64) __attribute__((amdgpu_waves_per_eu(4)))
chan_apply_dual4_kernel(ChanArgs c, int tiles_x, int tiles_y, int nbatch) {
  __shared__ __align__(16) unsigned char smem[dual_lds_bytes<BM, BN, BKC, DB>()];
  chan_apply_dual<LEFT, ROTK, OM, BM, BN, WTM, WTN, BKC, DB, AM, true>(c, tiles_x, tiles_y, nbatch, smem);
}

// ------------------------------------------------------------------ launchers

template <typename CT, int BM, int BN, int WTM, int WTN>
static void run_gemm(const GemmArgs& g0, int nbatch, hipStream_t s) {
  constexpr int NT = (BM / (16 * WTM)) * (BN / (16 * WTN)) * 64;
  GemmArgs g = g0;
  int tx = (g.N + BN - 1) / BN, ty = (g.M + BM - 1) / BM;
  if (g.herm) {
    if (BM != BN || g.M != g.N || g.mode != GEMM_NORMAL) {
      std::fprintf(stderr, "zgemm: Hermitian output needs square tiles and a square GEMM_NORMAL product\n");
      std::abort();
    }
    g.herm = tx;
    tx = tx * (tx + 1) / 2;
    ty = 1;
  }
  const long long T = (long long)tx * ty * nbatch;
  const int nblk = (int)((T + 7) / 8 * 8);
  hipLaunchKernelGGL((zgemm_kernel<CT, BM, BN, WTM, WTN>), dim3(nblk), dim3(NT), 0, s, g, tx, ty, nbatch);
  cfqmc_post_launch("zgemm_kernel");
}

void launch_zgemm(const GemmArgs& g, int nbatch, int mixed, int cfg, hipStream_t s) {
  if (nbatch <= 0 || g.M <= 0 || g.N <= 0) return;
  if (mixed) {
    switch (cfg) {
      case 0: run_gemm<float, 16, 16, 1, 1>(g, nbatch, s); break;
      case 1: run_gemm<float, 32, 32, 1, 1>(g, nbatch, s); break;
      case 2: run_gemm<float, 32, 32, 2, 2>(g, nbatch, s); break;
      default: run_gemm<float, 64, 64, 2, 2>(g, nbatch, s); break;
    }
  } else {
    switch (cfg) {
      case 0: run_gemm<double, 16, 16, 1, 1>(g, nbatch, s); break;
      case 1: run_gemm<double, 32, 32, 1, 1>(g, nbatch, s); break;
      case 2: run_gemm<double, 32, 32, 2, 2>(g, nbatch, s); break;
      default: run_gemm<double, 64, 64, 2, 2>(g, nbatch, s); break;
    }
  }
}

template <typename CT, bool LEFT, int ROTK, bool OM, int BM, int BN, int WTM, int WTN, int BKC, bool DB, int AM>
static void run_chan(const ChanArgs& c, int nbatch, hipStream_t s) {
  constexpr int NT = (BM / (16 * WTM)) * (BN / (16 * WTN)) * 64 * (AM == 4 ? 2 : 1);
  const int rows = LEFT ? c.N : c.n_other, cols = LEFT ? c.n_other : c.N;
  const int tx = (cols + BN - 1) / BN, ty = (rows + BM - 1) / BM;
  const long long T = (long long)tx * ty * nbatch;
  const int nblk = (int)((T + 7) / 8 * 8);
  hipLaunchKernelGGL((chan_apply_kernel<CT, LEFT, ROTK, OM, BM, BN, WTM, WTN, BKC, DB, AM>), dim3(nblk), dim3(NT), 0,
                     s, c, tx, ty, nbatch); cfqmc_post_launch("chan_apply_kernel");
}

template <typename CT, int BM, int BN, int WTM, int WTN, int BKC, bool DB, int AM = 0>
static void run_chan_any(const ChanArgs& c, int left, int rot, int nbatch, hipStream_t s) {
  // the accumulation modes concern the FP32 path only (FP64 keeps its one form);
  // AM = 4 is the FP64 valley split (FP32: accumulation mode 0)
  constexpr int F = sizeof(CT) == 8 ? (AM == 4 ? 4 : 0) : (AM == 4 ? 0 : AM);
  if (left) {
    if (rot == ROT_X) run_chan<CT, true, ROT_X, false, BM, BN, WTM, WTN, BKC, DB, F>(c, nbatch, s);
    else if (rot == ROT_Y) run_chan<CT, true, ROT_Y, false, BM, BN, WTM, WTN, BKC, DB, F>(c, nbatch, s);
    else if (c.one_minus) run_chan<CT, true, ROT_NONE, true, BM, BN, WTM, WTN, BKC, DB, F>(c, nbatch, s);
    else run_chan<CT, true, ROT_NONE, false, BM, BN, WTM, WTN, BKC, DB, F>(c, nbatch, s);
  } else {
    if (rot == ROT_X) run_chan<CT, false, ROT_X, false, BM, BN, WTM, WTN, BKC, DB, F>(c, nbatch, s);
    else if (rot == ROT_Y) run_chan<CT, false, ROT_Y, false, BM, BN, WTM, WTN, BKC, DB, F>(c, nbatch, s);
    else run_chan<CT, false, ROT_NONE, false, BM, BN, WTM, WTN, BKC, DB, F>(c, nbatch, s);
  }
}

template <typename CT>
static void chan_cfg(const ChanArgs& c, int left, int rot, int nbatch, int cfg, hipStream_t s) {
  switch (cfg) {
    case 0: run_chan_any<CT, 16, 16, 1, 1, 16, false>(c, left, rot, nbatch, s); break;
    case 1: run_chan_any<CT, 32, 32, 1, 1, 16, false>(c, left, rot, nbatch, s); break;
    case 2: run_chan_any<CT, 32, 32, 1, 1, 8, true>(c, left, rot, nbatch, s); break;
    case 3: run_chan_any<CT, 32, 32, 1, 1, 16, true>(c, left, rot, nbatch, s); break;
    case 4: run_chan_any<CT, 64, 32, 1, 1, 16, true>(c, left, rot, nbatch, s); break;
    case 5: run_chan_any<CT, 32, 64, 1, 1, 16, true>(c, left, rot, nbatch, s); break;
    case 6: run_chan_any<CT, 64, 64, 2, 2, 8, true>(c, left, rot, nbatch, s); break;
    case 7: run_chan_any<CT, 16, 16, 1, 1, 8, true>(c, left, rot, nbatch, s); break;
    // FP32 accumulation over the whole k range (FP64 configurations: the same tiles)
    case 8: run_chan_any<CT, 32, 32, 1, 1, 16, false, 1>(c, left, rot, nbatch, s); break;
    case 9: run_chan_any<CT, 64, 64, 2, 2, 16, true, 1>(c, left, rot, nbatch, s); break;
    case 10: run_chan_any<CT, 64, 32, 2, 1, 16, true, 1>(c, left, rot, nbatch, s); break;
    case 11: run_chan_any<CT, 32, 64, 1, 2, 16, true, 1>(c, left, rot, nbatch, s); break;
    // FP32 three-product form, FP32 accumulation
    case 12: run_chan_any<CT, 32, 32, 1, 1, 16, false, 2>(c, left, rot, nbatch, s); break;
    case 13: run_chan_any<CT, 64, 32, 2, 1, 16, true, 2>(c, left, rot, nbatch, s); break;
    // FP32 three-product slabs with an FP64 accumulation point per slab
    case 14: run_chan_any<CT, 32, 32, 1, 1, 16, false, 3>(c, left, rot, nbatch, s); break;
    // 8- and 16-wave workgroups of 16 x 16 wave tiles, one LDS stage: each staged
    // operand element serves more waves for the same LDS per wave
    case 15: run_chan_any<CT, 64, 32, 1, 1, 16, false>(c, left, rot, nbatch, s); break;
    case 16: run_chan_any<CT, 64, 64, 1, 1, 16, false>(c, left, rot, nbatch, s); break;
    case 17: run_chan_any<CT, 64, 32, 1, 1, 16, false, 2>(c, left, rot, nbatch, s); break;
    case 18: run_chan_any<CT, 64, 64, 1, 1, 16, false, 2>(c, left, rot, nbatch, s); break;
    // FP64: the 32 x 32 tile with its two valley products on eight waves
    default: run_chan_any<CT, 32, 32, 1, 1, 16, false, 4>(c, left, rot, nbatch, s); break;
  }
}

void launch_chan_apply(const ChanArgs& c, int left, int rot, int nbatch, int mixed, int cfg, hipStream_t s) {
  if (nbatch <= 0) return;
  if (mixed) chan_cfg<float>(c, left, rot, nbatch, cfg, s);
  else chan_cfg<double>(c, left, rot, nbatch, cfg, s);
}

template <bool LEFT, int ROTK, bool OM, int AM, bool W4>
static void run_chan_dual(const ChanArgs& c, int nbatch, hipStream_t s) {
  constexpr int BM = 32, BN = 32;
  const int rows = LEFT ? c.N : c.n_other, cols = LEFT ? c.n_other : c.N;
  const int tx = (cols + BN - 1) / BN, ty = (rows + BM - 1) / BM;
  const long long T = (long long)tx * ty * nbatch;
  const int nblk = (int)((T + 7) / 8 * 8);
  if (W4)
    hipLaunchKernelGGL((chan_apply_dual4_kernel<LEFT, ROTK, OM, BM, BN, 1, 1, 16, false, AM>), dim3(nblk), dim3(256),
                       0, s, c, tx, ty, nbatch);
  else
    hipLaunchKernelGGL((chan_apply_dual_kernel<LEFT, ROTK, OM, BM, BN, 1, 1, 16, false, AM>), dim3(nblk), dim3(256),
                       0, s, c, tx, ty, nbatch);
  cfqmc_post_launch("chan_apply_dual_kernel");
}

template <int AM, bool W4>
static void run_chan_dual_any(const ChanArgs& c, int left, int rot, int nbatch, hipStream_t s) {
  if (left) {
    if (rot == ROT_X) run_chan_dual<true, ROT_X, false, AM, W4>(c, nbatch, s);
    else if (rot == ROT_Y) run_chan_dual<true, ROT_Y, false, AM, W4>(c, nbatch, s);
    else if (c.one_minus) run_chan_dual<true, ROT_NONE, true, AM, W4>(c, nbatch, s);
    else run_chan_dual<true, ROT_NONE, false, AM, W4>(c, nbatch, s);
  } else {
    if (rot == ROT_X) run_chan_dual<false, ROT_X, false, AM, W4>(c, nbatch, s);
    else if (rot == ROT_Y) run_chan_dual<false, ROT_Y, false, AM, W4>(c, nbatch, s);
    else run_chan_dual<false, ROT_NONE, false, AM, W4>(c, nbatch, s);
  }
}

// Configurations 1 (FP64 accumulation points) and 12 (three-product FP32
// accumulation) have single-launch forms; every FP64 configuration of their
// 32 x 32 single-stage tile (1, 8, 12, 14, 19) can join them.
bool launch_chan_apply_dual(const ChanArgs& c, int left, int rot, int nbatch, int cfg32, int cfg64, int variant,
                            hipStream_t s) {
  const bool geo64 = cfg64 == 1 || cfg64 == 8 || cfg64 == 12 || cfg64 == 14 || cfg64 == 19;
  if ((cfg32 != 1 && cfg32 != 12) || !geo64 || !c.chain_sel || variant < 1 || variant > 2) return false;
  if (nbatch <= 0) return true;
  const bool w4 = variant == 2;
  if (cfg32 == 1) {
    if (w4) run_chan_dual_any<0, true>(c, left, rot, nbatch, s);
    else run_chan_dual_any<0, false>(c, left, rot, nbatch, s);
  } else {
    if (w4) run_chan_dual_any<2, true>(c, left, rot, nbatch, s);
    else run_chan_dual_any<2, false>(c, left, rot, nbatch, s);
  }
  return true;
}
