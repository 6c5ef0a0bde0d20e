// Float64 matrix-core (v_mfma_f64_16x16x4) tiles of the library's GEMMs, shared by k_gemm_f64.hip,
// the persistent batch kernel and the merge products of the tridiagonal eigensolver.
//
// Block tile 64 x 64 x 16, 256 threads = 4 waves in a 2 x 2 arrangement, each wave owning a
// 32 x 32 sub-tile = 2 x 2 MFMA blocks of 16 x 16.  Operands are staged through LDS stored
// k-major ([k][m] and [k][n]), which is the order in which the f64 MFMA consumes them (lane l
// supplies A[m = l%16][k = l/16] and B[k = l/16][n = l%16]; the result element (l/16 + 4*j, l%16)
// sits in component j of lane l).  Register prefetch of the next k-slab overlaps global loads
// with the matrix-core work.
#pragma once
#include "common.h"

namespace pnof {
namespace f64t {

constexpr int TM = 64, TN = 64, TK = 16, LPAD = 2;

struct F64Smem {
  double a[TK][TM + LPAD];
  double b[TK][TN + LPAD];
};

// Strided view helper: element (r, k) of an operand, with r the output-side index.
template <bool RCONTIG>
__device__ __forceinline__ void load_slab(const double* __restrict__ P, long long sr, long long sk,
                                          int R, int K, int r0, int k0, double (&reg)[4]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int r, k;
    if (RCONTIG) { r = t & 63; k = (t >> 6) + 4 * i; }
    else         { r = t >> 2; k = ((t & 3) << 2) + i; }
    const int gr = r0 + r, gk = k0 + k;
    reg[i] = (gr < R && gk < K) ? P[(long long)gr * sr + (long long)gk * sk] : 0.0;
  }
}

template <bool RCONTIG>
__device__ __forceinline__ void store_slab(double (*S)[TM + LPAD], const double (&reg)[4]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int r, k;
    if (RCONTIG) { r = t & 63; k = (t >> 6) + 4 * i; }
    else         { r = t >> 2; k = ((t & 3) << 2) + i; }
    S[k][r] = reg[i];
  }
}

// acc[mi][ni] += A(m0.., :) B(:, n0..) over k in [kb, ke).
template <bool AM, bool BN>
__device__ __forceinline__ void tile_f64(F64Smem& sm, const double* __restrict__ A, long long sam,
                                         long long sak, const double* __restrict__ B, long long sbk,
                                         long long sbn, int M, int N, int kb, int ke, int m0, int n0,
                                         f64x4 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int K = ke;
  double ra[4], rb[4];
  load_slab<AM>(A, sam, sak, M, K, m0, kb, ra);
  load_slab<BN>(B, sbn, sbk, N, K, n0, kb, rb);
  for (int k0 = kb; k0 < ke; k0 += TK) {
    __syncthreads();
    store_slab<AM>(sm.a, ra);
    store_slab<BN>(sm.b, rb);
    __syncthreads();
    if (k0 + TK < K) {
      load_slab<AM>(A, sam, sak, M, K, m0, k0 + TK, ra);
      load_slab<BN>(B, sbn, sbk, N, K, n0, k0 + TK, rb);
    }
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a0 = sm.a[kr][wm + (lane & 15)], a1 = sm.a[kr][wm + 16 + (lane & 15)];
      double b0 = sm.b[kr][wn + (lane & 15)], b1 = sm.b[kr][wn + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
}

__device__ __forceinline__ void zero_acc(f64x4 (&acc)[2][2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
}

// Row / column of component j of acc[mi][ni] relative to the block tile origin.
__device__ __forceinline__ int acc_row(int mi, int j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave >> 1) * 32 + mi * 16 + (lane >> 4) + 4 * j;
}
__device__ __forceinline__ int acc_col(int ni) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave & 1) * 32 + ni * 16 + (lane & 15);
}


// Tile t of product g of a grouped GEMM (C = alpha A B + beta C with g's strides); tiles beyond the
// product's extent do nothing.
template <bool AM, bool BN>
__device__ __forceinline__ void grouped_tile(const F64Gemm& g, int t, F64Smem& sm) {
  const int tiles_n = (g.N + TN - 1) / TN;
  if (t >= tiles_n * ((g.M + TM - 1) / TM)) return;
  const int m0 = (t / tiles_n) * TM, n0 = (t % tiles_n) * TN;
  f64x4 acc[2][2];
  zero_acc(acc);
  tile_f64<AM, BN>(sm, g.A, g.sam, g.sak, g.B, g.sbk, g.sbn, g.M, g.N, 0, g.K, m0, n0, acc);
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + acc_row(mi, j), n = n0 + acc_col(ni);
        if (m < g.M && n < g.N) {
          double* c = g.C + (long long)m * g.scm + (long long)n * g.scn;
          *c = g.alpha * acc[mi][ni][j] + (g.beta != 0.0 ? g.beta * *c : 0.0);
        }
      }
}
// Tiles of product g.
__host__ __device__ inline int grouped_tiles(int M, int N) { return ((M + TM - 1) / TM) * ((N + TN - 1) / TN); }


// Finer tile for single products: block 64 x 32 (4 waves of 32 x 16, each two 16 x 16 MFMA
// blocks), k-slabs of 16 through two LDS stages, each slab loaded into registers two slabs ahead of
// its multiplication; one barrier per slab separates the writes of one stage from the reads of the
// other.
namespace wide {
constexpr int BM = 64, BNT = 32, BK = 16, PAD = 2;
struct Smem {
  double a[2][BK][BM + PAD];
  double b[2][BK][BNT + PAD];
};
// A slab (BM x BK, 4 per thread): m contiguous (AM) or k contiguous.
template <bool AM>
__device__ __forceinline__ void load_a(const double* __restrict__ A, long long sam, long long sak, int M, int K, int m0,
                                       int k0, double (&r)[BK / 4]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < BK / 4; ++i) {
    const int m = AM ? (t & 63) : (t >> 2), k = AM ? ((t >> 6) + 4 * i) : ((t & 3) * (BK / 4) + i);
    const int gm = m0 + m, gk = k0 + k;
    r[i] = (gm < M && gk < K) ? A[(long long)gm * sam + (long long)gk * sak] : 0.0;
  }
}
template <bool AM>
__device__ __forceinline__ void store_a(double (*S)[BM + PAD], const double (&r)[BK / 4]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < BK / 4; ++i) {
    const int m = AM ? (t & 63) : (t >> 2), k = AM ? ((t >> 6) + 4 * i) : ((t & 3) * (BK / 4) + i);
    S[k][m] = r[i];
  }
}
// B slab (BK x BNT, 2 per thread): n contiguous (BN) or k contiguous.
template <bool BN>
__device__ __forceinline__ void load_b(const double* __restrict__ B, long long sbk, long long sbn, int N, int K, int n0,
                                       int k0, double (&r)[BK / 8]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < BK / 8; ++i) {
    const int n = BN ? (t & 31) : (t >> 3), k = BN ? ((t >> 5) + 8 * i) : ((t & 7) * (BK / 8) + i);
    const int gn = n0 + n, gk = k0 + k;
    r[i] = (gn < N && gk < K) ? B[(long long)gk * sbk + (long long)gn * sbn] : 0.0;
  }
}
template <bool BN>
__device__ __forceinline__ void store_b(double (*S)[BNT + PAD], const double (&r)[BK / 8]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < BK / 8; ++i) {
    const int n = BN ? (t & 31) : (t >> 3), k = BN ? ((t >> 5) + 8 * i) : ((t & 7) * (BK / 8) + i);
    S[k][n] = r[i];
  }
}



// acc[mi] (rows wide_row(mi, j), column wide_col() of the tile at (m0, n0)) = A(m0.., :) B(:, n0..)
// over k in [0, K).  Every thread of the block must call it (it synchronises the block).
template <bool AM, bool BN>
__device__ __forceinline__ void wide_tile(Smem& sm, const double* __restrict__ A, long long sam, long long sak,
                                          const double* __restrict__ B, long long sbk, long long sbn, int M, int N,
                                          int K, int m0, int n0, f64x4 (&acc)[2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 16;
  acc[0] = f64x4{0.0, 0.0, 0.0, 0.0};
  acc[1] = f64x4{0.0, 0.0, 0.0, 0.0};
  // slab j travels in register set j % 2, loaded two slabs ahead of its multiplication; LDS stage
  // j % 2 holds it while it is multiplied
  double ra[2][BK / 4], rb[2][BK / 8];
  const int ns = (K + BK - 1) / BK;
  auto mul = [&](int st) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      const double a0 = sm.a[st][kr][wm + (lane & 15)], a1 = sm.a[st][kr][wm + 16 + (lane & 15)];
      const double b0 = sm.b[st][kr][wn + (lane & 15)];
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1], 0, 0, 0);
    }
  };
  load_a<AM>(A, sam, sak, M, K, m0, 0, ra[0]);
  load_b<BN>(B, sbk, sbn, N, K, n0, 0, rb[0]);
  store_a<AM>(sm.a[0], ra[0]);
  store_b<BN>(sm.b[0], rb[0]);
  if (1 < ns) {
    load_a<AM>(A, sam, sak, M, K, m0, BK, ra[1]);
    load_b<BN>(B, sbk, sbn, N, K, n0, BK, rb[1]);
  }
  __syncthreads();
  for (int s0 = 0; s0 < ns; s0 += 2) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int ss = s0 + d;
      if (ss < ns) {
        if (ss + 2 < ns) {
          load_a<AM>(A, sam, sak, M, K, m0, (ss + 2) * BK, ra[d]);
          load_b<BN>(B, sbk, sbn, N, K, n0, (ss + 2) * BK, rb[d]);
        }
        mul(d);
        if (ss + 1 < ns) {
          store_a<AM>(sm.a[d ^ 1], ra[d ^ 1]);
          store_b<BN>(sm.b[d ^ 1], rb[d ^ 1]);
        }
        __syncthreads();
      }
    }
  }
}
// Row / column (relative to the tile origin) of component j of acc[mi] of wide_tile.
__device__ __forceinline__ int wide_row(int mi, int j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave >> 1) * 32 + mi * 16 + (lane >> 4) + 4 * j;
}
__device__ __forceinline__ int wide_col() {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave & 1) * 16 + (lane & 15);
}
}  // namespace wide

}  // namespace f64t
}  // namespace pnof
