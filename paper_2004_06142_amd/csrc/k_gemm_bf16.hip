// bfloat16 matrix-core (v_mfma_f32_16x16x32_bf16) contractions with float32 accumulation.
//
// Every product here is "NT": both operands are stored with the contraction index k contiguous
// (A row m = A[m*lda + k], B row n = B[n*ldb + k]), which is the order in which one MFMA lane
// consumes eight consecutive k values.  An operand may be carried as a hi + lo pair of bf16
// values (x ~= hi + lo to about 16 significant bits); the accumulator then receives
//   terms = 1: hi*hi
//   terms = 2: Ahi*Bhi + Alo*Bhi                  (B exact in bf16)
//   terms = 3: Ahi*Bhi + Ahi*Blo + Alo*Bhi        (the lo*lo product is below float32 rounding)
// Block tile 128 x 128 x 32, 256 threads = 4 waves in a 2 x 2 arrangement, each wave owning
// 64 x 64 = 4 x 4 MFMA blocks; operands are staged through LDS rows padded by 16 bytes, with
// register prefetch of the next k-slab.  MFMA lane layout: lane l supplies row l%16 and the
// eight k values 8*(l/16)..8*(l/16)+7; result element (4*(l/16)+j, l%16) is component j.
#include "common.h"

namespace pnof {
namespace {

constexpr int BM = 128, BN = 128, BK = 32, KP = BK + 8;  // LDS row pitch in bf16 elements

struct Operand {
  const u16* hi;
  const u16* lo;
  long long ld;     // elements between rows
  int rows;         // valid rows
  int K;            // valid k
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// One 16-byte chunk (8 bf16) of row r, k in [k, k+8); zeros outside the valid region.
__device__ __forceinline__ u32x4 load_chunk(const u16* __restrict__ p, long long ld, int rows, int K,
                                            int r, int k) {
  u32x4 v = {0u, 0u, 0u, 0u};
  if (r >= rows) return v;
  const u16* src = p + (long long)r * ld + k;
  if (k + 8 <= K && ((ld & 7) == 0) && ((((uintptr_t)p) & 15) == 0)) {
    v = *reinterpret_cast<const u32x4*>(src);
  } else {
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 8; ++i)
      if (k + i < K) w[i >> 1] |= ((uint32_t)src[i]) << (16 * (i & 1));
    v = u32x4{w[0], w[1], w[2], w[3]};
  }
  return v;
}

struct Smem {
  u16 a[2][BM][KP];
  u16 b[2][BN][KP];
};

template <int TERMS, bool ALO, bool BLO>
struct Tile {
  u32x4 ra[2][2], rb[2][2];  // [hi/lo][chunk]

  __device__ __forceinline__ void load(const Operand& A, const Operand& B, int m0, int n0, int k0) {
    const int t = threadIdx.x;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int idx = t + 256 * c;          // 512 chunks = 128 rows x 4 chunks
      const int r = idx >> 2, kc = (idx & 3) * 8;
      ra[0][c] = load_chunk(A.hi, A.ld, A.rows, A.K, m0 + r, k0 + kc);
      if (ALO) ra[1][c] = load_chunk(A.lo, A.ld, A.rows, A.K, m0 + r, k0 + kc);
      rb[0][c] = load_chunk(B.hi, B.ld, B.rows, B.K, n0 + r, k0 + kc);
      if (BLO) rb[1][c] = load_chunk(B.lo, B.ld, B.rows, B.K, n0 + r, k0 + kc);
    }
  }
  __device__ __forceinline__ void store(Smem& sm) {
    const int t = threadIdx.x;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int idx = t + 256 * c;
      const int r = idx >> 2, kc = (idx & 3) * 8;
      *reinterpret_cast<u32x4*>(&sm.a[0][r][kc]) = ra[0][c];
      if (ALO) *reinterpret_cast<u32x4*>(&sm.a[1][r][kc]) = ra[1][c];
      *reinterpret_cast<u32x4*>(&sm.b[0][r][kc]) = rb[0][c];
      if (BLO) *reinterpret_cast<u32x4*>(&sm.b[1][r][kc]) = rb[1][c];
    }
  }
};

__device__ __forceinline__ bf16x8 frag(const u16* p) {
  return *reinterpret_cast<const bf16x8*>(p);
}

// acc += A(m0.., :) B(n0.., :)^T over k in [0, K).
template <int TERMS, bool ALO, bool BLO>
__device__ __forceinline__ void tile_bf16(Smem& sm, const Operand& A, const Operand& B, int m0,
                                          int n0, f32x4 (&acc)[4][4]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int K = A.K;
  Tile<TERMS, ALO, BLO> tl;
  tl.load(A, B, m0, n0, 0);
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    tl.store(sm);
    __syncthreads();
    if (k0 + BK < K) tl.load(A, B, m0, n0, k0 + BK);
    bf16x8 ah[4], bh[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ah[i] = frag(&sm.a[0][wm + i * 16 + fr][fk]);
      bh[i] = frag(&sm.b[0][wn + i * 16 + fr][fk]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
    if (TERMS >= 2) {
      if (BLO) {
        bf16x8 bl[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) bl[j] = frag(&sm.b[1][wn + j * 16 + fr][fk]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
      }
      if (ALO) {
        bf16x8 al[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) al[i] = frag(&sm.a[1][wm + i * 16 + fr][fk]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
      }
    }
  }
}

__device__ __forceinline__ void zero4(f32x4 (&acc)[4][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
}

__device__ __forceinline__ int row_of(int i, int j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave >> 1) * 64 + i * 16 + 4 * (lane >> 4) + j;
}
__device__ __forceinline__ int col_of(int jn) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave & 1) * 64 + jn * 16 + (lane & 15);
}

__device__ __forceinline__ void tri_tile(int t, int& tm, int& tn) {
  int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  tm = r;
  tn = t - r * (r + 1) / 2;
}

// gemm1: XT_P[p][mu] = sum_nu Ct[p][nu] B_P[mu][nu]; written split as XT (p-major) and X (mu-major).
template <int TERMS, bool BLO>
__global__ __launch_bounds__(256) void gemm1_kernel(int nbf, int nact, const u16* __restrict__ ct_hi,
                                                    const u16* __restrict__ ct_lo, int ldk,
                                                    const u16* __restrict__ b_hi,
                                                    const u16* __restrict__ b_lo, long long bstride,
                                                    int ldb, u16* __restrict__ xt_hi,
                                                    u16* __restrict__ xt_lo, int ldx,
                                                    u16* __restrict__ x_hi, u16* __restrict__ x_lo,
                                                    int ldxx) {
  __shared__ Smem sm;
  const int tiles_n = (nbf + BN - 1) / BN;
  const int m0 = (blockIdx.x / tiles_n) * BM, n0 = (blockIdx.x % tiles_n) * BN;
  const long long P = blockIdx.y;
  Operand A{ct_hi, ct_lo, ldk, nact, nbf};
  Operand B{b_hi + P * bstride, BLO ? b_lo + P * bstride : nullptr, ldb, nbf, nbf};
  f32x4 acc[4][4];
  zero4(acc);
  tile_bf16<TERMS, (TERMS >= 2), BLO>(sm, A, B, m0, n0, acc);
  u16* XTh = xt_hi + P * (long long)nact * ldx;
  u16* XTl = xt_lo ? xt_lo + P * (long long)nact * ldx : nullptr;
  u16* Xh = x_hi + P * (long long)nbf * ldxx;
  u16* Xl = x_lo ? x_lo + P * (long long)nbf * ldxx : nullptr;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jn = 0; jn < 4; ++jn) {
      const int mu = n0 + col_of(jn);
      const int pb = m0 + row_of(i, 0);
      if (mu >= nbf) continue;
      u16 h[4], l[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (TERMS == 1) { h[j] = f32_to_bf16_bits(acc[i][jn][j]); l[j] = 0; }
        else split_f32(acc[i][jn][j], h[j], l[j]);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = pb + j;
        if (p < nact) {
          XTh[(long long)p * ldx + mu] = h[j];
          if (XTl) XTl[(long long)p * ldx + mu] = l[j];
        }
      }
      if (pb + 3 < nact) {  // four consecutive p of row mu: one 8-byte store per array
        uint2 vh = {(uint32_t)h[0] | ((uint32_t)h[1] << 16), (uint32_t)h[2] | ((uint32_t)h[3] << 16)};
        *reinterpret_cast<uint2*>(&Xh[(long long)mu * ldxx + pb]) = vh;
        if (Xl) {
          uint2 vl = {(uint32_t)l[0] | ((uint32_t)l[1] << 16), (uint32_t)l[2] | ((uint32_t)l[3] << 16)};
          *reinterpret_cast<uint2*>(&Xl[(long long)mu * ldxx + pb]) = vl;
        }
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (pb + j < nact) {
            Xh[(long long)mu * ldxx + pb + j] = h[j];
            if (Xl) Xl[(long long)mu * ldxx + pb + j] = l[j];
          }
      }
    }
}

// gemm2: b_P = Ct XT_P^T on lower tiles; Kpart[s] += sum_{P in s} b^2 (lower triangle, summed over
// the successive P-chunks of one call), D[P][p] = b_pp,
// W_P = b o beta (symmetric, each unordered pair written once, split hi/lo).
template <int TERMS>
__global__ __launch_bounds__(256) void gemm2_kernel(int nbf, int nact, int np, int nsplit,
                                                    const u16* __restrict__ ct_hi,
                                                    const u16* __restrict__ ct_lo, int ldk,
                                                    const u16* __restrict__ xt_hi,
                                                    const u16* __restrict__ xt_lo, int ldx,
                                                    const float* __restrict__ beta32,
                                                    double* __restrict__ Kpart,
                                                    double* __restrict__ Dc,
                                                    u16* __restrict__ w_hi, u16* __restrict__ w_lo,
                                                    int ldw) {
  __shared__ Smem sm;
  int tm, tn;
  tri_tile(blockIdx.x, tm, tn);
  const int m0 = tm * BM, n0 = tn * BN;
  const int s = blockIdx.y;
  const int pb = (int)((long long)np * s / nsplit), pe = (int)((long long)np * (s + 1) / nsplit);
  f32x4 kacc[4][4];
  zero4(kacc);
  Operand A{ct_hi, ct_lo, ldk, nact, nbf};
  for (int P = pb; P < pe; ++P) {
    const long long off = (long long)P * nact * ldx;
    Operand B{xt_hi + off, xt_lo ? xt_lo + off : nullptr, ldx, nact, nbf};
    f32x4 acc[4][4];
    zero4(acc);
    tile_bf16<TERMS, (TERMS >= 2), (TERMS >= 3)>(sm, A, B, m0, n0, acc);
    u16* Wh = w_hi + (long long)P * nact * ldw;
    u16* Wl = w_lo ? w_lo + (long long)P * nact * ldw : nullptr;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int jn = 0; jn < 4; ++jn)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int p = m0 + row_of(i, j), q = n0 + col_of(jn);
          const float b = acc[i][jn][j];
          kacc[i][jn][j] += b * b;
          if (p < nact && q <= p) {
            const float w = b * beta32[(long long)p * nact + q];
            u16 h, l;
            if (TERMS == 1) { h = f32_to_bf16_bits(w); l = 0; }
            else split_f32(w, h, l);
            Wh[(long long)p * ldw + q] = h;
            Wh[(long long)q * ldw + p] = h;
            if (Wl) { Wl[(long long)p * ldw + q] = l; Wl[(long long)q * ldw + p] = l; }
            if (p == q) Dc[(long long)P * nact + p] = (double)b;
          }
        }
  }
  double* Kp = Kpart + (long long)s * nact * nact;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jn = 0; jn < 4; ++jn)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = m0 + row_of(i, j), q = n0 + col_of(jn);
        if (p < nact && q <= p) Kp[(long long)p * nact + q] += (double)kacc[i][jn][j];
      }
}

// gemm3: Ypart[s][mu][q] = sum_{P in s} sum_r X_P[mu][r] W_P[q][r]  (W symmetric).
template <int TERMS>
__global__ __launch_bounds__(256) void gemm3_kernel(int nbf, int nact, int np, int nsplit,
                                                    const u16* __restrict__ x_hi,
                                                    const u16* __restrict__ x_lo, int ldxx,
                                                    const u16* __restrict__ w_hi,
                                                    const u16* __restrict__ w_lo, int ldw,
                                                    float* __restrict__ Ypart) {
  __shared__ Smem sm;
  const int tiles_n = (nact + BN - 1) / BN;
  const int m0 = (blockIdx.x / tiles_n) * BM, n0 = (blockIdx.x % tiles_n) * BN;
  const int s = blockIdx.y;
  const int pb = (int)((long long)np * s / nsplit), pe = (int)((long long)np * (s + 1) / nsplit);
  f32x4 acc[4][4];
  zero4(acc);
  for (int P = pb; P < pe; ++P) {
    const long long ox = (long long)P * nbf * ldxx, ow = (long long)P * nact * ldw;
    Operand A{x_hi + ox, x_lo ? x_lo + ox : nullptr, ldxx, nbf, nact};
    Operand B{w_hi + ow, w_lo ? w_lo + ow : nullptr, ldw, nact, nact};
    tile_bf16<TERMS, (TERMS >= 2), (TERMS >= 3)>(sm, A, B, m0, n0, acc);
  }
  float* Y = Ypart + (long long)s * nbf * nact;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jn = 0; jn < 4; ++jn)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + row_of(i, j), n = n0 + col_of(jn);
        if (m < nbf && n < nact) Y[(long long)m * nact + n] = acc[i][jn][j];
      }
}

}  // namespace

hipError_t df_bf16_gemm1(hipStream_t s, int nbf, int nact, int np, int terms, SplitPtr Ct, int ldk,
                         SplitPtr Bp, long long bstride, int ldb, u16* XT_hi, u16* XT_lo, int ldx,
                         u16* X_hi, u16* X_lo, int ldxx) {
  if (np <= 0) return hipSuccess;
  dim3 grid(cdiv(nact, BM) * cdiv(nbf, BN), np);
  if (terms == 1)
    hipLaunchKernelGGL((gemm1_kernel<1, false>), grid, dim3(256), 0, s, nbf, nact, Ct.hi, Ct.lo, ldk, Bp.hi, Bp.lo, bstride, ldb, XT_hi, XT_lo, ldx, X_hi, X_lo, ldxx);
  else if (Bp.lo == nullptr)
    hipLaunchKernelGGL((gemm1_kernel<2, false>), grid, dim3(256), 0, s, nbf, nact, Ct.hi, Ct.lo, ldk, Bp.hi, Bp.lo, bstride, ldb, XT_hi, XT_lo, ldx, X_hi, X_lo, ldxx);
  else
    hipLaunchKernelGGL((gemm1_kernel<3, true>), grid, dim3(256), 0, s, nbf, nact, Ct.hi, Ct.lo, ldk, Bp.hi, Bp.lo, bstride, ldb, XT_hi, XT_lo, ldx, X_hi, X_lo, ldxx);
  return hipGetLastError();
}

hipError_t df_bf16_gemm2(hipStream_t s, int nbf, int nact, int np, int nsplit, int terms,
                         SplitPtr Ct, int ldk, SplitPtr XT, int ldx, const float* beta32,
                         double* Kpart, double* Dchunk, u16* W_hi, u16* W_lo, int ldw) {
  if (np <= 0) return hipSuccess;
  const int t = cdiv(nact, BM);
  dim3 grid(t * (t + 1) / 2, nsplit);
  if (terms == 1)
    hipLaunchKernelGGL((gemm2_kernel<1>), grid, dim3(256), 0, s, nbf, nact, np, nsplit, Ct.hi, Ct.lo, ldk, XT.hi, XT.lo, ldx, beta32, Kpart, Dchunk, W_hi, W_lo, ldw);
  else
    hipLaunchKernelGGL((gemm2_kernel<3>), grid, dim3(256), 0, s, nbf, nact, np, nsplit, Ct.hi, Ct.lo, ldk, XT.hi, XT.lo, ldx, beta32, Kpart, Dchunk, W_hi, W_lo, ldw);
  return hipGetLastError();
}

hipError_t df_bf16_gemm3(hipStream_t s, int nbf, int nact, int np, int nsplit, int terms, SplitPtr X,
                         int ldxx, SplitPtr W, int ldw, float* Ypart) {
  if (np <= 0) return hipSuccess;
  dim3 grid(cdiv(nbf, BM) * cdiv(nact, BN), nsplit);
  if (terms == 1)
    hipLaunchKernelGGL((gemm3_kernel<1>), grid, dim3(256), 0, s, nbf, nact, np, nsplit, X.hi, X.lo, ldxx, W.hi, W.lo, ldw, Ypart);
  else
    hipLaunchKernelGGL((gemm3_kernel<3>), grid, dim3(256), 0, s, nbf, nact, np, nsplit, X.hi, X.lo, ldxx, W.hi, W.lo, ldw, Ypart);
  return hipGetLastError();
}

}  // namespace pnof
