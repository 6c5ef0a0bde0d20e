// Float64 matrix-core (v_mfma_f64_16x16x4) contractions.
//
// Block tile 64 x 64 x 16, 256 threads = 4 waves in a 2 x 2 arrangement, each wave owning a
// 32 x 32 sub-tile = 2 x 2 MFMA blocks of 16 x 16.  Operands are staged through LDS stored
// k-major ([k][m] and [k][n]), which is the order in which the f64 MFMA consumes them (lane l
// supplies A[m = l%16][k = l/16] and B[k = l/16][n = l%16]; the result element (l/16 + 4*j, l%16)
// sits in component j of lane l).  Register prefetch of the next k-slab overlaps global loads
// with the matrix-core work.
#include "common.h"
#include "f64_tile.h"

namespace pnof {
namespace {

using namespace f64t;

template <bool AM, bool BN>
__global__ __launch_bounds__(256) void gemm_f64_kernel(int M, int N, int K, double alpha,
                                                       const double* __restrict__ A, long long sam,
                                                       long long sak, long long sab,
                                                       const double* __restrict__ B, long long sbk,
                                                       long long sbn, long long sbb, double beta,
                                                       double* __restrict__ C, long long scm,
                                                       long long scn, long long scb) {
  __shared__ F64Smem sm;
  const int tiles_n = (N + TN - 1) / TN;
  const int m0 = (blockIdx.x / tiles_n) * TM, n0 = (blockIdx.x % tiles_n) * TN;
  const long long b = blockIdx.y;
  f64x4 acc[2][2];
  zero_acc(acc);
  tile_f64<AM, BN>(sm, A + b * sab, sam, sak, B + b * sbb, sbk, sbn, M, N, 0, K, m0, n0, acc);
  double* Cb = C + b * scb;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + acc_row(mi, j), n = n0 + acc_col(ni);
        if (m < M && n < N) {
          double* c = Cb + (long long)m * scm + (long long)n * scn;
          *c = alpha * acc[mi][ni][j] + (beta != 0.0 ? beta * *c : 0.0);
        }
      }
}

// Single products (the step's float64 products: H C_A, lambda = C^T Y, J = D^T D, Q Z and C U) on a
// finer grid: block tile 64 x 32 (4 waves of 32 x 16, each two 16 x 16 MFMA blocks), so that a
// 1200 x 1200 product makes 722 blocks, about 2.8 per compute unit, where 64 x 64 tiles made 361,
// about 1.4, and the units holding two of them set the time.  k-slabs of 16 go through two LDS
// stages, loaded into registers two slabs ahead of their multiplication; one barrier per slab
// separates the writes of one stage from the reads of the other (1200^3: 94-101 us, against
// 103-113 us with slabs of 32 one ahead and 117-130 us with 64 x 64 tiles).
template <bool AM, bool BN>
__global__ __launch_bounds__(256, 3) void gemm_f64_wide_kernel(int M, int N, int K, double alpha,
                                                              const double* __restrict__ A, long long sam,
                                                              long long sak, const double* __restrict__ B,
                                                              long long sbk, long long sbn, double beta,
                                                              double* __restrict__ C, long long scm, long long scn) {
  using namespace wide;
  __shared__ Smem sm;
  const int tn_n = (N + BNT - 1) / BNT;
  const int m0 = (blockIdx.x / tn_n) * BM, n0 = (blockIdx.x % tn_n) * BNT;
  f64x4 acc[2];
  wide_tile<AM, BN>(sm, A, sam, sak, B, sbk, sbn, M, N, K, m0, n0, acc);
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = m0 + wide_row(mi, j), n = n0 + wide_col();
      if (m < M && n < N) {
        double* c = C + (long long)m * scm + (long long)n * scn;
        *c = alpha * acc[mi][j] + (beta != 0.0 ? beta * *c : 0.0);
      }
    }
}

// One product of a grouped launch per blockIdx.y; blocks beyond that product's tiles exit.
template <bool AM, bool BN>
__global__ __launch_bounds__(256) void gemm_f64_grouped_kernel(const F64Gemm* __restrict__ tab) {
  __shared__ F64Smem sm;
  grouped_tile<AM, BN>(tab[blockIdx.y], blockIdx.x, sm);
}

// Split-K form for products with few output tiles: block (tile, s) sums k in the s-th of ks equal
// ranges and writes its partial to slab s of Cpart (ks dense M x N slabs, row-major).  The caller
// adds the slabs in slab order, so the result does not depend on the schedule.
template <bool AM, bool BN>
__global__ __launch_bounds__(256) void gemm_f64_splitk_kernel(int M, int N, int K, int ks, const double* __restrict__ A,
                                                              long long sam, long long sak,
                                                              const double* __restrict__ B, long long sbk,
                                                              long long sbn, double* __restrict__ Cpart) {
  __shared__ F64Smem sm;
  const int tiles_n = (N + TN - 1) / TN;
  const int tile = blockIdx.x / ks, sidx = blockIdx.x % ks;
  const int m0 = (tile / tiles_n) * TM, n0 = (tile % tiles_n) * TN;
  const int kb = (int)((long long)K * sidx / ks), ke = (int)((long long)K * (sidx + 1) / ks);
  f64x4 acc[2][2];
  zero_acc(acc);
  tile_f64<AM, BN>(sm, A, sam, sak, B, sbk, sbn, M, N, kb, ke, m0, n0, acc);
  double* Cs = Cpart + (long long)sidx * M * N;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + acc_row(mi, j), n = n0 + acc_col(ni);
        if (m < M && n < N) Cs[(long long)m * N + n] = acc[mi][ni][j];
      }
}

// Lower-triangle tile index t -> (tm, tn) with tn <= tm.
__device__ __forceinline__ void tri_tile(int t, int& tm, int& tn) {
  int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  tm = r;
  tn = t - r * (r + 1) / 2;
}

// gemm1: XT[P][p][mu] = sum_nu Ct[p][nu] B_P[nu][mu] (B_P symmetric, row-major).
__global__ __launch_bounds__(256) void df_gemm1_kernel(int nbf, int nact, const double* __restrict__ Ct,
                                                       int ldk, const double* __restrict__ Bc,
                                                       double* __restrict__ XT, int ldx) {
  __shared__ F64Smem sm;
  const int tiles_n = (nbf + TN - 1) / TN;
  const int m0 = (blockIdx.x / tiles_n) * TM, n0 = (blockIdx.x % tiles_n) * TN;
  const long long P = blockIdx.y;
  f64x4 acc[2][2];
  zero_acc(acc);
  // A(m=p, k=nu) = Ct[p*ldk + nu] (k contiguous); B(k=nu, n=mu) = B_P[nu*nbf + mu] (n contiguous)
  tile_f64<false, true>(sm, Ct, ldk, 1, Bc + P * nbf * nbf, nbf, 1, nact, nbf, 0, nbf, m0, n0, acc);
  double* X = XT + P * (long long)nact * ldx;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + acc_row(mi, j), n = n0 + acc_col(ni);
        if (m < nact && n < nbf) X[(long long)m * ldx + n] = acc[mi][ni][j];
      }
}

// gemm2: b_P = Ct XT_P^T on lower tiles of the nact x nact result, P in the block's split.
__global__ __launch_bounds__(256) void df_gemm2_kernel(int nbf, int nact, int np, int nsplit,
                                                       const double* __restrict__ Ct, int ldk,
                                                       const double* __restrict__ XT, int ldx,
                                                       const double* __restrict__ beta,
                                                       double* __restrict__ Kpart,
                                                       double* __restrict__ Dc,
                                                       double* __restrict__ W, int ldw) {
  __shared__ F64Smem sm;
  int tm, tn;
  tri_tile(blockIdx.x, tm, tn);
  const int m0 = tm * TM, n0 = tn * TN;
  const int s = blockIdx.y;
  const int pb = (int)((long long)np * s / nsplit), pe = (int)((long long)np * (s + 1) / nsplit);
  f64x4 kacc[2][2];
  zero_acc(kacc);
  for (int P = pb; P < pe; ++P) {
    f64x4 acc[2][2];
    zero_acc(acc);
    // A(m=p, k=mu) = Ct[p*ldk + mu]; B(k=mu, n=q) = XT_P[q*ldx + mu] (k contiguous)
    tile_f64<false, false>(sm, Ct, ldk, 1, XT + (long long)P * nact * ldx, 1, ldx, nact, nact, 0, nbf,
                           m0, n0, acc);
    double* Wp = W + (long long)P * nact * ldw;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int p = m0 + acc_row(mi, j), q = n0 + acc_col(ni);
          const double b = acc[mi][ni][j];
          kacc[mi][ni][j] += b * b;
          if (p < nact && q <= p) {  // each unordered pair written once: deterministic W
            const double w = b * beta[(long long)p * nact + q];
            Wp[(long long)p * ldw + q] = w;
            Wp[(long long)q * ldw + p] = w;
            if (p == q) Dc[(long long)P * nact + p] = b;
          }
        }
  }
  double* Kp = Kpart + (long long)s * nact * nact;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = m0 + acc_row(mi, j), q = n0 + acc_col(ni);
        if (p < nact && q <= p) Kp[(long long)p * nact + q] += kacc[mi][ni][j];
      }
}

// gemm3: Ypart[s][mu][q] = sum_{P in split s} sum_r XT_P[r][mu] W_P[r][q].
__global__ __launch_bounds__(256) void df_gemm3_kernel(int nbf, int nact, int np, int nsplit,
                                                       const double* __restrict__ XT, int ldx,
                                                       const double* __restrict__ W, int ldw,
                                                       double* __restrict__ Ypart) {
  __shared__ F64Smem sm;
  const int tiles_n = (nact + TN - 1) / TN;
  const int m0 = (blockIdx.x / tiles_n) * TM, n0 = (blockIdx.x % tiles_n) * TN;
  const int s = blockIdx.y;
  const int pb = (int)((long long)np * s / nsplit), pe = (int)((long long)np * (s + 1) / nsplit);
  f64x4 acc[2][2];
  zero_acc(acc);
  for (int P = pb; P < pe; ++P) {
    // A(m=mu, k=r) = XT_P[r*ldx + mu] (m contiguous); B(k=r, n=q) = W_P[r*ldw + q] (n contiguous)
    tile_f64<true, true>(sm, XT + (long long)P * nact * ldx, 1, ldx, W + (long long)P * nact * ldw,
                         ldw, 1, nbf, nact, 0, nact, m0, n0, acc);
  }
  double* Y = Ypart + (long long)s * nbf * nact;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + acc_row(mi, j), n = n0 + acc_col(ni);
        if (m < nbf && n < nact) Y[(long long)m * nact + n] = acc[mi][ni][j];
      }
}

// ------------------------------------------------------------------------------------------------
// float32 matrix-core (v_mfma_f32_16x16x4f32) forms of the three contractions (PNOF_FP32): the same
// 64 x 64 x 16 tiling and LDS staging, float operands, float32 accumulation within a P row; K sums
// b^2 in float64.  Lane layout of the operands as above; the result element (4*(l/16) + j, l%16)
// sits in component j of lane l.
struct F32Smem {
  float a[TK][TM + LPAD];
  float b[TK][TN + LPAD];
};

__device__ __forceinline__ float ldf(const float* p) { return *p; }
__device__ __forceinline__ float ldf(const double* p) { return (float)*p; }
__device__ __forceinline__ float ldf(const u16* p) { return bf16_bits_to_f32(*p); }

template <bool RCONTIG, typename S>
__device__ __forceinline__ void load_slab32(const S* __restrict__ P, long long sr, long long sk, int R, int K, int r0,
                                            int k0, float (&reg)[4]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int r, k;
    if (RCONTIG) { r = t & 63; k = (t >> 6) + 4 * i; }
    else         { r = t >> 2; k = ((t & 3) << 2) + i; }
    const int gr = r0 + r, gk = k0 + k;
    reg[i] = (gr < R && gk < K) ? ldf(P + (long long)gr * sr + (long long)gk * sk) : 0.0f;
  }
}

template <bool RCONTIG>
__device__ __forceinline__ void store_slab32(float (*S)[TM + LPAD], const float (&reg)[4]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int r, k;
    if (RCONTIG) { r = t & 63; k = (t >> 6) + 4 * i; }
    else         { r = t >> 2; k = ((t & 3) << 2) + i; }
    S[k][r] = reg[i];
  }
}

template <bool AM, bool BN, typename SA, typename SB>
__device__ __forceinline__ void tile_f32(F32Smem& sm, const SA* __restrict__ A, long long sam, long long sak,
                                         const SB* __restrict__ B, long long sbk, long long sbn, int M, int N, int kb,
                                         int ke, int m0, int n0, f32x4 (&acc)[2][2]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int K = ke;
  float ra[4], rb[4];
  load_slab32<AM>(A, sam, sak, M, K, m0, kb, ra);
  load_slab32<BN>(B, sbn, sbk, N, K, n0, kb, rb);
  for (int k0 = kb; k0 < ke; k0 += TK) {
    __syncthreads();
    store_slab32<AM>(sm.a, ra);
    store_slab32<BN>(sm.b, rb);
    __syncthreads();
    if (k0 + TK < K) {
      load_slab32<AM>(A, sam, sak, M, K, m0, k0 + TK, ra);
      load_slab32<BN>(B, sbn, sbk, N, K, n0, k0 + TK, rb);
    }
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int kr = kk + (lane >> 4);
      const float a0 = sm.a[kr][wm + (lane & 15)], a1 = sm.a[kr][wm + 16 + (lane & 15)];
      const float b0 = sm.b[kr][wn + (lane & 15)], b1 = sm.b[kr][wn + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
}

__device__ __forceinline__ void zero_acc32(f32x4 (&acc)[2][2]) {
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
}
__device__ __forceinline__ int acc_row32(int mi, int j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave >> 1) * 32 + mi * 16 + 4 * (lane >> 4) + j;
}

// gemm1: XT[P][p][mu] = sum_nu Ct[p][nu] B_P[nu][mu], B read as stored (bf16 or float64).
template <typename SB>
__global__ __launch_bounds__(256) void df32_gemm1_kernel(int nbf, int nact, const float* __restrict__ Ct, int ldk,
                                                         const SB* __restrict__ Bc, float* __restrict__ XT, int ldx) {
  __shared__ F32Smem sm;
  const int tiles_n = (nbf + TN - 1) / TN;
  const int m0 = (blockIdx.x / tiles_n) * TM, n0 = (blockIdx.x % tiles_n) * TN;
  const long long P = blockIdx.y;
  f32x4 acc[2][2];
  zero_acc32(acc);
  tile_f32<false, true>(sm, Ct, ldk, 1, Bc + P * nbf * nbf, nbf, 1, nact, nbf, 0, nbf, m0, n0, acc);
  float* X = XT + P * (long long)nact * ldx;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + acc_row32(mi, j), n = n0 + acc_col(ni);
        if (m < nact && n < nbf) X[(long long)m * ldx + n] = acc[mi][ni][j];
      }
}

// gemm2: b_P = Ct XT_P^T on lower tiles; K partials (float64 sums of b^2), D, W = b o beta.
__global__ __launch_bounds__(256) void df32_gemm2_kernel(int nbf, int nact, int np, int nsplit,
                                                         const float* __restrict__ Ct, int ldk,
                                                         const float* __restrict__ XT, int ldx,
                                                         const float* __restrict__ beta32, double* __restrict__ Kpart,
                                                         double* __restrict__ Dc, float* __restrict__ W, int ldw) {
  __shared__ F32Smem sm;
  int tm, tn;
  tri_tile(blockIdx.x, tm, tn);
  const int m0 = tm * TM, n0 = tn * TN;
  const int s = blockIdx.y;
  const int pb = (int)((long long)np * s / nsplit), pe = (int)((long long)np * (s + 1) / nsplit);
  f64x4 kacc[2][2];
  zero_acc(kacc);
  for (int P = pb; P < pe; ++P) {
    f32x4 acc[2][2];
    zero_acc32(acc);
    tile_f32<false, false>(sm, Ct, ldk, 1, XT + (long long)P * nact * ldx, 1, ldx, nact, nact, 0, nbf, m0, n0, acc);
    float* Wp = W + (long long)P * nact * ldw;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ni = 0; ni < 2; ++ni)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int p = m0 + acc_row32(mi, j), q = n0 + acc_col(ni);
          const float b = acc[mi][ni][j];
          kacc[mi][ni][j] += (double)b * (double)b;
          if (p < nact && q <= p) {
            const float w = b * beta32[(long long)p * nact + q];
            Wp[(long long)p * ldw + q] = w;
            Wp[(long long)q * ldw + p] = w;
            if (p == q) Dc[(long long)P * nact + p] = (double)b;
          }
        }
  }
  double* Kp = Kpart + (long long)s * nact * nact;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = m0 + acc_row32(mi, j), q = n0 + acc_col(ni);
        if (p < nact && q <= p) Kp[(long long)p * nact + q] += kacc[mi][ni][j];
      }
}

// gemm3: Ypart[s][mu][q] = sum_{P in split s} sum_r XT_P[r][mu] W_P[r][q].
__global__ __launch_bounds__(256) void df32_gemm3_kernel(int nbf, int nact, int np, int nsplit,
                                                         const float* __restrict__ XT, int ldx,
                                                         const float* __restrict__ W, int ldw,
                                                         float* __restrict__ Ypart) {
  __shared__ F32Smem sm;
  const int tiles_n = (nact + TN - 1) / TN;
  const int m0 = (blockIdx.x / tiles_n) * TM, n0 = (blockIdx.x % tiles_n) * TN;
  const int s = blockIdx.y;
  const int pb = (int)((long long)np * s / nsplit), pe = (int)((long long)np * (s + 1) / nsplit);
  f32x4 acc[2][2];
  zero_acc32(acc);
  for (int P = pb; P < pe; ++P)
    tile_f32<true, true>(sm, XT + (long long)P * nact * ldx, 1, ldx, W + (long long)P * nact * ldw, ldw, 1, nbf, nact,
                         0, nact, m0, n0, acc);
  float* Y = Ypart + (long long)s * nbf * nact;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + acc_row32(mi, j), n = n0 + acc_col(ni);
        if (m < nbf && n < nact) Y[(long long)m * nact + n] = acc[mi][ni][j];
      }
}

}  // namespace

hipError_t gemm_f64(hipStream_t s, int M, int N, int K, int batch, double alpha, const double* A,
                    long long sam, long long sak, long long sab, const double* B, long long sbk,
                    long long sbn, long long sbb, double beta, double* C, long long scm, long long scn,
                    long long scb) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  const bool am = (sam == 1), bn = (sbn == 1);
  if (batch == 1) {
    const dim3 g1((unsigned)(cdiv(M, wide::BM) * cdiv(N, wide::BNT)));
    if (am && bn)
      hipLaunchKernelGGL((gemm_f64_wide_kernel<true, true>), g1, dim3(256), 0, s, M, N, K, alpha, A, sam, sak, B, sbk, sbn, beta, C, scm, scn);
    else if (am)
      hipLaunchKernelGGL((gemm_f64_wide_kernel<true, false>), g1, dim3(256), 0, s, M, N, K, alpha, A, sam, sak, B, sbk, sbn, beta, C, scm, scn);
    else if (bn)
      hipLaunchKernelGGL((gemm_f64_wide_kernel<false, true>), g1, dim3(256), 0, s, M, N, K, alpha, A, sam, sak, B, sbk, sbn, beta, C, scm, scn);
    else
      hipLaunchKernelGGL((gemm_f64_wide_kernel<false, false>), g1, dim3(256), 0, s, M, N, K, alpha, A, sam, sak, B, sbk, sbn, beta, C, scm, scn);
    return hipGetLastError();
  }
  dim3 grid(cdiv(M, TM) * cdiv(N, TN), batch);
  if (am && bn)
    hipLaunchKernelGGL((gemm_f64_kernel<true, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, sam, sak, sab, B, sbk, sbn, sbb, beta, C, scm, scn, scb);
  else if (am && !bn)
    hipLaunchKernelGGL((gemm_f64_kernel<true, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, sam, sak, sab, B, sbk, sbn, sbb, beta, C, scm, scn, scb);
  else if (!am && bn)
    hipLaunchKernelGGL((gemm_f64_kernel<false, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, sam, sak, sab, B, sbk, sbn, sbb, beta, C, scm, scn, scb);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<false, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, sam, sak, sab, B, sbk, sbn, sbb, beta, C, scm, scn, scb);
  return hipGetLastError();
}

int gemm_f64_ksplit(int M, int N, int K) {
  const int tiles = cdiv(M, TM) * cdiv(N, TN);
  int ks = cdiv(512, tiles);                   // about two blocks per compute unit
  ks = ks < F64_KSPLIT_MAX ? ks : F64_KSPLIT_MAX;
  const int kmax = cdiv(K, 4 * TK);            // at least four k-slabs per block
  return ks < kmax ? ks : (kmax > 0 ? kmax : 1);
}

hipError_t gemm_f64_splitk(hipStream_t s, int M, int N, int K, int ks, const double* A, long long sam, long long sak,
                           const double* B, long long sbk, long long sbn, double* Cpart) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (ks < 1 || ks > F64_KSPLIT_MAX) return hipErrorInvalidValue;
  const dim3 grid(cdiv(M, TM) * cdiv(N, TN) * ks);
  const bool am = (sam == 1), bn = (sbn == 1);
  if (am && bn)
    hipLaunchKernelGGL((gemm_f64_splitk_kernel<true, true>), grid, dim3(256), 0, s, M, N, K, ks, A, sam, sak, B, sbk, sbn, Cpart);
  else if (am)
    hipLaunchKernelGGL((gemm_f64_splitk_kernel<true, false>), grid, dim3(256), 0, s, M, N, K, ks, A, sam, sak, B, sbk, sbn, Cpart);
  else if (bn)
    hipLaunchKernelGGL((gemm_f64_splitk_kernel<false, true>), grid, dim3(256), 0, s, M, N, K, ks, A, sam, sak, B, sbk, sbn, Cpart);
  else
    hipLaunchKernelGGL((gemm_f64_splitk_kernel<false, false>), grid, dim3(256), 0, s, M, N, K, ks, A, sam, sak, B, sbk, sbn, Cpart);
  return hipGetLastError();
}

hipError_t gemm_f64_grouped(hipStream_t s, int ngemm, int maxM, int maxN, bool a_unit_m, bool b_unit_n,
                            const F64Gemm* tab) {
  if (ngemm <= 0 || maxM <= 0 || maxN <= 0) return hipSuccess;
  dim3 grid(cdiv(maxM, TM) * cdiv(maxN, TN), ngemm);
  if (a_unit_m && b_unit_n) hipLaunchKernelGGL((gemm_f64_grouped_kernel<true, true>), grid, dim3(256), 0, s, tab);
  else if (a_unit_m) hipLaunchKernelGGL((gemm_f64_grouped_kernel<true, false>), grid, dim3(256), 0, s, tab);
  else if (b_unit_n) hipLaunchKernelGGL((gemm_f64_grouped_kernel<false, true>), grid, dim3(256), 0, s, tab);
  else hipLaunchKernelGGL((gemm_f64_grouped_kernel<false, false>), grid, dim3(256), 0, s, tab);
  return hipGetLastError();
}

hipError_t df_f64_gemm1(hipStream_t s, int nbf, int nact, int np, const double* Ct, int ldk,
                        const double* Bchunk, double* XT, int ldx) {
  if (np <= 0) return hipSuccess;
  dim3 grid(cdiv(nact, TM) * cdiv(nbf, TN), np);
  hipLaunchKernelGGL(df_gemm1_kernel, grid, dim3(256), 0, s, nbf, nact, Ct, ldk, Bchunk, XT, ldx);
  return hipGetLastError();
}

hipError_t df_f64_gemm2(hipStream_t s, int nbf, int nact, int np, int nsplit, const double* Ct,
                        int ldk, const double* XT, int ldx, const double* beta, double* Kpart,
                        double* Dchunk, double* W, int ldw) {
  if (np <= 0) return hipSuccess;
  const int t = cdiv(nact, TM);
  dim3 grid(t * (t + 1) / 2, nsplit);
  hipLaunchKernelGGL(df_gemm2_kernel, grid, dim3(256), 0, s, nbf, nact, np, nsplit, Ct, ldk, XT, ldx,
                     beta, Kpart, Dchunk, W, ldw);
  return hipGetLastError();
}

hipError_t df_f64_gemm3(hipStream_t s, int nbf, int nact, int np, int nsplit, const double* XT,
                        int ldx, const double* W, int ldw, double* Ypart) {
  if (np <= 0) return hipSuccess;
  dim3 grid(cdiv(nbf, TM) * cdiv(nact, TN), nsplit);
  hipLaunchKernelGGL(df_gemm3_kernel, grid, dim3(256), 0, s, nbf, nact, np, nsplit, XT, ldx, W, ldw,
                     Ypart);
  return hipGetLastError();
}

}  // namespace pnof

namespace pnof {

hipError_t df_f32_gemm1(hipStream_t s, int nbf, int nact, int np, const float* Ct, int ldk, const void* Bchunk,
                        int b_is_bf16, float* XT, int ldx) {
  if (np <= 0) return hipSuccess;
  dim3 grid(cdiv(nact, TM) * cdiv(nbf, TN), np);
  if (b_is_bf16)
    hipLaunchKernelGGL(df32_gemm1_kernel<u16>, grid, dim3(256), 0, s, nbf, nact, Ct, ldk,
                       static_cast<const u16*>(Bchunk), XT, ldx);
  else
    hipLaunchKernelGGL(df32_gemm1_kernel<double>, grid, dim3(256), 0, s, nbf, nact, Ct, ldk,
                       static_cast<const double*>(Bchunk), XT, ldx);
  return hipGetLastError();
}

hipError_t df_f32_gemm2(hipStream_t s, int nbf, int nact, int np, int nsplit, const float* Ct, int ldk,
                        const float* XT, int ldx, const float* beta32, double* Kpart, double* Dchunk, float* W,
                        int ldw) {
  if (np <= 0) return hipSuccess;
  const int t = cdiv(nact, TM);
  dim3 grid(t * (t + 1) / 2, nsplit);
  hipLaunchKernelGGL(df32_gemm2_kernel, grid, dim3(256), 0, s, nbf, nact, np, nsplit, Ct, ldk, XT, ldx, beta32, Kpart,
                     Dchunk, W, ldw);
  return hipGetLastError();
}

hipError_t df_f32_gemm3(hipStream_t s, int nbf, int nact, int np, int nsplit, const float* XT, int ldx,
                        const float* W, int ldw, float* Ypart) {
  if (np <= 0) return hipSuccess;
  dim3 grid(cdiv(nbf, TM) * cdiv(nact, TN), nsplit);
  hipLaunchKernelGGL(df32_gemm3_kernel, grid, dim3(256), 0, s, nbf, nact, np, nsplit, XT, ldx, W, ldw, Ypart);
  return hipGetLastError();
}

}  // namespace pnof
