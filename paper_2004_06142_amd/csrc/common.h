// Internal declarations shared by the libpnof translation units (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>

namespace pnof {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16;

// ---------------------------------------------------------------- orbital layout
// Strong orbital of pair g is g; the nsingle singly occupied orbitals (Omega_I) follow, each its own
// subspace; weak k of pair g is npairs + nsingle + ncwo*(npairs-1-g) + k.
__host__ __device__ inline int pair_of(int p, int npairs, int ncwo, int nsingle) {
  if (p < npairs + nsingle) return p;
  const int blk = (p - npairs - nsingle) / ncwo;
  return (blk < npairs) ? (npairs - 1 - blk) : -1;
}
__host__ __device__ inline bool is_single(int p, int npairs, int nsingle) { return p >= npairs && p < npairs + nsingle; }
__host__ __device__ inline int weak_index(int g, int k, int npairs, int ncwo, int nsingle) {
  return npairs + nsingle + ncwo * (npairs - 1 - g) + k;
}

// ---------------------------------------------------------------- PNOF coefficients
// alpha_pq, beta_pq of E_2 = sum_pq alpha_pq J_pq + beta_pq K_pq (Eqs. Eg, Efg, Efg_s).
// A singly occupied orbital has no intra-subspace term (beta_pp = 0).
__device__ inline void pnof_coeff(int p, int q, double np_, double nq, int npairs, int ncwo, int nsingle,
                                  int functional, double& a, double& b) {
  a = 0.0;
  if (pair_of(p, npairs, ncwo, nsingle) == pair_of(q, npairs, ncwo, nsingle)) {
    if (p == q) b = is_single(p, npairs, nsingle) ? 0.0 : np_;
    else {
      const double s = sqrt(np_ * nq);
      b = (p < npairs || q < npairs) ? -s : s;
    }
  } else {
    a = 2.0 * np_ * nq;
    if (functional == 5) b = -np_ * nq;
    else if (functional == 8) b = -np_ * nq - 4.0 * (np_ * (1.0 - np_)) * (nq * (1.0 - nq));
    else b = -np_ * nq - sqrt(np_ * (1.0 - np_)) * sqrt(nq * (1.0 - nq));
  }
}

// Term q != p of dE/dn_p at fixed J, K (derivative of Eqs. Eg, Efg); php = sqrt(n_p (1 - n_p)).
__device__ inline double grad_n_term(int p, int q, double np_, double nq, double php, double jpq, double kpq,
                                     int npairs, int ncwo, int nsingle, int functional) {
  if (pair_of(q, npairs, ncwo, nsingle) == pair_of(p, npairs, ncwo, nsingle)) {
    const double sg = (p < npairs || q < npairs) ? -1.0 : 1.0;
    return sg * sqrt(nq / np_) * kpq;
  }
  double s = 4.0 * nq * jpq - 2.0 * nq * kpq;
  if (functional == 7) s += -sqrt(nq * (1.0 - nq)) * (1.0 - 2.0 * np_) / php * kpq;
  else if (functional == 8) s += -8.0 * (1.0 - 2.0 * np_) * nq * (1.0 - nq) * kpq;
  return s;
}

// ---------------------------------------------------------------- ON maps (Section 3.1)
__device__ inline double sigm(double x) { return 1.0 / (1.0 + exp(-x)); }

// Adjoint of the ON map for subspace g (pair g < npairs, or a singly occupied orbital): the entries
// out[r] = sum_p dEdn[p] dn_p/dgamma_r of the gamma variables of that subspace.  kind 0: sigmoid map
// normalised per pair (one gamma per active orbital); kind 1: trigonometric map (Eqs. soo, woo).
__device__ inline void on_map_vjp_subspace(int kind, int npairs, int ncwo, int nsingle, const double* __restrict__ gamma,
                                           const double* __restrict__ dEdn, double* __restrict__ out, int g) {
  if (g >= npairs) {   // a singly occupied orbital: n = 1/2 whatever its gamma (sigmoid map; none in the other)
    if (kind == 0 && g < npairs + nsingle) out[g] = 0.0;
    return;
  }
  if (kind == 0) {
    double S = sigm(gamma[g]);
    for (int k = 0; k < ncwo; ++k) S += sigm(gamma[weak_index(g, k, npairs, ncwo, nsingle)]);
    // dE/dgamma_r = s'_r / S * (dEdn_r - sum_p n_p dEdn_p)
    double avg = 0.0;
    for (int a = -1; a < ncwo; ++a) {
      const int p = a < 0 ? g : weak_index(g, a, npairs, ncwo, nsingle);
      avg += sigm(gamma[p]) / S * dEdn[p];
    }
    for (int b = -1; b < ncwo; ++b) {
      const int r = b < 0 ? g : weak_index(g, b, npairs, ncwo, nsingle);
      const double sr = sigm(gamma[r]);
      out[r] = sr * (1.0 - sr) / S * (dEdn[r] - avg);
    }
  } else {
    // n_i = h * prod_{k<i} c_k^2 * f_i, f_i = s_i^2 (f = 1 for the last weak orbital),
    // c_k = cos(gamma_k), s_k = sin(gamma_k) of the pair's weak variables; h = sin^2(gamma_g)/2.
    const double gs = gamma[g];
    const double cg = cos(gs), sg = sin(gs);
    const double h = 0.5 * sg * sg, dh = sg * cg;
    const int base = npairs + g * (ncwo - 1);
    double acc_g = -cg * sg * dEdn[g];
    double prod = 1.0;
    for (int i = 0; i < ncwo; ++i) {
      const bool last = (i == ncwo - 1);
      const double si = last ? 0.0 : sin(gamma[base + i]);
      const double fi = last ? 1.0 : si * si;
      acc_g += dh * prod * fi * dEdn[weak_index(g, i, npairs, ncwo, nsingle)];
      if (!last) { const double ci = cos(gamma[base + i]); prod *= ci * ci; }
    }
    out[g] = acc_g;
    for (int j = 0; j < ncwo - 1; ++j) {
      const double cj = cos(gamma[base + j]), sj = sin(gamma[base + j]);
      double sum = 0.0;
      for (int i = j; i < ncwo; ++i) {
        const bool last = (i == ncwo - 1);
        double other = h;                           // prod over k < i, k != j of c_k^2
        for (int k = 0; k < i; ++k) {
          if (k == j) continue;
          const double ck = cos(gamma[base + k]);
          other *= ck * ck;
        }
        double d;
        if (i == j) d = other * 2.0 * sj * cj;      // d(s_j^2)
        else {
          const double si = last ? 0.0 : sin(gamma[base + i]);
          d = other * (-2.0 * cj * sj) * (last ? 1.0 : si * si);  // d(c_j^2) * f_i
        }
        sum += d * dEdn[weak_index(g, i, npairs, ncwo, nsingle)];
      }
      out[base + j] = sum;
    }
  }
}

// sum_{k < ns} p[k * stride], added in order of k, with the loads issued eight at a time: the partial
// sums of a split contraction lie far apart in memory, and with one load in flight per thread the
// reduction would wait out the memory latency once per split.
template <typename T>
__device__ __forceinline__ double sum_strided(const T* __restrict__ p, int ns, long long stride) {
  double s = 0.0;
  int k = 0;
  for (; k + 8 <= ns; k += 8) {
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(long long)(k + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += (double)v[u];
  }
  for (; k < ns; ++k) s += (double)p[(long long)k * stride];
  return s;
}

// ---------------------------------------------------------------- bf16 helpers
// Round-to-nearest-even float32 -> bfloat16 bits (inputs here are finite).
__device__ __forceinline__ u16 f32_to_bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(u16 b) { return __uint_as_float(((uint32_t)b) << 16); }

// x ~= hi + lo with hi = bf16(x), lo = bf16(x - hi).
__device__ __forceinline__ void split_f32(float x, u16& hi, u16& lo) {
  hi = f32_to_bf16_bits(x);
  lo = f32_to_bf16_bits(x - bf16_bits_to_f32(hi));
}
// Two floats to bf16 with the hardware round-to-nearest-even conversion (v_cvt_pk_bf16_f32):
// packed pair, first value in the low half.
__device__ __forceinline__ uint32_t cvt2_bf16(float a, float b) {
  typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
  const bf2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}
// hi/lo split of two floats (as split_f32), as packed pairs.
__device__ __forceinline__ void split2_f32(float a, float b, uint32_t& hi, uint32_t& lo) {
  hi = cvt2_bf16(a, b);
  lo = cvt2_bf16(a - __uint_as_float(hi << 16), b - __uint_as_float(hi & 0xFFFF0000u));
}

__device__ __forceinline__ void split_f64(double x, u16& hi, u16& lo) {
  hi = f32_to_bf16_bits((float)x);
  lo = f32_to_bf16_bits((float)(x - (double)bf16_bits_to_f32(hi)));
}

// Compact bf16 pair of an orbital coefficient: hi = bf16(x), lo = bf16(x - hi), except that a lo
// below 2^(e - 14) (2^e <= |hi| < 2^(e+1)) is rounded once more to the grid 2^(e - 21), where it
// needs at most 8 bits.  hi + lo then spans at most 22 bits: it is exact in float32, and after a
// power-of-two scaling it splits exactly into an fp16 pair (11 + 11 bits) while the scaled value
// stays above 2^-3 (|C~| >= 2^-14 max|C| with the scale sC), so the b contraction's fp16 operand is
// the same C~ as X's bf16 one; smaller entries differ by at most 2^-37 max|C|.
// |x - hi - lo| <= 2^-17 |x|.
__device__ __forceinline__ void split_compact(double x, u16& hi, u16& lo) {
  hi = f32_to_bf16_bits((float)x);
  const double h = (double)bf16_bits_to_f32(hi);
  lo = f32_to_bf16_bits((float)(x - h));
  const double l = (double)bf16_bits_to_f32(lo);
  if (h == 0.0 || l == 0.0) return;
  const int e = ilogb(h);
  if (ilogb(l) >= e - 14) return;
  const double q = ldexp(1.0, e - 21);
  lo = (u16)(__float_as_uint((float)(rint(l / q) * q)) >> 16);
}

// ---------------------------------------------------------------- fp16 pairs with a power-of-two scale
// In the split mode the operands of the b and Y contractions (and of X when B is float64) are carried
// as fp16 hi + lo pairs of the value times a power of two s: hi = fp16(x s), lo = fp16(x s - hi),
// |x s - hi - lo| <= 2^-22 |x s| while x s stays in fp16's normal range (absolute error at most 2^-25
// below it).  s is chosen from a bound of |x| so that |x s| <= 2^14.
__device__ __forceinline__ u16 f32_to_f16_bits(float x) {
  const _Float16 h = (_Float16)x;
  return __builtin_bit_cast(u16, h);
}
__device__ __forceinline__ float f16_bits_to_f32(u16 b) { return (float)__builtin_bit_cast(_Float16, b); }
__device__ __forceinline__ void split_f16(float xs, u16& hi, u16& lo) {
  hi = f32_to_f16_bits(xs);
  lo = f32_to_f16_bits(xs - f16_bits_to_f32(hi));
}
// Two values at once, as packed pairs (first value in the low half): two packed conversions
// (v_cvt_pk_f16_f32), two widenings and two subtractions.
__device__ __forceinline__ void split2_f16(float a, float b, uint32_t& hi, uint32_t& lo) {
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  typedef float f2 __attribute__((ext_vector_type(2)));
  const f2 x = {a, b};
  const h2 h = __builtin_convertvector(x, h2);
  const h2 l = __builtin_convertvector(x - __builtin_convertvector(h, f2), h2);
  hi = __builtin_bit_cast(uint32_t, h);
  lo = __builtin_bit_cast(uint32_t, l);
}

// Exponent e with bound < 2^e (0 for a zero or non-finite bound), clamped to [-60, 60].
__host__ __device__ inline int bound_exp(float bound) {
  if (!(bound > 0.0f) || !(bound < 3.0e38f)) return 0;
  int e;
  frexpf(bound, &e);
  return e > 60 ? 60 : (e < -60 ? -60 : e);
}

// Bounds that fix the scales of one problem (or one batch instance) and of one P-chunk of it, kept as
// the bits of non-negative floats (so an integer atomic max is a float max):
//   call-level  [0] max |C_pq| over active columns, [1] max column 1-norm of C_A,
//               [2] max |beta| + max row 1-norm of alpha;
//   per chunk c [SCL_CALL + 2c] max row 1-norm sum_nu |B_P mu nu| over the chunk's rows,
//               [SCL_CALL + 2c + 1] max |B| over the chunk (float64 B only).
constexpr int SCL_CALL = 4;
inline long long scl_words(long long nchunk) { return SCL_CALL + 2 * nchunk; }

// Multipliers of the split mode for one chunk, all powers of two (exact in float32):
//   sC    Chat = C~ sC (the fp16 pair of the b contraction, and of X when B is float64);
//   sB    Bhat = B sB (float64 B only);
//   xmul  X accumulator -> Xhat = X sX (1 * sX for bf16 B; sX / (sC sB) for float64 B);
//   invB  b accumulator (Chat^T Xhat) -> b;
//   sW    What = W sW;  wmul = invB sW (b accumulator times beta -> What);
//   invY  Y accumulator (Xhat^T What) -> Y;  invX = 1 / sX.
// |X_P mu q| <= sum_nu |B_P mu nu| |C~_nu q| <= rownorm(B) max|C~|; |b_pq| <= ||c~_p||_1 max|X|;
// |W_pq| <= max|b| (max|beta| + max_p sum_r |alpha_pr|) (the diagonal adds d = D alpha).  The 1 %
// margins cover the float32 rounding of the bounds and |C~| <= |C| (1 + 2^-16).
struct Scales {
  float sC, sB, xmul, invB, sW, wmul, invY, invX;
};
__device__ __forceinline__ Scales chunk_scales(const uint32_t* __restrict__ bnd, int chunk, bool f64b) {
  const int ec = bound_exp(__uint_as_float(bnd[0]) * 1.01f), ec1 = bound_exp(__uint_as_float(bnd[1]) * 1.01f),
            eab = bound_exp(__uint_as_float(bnd[2]) * 1.01f);
  const int ebn = bound_exp(__uint_as_float(bnd[SCL_CALL + 2 * chunk]) * 1.01f);
  const int ebm = f64b ? bound_exp(__uint_as_float(bnd[SCL_CALL + 2 * chunk + 1]) * 1.01f) : 0;
  const int kC = 13 - ec, kB = f64b ? 13 - ebm : 0;
  const int kX = 14 - (ebn + ec);                // |X| < 2^(ebn + ec)
  const int kW = 14 - (ec1 + ebn + ec + eab);    // |W| < 2^(ec1 + ebn + ec + eab)
  Scales s;
  s.sC = ldexpf(1.0f, kC);
  s.sB = ldexpf(1.0f, kB);
  s.xmul = ldexpf(1.0f, f64b ? kX - kC - kB : kX);
  s.invB = ldexpf(1.0f, -kC - kX);
  s.sW = ldexpf(1.0f, kW);
  s.wmul = ldexpf(1.0f, kW - kC - kX);
  s.invY = ldexpf(1.0f, -kX - kW);
  s.invX = ldexpf(1.0f, -kX);
  return s;
}

__host__ __device__ inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }
__host__ __device__ inline long long round_up(long long a, long long b) { return (a + b - 1) / b * b; }

// ---------------------------------------------------------------- f64 GEMM (k_gemm_f64.hip)
// C[b] = alpha * A[b] B[b] + beta * C[b] with strided views
//   A(m,k) = A[b*sab + m*sam + k*sak], B(k,n) = B[b*sbb + k*sbk + n*sbn], C(m,n) = C[b*scb + m*scm + n*scn]
// Exactly one of sam/sak and one of sbk/sbn must be 1.
// Eigenvalues (ascending, overwriting d) and eigenvectors (Z, n x n column-major) of the symmetric
// tridiagonal matrix with diagonal d and off-diagonal e (n - 1 entries), by divide and conquer;
// ws holds tridiag_dc_ws_doubles(n) doubles; info (device) is set nonzero if a secular equation
// did not converge.  1 <= n <= TRIDIAG_MAX_N.
long long tridiag_dc_ws_doubles(int n);
hipError_t tridiag_eig_dc(hipStream_t s, int n, double* d, const double* e, double* Z, double* ws, int* info);
hipError_t gemm_f64(hipStream_t s, int M, int N, int K, int batch, double alpha, const double* A,
                    long long sam, long long sak, long long sab, const double* B, long long sbk,
                    long long sbn, long long sbb, double beta, double* C, long long scm, long long scn,
                    long long scb);

// Grouped form: product g of tab (device memory) is C = alpha A B + beta C with its own sizes and
// pointers; all products share the unit-stride pattern (a_unit_m: sam == 1, b_unit_n: sbn == 1).
struct F64Gemm {
  int M, N, K;
  double alpha;
  const double* A;
  long long sam, sak;
  const double* B;
  long long sbk, sbn;
  double beta;
  double* C;
  long long scm, scn;
};
hipError_t gemm_f64_grouped(hipStream_t s, int ngemm, int maxM, int maxN, bool a_unit_m, bool b_unit_n,
                            const F64Gemm* tab);

// FP64 three-index contractions of one P-chunk (np rows of B).
//  gemm1: XT[P][p][mu] = sum_nu Ct[p][nu] B_P[mu][nu]      (Ct: nact x ldk, XT: ld ldx)
//  gemm2: b_P = Ct XT_P^T on lower tiles; Kpart[s] += b^2; D[P][p] = b_pp; W[P] = b o beta
//  gemm3: Ypart[s][mu][q] = sum_{P in split s} sum_r XT[P][r][mu] W[P][r][q]
hipError_t df_f64_gemm1(hipStream_t s, int nbf, int nact, int np, const double* Ct, int ldk,
                        const double* Bchunk, double* XT, int ldx);
hipError_t df_f64_gemm2(hipStream_t s, int nbf, int nact, int np, int nsplit, const double* Ct,
                        int ldk, const double* XT, int ldx, const double* beta, double* Kpart,
                        double* Dchunk, double* W, int ldw);
hipError_t df_f64_gemm3(hipStream_t s, int nbf, int nact, int np, int nsplit, const double* XT,
                        int ldx, const double* W, int ldw, double* Ypart);
// Float32 forms (PNOF_FP32): float operands and accumulation, float64 K sums and D; gemm1 reads B as
// stored (bf16 when b_is_bf16, else float64) and rounds it to float.
hipError_t df_f32_gemm1(hipStream_t s, int nbf, int nact, int np, const float* Ct, int ldk, const void* Bchunk,
                        int b_is_bf16, float* XT, int ldx);
hipError_t df_f32_gemm2(hipStream_t s, int nbf, int nact, int np, int nsplit, const float* Ct, int ldk,
                        const float* XT, int ldx, const float* beta32, double* Kpart, double* Dchunk, float* W,
                        int ldw);
hipError_t df_f32_gemm3(hipStream_t s, int nbf, int nact, int np, int nsplit, const float* XT, int ldx,
                        const float* W, int ldw, float* Ypart);

// ---------------------------------------------------------------- bf16 split GEMMs (k_gemm_bf16.hip)
// terms: 1 = hi*hi; 3 = hi*hi + hi*lo + lo*hi.  variant: 0 = 128 x 128 block tiles (two blocks per
// CU), 1 = 128 x 256 (X) or 256 x 128 (Y) block tiles (one block per CU).  B_P given as bf16 (exact, 2 products against the
// split Ct) or as a pre-split hi/lo pair (3 products).
struct SplitPtr {
  const u16* hi;
  const u16* lo;  // may be null when terms == 1 or the operand is exact
};
// Geometry of the split-path workspace operands (see k_gemm_bf16.hip).
struct WsDims {
  int nact32;
  long long ct_bytes, xt_bytes, w_bytes;
};
// Arguments of one launch of each contraction, for one problem (or one instance of a batch).
struct G1Args {   // XT_P[p][mu] = sum_nu Ct[p][nu] B_P[mu][nu]
  int nbf, nact, np;
  const u16* ct_hi;
  const u16* ct_lo;
  int ldk;
  const u16* b_hi;
  const u16* b_lo;
  long long bstride;   // elements between B_P and B_{P+1}
  int ldb;
  long long b_bytes;   // readable bytes from b_hi (and b_lo) onwards
  u16* xt_hi;
  u16* xt_lo;
  int ldx;
  WsDims ws;
  const uint32_t* bnd;   // split mode: the bounds that fix the scales (see chunk_scales)
  int chunk;
};
struct G2Args {   // b_P = Ct XT_P^T; K partials, D, W
  int nbf, nact, np, nsplit;
  const u16* ct_hi;
  const u16* ct_lo;
  int ldk;
  const u16* xt_hi;
  const u16* xt_lo;
  int ldx;
  const float* beta32;
  double* Kpart;
  double* Dc;
  u16* w_hi;
  u16* w_lo;
  int ldw;
  WsDims ws;
  const uint32_t* bnd;
  int chunk;
  // W stored once per 128 x 128 block pair, W_P being symmetric: each tile (on or below the
  // diagonal) writes only its transposed image W[q][p], so W holds the blocks on and above the
  // diagonal; gemm3 with wsym reads it that way
  int wsym = 0;
};
struct G3Args {   // Ypart[s] = sum_{P in s} X_P W_P
  int nbf, nact, np, nsplit;
  const u16* xt_hi;
  const u16* xt_lo;
  int ldx;
  const u16* w_hi;
  const u16* w_lo;
  int ldw;
  float* Ypart;
  WsDims ws;
  const uint32_t* bnd;
  int chunk;
  int wsym = 0;   // W as gemm2 writes it with wsym (see G2Args)
};
// Work items of one launch.  The stacked form of X treats the rows (P, mu) of np consecutive B_P
// as one matrix (B_P rows padded to ldb, bstride == nbf * ldb), so short rows do not waste tiles.
// g1m x g1n: the block tile along (p, mu); grid and kernel must use the same values.
__host__ __device__ inline int g1_items(const G1Args& a, int g1m, int g1n, bool stacked) {
  return cdiv(a.nact, g1m) * (stacked ? cdiv((long long)a.np * a.nbf, g1n) : a.np * cdiv(a.nbf, g1n));
}
// tt: the square tile of the b contraction (128; 64 for the grouped form of short active spaces)
__host__ __device__ inline int g2_items(const G2Args& a, int tt) {
  const int t = cdiv(a.nact, tt);
  return a.nsplit * t * (t + 1) / 2;
}
// g3m x g3n: the block tile along (mu, q); the launch grid and the kernel's decoding of its block
// index must use the same values.
__host__ __device__ inline int g3_items(const G3Args& a, int g3m, int g3n) {
  return a.nsplit * cdiv(a.nbf, g3m) * cdiv(a.nact, g3n);
}

// Grouped launches over the instances of a batch: tab[i] are the arguments of instance i (device
// memory), off[i] the first work item of instance i (off[ninst] = total).  terms as above;
// B must be bf16 (exact) with padded rows, and every leading dimension a multiple of 32.
// tile: width of the tiles along the active orbitals, 128 or 64 (the work-item offsets must be counted
// with the same width: g1_items(.., tile, 128, true), g2_items(.., tile), g3_items(.., 128, tile)).
// The grouped b contraction covers every P of its instances, so it stores its K sums into Kpart
// (no prior clearing) where the single-problem form adds them.
hipError_t df_bf16_gemm1_grouped(hipStream_t s, int ninst, int total, int terms, int tile, const G1Args* tab,
                                 const int* off);
hipError_t df_bf16_gemm2_grouped(hipStream_t s, int ninst, int total, int terms, int tile, const G2Args* tab,
                                 const int* off);
hipError_t df_bf16_gemm3_grouped(hipStream_t s, int ninst, int total, int terms, int tile, const G3Args* tab,
                                 const int* off);

// Split mode (terms > 1): bnd / chunk give the scales of the chunk (chunk_scales); the X output, the
// b operands Ct (fp16 pair of C~ sC) and XT, W and the Y operands are fp16 pairs; X from a float64 B
// takes Ct and B as fp16 pairs (terms 3), from a bf16 B the compact bf16 pair of C (terms 2).
hipError_t df_bf16_gemm1(hipStream_t s, int nbf, int nact, int np, int terms, SplitPtr Ct, int ldk, SplitPtr Bp,
                         long long bstride, int ldb, long long b_bytes, u16* XT_hi, u16* XT_lo, int ldx, int variant,
                         const WsDims& d, const uint32_t* bnd, int chunk);
// wsym: W is written only as the transposed image of b's tiles, i.e. its 128 x 128 blocks on and
// above the diagonal (gemm2), and Y reads each block of W in the orientation that holds it (gemm3);
// split mode, 128 x 128 b tiles, Y on the direct-load path only.
hipError_t df_bf16_gemm2(hipStream_t s, int nbf, int nact, int np, int nsplit, int terms,
                         SplitPtr Ct, int ldk, SplitPtr XT, int ldx, const float* beta32,
                         double* Kpart, double* Dchunk, u16* W_hi, u16* W_lo, int ldw, const WsDims& d,
                         const uint32_t* bnd, int chunk, bool wsym = false);
hipError_t df_bf16_gemm3(hipStream_t s, int nbf, int nact, int np, int nsplit, int terms, SplitPtr XT,
                         int ldx, SplitPtr W, int ldw, float* Ypart, int variant, const WsDims& d,
                         const uint32_t* bnd, int chunk, bool wsym = false);

// ---------------------------------------------------------------- batches (k_batch.hip)
// One instance of a batch: sizes, the caller's inputs and outputs, and its slices of the batch
// workspace.  Leading dimensions: ldk = ldx = round_up(nbf, 32), ldw = nact32 = round_up(nact, 32).
struct BInst {
  int nbf, nact, naux, npairs, ncwo, nsingle, functional, terms;
  int ldk, ldw, nact32, ns2, ns3;
  const double* C;
  const double* n;
  const double* H;
  const u16* B;         // caller's bf16 B, naux x nbf x nbf
  double* lam;          // caller's outputs (dEdC, dEdn, asym may be null)
  double* E;
  double* dEdC;
  double* dEdn;
  double* asym;
  u16* Bp;              // packed B: naux x nbf x ldk, zero pads
  double *alpha, *beta, *HC, *Hpp, *J, *K, *Kpart, *D, *dbuf, *Y2e, *Y;
  double* epart;        // BATCH_EPARTS energy partials, summed in order by the last launch
  float* beta32;
  float* Ypart;
  u16 *cth, *ctl, *xth, *xtl, *wh, *wl;
  u16 *ch16, *cl16;     // split mode: fp16 pair of C~ sC (the b contraction's operand)
  uint32_t* bnd;        // split mode: scale bounds (SCL_CALL call-level words, then the words of B)
  float* colb;          // split mode: per-orbital bounds (4 nact)
  const double* gamma;  // optional: ON-map variables (on_kind), for dE/dgamma
  double* dEdgamma;     // optional output
  int on_kind;
};
// Blocks per instance that sum the energy (each writes one partial to epart).
constexpr int BATCH_EPARTS = 32;
// Each launch covers every instance (blockIdx.y = instance); maxima size the grids.
struct BMax {
  int nbf, nact;
  long long pack, zero, prep, y, k, diag, rows;
};
hipError_t batch_pack(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);   // B -> Bp, zero workspace
hipError_t batch_b_bounds(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);   // row bounds of B (at bind)
hipError_t batch_bounds(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);     // call-level scale bounds
hipError_t batch_prep(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);   // coeffs, split C_A
hipError_t batch_hpp(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);
hipError_t batch_add_diag(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);
hipError_t batch_reduce(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);  // Y2e, K
hipError_t batch_energy_y(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);
hipError_t batch_finish(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);  // lambda cols, dE/dC, dE/dn, asym
hipError_t batch_vjp(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);     // dE/dgamma (instances with gamma)

// ---------------------------------------------------------------- persistent batch kernel (k_gemm_bf16.hip)
// One launch runs every step of every instance: blocks claim work items of an instance's current
// phase (all items of the previous phase complete), in instance order.  Phases of one instance:
enum {
  PH_PREP = 0,   // scale bounds, alpha/beta, C split (one item)
  PH_X,          // X tiles, then the float64 tiles of H C_A
  PH_B,          // b tiles (64-wide), then H_pp (one item)
  PH_DJ,         // float64 tiles of D alpha, then of J = D^T D
  PH_DIAG,       // W diagonal
  PH_Y,          // Y tiles
  PH_RED,        // Y2e and K reductions
  PH_EY,         // BATCH_EPARTS energy partials, then Y = n o (H C_A) + Y2e
  PH_LAM,        // float64 tiles of lambda = C^T Y
  PH_FIN,        // E, lambda columns, dE/dC, asymmetry, dE/dn
  PH_VJP,        // dE/dgamma; the instance's completion time
  PH_N
};
constexpr int PERSIST_PARTS = 8;   // items of the element-wise phases (W diagonal, reductions, Y, finish)
constexpr int PERSIST_XG = 4;      // X tiles per work item (consecutive tiles share their rows of B)
constexpr int PERSIST_MAX_DIES = 16;   // accelerator complex dies (one L2 each) a device may have
// Scheduling state (device memory, cleared by batch_persist before each run).
struct PSched {
  const int* cnt;                 // [ninst][PH_N] items of each phase
  int* claim;                     // [ninst][PH_N] items handed out
  int* done;                      // [ninst][PH_N] items completed
  int* phase;                     // [ninst] first phase not complete
  unsigned long long* t_end;      // [ninst] device wall clock when the instance completed
  unsigned long long* t_start;    // device wall clock when the run started
  int* prog;                      // [0] items completed, [1] instances completed, [2] stalled
  const int* order;               // instances grouped by the die that runs them, each group ascending
  const int* xoff;                // [ndie + 1]: group x is order[xoff[x] .. xoff[x + 1])
  int* die_of;                    // [ndie]: the hardware die id that took group x (-1 before)
  int ndie;                       // the device's dies; a block of die id d serves group d % ndie
  unsigned long long stall_ticks; // device-clock ticks with no progress anywhere before a block gives up
};
struct PArgs {
  int ninst, terms;
  const BInst* inst;
  const G1Args* g1;
  const G2Args* g2;
  const G3Args* g3;
  const F64Gemm* f64;             // [4][ninst]: H C_A, D alpha, D^T D, C^T Y
  PSched sc;
};
// Items of instance i in each phase for X / Y tile widths tx, ty (the b contraction runs 64-wide).
void persist_counts(const BInst& d, const G1Args& g1, const G2Args& g2, const G3Args& g3, int tx, int ty, int* cnt);
// Clears the scheduling state, stamps the start and runs the persistent kernel (grid: blocks).
hipError_t batch_persist(hipStream_t s, const PArgs& a, int ninst_state_words, int tx, int ty, int blocks);

// ---------------------------------------------------------------- small kernels (k_small.hip)
hipError_t fill_f64(hipStream_t s, double* p, long long n, double v);
hipError_t fill_u16(hipStream_t s, u16* p, long long n, u16 v);
// zero columns [cols, ld) of rows [0, rows) and rows [rows, rows_pad) of nslice slices
hipError_t zero_pads_u16(hipStream_t s, u16* base, int nslice, long long sstride, int rows, int rows_pad, int ld,
                         int cols);
hipError_t coeffs(hipStream_t s, int nact, int npairs, int ncwo, int nsingle, int functional, const double* n,
                  double* alpha, double* beta, float* beta32);
hipError_t transpose_ca(hipStream_t s, int nbf, int nact, const double* C, double* Ct, int ldk);
hipError_t transpose_ca_f32(hipStream_t s, int nbf, int nact, const double* C, float* Ct, int ldk);
// The occupations and the subspace layout (the structure of the Coulomb coefficients alpha).
struct OccLayout {
  const double* n;
  int npairs, ncwo, nsingle;
};
// float32 W: d = Dchunk alpha as in add_diag_f64, then W_P[p][p] += d[P][p].
hipError_t add_diag_f32(hipStream_t s, int nact, int np, const double* Dchunk, const OccLayout& oc, double* dbuf,
                        float* W, int ldw);
// C_A^T as bf16 (terms 1) or, in the split mode, the compact bf16 pair (hi, lo) plus the fp16 pair
// (h16, l16) of the same value times sC (bnd: call-level words already formed).
hipError_t split_ca(hipStream_t s, int nbf, int nact, int terms, const double* C, u16* Ct_hi,
                    u16* Ct_lo, u16* Ct_h16, u16* Ct_l16, int ldk, const uint32_t* bnd);
// float64 B rows of one chunk as the fp16 pair of B sB.
hipError_t split_b(hipStream_t s, long long n, const double* B, u16* hi, u16* lo, const uint32_t* bnd, int chunk);
// Call-level scale bounds from C_A and n (col: 4 nact floats of scratch) into bnd[0..SCL_CALL), and
// the nclear per-chunk words after them cleared.
hipError_t scale_bounds(hipStream_t s, int nbf, int nact, const double* C, const double* n, int npairs, int ncwo,
                        int nsingle, int functional, float* col, uint32_t* bnd, int nclear);
// Per chunk of rows_per_chunk rows of B (nrows rows, ncols used of ld): the largest row 1-norm and the
// largest |B|, raised into slot[2c], slot[2c + 1] (the words must start at zero).
hipError_t b_bounds(hipStream_t s, const void* B, int is_f64, long long nrows, int ncols, long long ld,
                    long long rows_per_chunk, uint32_t* slot);
hipError_t widen_bf16(hipStream_t s, long long n, const u16* src, double* dst);
hipError_t hpp_from_hc(hipStream_t s, int nbf, int nact, const double* C, const double* HC, double* Hpp);
// Split-K float64 product for few output tiles: ks (<= F64_KSPLIT_MAX) dense M x N partial slabs in
// Cpart, summed by the caller in slab order.  gemm_f64_ksplit gives the split used for a shape.
constexpr int F64_KSPLIT_MAX = 8;
int gemm_f64_ksplit(int M, int N, int K);
hipError_t gemm_f64_splitk(hipStream_t s, int M, int N, int K, int ks, const double* A, long long sam, long long sak,
                           const double* B, long long sbk, long long sbn, double* Cpart);
// d = Dchunk alpha (np x nact into dbuf), formed from the structure of alpha (2 n_p n_q between
// subspaces, 0 within one) in O(np nact), then W_P[p][p] += d[P][p].  The split form rebuilds the
// diagonal from Dchunk (the b contraction's float accumulators b^P_pp) as float(b^P_pp * beta32_pp) +
// d[P][p] and only writes it, so W's scattered diagonal is never read back.
hipError_t add_diag_f64(hipStream_t s, int nact, int np, const double* Dchunk, const OccLayout& oc,
                        double* dbuf, double* W, int ldw);
hipError_t add_diag_bf16(hipStream_t s, int nact, int np, const double* Dchunk, const OccLayout& oc,
                         const float* beta32, double* dbuf, u16* W_hi, u16* W_lo, int ldw, long long pstride,
                         const uint32_t* bnd, int chunk);
hipError_t reduce_k(hipStream_t s, int nact, int nsplit, const double* Kpart, double* K);
hipError_t reduce_y_f64(hipStream_t s, long long n, int nsplit, const double* Ypart, double* Y);
hipError_t reduce_y_f32(hipStream_t s, long long n, int nsplit, const float* Ypart, double* Y);
hipError_t energy(hipStream_t s, int nbf, int nact, const double* n, const double* Hpp,
                  const double* alpha, const double* beta, const double* J, const double* K,
                  const double* Y2e, const double* C, const u16* Ct_hi, const u16* Ct_lo, const float* Ct32, int ldk,
                  int corr_terms, double* partials, double* E);
hipError_t assemble_y(hipStream_t s, int nbf, int nact, const double* n, const double* HC,
                      const double* Y2e, double* Y);
hipError_t grad_c(hipStream_t s, int nbf, int nact, const double* Y, double* dEdC);
hipError_t zero_cols(hipStream_t s, int nbf, int col0, double* M);
hipError_t max_asym(hipStream_t s, int nbf, const double* lam, double* partials, double* out);
hipError_t grad_n(hipStream_t s, int nact, int npairs, int ncwo, int nsingle, int functional, const double* n,
                  const double* Hpp, const double* J, const double* K, double* dEdn);
hipError_t on_map(hipStream_t s, int kind, int npairs, int ncwo, int nsingle, const double* gamma, double* n,
                  double* jac);
hipError_t on_map_vjp(hipStream_t s, int kind, int npairs, int ncwo, int nsingle, const double* gamma,
                      const double* dEdn, double* dEdgamma);
hipError_t build_s(hipStream_t s, int nbf, const double* lam, const double* diag_prev, double zeta,
                   double* S);
hipError_t sign_fix_cols(hipStream_t s, int nbf, double* Ucm);
// Householder reduction to tridiagonal form (k_eig.hip), one launch per column: A (n x n symmetric,
// row-major) is overwritten; d (n), e (n - 1), tau (n - 1) and the reflectors as rows of Vh (n x n,
// read column-major: the lower-storage layout of ormtr); p2: 2n doubles of scratch.
constexpr int TRIDIAG_MAX_N = 2048;   // three float64 vectors of n in LDS
hipError_t tridiag_f64(hipStream_t s, int n, double* A, double* Vh, double* p2, double* d, double* e, double* tau);
// Q = H_0 ... H_{n-2} (column-major n x n) from the reflectors of tridiag_f64 (Vh, tau), applied in
// blocks of QNB as float64 GEMMs.  ws: form_q_ws_doubles(n) doubles.  3 <= n <= TRIDIAG_MAX_N.
constexpr int QNB = 128;
constexpr int FORMQ_KS = 8;   // k-splits of Q's skinny products
inline int formq_blocks(int n) { return (n - 1 + QNB - 1) / QNB; }
long long form_q_ws_doubles(int n);
hipError_t form_q_f64(hipStream_t s, int n, const double* Vh, const double* tau, double* ws, double* Q);
hipError_t offdiag_copy(hipStream_t s, int nbf, const double* src, double* dst);
// E_hf and E_sta (device scalars) from n, H_pp, J, K; partials: 256 doubles of scratch.
hipError_t nofmp2_terms(hipStream_t s, int nact, int npairs, int ncwo, int nsingle, const double* n, const double* Hpp,
                        const double* J, const double* K, double* partials, double* E_hf, double* E_sta);
hipError_t count_nonfinite(hipStream_t s, const void* p, long long n, int is_bf16, int* flag);
// explicit four-index integrals (nbf <= 64)
hipError_t eri_jk_ao(hipStream_t s, int nbf, int nact, const double* ERI, const double* C,
                     double* Jr, double* Kr);
hipError_t eri_jk_no(hipStream_t s, int nbf, int nact, const double* C, const double* Jr,
                     const double* Kr, double* J, double* K);
hipError_t eri_y(hipStream_t s, int nbf, int nact, const double* C, const double* n,
                 const double* HC, const double* alpha, const double* beta, const double* Jr,
                 const double* Kr, double* Y2e);
hipError_t gather_ao(hipStream_t s, int nbf, int nq, const int32_t* q_idx, const double* src,
                     double* dst);
hipError_t eri_fock_ao(hipStream_t s, int nbf, int nact, int nq, const int32_t* q_idx,
                       const double* n, const double* H, const double* alpha, const double* beta,
                       const double* Jr, const double* Kr, double* Fq);
// density-fitted per-orbital AO matrices, accumulated one P-chunk at a time
hipError_t df_ao_accum(hipStream_t s, int nbf, int nact, int np, int nq, const int32_t* q_idx,
                       const void* Bchunk, int b_is_bf16, const double* Dchunk,
                       const double* alpha, const double* beta, const double* XT, const float* XT32, const u16* XT_hi,
                       const u16* XT_lo, int ldx, long long xps, double* Jq, double* Kq, double* Fq,
                       const uint32_t* bnd, int chunk);
hipError_t fock_ao_h(hipStream_t s, int nbf, int nq, const int32_t* q_idx, const double* n,
                     const double* H, double* Fq);

}  // namespace pnof
