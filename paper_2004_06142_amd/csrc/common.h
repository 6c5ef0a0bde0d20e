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

__host__ __device__ inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }
__host__ __device__ inline long long round_up(long long a, long long b) { return (a + b - 1) / b * b; }

// ---------------------------------------------------------------- f64 GEMM (k_gemm_f64.hip)
// C[b] = alpha * A[b] B[b] + beta * C[b] with strided views
//   A(m,k) = A[b*sab + m*sam + k*sak], B(k,n) = B[b*sbb + k*sbk + n*sbn], C(m,n) = C[b*scb + m*scm + n*scn]
// Exactly one of sam/sak and one of sbk/sbn must be 1.
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

hipError_t df_bf16_gemm1(hipStream_t s, int nbf, int nact, int np, int terms, SplitPtr Ct, int ldk, SplitPtr Bp,
                         long long bstride, int ldb, long long b_bytes, u16* XT_hi, u16* XT_lo, int ldx, int variant,
                         const WsDims& d);
hipError_t df_bf16_gemm2(hipStream_t s, int nbf, int nact, int np, int nsplit, int terms,
                         SplitPtr Ct, int ldk, SplitPtr XT, int ldx, const float* beta32,
                         double* Kpart, double* Dchunk, u16* W_hi, u16* W_lo, int ldw, const WsDims& d);
hipError_t df_bf16_gemm3(hipStream_t s, int nbf, int nact, int np, int nsplit, int terms, SplitPtr XT,
                         int ldx, SplitPtr W, int ldw, float* Ypart, int variant, const WsDims& d);

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
};
// Blocks per instance that sum the energy (each writes one partial to epart).
constexpr int BATCH_EPARTS = 32;
// Each launch covers every instance (blockIdx.y = instance); maxima size the grids.
struct BMax {
  int nbf, nact;
  long long pack, zero, prep, y, k, diag;
};
hipError_t batch_pack(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);   // B -> Bp, zero workspace
hipError_t batch_prep(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);   // coeffs, split C_A, zero K partials
hipError_t batch_hpp(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);
hipError_t batch_add_diag(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);
hipError_t batch_reduce(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);  // Y2e, K
hipError_t batch_energy_y(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);
hipError_t batch_finish(hipStream_t s, int ninst, const BInst* tab, const BMax& mx);  // lambda cols, dE/dC, dE/dn, asym

// ---------------------------------------------------------------- small kernels (k_small.hip)
hipError_t fill_f64(hipStream_t s, double* p, long long n, double v);
hipError_t fill_u16(hipStream_t s, u16* p, long long n, u16 v);
// zero columns [cols, ld) of rows [0, rows) and rows [rows, rows_pad) of nslice slices
hipError_t zero_pads_u16(hipStream_t s, u16* base, int nslice, long long sstride, int rows, int rows_pad, int ld,
                         int cols);
hipError_t coeffs(hipStream_t s, int nact, int npairs, int ncwo, int nsingle, int functional, const double* n,
                  double* alpha, double* beta, float* beta32);
hipError_t transpose_ca(hipStream_t s, int nbf, int nact, const double* C, double* Ct, int ldk);
hipError_t split_ca(hipStream_t s, int nbf, int nact, int terms, const double* C, u16* Ct_hi,
                    u16* Ct_lo, int ldk);
hipError_t split_b(hipStream_t s, long long n, const double* B, u16* hi, u16* lo);
hipError_t widen_bf16(hipStream_t s, long long n, const u16* src, double* dst);
hipError_t hpp_from_hc(hipStream_t s, int nbf, int nact, const double* C, const double* HC, double* Hpp);
// Split-K float64 product for few output tiles: ks (<= F64_KSPLIT_MAX) dense M x N partial slabs in
// Cpart, summed by the caller in slab order.  gemm_f64_ksplit gives the split used for a shape.
constexpr int F64_KSPLIT_MAX = 8;
int gemm_f64_ksplit(int M, int N, int K);
hipError_t gemm_f64_splitk(hipStream_t s, int M, int N, int K, int ks, const double* A, long long sam, long long sak,
                           const double* B, long long sbk, long long sbn, double* Cpart);
// d = Dchunk alpha (float64 matrix cores, split over k into the F64_KSPLIT_MAX * np * nact doubles of
// dbuf), then W_P[p][p] += d[P][p].  The split form rebuilds the diagonal from Dchunk (the b
// contraction's float accumulators b^P_pp) as float(b^P_pp * beta32_pp) + d[P][p] and only writes it,
// so W's scattered diagonal is never read back.
hipError_t add_diag_f64(hipStream_t s, int nact, int np, const double* Dchunk, const double* alpha,
                        double* dbuf, double* W, int ldw);
hipError_t add_diag_bf16(hipStream_t s, int nact, int np, const double* Dchunk, const double* alpha,
                         const float* beta32, double* dbuf, u16* W_hi, u16* W_lo, int ldw, long long pstride);
hipError_t reduce_k(hipStream_t s, int nact, int nsplit, const double* Kpart, double* K);
hipError_t reduce_y_f64(hipStream_t s, long long n, int nsplit, const double* Ypart, double* Y);
hipError_t reduce_y_f32(hipStream_t s, long long n, int nsplit, const float* Ypart, double* Y);
hipError_t energy(hipStream_t s, int nbf, int nact, const double* n, const double* Hpp,
                  const double* alpha, const double* beta, const double* J, const double* K,
                  const double* Y2e, const double* C, const u16* Ct_hi, const u16* Ct_lo, int ldk,
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
// blocks of ORMTR_NB.  Tall: workspace of ormtr_tblocks(n) * ORMTR_NB^2 doubles.  3 <= n <= TRIDIAG_MAX_N.
constexpr int ORMTR_NB = 32;
inline int ormtr_tblocks(int n) { return (n - 1 + ORMTR_NB - 1) / ORMTR_NB; }
hipError_t form_q_f64(hipStream_t s, int n, const double* Vh, const double* tau, double* Tall, double* Q);
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
                       const double* alpha, const double* beta, const double* XT, const u16* XT_hi,
                       const u16* XT_lo, int ldx, long long xps, double* Jq, double* Kq, double* Fq);
hipError_t fock_ao_h(hipStream_t s, int nbf, int nq, const int32_t* q_idx, const double* n,
                     const double* H, double* Fq);

}  // namespace pnof
