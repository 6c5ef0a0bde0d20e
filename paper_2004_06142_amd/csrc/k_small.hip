// Element-wise, reduction and small-matrix kernels of the PNOF step (float64 throughout).
#include <algorithm>

#include "common.h"

namespace pnof {
namespace {

constexpr int NT = 256;

inline dim3 grid1(long long n, int per = NT) {
  long long b = (n + per - 1) / per;
  if (b < 1) b = 1;
  if (b > 65535LL * 16) b = 65535LL * 16;
  return dim3((unsigned)b);
}

#define GRID_STRIDE(i, n) \
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)

__global__ void fill_f64_k(double* p, long long n, double v) { GRID_STRIDE(i, n) p[i] = v; }
__global__ void fill_u16_k(u16* p, long long n, u16 v) { GRID_STRIDE(i, n) p[i] = v; }

// Zero the pads of nslice row-major slices (slice stride sstride): columns [cols, ld) of rows
// [0, rows), and rows [rows, rows_pad) in full.
__global__ void zero_pads_u16_k(u16* __restrict__ base, int nslice, long long sstride, int rows, int rows_pad, int ld,
                                int cols) {
  const long long side = (long long)rows * (ld - cols), per = side + (long long)(rows_pad - rows) * ld;
  GRID_STRIDE(i, (long long)nslice * per) {
    const long long sl = i / per, j = i % per;
    long long r, c;
    if (j < side) {
      r = j / (ld - cols);
      c = cols + j % (ld - cols);
    } else {
      r = rows + (j - side) / ld;
      c = (j - side) % ld;
    }
    base[sl * sstride + r * ld + c] = 0;
  }
}

// alpha, beta of E_2 = sum_pq alpha_pq J_pq + beta_pq K_pq (Eqs. Eg, Efg, Efg_s).
__global__ void coeffs_k(int nact, int npairs, int ncwo, int nsingle, int functional, const double* __restrict__ n,
                         double* __restrict__ alpha, double* __restrict__ beta, float* __restrict__ beta32) {
  GRID_STRIDE(i, (long long)nact * nact) {
    const int p = (int)(i / nact), q = (int)(i % nact);
    double a, b;
    pnof_coeff(p, q, n[p], n[q], npairs, ncwo, nsingle, functional, a, b);
    alpha[i] = a;
    beta[i] = b;
    if (beta32) beta32[i] = (float)b;
  }
}

__global__ void transpose_ca_k(int nbf, int nact, const double* __restrict__ C, double* __restrict__ Ct, int ldk) {
  GRID_STRIDE(i, (long long)nact * nbf) {
    const int p = (int)(i / nbf), mu = (int)(i % nbf);
    Ct[(long long)p * ldk + mu] = C[(long long)mu * nbf + p];
  }
}
__global__ void transpose_ca_f32_k(int nbf, int nact, const double* __restrict__ C, float* __restrict__ Ct, int ldk) {
  GRID_STRIDE(i, (long long)nact * nbf) {
    const int p = (int)(i / nbf), mu = (int)(i % nbf);
    Ct[(long long)p * ldk + mu] = (float)C[(long long)mu * nbf + p];
  }
}

// C_A^T as bf16: one value (terms 1), or the compact bf16 pair C~ = hi + lo of X's contraction plus
// the exact fp16 pair of C~ sC for the b contraction (and X from a float64 B).
__global__ void split_ca_k(int nbf, int nact, int terms, const double* __restrict__ C, u16* __restrict__ hi,
                           u16* __restrict__ lo, u16* __restrict__ h16, u16* __restrict__ l16, int ldk,
                           const uint32_t* __restrict__ bnd) {
  const float sC = terms > 1 ? chunk_scales(bnd, 0, false).sC : 1.0f;
  GRID_STRIDE(i, (long long)nact * nbf) {
    const int p = (int)(i / nbf), mu = (int)(i % nbf);
    const long long o = (long long)p * ldk + mu;
    const double x = C[(long long)mu * nbf + p];
    if (terms == 1) {
      hi[o] = f32_to_bf16_bits((float)x);
      continue;
    }
    u16 h, l;
    split_compact(x, h, l);
    hi[o] = h;
    lo[o] = l;
    // hi + lo spans at most 22 bits: exact in float32, and its fp16 pair is exact (split_compact)
    const float xs = (bf16_bits_to_f32(h) + bf16_bits_to_f32(l)) * sC;
    u16 a, b;
    split_f16(xs, a, b);
    h16[o] = a;
    l16[o] = b;
  }
}

// float64 B as the fp16 pair of B sB (sB of the chunk), or as one bf16 value when bnd is null.
__global__ void split_b_k(long long n, const double* __restrict__ B, u16* __restrict__ hi, u16* __restrict__ lo,
                          const uint32_t* __restrict__ bnd, int chunk) {
  if (!bnd) {
    GRID_STRIDE(i, n) hi[i] = f32_to_bf16_bits((float)B[i]);
    return;
  }
  const float sB = chunk_scales(bnd, chunk, true).sB;
  GRID_STRIDE(i, n) {
    u16 h, l;
    const double xs = B[i] * (double)sB;
    h = f32_to_f16_bits((float)xs);
    l = f32_to_f16_bits((float)(xs - (double)f16_bits_to_f32(h)));
    hi[i] = h;
    lo[i] = l;
  }
}

// Scale bounds, stage 1: one wavefront per active orbital q writes col[4q..4q+3] = sum_mu |C_mu q|,
// max_mu |C_mu q|, sum_r |alpha_qr|, max_r |beta_qr| (alpha, beta of Eqs. Eg, Efg from n; zero when
// n is absent).
__global__ void col_bounds_k(int nbf, int nact, const double* __restrict__ C, const double* __restrict__ n,
                             int npairs, int ncwo, int nsingle, int functional, float* __restrict__ col) {
  const int lane = threadIdx.x & 63;
  const int q = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (q >= nact) return;
  double s1 = 0.0, cm = 0.0, sa = 0.0, bm = 0.0;
  for (int mu = lane; mu < nbf; mu += 64) {
    const double c = fabs(C[(long long)mu * nbf + q]);
    s1 += c;
    cm = fmax(cm, c);
  }
  if (n) {
    for (int r = lane; r < nact; r += 64) {
      double a, b;
      pnof_coeff(q, r, n[q], n[r], npairs, ncwo, nsingle, functional, a, b);
      sa += fabs(a);
      bm = fmax(bm, fabs(b));
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    s1 += __shfl_down(s1, off, 64);
    sa += __shfl_down(sa, off, 64);
    cm = fmax(cm, __shfl_down(cm, off, 64));
    bm = fmax(bm, __shfl_down(bm, off, 64));
  }
  if (lane == 0) {
    col[4 * q + 0] = (float)s1;
    col[4 * q + 1] = (float)cm;
    col[4 * q + 2] = (float)sa;
    col[4 * q + 3] = (float)bm;
  }
}

// Scale bounds, stage 2 (one block): the call-level words of bnd, and the per-chunk words cleared.
__global__ void bounds_reduce_k(int nact, const float* __restrict__ col, uint32_t* __restrict__ bnd, int nclear) {
  __shared__ float red[4][NT / 64];
  float v[4] = {0.f, 0.f, 0.f, 0.f};
  for (int q = threadIdx.x; q < nact; q += blockDim.x)
    for (int k = 0; k < 4; ++k) v[k] = fmaxf(v[k], col[4 * q + k]);
  for (int off = 32; off > 0; off >>= 1)
    for (int k = 0; k < 4; ++k) v[k] = fmaxf(v[k], __shfl_down(v[k], off, 64));
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < 4; ++k)
      for (int w = 1; w < NT / 64; ++w) red[k][0] = fmaxf(red[k][0], red[k][w]);
    bnd[0] = __float_as_uint(red[1][0]);                 // max |C|
    bnd[1] = __float_as_uint(red[0][0]);                 // max column 1-norm
    bnd[2] = __float_as_uint(red[3][0] + red[2][0]);     // max |beta| + max row 1-norm of alpha
    bnd[3] = 0u;
  }
  for (int i = threadIdx.x; i < nclear; i += blockDim.x) bnd[SCL_CALL + i] = 0u;
}

// Row bounds of B (nrows rows of ncols elements, leading dimension ld): for every chunk of
// rows_per_chunk consecutive rows, the largest row 1-norm and the largest |B|, raised into
// slot[2c], slot[2c + 1] with integer atomic maxima on the bits of the non-negative floats.  One
// wavefront per row; each wavefront walks a contiguous range of rows and raises a chunk's words when
// it leaves that chunk.
template <bool F64, bool VEC>
__global__ void b_bounds_k(const void* __restrict__ B, long long nrows, int ncols, long long ld,
                           long long rows_per_chunk, uint32_t* __restrict__ slot) {
  const int lane = threadIdx.x & 63;
  const long long nw = (long long)gridDim.x * (blockDim.x >> 6);
  const long long w = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const long long per = (nrows + nw - 1) / nw;
  const long long r0 = w * per, r1 = r0 + per < nrows ? r0 + per : nrows;
  float rmax = 0.f, amax = 0.f;
  long long cur = r0 < r1 ? r0 / rows_per_chunk : -1;
  auto flush = [&]() {
    if (lane == 0 && cur >= 0) {
      if (rmax > 0.f) atomicMax(slot + 2 * cur, __float_as_uint(rmax));
      if (amax > 0.f) atomicMax(slot + 2 * cur + 1, __float_as_uint(amax));
    }
    rmax = 0.f;
    amax = 0.f;
  };
  for (long long r = r0; r < r1; ++r) {
    if (r / rows_per_chunk != cur) {
      flush();
      cur = r / rows_per_chunk;
    }
    float s = 0.f, a = 0.f;
    if constexpr (F64) {
      const double* row = static_cast<const double*>(B) + r * ld;
      for (int c = lane; c < ncols; c += 64) {
        const float v = (float)fabs(row[c]);
        s += v;
        a = fmaxf(a, v);
      }
    } else if constexpr (VEC) {
      const u16* row = static_cast<const u16*>(B) + r * ld;
      for (int c = 8 * lane; c < ncols; c += 512) {
        const uint4 v = *reinterpret_cast<const uint4*>(row + c);
        const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float x = fabsf(__uint_as_float(wd[k] << 16)), y = fabsf(__uint_as_float(wd[k] & 0xFFFF0000u));
          s += x + y;
          a = fmaxf(a, fmaxf(x, y));
        }
      }
    } else {
      const u16* row = static_cast<const u16*>(B) + r * ld;
      for (int c = lane; c < ncols; c += 64) {
        const float v = fabsf(bf16_bits_to_f32(row[c]));
        s += v;
        a = fmaxf(a, v);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      s += __shfl_down(s, off, 64);
      a = fmaxf(a, __shfl_down(a, off, 64));
    }
    rmax = fmaxf(rmax, __shfl(s, 0, 64));
    amax = fmaxf(amax, __shfl(a, 0, 64));
  }
  flush();
}

// Hpp[p] = sum_mu C[mu][p] HC[mu][p]: one wavefront per orbital, fixed reduction order.
__global__ void hpp_k(int nbf, int nact, const double* __restrict__ C, const double* __restrict__ HC,
                      double* __restrict__ Hpp) {
  const int p = blockIdx.x;
  const int lane = threadIdx.x;
  double s = 0.0;
  for (int mu = lane; mu < nbf; mu += 64) s += C[(long long)mu * nbf + p] * HC[(long long)mu * nact + p];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) Hpp[p] = s;
}

// W_P[p][p] += d[P][p], with d = D alpha (d_Pp = sum_q D_Pq alpha_qp) computed beforehand as ks
// partial slabs over ranges of q, added here in slab order.
__device__ __forceinline__ double sum_slabs(const double* __restrict__ d, int ks, long long slab, long long i) {
  double v = 0.0;
  for (int s = 0; s < ks; ++s) v += d[s * slab + i];
  return v;
}

// d[P][q] = sum_p D[P][p] alpha_pq.  The Coulomb coefficients are alpha_pq = 2 n_p n_q between
// different subspaces and 0 within one (Eqs. Eg, Efg), so d = 2 n_q (s_P - S_P,g(q)) with
// s_P = sum_p n_p D[P][p] and S_P,g the same sum over q's own subspace (a strong orbital and its weak
// ones, or one singly occupied orbital): O(nact) per row instead of a product with alpha.  One
// workgroup per row P; the row sum is reduced in a fixed order.
__global__ void d_alpha_k(int nact, int npairs, int ncwo, int nsingle, const double* __restrict__ n,
                          const double* __restrict__ Dc, double* __restrict__ d) {
  const int P = blockIdx.x, tid = threadIdx.x;
  const double* Dr = Dc + (long long)P * nact;
  __shared__ double red[NT / 64];
  double v = 0.0;
  for (int p = tid; p < nact; p += NT) v += n[p] * Dr[p];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double sP = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) sP += red[w];
  for (int q = tid; q < nact; q += NT) {
    const int g = pair_of(q, npairs, ncwo, nsingle);
    double Sg;
    if (g < npairs) {
      Sg = n[g] * Dr[g];
      for (int k = 0; k < ncwo; ++k) {
        const int w = weak_index(g, k, npairs, ncwo, nsingle);
        Sg += n[w] * Dr[w];
      }
    } else {
      Sg = n[q] * Dr[q];
    }
    d[(long long)P * nact + q] = 2.0 * n[q] * (sP - Sg);
  }
}

__global__ void add_diag_f64_k(int nact, int np, int ks, const double* __restrict__ d, double* __restrict__ W,
                               int ldw) {
  const long long slab = (long long)np * nact;
  GRID_STRIDE(i, slab) {
    const long long P = i / nact;
    const int p = (int)(i % nact);
    W[P * nact * ldw + (long long)p * ldw + p] += sum_slabs(d, ks, slab, i);
  }
}

__global__ void add_diag_f32_k(int nact, int np, int ks, const double* __restrict__ d, float* __restrict__ W, int ldw) {
  const long long slab = (long long)np * nact;
  GRID_STRIDE(i, slab) {
    const long long P = i / nact;
    const int p = (int)(i % nact);
    float* w = W + P * nact * ldw + (long long)p * ldw + p;
    *w = (float)((double)*w + sum_slabs(d, ks, slab, i));
  }
}

__global__ void add_diag_bf16_k(int nact, int np, int ks, const double* __restrict__ d, const double* __restrict__ Dc,
                                const float* __restrict__ beta32, u16* __restrict__ Wh, u16* __restrict__ Wl, int ldw,
                                long long pstride, const uint32_t* __restrict__ bnd, int chunk) {
  const long long slab = (long long)np * nact;
  const float sW = Wl ? chunk_scales(bnd, chunk, false).sW : 1.0f;
  GRID_STRIDE(i, slab) {
    const long long P = i / nact;
    const int p = (int)(i % nact);
    const long long o = P * pstride + (long long)p * ldw + p;
    const float wv = (float)Dc[i] * beta32[(long long)p * nact + p];
    const double w = (double)wv + sum_slabs(d, ks, slab, i);
    if (Wl) {   // split mode: the fp16 pair of W sW
      u16 h, l;
      split_f16((float)(w * (double)sW), h, l);
      Wh[o] = h;
      Wl[o] = l;
    } else {
      Wh[o] = f32_to_bf16_bits((float)w);
    }
  }
}

// K[p][q] += sum_s Kpart[s][max][min], mirrored: each lower-triangle position is read along rows
// (coalesced) and added to both halves.
__global__ void reduce_k_k(int nact, int nsplit, const double* __restrict__ Kpart, double* __restrict__ K) {
  GRID_STRIDE(i, (long long)nact * nact) {
    const int p = (int)(i / nact), q = (int)(i % nact);
    if (q > p) continue;
    const double s = sum_strided(Kpart + i, nsplit, (long long)nact * nact);
    K[i] += s;
    if (q != p) K[(long long)q * nact + p] += s;
  }
}

template <typename T>
__global__ void reduce_y_k(long long n, int nsplit, const T* __restrict__ Yp, double* __restrict__ Y) {
  GRID_STRIDE(i, n) {
    Y[i] += sum_strided(Yp + i, nsplit, n);
  }
}

// Energy (Eqs. EPNOF7, Eg, Efg) and, for split arithmetic, the first-order correction
// 4 <Y2e, C_A - C~_A>.  Stage 1: fixed-range block partial sums; stage 2: one block.
__device__ inline double block_sum(double v) {
  __shared__ double red[NT / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

__global__ void energy_stage1_k(int nbf, int nact, const double* __restrict__ n, const double* __restrict__ Hpp,
                                const double* __restrict__ alpha, const double* __restrict__ beta,
                                const double* __restrict__ J, const double* __restrict__ K,
                                const double* __restrict__ Y2e, const double* __restrict__ C,
                                const u16* __restrict__ cth, const u16* __restrict__ ctl,
                                const float* __restrict__ ct32, int ldk, int corr_terms,
                                double* __restrict__ partials) {
  const long long n2 = (long long)nact * nact;
  const long long ncorr = corr_terms > 0 ? (long long)nbf * nact : 0;
  const long long total = nact + n2 + ncorr;
  const long long per = (total + gridDim.x - 1) / gridDim.x;
  const long long b0 = blockIdx.x * per, b1 = min(total, b0 + per);
  double s = 0.0;
  for (long long i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
    if (i < nact) s += 2.0 * n[i] * Hpp[i];
    else if (i < nact + n2) { const long long k = i - nact; s += alpha[k] * J[k] + beta[k] * K[k]; }
    else {
      const long long k = i - nact - n2;
      const int mu = (int)(k / nact), p = (int)(k % nact);
      double ct;
      if (ct32) ct = (double)ct32[(long long)p * ldk + mu];
      else {
        ct = (double)bf16_bits_to_f32(cth[(long long)p * ldk + mu]);
        if (corr_terms > 1) ct += (double)bf16_bits_to_f32(ctl[(long long)p * ldk + mu]);
      }
      s += 4.0 * Y2e[k] * (C[(long long)mu * nbf + p] - ct);
    }
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void sum_partials_k(int nparts, const double* __restrict__ partials, double* __restrict__ out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += partials[i];
  s = block_sum(s);
  if (threadIdx.x == 0) *out = s;
}

// NOF-MP2 reference terms (Eqs. HFL, Esta): block partial sums of E_hf and E_sta over a fixed
// range of the index space [0, nom) + [0, nom^2) + [0, nact^2), nom = npairs + nsingle (the
// subspace-defining orbitals, weight A = 1 strong, 1/2 single); stage 2 adds the partials in order.
__global__ void nofmp2_stage1_k(int nact, int npairs, int ncwo, int nsingle, const double* __restrict__ n,
                                const double* __restrict__ Hpp, const double* __restrict__ J,
                                const double* __restrict__ K, double* __restrict__ partials) {
  const long long n2 = (long long)nact * nact;
  const int nom = npairs + nsingle;
  const long long total = nom + (long long)nom * nom + n2;
  const long long per = (total + gridDim.x - 1) / gridDim.x;
  const long long b0 = blockIdx.x * per, b1 = min(total, b0 + per);
  double hf = 0.0, sta = 0.0;
  for (long long i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
    if (i < nom) {
      const int g = (int)i;
      // 2 A_g H_gg, and minus the self-Coulomb J_gg / 4 of a single orbital
      hf += g < npairs ? 2.0 * Hpp[g] : Hpp[g] - 0.25 * J[(long long)g * nact + g];
    } else if (i < nom + (long long)nom * nom) {
      const long long k = i - nom;
      const int f = (int)(k / nom), g = (int)(k % nom);
      const double af = f < npairs ? 1.0 : 0.5, ag = g < npairs ? 1.0 : 0.5;
      hf += af * ag * (2.0 * J[(long long)f * nact + g] - K[(long long)f * nact + g]);
    } else {
      const long long k = i - nom - (long long)nom * nom;
      const int p = (int)(k / nact), q = (int)(k % nact);
      if (p == q) continue;
      const double np_ = n[p], nq = n[q];
      if (pair_of(p, npairs, ncwo, nsingle) == pair_of(q, npairs, ncwo, nsingle)) {
        const double lp = 1.0 - fabs(1.0 - 2.0 * np_), lq = 1.0 - fabs(1.0 - 2.0 * nq);
        const double sg = (p < npairs || q < npairs) ? -1.0 : 1.0;
        sta += sqrt(lp * lq) * sg * sqrt(np_ * nq) * K[k];
      } else {
        sta += -4.0 * (nq * (1.0 - nq)) * (np_ * (1.0 - np_)) * K[k];
      }
    }
  }
  hf = block_sum(hf);
  sta = block_sum(sta);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = hf;
    partials[2 * blockIdx.x + 1] = sta;
  }
}

__global__ void sum2_partials_k(int nparts, const double* __restrict__ partials, double* __restrict__ a,
                                double* __restrict__ b) {
  double x = 0.0, y = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    x += partials[2 * i];
    y += partials[2 * i + 1];
  }
  x = block_sum(x);
  y = block_sum(y);
  if (threadIdx.x == 0) {
    *a = x;
    *b = y;
  }
}

__global__ void assemble_y_k(int nbf, int nact, const double* __restrict__ n, const double* __restrict__ HC,
                             const double* __restrict__ Y2e, double* __restrict__ Y) {
  GRID_STRIDE(i, (long long)nbf * nact) {
    const int q = (int)(i % nact);
    Y[i] = n[q] * HC[i] + Y2e[i];
  }
}

__global__ void grad_c_k(int nbf, int nact, const double* __restrict__ Y, double* __restrict__ G) {
  GRID_STRIDE(i, (long long)nbf * nbf) {
    const int mu = (int)(i / nbf), q = (int)(i % nbf);
    G[i] = q < nact ? 4.0 * Y[(long long)mu * nact + q] : 0.0;
  }
}

__global__ void zero_cols_k(int nbf, int col0, double* __restrict__ M) {
  const long long w = nbf - col0;
  GRID_STRIDE(i, (long long)nbf * w) {
    const long long r = i / w;
    const int c = col0 + (int)(i % w);
    M[r * nbf + c] = 0.0;
  }
}

__device__ inline double block_max(double v) {
  __shared__ double red[NT / 64];
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) s = fmax(s, red[i]);
  return s;
}

__global__ void asym_stage1_k(int nbf, const double* __restrict__ lam, double* __restrict__ partials) {
  double m = 0.0;
  GRID_STRIDE(i, (long long)nbf * nbf) {
    const long long p = i / nbf, q = i % nbf;
    m = fmax(m, fabs(lam[i] - lam[q * nbf + p]));
  }
  m = block_max(m);
  if (threadIdx.x == 0) partials[blockIdx.x] = m;
}

__global__ void max_partials_k(int nparts, const double* __restrict__ partials, double* __restrict__ out) {
  double m = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) m = fmax(m, partials[i]);
  m = block_max(m);
  if (threadIdx.x == 0) *out = m;
}

// dE/dn_p (derivative of Eqs. Eg, Efg at fixed J, K, H_pp): one wavefront per orbital.
__global__ void grad_n_k(int nact, int npairs, int ncwo, int nsingle, int functional, const double* __restrict__ n,
                         const double* __restrict__ Hpp, const double* __restrict__ J,
                         const double* __restrict__ K, double* __restrict__ g) {
  const int p = blockIdx.x, lane = threadIdx.x;
  const double np_ = n[p];
  const double php = sqrt(np_ * (1.0 - np_));
  double s = 0.0;
  for (int q = lane; q < nact; q += 64) {
    if (q == p) continue;
    s += grad_n_term(p, q, np_, n[q], php, J[(long long)p * nact + q], K[(long long)p * nact + q], npairs, ncwo,
                     nsingle, functional);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  // a singly occupied orbital has no K_pp term (beta_pp = 0); its n is fixed at 1/2
  if (lane == 0) g[p] = 2.0 * Hpp[p] + (is_single(p, npairs, nsingle) ? 0.0 : K[(long long)p * nact + p]) + s;
}


// ON maps, one thread per pair (Section 3.1); singly occupied orbitals get n = 1/2 (their rows of
// the Jacobian stay zero).
__global__ void on_map_k(int kind, int npairs, int ncwo, int nsingle, const double* __restrict__ gamma,
                         double* __restrict__ n, double* __restrict__ jac) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < nsingle) n[npairs + g] = 0.5;
  if (g >= npairs) return;
  const int nact = npairs * (ncwo + 1) + nsingle;
  const int ngam = kind == 0 ? nact : npairs * ncwo;
  if (kind == 0) {
    double S = sigm(gamma[g]);
    for (int k = 0; k < ncwo; ++k) S += sigm(gamma[weak_index(g, k, npairs, ncwo, nsingle)]);
    for (int a = -1; a < ncwo; ++a) {
      const int p = a < 0 ? g : weak_index(g, a, npairs, ncwo, nsingle);
      const double sp = sigm(gamma[p]);
      n[p] = sp / S;
      if (jac) {
        for (int b = -1; b < ncwo; ++b) {
          const int r = b < 0 ? g : weak_index(g, b, npairs, ncwo, nsingle);
          const double sr = sigm(gamma[r]);
          const double dsr = sr * (1.0 - sr);
          jac[(long long)p * ngam + r] = ((p == r ? dsr : 0.0) * S - sp * dsr) / (S * S);
        }
      }
    }
  } else {
    const double gs = gamma[g];
    const double cg = cos(gs), sg = sin(gs);
    n[g] = 0.5 * (1.0 + cg * cg);
    const double h = 0.5 * sg * sg, dh = sg * cg;
    if (jac) jac[(long long)g * ngam + g] = -cg * sg;
    double prod = 1.0;
    for (int i = 0; i < ncwo; ++i) {
      const int p = weak_index(g, i, npairs, ncwo, nsingle);
      const bool last = (i == ncwo - 1);
      const double gi = last ? 0.0 : gamma[npairs + g * (ncwo - 1) + i];
      const double si2 = last ? 1.0 : sin(gi) * sin(gi);
      n[p] = h * prod * si2;
      if (jac) {
        jac[(long long)p * ngam + g] = dh * prod * si2;
        // derivative w.r.t. the earlier weak variables j < i (cos^2 factors)
        for (int j = 0; j < i && j < ncwo - 1; ++j) {
          const double gj = gamma[npairs + g * (ncwo - 1) + j];
          double other = h * si2;
          for (int k = 0; k < i && k < ncwo - 1; ++k) {
            if (k == j) continue;
            const double gk = gamma[npairs + g * (ncwo - 1) + k];
            other *= cos(gk) * cos(gk);
          }
          jac[(long long)p * ngam + npairs + g * (ncwo - 1) + j] = other * (-2.0 * cos(gj) * sin(gj));
        }
        if (!last) jac[(long long)p * ngam + npairs + g * (ncwo - 1) + i] = h * prod * 2.0 * sin(gi) * cos(gi);
      }
      if (!last) prod *= cos(gi) * cos(gi);
    }
  }
}

// dE/dgamma = (dn/dgamma)^T dE/dn, pair by pair (the sigmoid variables of singly occupied orbitals
// do not enter: zero).
__global__ void on_map_vjp_k(int kind, int npairs, int ncwo, int nsingle, const double* __restrict__ gamma,
                             const double* __restrict__ dEdn, double* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < npairs + nsingle) on_map_vjp_subspace(kind, npairs, ncwo, nsingle, gamma, dEdn, out, g);
}

// dst = src with a zero diagonal (the error vector of the DIIS extrapolation).
__global__ void offdiag_k(int nbf, const double* __restrict__ src, double* __restrict__ dst) {
  GRID_STRIDE(i, (long long)nbf * nbf) dst[i] = (i / nbf == i % nbf) ? 0.0 : src[i];
}

// Matrix diagonalised by the orbital step.
__global__ void build_s_k(int nbf, const double* __restrict__ lam, const double* __restrict__ dprev, double zeta,
                          double* __restrict__ S) {
  GRID_STRIDE(i, (long long)nbf * nbf) {
    const long long p = i / nbf, q = i % nbf;
    const double a = lam[p * nbf + q], b = lam[q * nbf + p];
    double v;
    if (!dprev) v = 0.5 * (a + b);
    else if (p == q) v = dprev[p];
    else {
      v = (p < q) ? (b - a) : (a - b);   // S_pq = lambda_qp - lambda_pq for p < q, mirrored
      if (zeta > 0.0)
        while (fabs(v) > zeta) v /= 10.0;
    }
    S[i] = v;
  }
}

// Column j of the column-major eigenvector matrix: make its largest-|.| entry (lowest index on
// ties) positive.  One block per column.
__global__ void sign_fix_k(int nbf, double* __restrict__ U) {
  const int j = blockIdx.x;
  double* col = U + (long long)j * nbf;
  __shared__ double bv[NT];
  __shared__ int bi[NT];
  double best = -1.0;
  int idx = 0;
  for (int i = threadIdx.x; i < nbf; i += blockDim.x) {
    const double a = fabs(col[i]);
    if (a > best) { best = a; idx = i; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = idx;
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double o = bv[threadIdx.x + off];
      const int oi = bi[threadIdx.x + off];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const bool neg = col[bi[0]] < 0.0;
  __syncthreads();
  if (neg)
    for (int i = threadIdx.x; i < nbf; i += blockDim.x) col[i] = -col[i];
}

__global__ void nonfinite_k(const void* p, long long n, int is_bf16, int* flag) {
  int bad = 0;
  GRID_STRIDE(i, n) {
    double v = is_bf16 ? (double)bf16_bits_to_f32(reinterpret_cast<const u16*>(p)[i])
                       : reinterpret_cast<const double*>(p)[i];
    if (!isfinite(v)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

// ---- explicit four-index integrals (nbf <= 64) ----
// Jr[r][m][n] = sum_ls (mn|ls) C_lr C_sr ; Kr[r][m][n] = sum_ls (ml|ns) C_lr C_sr (Eq. Gpmn).
__global__ void eri_jk_ao_k(int nbf, int nact, const double* __restrict__ ERI, const double* __restrict__ C,
                            double* __restrict__ Jr, double* __restrict__ Kr) {
  const long long n2 = (long long)nbf * nbf;
  GRID_STRIDE(i, (long long)nact * n2) {
    const int r = (int)(i / n2);
    const int m = (int)((i % n2) / nbf), n = (int)(i % nbf);
    double sj = 0.0, sk = 0.0;
    for (int l = 0; l < nbf; ++l) {
      const double cl = C[(long long)l * nbf + r];
      double tj = 0.0, tk = 0.0;
      for (int s = 0; s < nbf; ++s) {
        const double cs = C[(long long)s * nbf + r];
        tj += ERI[(((long long)m * nbf + n) * nbf + l) * nbf + s] * cs;
        tk += ERI[(((long long)m * nbf + l) * nbf + n) * nbf + s] * cs;
      }
      sj += cl * tj;
      sk += cl * tk;
    }
    Jr[i] = sj;
    Kr[i] = sk;
  }
}

// J_pq = c_p^T J^q c_p, K_pq = c_p^T K^q c_p (Eq. JKpq).
__global__ void eri_jk_no_k(int nbf, int nact, const double* __restrict__ C, const double* __restrict__ Jr,
                            const double* __restrict__ Kr, double* __restrict__ J, double* __restrict__ K) {
  GRID_STRIDE(i, (long long)nact * nact) {
    const int p = (int)(i / nact), q = (int)(i % nact);
    const double* Jq = Jr + (long long)q * nbf * nbf;
    const double* Kq = Kr + (long long)q * nbf * nbf;
    double sj = 0.0, sk = 0.0;
    for (int m = 0; m < nbf; ++m) {
      double tj = 0.0, tk = 0.0;
      for (int n = 0; n < nbf; ++n) {
        const double cn = C[(long long)n * nbf + p];
        tj += Jq[(long long)m * nbf + n] * cn;
        tk += Kq[(long long)m * nbf + n] * cn;
      }
      const double cm = C[(long long)m * nbf + p];
      sj += cm * tj;
      sk += cm * tk;
    }
    J[i] = sj;
    K[i] = sk;
  }
}

// Y2e[m][q] = sum_r (alpha_qr J^r + beta_qr K^r) c_q.
__global__ void eri_y_k(int nbf, int nact, const double* __restrict__ C, const double* __restrict__ alpha,
                        const double* __restrict__ beta, const double* __restrict__ Jr,
                        const double* __restrict__ Kr, double* __restrict__ Y2e) {
  GRID_STRIDE(i, (long long)nbf * nact) {
    const int m = (int)(i / nact), q = (int)(i % nact);
    double s = 0.0;
    for (int r = 0; r < nact; ++r) {
      const double a = alpha[(long long)q * nact + r], b = beta[(long long)q * nact + r];
      const double* Jm = Jr + ((long long)r * nbf + m) * nbf;
      const double* Km = Kr + ((long long)r * nbf + m) * nbf;
      double tj = 0.0, tk = 0.0;
      for (int n = 0; n < nbf; ++n) {
        const double cn = C[(long long)n * nbf + q];
        tj += Jm[n] * cn;
        tk += Km[n] * cn;
      }
      s += a * tj + b * tk;
    }
    Y2e[i] = s;
  }
}

__global__ void gather_ao_k(int nbf, int nq, const int32_t* __restrict__ q_idx, const double* __restrict__ src,
                            double* __restrict__ dst) {
  const long long n2 = (long long)nbf * nbf;
  GRID_STRIDE(i, (long long)nq * n2) {
    const int k = (int)(i / n2);
    dst[i] = src[(long long)q_idx[k] * n2 + i % n2];
  }
}

__global__ void eri_fock_ao_k(int nbf, int nact, int nq, const int32_t* __restrict__ q_idx,
                              const double* __restrict__ n, const double* __restrict__ H,
                              const double* __restrict__ alpha, const double* __restrict__ beta,
                              const double* __restrict__ Jr, const double* __restrict__ Kr,
                              double* __restrict__ Fq) {
  const long long n2 = (long long)nbf * nbf;
  GRID_STRIDE(i, (long long)nq * n2) {
    const int k = (int)(i / n2);
    const long long e = i % n2;
    const int q = q_idx[k];
    double s = n[q] * H[e];
    for (int r = 0; r < nact; ++r)
      s += alpha[(long long)q * nact + r] * Jr[(long long)r * n2 + e] + beta[(long long)q * nact + r] * Kr[(long long)r * n2 + e];
    Fq[i] = s;
  }
}

__global__ void fock_ao_h_k(int nbf, int nq, const int32_t* __restrict__ q_idx, const double* __restrict__ n,
                            const double* __restrict__ H, double* __restrict__ Fq) {
  const long long n2 = (long long)nbf * nbf;
  GRID_STRIDE(i, (long long)nq * n2) {
    const int k = (int)(i / n2);
    Fq[i] += n[q_idx[k]] * H[i % n2];
  }
}

// Per-orbital AO matrices from one P-chunk:  J^q += sum_P D_Pq B_P,  K^q += sum_P x_Pq x_Pq^T,
// F^q += sum_P [d_Pq B_P + sum_r beta_qr x_Pr x_Pr^T]  with x_Pr[mu] = XT[P][r][mu].
// XT is float64, one bf16 value (terms 1), or the fp16 pair of X sX (split mode; invX = 1 / sX).
__device__ inline double xt_val(const double* XT, const float* XT32, const u16* xh, const u16* xl, double invX,
                                long long o) {
  if (XT) return XT[o];
  if (XT32) return (double)XT32[o];
  if (!xl) return (double)bf16_bits_to_f32(xh[o]);
  return ((double)f16_bits_to_f32(xh[o]) + (double)f16_bits_to_f32(xl[o])) * invX;
}

__global__ void df_ao_accum_k(int nbf, int nact, int np, int nq, const int32_t* __restrict__ q_idx,
                              const void* __restrict__ Bc, int b_bf16, const double* __restrict__ Dc,
                              const double* __restrict__ alpha, const double* __restrict__ beta,
                              const double* __restrict__ XT, const float* __restrict__ XT32, const u16* __restrict__ xh,
                              const u16* __restrict__ xl, int ldx, long long xps, double* __restrict__ Jq,
                              double* __restrict__ Kq, double* __restrict__ Fq, const uint32_t* __restrict__ bnd,
                              int chunk) {
  const long long n2 = (long long)nbf * nbf;
  const double invX = xl ? (double)chunk_scales(bnd, chunk, false).invX : 1.0;
  GRID_STRIDE(i, (long long)nq * n2) {
    const int k = (int)(i / n2);
    const long long e = i % n2;
    const int m = (int)(e / nbf), nn = (int)(e % nbf);
    const int q = q_idx[k];
    double sj = 0.0, sk = 0.0, sf = 0.0;
    for (int P = 0; P < np; ++P) {
      const long long bo = (long long)P * n2 + e;
      const double b = b_bf16 ? (double)bf16_bits_to_f32(reinterpret_cast<const u16*>(Bc)[bo])
                              : reinterpret_cast<const double*>(Bc)[bo];
      const double* Dp = Dc + (long long)P * nact;
      const long long xo = (long long)P * xps;
      sj += Dp[q] * b;
      const double xm = xt_val(XT, XT32, xh, xl, invX, xo + (long long)q * ldx + m);
      const double xn = xt_val(XT, XT32, xh, xl, invX, xo + (long long)q * ldx + nn);
      sk += xm * xn;
      if (Fq) {
        double d = 0.0, kk = 0.0;
        for (int r = 0; r < nact; ++r) {
          d += alpha[(long long)q * nact + r] * Dp[r];
          kk += beta[(long long)q * nact + r] * xt_val(XT, XT32, xh, xl, invX, xo + (long long)r * ldx + m) *
                xt_val(XT, XT32, xh, xl, invX, xo + (long long)r * ldx + nn);
        }
        sf += d * b + kk;
      }
    }
    if (Jq) Jq[i] += sj;
    if (Kq) Kq[i] += sk;
    if (Fq) Fq[i] += sf;
  }
}

}  // namespace

#define LAUNCH(kern, grid, block, ...)                              \
  do {                                                              \
    hipLaunchKernelGGL(kern, grid, block, 0, s, __VA_ARGS__);       \
    return hipGetLastError();                                       \
  } while (0)

hipError_t fill_f64(hipStream_t s, double* p, long long n, double v) {
  if (n <= 0) return hipSuccess;
  LAUNCH(fill_f64_k, grid1(n), dim3(NT), p, n, v);
}
hipError_t fill_u16(hipStream_t s, u16* p, long long n, u16 v) {
  if (n <= 0) return hipSuccess;
  LAUNCH(fill_u16_k, grid1(n), dim3(NT), p, n, v);
}
hipError_t zero_pads_u16(hipStream_t s, u16* base, int nslice, long long sstride, int rows, int rows_pad, int ld,
                         int cols) {
  if (nslice <= 0 || rows < 0 || rows_pad < rows || cols < 0 || ld < cols || sstride < (long long)rows_pad * ld)
    return hipErrorInvalidValue;
  const long long n = (long long)nslice * ((long long)rows * (ld - cols) + (long long)(rows_pad - rows) * ld);
  if (n == 0) return hipSuccess;
  LAUNCH(zero_pads_u16_k, grid1(n), dim3(NT), base, nslice, sstride, rows, rows_pad, ld, cols);
}
hipError_t coeffs(hipStream_t s, int nact, int npairs, int ncwo, int nsingle, int functional, const double* n,
                  double* alpha, double* beta, float* beta32) {
  LAUNCH(coeffs_k, grid1((long long)nact * nact), dim3(NT), nact, npairs, ncwo, nsingle, functional, n, alpha, beta,
         beta32);
}
hipError_t transpose_ca(hipStream_t s, int nbf, int nact, const double* C, double* Ct, int ldk) {
  LAUNCH(transpose_ca_k, grid1((long long)nbf * nact), dim3(NT), nbf, nact, C, Ct, ldk);
}
hipError_t transpose_ca_f32(hipStream_t s, int nbf, int nact, const double* C, float* Ct, int ldk) {
  LAUNCH(transpose_ca_f32_k, grid1((long long)nbf * nact), dim3(NT), nbf, nact, C, Ct, ldk);
}
hipError_t add_diag_f32(hipStream_t s, int nact, int np, const double* Dc, const OccLayout& oc, double* dbuf, float* W,
                        int ldw) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(d_alpha_k, dim3(np), dim3(NT), 0, s, nact, oc.npairs, oc.ncwo, oc.nsingle, oc.n, Dc, dbuf);
  LAUNCH(add_diag_f32_k, grid1((long long)np * nact), dim3(NT), nact, np, 1, dbuf, W, ldw);
}
hipError_t split_ca(hipStream_t s, int nbf, int nact, int terms, const double* C, u16* hi, u16* lo, u16* h16,
                    u16* l16, int ldk, const uint32_t* bnd) {
  LAUNCH(split_ca_k, grid1((long long)nbf * nact), dim3(NT), nbf, nact, terms, C, hi, lo, h16, l16, ldk, bnd);
}
hipError_t split_b(hipStream_t s, long long n, const double* B, u16* hi, u16* lo, const uint32_t* bnd, int chunk) {
  if (n <= 0) return hipSuccess;
  LAUNCH(split_b_k, grid1(n), dim3(NT), n, B, hi, lo, bnd, chunk);
}
hipError_t scale_bounds(hipStream_t s, int nbf, int nact, const double* C, const double* n, int npairs, int ncwo,
                        int nsingle, int functional, float* col, uint32_t* bnd, int nclear) {
  hipLaunchKernelGGL(col_bounds_k, dim3((unsigned)cdiv(nact, NT / 64)), dim3(NT), 0, s, nbf, nact, C, n, npairs, ncwo,
                     nsingle, functional, col);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  LAUNCH(bounds_reduce_k, dim3(1), dim3(NT), nact, col, bnd, nclear);
}
hipError_t b_bounds(hipStream_t s, const void* B, int is_f64, long long nrows, int ncols, long long ld,
                    long long rows_per_chunk, uint32_t* slot) {
  if (nrows <= 0) return hipSuccess;
  const dim3 g((unsigned)std::min<long long>(cdiv(nrows, NT / 64), 4096));
  const bool vec = !is_f64 && (ld % 8 == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
  if (is_f64) LAUNCH((b_bounds_k<true, false>), g, dim3(NT), B, nrows, ncols, ld, rows_per_chunk, slot);
  if (vec) LAUNCH((b_bounds_k<false, true>), g, dim3(NT), B, nrows, ncols, ld, rows_per_chunk, slot);
  LAUNCH((b_bounds_k<false, false>), g, dim3(NT), B, nrows, ncols, ld, rows_per_chunk, slot);
}
hipError_t hpp_from_hc(hipStream_t s, int nbf, int nact, const double* C, const double* HC, double* Hpp) {
  LAUNCH(hpp_k, dim3(nact), dim3(64), nbf, nact, C, HC, Hpp);
}
hipError_t add_diag_f64(hipStream_t s, int nact, int np, const double* Dc, const OccLayout& oc, double* dbuf,
                        double* W, int ldw) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(d_alpha_k, dim3(np), dim3(NT), 0, s, nact, oc.npairs, oc.ncwo, oc.nsingle, oc.n, Dc, dbuf);
  LAUNCH(add_diag_f64_k, grid1((long long)np * nact), dim3(NT), nact, np, 1, dbuf, W, ldw);
}
hipError_t add_diag_bf16(hipStream_t s, int nact, int np, const double* Dc, const OccLayout& oc, const float* beta32,
                         double* dbuf, u16* Wh, u16* Wl, int ldw, long long pstride, const uint32_t* bnd, int chunk) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(d_alpha_k, dim3(np), dim3(NT), 0, s, nact, oc.npairs, oc.ncwo, oc.nsingle, oc.n, Dc, dbuf);
  LAUNCH(add_diag_bf16_k, grid1((long long)np * nact), dim3(NT), nact, np, 1, dbuf, Dc, beta32, Wh, Wl, ldw, pstride,
         bnd, chunk);
}
hipError_t nofmp2_terms(hipStream_t s, int nact, int npairs, int ncwo, int nsingle, const double* n,
                        const double* Hpp, const double* J, const double* K, double* partials, double* E_hf,
                        double* E_sta) {
  const int nb = 128;   // partials holds 2 * nb doubles
  hipLaunchKernelGGL(nofmp2_stage1_k, dim3(nb), dim3(NT), 0, s, nact, npairs, ncwo, nsingle, n, Hpp, J, K, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  LAUNCH(sum2_partials_k, dim3(1), dim3(NT), nb, partials, E_hf, E_sta);
}
hipError_t offdiag_copy(hipStream_t s, int nbf, const double* src, double* dst) {
  LAUNCH(offdiag_k, grid1((long long)nbf * nbf), dim3(NT), nbf, src, dst);
}
hipError_t reduce_k(hipStream_t s, int nact, int nsplit, const double* Kpart, double* K) {
  LAUNCH(reduce_k_k, grid1((long long)nact * nact), dim3(NT), nact, nsplit, Kpart, K);
}
hipError_t reduce_y_f64(hipStream_t s, long long n, int nsplit, const double* Yp, double* Y) {
  LAUNCH(reduce_y_k<double>, grid1(n), dim3(NT), n, nsplit, Yp, Y);
}
hipError_t reduce_y_f32(hipStream_t s, long long n, int nsplit, const float* Yp, double* Y) {
  LAUNCH(reduce_y_k<float>, grid1(n), dim3(NT), n, nsplit, Yp, Y);
}
hipError_t energy(hipStream_t s, int nbf, int nact, const double* n, const double* Hpp,
                  const double* alpha, const double* beta, const double* J, const double* K,
                  const double* Y2e, const double* C, const u16* cth, const u16* ctl, const float* ct32, int ldk,
                  int corr_terms, double* partials, double* E) {
  const int nb = 256;
  hipLaunchKernelGGL(energy_stage1_k, dim3(nb), dim3(NT), 0, s, nbf, nact, n, Hpp, alpha, beta, J, K, Y2e,
                     C, cth, ctl, ct32, ldk, corr_terms, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  LAUNCH(sum_partials_k, dim3(1), dim3(NT), nb, partials, E);
}
hipError_t assemble_y(hipStream_t s, int nbf, int nact, const double* n, const double* HC, const double* Y2e,
                      double* Y) {
  LAUNCH(assemble_y_k, grid1((long long)nbf * nact), dim3(NT), nbf, nact, n, HC, Y2e, Y);
}
hipError_t grad_c(hipStream_t s, int nbf, int nact, const double* Y, double* G) {
  LAUNCH(grad_c_k, grid1((long long)nbf * nbf), dim3(NT), nbf, nact, Y, G);
}
hipError_t zero_cols(hipStream_t s, int nbf, int col0, double* M) {
  if (col0 >= nbf) return hipSuccess;
  LAUNCH(zero_cols_k, grid1((long long)nbf * (nbf - col0)), dim3(NT), nbf, col0, M);
}
hipError_t max_asym(hipStream_t s, int nbf, const double* lam, double* partials, double* out) {
  const int nb = 256;
  hipLaunchKernelGGL(asym_stage1_k, dim3(nb), dim3(NT), 0, s, nbf, lam, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  LAUNCH(max_partials_k, dim3(1), dim3(NT), nb, partials, out);
}
hipError_t grad_n(hipStream_t s, int nact, int npairs, int ncwo, int nsingle, int functional, const double* n,
                  const double* Hpp, const double* J, const double* K, double* dEdn) {
  LAUNCH(grad_n_k, dim3(nact), dim3(64), nact, npairs, ncwo, nsingle, functional, n, Hpp, J, K, dEdn);
}
hipError_t on_map(hipStream_t s, int kind, int npairs, int ncwo, int nsingle, const double* gamma, double* n,
                  double* jac) {
  LAUNCH(on_map_k, dim3(cdiv(std::max(npairs, nsingle), 64)), dim3(64), kind, npairs, ncwo, nsingle, gamma, n, jac);
}
hipError_t on_map_vjp(hipStream_t s, int kind, int npairs, int ncwo, int nsingle, const double* gamma,
                      const double* dEdn, double* out) {
  LAUNCH(on_map_vjp_k, dim3(cdiv(npairs + nsingle, 64)), dim3(64), kind, npairs, ncwo, nsingle, gamma, dEdn, out);
}
hipError_t build_s(hipStream_t s, int nbf, const double* lam, const double* dprev, double zeta, double* S) {
  LAUNCH(build_s_k, grid1((long long)nbf * nbf), dim3(NT), nbf, lam, dprev, zeta, S);
}
hipError_t sign_fix_cols(hipStream_t s, int nbf, double* U) {
  LAUNCH(sign_fix_k, dim3(nbf), dim3(NT), nbf, U);
}
hipError_t count_nonfinite(hipStream_t s, const void* p, long long n, int is_bf16, int* flag) {
  if (n <= 0) return hipSuccess;
  LAUNCH(nonfinite_k, grid1(n), dim3(NT), p, n, is_bf16, flag);
}
hipError_t eri_jk_ao(hipStream_t s, int nbf, int nact, const double* ERI, const double* C, double* Jr, double* Kr) {
  LAUNCH(eri_jk_ao_k, grid1((long long)nact * nbf * nbf), dim3(NT), nbf, nact, ERI, C, Jr, Kr);
}
hipError_t eri_jk_no(hipStream_t s, int nbf, int nact, const double* C, const double* Jr, const double* Kr,
                     double* J, double* K) {
  LAUNCH(eri_jk_no_k, grid1((long long)nact * nact), dim3(NT), nbf, nact, C, Jr, Kr, J, K);
}
hipError_t eri_y(hipStream_t s, int nbf, int nact, const double* C, const double* /*n*/, const double* /*HC*/,
                 const double* alpha, const double* beta, const double* Jr, const double* Kr, double* Y2e) {
  LAUNCH(eri_y_k, grid1((long long)nbf * nact), dim3(NT), nbf, nact, C, alpha, beta, Jr, Kr, Y2e);
}
hipError_t gather_ao(hipStream_t s, int nbf, int nq, const int32_t* q_idx, const double* src, double* dst) {
  if (nq <= 0) return hipSuccess;
  LAUNCH(gather_ao_k, grid1((long long)nq * nbf * nbf), dim3(NT), nbf, nq, q_idx, src, dst);
}
hipError_t eri_fock_ao(hipStream_t s, int nbf, int nact, int nq, const int32_t* q_idx, const double* n,
                       const double* H, const double* alpha, const double* beta, const double* Jr,
                       const double* Kr, double* Fq) {
  if (nq <= 0) return hipSuccess;
  LAUNCH(eri_fock_ao_k, grid1((long long)nq * nbf * nbf), dim3(NT), nbf, nact, nq, q_idx, n, H, alpha, beta, Jr, Kr, Fq);
}
hipError_t df_ao_accum(hipStream_t s, int nbf, int nact, int np, int nq, const int32_t* q_idx,
                       const void* Bchunk, int b_is_bf16, const double* Dchunk, const double* alpha,
                       const double* beta, const double* XT, const float* XT32, const u16* XT_hi, const u16* XT_lo,
                       int ldx, long long xps, double* Jq, double* Kq, double* Fq, const uint32_t* bnd, int chunk) {
  if (nq <= 0 || np <= 0) return hipSuccess;
  LAUNCH(df_ao_accum_k, grid1((long long)nq * nbf * nbf), dim3(NT), nbf, nact, np, nq, q_idx, Bchunk,
         b_is_bf16, Dchunk, alpha, beta, XT, XT32, XT_hi, XT_lo, ldx, xps, Jq, Kq, Fq, bnd, chunk);
}
hipError_t fock_ao_h(hipStream_t s, int nbf, int nq, const int32_t* q_idx, const double* n, const double* H,
                     double* Fq) {
  if (nq <= 0) return hipSuccess;
  LAUNCH(fock_ao_h_k, grid1((long long)nq * nbf * nbf), dim3(NT), nbf, nq, q_idx, n, H, Fq);
}

}  // namespace pnof

namespace pnof {
namespace {
__global__ void widen_bf16_k(long long n, const u16* __restrict__ src, double* __restrict__ dst) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = (double)bf16_bits_to_f32(src[i]);
}
}  // namespace
hipError_t widen_bf16(hipStream_t s, long long n, const u16* src, double* dst) {
  if (n <= 0) return hipSuccess;
  long long b = (n + 255) / 256;
  if (b > 65535LL * 16) b = 65535LL * 16;
  hipLaunchKernelGGL(widen_bf16_k, dim3((unsigned)b), dim3(256), 0, s, n, src, dst);
  return hipGetLastError();
}
}  // namespace pnof
