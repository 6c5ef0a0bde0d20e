// Device bodies of the element-wise, reduction and small-matrix steps of a batch instance (the
// formulas of the single-problem kernels: Section 2, Eqs. Eg, Efg; Section 3.2, Eqs. lowdin, lag;
// Section 3.1 for the ON-map adjoint).  Each body covers the instance with `nparts` cooperating
// blocks of which this is block `part`; the grouped launches of k_batch.hip call them with
// (blockIdx.x, gridDim.x), the persistent batch kernel with the parts of its work items.
#pragma once
#include "common.h"

namespace pnof {
namespace bdev {

constexpr int BT = 256;   // threads per block of every caller

#define BDEV_STRIDE(i, n)                                                                       \
  for (long long i = (long long)part * blockDim.x + threadIdx.x; i < (n); i += (long long)nparts * blockDim.x)

__device__ inline double block_sum(double v) {
  __shared__ double red[BT / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < BT / 64; ++i) s += red[i];
  return s;
}

__device__ inline double block_max(double v) {
  __shared__ double red[BT / 64];
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < BT / 64; ++i) s = fmax(s, red[i]);
  return s;
}

// Call-level scale bounds, stage 1: one wavefront per active orbital q, colb[4q..4q+3] =
// sum_mu |C_mu q|, max_mu |C_mu q|, sum_r |alpha_qr|, max_r |beta_qr|.
__device__ inline void col_bounds(const BInst& d, int part, int nparts) {
  const int lane = threadIdx.x & 63;
  for (int q = part * (blockDim.x >> 6) + (threadIdx.x >> 6); q < d.nact; q += nparts * (blockDim.x >> 6)) {
    double s1 = 0.0, cm = 0.0, sa = 0.0, bm = 0.0;
    for (int mu = lane; mu < d.nbf; mu += 64) {
      const double c = fabs(d.C[(long long)mu * d.nbf + q]);
      s1 += c;
      cm = fmax(cm, c);
    }
    for (int r = lane; r < d.nact; r += 64) {
      double a, b;
      pnof_coeff(q, r, d.n[q], d.n[r], d.npairs, d.ncwo, d.nsingle, d.functional, a, b);
      sa += fabs(a);
      bm = fmax(bm, fabs(b));
    }
    for (int off = 32; off > 0; off >>= 1) {
      s1 += __shfl_down(s1, off, 64);
      sa += __shfl_down(sa, off, 64);
      cm = fmax(cm, __shfl_down(cm, off, 64));
      bm = fmax(bm, __shfl_down(bm, off, 64));
    }
    if (lane == 0) {
      d.colb[4 * q + 0] = (float)s1;
      d.colb[4 * q + 1] = (float)cm;
      d.colb[4 * q + 2] = (float)sa;
      d.colb[4 * q + 3] = (float)bm;
    }
  }
}

// Stage 2 (one block): the call-level words bnd[0..3); returns them to thread 0 as well.
__device__ inline void bounds_reduce(const BInst& d, uint32_t (&out)[3]) {
  __shared__ float red[4][BT / 64];
  float v[4] = {0.f, 0.f, 0.f, 0.f};
  for (int q = threadIdx.x; q < d.nact; q += blockDim.x)
    for (int k = 0; k < 4; ++k) v[k] = fmaxf(v[k], d.colb[4 * q + k]);
  for (int off = 32; off > 0; off >>= 1)
    for (int k = 0; k < 4; ++k) v[k] = fmaxf(v[k], __shfl_down(v[k], off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < 4; ++k)
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) red[k][0] = fmaxf(red[k][0], red[k][w]);
    out[0] = __float_as_uint(red[1][0]);
    out[1] = __float_as_uint(red[0][0]);
    out[2] = __float_as_uint(red[3][0] + red[2][0]);
    d.bnd[0] = out[0];
    d.bnd[1] = out[1];
    d.bnd[2] = out[2];
  }
}

// alpha, beta (float64 and float32), C_A^T as bf16 (terms 1) or the compact bf16 pair and the fp16
// pair of C~ sC (split mode).
__device__ inline void prep(const BInst& d, int part, int nparts, float sC) {
  const int nact = d.nact, nbf = d.nbf;
  const long long n2 = (long long)nact * nact;
  BDEV_STRIDE(i, n2) {
    const int p = (int)(i / nact), q = (int)(i % nact);
    double a, b;
    pnof_coeff(p, q, d.n[p], d.n[q], d.npairs, d.ncwo, d.nsingle, d.functional, a, b);
    d.alpha[i] = a;
    d.beta[i] = b;
    d.beta32[i] = (float)b;
  }
  BDEV_STRIDE(i, (long long)nact * nbf) {
    const int p = (int)(i / nbf), mu = (int)(i % nbf);
    const long long o = (long long)p * d.ldk + mu;
    const double x = d.C[(long long)mu * nbf + p];
    if (d.terms == 1) {
      d.cth[o] = f32_to_bf16_bits((float)x);
      continue;
    }
    u16 h, l;
    split_compact(x, h, l);
    d.cth[o] = h;
    d.ctl[o] = l;
    u16 a, b;
    split_f16((bf16_bits_to_f32(h) + bf16_bits_to_f32(l)) * sC, a, b);
    d.ch16[o] = a;
    d.cl16[o] = b;
  }
}

// Hpp[p] = sum_mu C[mu][p] HC[mu][p]: one wavefront per orbital.
__device__ inline void hpp(const BInst& d, int part, int nparts) {
  const int lane = threadIdx.x & 63;
  for (int p = part * (blockDim.x >> 6) + (threadIdx.x >> 6); p < d.nact; p += nparts * (blockDim.x >> 6)) {
    double s = 0.0;
    for (int mu = lane; mu < d.nbf; mu += 64) s += d.C[(long long)mu * d.nbf + p] * d.HC[(long long)mu * d.nact + p];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) d.Hpp[p] = s;
  }
}

// W_P[p][p] = float(b^P_pp beta_pp) + (D alpha)[P][p], as the fp16 pair of W sW (split mode) or one
// bf16 value.  D holds the b contraction's diagonal, so the entry is rebuilt and only written.
__device__ inline void add_diag(const BInst& d, int part, int nparts) {
  const long long pstride = (long long)d.nact32 * d.ldw;
  const float sW = d.wl ? chunk_scales(d.bnd, 0, false).sW : 1.0f;
  BDEV_STRIDE(i, (long long)d.naux * d.nact) {
    const long long P = i / d.nact;
    const int p = (int)(i % d.nact);
    const long long o = P * pstride + (long long)p * d.ldw + p;
    const float wv = (float)d.D[i] * d.beta32[(long long)p * d.nact + p];
    const double w = (double)wv + d.dbuf[i];
    if (d.wl) {
      u16 h, l;
      split_f16((float)(w * (double)sW), h, l);
      d.wh[o] = h;
      d.wl[o] = l;
    } else {
      d.wh[o] = f32_to_bf16_bits((float)w);
    }
  }
}

// Y2e = sum_s Ypart[s]; K[p][q] = K[q][p] = sum_s Kpart[s][p][q] for q <= p (rows read coalesced).
__device__ inline void reduce(const BInst& d, int part, int nparts) {
  const long long ny = (long long)d.nbf * d.nact, n2 = (long long)d.nact * d.nact;
  BDEV_STRIDE(i, ny) { d.Y2e[i] = sum_strided(d.Ypart + i, d.ns3, ny); }
  BDEV_STRIDE(i, n2) {
    const int p = (int)(i / d.nact), q = (int)(i % d.nact);
    if (q > p) continue;
    const double s = sum_strided(d.Kpart + i, d.ns2, n2);
    d.K[i] = s;
    d.K[(long long)q * d.nact + p] = s;
  }
}

// Energy of Eq. EPNOF7 with the first-order correction of the split orbitals: partial e of
// BATCH_EPARTS, one contiguous range of the terms summed in a fixed order into epart[e].  Partial 0
// also clears the asymmetry maximum that finish raises.
__device__ inline void energy_part(const BInst& d, int e) {
  const int nbf = d.nbf, nact = d.nact;
  const long long ny = (long long)nbf * nact, n2 = (long long)nact * nact;
  const long long total = nact + n2 + ny, per = (total + BATCH_EPARTS - 1) / BATCH_EPARTS;
  const long long lo = (long long)e * per, hi = lo + per < total ? lo + per : total;
  double s = 0.0;
  const long long e0 = lo < nact ? lo : nact, e1 = hi < nact ? hi : nact;
  for (long long i = e0 + threadIdx.x; i < e1; i += blockDim.x) s += 2.0 * d.n[i] * d.Hpp[i];
  const long long j0 = (lo > nact ? lo : nact) - nact, j1 = (hi < nact + n2 ? hi : nact + n2) - nact;
  for (long long k = j0 + threadIdx.x; k < j1; k += blockDim.x) s += d.alpha[k] * d.J[k] + d.beta[k] * d.K[k];
  const long long y0 = (lo > nact + n2 ? lo : nact + n2) - nact - n2, y1 = hi - nact - n2;
  for (long long k = y0 + threadIdx.x; k < y1; k += blockDim.x) {
    const int mu = (int)(k / nact), p = (int)(k % nact);
    double ct = (double)bf16_bits_to_f32(d.cth[(long long)p * d.ldk + mu]);
    if (d.terms > 1) ct += (double)bf16_bits_to_f32(d.ctl[(long long)p * d.ldk + mu]);
    s += 4.0 * d.Y2e[k] * (d.C[(long long)mu * nbf + p] - ct);
  }
  s = block_sum(s);
  if (threadIdx.x == 0) {
    d.epart[e] = s;
    if (e == 0 && d.asym) *d.asym = 0.0;
  }
}

// Y = n o (H C_A) + Y2e.
__device__ inline void y_assemble(const BInst& d, int part, int nparts) {
  const long long ny = (long long)d.nbf * d.nact;
  BDEV_STRIDE(i, ny) { d.Y[i] = d.n[i % d.nact] * d.HC[i] + d.Y2e[i]; }
}

// E = sum of the energy partials in order (part 0); lambda columns >= nact zeroed, dE/dC = 4 Y (zero
// columns beyond nact), max |lambda - lambda^T| (each block raises the instance's maximum with an
// integer atomic max on the bits, exact for non-negative doubles), dE/dn (one wavefront per orbital).
__device__ inline void finish(const BInst& d, int part, int nparts) {
  const int nbf = d.nbf, nact = d.nact;
  if (part == 0 && threadIdx.x == 0) {
    double e = 0.0;
    for (int b = 0; b < BATCH_EPARTS; ++b) e += d.epart[b];
    *d.E = e;
  }
  const long long nthreads = (long long)nparts * blockDim.x;
  const long long t0 = (long long)part * blockDim.x + threadIdx.x;
  double m = 0.0;
  for (long long i = t0; i < (long long)nbf * nbf; i += nthreads) {
    const long long r = i / nbf;
    const int c = (int)(i % nbf);
    if (d.asym) {
      const double a = c < nact ? d.lam[i] : 0.0, b = r < nact ? d.lam[(long long)c * nbf + r] : 0.0;
      m = fmax(m, fabs(a - b));
    }
    if (c >= nact) d.lam[i] = 0.0;
    if (d.dEdC) d.dEdC[i] = c < nact ? 4.0 * d.Y[r * nact + c] : 0.0;
  }
  if (d.asym) {
    m = block_max(m);
    if (threadIdx.x == 0 && m > 0.0)
      atomicMax(reinterpret_cast<unsigned long long*>(d.asym), (unsigned long long)__double_as_longlong(m));
  }
  if (!d.dEdn) return;
  const int lane = threadIdx.x & 63;
  for (long long wv = t0 >> 6; wv < nact; wv += nthreads >> 6) {
    const int p = (int)wv;
    const double np_ = d.n[p];
    const double php = sqrt(np_ * (1.0 - np_));
    double s = 0.0;
    for (int q = lane; q < nact; q += 64) {
      if (q == p) continue;
      s += grad_n_term(p, q, np_, d.n[q], php, d.J[(long long)p * nact + q], d.K[(long long)p * nact + q], d.npairs,
                       d.ncwo, d.nsingle, d.functional);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0)
      d.dEdn[p] = 2.0 * d.Hpp[p] + (is_single(p, d.npairs, d.nsingle) ? 0.0 : d.K[(long long)p * nact + p]) + s;
  }
}

// dE/dgamma = (dn/dgamma)^T dE/dn through the instance's ON map (one thread per subspace).
__device__ inline void vjp(const BInst& d, int part, int nparts) {
  if (!d.gamma || !d.dEdgamma || !d.dEdn) return;
  for (int g = part * blockDim.x + threadIdx.x; g < d.npairs + d.nsingle; g += nparts * blockDim.x)
    on_map_vjp_subspace(d.on_kind, d.npairs, d.ncwo, d.nsingle, d.gamma, d.dEdn, d.dEdgamma, g);
}

#undef BDEV_STRIDE

}  // namespace bdev
}  // namespace pnof
