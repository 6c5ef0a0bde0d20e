// Grouped element-wise, reduction and small-matrix kernels of a batch of independent PNOF problems
// (a potential-energy-surface scan): every launch covers all instances, blockIdx.y = instance, so
// one step of the batch is a fixed, short sequence of launches (graph-capturable).  The formulas are
// those of the single-problem kernels (Section 2, Eqs. Eg, Efg; Section 3.2, Eqs. lowdin, lag).
#include "common.h"

namespace pnof {
namespace {

constexpr int NT = 256;

#define INST_STRIDE(i, n) \
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)

inline dim3 grid2(long long per_inst, int ninst, int cap = 2048) {
  long long b = (per_inst + NT - 1) / NT;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return dim3((unsigned)b, (unsigned)ninst);
}

// Packed copy of B (rows padded to ldk with zeros) and zeroed tile workspace (the zero pads are part
// of the contract of the contraction kernels; only valid blocks are written afterwards).
__global__ void pack_k(const BInst* __restrict__ tab) {
  const BInst& d = tab[blockIdx.y];
  const long long nb = (long long)d.naux * d.nbf * d.ldk;
  INST_STRIDE(i, nb) {
    const long long row = i / d.ldk;
    const int k = (int)(i % d.ldk);
    d.Bp[i] = k < d.nbf ? d.B[row * d.nbf + k] : (u16)0;
  }
  const long long nct = (long long)d.nact32 * d.ldk, nxt = (long long)d.naux * d.nact32 * d.ldk,
                  nw = (long long)d.naux * d.nact32 * d.ldw;
  INST_STRIDE(i, nct) {
    d.cth[i] = 0;
    if (d.ctl) d.ctl[i] = 0;
    if (d.ch16) {
      d.ch16[i] = 0;
      d.cl16[i] = 0;
    }
  }
  if (d.bnd && blockIdx.x == 0 && threadIdx.x < SCL_CALL + 2) d.bnd[threadIdx.x] = 0u;
  INST_STRIDE(i, nxt) {
    d.xth[i] = 0;
    if (d.xtl) d.xtl[i] = 0;
  }
  INST_STRIDE(i, nw) {
    d.wh[i] = 0;
    if (d.wl) d.wl[i] = 0;
  }
}

// Row bounds of each instance's packed B (zero pads add nothing): the largest row 1-norm into
// bnd[SCL_CALL] with an integer atomic max on the bits (one wavefront per row).
__global__ void b_bounds_k(const BInst* __restrict__ tab) {
  const BInst& d = tab[blockIdx.y];
  if (!d.bnd) return;
  __shared__ float red[NT / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long long nrows = (long long)d.naux * d.nbf;
  float rmax = 0.f;
  for (long long r = (long long)blockIdx.x * (NT / 64) + w; r < nrows; r += (long long)gridDim.x * (NT / 64)) {
    const u16* row = d.Bp + r * d.ldk;
    float s = 0.f;
    for (int c = 8 * lane; c < d.ldk; c += 512) {
      const uint4 v = *reinterpret_cast<const uint4*>(row + c);
      const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) s += fabsf(__uint_as_float(wd[k] << 16)) + fabsf(__uint_as_float(wd[k] & 0xFFFF0000u));
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    rmax = fmaxf(rmax, __shfl(s, 0, 64));
  }
  if (lane == 0) red[w] = rmax;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < NT / 64; ++k) red[0] = fmaxf(red[0], red[k]);
    if (red[0] > 0.f) atomicMax(d.bnd + SCL_CALL, __float_as_uint(red[0]));
  }
}

// Call-level scale bounds, stage 1: one wavefront per active orbital q of each instance,
// colb[4q..4q+3] = sum_mu |C_mu q|, max_mu |C_mu q|, sum_r |alpha_qr|, max_r |beta_qr|.
__global__ void col_bounds_k(const BInst* __restrict__ tab) {
  const BInst& d = tab[blockIdx.y];
  if (!d.bnd) return;
  const int lane = threadIdx.x & 63;
  const int q = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
  if (q >= d.nact) return;
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

// Stage 2, one block per instance: the call-level words bnd[0..3).
__global__ void bounds_reduce_k(const BInst* __restrict__ tab) {
  const BInst& d = tab[blockIdx.y];
  if (!d.bnd) return;
  __shared__ float red[4][NT / 64];
  float v[4] = {0.f, 0.f, 0.f, 0.f};
  for (int q = threadIdx.x; q < d.nact; q += blockDim.x)
    for (int k = 0; k < 4; ++k) v[k] = fmaxf(v[k], d.colb[4 * q + k]);
  for (int off = 32; off > 0; off >>= 1)
    for (int k = 0; k < 4; ++k) v[k] = fmaxf(v[k], __shfl_down(v[k], off, 64));
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < 4; ++k)
      for (int w = 1; w < NT / 64; ++w) red[k][0] = fmaxf(red[k][0], red[k][w]);
    d.bnd[0] = __float_as_uint(red[1][0]);
    d.bnd[1] = __float_as_uint(red[0][0]);
    d.bnd[2] = __float_as_uint(red[3][0] + red[2][0]);
  }
}

// alpha, beta (float64 and float32), C_A^T as bf16 (terms 1) or, in the split mode, the compact bf16
// pair and the fp16 pair of the same value times sC.  The K partials need no clearing: the grouped b
// contraction stores (not adds) every lower-triangle position of every split.
__global__ void prep_k(const BInst* __restrict__ tab) {
  const BInst& d = tab[blockIdx.y];
  const int nact = d.nact, nbf = d.nbf;
  const long long n2 = (long long)nact * nact;
  INST_STRIDE(i, n2) {
    const int p = (int)(i / nact), q = (int)(i % nact);
    double a, b;
    pnof_coeff(p, q, d.n[p], d.n[q], d.npairs, d.ncwo, d.nsingle, d.functional, a, b);
    d.alpha[i] = a;
    d.beta[i] = b;
    d.beta32[i] = (float)b;
  }
  const float sC = d.terms > 1 ? chunk_scales(d.bnd, 0, false).sC : 1.0f;
  INST_STRIDE(i, (long long)nact * nbf) {
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
__global__ void hpp_k(const BInst* __restrict__ tab) {
  const BInst& d = tab[blockIdx.y];
  const int p = blockIdx.x;
  if (p >= d.nact) return;
  double s = 0.0;
  for (int mu = threadIdx.x; mu < d.nbf; mu += 64) s += d.C[(long long)mu * d.nbf + p] * d.HC[(long long)mu * d.nact + p];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (threadIdx.x == 0) d.Hpp[p] = s;
}

// W_P[p][p] = float(b^P_pp beta_pp) + (D alpha)[P][p], as the fp16 pair of W sW (split mode) or one
// bf16 value.  D holds the b contraction's diagonal, so the entry is rebuilt and only written: the
// scattered diagonal of W is never read back.
__global__ void add_diag_k(const BInst* __restrict__ tab) {
  const BInst& d = tab[blockIdx.y];
  const long long pstride = (long long)d.nact32 * d.ldw;
  const float sW = d.wl ? chunk_scales(d.bnd, 0, false).sW : 1.0f;
  INST_STRIDE(i, (long long)d.naux * d.nact) {
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
__global__ void reduce_k(const BInst* __restrict__ tab) {
  const BInst& d = tab[blockIdx.y];
  const long long ny = (long long)d.nbf * d.nact, n2 = (long long)d.nact * d.nact;
  INST_STRIDE(i, ny) {
    d.Y2e[i] = sum_strided(d.Ypart + i, d.ns3, ny);
  }
  INST_STRIDE(i, n2) {
    const int p = (int)(i / d.nact), q = (int)(i % d.nact);
    if (q > p) continue;
    const double s = sum_strided(d.Kpart + i, d.ns2, n2);
    d.K[i] = s;
    d.K[(long long)q * d.nact + p] = s;
  }
}

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

// Energy of Eq. EPNOF7 with the first-order correction of the split orbitals: blocks
// 0 .. BATCH_EPARTS-1 of each instance each sum one contiguous range of the terms (fixed order) into
// epart; the last launch adds the partials in order.  The other blocks form Y = n o (H C_A) + Y2e.
// Block 0 also clears the asymmetry maximum that the last launch raises.
__global__ void energy_y_k(const BInst* __restrict__ tab) {
  const BInst& d = tab[blockIdx.y];
  const int nbf = d.nbf, nact = d.nact;
  const long long ny = (long long)nbf * nact, n2 = (long long)nact * nact;
  if (blockIdx.x < BATCH_EPARTS) {
    const long long total = nact + n2 + ny, per = (total + BATCH_EPARTS - 1) / BATCH_EPARTS;
    const long long lo = (long long)blockIdx.x * per, hi = lo + per < total ? lo + per : total;
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
      d.epart[blockIdx.x] = s;
      if (blockIdx.x == 0 && d.asym) *d.asym = 0.0;
    }
    return;
  }
  for (long long i = (long long)(blockIdx.x - BATCH_EPARTS) * blockDim.x + threadIdx.x; i < ny;
       i += (long long)(gridDim.x - BATCH_EPARTS) * blockDim.x)
    d.Y[i] = d.n[i % nact] * d.HC[i] + d.Y2e[i];
}

// E = sum of the energy partials in order; lambda columns >= nact zeroed, dE/dC = 4 Y (zero columns
// beyond nact), max |lambda - lambda^T| (every block takes its own maximum and raises the instance's
// with an integer atomic max on the bits, exact for non-negative doubles), dE/dn (one wavefront per
// orbital).
__global__ void finish_k(const BInst* __restrict__ tab) {
  const BInst& d = tab[blockIdx.y];
  const int nbf = d.nbf, nact = d.nact;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double e = 0.0;
    for (int b = 0; b < BATCH_EPARTS; ++b) e += d.epart[b];
    *d.E = e;
  }
  const long long nthreads = (long long)gridDim.x * blockDim.x;
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
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

}  // namespace

#define LAUNCH2(kern, grid, ...)                                  \
  do {                                                            \
    hipLaunchKernelGGL(kern, grid, dim3(NT), 0, s, __VA_ARGS__);  \
    return hipGetLastError();                                     \
  } while (0)

hipError_t batch_pack(hipStream_t s, int ninst, const BInst* tab, const BMax& mx) {
  LAUNCH2(pack_k, grid2(mx.pack, ninst, 8192), tab);
}
hipError_t batch_b_bounds(hipStream_t s, int ninst, const BInst* tab, const BMax& mx) {
  LAUNCH2(b_bounds_k, grid2(mx.rows, ninst, 1024), tab);
}
hipError_t batch_bounds(hipStream_t s, int ninst, const BInst* tab, const BMax& mx) {
  hipLaunchKernelGGL(col_bounds_k, dim3((unsigned)cdiv(mx.nact, NT / 64), (unsigned)ninst), dim3(NT), 0, s, tab);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  LAUNCH2(bounds_reduce_k, dim3(1, (unsigned)ninst), tab);
}
hipError_t batch_prep(hipStream_t s, int ninst, const BInst* tab, const BMax& mx) {
  LAUNCH2(prep_k, grid2(mx.prep, ninst), tab);
}
hipError_t batch_hpp(hipStream_t s, int ninst, const BInst* tab, const BMax& mx) {
  hipLaunchKernelGGL(hpp_k, dim3((unsigned)mx.nact, (unsigned)ninst), dim3(64), 0, s, tab);
  return hipGetLastError();
}
hipError_t batch_add_diag(hipStream_t s, int ninst, const BInst* tab, const BMax& mx) {
  LAUNCH2(add_diag_k, grid2(mx.diag, ninst), tab);
}
hipError_t batch_reduce(hipStream_t s, int ninst, const BInst* tab, const BMax& mx) {
  LAUNCH2(reduce_k, grid2(mx.y > mx.k ? mx.y : mx.k, ninst), tab);
}
hipError_t batch_energy_y(hipStream_t s, int ninst, const BInst* tab, const BMax& mx) {
  dim3 g = grid2(mx.y, ninst);
  g.x += BATCH_EPARTS;
  LAUNCH2(energy_y_k, g, tab);
}
hipError_t batch_finish(hipStream_t s, int ninst, const BInst* tab, const BMax& mx) {
  dim3 g = grid2((long long)mx.nbf * mx.nbf, ninst);
  if (g.x * NT / 64 < (unsigned)mx.nact) g.x = (unsigned)((mx.nact * 64LL + NT - 1) / NT);
  LAUNCH2(finish_k, g, tab);
}

}  // namespace pnof
