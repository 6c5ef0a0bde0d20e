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
  }
  INST_STRIDE(i, nxt) {
    d.xth[i] = 0;
    if (d.xtl) d.xtl[i] = 0;
  }
  INST_STRIDE(i, nw) {
    d.wh[i] = 0;
    if (d.wl) d.wl[i] = 0;
  }
}

// alpha, beta (float64 and float32), C_A^T split into hi/lo.  The K partials need no clearing: the
// grouped b contraction stores (not adds) every lower-triangle position of every split.
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
  INST_STRIDE(i, (long long)nact * nbf) {
    const int p = (int)(i / nbf), mu = (int)(i % nbf);
    u16 h, l;
    split_f64(d.C[(long long)mu * nbf + p], h, l);
    d.cth[(long long)p * d.ldk + mu] = h;
    if (d.terms > 1) d.ctl[(long long)p * d.ldk + mu] = l;
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

// W_P[p][p] = float(b^P_pp beta_pp) + (D alpha)[P][p], split into hi/lo.  D holds the b contraction's
// float accumulators of the diagonal, so the entry is rebuilt and only written: the scattered
// diagonal of W is never read back.
__global__ void add_diag_k(const BInst* __restrict__ tab) {
  const BInst& d = tab[blockIdx.y];
  const long long pstride = (long long)d.nact32 * d.ldw;
  INST_STRIDE(i, (long long)d.naux * d.nact) {
    const long long P = i / d.nact;
    const int p = (int)(i % d.nact);
    const long long o = P * pstride + (long long)p * d.ldw + p;
    const float wv = (float)d.D[i] * d.beta32[(long long)p * d.nact + p];
    u16 h, l;
    split_f64((double)wv + d.dbuf[i], h, l);
    d.wh[o] = h;
    if (d.wl) d.wl[o] = l;
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
