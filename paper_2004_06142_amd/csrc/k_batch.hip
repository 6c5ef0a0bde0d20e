// Grouped element-wise, reduction and small-matrix kernels of a batch of independent PNOF problems
// (a potential-energy-surface scan): every launch covers all instances, blockIdx.y = instance, so
// one step of the batch is a fixed, short sequence of launches (graph-capturable).  The formulas are
// those of the single-problem kernels (Section 2, Eqs. Eg, Efg; Section 3.2, Eqs. lowdin, lag).
#include "batch_dev.h"
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

// The steps of the batch as grouped launches: blockIdx.y = instance, the blocks of x one instance's
// parts (bodies in batch_dev.h, shared with the persistent batch kernel).
__global__ void col_bounds_k(const BInst* __restrict__ tab) {
  const BInst& d = tab[blockIdx.y];
  if (d.bnd) bdev::col_bounds(d, blockIdx.x, gridDim.x);
}
__global__ void bounds_reduce_k(const BInst* __restrict__ tab) {
  const BInst& d = tab[blockIdx.y];
  uint32_t w[3];
  if (d.bnd) bdev::bounds_reduce(d, w);
}
__global__ void prep_k(const BInst* __restrict__ tab) {
  const BInst& d = tab[blockIdx.y];
  bdev::prep(d, blockIdx.x, gridDim.x, d.terms > 1 ? chunk_scales(d.bnd, 0, false).sC : 1.0f);
}
__global__ void hpp_k(const BInst* __restrict__ tab) { bdev::hpp(tab[blockIdx.y], blockIdx.x, gridDim.x); }
__global__ void add_diag_k(const BInst* __restrict__ tab) { bdev::add_diag(tab[blockIdx.y], blockIdx.x, gridDim.x); }
__global__ void reduce_k(const BInst* __restrict__ tab) { bdev::reduce(tab[blockIdx.y], blockIdx.x, gridDim.x); }
// blocks 0 .. BATCH_EPARTS-1: the energy partials; the others: Y = n o (H C_A) + Y2e
__global__ void energy_y_k(const BInst* __restrict__ tab) {
  const BInst& d = tab[blockIdx.y];
  if (blockIdx.x < BATCH_EPARTS) bdev::energy_part(d, blockIdx.x);
  else bdev::y_assemble(d, blockIdx.x - BATCH_EPARTS, gridDim.x - BATCH_EPARTS);
}
__global__ void finish_k(const BInst* __restrict__ tab) { bdev::finish(tab[blockIdx.y], blockIdx.x, gridDim.x); }
__global__ void vjp_k(const BInst* __restrict__ tab) { bdev::vjp(tab[blockIdx.y], blockIdx.x, gridDim.x); }

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
  LAUNCH2(hpp_k, dim3((unsigned)cdiv(mx.nact, NT / 64), (unsigned)ninst), tab);
}
hipError_t batch_vjp(hipStream_t s, int ninst, const BInst* tab, const BMax& mx) {
  LAUNCH2(vjp_k, dim3(1, (unsigned)ninst), tab);
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
