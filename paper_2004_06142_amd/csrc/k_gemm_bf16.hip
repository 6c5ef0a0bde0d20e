// 16-bit matrix-core (v_mfma_f32_16x16x32_bf16 / _f16) contractions with float32 accumulation.
//
// Operands may be carried as a hi + lo pair of 16-bit values; the accumulator then receives
//   terms = 1: hi*hi                              (bf16, one pass)
//   terms = 2: Ahi*Bhi + Alo*Bhi                  (B exact in bf16: X from a bf16 B)
//   terms = 3: Ahi*Bhi + Ahi*Blo + Alo*Bhi        (the lo*lo product is below float32 rounding)
// In the split mode the pairs of the b and Y contractions (and of X when B is float64) are fp16
// pairs of the value times a power of two (11 + 11 significant bits; the scales are fixed per P-chunk
// from bounds, see chunk_scales), multiplied by the fp16 matrix-core instruction; X from a bf16 B
// multiplies the compact bf16 pair of C by B and writes fp16 pairs.
//
// Block tiles BM x BN x 32 (128 x 256 for X, 128 x 128 for the symmetric b, 256 x 128 for Y),
// 256 threads = 4 waves (2 x 2), each wave owning (BM/2) x (BN/2) in 16 x 16 MFMA blocks.  Operand
// k-tiles go global -> registers (one tile ahead) -> LDS (two buffers), one barrier per k-tile.  MFMA lane layout (16x16x32): lane l supplies row l%16 and the eight k
// values 8*(l/16)..+7 of each operand; result element (4*(l/16)+j, l%16) is component j.
//
// Operand storage in global memory:
//   "row" operand: row r (an output index) is contiguous in k  -> LDS [r][k] (16-byte chunks
//     XOR-swizzled within the row), 16-byte reads;
//   "col" operand: row k is contiguous in the output index    -> LDS [k][r], read with the
//     transposing LDS load (ds_read_b64_tr_b16), which within each 16-lane group hands lane i
//     element i%4 of the 8-byte chunks fetched by lanes 4j + i/4 (j = 0..3), i.e. four consecutive
//     k of one row when lane 4j+q fetched rows 4q..4q+3 of k-row j.
// Blocks are numbered so that the eight XCDs each receive one contiguous range of work items:
// items sharing an operand (same P, or same split of P) run on the same XCD and share its L2.
#include <type_traits>

#include "batch_dev.h"
#include "common.h"
#include "f64_tile.h"

namespace pnof {
namespace {

constexpr int BK = 32;
constexpr int RP = BK;              // row-layout LDS pitch (bf16 elements): 64 bytes, chunks swizzled
constexpr int NXCD = 8;
constexpr int T2 = 128;             // tile of the symmetric nact x nact products

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// One 16 x 16 x 32 product; fragments hold raw 16-bit patterns (bf16 or fp16 by F16).
template <bool F16>
__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
  if constexpr (F16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

struct Opnd {
  const u16* hi;
  const u16* lo;
  long long ld;   // elements between consecutive storage rows
  int R;          // valid output-index extent (rows of a row operand, columns of a col operand)
  int K;          // valid k extent
  bool col;       // storage rows run along k (read through the transposing LDS load)
};

__device__ __forceinline__ bool aligned16(const void* p, long long ld) {
  return ((ld & 7) == 0) && ((reinterpret_cast<uintptr_t>(p) & 15) == 0);
}

// 8 consecutive elements src[0..7] of a storage row, zero beyond `valid` elements.
__device__ __forceinline__ u32x4 ld8(const u16* __restrict__ src, int valid, bool vec) {
  if (valid >= 8 && vec) return *reinterpret_cast<const u32x4*>(src);
  uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int i = 0; i < 8; ++i)
    if (i < valid) w[i >> 1] |= ((uint32_t)src[i]) << (16 * (i & 1));
  return u32x4{w[0], w[1], w[2], w[3]};
}

// LDS bank model of gfx950 (measured with the bank-conflict counter): 64 banks of 4 bytes; a 16-byte
// read is served in four 16-lane groups, lane L in group (bit 5, bit 2 ^ bit 3 ^ bit 4) of L, and a
// group is conflict-free when its 16 addresses fall in distinct 16-byte slots of a 256-byte line;
// an 8-byte read is served in two groups of 32 consecutive lanes, each needing distinct 8-byte slots.
// Row layout swizzle: in a fragment read (lane L: row L % 16, chunk L / 16), the four lanes of one
// group that share row % 4 are rows r, r + 12 (chunk g) and r + 4, r + 8 (chunk g ^ 1); flipping
// bit 1 of the chunk on rows with bit 3 set spreads them over four distinct slots.
__device__ __forceinline__ int swz(int r) { return 2 * ((r >> 3) & 1); }

// LDS geometry of one operand slice with D output-index rows.
template <int D>
struct Geo {
  static constexpr int CP = D + 16;                          // col-layout pitch (bf16)
  static constexpr int SLOT = (D * RP > BK * CP) ? D * RP : BK * CP;
  static constexpr int NCH = D * BK / 8 / 256;               // 16-byte chunks per thread
};

// Global -> registers: one BK-deep k-tile of one operand slice (D x BK elements), as raw 16-byte
// chunks plus the number of valid elements of each.  VEC: every storage row starts 16-byte aligned
// and may be read in whole chunks up to the next multiple of 8 past K (or R); the load is issued
// unconditionally from a clamped address, and the invalid elements are cleared only when the chunk
// is written to LDS, so nothing waits on the load before the matrix-core work of the k-tile.
template <int D>
struct Chunks {
  u32x4 v[Geo<D>::NCH];
  int valid[Geo<D>::NCH];
};

template <int D, bool VEC>
__device__ __forceinline__ void fetch(const u16* __restrict__ base, const Opnd& o, int r0, int k0, Chunks<D>& ch) {
  const int t = threadIdx.x;
#pragma unroll
  for (int c = 0; c < Geo<D>::NCH; ++c) {
    const int idx = t + 256 * c;
    int gr, gk, valid;
    long long off;
    if (!o.col) {  // D rows x 4 chunks along k
      gr = r0 + (idx >> 2);
      gk = k0 + (idx & 3) * 8;
      off = (long long)gr * o.ld + gk;
      valid = o.K - gk;
    } else {       // BK k-rows x D/8 chunks along the output index
      gk = k0 + idx / (D / 8);
      gr = r0 + (idx % (D / 8)) * 8;
      off = (long long)gk * o.ld + gr;
      valid = o.R - gr;
    }
    const bool ok = gr < o.R && gk < o.K;
    ch.valid[c] = ok ? (valid < 8 ? valid : 8) : 0;
    if (VEC) ch.v[c] = *reinterpret_cast<const u32x4*>(base + (ok ? off : 0));
    else ch.v[c] = ok ? ld8(base + off, valid, false) : u32x4{0u, 0u, 0u, 0u};
  }
}

__device__ __forceinline__ u32x4 mask8(u32x4 v, int valid) {
  uint32_t w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
    w[i] = (2 * i < valid ? (v[i] & 0xFFFFu) : 0u) | (2 * i + 1 < valid ? (v[i] & 0xFFFF0000u) : 0u);
  return u32x4{w[0], w[1], w[2], w[3]};
}

// Row layout: the four 16-byte chunks of row r are stored permuted, chunk c at c ^ swz(r), so that
// fragment reads (one chunk of 16 consecutive rows per lane group) are free of bank conflicts.
template <int D>
__device__ __forceinline__ void stash(u16* __restrict__ s, bool col, const Chunks<D>& ch) {
  const int t = threadIdx.x;
#pragma unroll
  for (int c = 0; c < Geo<D>::NCH; ++c) {
    const int idx = t + 256 * c;
    u16* dst = !col ? s + (idx >> 2) * RP + (((idx & 3) ^ swz(idx >> 2)) * 8)
                    : s + (idx / (D / 8)) * Geo<D>::CP + (idx % (D / 8)) * 8;
    *reinterpret_cast<u32x4*>(dst) = mask8(ch.v[c], ch.valid[c]);
  }
}

// MFMA operand fragment for the 16 output rows starting at r: lane l gets row r + l%16 and the
// eight k values 8*(l/16)..+7 of the current k-tile.
template <int D>
__device__ __forceinline__ bf16x8 frag(const u16* __restrict__ s, bool col, int r) {
  const int lane = threadIdx.x & 63;
  if (!col) {
    const int rr = r + (lane & 15);
    return *reinterpret_cast<const bf16x8*>(s + rr * RP + (((lane >> 4) ^ swz(rr)) * 8));
  }
  const int g = lane >> 4, L = lane & 15, j = L >> 2, q = L & 3;
  typedef __attribute__((address_space(3))) v4s* lds_v4s;
  const u16* p0 = s + (8 * g + j) * Geo<D>::CP + r + 4 * q;
  const u16* p1 = s + (8 * g + 4 + j) * Geo<D>::CP + r + 4 * q;
  union { v4s h[2]; bf16x8 v; } u;
  u.h[0] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s)(p0));
  u.h[1] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s)(p1));
  return u.v;
}

template <int BM, int BN, bool ALO, bool BLO>
struct Stage {
  u16 a[2][ALO ? 2 : 1][Geo<BM>::SLOT];
  u16 b[2][BLO ? 2 : 1][Geo<BN>::SLOT];
};

template <int MI, int NI>
__device__ __forceinline__ void zero(f32x4 (&acc)[MI][NI]) {
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// Main loop over a sequence of segments (one per P), each a contraction over k in [0, K), for a
// BM x BN block tile; 4 waves in 2 x 2, each owning (BM/2) x (BN/2).  acc is reset at the start of
// each segment when RESET; epi(seg, acc) runs at the end of each.  A(seg, k0) / B(seg, k0) give
// the operand descriptors of a k-tile (the storage order may change from one k-tile to the next).
template <int BM, int BN, bool ALO, bool BLO, bool ACOL, bool BCOL, bool RESET, bool F16, typename FA, typename FB,
          typename EPI>
__device__ __forceinline__ void mainloop(Stage<BM, BN, ALO, BLO>& sm, int nseg, int kb, int ke, int m0, int n0, FA A,
                                         FB B, f32x4 (&acc)[BM / 32][BN / 32], EPI epi) {
  constexpr int MI = BM / 32, NI = BN / 32;
  const int wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
  const int KT = (ke - kb + BK - 1) / BK;
  const int total = nseg * KT;
  if (total <= 0) return;
  Chunks<BM> ra[ALO ? 2 : 1];
  Chunks<BN> rb[BLO ? 2 : 1];
  int lseg = 0, lk = kb;
  auto load = [&]() {
    Opnd a = A(lseg), b = B(lseg);
    a.col = ACOL;
    b.col = BCOL;
    fetch<BM, false>(a.hi, a, m0, lk, ra[0]);
    if (ALO) fetch<BM, false>(a.lo, a, m0, lk, ra[ALO ? 1 : 0]);
    fetch<BN, false>(b.hi, b, n0, lk, rb[0]);
    if (BLO) fetch<BN, false>(b.lo, b, n0, lk, rb[BLO ? 1 : 0]);
    lk += BK;
    if (lk >= ke) { lk = kb; ++lseg; }
  };
  auto store = [&](int buf) {
    stash<BM>(sm.a[buf][0], ACOL, ra[0]);
    if (ALO) stash<BM>(sm.a[buf][ALO ? 1 : 0], ACOL, ra[ALO ? 1 : 0]);
    stash<BN>(sm.b[buf][0], BCOL, rb[0]);
    if (BLO) stash<BN>(sm.b[buf][BLO ? 1 : 0], BCOL, rb[BLO ? 1 : 0]);
  };
  load();
  store(0);
  __syncthreads();
  if (RESET) zero(acc);
  int it = 0;
  for (int seg = 0; seg < nseg; ++seg) {
    for (int kt = 0; kt < KT; ++kt, ++it) {
      const int buf = it & 1;
      const bool more = it + 1 < total;
      if (more) load();
      bf16x8 ah[MI], bh[NI];
#pragma unroll
      for (int i = 0; i < MI; ++i) ah[i] = frag<BM>(sm.a[buf][0], ACOL, wm + 16 * i);
#pragma unroll
      for (int j = 0; j < NI; ++j) bh[j] = frag<BN>(sm.b[buf][0], BCOL, wn + 16 * j);
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
          acc[i][j] = mma<F16>(ah[i], bh[j], acc[i][j]);
      if (BLO) {
        bf16x8 bl[NI];
#pragma unroll
        for (int j = 0; j < NI; ++j) bl[j] = frag<BN>(sm.b[buf][BLO ? 1 : 0], BCOL, wn + 16 * j);
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NI; ++j)
            acc[i][j] = mma<F16>(ah[i], bl[j], acc[i][j]);
      }
      if (ALO) {
#pragma unroll
        for (int i = 0; i < MI; ++i) {
          const bf16x8 al = frag<BM>(sm.a[buf][ALO ? 1 : 0], ACOL, wm + 16 * i);
#pragma unroll
          for (int j = 0; j < NI; ++j)
            acc[i][j] = mma<F16>(al, bh[j], acc[i][j]);
        }
      }
      if (more) store(buf ^ 1);
      __syncthreads();
    }
    epi(seg, acc);
    if (RESET) zero(acc);
  }
}

// ------------------------------------------------------------------------------------------
// Direct-to-LDS pipeline (aligned operands).  Each k-tile slice is fetched by buffer loads that
// write LDS directly (16 bytes per lane, a wave filling one contiguous 1 KB block), S stages deep,
// so S-1 k-tiles are in flight while the matrix cores work on the oldest one; no registers are
// spent on staging.  Loads past the buffer's record limit return zeros.  Requirements: every
// storage row starts 16-byte aligned; rows of the workspace operands are zero-padded to a
// multiple of 32 in k, so the k-tail of the last tile contributes nothing.
// Slice layouts (no padding): row mode element (r, k) at r*BK + ((k/8) ^ swz(r))*8 + k%8;
// col mode element (kr, r) at kr*D + ((r/8) ^ cswz(kr))*8 + r%8.  A transposing fragment read
// serves lanes 0-31 together: k rows kr and kr + 8 land on one bank set unless bit 3 of kr also
// moves the chunk (possible when a row holds at least 16 chunks).
template <int D>
__device__ __forceinline__ int cswz(int kr) {
  return 2 * (kr & 3) ^ (D >= 128 ? 8 * ((kr >> 3) & 1) : 0);
}

constexpr int waitcnt_vm(int n) {
  // gfx9 s_waitcnt immediate: vmcnt[3:0] bits 3:0, vmcnt[5:4] bits 15:14; expcnt and lgkmcnt maxed
  return (n & 0xF) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8);
}

struct Rsrc {
  __amdgpu_buffer_rsrc_t r;
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, long long bytes) {
  const int nrec = bytes > 0x7FFFFFFFLL ? 0x7FFFFFFF : (int)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, nrec, 0x00020000);
}

// Operand of one k-tile for the direct path: slice base, its record limit, storage layout.
struct DOpnd {
  const u16* hi;
  const u16* lo;
  long long ld;
  long long bytes;   // readable bytes from hi (and from lo) onwards
};

template <int D, int NW = 4>
__device__ __forceinline__ void dl_issue(u16* lds_slice, const u16* base, long long bytes, long long ld, const bool col,
                                         int r0, int k0) {
  constexpr int PER_WAVE = D / (16 * NW);   // (D * BK / 8 chunks) / 64 lanes / NW waves
  static_assert(D % (16 * NW) == 0, "slice rows per wave");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(base, bytes);
#pragma unroll
  for (int i = 0; i < PER_WAVE; ++i) {
    const int blk = wave * PER_WAVE + i;
    const int q = blk * 64 + lane;
    long long off;
    if (!col) {
      const int row = q >> 2, c = (q & 3) ^ swz(q >> 2);
      off = (long long)(r0 + row) * ld + k0 + c * 8;
    } else {
      const int kr = q / (D / 8), c = (q % (D / 8)) ^ cswz<D>(q / (D / 8));
      off = (long long)(k0 + kr) * ld + r0 + c * 8;
    }
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)(lds_slice + blk * 512),
                                             16, (unsigned)(off * 2), 0, 0, 0);
  }
}

template <int D, bool COL>
__device__ __forceinline__ bf16x8 dl_frag(const u16* __restrict__ s, int r) {
  const int lane = threadIdx.x & 63;
  if constexpr (!COL) {
    const int rr = r + (lane & 15);
    return *reinterpret_cast<const bf16x8*>(s + rr * BK + (((lane >> 4) ^ swz(rr)) * 8));
  }
  const int g = lane >> 4, L = lane & 15, j = L >> 2, q = L & 3;
  typedef __attribute__((address_space(3))) v4s* lds_v4s;
  const int m = r + 4 * q;
  const int k0 = 8 * g + j, k1 = 8 * g + 4 + j;
  const u16* p0 = s + k0 * D + (((m >> 3) ^ cswz<D>(k0)) << 3) + (m & 7);
  const u16* p1 = s + k1 * D + (((m >> 3) ^ cswz<D>(k1)) << 3) + (m & 7);
  union { v4s h[2]; bf16x8 v; } u;
  u.h[0] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s)(p0));
  u.h[1] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s)(p1));
  return u.v;
}

// Pipeline depth that fits `budget` bytes of LDS (at most 5 stages: up to four k-tiles in flight
// while one is consumed, which is what covers the latency of operands streamed from HBM).
constexpr int ring_depth(int BM, int BN, bool ALO, bool BLO, int budget) {
  const int stage = 2 * BK * (BM * (ALO ? 2 : 1) + BN * (BLO ? 2 : 1));
  const int s = budget / stage;
  return s > 5 ? 5 : s;
}

template <int BM, int BN, bool ALO, bool BLO, int S>
struct Ring {
  u16 a[S][ALO ? 2 : 1][BM * BK];
  u16 b[S][BLO ? 2 : 1][BN * BK];
};

// The ring of a contraction body: the caller's (EXT: e.g. one union shared by the bodies of a
// persistent kernel, ext pointing into LDS) or the body's own static LDS.
template <typename RT, bool EXT>
__device__ __forceinline__ RT& ring_of(void* ext) {
  if constexpr (EXT) {
    return *reinterpret_cast<RT*>(ext);
  } else {
    __shared__ RT sm;
    return sm;
  }
}

// Contraction over segments seg = 0..nseg-1 and k in [kb, ke) of each; ACOL / BCOL fix the storage
// order of the operands at compile time.
// ILV: the k-tile's products run row block by row block (i-major), with the A fragments of block
// i + 1 read while the products of block i issue, in an order pinned by scheduling groups: a wave
// then waits only for its B fragments and first A block after the barrier, instead of for most of
// the k-tile's fragment reads, and the LDS stays busy through the tile.
// BSYM: the B operand is W as gemm2 writes it with wsym (the 128 x 128 blocks on and above the
// diagonal), read per 128-wide part of the tile: block (q-block, k-block) is read row-wise (W[q][k])
// when k-block >= q-block and column-wise (W[k][q], its transpose) otherwise; each part of the stage
// is laid out for its view.
template <int BM, int BN, bool ALO, bool BLO, int S, bool ACOL, bool BCOL, bool RESET, bool F16, int WGM = 2,
          int WGN = 2, bool ILV = false, bool BSYM = false, typename FA, typename FB, typename EPI>
__device__ __forceinline__ void mainloop_dl(Ring<BM, BN, ALO, BLO, S>& sm, int nseg, int kb, int ke, int m0, int n0,
                                            FA A, FB B, f32x4 (&acc)[BM / (16 * WGM)][BN / (16 * WGN)], EPI epi) {
  constexpr int SH = 128;         // BSYM: width of one part of the B tile (the b tile of W)
  static_assert(!BSYM || (BN % SH == 0 && !BCOL && (BN / WGN) <= SH), "BSYM: parts of 128, one per wave");
  constexpr int NW = WGM * WGN;   // waves in a WGM x WGN grid, each owning (BM / WGM) x (BN / WGN)
  constexpr int MI = BM / (16 * WGM), NI = BN / (16 * WGN);
  constexpr int L = (ALO ? 2 : 1) * (BM / (16 * NW)) + (BLO ? 2 : 1) * (BN / (16 * NW));   // loads per wave per tile
  static_assert(L * (S - 2) < 64, "vmcnt range");
  const int wave = threadIdx.x >> 6;
  const int wm = (wave / WGN) * (BM / WGM), wn = (wave % WGN) * (BN / WGN);
  const int KT = (ke - kb + BK - 1) / BK;
  const int total = nseg * KT;
  if (total <= 0) return;
  int lseg = 0, lk = kb;
  auto issue = [&](int stage) {
    const DOpnd a = A(lseg), b = B(lseg);
    dl_issue<BM, NW>(sm.a[stage][0], a.hi, a.bytes, a.ld, ACOL, m0, lk);
    if (ALO) dl_issue<BM, NW>(sm.a[stage][ALO ? 1 : 0], a.lo, a.bytes, a.ld, ACOL, m0, lk);
    if constexpr (BSYM) {
#pragma unroll
      for (int h = 0; h < BN / SH; ++h) {
        const bool col = lk / SH < (n0 + SH * h) / SH;
        dl_issue<SH, NW>(sm.b[stage][0] + h * SH * BK, b.hi, b.bytes, b.ld, col, n0 + SH * h, lk);
        if (BLO) dl_issue<SH, NW>(sm.b[stage][BLO ? 1 : 0] + h * SH * BK, b.lo, b.bytes, b.ld, col, n0 + SH * h, lk);
      }
    } else {
      dl_issue<BN, NW>(sm.b[stage][0], b.hi, b.bytes, b.ld, BCOL, n0, lk);
      if (BLO) dl_issue<BN, NW>(sm.b[stage][BLO ? 1 : 0], b.lo, b.bytes, b.ld, BCOL, n0, lk);
    }
    lk += BK;
    if (lk >= ke) { lk = kb; ++lseg; }
  };
#pragma unroll
  for (int t = 0; t < S - 1; ++t)
    if (t < total) issue(t);
  if (RESET) zero(acc);
  // segments outside, k-tiles inside: the epilogue sits outside the inner loop, so the register
  // allocator keeps the accumulators in place through the k-loop (an epilogue inside the k-loop made
  // it shuttle them between AGPRs and VGPRs on every k-tile)
  // B fragment at wave column c (0 .. BN / WGN) of the stage; bv: the part is read column-wise
  // (BSYM; the wave's columns lie in one part)
  auto bfrag = [&](auto bv, const u16* base, int c) -> bf16x8 {
    if constexpr (BSYM) {
      return dl_frag<SH, decltype(bv)::value>(base + (wn / SH) * SH * BK, wn % SH + c);
    } else {
      return dl_frag<BN, BCOL>(base, wn + c);
    }
  };
  int stage = 0, it = 0;
  // one k-tile's products from stage `stage`; bv as for bfrag (a compile-time view, so that each
  // form is straight-line code with its own read counts in the scheduling groups)
  auto ktile = [&](auto bv) {
    constexpr bool BC = BSYM ? decltype(bv)::value : BCOL;   // B read with transposing reads
    if constexpr (ILV) {
      // reads of one A block: 1 (row layout) or 2 (transposing) instructions per hi / lo part
      constexpr int RA = (ACOL ? 2 : 1) * (ALO ? 2 : 1);
      constexpr int RB = (BC ? 2 : 1) * (BLO ? 2 : 1) * NI;
      constexpr int PR = NI * (1 + (BLO ? 1 : 0) + (ALO ? 1 : 0));   // products per A block
      bf16x8 bh[NI], bl[NI], ah[2], al[2];
#pragma unroll
      for (int j = 0; j < NI; ++j) {
        bh[j] = bfrag(bv, sm.b[stage][0], 16 * j);
        if (BLO) bl[j] = bfrag(bv, sm.b[stage][BLO ? 1 : 0], 16 * j);
      }
      ah[0] = dl_frag<BM, ACOL>(sm.a[stage][0], wm);
      if (ALO) al[0] = dl_frag<BM, ACOL>(sm.a[stage][ALO ? 1 : 0], wm);
      __builtin_amdgcn_sched_group_barrier(0x100, RB + RA, 0);
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const int c = i & 1, n = c ^ 1;
        if (i + 1 < MI) {
          ah[n] = dl_frag<BM, ACOL>(sm.a[stage][0], wm + 16 * (i + 1));
          if (ALO) al[n] = dl_frag<BM, ACOL>(sm.a[stage][ALO ? 1 : 0], wm + 16 * (i + 1));
          __builtin_amdgcn_sched_group_barrier(0x100, RA, 0);
        }
        // products in passes over j, so no two consecutive products share an accumulator
#pragma unroll
        for (int j = 0; j < NI; ++j) acc[i][j] = mma<F16>(ah[c], bh[j], acc[i][j]);
        if (BLO) {
#pragma unroll
          for (int j = 0; j < NI; ++j) acc[i][j] = mma<F16>(ah[c], bl[j], acc[i][j]);
        }
        if (ALO) {
#pragma unroll
          for (int j = 0; j < NI; ++j) acc[i][j] = mma<F16>(al[c], bh[j], acc[i][j]);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, PR, 0);
      }
    } else {
      bf16x8 ah[MI], bh[NI];
#pragma unroll
      for (int i = 0; i < MI; ++i) ah[i] = dl_frag<BM, ACOL>(sm.a[stage][0], wm + 16 * i);
#pragma unroll
      for (int j = 0; j < NI; ++j) bh[j] = bfrag(bv, sm.b[stage][0], 16 * j);
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
          acc[i][j] = mma<F16>(ah[i], bh[j], acc[i][j]);
      if (BLO) {
        bf16x8 bl[NI];
#pragma unroll
        for (int j = 0; j < NI; ++j) bl[j] = bfrag(bv, sm.b[stage][BLO ? 1 : 0], 16 * j);
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NI; ++j)
            acc[i][j] = mma<F16>(ah[i], bl[j], acc[i][j]);
      }
      if (ALO) {
#pragma unroll
        for (int i = 0; i < MI; ++i) {
          const bf16x8 al = dl_frag<BM, ACOL>(sm.a[stage][ALO ? 1 : 0], wm + 16 * i);
#pragma unroll
          for (int j = 0; j < NI; ++j)
            acc[i][j] = mma<F16>(al, bh[j], acc[i][j]);
        }
      }
    }
  };
  for (int seg = 0; seg < nseg; ++seg) {
    for (int kt = 0; kt < KT; ++kt, ++it) {
      if (it + S - 2 < total) __builtin_amdgcn_s_waitcnt(waitcnt_vm(L * (S - 2)));
      else __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
      __builtin_amdgcn_s_barrier();
      if (it + S - 1 < total) issue((stage + S - 1) % S);
      if constexpr (BSYM) {
        // this wave's part is read column-wise when the k-tile's 128-block lies before the part's
        if ((kb + kt * BK) / SH < (n0 + wn) / SH) ktile(std::true_type{});
        else ktile(std::false_type{});
      } else {
        ktile(std::false_type{});
      }
      stage = (stage + 1 == S) ? 0 : stage + 1;
    }
    epi(seg, acc);
    if (RESET) zero(acc);
  }
  __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
  __builtin_amdgcn_s_barrier();
}

// Output row / column of component j of acc[i][jn] relative to the block tile origin.
template <int BM, int WGM = 2, int WGN = 2>
__device__ __forceinline__ int row_of(int i, int j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave / WGN) * (BM / WGM) + i * 16 + 4 * (lane >> 4) + j;
}
template <int BN, int WGM = 2, int WGN = 2>
__device__ __forceinline__ int col_of(int jn) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  return (wave % WGN) * (BN / WGN) + jn * 16 + (lane & 15);
}

// Lower-triangle tile t of a tt x tt tiling, ordered by column (tiles sharing tn are consecutive,
// so the blocks an XCD holds at once read few distinct column panels).
__device__ __forceinline__ void tri_tile(int t, int tt, int& tm, int& tn) {
  int r = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= t) ++r;
  while (r * (r + 1) / 2 > t) --r;
  tn = tt - 1 - r;
  tm = tt - 1 - (t - r * (r + 1) / 2);
}

// Tile t of a tm_n x tn_n grid in groups of G rows: consecutive tiles sweep G rows of one column,
// then the next column, so a run of consecutive tiles covers a compact G x (run / G) patch.
template <int G>
__device__ __forceinline__ void grouped_tile(int t, int tm_n, int tn_n, int& tm, int& tn) {
  const int per_group = G * tn_n;
  const int g = t / per_group, r = t % per_group;
  const int rows = min(G, tm_n - g * G);
  tm = g * G + r % rows;
  tn = r / rows;
}

// Block id -> work item, each XCD taking one contiguous range of items (-1: padding block).
__device__ __forceinline__ int xcd_item(int total) {
  const int per = (total + NXCD - 1) / NXCD;
  const int w = (int)(blockIdx.x % NXCD) * per + (int)(blockIdx.x / NXCD);
  return w < total ? w : -1;
}

// Shapes of the workspace operands (WsDims): Ct is nact32 x ldk, each XT_P is nact32 x ldx and each
// W_P is nact32 x ldw (nact32 = nact rounded up to 32), row-major, zero outside the valid block.

// Instance of a grouped launch that owns work item w: off[i] <= w < off[i+1].
__device__ __forceinline__ int find_instance(const int* __restrict__ off, int ninst, int w) {
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// gemm1: XT_P[p][mu] = sum_nu Ct[p][nu] B_P[mu][nu], written as a hi/lo pair.  Tile G1M (p) x G1N (mu)
// in a WGM x WGN wave grid, one P per work item (items covering several P measured slower: the
// epilogue's stores then stall the next P's operand waits, as the vector-memory counter retires loads
// and stores in order).
// STACK: the n-tiles run over the stacked rows (P, mu) of all np rows of B.
// EXT / ext: the ring is the caller's (see ring_of); BUDGET: LDS bytes for the ring (0: the whole
// unit's LDS shared by MINB blocks).
template <int TERMS, bool BLO, int G1M, int G1N, int WGM, int WGN, int MINB, bool VEC, bool STACK, bool EXT = false,
          int BUDGET = 0>
__device__ __forceinline__ void gemm1_body(int w, const G1Args& g, void* ext = nullptr) {
  constexpr bool ALO = TERMS >= 2;
  constexpr int MI = G1M / (16 * WGM), NI = G1N / (16 * WGN);
  const int nbf = g.nbf, nact = g.nact, ldx = g.ldx;
  const int tm_n = (nact + G1M - 1) / G1M;
  int P = 0, m0, n0;
  if constexpr (STACK) {
    m0 = (w % tm_n) * G1M;
    n0 = (w / tm_n) * G1N;
  } else {
    const int tn_n = (nbf + G1N - 1) / G1N;
    P = w / (tm_n * tn_n);
    const int tile = w % (tm_n * tn_n);
    m0 = (tile / tn_n) * G1M;
    n0 = (tile % tn_n) * G1N;
  }
  const long long pstride = (long long)g.ws.nact32 * ldx;
  u16* XTh = g.xt_hi + (STACK ? 0 : P * pstride);
  u16* XTl = g.xt_lo ? g.xt_lo + (STACK ? 0 : P * pstride) : nullptr;
  const long long nrows = (long long)g.np * nbf;
  // split mode: X is written as the fp16 pair of X sX
  const float xmul = TERMS >= 2 ? chunk_scales(g.bnd, g.chunk, TERMS == 3).xmul : 1.0f;
  f32x4 acc[MI][NI];
  auto epi = [&](int, f32x4(&a)[MI][NI]) {
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int jn = 0; jn < NI; ++jn) {
        long long xo;
        if constexpr (STACK) {
          const int c = n0 + col_of<G1N, WGM, WGN>(jn);
          if (c >= nrows) continue;
          const int Pc = c / nbf;
          xo = Pc * pstride + (c - Pc * nbf);
        } else {
          const int mu = n0 + col_of<G1N, WGM, WGN>(jn);
          if (mu >= nbf) continue;
          xo = mu;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int p = m0 + row_of<G1M, WGM, WGN>(i, j);
          if (p >= nact) continue;
          u16 h, l;
          if (TERMS == 1) { h = f32_to_bf16_bits(a[i][jn][j]); l = 0; }
          else split_f16(a[i][jn][j] * xmul, h, l);
          XTh[(long long)p * ldx + xo] = h;
          if (XTl) XTl[(long long)p * ldx + xo] = l;
        }
      }
  };
  if constexpr (VEC) {
    // the LDS of one compute unit is shared by MINB blocks
    constexpr int S = ring_depth(G1M, G1N, ALO, BLO, BUDGET > 0 ? BUDGET : (MINB == 2 ? 81920 : 163840));
    auto& sm = ring_of<Ring<G1M, G1N, ALO, BLO, S>, EXT>(ext);
    auto A = [&](int) { return DOpnd{g.ct_hi, g.ct_lo, g.ldk, g.ws.ct_bytes}; };
    auto B = [&](int) {
      const long long o = (long long)P * g.bstride;
      return DOpnd{g.b_hi + o, BLO ? g.b_lo + o : nullptr, g.ldb, g.b_bytes - 2 * o};
    };
    mainloop_dl<G1M, G1N, ALO, BLO, S, false, false, true, (TERMS == 3), WGM, WGN, (WGM * WGN == 8)>(sm, 1, 0, nbf, m0, n0,
                                                                                                     A, B, acc,
                                                                                      epi);
  } else {
    static_assert(VEC || (WGM == 2 && WGN == 2), "register-staged path: 2 x 2 waves");
    __shared__ Stage<G1M, G1N, ALO, BLO> sm;
    auto A = [&](int) { return Opnd{g.ct_hi, g.ct_lo, g.ldk, nact, nbf, false}; };
    auto B = [&](int) {
      const long long o = (long long)P * g.bstride;
      return Opnd{g.b_hi + o, BLO ? g.b_lo + o : nullptr, g.ldb, STACK ? (int)nrows : nbf, nbf, false};
    };
    mainloop<G1M, G1N, ALO, BLO, false, false, true, (TERMS == 3)>(sm, 1, 0, nbf, m0, n0, A, B, acc, epi);
  }
}

// gemm2: b_P = Ct XT_P^T on lower-triangle tiles; Kpart[s] += sum_{P in s} b^2 (lower triangle, summed
// over the successive P-chunks of one call), D[P][p] = b_pp, W_P = b o beta as a hi/lo pair.  W is
// written in full (off-diagonal tiles store their mirror image as well), or with wsym only as the
// transposed image of each tile: the 128 x 128 blocks on and above the diagonal, which gemm3 with
// wsym reads.
// waves along q of a gemm2 block (2 x g2_wgn grid)
constexpr int g2_wgn(bool vec) { return vec ? 4 : 2; }

// TT: the square tile (128, or 64 for the short active spaces of batch instances, with 4 waves).
// KSET: store the K sums instead of adding them (a launch that covers every P of the problem).
template <int TERMS, bool VEC, int TT = T2, bool KSET = false, bool EXT = false, int BUDGET = 0>
__device__ __forceinline__ void gemm2_body(int w, const G2Args& g, void* ext = nullptr) {
  constexpr bool LO = TERMS >= 3;
  // the direct-load form of the 128 tile runs 8 waves (2 x 4, each 64 x 32): half the accumulators,
  // beta and K sums per wave, so they stay in registers, and two waves per SIMD hide each other's
  // epilogue latency; the 64 tile runs 4 waves of 32 x 32
  constexpr int WGN = g2_wgn(VEC && TT == 128), NI = TT / (16 * WGN), MI = TT / 32;
  const int nbf = g.nbf, nact = g.nact, np = g.np, nsplit = g.nsplit, ldw = g.ldw, ldx = g.ldx;
  const int tt = (nact + TT - 1) / TT;
  const int ntri = tt * (tt + 1) / 2;
  const int s = w / ntri;
  int tm, tn;
  tri_tile(w % ntri, tt, tm, tn);
  const int m0 = tm * TT, n0 = tn * TT;
  const int pb = (int)((long long)np * s / nsplit), pe = (int)((long long)np * (s + 1) / nsplit);
  // split mode: the accumulator holds b sC sX; W is written as the fp16 pair of W sW
  float invB = 1.0f, wmul = 1.0f;
  if constexpr (LO) {
    const Scales sc = chunk_scales(g.bnd, g.chunk, false);
    invB = sc.invB;
    wmul = sc.wmul;
  }
  // beta (times the W scale) of this lane's accumulator positions, kept in registers for the whole
  // P-range
  f32x4 bet[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int jn = 0; jn < NI; ++jn)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = m0 + row_of<TT, 2, WGN>(i, j), q = n0 + col_of<TT, 2, WGN>(jn);
        bet[i][jn][j] = (p < nact && q < nact) ? g.beta32[(long long)p * nact + q] * wmul : 0.f;
      }
  f32x4 kacc[MI][NI], acc[MI][NI];
  zero(kacc);
  const bool diag = (tm == tn);
  auto epi = [&](int seg, f32x4(&a)[MI][NI]) {
    const int P = pb + seg;
    u16* Wh = g.w_hi + (long long)P * g.ws.nact32 * ldw;
    u16* Wl = LO ? g.w_lo + (long long)P * g.ws.nact32 * ldw : nullptr;
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int jn = 0; jn < NI; ++jn) {
        const int p0 = m0 + row_of<TT, 2, WGN>(i, 0), q = n0 + col_of<TT, 2, WGN>(jn);
        float wv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float b = a[i][jn][j] * invB;
          kacc[i][jn][j] += b * b;
          wv[j] = a[i][jn][j] * bet[i][jn][j];
        }
        uint32_t h01, h23, l01 = 0, l23 = 0;
        if constexpr (LO) {
          split2_f16(wv[0], wv[1], h01, l01);
          split2_f16(wv[2], wv[3], h23, l23);
        } else {
          h01 = cvt2_bf16(wv[0], wv[1]);
          h23 = cvt2_bf16(wv[2], wv[3]);
        }
        if (q < nact && g.wsym) {
          // the transposed image only: W[q][p0 .. p0 + 3] in one 8-byte store (the padding columns
          // past nact receive zeros), covering the blocks on and above the diagonal
          if (p0 < nact) {
            const long long o = (long long)q * ldw + p0;
            *reinterpret_cast<uint2*>(Wh + o) = uint2{h01, h23};
            if (LO) *reinterpret_cast<uint2*>(Wl + o) = uint2{l01, l23};
          }
          if (diag) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (p0 + j == q) g.Dc[(long long)P * nact + q] = (double)(a[i][jn][j] * invB);
          }
        } else if (q < nact) {
          const u16 hv[4] = {(u16)h01, (u16)(h01 >> 16), (u16)h23, (u16)(h23 >> 16)};
          const u16 lv[4] = {(u16)l01, (u16)(l01 >> 16), (u16)l23, (u16)(l23 >> 16)};
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int p = p0 + j;
            if (p < nact) {
              Wh[(long long)p * ldw + q] = hv[j];
              if (LO) Wl[(long long)p * ldw + q] = lv[j];
              if (diag && p == q) g.Dc[(long long)P * nact + p] = (double)(a[i][jn][j] * invB);
            }
          }
          if (!diag && p0 < nact) {
            const long long o = (long long)q * ldw + p0;
            if ((ldw & 3) == 0) {
              *reinterpret_cast<uint2*>(Wh + o) = uint2{h01, h23};
              if (LO) *reinterpret_cast<uint2*>(Wl + o) = uint2{l01, l23};
            } else {
#pragma unroll
              for (int j = 0; j < 4; ++j)
                if (p0 + j < nact) {
                  Wh[o + j] = hv[j];
                  if (LO) Wl[o + j] = lv[j];
                }
            }
          }
        }
      }
  };
  if constexpr (VEC) {
    constexpr int S = ring_depth(TT, TT, LO, LO, BUDGET > 0 ? BUDGET : (TT == 128 ? 163840 : 81920));
    auto& sm = ring_of<Ring<TT, TT, LO, LO, S>, EXT>(ext);
    auto A = [&](int) { return DOpnd{g.ct_hi, g.ct_lo, g.ldk, g.ws.ct_bytes}; };
    auto B = [&](int seg) {
      const long long off = (long long)(pb + seg) * g.ws.nact32 * ldx;
      return DOpnd{g.xt_hi + off, LO ? g.xt_lo + off : nullptr, ldx, g.ws.xt_bytes - 2 * off};
    };
    mainloop_dl<TT, TT, LO, LO, S, false, false, true, LO, 2, WGN>(sm, pe - pb, 0, nbf, m0, n0, A, B, acc, epi);
  } else {
    __shared__ Stage<TT, TT, LO, LO> sm;
    auto A = [&](int) { return Opnd{g.ct_hi, g.ct_lo, g.ldk, nact, nbf, false}; };
    auto B = [&](int seg) {
      const long long off = (long long)(pb + seg) * g.ws.nact32 * ldx;
      return Opnd{g.xt_hi + off, LO ? g.xt_lo + off : nullptr, ldx, nact, nbf, false};
    };
    mainloop<TT, TT, LO, LO, false, false, true, LO>(sm, pe - pb, 0, nbf, m0, n0, A, B, acc, epi);
  }
  double* Kp = g.Kpart + (long long)s * nact * nact;
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int jn = 0; jn < NI; ++jn)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = m0 + row_of<TT, 2, WGN>(i, j), q = n0 + col_of<TT, 2, WGN>(jn);
        if (p < nact && q <= p) {
          if constexpr (KSET) Kp[(long long)p * nact + q] = (double)kacc[i][jn][j];
          else Kp[(long long)p * nact + q] += (double)kacc[i][jn][j];
        }
      }
}

// gemm3: Ypart[s][mu][q] = sum_{P in s} sum_r XT_P[r][mu] W_P[q][r].  XT is read as a col operand,
// W as a row operand (with wsym, each 128-wide block from the orientation gemm2 stored it in: rows
// on and above the diagonal, columns below); every block walks (P, r) in the same order, so blocks of one
// split that share an operand panel read it at about the same time.  Split mode: 3 fp16 products
// (2 products, dropping X_lo W_hi at about 2^-12 relative, left lambda 2.2e-5 from the exact values on
// a 77-function edge shape).
// Tile G3M (mu) x G3N (q), waves in a WGM x WGN grid.  Each wave's share of the tile sets how many
// matrix-core products one byte read from LDS feeds: a 64 x 64 wave reads 16 KB per k-tile for 48
// products, a 128 x 64 wave 24 KB for 96; LDS bandwidth (about 128 bytes per clock per compute unit)
// is what limits the 64 x 64 form.
template <int TERMS, int G3M, int G3N, int WGM, int WGN, int MINB, bool VEC, bool EXT = false, int BUDGET = 0,
          bool WSYM = false>
__device__ __forceinline__ void gemm3_body(int w, const G3Args& g, void* ext = nullptr) {
  constexpr bool LO = TERMS >= 3;
  constexpr int MI = G3M / (16 * WGM), NI = G3N / (16 * WGN);
  const int nbf = g.nbf, nact = g.nact, np = g.np, nsplit = g.nsplit, ldx = g.ldx, ldw = g.ldw;
  const int tm_n = (nbf + G3M - 1) / G3M, tn_n = (nact + G3N - 1) / G3N;
  const int s = w / (tm_n * tn_n);
  int tm, tn;
  grouped_tile<4>(w % (tm_n * tn_n), tm_n, tn_n, tm, tn);
  const int m0 = tm * G3M, n0 = tn * G3N;
  const int pb = (int)((long long)np * s / nsplit), pe = (int)((long long)np * (s + 1) / nsplit);
  f32x4 acc[MI][NI];
  zero(acc);
  auto none = [&](int, f32x4(&)[MI][NI]) {};
  if constexpr (VEC) {
    // the 128 x 128 tile runs two blocks per compute unit (two-stage ring each): while one block
    // waits on its fragment reads or barrier, the other keeps the matrix cores busy
    constexpr int S = ring_depth(G3M, G3N, LO, LO, BUDGET > 0 ? BUDGET : (MINB == 2 ? 81920 : 163840));
    auto& sm = ring_of<Ring<G3M, G3N, LO, LO, S>, EXT>(ext);
    auto A = [&](int seg) {
      const long long off = (long long)(pb + seg) * g.ws.nact32 * ldx;
      return DOpnd{g.xt_hi + off, LO ? g.xt_lo + off : nullptr, ldx, g.ws.xt_bytes - 2 * off};
    };
    auto B = [&](int seg) {
      const long long off = (long long)(pb + seg) * g.ws.nact32 * ldw;
      return DOpnd{g.w_hi + off, LO ? g.w_lo + off : nullptr, ldw, g.ws.w_bytes - 2 * off};
    };
    mainloop_dl<G3M, G3N, LO, LO, S, true, false, false, LO, WGM, WGN, (WGM * WGN == 8), WSYM>(sm, pe - pb, 0, nact,
                                                                                             m0, n0, A, B, acc, none);
  } else {
    static_assert(VEC || (WGM == 2 && WGN == 2), "register-staged path: 2 x 2 waves");
    static_assert(!WSYM, "the symmetric W layout is read on the direct-load path only");
    __shared__ Stage<G3M, G3N, LO, LO> sm;
    auto A = [&](int seg) {
      const long long off = (long long)(pb + seg) * g.ws.nact32 * ldx;
      return Opnd{g.xt_hi + off, LO ? g.xt_lo + off : nullptr, ldx, nbf, nact, true};
    };
    auto B = [&](int seg) {
      const long long off = (long long)(pb + seg) * g.ws.nact32 * ldw;
      return Opnd{g.w_hi + off, LO ? g.w_lo + off : nullptr, ldw, nact, nact, false};
    };
    mainloop<G3M, G3N, LO, LO, true, false, false, LO>(sm, pe - pb, 0, nact, m0, n0, A, B, acc, none);
  }
  float* Y = g.Ypart + (long long)s * nbf * nact;
  const float invY = LO ? chunk_scales(g.bnd, g.chunk, false).invY : 1.0f;   // acc = Y sX sW
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int jn = 0; jn < NI; ++jn)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + row_of<G3M, WGM, WGN>(i, j), n = n0 + col_of<G3N, WGM, WGN>(jn);
        if (m < nbf && n < nact) Y[(long long)m * nact + n] = acc[i][jn][j] * invY;
      }
}

template <int TERMS, bool BLO, int G1M, int G1N, int WGM, int WGN, int MINB, bool VEC>
__global__ __launch_bounds__(64 * WGM * WGN, MINB) void gemm1_kernel(G1Args g) {
  const int w = xcd_item(g1_items(g, G1M, G1N, false));
  if (w < 0) return;
  gemm1_body<TERMS, BLO, G1M, G1N, WGM, WGN, MINB, VEC, false>(w, g);
}
template <int TERMS, bool VEC>
__global__ __launch_bounds__(128 * g2_wgn(VEC), 1) void gemm2_kernel(G2Args g) {
  const int w = xcd_item(g2_items(g, T2));
  if (w < 0) return;
  gemm2_body<TERMS, VEC>(w, g);
}
template <int TERMS, int G3M, int G3N, int WGM, int WGN, int MINB, bool VEC, bool WSYM = false>
__global__ __launch_bounds__(64 * WGM * WGN, MINB) void gemm3_kernel(G3Args g) {
  const int w = xcd_item(g3_items(g, G3M, G3N));
  if (w < 0) return;
  gemm3_body<TERMS, G3M, G3N, WGM, WGN, MINB, VEC, false, 0, WSYM>(w, g);
}

// Grouped forms: one launch over the work items of every instance of a batch.  The tile width along
// the active orbitals is a template parameter (128, or 64 when the instances' active spaces are
// short); the 64-wide forms run 4 waves and two blocks per compute unit.
// (X at two blocks per compute unit, as the single-problem 128 x 128 form: 8.6 -> 7.7 ms per
// 64-instance PES batch)
template <int TERMS, int TM>
__global__ __launch_bounds__(256, 2) void gemm1_grouped(const G1Args* __restrict__ tab, const int* __restrict__ off,
                                                        int ninst, int total) {
  const int w = xcd_item(total);
  if (w < 0) return;
  const int i = find_instance(off, ninst, w);
  const G1Args g = tab[i];
  gemm1_body<TERMS, false, TM, 128, 2, 2, 2, true, true>(w - off[i], g);
}
template <int TERMS, int TT>
__global__ __launch_bounds__(TT == 128 ? 128 * g2_wgn(true) : 256, TT == 128 ? 1 : 2) void gemm2_grouped(
    const G2Args* __restrict__ tab, const int* __restrict__ off, int ninst, int total) {
  const int w = xcd_item(total);
  if (w < 0) return;
  const int i = find_instance(off, ninst, w);
  const G2Args g = tab[i];
  gemm2_body<TERMS, true, TT, true>(w - off[i], g);
}
template <int TERMS, int TN>
__global__ __launch_bounds__(256, 2) void gemm3_grouped(const G3Args* __restrict__ tab, const int* __restrict__ off,
                                                        int ninst, int total) {
  const int w = xcd_item(total);
  if (w < 0) return;
  const int i = find_instance(off, ninst, w);
  const G3Args g = tab[i];
  gemm3_body<TERMS, 128, TN, 2, 2, 2, true>(w - off[i], g);
}

// ------------------------------------------------------------------------------------------
// Persistent batch kernel.  Every block loops: claim a work item of the first instance (in index
// order) whose current phase still has unclaimed items -- every item of the phases before it being
// complete, a claimed item never waits -- run it, publish it.  The block that completes a phase's
// last item moves the instance to the next phase; the instance's last phase stamps its completion
// time.  A block that finds nothing to claim polls; once stall_ticks of the device clock pass with
// no item completed anywhere it raises the stall flag and exits, and the others exit on seeing the
// flag, so every block ends whatever happens.
constexpr int PBUDGET = 79872;   // LDS of the largest ring; with the small arrays, two blocks per unit

template <int TX, int TY>
union PersistLds {
  Ring<TX, 128, true, false, ring_depth(TX, 128, true, false, PBUDGET)> x;
  Ring<64, 64, true, true, ring_depth(64, 64, true, true, PBUDGET)> b;
  Ring<128, TY, true, true, ring_depth(128, TY, true, true, PBUDGET)> y;
  f64t::F64Smem f;
};

__device__ __forceinline__ int ld_dev(const int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ int ld_uni(const int* p) { return __builtin_amdgcn_readfirstlane(ld_dev(p)); }

// The prep item (one block): the call-level scale bounds reduced in LDS (the grouped launches take
// two launches and a global array for them; the words are the same), then alpha, beta and C's split.
__device__ inline void persist_prep(const BInst& d) {
  __shared__ uint32_t m[4];
  if (threadIdx.x < 4) m[threadIdx.x] = 0u;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  for (int q = threadIdx.x >> 6; q < d.nact; q += blockDim.x >> 6) {
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
      atomicMax(&m[0], __float_as_uint((float)s1));
      atomicMax(&m[1], __float_as_uint((float)cm));
      atomicMax(&m[2], __float_as_uint((float)sa));
      atomicMax(&m[3], __float_as_uint((float)bm));
    }
  }
  __syncthreads();
  const uint32_t w0 = m[1], w1 = m[0], w2 = __float_as_uint(__uint_as_float(m[3]) + __uint_as_float(m[2]));
  if (threadIdx.x == 0) {
    d.bnd[0] = w0;
    d.bnd[1] = w1;
    d.bnd[2] = w2;
  }
  // sC exactly as chunk_scales forms it from bnd[0]
  bdev::prep(d, 0, 1, ldexpf(1.0f, 13 - bound_exp(__uint_as_float(w0) * 1.01f)));
}

template <int TX, int TY>
__device__ __forceinline__ void persist_item(const PArgs& a, int i, int ph, int idx, void* lds) {
  const BInst& d = a.inst[i];
  f64t::F64Smem& fs = *reinterpret_cast<f64t::F64Smem*>(lds);
  const int n = a.ninst;
  switch (ph) {
    case PH_PREP:
      persist_prep(d);
      break;
    case PH_X: {
      const G1Args g = a.g1[i];
      const int nt = g1_items(g, TX, 128, true), nx = cdiv(nt, PERSIST_XG);
      if (idx < nx) {
        const int t0 = idx * PERSIST_XG, t1 = t0 + PERSIST_XG < nt ? t0 + PERSIST_XG : nt;
        for (int t = t0; t < t1; ++t) {
          if (t > t0) __syncthreads();   // the ring of the tile before is free again
          gemm1_body<2, false, TX, 128, 2, 2, 2, true, true, true, PBUDGET>(t, g, lds);
        }
      } else {
        f64t::grouped_tile<false, true>(a.f64[i], idx - nx, fs);                           // H C_A
      }
      break;
    }
    case PH_B: {
      const G2Args g = a.g2[i];
      const int nb = g2_items(g, 64);
      if (idx < nb) gemm2_body<3, true, 64, true, true, PBUDGET>(idx, g, lds);
      else bdev::hpp(d, 0, 1);
      break;
    }
    case PH_DJ: {
      const int nd = f64t::grouped_tiles(d.naux, d.nact);
      if (idx < nd) f64t::grouped_tile<false, true>(a.f64[n + i], idx, fs);                // D alpha
      else f64t::grouped_tile<true, true>(a.f64[2 * n + i], idx - nd, fs);                // J = D^T D
      break;
    }
    case PH_DIAG:
      bdev::add_diag(d, idx, PERSIST_PARTS);
      break;
    case PH_Y: {
      const G3Args g = a.g3[i];
      gemm3_body<3, 128, TY, 2, 2, 2, true, true, PBUDGET>(idx, g, lds);
      break;
    }
    case PH_RED:
      bdev::reduce(d, idx, PERSIST_PARTS);
      break;
    case PH_EY:
      if (idx < BATCH_EPARTS) bdev::energy_part(d, idx);
      else bdev::y_assemble(d, idx - BATCH_EPARTS, PERSIST_PARTS);
      break;
    case PH_LAM:
      f64t::grouped_tile<true, true>(a.f64[3 * n + i], idx, fs);                          // lambda = C^T Y
      break;
    case PH_FIN:
      bdev::finish(d, idx, PERSIST_PARTS);
      break;
    default:
      bdev::vjp(d, 0, 1);
      break;
  }
}

// Every instance runs on one die: a block reads the id of the die it runs on from the hardware and
// claims items of that die's group of instances only (group = id modulo the device's die count;
// the first block of a group records its die id, and a block of another die mapping to the same
// group stops the run with the error flag rather than share an L2-resident instance).  All of an instance's intermediate data then stays in
// one L2, so a block makes its item's stores visible by waiting for them to reach L2 (before the
// barrier that ends the item) and sees the other blocks' stores after invalidating its compute
// unit's L1 (after claiming); no L2 write-back or invalidation is needed.  The scheduling words are
// touched with device-scope atomics and coherent loads only.
// The scheduling runs in wavefront 0 as a whole; the other wavefronts wait at the barrier.  Lane l
// of wavefront 0 looks at the die's instance base + l, a ballot picks the first one with unclaimed
// items of its open phase, and lane 0 alone performs the atomics (every value the lanes branch on
// is uniform).  Publishing an item and claiming the next form a single region of wavefront 0 at
// the top of the loop, so that no code path of the loop distinguishes lanes of one wavefront around
// a barrier: were the two separate lane-0 regions on either side of the loop's back edge, the
// compiler may join them into one and leave lanes 1..63 cycling through the barriers without lane 0.
__device__ __forceinline__ int die_id() { return (int)__builtin_amdgcn_s_getreg((3 << 11) | 20); }   // XCC_ID[3:0]
__device__ __forceinline__ void l1_invalidate() { asm volatile("buffer_inv sc0" ::: "memory"); }

template <int TX, int TY>
__global__ __launch_bounds__(256, 2) void batch_persist_k(PArgs a) {
  __shared__ PersistLds<TX, TY> u;
  __shared__ int s_it[3];
  const PSched& sc = a.sc;
  const int die = die_id(), grp = die % sc.ndie;
  if (threadIdx.x == 0) {
    const int prev = atomicCAS(sc.die_of + grp, -1, die);
    s_it[0] = (prev == -1 || prev == die) ? 0 : 1;
    if (s_it[0]) atomicExch(sc.prog + 2, 2);   // two dies in one group: stop every block
  }
  __syncthreads();
  if (s_it[0]) return;
  const int lo = __builtin_amdgcn_readfirstlane(sc.xoff[grp]), hi = __builtin_amdgcn_readfirstlane(sc.xoff[grp + 1]);
  const int lane = threadIdx.x;   // in wavefront 0
  const bool lead = threadIdx.x == 0;
  int last = -1;   // state word (instance * PH_N + phase) of the item this block completed last
  for (;;) {
    if (threadIdx.x < 64) {
      if (last >= 0 && lead) {   // publish it
        const int dn = atomicAdd(sc.done + last, 1) + 1;
        if (dn == sc.cnt[last]) {
          const int i = last / PH_N, ph = last % PH_N;
          if (ph + 1 == PH_N) __hip_atomic_store(sc.t_end + i, wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          atomicExch(sc.phase + i, ph + 1);
          if (ph + 1 == PH_N) atomicAdd(sc.prog + 1, 1);
        }
        atomicAdd(sc.prog, 1);
      }
      int inst = -1, ph = 0, idx = 0;
      int seen = ld_uni(sc.prog);
      unsigned long long t_seen = wall_clock64();
      for (;;) {
        if (ld_uni(sc.prog + 1) >= a.ninst || ld_uni(sc.prog + 2) != 0) break;
        for (int base = lo; base < hi && inst < 0; base += 64) {
          int i = -1, p = PH_N, k = 0, cnt = 0;
          bool open = false;
          if (base + lane < hi) {
            i = sc.order[base + lane];
            p = ld_dev(sc.phase + i);
            if (p < PH_N) {
              k = i * PH_N + p;
              cnt = sc.cnt[k];
              open = ld_dev(sc.claim + k) < cnt;
            }
          }
          unsigned long long m = __ballot(open);
          while (m) {
            const int l = __ffsll((long long)m) - 1;
            const int kk = __builtin_amdgcn_readlane(k, l), cc = __builtin_amdgcn_readlane(cnt, l);
            int c = 0;
            if (lead) c = atomicAdd(sc.claim + kk, 1);
            c = __builtin_amdgcn_readlane(c, 0);
            if (c < cc) {
              inst = __builtin_amdgcn_readlane(i, l);
              ph = __builtin_amdgcn_readlane(p, l);
              idx = c;
              break;
            }
            m &= m - 1;   // that phase ran out meanwhile: the next instance
          }
        }
        if (inst >= 0) break;
        __builtin_amdgcn_s_sleep(8);
        const int now = ld_uni(sc.prog);
        const unsigned long long t = wall_clock64();
        if (now != seen) {
          seen = now;
          t_seen = t;
        } else if (t - t_seen > sc.stall_ticks) {
          if (lead) atomicExch(sc.prog + 2, 1);
          break;
        }
      }
      if (inst >= 0) l1_invalidate();
      if (lead) {
        s_it[0] = inst;
        s_it[1] = ph;
        s_it[2] = idx;
      }
    }
    __syncthreads();
    const int inst = __builtin_amdgcn_readfirstlane(s_it[0]), ph = __builtin_amdgcn_readfirstlane(s_it[1]),
              idx = __builtin_amdgcn_readfirstlane(s_it[2]);
    if (inst < 0) return;
    persist_item<TX, TY>(a, inst, ph, idx, &u);
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));   // this wavefront's stores have reached L2
    __syncthreads();
    last = inst * PH_N + ph;
  }
}

// Clears the scheduling state of a run and stamps its start.
__global__ void persist_reset_k(PSched sc, int nwords_inst, int ninst) {
  for (int i = threadIdx.x; i < nwords_inst; i += blockDim.x) {
    sc.claim[i] = 0;
    sc.done[i] = 0;
  }
  for (int i = threadIdx.x; i < ninst; i += blockDim.x) sc.phase[i] = 0;
  for (int i = threadIdx.x; i < sc.ndie; i += blockDim.x) sc.die_of[i] = -1;
  if (threadIdx.x < 3) sc.prog[threadIdx.x] = 0;
  if (threadIdx.x == 0) *sc.t_start = wall_clock64();
}

inline dim3 xcd_grid(long long items) { return dim3((unsigned)(cdiv(items, NXCD) * NXCD)); }

}  // namespace

inline bool al16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }
template <int TERMS, bool BLO, int G1M, int G1N, int WGM, int WGN, int MINB>
static void launch_g1(hipStream_t s, const G1Args& g) {
  const dim3 grid = xcd_grid(g1_items(g, G1M, G1N, false));
  // direct-to-LDS needs 16-byte aligned rows of the caller's B (nbf % 8 == 0)
  const bool vec = (g.ldb % 8 == 0) && (g.nbf % 8 == 0) && (g.bstride % 8 == 0) && al16(g.b_hi) &&
                   (!g.b_lo || al16(g.b_lo)) && al16(g.ct_hi) && (!g.ct_lo || al16(g.ct_lo)) && (g.ldk % 32 == 0) &&
                   (g.ldx % 32 == 0);
  // operands without aligned rows take the register-staged 128 x 128 form whatever the variant
  if (vec)
    hipLaunchKernelGGL((gemm1_kernel<TERMS, BLO, G1M, G1N, WGM, WGN, MINB, true>), grid, dim3(64 * WGM * WGN), 0, s, g);
  else
    hipLaunchKernelGGL((gemm1_kernel<TERMS, BLO, 128, 128, 2, 2, 2, false>), xcd_grid(g1_items(g, 128, 128, false)),
                       dim3(256), 0, s, g);
}

// variant (resolved by the planner): 1 = 128 x 128 (4 waves of 64 x 64, two blocks per CU),
// 2 = 128 x 256 (4 waves of 64 x 128), 3 = 256 x 256 (8 waves of 128 x 64)
template <int TERMS, bool BLO>
static void launch_g1v(hipStream_t s, const G1Args& g, int variant) {
  switch (variant) {
    case 2: launch_g1<TERMS, BLO, 128, 256, 2, 2, 1>(s, g); break;
    case 3: launch_g1<TERMS, BLO, 256, 256, 2, 4, 1>(s, g); break;
    default: launch_g1<TERMS, BLO, 128, 128, 2, 2, 2>(s, g); break;
  }
}

hipError_t df_bf16_gemm1(hipStream_t s, int nbf, int nact, int np, int terms, SplitPtr Ct, int ldk, SplitPtr Bp,
                         long long bstride, int ldb, long long b_bytes, u16* XT_hi, u16* XT_lo, int ldx, int variant,
                         const WsDims& d, const uint32_t* bnd, int chunk) {
  if (np <= 0) return hipSuccess;
  const G1Args g{nbf, nact, np, Ct.hi, Ct.lo, ldk, Bp.hi, Bp.lo, bstride, ldb, b_bytes, XT_hi, XT_lo, ldx, d, bnd, chunk};
  if (terms == 1) launch_g1v<1, false>(s, g, variant);
  else if (Bp.lo == nullptr) launch_g1v<2, false>(s, g, variant);
  else launch_g1v<3, true>(s, g, variant);
  return hipGetLastError();
}

hipError_t df_bf16_gemm2(hipStream_t s, int nbf, int nact, int np, int nsplit, int terms, SplitPtr Ct, int ldk,
                         SplitPtr XT, int ldx, const float* beta32, double* Kpart, double* Dchunk, u16* W_hi,
                         u16* W_lo, int ldw, const WsDims& d, const uint32_t* bnd, int chunk, bool wsym) {
  if (np <= 0) return hipSuccess;
  const G2Args g{nbf,   nact,  np,     nsplit, Ct.hi, Ct.lo, ldk, XT.hi, XT.lo, ldx, beta32,
                 Kpart, Dchunk, W_hi, W_lo,   ldw,   d,     bnd, chunk, wsym ? 1 : 0};
  const dim3 grid = xcd_grid(g2_items(g, T2));
  const bool vec = (ldk % 32 == 0) && (ldx % 32 == 0) && al16(Ct.hi) && (!Ct.lo || al16(Ct.lo)) && al16(XT.hi) &&
                   (!XT.lo || al16(XT.lo));
  if (terms == 1) {
    if (vec) hipLaunchKernelGGL((gemm2_kernel<1, true>), grid, dim3(128 * g2_wgn(true)), 0, s, g);
    else hipLaunchKernelGGL((gemm2_kernel<1, false>), grid, dim3(128 * g2_wgn(false)), 0, s, g);
  } else {
    if (vec) hipLaunchKernelGGL((gemm2_kernel<3, true>), grid, dim3(128 * g2_wgn(true)), 0, s, g);
    else hipLaunchKernelGGL((gemm2_kernel<3, false>), grid, dim3(128 * g2_wgn(false)), 0, s, g);
  }
  return hipGetLastError();
}

static bool g3_vec(const G3Args& g) {
  return (g.ldx % 32 == 0) && (g.ldw % 32 == 0) && al16(g.xt_hi) && (!g.xt_lo || al16(g.xt_lo)) && al16(g.w_hi) &&
         (!g.w_lo || al16(g.w_lo));
}

template <int TERMS, int G3M, int G3N, int WGM, int WGN, int MINB>
static void launch_g3(hipStream_t s, const G3Args& g) {
  const dim3 grid = xcd_grid(g3_items(g, G3M, G3N));
  const bool vec = g3_vec(g);
  // operands without aligned rows take the register-staged 128 x 128 form whatever the variant
  if (vec && g.wsym)
    hipLaunchKernelGGL((gemm3_kernel<TERMS, G3M, G3N, WGM, WGN, MINB, true, true>), grid, dim3(64 * WGM * WGN), 0, s, g);
  else if (vec)
    hipLaunchKernelGGL((gemm3_kernel<TERMS, G3M, G3N, WGM, WGN, MINB, true>), grid, dim3(64 * WGM * WGN), 0, s, g);
  else
    hipLaunchKernelGGL((gemm3_kernel<TERMS, 128, 128, 2, 2, 2, false>), xcd_grid(g3_items(g, 128, 128)), dim3(256), 0,
                       s, g);
}

hipError_t df_bf16_gemm3(hipStream_t s, int nbf, int nact, int np, int nsplit, int terms, SplitPtr XT, int ldx,
                         SplitPtr W, int ldw, float* Ypart, int variant, const WsDims& d, const uint32_t* bnd,
                         int chunk, bool wsym) {
  if (np <= 0) return hipSuccess;
  const G3Args g{nbf, nact, np, nsplit, XT.hi, XT.lo, ldx, W.hi, W.lo, ldw, Ypart, d, bnd, chunk, wsym ? 1 : 0};
  if (wsym && !g3_vec(g)) return hipErrorInvalidValue;   // the symmetric layout needs the direct-load path
  // variant (resolved by the planner): 1 = 128 x 128 (4 waves of 64 x 64, two blocks per CU),
  // 2 = 256 x 128 (4 waves of 128 x 64), 3 = 256 x 256 (8 waves of 128 x 64)
  if (terms == 1) {
    switch (variant) {
      case 2: launch_g3<1, 256, 128, 2, 2, 1>(s, g); break;
      case 3: launch_g3<1, 256, 256, 2, 4, 1>(s, g); break;
      default: launch_g3<1, 128, 128, 2, 2, 2>(s, g); break;
    }
  } else {
    switch (variant) {
      case 2: launch_g3<3, 256, 128, 2, 2, 1>(s, g); break;
      case 3: launch_g3<3, 256, 256, 2, 4, 1>(s, g); break;
      default: launch_g3<3, 128, 128, 2, 2, 2>(s, g); break;
    }
  }
  return hipGetLastError();
}

hipError_t df_bf16_gemm1_grouped(hipStream_t s, int ninst, int total, int terms, int tile, const G1Args* tab,
                                 const int* off) {
  if (total <= 0) return hipSuccess;
  const dim3 gr = xcd_grid(total);
  if (tile == 64) {
    if (terms == 1) hipLaunchKernelGGL((gemm1_grouped<1, 64>), gr, dim3(256), 0, s, tab, off, ninst, total);
    else hipLaunchKernelGGL((gemm1_grouped<2, 64>), gr, dim3(256), 0, s, tab, off, ninst, total);
  } else {
    if (terms == 1) hipLaunchKernelGGL((gemm1_grouped<1, 128>), gr, dim3(256), 0, s, tab, off, ninst, total);
    else hipLaunchKernelGGL((gemm1_grouped<2, 128>), gr, dim3(256), 0, s, tab, off, ninst, total);
  }
  return hipGetLastError();
}
hipError_t df_bf16_gemm2_grouped(hipStream_t s, int ninst, int total, int terms, int tile, const G2Args* tab,
                                 const int* off) {
  if (total <= 0) return hipSuccess;
  const dim3 gr = xcd_grid(total);
  if (tile == 64) {
    if (terms == 1) hipLaunchKernelGGL((gemm2_grouped<1, 64>), gr, dim3(256), 0, s, tab, off, ninst, total);
    else hipLaunchKernelGGL((gemm2_grouped<3, 64>), gr, dim3(256), 0, s, tab, off, ninst, total);
  } else {
    const dim3 bl(128 * g2_wgn(true));
    if (terms == 1) hipLaunchKernelGGL((gemm2_grouped<1, 128>), gr, bl, 0, s, tab, off, ninst, total);
    else hipLaunchKernelGGL((gemm2_grouped<3, 128>), gr, bl, 0, s, tab, off, ninst, total);
  }
  return hipGetLastError();
}
hipError_t df_bf16_gemm3_grouped(hipStream_t s, int ninst, int total, int terms, int tile, const G3Args* tab,
                                 const int* off) {
  if (total <= 0) return hipSuccess;
  const dim3 gr = xcd_grid(total);
  if (tile == 64) {
    if (terms == 1) hipLaunchKernelGGL((gemm3_grouped<1, 64>), gr, dim3(256), 0, s, tab, off, ninst, total);
    else hipLaunchKernelGGL((gemm3_grouped<3, 64>), gr, dim3(256), 0, s, tab, off, ninst, total);
  } else {
    if (terms == 1) hipLaunchKernelGGL((gemm3_grouped<1, 128>), gr, dim3(256), 0, s, tab, off, ninst, total);
    else hipLaunchKernelGGL((gemm3_grouped<3, 128>), gr, dim3(256), 0, s, tab, off, ninst, total);
  }
  return hipGetLastError();
}

}  // namespace pnof

namespace pnof {

void persist_counts(const BInst& d, const G1Args& g1, const G2Args& g2, const G3Args& g3, int tx, int ty, int* cnt) {
  cnt[PH_PREP] = 1;
  cnt[PH_X] = cdiv(g1_items(g1, tx, 128, true), PERSIST_XG) + f64t::grouped_tiles(d.nbf, d.nact);
  cnt[PH_B] = g2_items(g2, 64) + 1;
  cnt[PH_DJ] = f64t::grouped_tiles(d.naux, d.nact) + f64t::grouped_tiles(d.nact, d.nact);
  cnt[PH_DIAG] = PERSIST_PARTS;
  cnt[PH_Y] = g3_items(g3, 128, ty);
  cnt[PH_RED] = PERSIST_PARTS;
  cnt[PH_EY] = BATCH_EPARTS + PERSIST_PARTS;
  cnt[PH_LAM] = f64t::grouped_tiles(d.nbf, d.nact);
  cnt[PH_FIN] = PERSIST_PARTS;
  cnt[PH_VJP] = 1;
}

hipError_t batch_persist(hipStream_t s, const PArgs& a, int ninst_state_words, int tx, int ty, int blocks) {
  hipLaunchKernelGGL(persist_reset_k, dim3(1), dim3(256), 0, s, a.sc, ninst_state_words, a.ninst);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (tx == 64 && ty == 64) hipLaunchKernelGGL((batch_persist_k<64, 64>), dim3(blocks), dim3(256), 0, s, a);
  else if (tx == 64) hipLaunchKernelGGL((batch_persist_k<64, 128>), dim3(blocks), dim3(256), 0, s, a);
  else if (ty == 64) hipLaunchKernelGGL((batch_persist_k<128, 64>), dim3(blocks), dim3(256), 0, s, a);
  else hipLaunchKernelGGL((batch_persist_k<128, 128>), dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace pnof
