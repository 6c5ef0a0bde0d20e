// Householder reduction of a symmetric float64 matrix to tridiagonal form, one kernel per column.
//
// The orbital step diagonalises an n x n symmetric matrix every iteration (n = 1200 at the largest
// workload).  The reduction is a chain of n dependent steps, so its cost is per-step latency, not
// bandwidth.  Each step here is a single launch: it applies the previous step's rank-2 update to
// the rows it owns and, in the same pass over each row, accumulates that row's product with the new
// Householder vector.  The update is never a separate kernel, and no step reads the matrix twice.
//
// Step k (0 <= k < n), with v_{k-1}, tau_{k-1} and p_{k-1} = tau_{k-1} A v_{k-1} from step k - 1:
//   w_{k-1} = p_{k-1} - (tau_{k-1} / 2) (p_{k-1} . v_{k-1}) v_{k-1};
//   c = row k of A with the pending update A -= v w^T + w v^T applied (A is symmetric, so row k is
//       column k); d_k = c_k;
//   Householder vector of c_{k+1..n-1}: v_k (v_k[k+1] = 1), tau_k, e_k = beta (LAPACK's dlarfg
//       convention: beta = -sign(alpha) |c_{k+1..}|, tau = (beta - alpha) / beta; tau = 0 when the
//       column below the subdiagonal is already zero);
//   rows i > k: apply the pending update, store, p_k[i] = tau_k (row i . v_k).
// Every block recomputes w_{k-1}, c and v_k identically (same data, same reduction order); block 0
// stores v_k as row k of Vh, which read column-major is the lower-storage reflector layout that
// LAPACK-style routines (ormtr) take: Q = H_0 H_1 ... H_{n-2}, H_k = I - tau_k v_k v_k^T, A = Q T Q^T.
#include "common.h"

namespace pnof {
namespace {

// Sums over the lanes of a wavefront with DPP lane moves, which stay in the vector unit (a shuffle
// goes through the LDS crossbar on every level).  Quad permutes (lane ^ 1, lane ^ 2) and the
// half-row and row mirrors (lane i <-> 7 - i, 15 - i) leave every lane of a row of 16 with the row's
// sum; two row broadcasts (lane 15 into rows 1 and 3, lane 31 into rows 2 and 3) then carry the row
// sums into lane 63, which is read back.  All 64 lanes must be active.
template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xf, false);
  return __hiloint2double(hi, lo);
}
// sum over each group of 8 lanes (lanes 8g .. 8g + 7), in every lane of the group
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_mov<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_mov<0x141>(v);   // row_half_mirror
  return v;
}
// sum over the 64 lanes, returned in every lane
__device__ __forceinline__ double wave_sum(double v) {
  v = group8_sum(v);
  v += dpp_mov<0x140>(v);        // row_mirror
  v += dpp_mov<0x142, 0xa>(v);   // row_bcast:15
  v += dpp_mov<0x143, 0xc>(v);   // row_bcast:31
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

constexpr int TNT = 256;   // threads per block
constexpr int TROWS = 4;   // rows of the trailing matrix per block (one per wavefront)
constexpr int TPQ = 4;     // prologue elements per thread held in registers (loops cover the rest)
constexpr int TPRE = 24;   // row elements per lane loaded before the prologue (loops cover the rest)

__device__ double tblock_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < TNT / 64; ++i) s += red[i];
  return s;
}

__global__ __launch_bounds__(TNT) void trd_step_k(int n, int k, double* __restrict__ A, double* __restrict__ Vh,
                                                  const double* __restrict__ pprev, double* __restrict__ pcur,
                                                  double* __restrict__ d, double* __restrict__ e,
                                                  double* __restrict__ tau) {
  extern __shared__ double sh[];
  const int m = n - k;          // active indices k .. n-1, stored from 0
  double* vp = sh;              // v_{k-1}
  double* wp = sh + m;          // p_{k-1}, then w_{k-1}
  double* vk = sh + 2 * m;      // c, then v_k
  __shared__ double red[TNT / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  // this wavefront's row: its first TPRE * 64 elements are loaded before the prologue, so their
  // latency overlaps the prologue's
  const int irow = k + 1 + blockIdx.x * TROWS + wv;
  const bool has_row = (irow < n) && (m >= 2);
  double* __restrict__ row = A + (long long)(has_row ? irow : k) * n + k;
  double a[TPRE];
#pragma unroll
  for (int c = 0; c < TPRE; ++c) {
    const int jl = 1 + lane + 64 * c;
    a[c] = (has_row && jl < m) ? row[jl] : 0.0;
  }
  // prologue: v_{k-1}, p_{k-1} and row k loaded together
  const double* vprev = Vh + (long long)(k > 0 ? k - 1 : 0) * n + k;
  const double* pp = pprev + k;
  const double* rowk = A + (long long)k * n + k;
  double rv[TPQ], rp[TPQ], rc[TPQ];
#pragma unroll
  for (int q = 0; q < TPQ; ++q) {
    const int i = t + TNT * q;
    const bool ok = i < m;
    rv[q] = (ok && k > 0) ? vprev[i] : 0.0;
    rp[q] = (ok && k > 0) ? pp[i] : 0.0;
    rc[q] = ok ? rowk[i] : 0.0;
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < TPQ; ++q) {
    const int i = t + TNT * q;
    if (i < m) {
      vp[i] = rv[q];
      s += rv[q] * rp[q];
    }
  }
  for (int i = t + TNT * TPQ; i < m; i += TNT) {
    const double v = k > 0 ? vprev[i] : 0.0, p = k > 0 ? pp[i] : 0.0;
    vp[i] = v;
    wp[i] = p;
    s += v * p;
  }
  s = tblock_sum(s, red);   // its syncs also publish vp and wp
  const double half = k > 0 ? 0.5 * tau[k - 1] * s : 0.0;
  const double v0 = vp[0], w0 = (k > 0 ? pp[0] : 0.0) - half * v0;
  double sig = 0.0;
#pragma unroll
  for (int q = 0; q < TPQ; ++q) {
    const int i = t + TNT * q;
    if (i < m) {
      const double w = rp[q] - half * rv[q];
      wp[i] = w;
      const double c = rc[q] - v0 * w - w0 * rv[q];
      rc[q] = c;
      vk[i] = c;
      if (i >= 2) sig += c * c;
    }
  }
  for (int i = t + TNT * TPQ; i < m; i += TNT) {
    const double w = wp[i] - half * vp[i];
    wp[i] = w;
    const double c = rowk[i] - v0 * w - w0 * vp[i];
    vk[i] = c;
    if (i >= 2) sig += c * c;
  }
  sig = tblock_sum(sig, red);   // also publishes wp and vk
  double tk = 0.0, beta = 0.0, scal = 0.0;
  if (m >= 2) {
    const double alpha = vk[1];
    if (sig == 0.0) {
      beta = alpha;
    } else {
      beta = -copysign(sqrt(alpha * alpha + sig), alpha);
      tk = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
  }
  const double dk = vk[0];
  __syncthreads();   // every thread has read vk[0] and vk[1]
#pragma unroll
  for (int q = 0; q < TPQ; ++q) {
    const int i = t + TNT * q;
    if (i < m) vk[i] = (i == 0) ? 0.0 : (i == 1 ? 1.0 : rc[q] * scal);
  }
  for (int i = t + TNT * TPQ; i < m; i += TNT) vk[i] = (i == 0) ? 0.0 : (i == 1 ? 1.0 : vk[i] * scal);
  __syncthreads();
  if (blockIdx.x == 0) {
    double* vrow = Vh + (long long)k * n + k;
    for (int i = t; i < m; i += TNT) vrow[i] = vk[i];
    if (t == 0) {
      d[k] = dk;
      if (m >= 2) {
        e[k] = beta;
        tau[k] = tk;
      }
    }
  }
  if (!has_row) return;
  const int il = irow - k;
  const double vpi = vp[il], wpi = wp[il];
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < TPRE; ++c) {
    const int jl = 1 + lane + 64 * c;
    if (jl < m) {
      const double x = a[c] - vpi * wp[jl] - wpi * vp[jl];
      row[jl] = x;
      acc += x * vk[jl];
    }
  }
  constexpr int CH = 8;
  for (int j0 = 1 + 64 * TPRE; j0 < m; j0 += 64 * CH) {
    double b[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int jl = j0 + lane + 64 * c;
      b[c] = jl < m ? row[jl] : 0.0;
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int jl = j0 + lane + 64 * c;
      if (jl < m) {
        const double x = b[c] - vpi * wp[jl] - wpi * vp[jl];
        row[jl] = x;
        acc += x * vk[jl];
      }
    }
  }
  acc = wave_sum(acc);
  if (lane == 0) pcur[irow] = tk * acc;
}

// ---------------------------------------------------------------- the last columns
// Once n - k <= TAILM the trailing block fits in one workgroup's LDS: a single launch of TAILNT
// threads finishes the reduction there (same Householder convention, the rank-2 update applied
// eagerly), with block barriers in place of one launch per column.
constexpr int TAILM = 128;
constexpr int TAILNT = 1024;

__device__ double tail_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < TAILNT / 64; ++i) s += red[i];
  return s;
}

__global__ __launch_bounds__(TAILNT) void trd_tail_k(int n, int k0, const double* __restrict__ A,
                                                     double* __restrict__ Vh, const double* __restrict__ pprev,
                                                     double* __restrict__ d, double* __restrict__ e,
                                                     double* __restrict__ tau) {
  constexpr int LD = TAILM + 1;
  __shared__ double As[TAILM * LD];
  __shared__ double vs[TAILM], ps[TAILM], ws[TAILM];
  static_assert(TAILNT / 8 >= TAILM, "one group of 8 lanes per row");
  __shared__ double red[TAILNT / 64];
  const int t = threadIdx.x, m0 = n - k0;
  for (int q = t; q < m0 * m0; q += TAILNT) {
    const int i = q / m0, j = q % m0;
    As[i * LD + j] = A[(long long)(k0 + i) * n + k0 + j];
  }
  if (k0 > 0) {
    // the update pending from column k0 - 1: w = p - (tau/2)(p.v) v, A -= v w^T + w v^T
    for (int i = t; i < m0; i += TAILNT) {
      vs[i] = Vh[(long long)(k0 - 1) * n + k0 + i];
      ps[i] = pprev[k0 + i];
    }
    __syncthreads();
    double s = 0.0;
    for (int i = t; i < m0; i += TAILNT) s += vs[i] * ps[i];
    s = tail_sum(s, red);
    const double half = 0.5 * tau[k0 - 1] * s;
    for (int i = t; i < m0; i += TAILNT) ws[i] = ps[i] - half * vs[i];
    __syncthreads();
    for (int q = t; q < m0 * m0; q += TAILNT) {
      const int i = q / m0, j = q % m0;
      As[i * LD + j] = As[i * LD + j] - vs[i] * ws[j] - ws[i] * vs[j];
    }
  }
  __syncthreads();
  // rows of the trailing block go to groups of 8 lanes (TAILNT / 8 = TAILM groups): row i = 1 + grp,
  // columns 1 + sub + 8u
  const int grp = t >> 3, sub = t & 7;
  for (int k = k0; k < n; ++k) {
    const int l = k - k0, m = n - k;
    const double* __restrict__ col = As + l * LD + l;   // row l from the diagonal on (= column l)
    // every wavefront forms |c_{2..}|^2 itself from LDS (no barrier)
    double sig = 0.0;
    for (int i = 2 + (t & 63); i < m; i += 64) sig += col[i] * col[i];
    sig = wave_sum(sig);
    const double dk = col[0], alpha = m >= 2 ? col[1] : 0.0;
    double tk = 0.0, beta = alpha, scal = 0.0;
    if (m >= 2 && sig != 0.0) {
      beta = -copysign(sqrt(alpha * alpha + sig), alpha);
      tk = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    for (int i = t; i < m; i += TAILNT) vs[i] = i == 0 ? 0.0 : (i == 1 ? 1.0 : col[i] * scal);
    if (t == 0) {
      d[k] = dk;
      if (m >= 2) {
        e[k] = beta;
        tau[k] = tk;
      }
    }
    __syncthreads();
    for (int i = t; i < m; i += TAILNT) Vh[(long long)k * n + k + i] = vs[i];
    // p_i = tau (A v)_i for the rows i >= 1 below k: 8 lanes per row, 3 shuffle levels
    const int i = 1 + grp;
    const bool has_row = i < m;
    const double* __restrict__ row = As + (l + (has_row ? i : 0)) * LD + l;
    double a = 0.0;
    if (has_row)
      for (int j = 1 + sub; j < m; j += 8) a += row[j] * vs[j];
    a = group8_sum(a);
    const double pi = tk * a, vi = has_row ? vs[i] : 0.0;
    if (sub == 0) ps[i - 1] = has_row ? pi * vi : 0.0;
    __syncthreads();
    // p . v, formed by every wavefront from the staged products (same order in each)
    double s2 = 0.0;
    for (int r = t & 63; r < TAILM; r += 64) s2 += ps[r];
    s2 = wave_sum(s2);
    const double half = 0.5 * tk * s2, wi = pi - half * vi;
    if (has_row && sub == 0) ws[i] = wi;
    __syncthreads();
    if (has_row) {
      double* __restrict__ ar = As + (l + i) * LD + l;
      for (int j = 1 + sub; j < m; j += 8) ar[j] = ar[j] - vi * ws[j] - wi * vs[j];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- back-transformation
// Q = H_0 ... H_{n-2} formed explicitly (column-major n x n); the eigenvectors are then Q times
// those of the tridiagonal matrix.  The reflectors are taken in blocks of ONB:
// Q_b = H_{k0} ... H_{k0+nb-1} = I - V T V^T with V the block's vectors as columns and T upper
// triangular (the compact WY form of a product of reflectors, Schreiber and Van Loan 1989).
// Columns are independent, so each workgroup owns OCW of them in LDS and applies Q_last, ..., Q_0
// to the identity in turn; no step waits on another workgroup.
constexpr int ONB = ORMTR_NB;                 // reflectors per block
constexpr int OCW = 8;                        // eigenvector columns per workgroup
constexpr int ORPT = TRIDIAG_MAX_N / TNT;     // rows per thread in the update

// T of every block (one workgroup each): G[i][j] = v_i . v_j (i < j), then T[j][j] = tau_j and
// T[0:j][j] = -tau_j T[0:j][0:j] G[0:j][j], stored full ONB x ONB with zeros outside the block.
__global__ __launch_bounds__(TNT) void larft_k(int n, int nref, const double* __restrict__ Vh,
                                               const double* __restrict__ tau, double* __restrict__ Tall) {
  __shared__ double Vs[64][ONB + 1];
  __shared__ double G[ONB][ONB + 1];
  __shared__ double T[ONB][ONB + 1];
  const int t = threadIdx.x, k0 = blockIdx.x * ONB, nb = min(ONB, nref - k0);
  constexpr int NQ = ONB * ONB / TNT;
  double g[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) g[q] = 0.0;
  for (int r0 = k0 + 1; r0 < n; r0 += 64) {
    __syncthreads();
    for (int e = t; e < 64 * ONB; e += TNT) {
      const int j = e / 64, rr = e % 64, r = r0 + rr, k = k0 + j;
      Vs[rr][j] = (j < nb && r < n && r > k) ? (r == k + 1 ? 1.0 : Vh[(long long)k * n + r]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int e = t + TNT * q, i = e / ONB, j = e % ONB;
      if (i < j) {
        double a = g[q];
        for (int rr = 0; rr < 64; ++rr) a += Vs[rr][i] * Vs[rr][j];
        g[q] = a;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = t + TNT * q;
    G[e / ONB][e % ONB] = g[q];
    T[e / ONB][e % ONB] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const double tj = tau[k0 + j];
    if (t < j) {
      double a = 0.0;
      for (int l = t; l < j; ++l) a += T[t][l] * G[l][j];
      T[t][j] = -tj * a;
    } else if (t == j) {
      T[j][j] = tj;
    }
    __syncthreads();
  }
  for (int e = t; e < ONB * ONB; e += TNT) Tall[(long long)blockIdx.x * ONB * ONB + e] = T[e / ONB][e % ONB];
}

// Q = Q I on OCW columns per workgroup (Z starts as the identity panel): for each block b, last to
// first, W1 = V^T Z (threads (j, g) sum rows r = g mod 8, then the 8 partials are added in order),
// W2 = T W1, Z -= V W2.  Column c of the identity is left alone by every reflector k >= c (its
// vector is zero on rows <= k), so a panel starts at the first block that reaches its columns.
// Loads of V are issued in batches (16 per thread in W1, 32 in the update) so that their latency
// is paid once per batch.
__global__ __launch_bounds__(TNT) void ormtr_k(int n, int nref, const double* __restrict__ Vh,
                                               const double* __restrict__ Tall, double* __restrict__ Z) {
  __shared__ double Zs[TRIDIAG_MAX_N * OCW];
  __shared__ double Wp[8][ONB][OCW];
  __shared__ double W1[ONB][OCW];
  __shared__ double W2[ONB][OCW];
  __shared__ double Ts[ONB][ONB];
  const int t = threadIdx.x, c0 = blockIdx.x * OCW;
  for (int e = t; e < n * OCW; e += TNT) {
    const int c = e / n, r = e % n;
    Zs[r * OCW + c] = (c0 + c < n && r == c0 + c) ? 1.0 : 0.0;
  }
  const int nblk = (nref + ONB - 1) / ONB;
  const int bstart = min(nblk - 1, max(0, c0 + OCW - 2) / ONB);
  constexpr int U1 = 16, JG = 4;
  for (int b = bstart; b >= 0; --b) {
    const int k0 = b * ONB, nb = min(ONB, nref - k0);
    for (int e = t; e < ONB * ONB; e += TNT) Ts[e / ONB][e % ONB] = Tall[(long long)b * ONB * ONB + e];
    __syncthreads();   // Zs (panel load or previous block's update) and Ts visible
    {
      const int j = t >> 3, g = t & 7, k = k0 + j;
      double acc[OCW];
#pragma unroll
      for (int c = 0; c < OCW; ++c) acc[c] = 0.0;
      if (j < nb) {
        const double* __restrict__ v = Vh + (long long)k * n;
        for (int r0 = k + 1 + g; r0 < n; r0 += 8 * U1) {
          double vv[U1];
#pragma unroll
          for (int u = 0; u < U1; ++u) {
            const int r = r0 + 8 * u;
            vv[u] = r < n ? (r == k + 1 ? 1.0 : v[r]) : 0.0;
          }
#pragma unroll
          for (int u = 0; u < U1; ++u) {
            const int r = r0 + 8 * u;
            if (r < n) {
#pragma unroll
              for (int c = 0; c < OCW; ++c) acc[c] += vv[u] * Zs[r * OCW + c];
            }
          }
        }
      }
#pragma unroll
      for (int c = 0; c < OCW; ++c) Wp[g][j][c] = acc[c];
    }
    __syncthreads();
    {
      const int j = t >> 3, c = t & 7;
      double a = 0.0;
#pragma unroll
      for (int g = 0; g < 8; ++g) a += Wp[g][j][c];
      W1[j][c] = a;
    }
    __syncthreads();
    {
      const int i = t >> 3, c = t & 7;
      double a = 0.0;
      for (int l = i; l < nb; ++l) a += Ts[i][l] * W1[l][c];
      W2[i][c] = a;   // zero for i >= nb
    }
    __syncthreads();
    double z[ORPT][OCW];
#pragma unroll
    for (int q = 0; q < ORPT; ++q) {
      const int r = k0 + 1 + t + TNT * q;
#pragma unroll
      for (int c = 0; c < OCW; ++c) z[q][c] = r < n ? Zs[r * OCW + c] : 0.0;
    }
    for (int j0 = 0; j0 < nb; j0 += JG) {
      double vv[JG][ORPT];
#pragma unroll
      for (int jj = 0; jj < JG; ++jj) {
        const int k = k0 + j0 + jj;
#pragma unroll
        for (int q = 0; q < ORPT; ++q) {
          const int r = k0 + 1 + t + TNT * q;
          vv[jj][q] = (j0 + jj < nb && r > k && r < n) ? (r == k + 1 ? 1.0 : Vh[(long long)k * n + r]) : 0.0;
        }
      }
#pragma unroll
      for (int jj = 0; jj < JG; ++jj) {
        double w[OCW];
#pragma unroll
        for (int c = 0; c < OCW; ++c) w[c] = W2[min(j0 + jj, ONB - 1)][c];
#pragma unroll
        for (int q = 0; q < ORPT; ++q)
#pragma unroll
          for (int c = 0; c < OCW; ++c) z[q][c] -= vv[jj][q] * w[c];
      }
    }
#pragma unroll
    for (int q = 0; q < ORPT; ++q) {
      const int r = k0 + 1 + t + TNT * q;
      if (r < n) {
#pragma unroll
        for (int c = 0; c < OCW; ++c) Zs[r * OCW + c] = z[q][c];
      }
    }
    __syncthreads();   // Wp, W1, W2 and Ts are rewritten by the next block
  }
  __syncthreads();
  for (int e = t; e < n * OCW; e += TNT) {
    const int c = e / n, r = e % n;
    if (c0 + c < n) Z[(long long)(c0 + c) * n + r] = Zs[r * OCW + c];
  }
}

}  // namespace

hipError_t form_q_f64(hipStream_t s, int n, const double* Vh, const double* tau, double* Tall, double* Q) {
  if (n < 3 || n > TRIDIAG_MAX_N) return hipErrorInvalidValue;
  const int nref = n - 1, nblk = cdiv(nref, ONB);
  hipLaunchKernelGGL(larft_k, dim3(nblk), dim3(TNT), 0, s, n, nref, Vh, tau, Tall);
  hipLaunchKernelGGL(ormtr_k, dim3(cdiv(n, OCW)), dim3(TNT), 0, s, n, nref, Vh, Tall, Q);
  return hipGetLastError();
}

hipError_t tridiag_f64(hipStream_t s, int n, double* A, double* Vh, double* p2, double* d, double* e, double* tau) {
  if (n <= 0 || n > TRIDIAG_MAX_N) return hipErrorInvalidValue;
  const size_t shm = 3 * (size_t)n * sizeof(double);
  const int k0 = std::max(0, n - TAILM);   // columns k0 .. n-1: one workgroup, trailing block in LDS
  for (int k = 0; k < k0; ++k) {
    const int blocks = std::max(1, cdiv(n - k - 1, TROWS));
    hipLaunchKernelGGL(trd_step_k, dim3(blocks), dim3(TNT), shm, s, n, k, A, Vh, p2 + ((k + 1) & 1) * (long long)n,
                       p2 + (k & 1) * (long long)n, d, e, tau);
  }
  hipLaunchKernelGGL(trd_tail_k, dim3(1), dim3(TAILNT), 0, s, n, k0, A, Vh,
                     p2 + ((k0 + 1) & 1) * (long long)n, d, e, tau);
  return hipGetLastError();
}

}  // namespace pnof
