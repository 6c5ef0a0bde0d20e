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

__host__ __device__ inline int trd_group_base(int k) { return ((k + 1) / TROWS) & ~7; }

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
  // row group g = irow / TROWS goes to block g - gb, with gb a multiple of 8: workgroups are dealt to
  // the 8 XCDs round-robin, so each row stays on one XCD (and its L2) from step to step
  const int gb = trd_group_base(k);
  const int irow = (gb + (int)blockIdx.x) * TROWS + wv;
  const bool has_row = (irow > k) && (irow < n) && (m >= 2);
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
// those of the tridiagonal matrix.  The reflectors are taken in blocks of QNB:
// Q_b = H_{k0} ... H_{k0+QNB-1} = I - V T V^T with V the block's vectors as columns and T upper
// triangular (the compact WY form of a product of reflectors, Schreiber and Van Loan 1989).  Q is
// built from the identity by applying Q_last, ..., Q_0 in turn, each as three float64 GEMMs on the
// trailing part [k0 + 1, n) x [k0 + 1, n) (columns at or before k0 are still unit columns there, and
// rows at or before k0 are untouched by the block).

// V as explicit columns (zero above the unit entry, zero past the last reflector), and Q = I.
__global__ __launch_bounds__(256) void formq_init_k(int n, int nref, int ncol, const double* __restrict__ Vh,
                                                    double* __restrict__ Vc, double* __restrict__ Q) {
  const long long tot = (long long)n * ncol, i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < tot) {
    const int c = (int)(i / n), r = (int)(i % n);
    Vc[i] = (c < nref && r > c) ? (r == c + 1 ? 1.0 : Vh[(long long)c * n + r]) : 0.0;
  }
  if (i < (long long)n * n) Q[i] = (i / n == i % n) ? 1.0 : 0.0;
}

// T of every block (one workgroup each) from the block's Gram matrix G = V^T V (row-major QNB x QNB).
// Within a run of 32 reflectors, column j follows from the earlier ones: T[j][j] = tau_j,
// T[0:j][j] = -tau_j T[0:j][0:j] G[0:j][j] (one wavefront per run, in parallel).  Adjacent triangles
// then merge as T = [[T1, -T1 G12 T2], [0, T2]] (the product of two compact WY factors), 32 + 32 and
// then 64 + 64; the scratch X = G12 T2 lives in T's empty lower triangle.  Zero past the block's last
// reflector.
__device__ __forceinline__ void formq_merge(double (*T)[QNB + 1], const double* __restrict__ G, int off, int h, int t0,
                                            int nt) {
  // X[i][c] = sum_{l <= c} G[off + i][off + h + l] T[off + h + l][off + h + c], stored at T[off + h + i][off + c]
  for (int e = t0; e < h * h; e += nt) {
    const int i = e / h, c = e % h;
    double a = 0.0;
    for (int l = 0; l <= c; ++l) a += G[(off + i) * QNB + off + h + l] * T[off + h + l][off + h + c];
    T[off + h + i][off + c] = a;
  }
}
__device__ __forceinline__ void formq_merge2(double (*T)[QNB + 1], int off, int h, int t0, int nt) {
  // T[off + i][off + h + c] = -sum_{l >= i} T[off + i][off + l] X[l][c]
  for (int e = t0; e < h * h; e += nt) {
    const int i = e / h, c = e % h;
    double a = 0.0;
    for (int l = i; l < h; ++l) a += T[off + i][off + l] * T[off + h + l][off + c];
    T[off + i][off + h + c] = -a;
  }
}

__global__ __launch_bounds__(TNT) void formq_t_k(int nref, const double* __restrict__ tau, const double* __restrict__ Gall,
                                                 double* __restrict__ Tall) {
  __shared__ double T[QNB][QNB + 1];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int k0 = blockIdx.x * QNB, nb = min(QNB, nref - k0);
  const double* G = Gall + (long long)blockIdx.x * QNB * QNB;
  for (int e = t; e < QNB * QNB; e += TNT) T[e / QNB][e % QNB] = 0.0;
  __syncthreads();
  const int c0 = 32 * wv;
  for (int jj = 0; jj < 32; ++jj) {
    const int j = c0 + jj;
    if (j < nb) {
      if (lane < jj) {
        double a = 0.0;
        for (int l = lane; l < jj; ++l) a += T[c0 + lane][c0 + l] * G[(c0 + l) * QNB + j];
        T[c0 + lane][j] = -tau[k0 + j] * a;
      } else if (lane == jj) {
        T[j][j] = tau[k0 + j];
      }
    }
    __syncthreads();
  }
  // 32 + 32 (two merges at once, half the block each), then 64 + 64
  formq_merge(T, G, (t >> 7) * 64, 32, t & 127, 128);
  __syncthreads();
  formq_merge2(T, (t >> 7) * 64, 32, t & 127, 128);
  __syncthreads();
  for (int e = t; e < 2 * 32 * 32; e += TNT) {   // clear the scratch
    const int q = e >> 10, i = (e >> 5) & 31, c = e & 31;
    T[q * 64 + 32 + i][q * 64 + c] = 0.0;
  }
  __syncthreads();
  formq_merge(T, G, 0, 64, t, TNT);
  __syncthreads();
  formq_merge2(T, 0, 64, t, TNT);
  __syncthreads();
  double* Tb = Tall + (long long)blockIdx.x * QNB * QNB;
  for (int e = t; e < QNB * QNB; e += TNT) {
    const int i = e / QNB, c = e % QNB;
    Tb[e] = c >= i ? T[i][c] : 0.0;
  }
}

// W1 (QNB x mb, ld n) = the sum of the ks split-K slabs (each QNB x mb, dense).
__global__ __launch_bounds__(256) void formq_sum_k(int mb, int n, int ks, const double* __restrict__ part,
                                                   double* __restrict__ W1) {
  const long long tot = (long long)QNB * mb, e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= tot) return;
  double a = 0.0;
  for (int s = 0; s < ks; ++s) a += part[s * tot + e];
  W1[(e / mb) * n + e % mb] = a;
}

}  // namespace

long long form_q_ws_doubles(int n) {
  const long long nb = formq_blocks(n);
  return nb * QNB * n + 2 * nb * QNB * QNB + (2LL + FORMQ_KS) * QNB * n + 64;
}

hipError_t form_q_f64(hipStream_t s, int n, const double* Vh, const double* tau, double* ws, double* Q) {
  if (n < 3 || n > TRIDIAG_MAX_N) return hipErrorInvalidValue;
  const int nref = n - 1, nb = formq_blocks(n), ncol = nb * QNB;
  double* Vc = ws;                                  // n x ncol, column-major
  double* G = Vc + (long long)n * ncol;             // nb x QNB x QNB
  double* T = G + (long long)nb * QNB * QNB;        // nb x QNB x QNB
  double* W1 = T + (long long)nb * QNB * QNB;       // QNB x n, row-major (ld n)
  double* W2 = W1 + (long long)QNB * n;             // QNB x n
  double* part = W2 + (long long)QNB * n;           // FORMQ_KS slabs of QNB x mb
  const long long tot = (long long)n * std::max(ncol, n);
  hipLaunchKernelGGL(formq_init_k, dim3((unsigned)cdiv(tot, 256)), dim3(256), 0, s, n, nref, ncol, Vh, Vc, Q);
  // G_b = V_b^T V_b
  hipError_t e = gemm_f64(s, QNB, QNB, n, nb, 1.0, Vc, n, 1, (long long)QNB * n, Vc, 1, n, (long long)QNB * n, 0.0,
                          G, QNB, 1, (long long)QNB * QNB);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(formq_t_k, dim3(nb), dim3(TNT), 0, s, nref, tau, G, T);
  for (int b = nb - 1; b >= 0; --b) {
    const int k0 = b * QNB, mb = n - k0 - 1;
    const double* Vb = Vc + (long long)k0 * n + k0 + 1;   // V_b(r, i) = Vb[i * n + r], rows k0 + 1 ..
    double* Zb = Q + (long long)(k0 + 1) * n + k0 + 1;    // Z(r, c) = Zb[c * n + r]
    // W1 = V_b^T Z, W2 = T_b W1, Z -= V_b W2
    // the first product has few output tiles (QNB x mb) and a long k: split over k, slabs summed
    const int ks = std::min(FORMQ_KS, std::max(1, mb / 128));
    if ((e = gemm_f64_splitk(s, QNB, mb, mb, ks, Vb, n, 1, Zb, 1, n, part)) != hipSuccess) return e;
    hipLaunchKernelGGL(formq_sum_k, dim3((unsigned)cdiv((long long)QNB * mb, 256)), dim3(256), 0, s, mb, n, ks, part, W1);
    if ((e = gemm_f64(s, QNB, mb, QNB, 1, 1.0, T + (long long)b * QNB * QNB, QNB, 1, 0, W1, n, 1, 0, 0.0, W2, n, 1, 0)) !=
        hipSuccess)
      return e;
    if ((e = gemm_f64(s, mb, mb, QNB, 1, -1.0, Vb, 1, n, 0, W2, n, 1, 0, 1.0, Zb, 1, n, 0)) != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t tridiag_f64(hipStream_t s, int n, double* A, double* Vh, double* p2, double* d, double* e, double* tau) {
  if (n <= 0 || n > TRIDIAG_MAX_N) return hipErrorInvalidValue;
  const size_t shm = 3 * (size_t)n * sizeof(double);
  const int k0 = std::max(0, n - TAILM);   // columns k0 .. n-1: one workgroup, trailing block in LDS
  for (int k = 0; k < k0; ++k) {
    const int blocks = std::max(1, (n - 1) / TROWS - trd_group_base(k) + 1);
    hipLaunchKernelGGL(trd_step_k, dim3(blocks), dim3(TNT), shm, s, n, k, A, Vh, p2 + ((k + 1) & 1) * (long long)n,
                       p2 + (k & 1) * (long long)n, d, e, tau);
  }
  hipLaunchKernelGGL(trd_tail_k, dim3(1), dim3(TAILNT), 0, s, n, k0, A, Vh,
                     p2 + ((k0 + 1) & 1) * (long long)n, d, e, tau);
  return hipGetLastError();
}

}  // namespace pnof
