// Eigenvalues and eigenvectors of a symmetric tridiagonal matrix by divide and conquer (Cuppen's
// splitting, with the secular equation solved per root and the eigenvectors of each rank-one
// update formed from recomputed weights after Gu and Eisenstat, which keeps them orthogonal to
// working precision however close the roots lie).  This is the middle step of the orbital step's
// diagonalisation (Sections 3.2 and 3.4): the Householder reduction hands over the diagonal d and
// off-diagonal e, and the eigenvectors Z returned here are rotated back by Q.
//
// The matrix (scaled by its largest entry) is cut recursively in halves down to leaves of at most
// DC_LEAF rows.  Segment j at depth t covers rows [floor(j n / 2^t), floor((j + 1) n / 2^t)), so the
// whole tree is implied by n and every kernel finds its segment by arithmetic.  At each cut the
// coupling b = e[cut - 1] is taken out as a rank-one term: both adjacent diagonal entries lose |b|,
// and the parent is blockdiag(T1, T2) + |b| v v^T with v = e_last(T1) + sign(b) e_first(T2).
//
// Leaves: one wavefront each, cyclic Jacobi (round-robin pairs, the matrix in LDS).
// Merge of two children with eigen-decompositions T1 = Q1 D1 Q1^T, T2 = Q2 D2 Q2^T, per level, for
// all parents of the level at once (kernels in launch order):
//   deflate  z = [last row of Q1, sign(b) first row of Q2] / sqrt 2, rho = 2 |b|; the children's
//            eigenvalues merged into one ascending list; entries with rho |z_j| <= tol leave as they
//            are, and a neighbour pair whose rotation zeroing one z entry perturbs the matrix by
//            less than tol is rotated (the rotated entry leaves); tol = 8 eps max(|d|, |z|).  The
//            rotations form chains (each continues with the surviving entry), replayed later on
//            the eigenvector columns.  The k survivors keep strictly increasing d.  Only the
//            rotations are sequential: the z test, and the rotation test of every neighbour pair
//            on the values before any rotation, run in parallel; a chain is walked serially from
//            each pair that passes (a pair after a chain's end sees unrotated values again).
//   secular  root i of 1/rho + sum_j z_j^2 / (d_j - x) = 0 in (d_i, d_i+1) (the last one in
//            (d_k-1, d_k-1 + rho |z|^2]), one wavefront per root, stored as an offset tau from
//            the nearer pole so that every d_j - x is formed without cancellation.  Iteration:
//            the function's two nearest poles modelled exactly and the rest by a constant fitted
//            to value and slope (the "middle way" of R.-C. Li's secular-equation solvers), kept
//            inside a bisection bracket, with a bisection step every 16th iteration.
//   rank     every eigenvalue of the parent (roots and deflated entries) gets its place in the
//            ascending output.
//   zhat     the weights recomputed from the roots: zhat_j^2 = prod_r (x_r - d_j) /
//            (rho prod_{r != j} (d_r - d_j)), sign of z_j.
//   vec      eigenvector i of diag(d) + rho zhat zhat^T: u_j = zhat_j / (d_j - x_i), normalised.
//   gather   columns of blockdiag(Q1, Q2) that no rotation touches: deflated ones straight to their
//            output place, survivors into a compact matrix ordered [first child only | both |
//            second child only] (the middle group holds columns mixed by rotations).
//   chain    rotation chains replayed row by row on the affected columns.
//   gemm     the survivors' eigenvectors: first child's rows = compact[rows of T1, first two
//            groups] U[first two groups, :], second child's rows likewise with the last two groups,
//            so the zero blocks of blockdiag(Q1, Q2) are never multiplied.
// Launches per level: deflate | secular | rank + zhat | vec + gather + chain | gemm.  Eigenvalues and
// vectors ping-pong between the caller's (w, Z) and a workspace pair by level parity, so that the
// last merge writes the caller's arrays.
#include "common.h"
#include "f64_tile.h"

namespace pnof {
namespace {

constexpr int DC_LEAF = 16;                 // rows of a leaf at most (Jacobi in one wavefront)
constexpr int DC_LP = DC_LEAF + 1;          // leaf LDS row pitch
constexpr int DMAX = TRIDIAG_MAX_N;
constexpr int SQ = DMAX / 64;               // entries per lane of a wavefront over one parent
constexpr double UEPS = 1.1102230246251565e-16;   // unit roundoff 2^-53

struct DcPar {      // one parent of the current level, written by the deflation kernel
  int k;           // survivors (roots of the secular equation)
  int n1, n12, n3; // survivors touching only the first child's rows, both, only the second
  int ndef;        // deflated entries (m - k)
  int nchain;      // rotation chains
  double rho;      // 2 |b|
};

struct DcWs {
  int n, T;
  double* dS;        // scaled diagonal with the cuts' corrections
  double* es;        // scaled off-diagonal
  double* scale;     // the matrix was divided by scale[0]
  double* dbuf[2];   // eigenvalues; [0] is the caller's array
  double* zbuf[2];   // eigenvectors (n x n, column-major); [0] is the caller's
  double* Qc;        // compact surviving columns of the current merge (n x n)
  double* Mm;        // eigenvectors of the rank-one updates (n x n)
  double *dl, *zl, *zh, *tau, *val, *rc, *rs;   // per parent at the parent's first row
  int *orig, *rank, *qpos, *dest, *inch, *cm, *chs, *chl;
  DcPar* par;
  int* info;
};

__device__ __forceinline__ int seg_lo(int n, int t, int j) { return (int)(((long long)j * n) >> t); }
__device__ __forceinline__ int parent_of(int n, int t, int p) {
  int j = (int)(((long long)p << t) / n);
  while (seg_lo(n, t, j + 1) <= p) ++j;
  return j;
}

// Butterfly sums over the 64 lanes: every lane ends with the same bits (each step adds the same
// two values in either order).
__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}
__device__ __forceinline__ double wprod(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v *= __shfl_xor(v, m, 64);
  return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
  return v;
}

// Scale by the largest entry, and take each cut's coupling out of the two diagonal entries beside it.
__global__ __launch_bounds__(1024) void dc_prep_k(DcWs w, const double* __restrict__ d, const double* __restrict__ e) {
  const int n = w.n, T = w.T, tid = threadIdx.x;
  __shared__ double red[16];
  double mx = 0.0;
  for (int i = tid; i < n; i += 1024) {
    mx = fmax(mx, fabs(d[i]));
    if (i + 1 < n) mx = fmax(mx, fabs(e[i]));
  }
  mx = wmax(mx);
  if ((tid & 63) == 0) red[tid >> 6] = mx;
  __syncthreads();
  if (tid < 64) {
    double v = tid < 16 ? red[tid] : 0.0;
    v = wmax(v);
    if (tid == 0) red[0] = v > 0.0 ? v : 1.0;
  }
  __syncthreads();
  const double sc = red[0], inv = 1.0 / sc;
  if (tid == 0) {
    w.scale[0] = sc;
    w.info[0] = 0;
  }
  const int nl = 1 << T;
  for (int i = tid; i < n; i += 1024) {
    const int j = parent_of(n, T, i);
    double v = d[i] * inv;
    if (i == seg_lo(n, T, j) && j > 0) v -= fabs(e[i - 1] * inv);
    if (i == seg_lo(n, T, j + 1) - 1 && j + 1 < nl) v -= fabs(e[i] * inv);
    w.dS[i] = v;
    w.es[i] = i + 1 < n ? e[i] * inv : 0.0;
  }
}

// One leaf per wavefront: cyclic Jacobi with round-robin pairs (every round rotates m/2 disjoint
// pairs at once), until a sweep rotates nothing.  A pair is left alone when its off-diagonal entry
// is below eps sqrt(|a_pp a_qq|) or 1e-3 eps of the leaf's largest entry.  Odd sizes add a zero
// row and column whose pair never rotates.
__global__ __launch_bounds__(64) void dc_leaf_k(DcWs w) {
  const int n = w.n, T = w.T, tid = threadIdx.x;
  const int o = seg_lo(n, T, blockIdx.x), m = seg_lo(n, T, blockIdx.x + 1) - o;
  const int mp = m + (m & 1), np = mp / 2;
  __shared__ double A[DC_LEAF][DC_LP], V[DC_LEAF][DC_LP];
  __shared__ double pc[DC_LEAF / 2], ps[DC_LEAF / 2], pt[DC_LEAF / 2];
  __shared__ int pp[DC_LEAF / 2], pq[DC_LEAF / 2], prot[DC_LEAF / 2];
  __shared__ int any;
  double mx = 0.0;
  for (int x = tid; x < mp * mp; x += 64) {
    const int r = x / mp, c = x % mp;
    double a = 0.0;
    if (r < m && c < m) {
      if (r == c) a = w.dS[o + r];
      else if (c == r + 1) a = w.es[o + r];
      else if (r == c + 1) a = w.es[o + c];
    }
    A[r][c] = a;
    V[r][c] = r == c ? 1.0 : 0.0;
    mx = fmax(mx, fabs(a));
  }
  const double athr = 1e-3 * UEPS * wmax(mx);
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) any = 0;
    __syncthreads();
    for (int r = 0; r < mp - 1; ++r) {
      if (tid < np) {
        int p, q;
        if (tid == 0) { p = r; q = mp - 1; }
        else { p = (r + tid) % (mp - 1); q = (r - tid + mp - 1) % (mp - 1); }
        if (p > q) { const int x = p; p = q; q = x; }
        double c = 1.0, sn = 0.0, tt = 0.0;
        int rot = 0;
        if (q < m) {
          const double apq = A[p][q], app = A[p][p], aqq = A[q][q];
          if (fabs(apq) > athr && fabs(apq) > UEPS * sqrt(fabs(app * aqq))) {
            const double th = (aqq - app) / (2.0 * apq);
            tt = fabs(th) > 1e150 ? 0.5 / th : copysign(1.0, th) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + tt * tt);
            sn = tt * c;
            rot = 1;
          }
        }
        pp[tid] = p; pq[tid] = q; pc[tid] = c; ps[tid] = sn; pt[tid] = tt; prot[tid] = rot;
        if (rot) any = 1;
      }
      __syncthreads();
      // A <- J^T A J on 2 x 2 blocks (pair P1 <= P2, mirrored), V <- V J
      const int nblk = np * (np + 1) / 2;
      for (int bk = tid; bk < nblk; bk += 64) {
        int P1 = 0, rem = bk;
        while (rem >= np - P1) { rem -= np - P1; ++P1; }
        const int P2 = P1 + rem;
        if (!prot[P1] && !prot[P2]) continue;
        const int p1 = pp[P1], q1 = pq[P1], p2 = pp[P2], q2 = pq[P2];
        if (P1 == P2) {
          const double apq = A[p1][q1];
          A[p1][p1] -= pt[P1] * apq;
          A[q1][q1] += pt[P1] * apq;
          A[p1][q1] = 0.0;
          A[q1][p1] = 0.0;
          continue;
        }
        const double c1 = pc[P1], s1 = ps[P1], c2 = pc[P2], s2 = ps[P2];
        const double a = A[p1][p2], bb = A[p1][q2], cc = A[q1][p2], dd = A[q1][q2];
        const double rp0 = c1 * a - s1 * cc, rp1 = c1 * bb - s1 * dd;
        const double rq0 = s1 * a + c1 * cc, rq1 = s1 * bb + c1 * dd;
        const double n00 = c2 * rp0 - s2 * rp1, n01 = s2 * rp0 + c2 * rp1;
        const double n10 = c2 * rq0 - s2 * rq1, n11 = s2 * rq0 + c2 * rq1;
        A[p1][p2] = n00; A[p2][p1] = n00;
        A[p1][q2] = n01; A[q2][p1] = n01;
        A[q1][p2] = n10; A[p2][q1] = n10;
        A[q1][q2] = n11; A[q2][q1] = n11;
      }
      for (int x = tid; x < mp * np; x += 64) {
        const int row = x / np, P = x % np;
        if (!prot[P]) continue;
        const int p = pp[P], q = pq[P];
        const double c = pc[P], sn = ps[P], vp = V[row][p], vq = V[row][q];
        V[row][p] = c * vp - sn * vq;
        V[row][q] = sn * vp + c * vq;
      }
      __syncthreads();
    }
    const int again = any;
    __syncthreads();
    if (!again) break;
  }
  // ascending order (ties by index), written at the leaf's block of the level-T buffers
  const int ob = T & 1;
  const double sc = T == 0 ? w.scale[0] : 1.0;
  for (int i = tid; i < m; i += 64) {
    const double v = A[i][i];
    int rk = 0;
    for (int y = 0; y < m; ++y) {
      const double u = A[y][y];
      rk += (u < v) || (u == v && y < i);
    }
    w.dbuf[ob][o + rk] = v * sc;
    double* col = w.zbuf[ob] + (long long)(o + rk) * n + o;
    for (int r = 0; r < m; ++r) col[r] = V[r][i];
  }
}

// Exclusive prefix over the 256 threads of a block of each thread's count v; total in `total`.
__device__ __forceinline__ int block_scan(int v, int* sh, int& total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) sh[wv] = x;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = sh[i];
    base += i < wv ? c : 0;
    tot += c;
  }
  __syncthreads();
  total = tot;
  return base + x - v;
}

// Rotation of the neighbour pair (pj, s) of the merged list that zeroes z[pj], and whether the
// matrix it leaves out, |(d_s - d_pj) C S|, is within tol.
__device__ __forceinline__ bool pair_rot(double zp, double zs, double dp, double ds, double tol, double& C, double& S,
                                         double& tau) {
  tau = hypot(zs, zp);
  C = zs / tau;
  S = -zp / tau;
  return fabs((ds - dp) * C * S) <= tol;
}

// Deflation, one workgroup per parent.  Each thread owns 8 consecutive places of the merged list
// (TRIDIAG_MAX_N = 256 x 8); compactions go through block prefix sums.
__global__ __launch_bounds__(256) void dc_deflate_k(DcWs w, int t) {
  const int n = w.n, tid = threadIdx.x, j0 = blockIdx.x;
  const int o = seg_lo(n, t, j0), m = seg_lo(n, t, j0 + 1) - o;
  const int m1 = seg_lo(n, t + 1, 2 * j0 + 1) - o, m2 = m - m1;
  const int in = (t + 1) & 1;
  const double* din = w.dbuf[in] + o;
  const double* Z = w.zbuf[in];
  const double b = w.es[o + m1 - 1];
  const double rho = 2.0 * fabs(b), sg = b < 0.0 ? -1.0 : 1.0;
  // by place in the merged ascending list
  __shared__ double sd[DMAX], sz[DMAX];
  __shared__ short ssrc[DMAX];   // local source column
  __shared__ short sl[DMAX];     // survivors of the z test, in order
  __shared__ short sx[DMAX];     // flagged pairs, then the final survivors
  __shared__ short sdf[DMAX];    // deflated places
  __shared__ unsigned char smask[DMAX];   // rows touched: 1 first child, 2 second
  __shared__ unsigned char sflg[DMAX];    // 1 z-deflated, 2 rotated out, 4 in a chain
  __shared__ double red[8];
  __shared__ int sh[4];
  __shared__ int snc;
  double md = 0.0, mz = 0.0;
  for (int j = tid; j < m; j += 256) {
    const double dj = din[j];
    double zj = j < m1 ? Z[(long long)(o + j) * n + o + m1 - 1] : sg * Z[(long long)(o + j) * n + o + m1];
    zj *= 0.70710678118654752440;
    int rk;
    if (j < m1) {   // children ascending; the first child's entry goes first on ties
      int lo = 0, hi = m2;
      while (lo < hi) { const int mid = (lo + hi) >> 1; if (din[m1 + mid] < dj) lo = mid + 1; else hi = mid; }
      rk = j + lo;
    } else {
      int lo = 0, hi = m1;
      while (lo < hi) { const int mid = (lo + hi) >> 1; if (din[mid] <= dj) lo = mid + 1; else hi = mid; }
      rk = (j - m1) + lo;
    }
    sd[rk] = dj;
    sz[rk] = zj;
    ssrc[rk] = (short)j;
    smask[rk] = j < m1 ? 1 : 2;
    md = fmax(md, fabs(dj));
    mz = fmax(mz, fabs(zj));
  }
  md = wmax(md);
  mz = wmax(mz);
  if ((tid & 63) == 0) { red[tid >> 6] = md; red[4 + (tid >> 6)] = mz; }
  __syncthreads();
  const double tol = 8.0 * UEPS * fmax(fmax(fmax(red[0], red[1]), fmax(red[2], red[3])),
                                       fmax(fmax(red[4], red[5]), fmax(red[6], red[7])));
  const int e0 = tid * 8, e1 = min(m, e0 + 8);
  // z test; survivors compacted in order
  int cnt = 0;
  for (int x = e0; x < e1; ++x) {
    const bool dz = rho * fabs(sz[x]) <= tol;
    sflg[x] = dz ? 1 : 0;
    cnt += !dz;
  }
  int ns;
  int pos = block_scan(cnt, sh, ns);
  for (int x = e0; x < e1; ++x)
    if (!sflg[x]) sl[pos++] = (short)x;
  __syncthreads();
  // neighbour pairs of survivors that rotate on unrotated values
  cnt = 0;
  unsigned pf = 0;
  for (int q = e0; q < min(ns - 1, e0 + 8); ++q) {
    double C, S, tau;
    const int a = sl[q], c = sl[q + 1];
    if (pair_rot(sz[a], sz[c], sd[a], sd[c], tol, C, S, tau)) { pf |= 1u << (q - e0); ++cnt; }
  }
  int nfl;
  pos = block_scan(cnt, sh, nfl);
  for (int q = e0; q < min(ns - 1, e0 + 8); ++q)
    if (pf >> (q - e0) & 1) sx[pos++] = (short)q;
  __syncthreads();
  // rotation chains, walked serially from each flagged pair not yet consumed
  if (tid == 0) {
    int nc = 0, cpos = 0, next = 0;
    int* cm = w.cm + o;
    double* rc = w.rc + o;
    double* rs = w.rs + o;
    for (int f = 0; f < nfl; ++f) {
      int q = sx[f];
      if (q < next) continue;
      int pj = sl[q];
      bool open = false;
      while (q + 1 < ns) {
        const int x = sl[q + 1];
        double C, S, tau;
        if (!pair_rot(sz[pj], sz[x], sd[pj], sd[x], tol, C, S, tau)) break;
        if (!open) {
          w.chs[o + nc] = cpos;
          cm[cpos++] = ssrc[pj];
          sflg[pj] |= 4;
          open = true;
        }
        rc[cpos - 1] = C;
        rs[cpos - 1] = S;
        cm[cpos++] = ssrc[x];
        sflg[x] |= 4;
        sz[x] = tau;
        sz[pj] = 0.0;
        const double dp = sd[pj], dn = sd[x];
        sd[pj] = dp * C * C + dn * S * S;
        sd[x] = dp * S * S + dn * C * C;
        smask[x] |= smask[pj];
        sflg[pj] |= 2;
        pj = x;
        ++q;
      }
      if (open) { w.chl[o + nc] = cpos - 1 - w.chs[o + nc]; ++nc; }
      next = q + 1;
    }
    snc = nc;
  }
  __syncthreads();
  // final survivors in order, with their groups; deflated places in order
  int c1 = 0, c3 = 0, c2 = 0;
  cnt = 0;
  for (int q = e0; q < min(ns, e0 + 8); ++q) {
    const int x = sl[q];
    if (sflg[x] & 2) continue;
    ++cnt;
    const int g = smask[x];
    c1 += g == 1; c3 += g == 3; c2 += g == 2;
  }
  int k, n1, n12, n3, nd;
  pos = block_scan(cnt, sh, k);
  int b1 = block_scan(c1, sh, n1), b3 = block_scan(c3, sh, n12), b2 = block_scan(c2, sh, n3);
  for (int q = e0; q < min(ns, e0 + 8); ++q) {
    const int x = sl[q];
    if (sflg[x] & 2) continue;
    const int g = smask[x];
    const int cp = g == 1 ? b1++ : (g == 3 ? n1 + b3++ : n1 + n12 + b2++);
    w.dl[o + pos] = sd[x];
    w.zl[o + pos] = sz[x];
    w.qpos[o + pos] = cp;
    w.dest[o + ssrc[x]] = cp;
    ++pos;
  }
  cnt = 0;
  for (int x = e0; x < e1; ++x) cnt += (sflg[x] & 3) != 0;
  pos = block_scan(cnt, sh, nd);
  for (int x = e0; x < e1; ++x)
    if (sflg[x] & 3) {
      w.val[o + k + pos] = sd[x];
      w.dest[o + ssrc[x]] = -1 - pos;
      ++pos;
    }
  for (int x = e0; x < e1; ++x) w.inch[o + ssrc[x]] = (sflg[x] & 4) ? 1 : 0;
  if (tid == 0) {
    DcPar P;
    P.k = k; P.n1 = n1; P.n12 = n12; P.n3 = n3; P.ndef = nd; P.nchain = snc; P.rho = rho;
    w.par[j0] = P;
  }
}

// Root i of the secular equation of its parent, one wavefront per root.
__global__ __launch_bounds__(256) void dc_secular_k(DcWs w, int t) {
  const int gw = (int)((blockIdx.x * 256u + threadIdx.x) >> 6), lane = threadIdx.x & 63;
  if (gw >= w.n) return;
  const int par = parent_of(w.n, t, gw), o = seg_lo(w.n, t, par);
  const DcPar P = w.par[par];
  const int i = gw - o, k = P.k;
  if (i >= k) return;
  const double* dl = w.dl + o;
  const double* zl = w.zl + o;
  const double rho = P.rho, rinv = 1.0 / rho;
  double dj[SQ], z2[SQ];
#pragma unroll
  for (int q = 0; q < SQ; ++q) {
    const int j = lane + 64 * q;
    dj[q] = j < k ? dl[j] : 0.0;
    z2[q] = j < k ? zl[j] * zl[j] : 0.0;
  }
  int org;
  double lo, hi;
  if (i < k - 1) {
    const double di = dl[i], h = 0.5 * (dl[i + 1] - di);
    double f = 0.0;
#pragma unroll
    for (int q = 0; q < SQ; ++q)
      if (lane + 64 * q < k) f += z2[q] / ((dj[q] - di) - h);
    f = wsum(f) + rinv;
    if (f >= 0.0) { org = i; lo = 0.0; hi = h; }
    else { org = i + 1; lo = -h; hi = 0.0; }
  } else {
    double s2 = 0.0;
#pragma unroll
    for (int q = 0; q < SQ; ++q) s2 += z2[q];
    org = k - 1;
    lo = 0.0;
    hi = rho * wsum(s2);
  }
  const double dorg = dl[org], di = dl[i], di1 = i + 1 < k ? dl[i + 1] : 0.0;
  double tau = 0.5 * (lo + hi);
  bool ok = false;
  for (int it = 0; it < 200; ++it) {
    double psi = 0.0, phi = 0.0, dpsi = 0.0, dphi = 0.0, sab = 0.0;
#pragma unroll
    for (int q = 0; q < SQ; ++q) {
      const int j = lane + 64 * q;
      if (j < k) {
        const double rd = 1.0 / ((dj[q] - dorg) - tau);
        const double t1 = z2[q] * rd, t2 = t1 * rd;
        if (j <= i) { psi += t1; dpsi += t2; }
        else { phi += t1; dphi += t2; }
        sab += fabs(t1);
      }
    }
    psi = wsum(psi); phi = wsum(phi); dpsi = wsum(dpsi); dphi = wsum(dphi); sab = wsum(sab);
    const double wv = rinv + psi + phi;
    const double err = UEPS * (8.0 * sab + 2.0 * rinv + 3.0 * fabs(tau) * (dpsi + dphi));
    if (wv < 0.0) lo = tau;
    else hi = tau;
    if (fabs(wv) <= err || hi - lo <= 4.0 * UEPS * fmax(fabs(lo), fabs(hi))) { ok = true; break; }
    const double a = (di - dorg) - tau;   // distance to the left pole (negative)
    double eta = 0.0;
    bool have = false;
    if (i < k - 1) {
      const double bq = (di1 - dorg) - tau;   // distance to the right pole (positive)
      const double Aq = a * a * dpsi, Bq = bq * bq * dphi, c = wv - a * dpsi - bq * dphi;
      const double qb = c * (a + bq) + Aq + Bq, qc = c * a * bq + Aq * bq + Bq * a;
      if (c == 0.0) {
        if (qb != 0.0) { eta = qc / qb; have = eta > a && eta < bq; }
      } else {
        const double sq = sqrt(fmax(qb * qb - 4.0 * c * qc, 0.0));
        double r1, r2;
        if (qb >= 0.0) { r1 = (qb + sq) / (2.0 * c); r2 = (qb + sq) != 0.0 ? 2.0 * qc / (qb + sq) : r1; }
        else { r1 = 2.0 * qc / (qb - sq); r2 = (qb - sq) / (2.0 * c); }
        const bool in1 = r1 > a && r1 < bq, in2 = r2 > a && r2 < bq;
        if (in1 && in2) { eta = fabs(r1) < fabs(r2) ? r1 : r2; have = true; }
        else if (in1) { eta = r1; have = true; }
        else if (in2) { eta = r2; have = true; }
      }
    } else {
      const double c = wv - a * dpsi;
      if (c > 0.0) { eta = a + a * a * dpsi / c; have = true; }
    }
    double tn = 0.5 * (lo + hi);
    if (have && (it & 15) != 15) {
      const double tc = tau + eta;
      if (tc > lo && tc < hi) tn = tc;
    }
    if (tn == tau) { ok = true; break; }
    tau = tn;
  }
  if (lane == 0) {
    w.tau[o + i] = tau;
    w.orig[o + i] = org;
    w.val[o + i] = dorg + tau;
    if (!ok) atomicOr(w.info, 1);
  }
}

// Place of every eigenvalue of a parent in its ascending output (ties by index); block (parent,
// 64 values), the four wavefronts counting over quarters of the parent.
__device__ __forceinline__ void rank_blk(const DcWs& w, int t, int par, int tile) {
  const int n = w.n, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int o = seg_lo(n, t, par), m = seg_lo(n, t, par + 1) - o;
  if (tile * 64 >= m) return;
  __shared__ double sv[DMAX];
  __shared__ int part[4][64];
  for (int x = tid; x < m; x += 256) sv[x] = w.val[o + x];
  __syncthreads();
  const int x = tile * 64 + lane;
  const double v = x < m ? sv[x] : 0.0;
  const int y0 = (m * wv) >> 2, y1 = (m * (wv + 1)) >> 2;
  int r = 0;
  for (int y = y0; y < y1; ++y) {
    const double u = sv[y];
    r += (u < v) || (u == v && y < x);
  }
  part[wv][lane] = r;
  __syncthreads();
  if (wv == 0 && x < m) {
    r = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
    w.rank[o + x] = r;
    w.dbuf[t & 1][o + r] = t == 0 ? v * w.scale[0] : v;
  }
}

// Recomputed weight of survivor j (global wavefront index gw), one wavefront per survivor.
__device__ __forceinline__ void zhat_wave(const DcWs& w, int t, int gw) {
  const int lane = threadIdx.x & 63;
  if (gw >= w.n) return;
  const int par = parent_of(w.n, t, gw), o = seg_lo(w.n, t, par);
  const DcPar P = w.par[par];
  const int j = gw - o, k = P.k;
  if (j >= k) return;
  const double* dl = w.dl + o;
  const double dj = dl[j];
  double prod = 1.0;
  for (int r = lane; r < k; r += 64) {
    const double num = (dl[w.orig[o + r]] - dj) + w.tau[o + r];
    const double den = r == k - 1 ? P.rho : (r < j ? dl[r] - dj : dl[r + 1] - dj);
    prod *= num / den;
  }
  prod = wprod(prod);
  if (lane == 0) w.zh[o + j] = copysign(sqrt(fmax(prod, 0.0)), w.zl[o + j]);
}

// Eigenvector i of diag(d) + rho zhat zhat^T, one wavefront per root, into column i of the
// parent's block of Mm, rows in the compact order.
__device__ __forceinline__ void vec_wave(const DcWs& w, int t, int gw) {
  const int n = w.n, lane = threadIdx.x & 63;
  if (gw >= n) return;
  const int par = parent_of(n, t, gw), o = seg_lo(n, t, par);
  const DcPar P = w.par[par];
  const int i = gw - o, k = P.k;
  if (i >= k) return;
  const double* dl = w.dl + o;
  const double* zh = w.zh + o;
  const double dorg = dl[w.orig[o + i]], ti = w.tau[o + i];
  double ss = 0.0;
  for (int j = lane; j < k; j += 64) {
    const double u = zh[j] / ((dl[j] - dorg) - ti);
    ss += u * u;
  }
  const double inv = 1.0 / sqrt(wsum(ss));
  double* col = w.Mm + (long long)(o + i) * n + o;
  for (int j = lane; j < k; j += 64) col[w.qpos[o + j]] = zh[j] / ((dl[j] - dorg) - ti) * inv;
}

// Destination column of local source j of a parent: its compact place (survivors) or its output
// place (deflated).
__device__ __forceinline__ double* dest_col(const DcWs& w, int t, int o, int k, int j) {
  const int dst = w.dest[o + j];
  return dst >= 0 ? w.Qc + (long long)(o + dst) * w.n + o
                  : w.zbuf[t & 1] + (long long)(o + w.rank[o + k - 1 - dst]) * w.n + o;
}

// Columns of blockdiag(Q1, Q2) that no rotation touches; block (parent, 64 rows, 32 columns).
__device__ __forceinline__ void gather_blk(const DcWs& w, int t, int bx, int rt, int ct) {
  const int n = w.n;
  const int tc = bx % ct;
  bx /= ct;
  const int tr = bx % rt, par = bx / rt;
  const int o = seg_lo(n, t, par), m = seg_lo(n, t, par + 1) - o;
  const int m1 = seg_lo(n, t + 1, 2 * par + 1) - o;
  const int r = tr * 64 + (threadIdx.x & 63);
  if (tc * 32 >= m || r >= m) return;
  const int k = w.par[par].k;
  const double* Zin = w.zbuf[(t + 1) & 1];
  for (int c = threadIdx.x >> 6; c < 32; c += 4) {
    const int j = tc * 32 + c;
    if (j >= m) break;
    if (w.inch[o + j]) continue;
    const bool inblk = j < m1 ? r < m1 : r >= m1;
    dest_col(w, t, o, k, j)[r] = inblk ? Zin[(long long)(o + j) * n + o + r] : 0.0;
  }
}

// Rotation chains replayed on their columns, one thread per row; block (parent, 64 rows), the four
// wavefronts taking every fourth chain.
__device__ __forceinline__ void chain_blk(const DcWs& w, int t, int bx, int rt) {
  const int n = w.n, par = bx / rt, tr = bx % rt;
  const int o = seg_lo(n, t, par), m = seg_lo(n, t, par + 1) - o;
  const int m1 = seg_lo(n, t + 1, 2 * par + 1) - o;
  const DcPar P = w.par[par];
  const int r = tr * 64 + (threadIdx.x & 63);
  if (P.nchain == 0 || r >= m) return;
  const double* Zin = w.zbuf[(t + 1) & 1];
  auto val = [&](int j) {
    const bool inblk = j < m1 ? r < m1 : r >= m1;
    return inblk ? Zin[(long long)(o + j) * n + o + r] : 0.0;
  };
  for (int c = threadIdx.x >> 6; c < P.nchain; c += 4) {
    const int s0 = w.chs[o + c], L = w.chl[o + c];
    double x = val(w.cm[o + s0]);
    for (int l = 0; l < L; ++l) {
      const double y = val(w.cm[o + s0 + l + 1]);
      const double C = w.rc[o + s0 + l], S = w.rs[o + s0 + l];
      dest_col(w, t, o, P.k, w.cm[o + s0 + l])[r] = C * x + S * y;
      x = C * y - S * x;
    }
    dest_col(w, t, o, P.k, w.cm[o + s0 + L])[r] = x;
  }
}

// After the roots: ranks (blocks [0, nrank)) and recomputed weights (the rest).
__global__ __launch_bounds__(256) void dc_post1_k(DcWs w, int t, int tiles, int nrank) {
  const int bx = blockIdx.x;
  if (bx < nrank) rank_blk(w, t, bx / tiles, bx % tiles);
  else zhat_wave(w, t, (int)(((bx - nrank) * 256u + threadIdx.x) >> 6));
}

// After the weights and ranks: eigenvectors of the rank-one updates (blocks [0, nvec)), untouched
// columns (the next ngat), rotation chains (the rest).
__global__ __launch_bounds__(256) void dc_post2_k(DcWs w, int t, int nvec, int ngat, int rt, int ct) {
  const int bx = blockIdx.x;
  if (bx < nvec) vec_wave(w, t, (int)((bx * 256u + threadIdx.x) >> 6));
  else if (bx < nvec + ngat) gather_blk(w, t, bx - nvec, rt, ct);
  else chain_blk(w, t, bx - nvec - ngat, rt);
}

// The survivors' eigenvectors: block (parent, child half, 64 rows, 32 roots); each root's column
// goes to its place in the ascending output.
__global__ __launch_bounds__(256, 3) void dc_gemm_k(DcWs w, int t, int tm_n, int tn_n) {
  using namespace f64t::wide;
  __shared__ Smem sm;
  const int n = w.n;
  int bx = blockIdx.x;
  const int tn = bx % tn_n;
  bx /= tn_n;
  const int tm = bx % tm_n;
  bx /= tm_n;
  const int half = bx & 1, par = bx >> 1;
  const int o = seg_lo(n, t, par), m = seg_lo(n, t, par + 1) - o;
  const int m1 = seg_lo(n, t + 1, 2 * par + 1) - o;
  const DcPar P = w.par[par];
  const int rows = half ? m - m1 : m1, r0 = half ? m1 : 0;
  const int c0 = half ? P.n1 : 0, K = half ? P.n12 + P.n3 : P.n1 + P.n12;
  const int m0 = tm * BM, n0 = tn * BNT;
  if (m0 >= rows || n0 >= P.k) return;
  const double* A = w.Qc + (long long)(o + c0) * n + o + r0;   // A(r, c) at c * n + r
  const double* B = w.Mm + (long long)o * n + o + c0;          // B(c, i) at i * n + c
  f64x4 acc[2];
  wide_tile<true, false>(sm, A, 1, n, B, 1, n, rows, P.k, K, m0, n0, acc);
  double* Zout = w.zbuf[t & 1];
  const int i = n0 + wide_col();
  if (i >= P.k) return;
  double* col = Zout + (long long)(o + w.rank[o + i]) * n + o + r0;
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int r = m0 + wide_row(mi, jj);
      if (r < rows) col[r] = acc[mi][jj];
    }
}

inline int cdiv_i(int a, int b) { return (a + b - 1) / b; }

int dc_depth(int n) {
  int t = 0;
  while (cdiv_i(n, 1 << t) > DC_LEAF) ++t;
  return t;
}

}  // namespace

long long tridiag_dc_ws_doubles(int n) {
  const long long nn = (long long)n * n;
  return 3 * nn + 32LL * n + 512;
}

hipError_t tridiag_eig_dc(hipStream_t s, int n, double* d, const double* e, double* Z, double* ws, int* info) {
  if (n <= 0 || n > TRIDIAG_MAX_N) return hipErrorInvalidValue;
  const long long nn = (long long)n * n;
  DcWs w;
  w.n = n;
  w.T = dc_depth(n);
  double* p = ws;
  auto take = [&](long long cnt) { double* r = p; p += (cnt + 7) & ~7LL; return r; };
  w.zbuf[0] = Z;
  w.zbuf[1] = take(nn);
  w.Qc = take(nn);
  w.Mm = take(nn);
  w.dbuf[0] = d;
  w.dbuf[1] = take(n);
  w.dS = take(n);
  w.es = take(n);
  w.scale = take(1);
  w.dl = take(n); w.zl = take(n); w.zh = take(n); w.tau = take(n); w.val = take(n); w.rc = take(n); w.rs = take(n);
  auto itake = [&]() { return reinterpret_cast<int*>(take((n + 1) / 2)); };
  w.orig = itake(); w.rank = itake(); w.qpos = itake(); w.dest = itake(); w.inch = itake();
  w.cm = itake(); w.chs = itake(); w.chl = itake();
  w.par = reinterpret_cast<DcPar*>(take(4LL * n));
  w.info = info;
  hipLaunchKernelGGL(dc_prep_k, dim3(1), dim3(1024), 0, s, w, d, e);
  hipLaunchKernelGGL(dc_leaf_k, dim3(1u << w.T), dim3(64), 0, s, w);
  const int waves = cdiv_i(n * 64, 256);
  for (int t = w.T - 1; t >= 0; --t) {
    const int np = 1 << t, mmax = cdiv_i(n, np), mcmax = cdiv_i(n, 2 * np);
    hipLaunchKernelGGL(dc_deflate_k, dim3(np), dim3(256), 0, s, w, t);
    hipLaunchKernelGGL(dc_secular_k, dim3(waves), dim3(256), 0, s, w, t);
    const int tiles = cdiv_i(mmax, 64), nrank = np * tiles;
    hipLaunchKernelGGL(dc_post1_k, dim3(nrank + waves), dim3(256), 0, s, w, t, tiles, nrank);
    const int rt = cdiv_i(mmax, 64), ct = cdiv_i(mmax, 32), ngat = np * rt * ct;
    hipLaunchKernelGGL(dc_post2_k, dim3(waves + ngat + np * rt), dim3(256), 0, s, w, t, waves, ngat, rt, ct);
    const int tm_n = cdiv_i(mcmax, f64t::wide::BM), tn_n = cdiv_i(mmax, f64t::wide::BNT);
    hipLaunchKernelGGL(dc_gemm_k, dim3(np * 2 * tm_n * tn_n), dim3(256), 0, s, w, t, tm_n, tn_n);
  }
  return hipGetLastError();
}

}  // namespace pnof
