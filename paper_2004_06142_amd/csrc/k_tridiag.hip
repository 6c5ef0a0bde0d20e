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
// Leaves: one workgroup each, cyclic Jacobi (round-robin pairs, the matrix in LDS).
// Merge of two children with eigen-decompositions T1 = Q1 D1 Q1^T, T2 = Q2 D2 Q2^T, per level, for
// all parents of the level at once (kernels in launch order):
//   deflate  z = [last row of Q1, sign(b) first row of Q2] / sqrt 2, rho = 2 |b|; the children's
//            eigenvalues merged into one ascending list; entries with rho |z_j| <= tol leave as they
//            are, and a neighbour pair whose rotation zeroing one z entry perturbs the matrix by
//            less than tol is rotated (the rotated entry leaves); tol = 8 eps max(|d|, |z|).  The
//            rotations form chains (each continues with the surviving entry), replayed later on
//            the eigenvector columns.  The k survivors keep strictly increasing d.
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
// Eigenvalues and vectors ping-pong between the caller's (w, Z) and a workspace pair by level
// parity, so that the last merge writes the caller's arrays.
#include "common.h"
#include "f64_tile.h"

namespace pnof {
namespace {

constexpr int DC_LEAF = 48;                 // rows of a leaf at most (Jacobi in one workgroup)
constexpr int DC_LP = DC_LEAF + 2;          // leaf LDS row pitch (one padding row for odd sizes)
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

// One leaf per workgroup: cyclic Jacobi with round-robin pairs (every round rotates m/2 disjoint
// pairs at once), until a sweep rotates nothing.  A pair is left alone when its off-diagonal entry
// is below eps sqrt(|a_pp a_qq|) or 1e-3 eps of the leaf's largest entry.
__global__ __launch_bounds__(256) void dc_leaf_k(DcWs w) {
  const int n = w.n, T = w.T, tid = threadIdx.x;
  const int o = seg_lo(n, T, blockIdx.x), m = seg_lo(n, T, blockIdx.x + 1) - o;
  const int mp = m + (m & 1), np = mp / 2;
  __shared__ double A[DC_LEAF + 1][DC_LP], V[DC_LEAF + 1][DC_LP];
  __shared__ double pc[DC_LEAF / 2 + 1], ps[DC_LEAF / 2 + 1], pt[DC_LEAF / 2 + 1];
  __shared__ int pp[DC_LEAF / 2 + 1], pq[DC_LEAF / 2 + 1], prot[DC_LEAF / 2 + 1];
  __shared__ int any;
  __shared__ double anrm;
  for (int x = tid; x < mp * mp; x += 256) {
    const int r = x / mp, c = x % mp;
    double a = 0.0;
    if (r < m && c < m) {
      if (r == c) a = w.dS[o + r];
      else if (c == r + 1) a = w.es[o + r];
      else if (r == c + 1) a = w.es[o + c];
    }
    A[r][c] = a;
    V[r][c] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  if (tid < 64) {
    double v = 0.0;
    for (int x = tid; x < m * m; x += 64) v = fmax(v, fabs(A[x / m][x % m]));
    v = wmax(v);
    if (tid == 0) anrm = v;
  }
  __syncthreads();
  const double athr = 1e-3 * UEPS * anrm;
  for (int sweep = 0; sweep < 40 && mp > 1; ++sweep) {
    if (tid == 0) any = 0;
    __syncthreads();
    for (int r = 0; r < mp - 1; ++r) {
      if (tid < np) {
        int p, q;
        if (tid == 0) { p = r; q = mp - 1; }
        else { p = (r + tid) % (mp - 1); q = (r - tid + mp - 1) % (mp - 1); }
        if (p > q) { const int x = p; p = q; q = x; }
        double c = 1.0, s = 0.0, tt = 0.0;
        int rot = 0;
        if (q < m) {
          const double apq = A[p][q], app = A[p][p], aqq = A[q][q];
          if (fabs(apq) > athr && fabs(apq) > UEPS * sqrt(fabs(app * aqq))) {
            const double th = (aqq - app) / (2.0 * apq);
            tt = fabs(th) > 1e150 ? 0.5 / th : copysign(1.0, th) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
            rot = 1;
          }
        }
        pp[tid] = p; pq[tid] = q; pc[tid] = c; ps[tid] = s; pt[tid] = tt; prot[tid] = rot;
        if (rot) any = 1;
      }
      __syncthreads();
      // A <- J^T A J on 2 x 2 blocks (pair P1 <= P2, mirrored), V <- V J
      const int nblk = np * (np + 1) / 2;
      for (int b = tid; b < nblk; b += 256) {
        int P1 = 0, rem = b;
        while (rem >= np - P1) { rem -= np - P1; ++P1; }
        const int P2 = P1 + rem;
        const int p1 = pp[P1], q1 = pq[P1], p2 = pp[P2], q2 = pq[P2];
        if (!prot[P1] && !prot[P2]) continue;
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
      for (int x = tid; x < mp * np; x += 256) {
        const int row = x / np, P = x % np;
        if (!prot[P]) continue;
        const int p = pp[P], q = pq[P];
        const double c = pc[P], s = ps[P], vp = V[row][p], vq = V[row][q];
        V[row][p] = c * vp - s * vq;
        V[row][q] = s * vp + c * vq;
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
  for (int i = tid; i < m; i += 256) {
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

// Deflation, one workgroup per parent; the scan over the merged list is serial (thread 0), the rest
// is spread over the block.
__global__ __launch_bounds__(256) void dc_deflate_k(DcWs w, int t) {
  const int n = w.n, tid = threadIdx.x, j0 = blockIdx.x;
  const int o = seg_lo(n, t, j0), m = seg_lo(n, t, j0 + 1) - o;
  const int m1 = seg_lo(n, t + 1, 2 * j0 + 1) - o, m2 = m - m1;
  const int in = (t + 1) & 1;
  const double* din = w.dbuf[in] + o;
  const double* Z = w.zbuf[in];
  const double b = w.es[o + m1 - 1];
  const double rho = 2.0 * fabs(b), sg = b < 0.0 ? -1.0 : 1.0;
  // by position in the merged ascending list
  __shared__ double sd[DMAX], sz[DMAX];
  __shared__ short ssrc[DMAX], snd[DMAX], sdf[DMAX];
  __shared__ unsigned char smask[DMAX], sinch[DMAX];
  __shared__ double red[8];
  __shared__ int cnt[256][3];
  __shared__ int tot[5];
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
    sinch[rk] = 0;
    md = fmax(md, fabs(dj));
    mz = fmax(mz, fabs(zj));
  }
  md = wmax(md);
  mz = wmax(mz);
  if ((tid & 63) == 0) { red[tid >> 6] = md; red[4 + (tid >> 6)] = mz; }
  __syncthreads();
  const double tol = 8.0 * UEPS * fmax(fmax(fmax(red[0], red[1]), fmax(red[2], red[3])),
                                       fmax(fmax(red[4], red[5]), fmax(red[6], red[7])));
  if (tid == 0) {
    int k = 0, nd = 0, nc = 0, cpos = 0, pj = -1;
    bool open = false;
    int* cm = w.cm + o;
    double* rc = w.rc + o;
    double* rs = w.rs + o;
    for (int s = 0; s < m; ++s) {
      if (rho * fabs(sz[s]) <= tol) { sdf[nd++] = (short)s; continue; }
      if (pj < 0) { pj = s; continue; }
      const double zp = sz[pj], zs = sz[s];
      const double tau = hypot(zs, zp);
      const double C = zs / tau, S = -zp / tau;
      if (fabs((sd[s] - sd[pj]) * C * S) <= tol) {
        if (!open) {
          w.chs[o + nc] = cpos;
          cm[cpos++] = ssrc[pj];
          sinch[pj] = 1;
          open = true;
        }
        rc[cpos - 1] = C;
        rs[cpos - 1] = S;
        cm[cpos++] = ssrc[s];
        sinch[s] = 1;
        sz[s] = tau;
        sz[pj] = 0.0;
        const double dp = sd[pj], dn = sd[s];
        sd[pj] = dp * C * C + dn * S * S;
        sd[s] = dp * S * S + dn * C * C;
        smask[s] |= smask[pj];
        sdf[nd++] = (short)pj;
        pj = s;
      } else {
        if (open) { w.chl[o + nc] = cpos - 1 - w.chs[o + nc]; ++nc; open = false; }
        snd[k++] = (short)pj;
        pj = s;
      }
    }
    if (pj >= 0) {
      if (open) { w.chl[o + nc] = cpos - 1 - w.chs[o + nc]; ++nc; }
      snd[k++] = (short)pj;
    }
    tot[0] = k;
    tot[1] = nd;
    tot[2] = nc;
  }
  __syncthreads();
  const int k = tot[0], nd = tot[1];
  // survivors: groups by the rows they touch, compact positions in group order
  const int per = (k + 255) / 256, i0 = tid * per, i1 = min(k, i0 + per);
  int c1 = 0, c3 = 0, c2 = 0;
  for (int i = i0; i < i1; ++i) {
    const int g = smask[snd[i]];
    c1 += g == 1; c3 += g == 3; c2 += g == 2;
  }
  cnt[tid][0] = c1; cnt[tid][1] = c3; cnt[tid][2] = c2;
  __syncthreads();
  if (tid == 0) {
    int a1 = 0, a3 = 0, a2 = 0;
    for (int x = 0; x < 256; ++x) {
      const int v1 = cnt[x][0], v3 = cnt[x][1], v2 = cnt[x][2];
      cnt[x][0] = a1; cnt[x][1] = a3; cnt[x][2] = a2;
      a1 += v1; a3 += v3; a2 += v2;
    }
    tot[3] = a1;
    tot[4] = a3;
    DcPar P;
    P.k = k; P.n1 = a1; P.n12 = a3; P.n3 = a2; P.ndef = nd; P.nchain = tot[2]; P.rho = rho;
    w.par[j0] = P;
  }
  __syncthreads();
  {
    const int n1 = tot[3], n12 = tot[4];
    int b1 = cnt[tid][0], b3 = cnt[tid][1], b2 = cnt[tid][2];
    for (int i = i0; i < i1; ++i) {
      const int s = snd[i], g = smask[s];
      const int pos = g == 1 ? b1++ : (g == 3 ? n1 + b3++ : n1 + n12 + b2++);
      w.dl[o + i] = sd[s];
      w.zl[o + i] = sz[s];
      w.qpos[o + i] = pos;
      w.dest[o + ssrc[s]] = pos;
    }
  }
  for (int q = tid; q < nd; q += 256) {
    const int s = sdf[q];
    w.val[o + k + q] = sd[s];
    w.dest[o + ssrc[s]] = -1 - q;
  }
  for (int s = tid; s < m; s += 256) w.inch[o + ssrc[s]] = sinch[s];
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
        const double del = (dj[q] - dorg) - tau;
        const double t1 = z2[q] / del, t2 = t1 / del;
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

// Place of every eigenvalue of a parent in its ascending output (ties by index).
__global__ __launch_bounds__(256) void dc_rank_k(DcWs w, int t, int tiles) {
  const int n = w.n, par = blockIdx.x / tiles, tile = blockIdx.x % tiles;
  const int o = seg_lo(n, t, par), m = seg_lo(n, t, par + 1) - o;
  if (tile * 256 >= m) return;
  __shared__ double sv[DMAX];
  for (int x = threadIdx.x; x < m; x += 256) sv[x] = w.val[o + x];
  __syncthreads();
  const int x = tile * 256 + threadIdx.x;
  if (x >= m) return;
  const double v = sv[x];
  int r = 0;
  for (int y = 0; y < m; ++y) {
    const double u = sv[y];
    r += (u < v) || (u == v && y < x);
  }
  w.rank[o + x] = r;
  w.dbuf[t & 1][o + r] = t == 0 ? v * w.scale[0] : v;
}

// Recomputed weight of survivor j, one wavefront per survivor.
__global__ __launch_bounds__(256) void dc_zhat_k(DcWs w, int t) {
  const int gw = (int)((blockIdx.x * 256u + threadIdx.x) >> 6), lane = threadIdx.x & 63;
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
__global__ __launch_bounds__(256) void dc_vec_k(DcWs w, int t) {
  const int n = w.n;
  const int gw = (int)((blockIdx.x * 256u + threadIdx.x) >> 6), lane = threadIdx.x & 63;
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

// Columns of blockdiag(Q1, Q2) that no rotation touches; block (parent, 64 rows, 32 columns).
__global__ __launch_bounds__(256) void dc_gather_k(DcWs w, int t, int rt, int ct) {
  const int n = w.n;
  int bx = blockIdx.x;
  const int tc = bx % ct;
  bx /= ct;
  const int tr = bx % rt, par = bx / rt;
  const int o = seg_lo(n, t, par), m = seg_lo(n, t, par + 1) - o;
  const int m1 = seg_lo(n, t + 1, 2 * par + 1) - o;
  const int r = tr * 64 + (threadIdx.x & 63);
  if (tr * 64 >= m || tc * 32 >= m || r >= m) return;
  const int k = w.par[par].k;
  const double* Zin = w.zbuf[(t + 1) & 1];
  double* Zout = w.zbuf[t & 1];
  for (int c = threadIdx.x >> 6; c < 32; c += 4) {
    const int j = tc * 32 + c;
    if (j >= m) break;
    if (w.inch[o + j]) continue;
    const int dst = w.dest[o + j];
    double* col = dst >= 0 ? w.Qc + (long long)(o + dst) * n + o : Zout + (long long)(o + w.rank[o + k - 1 - dst]) * n + o;
    const bool inblk = j < m1 ? r < m1 : r >= m1;
    col[r] = inblk ? Zin[(long long)(o + j) * n + o + r] : 0.0;
  }
}

// Rotation chains replayed on their columns, one thread per row; block (parent, 64 rows), the four
// wavefronts taking every fourth chain.
__global__ __launch_bounds__(256) void dc_chain_k(DcWs w, int t, int rt) {
  const int n = w.n, par = blockIdx.x / rt, tr = blockIdx.x % rt;
  const int o = seg_lo(n, t, par), m = seg_lo(n, t, par + 1) - o;
  const int m1 = seg_lo(n, t + 1, 2 * par + 1) - o;
  const DcPar P = w.par[par];
  const int r = tr * 64 + (threadIdx.x & 63);
  if (P.nchain == 0 || r >= m) return;
  const double* Zin = w.zbuf[(t + 1) & 1];
  double* Zout = w.zbuf[t & 1];
  auto val = [&](int j) {
    const bool inblk = j < m1 ? r < m1 : r >= m1;
    return inblk ? Zin[(long long)(o + j) * n + o + r] : 0.0;
  };
  auto put = [&](int j, double v) {
    const int dst = w.dest[o + j];
    double* col = dst >= 0 ? w.Qc + (long long)(o + dst) * n + o : Zout + (long long)(o + w.rank[o + P.k - 1 - dst]) * n + o;
    col[r] = v;
  };
  for (int c = threadIdx.x >> 6; c < P.nchain; c += 4) {
    const int s0 = w.chs[o + c], L = w.chl[o + c];
    double x = val(w.cm[o + s0]);
    for (int l = 0; l < L; ++l) {
      const double y = val(w.cm[o + s0 + l + 1]);
      const double C = w.rc[o + s0 + l], S = w.rs[o + s0 + l];
      put(w.cm[o + s0 + l], C * x + S * y);
      x = C * y - S * x;
    }
    put(w.cm[o + s0 + L], x);
  }
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
  hipLaunchKernelGGL(dc_leaf_k, dim3(1u << w.T), dim3(256), 0, s, w);
  const unsigned waves = (unsigned)cdiv_i(n * 64, 256);
  for (int t = w.T - 1; t >= 0; --t) {
    const int np = 1 << t, mmax = cdiv_i(n, np), mcmax = cdiv_i(n, 2 * np);
    hipLaunchKernelGGL(dc_deflate_k, dim3(np), dim3(256), 0, s, w, t);
    hipLaunchKernelGGL(dc_secular_k, dim3(waves), dim3(256), 0, s, w, t);
    const int rtl = cdiv_i(mmax, 256);
    hipLaunchKernelGGL(dc_rank_k, dim3(np * rtl), dim3(256), 0, s, w, t, rtl);
    hipLaunchKernelGGL(dc_zhat_k, dim3(waves), dim3(256), 0, s, w, t);
    hipLaunchKernelGGL(dc_vec_k, dim3(waves), dim3(256), 0, s, w, t);
    const int rt = cdiv_i(mmax, 64), ct = cdiv_i(mmax, 32);
    hipLaunchKernelGGL(dc_gather_k, dim3(np * rt * ct), dim3(256), 0, s, w, t, rt, ct);
    hipLaunchKernelGGL(dc_chain_k, dim3(np * rt), dim3(256), 0, s, w, t, rt);
    const int tm_n = cdiv_i(mcmax, f64t::wide::BM), tn_n = cdiv_i(mmax, f64t::wide::BNT);
    hipLaunchKernelGGL(dc_gemm_k, dim3(np * 2 * tm_n * tn_n), dim3(256), 0, s, w, t, tm_n, tn_n);
  }
  return hipGetLastError();
}

}  // namespace pnof
