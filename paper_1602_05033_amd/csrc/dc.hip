// Divide and conquer for the symmetric band matrix T_m (half-bandwidth ell),
// returning every eigenvalue and only the first and last ell rows of the
// eigenvector matrix Q — the data Proposition 1 needs (Section 3.2 computes
// exactly these rows, E_1^T Q and E_m^T Q, from a band-to-tridiagonal
// reduction; here the band is split directly instead).
//
// Tree: leaves are diagonal blocks of T (size b = a multiple of ell, <= 64),
// solved by Jacobi.  Two adjacent nodes L, R are coupled only by the ell x ell
// block B = T[first rows of R, last rows of L]; with B = U diag(sigma) V^T,
//     T = diag(T_L, T_R) + sum_i sigma_i (w+ w+^T - w- w-^T),
//     w+- = (E_a v_i +- E_b u_i)/sqrt(2),
// i.e. 2*ell symmetric rank-one updates of signs +-sigma_i, and the children
// are never modified (their decompositions stay valid as T grows).  Each
// update of D + rho z z^T (in the current eigenbasis) is done as in Cuppen's
// method with the deflation of Dongarra-Sorensen, a safeguarded rational
// secular-equation iteration, and the Gu-Eisenstat recomputation of z so the
// eigenvectors are numerically orthogonal.  Only 4*ell rows of the eigenvector
// matrix are carried through a merge: the first/last ell rows of each child
// (to form z and to keep the merged node's first/last rows).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "dc.hpp"

namespace lyap {

constexpr int kMaxL = 16;              // ell <= 16
constexpr int kRows = 4 * kMaxL;       // tracked rows per merge (4*ell)
constexpr double kEps = 2.220446049250313e-16;

struct DcMerge {
  int a;    // first row of the merged node
  int K1;   // size of the left child
  int K;    // size of the merged node
  int pad;
};

struct DcScal {
  int Kn, Kd, sg, skip;
  double r;          // |rho| * ||z||^2 (normalised problem)
  double sigma[kMaxL];
  double U[kMaxL * kMaxL];  // column i = u_i (R side)
  double V[kMaxL * kMaxL];  // column i = v_i (L side)
};

// ------------------------------------------------------------------ leaves
// Leaves cover rows [r0 + i b, min(r0 + (i+1) b, k)).
__global__ void k_leaf_extract(const double* band, int ldb, int ell, int k, int b, int r0, double* A) {
  const int leaf = blockIdx.y;
  const int a0 = r0 + leaf * b;
  const int n = min(b, k - a0);
  double* M = A + (size_t)leaf * b * b;
  for (int e = threadIdx.x + blockIdx.x * blockDim.x; e < n * n; e += blockDim.x * gridDim.x) {
    const int i = e / n, j = e % n;
    const int d = i > j ? i - j : j - i;
    const int c = (i > j ? j : i) + a0;
    M[e] = d <= ell ? band[(size_t)c * ldb + d] : 0.0;
  }
}

__global__ void k_leaf_store(const double* Q, const double* lam, int b, int ell, int k, int r0, int ld, double* D,
                             double* F, double* L) {
  const int leaf = blockIdx.y;
  const int a0 = r0 + leaf * b;
  const int n = min(b, k - a0);
  const double* Ql = Q + (size_t)leaf * b * b;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    D[a0 + i] = lam[(size_t)leaf * b + i];
    for (int a = 0; a < ell; ++a) {
      F[(size_t)a * ld + a0 + i] = Ql[a * n + i];
      L[(size_t)a * ld + a0 + i] = Ql[(n - ell + a) * n + i];
    }
  }
}

// The root's eigenvalues and first / last ell eigenvector rows to the caller
// (internal stride ld, the caller's stride k).
__global__ void k_root_out(int k, int ell, int ld, const double* D, const double* F, const double* L, double* lam,
                           double* Fo, double* Lo) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < k; e += gridDim.x * blockDim.x) {
    lam[e] = D[e];
    for (int r = 0; r < ell; ++r) {
      Fo[(size_t)r * k + e] = F[(size_t)r * ld + e];
      Lo[(size_t)r * k + e] = L[(size_t)r * ld + e];
    }
  }
}

// ------------------------------------------------------------------ merge setup
// Builds the sorted eigenvalues of diag(T_L, T_R) and the 4*ell tracked rows
// [F_L 0; L_L 0; 0 F_R; 0 L_R] in that order.
__global__ void k_merge_setup(const DcMerge* md, DcScal* ms, const double* band, int ldb, int ell, int k,
                              const double* Dm, const double* Fm, const double* Lm, double* Dw, double* Rw) {
  const DcMerge g = md[blockIdx.y];
  const int a = g.a, K1 = g.K1, K2 = g.K - g.K1;
  const double* lamL = Dm + a;
  const double* lamR = Dm + a + K1;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < g.K; e += gridDim.x * blockDim.x) {
    int pos;
    const bool left = e < K1;
    const int i = left ? e : e - K1;
    const double v = left ? lamL[i] : lamR[i];
    if (left) {  // + number of right values < v
      int lo = 0, hi = K2;
      while (lo < hi) { int mid = (lo + hi) >> 1; if (lamR[mid] < v) lo = mid + 1; else hi = mid; }
      pos = i + lo;
    } else {     // + number of left values <= v
      int lo = 0, hi = K1;
      while (lo < hi) { int mid = (lo + hi) >> 1; if (lamL[mid] <= v) lo = mid + 1; else hi = mid; }
      pos = i + lo;
    }
    Dw[a + pos] = v;
    const int col = a + e;
    for (int r = 0; r < ell; ++r) {
      Rw[(size_t)r * k + a + pos] = left ? Fm[(size_t)r * k + col] : 0.0;
      Rw[(size_t)(ell + r) * k + a + pos] = left ? Lm[(size_t)r * k + col] : 0.0;
      Rw[(size_t)(2 * ell + r) * k + a + pos] = left ? 0.0 : Fm[(size_t)r * k + col];
      Rw[(size_t)(3 * ell + r) * k + a + pos] = left ? 0.0 : Lm[(size_t)r * k + col];
    }
  }
}

// SVD of every merge's coupling block (they depend on T only): one-sided
// Jacobi, one wave per merge of the whole tree, W and V in LDS.  Each sweep
// visits the column pairs in the parallel (round-robin) order, the disjoint
// pairs of a round together: lane k < ell/2 forms the pair's inner products
// over the rows (in row order) and its rotation, then the lanes apply the
// round's rotations row by row.  A sweep with no off-diagonal ratio above
// 2 eps ends it.  (One thread per merge with W in private memory and V
// updated in place in the output took 0.2 ms per launch.)
__global__ __launch_bounds__(64) void k_coupling_svd(const DcMerge* md, DcScal* ms, int nm, const double* band,
                                                     int ldb, int ell) {
  const int q = blockIdx.x;
  if (q >= nm) return;
  __shared__ double W[kMaxL * kMaxL], V[kMaxL * kMaxL];
  __shared__ double sc[kMaxL / 2], ss[kMaxL / 2], soff[kMaxL / 2];
  __shared__ int sp[kMaxL / 2], sq[kMaxL / 2];
  const DcMerge g = md[q];
  const int a = g.a, K1 = g.K1;
  const int t = threadIdx.x;
  // W[r][c] = T(a + K1 + r, a + K1 - ell + c), V = I
  for (int e = t; e < ell * ell; e += 64) {
    const int r = e / ell, c = e - r * ell;
    const int row = a + K1 + r, colT = a + K1 - ell + c;
    const int d = row - colT;
    W[e] = (d >= 0 && d <= ell) ? band[(size_t)colT * ldb + d] : 0.0;
    V[e] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  const int np = (ell + 1) & ~1;  // players (one dummy when ell is odd)
  const int rot = np - 1;
  const int half = np / 2;
  for (int sweep = 0; sweep < 60 && ell > 1; ++sweep) {
    double off = 0.0;
    for (int round = 0; round < rot; ++round) {
      if (t < half) {
        int p, qq;
        if (t == 0) { p = 0; qq = 1 + round; }
        else {
          p = round + t; if (p >= rot) p -= rot; p += 1;
          qq = round - t; if (qq < 0) qq += rot; qq += 1;
        }
        if (p > qq) { const int x = p; p = qq; qq = x; }
        double c = 1.0, sn = 0.0;
        if (qq < ell) {
          double al = 0, be = 0, ga = 0;
          for (int r = 0; r < ell; ++r) {
            const double wp = W[r * ell + p], wq = W[r * ell + qq];
            al += wp * wp;
            be += wq * wq;
            ga += wp * wq;
          }
          if (!(fabs(ga) <= 1e-300 || fabs(ga) <= kEps * sqrt(al * be))) {
            off = fmax(off, fabs(ga) / sqrt(al * be));
            const double zeta = (be - al) / (2.0 * ga);
            const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            c = 1.0 / sqrt(1.0 + tt * tt);
            sn = c * tt;
          }
        }
        sp[t] = p; sq[t] = qq; sc[t] = c; ss[t] = sn;
      }
      __syncthreads();
      for (int e = t; e < half * ell; e += 64) {
        const int k = e / ell, r = e - k * ell;
        const int p = sp[k], qq = sq[k];
        const double sn = ss[k];
        if (qq >= ell || sn == 0.0) continue;
        const double c = sc[k];
        const double wp = W[r * ell + p], wq = W[r * ell + qq];
        W[r * ell + p] = c * wp - sn * wq;
        W[r * ell + qq] = sn * wp + c * wq;
        const double vp = V[r * ell + p], vq = V[r * ell + qq];
        V[r * ell + p] = c * vp - sn * vq;
        V[r * ell + qq] = sn * vp + c * vq;
      }
      __syncthreads();
    }
    if (t < half) soff[t] = off;
    __syncthreads();
    double mo = 0.0;
    for (int k = 0; k < half; ++k) mo = fmax(mo, soff[k]);
    __syncthreads();
    if (mo <= 2 * kEps) break;  // the same value in every lane
  }
  DcScal& s = ms[q];
  for (int c = t; c < ell; c += 64) {
    double nn = 0;
    for (int r = 0; r < ell; ++r) nn += W[r * ell + c] * W[r * ell + c];
    nn = sqrt(nn);
    s.sigma[c] = nn;
    for (int r = 0; r < ell; ++r) s.U[r * ell + c] = nn > 0 ? W[r * ell + c] / nn : (r == c ? 1.0 : 0.0);
  }
  for (int e = t; e < ell * ell; e += 64) s.V[e] = V[e];
}


// Deflation, one 1024-thread workgroup per merge.  Working index w runs over
// the columns in ascending order of sg*D (sg = sign(rho)): column c(w) = w
// (sg > 0) or K-1-w.  Entries with negligible z deflate directly; the others
// are compacted in order (prefix sums); an adjacent pair that is close enough
// for a Givens rotation to zero one z component deflates too.  The rotation
// test of a pair depends on the previous pair's outcome, so when any pair
// qualifies one thread walks the compacted candidate list in order.
constexpr int kDefThreads = 1024;
constexpr int kDefLds = 2048;  // candidates staged in LDS for the run-by-run walk

__device__ __forceinline__ int block_excl_scan(int v, int* sh, int* total) {
  // Hillis-Steele over kDefThreads values in shared memory
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kDefThreads; off <<= 1) {
    const int x = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  const int incl = sh[t];
  if (total) *total = sh[kDefThreads - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kDefThreads) void k_deflate(const DcMerge* md, DcScal* ms, int ell, int k, int upd,
                                                         double* Dw, double* Rw, double* z, double* Dn,
                                                         double* zn, int* nd, int* defl, double* defv, int* sml,
                                                         double* smv, int* rdl, double* rdv) {
  __shared__ int sh[kDefThreads];
  __shared__ double redd[kDefThreads / 64 * 2];
  __shared__ int any_trig, s_Kc, s_Ks, s_Kn, s_Nr;
  __shared__ int s_nd[kDefLds], s_tr[kDefLds];
  __shared__ double s_dn[kDefLds], s_zn[kDefLds];
  const DcMerge g = md[blockIdx.x];
  DcScal& s = ms[blockIdx.x];
  const int a = g.a, K = g.K;
  const int i = upd >> 1;
  const int sg = (upd & 1) ? -1 : 1;
  const int t = threadIdx.x;
  const int chunk = (K + kDefThreads - 1) / kDefThreads;
  const int w0 = min(t * chunk, K), w1 = min(w0 + chunk, K);
  auto col = [&](int w) { return sg > 0 ? w : K - 1 - w; };
  // ---- z = (R_a^T v_i + sg R_b^T u_i) / sqrt(2) of update 2i + (sg < 0),
  // each thread for its own columns, visible to the workgroup after the barrier
  {
    const double zs = sg > 0 ? 1.0 : -1.0;
    for (int w = w0; w < w1; ++w) {
      const int cl = a + col(w);
      double zx = 0.0, zy = 0.0;
      for (int r = 0; r < ell; ++r) {
        zx = fma(Rw[(size_t)(ell + r) * k + cl], s.V[r * ell + i], zx);
        zy = fma(Rw[(size_t)(2 * ell + r) * k + cl], s.U[r * ell + i], zy);
      }
      z[cl] = (zx + zs * zy) * 0.70710678118654752440;
    }
    __syncthreads();
  }
  // ---- norms
  double nz2 = 0.0, dmax = 0.0;
  for (int w = w0; w < w1; ++w) {
    const int c = col(w);
    nz2 += z[a + c] * z[a + c];
    dmax = fmax(dmax, fabs(Dw[a + c]));
  }
  {
    const int lane = t & 63, wave = t >> 6;
    double v = wave_sum(nz2);
    const double m = wave_max(dmax);
    if (lane == 0) { redd[wave] = v; redd[kDefThreads / 64 + wave] = m; }
    __syncthreads();
    if (t == 0) {
      double sv = 0.0, mv = 0.0;
      for (int w = 0; w < kDefThreads / 64; ++w) { sv += redd[w]; mv = fmax(mv, redd[kDefThreads / 64 + w]); }
      redd[0] = sv;
      redd[1] = mv;
    }
    __syncthreads();
    nz2 = redd[0];
    dmax = redd[1];
  }
  const double r0 = s.sigma[i];
  if (t == 0) s.sg = sg;
  if (!(r0 > 0.0) || !(nz2 > 0.0)) {  // nothing to do: every entry deflates
    for (int w = w0; w < w1; ++w) {
      defl[a + w] = w;
      defv[a + w] = sg * Dw[a + col(w)];
    }
    if (t == 0) { s.skip = 1; s.Kn = 0; s.Kd = K; s.r = 0.0; }
    return;
  }
  const double r = r0 * nz2;
  const double inv = 1.0 / sqrt(nz2);
  const double tol = 8.0 * kEps * fmax(dmax, r);
  // ---- compaction of candidates (non-small z) and of small entries
  int cnt = 0;
  for (int w = w0; w < w1; ++w) cnt += (r * fabs(z[a + col(w)] * inv) > tol);
  int Kc = 0, Ks = 0;
  const int bc = block_excl_scan(cnt, sh, &Kc);
  const int bs = block_excl_scan((w1 - w0) - cnt, sh, &Ks);
  {
    int ic = bc, is = bs;
    for (int w = w0; w < w1; ++w) {
      const int c = col(w);
      const double zw = z[a + c] * inv;
      const double dw = sg * Dw[a + c];
      if (r * fabs(zw) > tol) { nd[a + ic] = w; Dn[a + ic] = dw; zn[a + ic] = zw; ++ic; }
      else { sml[a + is] = w; smv[a + is] = dw; ++is; }
    }
  }
  if (t == 0) any_trig = 0;
  __syncthreads();
  // ---- adjacent-pair rotation test with the original values
  for (int q = 1 + t; q < Kc; q += kDefThreads) {
    const double zp = zn[a + q - 1], zw = zn[a + q];
    const double tt = hypot(zw, zp);
    if (fabs((Dn[a + q] - Dn[a + q - 1]) * (zw / tt) * (zp / tt)) <= tol) any_trig = 1;
  }
  __syncthreads();
  if (!any_trig) {
    for (int e = t; e < Ks; e += kDefThreads) { defl[a + e] = sml[a + e]; defv[a + e] = smv[a + e]; }
    if (t == 0) { s.skip = 0; s.Kn = Kc; s.Kd = Ks; s.r = r; }
    return;
  }
  // ---- walk over the candidates (rotations depend on the order)
  if (Kc <= kDefLds) {
    // The walk's state only differs from the candidates' own values inside a
    // run of consecutive rotations, and a run can only start at a pair that
    // passes the test with the original values.  So one wave visits just the
    // runs (from the list of such pairs) with the candidates staged in LDS,
    // every lane taking the same decisions and rotating its own rows of R;
    // the survivors are then compacted by the whole workgroup.  Rotations,
    // values and order are those of the plain walk below.
    for (int q = t; q < Kc; q += kDefThreads) {
      s_nd[q] = nd[a + q];
      s_dn[q] = Dn[a + q];
      s_zn[q] = zn[a + q];
    }
    __syncthreads();
    const int qc = (Kc + kDefThreads - 1) / kDefThreads;
    const int q0 = min(t * qc, Kc), q1 = min(q0 + qc, Kc);
    auto pair_rot = [&](int q) {
      const double zp = s_zn[q - 1], zw = s_zn[q];
      const double tt = hypot(zw, zp);
      return fabs((s_dn[q] - s_dn[q - 1]) * (zw / tt) * (zp / tt)) <= tol;
    };
    int ntr = 0;
    for (int q = max(q0, 1); q < q1; ++q) ntr += pair_rot(q) ? 1 : 0;
    int T = 0;
    {
      int o = block_excl_scan(ntr, sh, &T);
      for (int q = max(q0, 1); q < q1; ++q)
        if (pair_rot(q)) s_tr[o++] = q;
    }
    __syncthreads();
    if (t < 64) {
      const int nr = 4 * ell;
      int last = -1, Nr = 0;
      for (int x = 0; x < T; ++x) {
        const int qs = s_tr[x];
        if (qs <= last) continue;
        int p = qs - 1;
        int pw = s_nd[p];
        double pz = s_zn[p], pd = s_dn[p];
        int q = qs;
        for (; q < Kc; ++q) {
          const int w = s_nd[q];
          const double zw = s_zn[q], dw = s_dn[q];
          const double tt = hypot(zw, pz);
          const double cc = zw / tt, ss = pz / tt;
          if (!(fabs((dw - pd) * cc * ss) <= tol)) break;
          const int cp = col(pw), cw = col(w);
          for (int row = t; row < nr; row += 64) {
            double* R = Rw + (size_t)row * k + a;
            const double qp = R[cp], qw = R[cw];
            R[cp] = cc * qp - ss * qw;
            R[cw] = ss * qp + cc * qw;
          }
          if (t == 0) {
            rdl[a + Nr] = pw;
            rdv[a + Nr] = pd * cc * cc + dw * ss * ss;
          }
          ++Nr;
          s_nd[p] = -1;  // rotated out
          p = q;
          pw = w;
          pz = tt;
          pd = pd * ss * ss + dw * cc * cc;
        }
        s_zn[p] = pz;  // the run's survivor
        s_dn[p] = pd;
        last = q;
      }
      if (t == 0) s_Nr = Nr;
    }
    __syncthreads();
    int kept = 0;
    for (int q = q0; q < q1; ++q) kept += s_nd[q] >= 0 ? 1 : 0;
    int Kn = 0;
    {
      int o = block_excl_scan(kept, sh, &Kn);
      for (int q = q0; q < q1; ++q)
        if (s_nd[q] >= 0) {
          nd[a + o] = s_nd[q];
          Dn[a + o] = s_dn[q];
          zn[a + o] = s_zn[q];
          ++o;
        }
    }
    if (t == 0) {
      const int Nr = s_Nr;
      for (int x = 1; x < Nr; ++x) {  // rotated-out values are nearly sorted
        const double v = rdv[a + x];
        const int iw = rdl[a + x];
        int y = x - 1;
        while (y >= 0 && rdv[a + y] > v) { rdv[a + y + 1] = rdv[a + y]; rdl[a + y + 1] = rdl[a + y]; --y; }
        rdv[a + y + 1] = v;
        rdl[a + y + 1] = iw;
      }
      s_Kn = Kn;
    }
  } else if (t == 0) {
    const int nr = 4 * ell;
    int p = -1, Kn = 0, Nr = 0;
    double pz = 0.0, pd = 0.0;
    for (int q = 0; q < Kc; ++q) {
      const int w = nd[a + q];
      const double zw = zn[a + q], dw = Dn[a + q];
      if (p < 0) { p = w; pz = zw; pd = dw; continue; }
      const double tt = hypot(zw, pz);
      const double cc = zw / tt, ss = pz / tt;
      if (fabs((dw - pd) * cc * ss) <= tol) {
        const int cp = col(p), cw = col(w);
        for (int row = 0; row < nr; ++row) {
          double* R = Rw + (size_t)row * k + a;
          const double qp = R[cp], qw = R[cw];
          R[cp] = cc * qp - ss * qw;
          R[cw] = ss * qp + cc * qw;
        }
        rdl[a + Nr] = p;
        rdv[a + Nr] = pd * cc * cc + dw * ss * ss;
        ++Nr;
        p = w; pz = tt; pd = pd * ss * ss + dw * cc * cc;
      } else {
        nd[a + Kn] = p; Dn[a + Kn] = pd; zn[a + Kn] = pz; ++Kn;  // in place: Kn <= q
        p = w; pz = zw; pd = dw;
      }
    }
    if (p >= 0) { nd[a + Kn] = p; Dn[a + Kn] = pd; zn[a + Kn] = pz; ++Kn; }
    for (int x = 1; x < Nr; ++x) {  // rotated-out values are nearly sorted
      const double v = rdv[a + x];
      const int iw = rdl[a + x];
      int y = x - 1;
      while (y >= 0 && rdv[a + y] > v) { rdv[a + y + 1] = rdv[a + y]; rdl[a + y + 1] = rdl[a + y]; --y; }
      rdv[a + y + 1] = v;
      rdl[a + y + 1] = iw;
    }
    s_Kn = Kn;
    s_Nr = Nr;
  }
  __syncthreads();
  const int Nr = s_Nr;
  // ---- merge the two sorted deflated lists (small-z first on ties)
  for (int e = t; e < Ks + Nr; e += kDefThreads) {
    if (e < Ks) {
      const double v = smv[a + e];
      int lo = 0, hi = Nr;
      while (lo < hi) { int mid = (lo + hi) >> 1; if (rdv[a + mid] < v) lo = mid + 1; else hi = mid; }
      defl[a + e + lo] = sml[a + e];
      defv[a + e + lo] = v;
    } else {
      const int x = e - Ks;
      const double v = rdv[a + x];
      int lo = 0, hi = Ks;
      while (lo < hi) { int mid = (lo + hi) >> 1; if (smv[a + mid] <= v) lo = mid + 1; else hi = mid; }
      defl[a + x + lo] = rdl[a + x];
      defv[a + x + lo] = v;
    }
  }
  if (t == 0) { s.skip = 0; s.Kn = s_Kn; s.Kd = Ks + Nr; s.r = r; }
}

// sum z_i^2 / (d_i - dO - t) and sum z_i^2 / (d_i - dO - t)^2 over i = i0, i0 + 64,
// ... < i1 (one lane's share), accumulated in that order; four terms per pass
// so that their loads are in flight together.
__device__ __forceinline__ void secular_terms(const double* d, const double* zz, double dO, double t, int i0, int i1,
                                              double& s1, double& s2) {
  int i = i0;
  for (; i + 192 < i1; i += 256) {
    double zv[4], dv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      zv[u] = zz[i + 64 * u];
      dv[u] = d[i + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double q = zv[u] / ((dv[u] - dO) - t);
      s1 = fma(zv[u], q, s1);
      s2 = fma(q, q, s2);
    }
  }
  for (; i < i1; i += 64) {
    const double q = zz[i] / ((d[i] - dO) - t);
    s1 = fma(zz[i], q, s1);
    s2 = fma(q, q, s2);
  }
}

// Root of a x^2 + b x + c0 = 0 in (L, R) when there is one (else the other
// root), from the cancellation-free pair q / a and c0 / q.
__device__ __forceinline__ double quad_root_in(double a, double b, double c0, double L, double R) {
  if (a == 0.0) return -c0 / b;
  const double sq = sqrt(fmax(b * b - 4.0 * a * c0, 0.0));
  const double q = -0.5 * (b >= 0.0 ? b + sq : b - sq);
  const double x1 = q / a;
  const double x2 = q != 0.0 ? c0 / q : x1;
  return (x1 > L && x1 < R) ? x1 : x2;
}

// Secular equation 1/r + sum_i z_i^2/(d_i - lambda) = 0.  Root j lies in
// (d_j, d_{j+1}) (last: (d_{K-1}, d_{K-1} + r||z||^2)); it is stored as the
// nearer pole index o_j and the offset tau_j = lambda_j - d_{o_j} so that every
// difference d_i - lambda_j is formed accurately.
//
// One iteration given the sums psi = sum_{i<=j} z_i^2/(d_i - lambda), phi (the
// rest) and their derivatives at t = lambda - d_o: updates the bracket
// (lo, hi) and t; returns true once t has converged.
__device__ __forceinline__ bool secular_step(double ir, double psi, double phi, double dpsi, double dphi, bool last,
                                             bool o_is_j, double Dj, double Dj1, int Kn, double& lo, double& hi,
                                             double& t) {
  const double f = ir + psi + phi;
  if (f < 0.0) lo = fmax(lo, t); else hi = fmin(hi, t);
  const double err = 8.0 * kEps * (ir + fabs(psi) + fabs(phi) + fabs(t) * (dpsi + dphi));
  if (fabs(f) <= err || (hi - lo) <= 4.0 * kEps * fmax(fabs(lo), fabs(hi))) return true;
  const double dlj = Dj - t;
  const double b1 = dpsi * dlj * dlj;
  const double a1 = psi - b1 / dlj;
  double tn;
  if (!last) {
    const double dlj1 = Dj1 - t;
    const double b2 = dphi * dlj1 * dlj1;
    const double a2 = phi - b2 / dlj1;
    const double c = ir + a1 + a2;
    const double dd = Dj1 - Dj;
    // root of c + b1/(Dj - x) + b2/(Dj1 - x), solved for its distance to the
    // origin pole (Dj or Dj1 is 0) so that a root next to that pole keeps
    // its relative accuracy: u = Dj - x in (-dd, 0) or w = Dj1 - x in (0, dd)
    if (o_is_j) tn = Dj - quad_root_in(c, c * dd + b1 + b2, b1 * dd, -dd, 0.0);
    else tn = Dj1 - quad_root_in(c, b1 + b2 - c * dd, -b2 * dd, 0.0, dd);
  } else {
    const double c = ir + a1;
    tn = c != 0.0 ? Dj + b1 / c : 0.5 * (lo + hi);
  }
  // The model matches f and f' at t and increases between its poles, so a
  // root of it on the side of t that the sign of f(t) points away from (or
  // t itself) comes either from f(t) being at the rounding level of the sum
  // (bound K eps sum|terms|: converged) or from a model without a root in
  // the bracket (bisect).
  if (f < 0.0 ? tn <= t : tn >= t) {
    if (fabs(f) <= kEps * Kn * (ir + fabs(psi) + fabs(phi))) return true;
    tn = 0.5 * (lo + hi);
  } else if (!(tn > lo && tn < hi)) {
    tn = 0.5 * (lo + hi);
  }
  t = tn;
  return false;
}

// Merges too large for LDS: one wave per root, the sums stream d and z from
// memory (L2) every iteration.
__global__ __launch_bounds__(256) void k_secular(const DcMerge* md, const DcScal* ms, const double* Dn,
                                                 const double* zn, int* orig, double* tau, double* lamn) {
  const DcMerge g = md[blockIdx.y];
  const DcScal& s = ms[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int Kn = s.Kn;
  if (j >= Kn) return;
  const double* d = Dn + g.a;
  const double* zz = zn + g.a;
  const double r = s.r;
  const double ir = 1.0 / r;
  const bool last = (j == Kn - 1);
  int o;
  double lo, hi;
  if (!last) {
    const double delta = d[j + 1] - d[j];
    const double mid = d[j] + 0.5 * delta;
    double f = 0.0;
    for (int i = lane; i < Kn; i += 64) f += zz[i] * zz[i] / (d[i] - mid);
    f = wave_sum(f) + ir;
    if (f >= 0.0) { o = j; lo = 0.0; hi = 0.5 * delta; }
    else { o = j + 1; lo = -0.5 * delta; hi = 0.0; }
  } else {
    double z2 = 0.0;
    for (int i = lane; i < Kn; i += 64) z2 += zz[i] * zz[i];
    z2 = wave_sum(z2);
    o = j; lo = 0.0; hi = r * z2;
  }
  const double dO = d[o];
  double t = 0.5 * (lo + hi);
  const double Dj = d[j] - dO;
  const double Dj1 = last ? 0.0 : d[j + 1] - dO;
  for (int it = 0; it < 120; ++it) {
    // with q = z_i / (d_i - lambda): z_i^2 / (d_i - lambda) = z_i q and its
    // derivative z_i^2 / (d_i - lambda)^2 = q^2 (one division per term)
    double psi = 0, phi = 0, dpsi = 0, dphi = 0;
    secular_terms(d, zz, dO, t, lane, j + 1, psi, dpsi);
    secular_terms(d, zz, dO, t, j + 1 + lane, Kn, phi, dphi);
    psi = wave_sum(psi); phi = wave_sum(phi); dpsi = wave_sum(dpsi); dphi = wave_sum(dphi);
    if (secular_step(ir, psi, phi, dpsi, dphi, last, o == j, Dj, Dj1, Kn, lo, hi, t)) break;
  }
  if (lane == 0) {
    orig[g.a + j] = o;
    tau[g.a + j] = t;
    lamn[g.a + j] = dO + t;
  }
}

// Large merges whose poles fit in LDS (Kn <= kSecLdsMax): a 1024-thread
// workgroup stages d and z once and its 16 waves (one root each) read them
// from LDS at every iteration instead of from L2.
constexpr int kSecLdsMax = 9216;  // 2 * 9216 doubles = 144 KB of LDS

__global__ __launch_bounds__(1024) void k_secular_lds(const DcMerge* md, const DcScal* ms, const double* Dn,
                                                      const double* zn, int* orig, double* tau, double* lamn) {
  extern __shared__ double sm[];
  const DcMerge g = md[blockIdx.y];
  const DcScal& s = ms[blockIdx.y];
  const int Kn = s.Kn;
  if (blockIdx.x * 16 >= Kn) return;  // the whole workgroup
  double* sd = sm;
  double* sz = sm + Kn;
  for (int i = threadIdx.x; i < Kn; i += 1024) {
    sd[i] = Dn[g.a + i];
    sz[i] = zn[g.a + i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 16 + (threadIdx.x >> 6);
  if (j >= Kn) return;
  const double r = s.r;
  const double ir = 1.0 / r;
  const bool last = (j == Kn - 1);
  int o;
  double lo, hi;
  if (!last) {
    const double delta = sd[j + 1] - sd[j];
    const double mid = sd[j] + 0.5 * delta;
    double f = 0.0;
    for (int i = lane; i < Kn; i += 64) f += sz[i] * sz[i] / (sd[i] - mid);
    f = wave_sum(f) + ir;
    if (f >= 0.0) { o = j; lo = 0.0; hi = 0.5 * delta; }
    else { o = j + 1; lo = -0.5 * delta; hi = 0.0; }
  } else {
    double z2 = 0.0;
    for (int i = lane; i < Kn; i += 64) z2 += sz[i] * sz[i];
    z2 = wave_sum(z2);
    o = j; lo = 0.0; hi = r * z2;
  }
  const double dO = sd[o];
  double t = 0.5 * (lo + hi);
  const double Dj = sd[j] - dO;
  const double Dj1 = last ? 0.0 : sd[j + 1] - dO;
  for (int it = 0; it < 120; ++it) {
    double psi = 0, phi = 0, dpsi = 0, dphi = 0;
    for (int i = lane; i <= j; i += 64) {
      const double q = sz[i] / ((sd[i] - dO) - t);
      psi = fma(sz[i], q, psi);
      dpsi = fma(q, q, dpsi);
    }
    for (int i = j + 1 + lane; i < Kn; i += 64) {
      const double q = sz[i] / ((sd[i] - dO) - t);
      phi = fma(sz[i], q, phi);
      dphi = fma(q, q, dphi);
    }
    psi = wave_sum(psi); phi = wave_sum(phi); dpsi = wave_sum(dpsi); dphi = wave_sum(dphi);
    if (secular_step(ir, psi, phi, dpsi, dphi, last, o == j, Dj, Dj1, Kn, lo, hi, t)) break;
  }
  if (lane == 0) {
    orig[g.a + j] = o;
    tau[g.a + j] = t;
    lamn[g.a + j] = dO + t;
  }
}

// Merges with Kn <= G * NR: a group of G lanes per root (64 / G roots per
// wave), each lane holding NR of the root's poles (i = lane-in-group + G u) in
// registers for every iteration; the sums are group butterflies.  Every lane
// takes part in every sum (a group whose root has converged keeps its state),
// and the wave stops when all of its groups have.
template <int G, int NR>
__global__ __launch_bounds__(256) void k_secular_reg(const DcMerge* md, const DcScal* ms, const double* Dn,
                                                     const double* zn, int* orig, double* tau, double* lamn) {
  constexpr int RPW = 64 / G;
  const DcMerge g = md[blockIdx.y];
  const DcScal& s = ms[blockIdx.y];
  const int Kn = s.Kn;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wave * RPW >= Kn) return;
  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);
  const int jr = wave * RPW + lane / G;
  const bool valid = jr < Kn;
  const int j = valid ? jr : Kn - 1;  // idle groups repeat the last root and store nothing
  const double* d = Dn + g.a;
  const double* zz = zn + g.a;
  const double r = s.r;
  const double ir = 1.0 / r;
  const bool last = (j == Kn - 1);
  double zr[NR], dr[NR];
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    const int i = gl + G * u;
    zr[u] = i < Kn ? zz[i] : 0.0;
    dr[u] = i < Kn ? d[i] : 0.0;
  }
  // f at the midpoint of (d_j, d_{j+1}) and ||z||^2 (the last root's bracket),
  // both formed by every group
  const double dj = d[j];
  const double delta = last ? 0.0 : d[j + 1] - dj;
  const double mid = dj + 0.5 * delta;
  double fm = 0.0, z2 = 0.0;
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    const bool in = gl + G * u < Kn;
    fm += in ? zr[u] * zr[u] / (dr[u] - mid) : 0.0;
    z2 += zr[u] * zr[u];
  }
  fm = group_sum<G>(fm) + ir;
  z2 = group_sum<G>(z2);
  int o;
  double lo, hi;
  if (last) { o = j; lo = 0.0; hi = r * z2; }
  else if (fm >= 0.0) { o = j; lo = 0.0; hi = 0.5 * delta; }
  else { o = j + 1; lo = -0.5 * delta; hi = 0.0; }
  const double dO = d[o];
  double t = 0.5 * (lo + hi);
  const double Dj = dj - dO;
  const double Dj1 = last ? 0.0 : d[j + 1] - dO;
  double er[NR];
#pragma unroll
  for (int u = 0; u < NR; ++u) er[u] = gl + G * u < Kn ? dr[u] - dO : 1e300;
  bool done = !valid;
  for (int it = 0; it < 120; ++it) {
    double psi = 0, phi = 0, dpsi = 0, dphi = 0;
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      const double q = zr[u] / (er[u] - t);
      if (gl + G * u <= j) {
        psi = fma(zr[u], q, psi);
        dpsi = fma(q, q, dpsi);
      } else {
        phi = fma(zr[u], q, phi);
        dphi = fma(q, q, dphi);
      }
    }
    psi = group_sum<G>(psi); phi = group_sum<G>(phi); dpsi = group_sum<G>(dpsi); dphi = group_sum<G>(dphi);
    if (!done) done = secular_step(ir, psi, phi, dpsi, dphi, last, o == j, Dj, Dj1, Kn, lo, hi, t);
    if (__ballot(!done) == 0) break;
  }
  if (valid && gl == 0) {
    orig[g.a + j] = o;
    tau[g.a + j] = t;
    lamn[g.a + j] = dO + t;
  }
}

void launch_secular(int Kmax, int nm, const DcMerge* md, const DcScal* ms, const double* Dn, const double* zn,
                    int* orig, double* tau, double* lamn, hipStream_t st) {
  // roots per 256-thread block: 4 * 64 / G
  auto grid = [&](int G) { return dim3((Kmax + 4 * (64 / G) - 1) / (4 * (64 / G)), nm); };
  if (Kmax <= 64)
    hipLaunchKernelGGL((k_secular_reg<8, 8>), grid(8), dim3(256), 0, st, md, ms, Dn, zn, orig, tau, lamn);
  else if (Kmax <= 128)
    hipLaunchKernelGGL((k_secular_reg<16, 8>), grid(16), dim3(256), 0, st, md, ms, Dn, zn, orig, tau, lamn);
  else if (Kmax <= 256)
    hipLaunchKernelGGL((k_secular_reg<32, 8>), grid(32), dim3(256), 0, st, md, ms, Dn, zn, orig, tau, lamn);
  else if (Kmax <= 512)
    hipLaunchKernelGGL((k_secular_reg<64, 8>), grid(64), dim3(256), 0, st, md, ms, Dn, zn, orig, tau, lamn);
  else if (Kmax <= 1024)
    hipLaunchKernelGGL((k_secular_reg<64, 16>), grid(64), dim3(256), 0, st, md, ms, Dn, zn, orig, tau, lamn);
  else if (Kmax <= kSecLdsMax) {
    static bool attr = false;  // more than the default 64 KB of dynamic LDS
    if (!attr) {
      LYAP_HIP(hipFuncSetAttribute((const void*)k_secular_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   2 * kSecLdsMax * (int)sizeof(double)));
      attr = true;
    }
    hipLaunchKernelGGL(k_secular_lds, dim3((Kmax + 15) / 16, nm), dim3(1024), 2 * (size_t)Kmax * sizeof(double), st,
                       md, ms, Dn, zn, orig, tau, lamn);
  } else {
    hipLaunchKernelGGL(k_secular, grid(64), dim3(256), 0, st, md, ms, Dn, zn, orig, tau, lamn);
  }
}

// Gu-Eisenstat: r zhat_i^2 = prod_j (lambda_j - d_i) / prod_{j != i} (d_j - d_i); one wave per i.
// The wave also gathers the tracked rows of candidate i, Rt[i][r] = Rw[r][c(nd_i)]
// (contiguous per candidate, zero-padded to npad rows: the layout k_vec reads).
__global__ __launch_bounds__(256) void k_zhat(const DcMerge* md, const DcScal* ms, int nr, int npad, int k,
                                              const double* Rw,
                                              const int* nd, const double* Dn, const double* zn, const int* orig,
                                              const double* tau, double* zh, double* Rt) {
  const DcMerge g = md[blockIdx.y];
  const DcScal& s = ms[blockIdx.y];
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int Kn = s.Kn;
  if (i >= Kn) return;
  if (lane < npad) {
    const int w = nd[g.a + i];
    const int c = s.sg > 0 ? w : g.K - 1 - w;
    Rt[(size_t)(g.a + i) * npad + lane] = lane < nr ? Rw[(size_t)lane * k + g.a + c] : 0.0;
  }
  const double* d = Dn + g.a;
  const int* og = orig + g.a;
  const double* tt = tau + g.a;
  const double di = d[i];
  double prod = 1.0;
  for (int j = lane; j < Kn; j += 64) {
    const double num = (d[og[j]] - di) + tt[j];  // lambda_j - d_i
    prod *= (j == i) ? num : num / (d[j] - di);
  }
  prod = wave_prod(prod);
  if (lane == 0) {
    const double v = sqrt(fmax(prod, 0.0) / s.r);
    zh[g.a + i] = zn[g.a + i] >= 0.0 ? v : -v;
  }
}

// Eigenvector j of D + r z z^T is zhat ./ (d - lambda_j), normalised; the
// tracked rows become Rows(:, nd) * u_j.  Lane = root j (64 roots per wave),
// wave = one of nsp slices of the candidates i; the candidate data (d_i,
// zhat_i, Rt[i][:]) is the same for every lane, so each wave streams it once
// for 64 roots.  Per slice sp, rows r < nr and (r = nr) the squared norm go to
// part[(sp (nr+1) + r) k + a + j]; k_vec_sum adds the slices up.
template <int NRP>
__global__ __launch_bounds__(256) void k_vec(const DcMerge* __restrict__ md, const DcScal* __restrict__ ms, int nr,
                                             int k, int nsp, const double* __restrict__ Rt,
                                             const double* __restrict__ Dn, const int* __restrict__ orig,
                                             const double* __restrict__ tau, const double* __restrict__ zh,
                                             double* __restrict__ part) {
  const DcMerge g = md[blockIdx.y];
  const int Kn = ms[blockIdx.y].Kn;
  const int nsp4 = nsp >> 2;
  const int chunk = blockIdx.x / nsp4;
  const int sp = (blockIdx.x % nsp4) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (chunk * 64 >= Kn) return;
  const int lane = threadIdx.x & 63;
  const int jr = chunk * 64 + lane;
  const int j = min(jr, Kn - 1);
  const double* d = Dn + g.a;
  const double dO = d[orig[g.a + j]];
  const double tj = tau[g.a + j];
  const int span = (Kn + nsp - 1) / nsp;
  const int i0 = min(Kn, sp * span), i1 = min(Kn, i0 + span);
  double acc[NRP];
#pragma unroll
  for (int r = 0; r < NRP; ++r) acc[r] = 0.0;
  double nn = 0.0;
#pragma unroll 2
  for (int i = i0; i < i1; ++i) {
    const double u = zh[g.a + i] / ((d[i] - dO) - tj);
    nn = fma(u, u, nn);
    const double* R = Rt + (size_t)(g.a + i) * NRP;  // rows >= nr are zero
#pragma unroll
    for (int r = 0; r < NRP; ++r) acc[r] = fma(R[r], u, acc[r]);
  }
  if (jr < Kn) {
    double* P = part + (size_t)sp * (nr + 1) * k + g.a + jr;
#pragma unroll
    for (int r = 0; r < NRP; ++r)
      if (r < nr) P[(size_t)r * k] = acc[r];
    P[(size_t)nr * k] = nn;
  }
}

constexpr int kMaxSplit = 16;

// NR[r][a + j] = sum over slices of part (rows r < nr), nrm[a + j] = the squared
// norm; one thread per (row, root).
__global__ void k_vec_sum(const DcMerge* md, const DcScal* ms, int nr, int k, int nsp, const double* part, double* NR,
                          double* nrm) {
  const DcMerge g = md[blockIdx.y];
  const int Kn = ms[blockIdx.y].Kn;
  const size_t ps = (size_t)(nr + 1) * k;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < (nr + 1) * Kn; e += gridDim.x * blockDim.x) {
    const int r = e / Kn, j = e - r * Kn;
    const double* P = part + (size_t)r * k + g.a + j;
    double v = 0.0;
    for (int sp = 0; sp < nsp; ++sp) v += P[sp * ps];
    if (r < nr) NR[(size_t)r * k + g.a + j] = v;
    else nrm[g.a + j] = v;
  }
}

inline int vec_pad(int nr) { return nr <= 8 ? 8 : nr <= 16 ? 16 : nr <= 32 ? 32 : 64; }

void launch_vec(dim3 grid, const DcMerge* md, const DcScal* ms, int nr, int k, int nsp, const double* Rt,
                const double* Dn, const int* orig, const double* tau, const double* zh, double* part,
                hipStream_t st) {
  if (nr <= 8)
    hipLaunchKernelGGL(k_vec<8>, grid, dim3(256), 0, st, md, ms, nr, k, nsp, Rt, Dn, orig, tau, zh, part);
  else if (nr <= 16)
    hipLaunchKernelGGL(k_vec<16>, grid, dim3(256), 0, st, md, ms, nr, k, nsp, Rt, Dn, orig, tau, zh, part);
  else if (nr <= 32)
    hipLaunchKernelGGL(k_vec<32>, grid, dim3(256), 0, st, md, ms, nr, k, nsp, Rt, Dn, orig, tau, zh, part);
  else
    hipLaunchKernelGGL(k_vec<64>, grid, dim3(256), 0, st, md, ms, nr, k, nsp, Rt, Dn, orig, tau, zh, part);
}

// New spectrum = deflated values U new roots, merged in ascending order (ties:
// deflated first), mapped back to the original orientation.
__global__ void k_assemble(const DcMerge* md, const DcScal* ms, int ell, int k, const double* Rin, const double* NR,
                           const double* nrm, const int* defl, const double* defv, const double* lamn, double* Dout,
                           double* Rout) {
  const DcMerge g = md[blockIdx.y];
  const DcScal& s = ms[blockIdx.y];
  const int a = g.a, K = g.K, Kn = s.Kn, Kd = s.Kd, sg = s.sg;
  const int nr = 4 * ell;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < K; e += gridDim.x * blockDim.x) {
    int pos;
    double v;
    if (e < Kd) {
      v = defv[a + e];
      int lo = 0, hi = Kn;
      while (lo < hi) { int mid = (lo + hi) >> 1; if (lamn[a + mid] < v) lo = mid + 1; else hi = mid; }
      pos = e + lo;
    } else {
      const int j = e - Kd;
      v = lamn[a + j];
      int lo = 0, hi = Kd;
      while (lo < hi) { int mid = (lo + hi) >> 1; if (defv[a + mid] <= v) lo = mid + 1; else hi = mid; }
      pos = j + lo;
    }
    const int P = sg > 0 ? pos : K - 1 - pos;
    Dout[a + P] = sg > 0 ? v : -v;
    if (e < Kd) {
      const int w = defl[a + e];
      const int c = sg > 0 ? w : K - 1 - w;
      for (int r = 0; r < nr; ++r) Rout[(size_t)r * k + a + P] = Rin[(size_t)r * k + a + c];
    } else {
      const int j = e - Kd;
      const double inv = 1.0 / sqrt(nrm[a + j]);
      for (int r = 0; r < nr; ++r) Rout[(size_t)r * k + a + P] = NR[(size_t)r * k + a + j] * inv;
    }
  }
}

__global__ void k_merge_finish(const DcMerge* md, int ell, int k, const double* Dw, const double* Rw, double* Dm,
                               double* Fm, double* Lm) {
  const DcMerge g = md[blockIdx.y];
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < g.K; e += gridDim.x * blockDim.x) {
    const int col = g.a + e;
    Dm[col] = Dw[col];
    for (int r = 0; r < ell; ++r) {
      Fm[(size_t)r * k + col] = Rw[(size_t)r * k + col];
      Lm[(size_t)r * k + col] = Rw[(size_t)(3 * ell + r) * k + col];
    }
  }
}

// ------------------------------------------------------------------ driver
struct DcWork::Impl {
  int ell;
  hipStream_t st;
  int cap = 0;
  int leaf = 32;
  DevBuf Da, Db, Ra, Rb, z, Dn, zn, nd, defl, defv, orig, tau, lamn, zh, Rt, part, NR, nrm, sml, smv, rdl, rdv;
  DevBuf leafA, leafQ, leafL, leafN;
  DevBuf md, ms;
  int md_cap = 0;
  // pinned staging of the leaf sizes and merge plan (a copy from pageable
  // memory would wait for the stream); reused once the previous run's copies
  // have executed
  HostBuf hleafN, hmd;
  hipEvent_t copied = nullptr;
  bool copy_pending = false;
  // node results (eigenvalues, first / last ell eigenvector rows), stride cap;
  // after a run, rows [0, kc) hold the root of the last band decomposed
  DevBuf Dres, Fres, Lres;
  int kc = 0;
  const double* cband = nullptr;
  int cldb = 0;

  void ensure(int k) {
    if (k <= cap) return;
    // geometric growth by 4 from 1024 rows: a reallocation frees the old
    // buffers (a free waits for the device) and drops the stored root
    int c = std::max({k, cap * 4, 1024});
    c = (c + 255) / 256 * 256;
    const size_t d = (size_t)c * sizeof(double), ii = (size_t)c * sizeof(int);
    Da.alloc(d); Db.alloc(d);
    Ra.alloc(d * 4 * ell); Rb.alloc(d * 4 * ell); Rt.alloc(d * vec_pad(4 * ell));
    part.alloc(d * (4 * ell + 1) * kMaxSplit);
    NR.alloc(d * 4 * ell);
    nrm.alloc(d);
    z.alloc(d); Dn.alloc(d); zn.alloc(d); defv.alloc(d); tau.alloc(d); lamn.alloc(d); zh.alloc(d);
    nd.alloc(ii); defl.alloc(ii); orig.alloc(ii); sml.alloc(ii); rdl.alloc(ii);
    smv.alloc(d); rdv.alloc(d);
    const int nl = (c + leaf - 1) / leaf;
    leafA.alloc((size_t)nl * leaf * leaf * sizeof(double));
    leafQ.alloc((size_t)nl * leaf * leaf * sizeof(double));
    leafL.alloc((size_t)nl * leaf * sizeof(double));
    leafN.alloc((size_t)nl * sizeof(int));
    Dres.alloc(d);
    Fres.alloc(d * ell);
    Lres.alloc(d * ell);
    kc = 0;  // the stored root is gone
    cap = c;
  }
};

DcWork::DcWork(int ell, hipStream_t st) : impl_(new Impl) {
  LYAP_REQUIRE(ell >= 1 && ell <= kMaxL, LYAP_E_UNSUPPORTED, "band eigensolver: ell=%d > %d", ell, kMaxL);
  impl_->ell = ell;
  impl_->st = st;
  // leaves of at least 16 rows, a multiple of ell: small dense Jacobi
  // problems (each leaf is one sequential wave) against a few more merge
  // levels (measured on the 64-problem batch: 8 rows 1.53 s, 16 rows 1.48 s,
  // 32 rows 1.67 s, 64 rows 2.89 s)
  int b = ell * std::max(1, 16 / ell);
  impl_->leaf = b;
}
DcWork::~DcWork() {
  if (impl_->copied) (void)hipEventDestroy(impl_->copied);
  delete impl_;
}

void DcWork::run(const double* band, int ldb, int k, double* lam, double* F, double* L) {
  Impl& w = *impl_;
  const int ell = w.ell;
  const int b = w.leaf;
  hipStream_t st = w.st;
  w.ensure(k);
  const int ld = w.cap;
  // T_k extends the band decomposed last (same rows 0..kc-1, which never change
  // once written): decompose only rows [kc, k) and merge that node with the
  // stored root of rows [0, kc) -- one merge at the top instead of the whole
  // tree below it.  Otherwise the whole tree.
  if (band == w.cband && ldb == w.cldb && k == w.kc) {  // decomposed already
    hipLaunchKernelGGL(k_root_out, dim3(std::min((k + 255) / 256, 1024)), dim3(256), 0, st, k, ell, ld,
                       w.Dres.as<double>(), w.Fres.as<double>(), w.Lres.as<double>(), lam, F, L);
    LYAP_LAUNCHED("dc root");
    return;
  }
  const bool grow = band == w.cband && ldb == w.cldb && w.kc >= ell && k - w.kc >= ell;
  const int r0 = grow ? w.kc : 0;
  // leaves of rows [r0, k)
  const int nl = (k - r0 + b - 1) / b;
  if (w.copy_pending) {
    LYAP_HIP(hipEventSynchronize(w.copied));
    w.copy_pending = false;
  }
  if (w.hleafN.bytes < nl * sizeof(int)) w.hleafN.alloc(std::max<size_t>(nl * sizeof(int), 4096));
  int* nlist = w.hleafN.as<int>();
  for (int i = 0; i < nl; ++i) nlist[i] = std::min(b, k - r0 - i * b);
  LYAP_HIP(hipMemcpyAsync(w.leafN.p, nlist, nl * sizeof(int), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_leaf_extract, dim3(4, nl), dim3(256), 0, st, band, ldb, ell, k, b, r0, w.leafA.as<double>());
  launch_jacobi(w.leafA.as<double>(), (int64_t)b * b, w.leafQ.as<double>(), (int64_t)b * b, w.leafL.as<double>(), b,
                w.leafN.as<int>(), b, nl, st);
  double* Dm = w.Dres.as<double>();
  double* Fm = w.Fres.as<double>();
  double* Lm = w.Lres.as<double>();
  hipLaunchKernelGGL(k_leaf_store, dim3(1, nl), dim3(64), 0, st, w.leafQ.as<double>(), w.leafL.as<double>(), b, ell,
                     k, r0, ld, Dm, Fm, Lm);
  LYAP_LAUNCHED("dc leaves");
  // the tree over [r0, k): merges of every level (offset, size), planned on the host
  std::vector<std::pair<int, int>> nodes;
  for (int i = 0; i < nl; ++i) nodes.emplace_back(r0 + i * b, nlist[i]);
  std::vector<DcMerge> all;
  std::vector<int> lvl_off, lvl_kmax;
  while (nodes.size() > 1) {
    std::vector<std::pair<int, int>> next;
    int Kmax = 0;
    lvl_off.push_back((int)all.size());
    for (size_t i = 0; i + 1 < nodes.size(); i += 2) {
      DcMerge g{nodes[i].first, nodes[i].second, nodes[i].second + nodes[i + 1].second, 0};
      all.push_back(g);
      next.emplace_back(g.a, g.K);
      Kmax = std::max(Kmax, g.K);
    }
    if (nodes.size() % 2) next.push_back(nodes.back());
    lvl_kmax.push_back(Kmax);
    nodes.swap(next);
  }
  if (grow) {  // the stored root [0, r0) with the new node [r0, k)
    lvl_off.push_back((int)all.size());
    all.push_back(DcMerge{0, r0, k, 0});
    lvl_kmax.push_back(k);
  }
  lvl_off.push_back((int)all.size());
  const int ntot = (int)all.size();
  if (ntot > w.md_cap) {
    w.md.alloc((size_t)ntot * sizeof(DcMerge));
    w.ms.alloc((size_t)ntot * sizeof(DcScal));
    w.md_cap = ntot;
  }
  if (ntot > 0) {
    if (w.hmd.bytes < ntot * sizeof(DcMerge)) w.hmd.alloc(std::max<size_t>(ntot * sizeof(DcMerge), 4096));
    std::memcpy(w.hmd.p, all.data(), ntot * sizeof(DcMerge));
    LYAP_HIP(hipMemcpyAsync(w.md.p, w.hmd.p, ntot * sizeof(DcMerge), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_coupling_svd, dim3(ntot), dim3(64), 0, st, w.md.as<DcMerge>(),
                       w.ms.as<DcScal>(), ntot, band, ldb, ell);
  }
  if (!w.copied) LYAP_HIP(hipEventCreateWithFlags(&w.copied, hipEventDisableTiming));
  LYAP_HIP(hipEventRecord(w.copied, st));
  w.copy_pending = true;
  for (size_t lv = 0; lv + 1 < lvl_off.size(); ++lv) {
    const int nm = lvl_off[lv + 1] - lvl_off[lv];
    const int Kmax = lvl_kmax[lv];
    const DcMerge* md = w.md.as<DcMerge>() + lvl_off[lv];
    DcScal* ms = w.ms.as<DcScal>() + lvl_off[lv];
    const int gx = std::min((Kmax + 255) / 256, 64);
    const int gw = (Kmax + 3) / 4;  // one wave per element, 4 waves per block
    // k_vec: 64 roots per wave, candidate slices so that a level has ~2048 waves
    const int nr = 4 * ell;
    const int nchunk = (Kmax + 63) / 64;
    int nsp = (2048 + nchunk * nm - 1) / (nchunk * nm);
    nsp = std::min(kMaxSplit, std::max(4, (nsp + 3) / 4 * 4));
    double* Dcur = w.Da.as<double>();
    double* Dnx = w.Db.as<double>();
    double* Rcur = w.Ra.as<double>();
    double* Rnx = w.Rb.as<double>();
    hipLaunchKernelGGL(k_merge_setup, dim3(gx, nm), dim3(256), 0, st, md, ms, band, ldb, ell, ld, Dm, Fm, Lm, Dcur,
                       Rcur);
    for (int u = 0; u < 2 * ell; ++u) {
      hipLaunchKernelGGL(k_deflate, dim3(nm), dim3(kDefThreads), 0, st, md, ms, ell, ld, u, Dcur, Rcur,
                         w.z.as<double>(), w.Dn.as<double>(), w.zn.as<double>(), w.nd.as<int>(), w.defl.as<int>(),
                         w.defv.as<double>(), w.sml.as<int>(), w.smv.as<double>(), w.rdl.as<int>(),
                         w.rdv.as<double>());
      launch_secular(Kmax, nm, md, ms, w.Dn.as<double>(), w.zn.as<double>(), w.orig.as<int>(), w.tau.as<double>(),
                     w.lamn.as<double>(), st);
      hipLaunchKernelGGL(k_zhat, dim3(gw, nm), dim3(256), 0, st, md, ms, nr, vec_pad(nr), ld, Rcur, w.nd.as<int>(),
                         w.Dn.as<double>(), w.zn.as<double>(), w.orig.as<int>(), w.tau.as<double>(),
                         w.zh.as<double>(), w.Rt.as<double>());
      launch_vec(dim3(nchunk * (nsp / 4), nm), md, ms, nr, ld, nsp, w.Rt.as<double>(), w.Dn.as<double>(),
                 w.orig.as<int>(), w.tau.as<double>(), w.zh.as<double>(), w.part.as<double>(), st);
      hipLaunchKernelGGL(k_vec_sum, dim3(std::min(((nr + 1) * Kmax + 255) / 256, 1024), nm), dim3(256), 0, st, md,
                         ms, nr, ld, nsp, w.part.as<double>(), w.NR.as<double>(), w.nrm.as<double>());
      hipLaunchKernelGGL(k_assemble, dim3(gx, nm), dim3(256), 0, st, md, ms, ell, ld, Rcur, w.NR.as<double>(),
                         w.nrm.as<double>(), w.defl.as<int>(), w.defv.as<double>(), w.lamn.as<double>(), Dnx, Rnx);
      std::swap(Dcur, Dnx);
      std::swap(Rcur, Rnx);
    }
    hipLaunchKernelGGL(k_merge_finish, dim3(gx, nm), dim3(256), 0, st, md, ell, ld, Dcur, Rcur, Dm, Fm, Lm);
    LYAP_LAUNCHED("dc merge level");
  }
  hipLaunchKernelGGL(k_root_out, dim3(std::min((k + 255) / 256, 1024)), dim3(256), 0, st, k, ell, ld, Dm, Fm, Lm, lam,
                     F, L);
  LYAP_LAUNCHED("dc root");
  w.cband = band;
  w.cldb = ldb;
  w.kc = k;
}

}  // namespace lyap
