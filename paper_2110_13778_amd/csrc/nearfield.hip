// Near-field Galerkin assembly (paper Sec. 2.3: linear-system entries over
// panel pairs of neighbouring leaf clusters; singular pairs by the
// singularity-removing relative-coordinate cubature of Sauter and Schwab) and
// the block-diagonal preconditioner of Sec. 2.6.
//
// Storage: for leaf c with n_c panels and S_c source panels (all panels of
// every c' in N(c), in list order), entries[ent_off[c] + i*S_c + k] holds the
// four operator blocks of the pair (target i of c, source k) as
// {B11, B12, B21, B22} with B11 = -(eps I3 - I2), B12 = -I1, B21 = -I6,
// B22 = -(I4 - I5/eps), plus the identity terms (1+eps)/2 A_i and
// (1+1/eps)/2 A_i on the diagonal.
//
// Pair classes: IDENT (same panel), EDGE (two shared vertices), VERTEX (one),
// CLOSE (centroid distance < near_ratio * max(sqrt(A_i), sqrt(A_j))), REGULAR.
//   REGULAR: 3 x 3 product of the symmetric 3-point rule.
//   CLOSE:   Duffy-collapsed n x n Gauss rule on each triangle.
//   IDENT:   the integrand depends on z = y - x only; the x-integral is the
//            area of a shrunken reference triangle, (1 - sigma(z))^2 / 2, and
//            the hexagon of z splits into six triangles with radial
//            coordinate xi: n^2 points per sector.
//   EDGE:    depends on (y1 - x1, x2, y2); four pyramids in those variables
//            with radial coordinate xi (Jacobian xi^2, times s on the two
//            Duffy-collapsed triangular faces) and weight (1 - sigma):
//            n^3 points per pyramid.
//   VERTEX:  Duffy on each triangle, the (x1, y1) square split on its
//            diagonal and collapsed to the shared vertex: 2 n^4 points.
// Each panel is parameterised as chi(x) = u + x1 (v - u) + x2 (w - v) on
// {0 <= x2 <= x1 <= 1}.  Every singular pair is integrated by one wavefront
// (lanes over quadrature points, fixed-order reduction), so FP64 results do
// not depend on scheduling.
#include "near.h"
#include "scan.h"

namespace fagbi {

// pass 0: count the singular / close pairs of each class per leaf (block);
// pass 1: regular entries, and the worklists at the scanned offsets.  Slots
// inside a block follow (iteration, wave, lane), so the worklists do not
// depend on scheduling.  blk is [4][nl]: counts (pass 0) or the exclusive
// scan of the counts over the flattened array (pass 1).
template <int PASS>
__global__ void __launch_bounds__(256) k_near_classify(NearArgs a, int64_t* blk, int nl, Item* w_ident,
                                                       Item* w_edge, Item* w_vertex, Item* w_close,
                                                       double4* ent) {
  __shared__ int wcnt[4][4];   // [wave][class - 1]
  const int c = blockIdx.x;
  const int nc = a.leaf_cnt[c];
  const int i0 = a.leaf_start[c];
  const int64_t so = a.src_off[c];
  const int S = (int)(a.src_off[c + 1] - so);
  const int64_t eo = a.ent_off[c];
  const int total = nc * S;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t run[4];
#pragma unroll
  for (int C = 0; C < 4; ++C) run[C] = PASS ? blk[(int64_t)C * nl + c] - blk[(int64_t)C * nl] : 0;
  for (int base = 0; base < total; base += blockDim.x) {
    const int e = base + threadIdx.x;
    const bool valid = e < total;
    int cls = -1, i = 0, j = 0;
    if (valid) {
      const int il = e / S;
      const int k = e - il * S;
      i = i0 + il;
      j = a.src_tree[so + k];
      cls = classify(a, i, j);
      // touching and close pairs are integrated once per unordered pair (for
      // the member whose target has the lower caller index) and mirrored
      if (cls >= C_EDGE && a.perm[i] > a.perm[j]) cls = -1;
      if (PASS == 1 && cls == C_REGULAR && ent) {
        double I[6];
        regular_pair(a, i, j, I);
        ent[eo + e] = combine(I, a.eps);
      }
    }
    unsigned long long mask[4];
#pragma unroll
    for (int C = 0; C < 4; ++C) {
      mask[C] = __ballot(cls == C + 1);
      if (lane == 0) wcnt[wave][C] = __popcll(mask[C]);
    }
    __syncthreads();
#pragma unroll
    for (int C = 0; C < 4; ++C) {
      int before = 0, all = 0;
      for (int w = 0; w < 4; ++w) {
        before += w < wave ? wcnt[w][C] : 0;
        all += wcnt[w][C];
      }
      if (PASS == 1 && cls == C + 1) {
        const int64_t pos = run[C] + before + __popcll(mask[C] & ((1ull << lane) - 1ull));
        Item* wl = C == 0 ? w_ident : C == 1 ? w_edge : C == 2 ? w_vertex : w_close;
        wl[pos] = Item{i, j, eo + e};
      }
      run[C] += all;
    }
    __syncthreads();
  }
  if (PASS == 0 && threadIdx.x == 0)
    for (int C = 0; C < 4; ++C) blk[(int64_t)C * nl + c] = run[C];
}

// The touching transforms write the separation as r = xi * R_hat (xi the
// radial coordinate), so every kernel is a power of xi times a function of
// u = kappa * xi * |R_hat|: the xi-rule of one ray is a power series in
// v = kappa * |R_hat| with precomputed coefficients (the class's radial
// table).  Up to the truncation (below 2^-56 relative, degree K) this is the
// same tensor-product rule as evaluating the n points of the ray.
// radial_order: the degree for a pair whose rays all have kappa |R_hat| <= vb,
// -1 if the table does not reach vb (then the rays are summed point by point).
// (vb is the same on every lane: one pair per wavefront; the degree is made
// wave-uniform so that the series loop and its table reads are scalar)
__device__ inline int radial_order(const double* tab, double vb) {
  int K = -1;
  for (int k = RAD_KMAX; k >= 2; --k)
    if (vb <= tab[RAD_VK + k]) K = k;
  return __builtin_amdgcn_readfirstlane(K);
}

// the four series of NR rays to degree K (Horner)
template <int K, int NR>
__device__ inline void radial_series(const double* tab, const double (&v)[NR], double (&t0)[NR],
                                     double (&t2)[NR], double (&t5a)[NR], double (&t5b)[NR]) {
  static_assert(K <= RAD_KMAX, "table degree");
#pragma unroll
  for (int k = K; k >= 0; --k) {
    const double* c = tab + 4 * k;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      t0[r] = fma(t0[r], v[r], c[0]);
      t2[r] = fma(t2[r], v[r], c[1]);
      t5a[r] = fma(t5a[r], v[r], c[2]);
      t5b[r] = fma(t5b[r], v[r], c[3]);
    }
  }
}

// adds the xi-rule of NR rays with weights W (the other coordinates' weights);
// the rays share the series' coefficient reads
template <int NR>
__device__ inline void radial_rays(const double (&R)[NR][3], const double (&W)[NR], const double* nx,
                                   const double* ny, double nn, double kappa, const double* tab, int K,
                                   double* acc) {
  double ir[NR], v[NR], p[NR], q[NR], t0[NR], t2[NR], t5a[NR], t5b[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double r2 = R[r][0] * R[r][0] + R[r][1] * R[r][1] + R[r][2] * R[r][2];
    p[r] = R[r][0] * nx[0] + R[r][1] * nx[1] + R[r][2] * nx[2];
    q[r] = R[r][0] * ny[0] + R[r][1] * ny[1] + R[r][2] * ny[2];
    ir[r] = inv_sqrt(r2);
    v[r] = kappa * (r2 * ir[r]);
    t0[r] = t2[r] = t5a[r] = t5b[r] = 0.0;
  }
  // degree rounded up to a multiple of 3 (more terms only add accuracy), so
  // that each series is unrolled with its table reads at fixed offsets
  switch ((K + 2) / 3) {
    case 0: case 1: case 2: radial_series<6, NR>(tab, v, t0, t2, t5a, t5b); break;
    case 3: radial_series<9, NR>(tab, v, t0, t2, t5a, t5b); break;
    case 4: radial_series<12, NR>(tab, v, t0, t2, t5a, t5b); break;
    case 5: radial_series<15, NR>(tab, v, t0, t2, t5a, t5b); break;
    case 6: radial_series<18, NR>(tab, v, t0, t2, t5a, t5b); break;
    case 7: radial_series<21, NR>(tab, v, t0, t2, t5a, t5b); break;
    default: radial_series<24, NR>(tab, v, t0, t2, t5a, t5b); break;
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double wi = W[r] * (1.0 / FOUR_PI);
    const double w3 = wi * ir[r] * ir[r] * ir[r];
    const double a1 = w3 * tab[RAD_T1], a2 = w3 * t2[r];
    acc[0] -= wi * t0[r] * ir[r];
    acc[1] += a1 * q[r];
    acc[2] += a2 * q[r];
    acc[3] -= a1 * p[r];
    acc[4] -= a2 * p[r];
    acc[5] += w3 * (nn * t5a[r] - p[r] * q[r] * (ir[r] * ir[r]) * t5b[r]);
  }
}

// rays per lane in the touching rules (they share the series' coefficient reads)
constexpr int NRAY = 2;

__device__ inline double norm3(const double* a) { return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }

// one wavefront per singular / close pair
// skip (optional): items already filled in by the surrogate; raw (optional):
// write the six integrals [n_items][6] instead of operator entries
template <int CLS>
__global__ void __launch_bounds__(256) k_near_singular(NearArgs a, const Item* items, int64_t n_items,
                                                       const double* gl, int n, double4* ent,
                                                       const uint8_t* skip, double* raw) {
  // the wave's pair (made provably wave-uniform, so that the returns below and
  // the loops after them stay scalar)
  const int64_t it = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (it >= n_items) return;
  if (skip && skip[it]) return;
  const Item item = items[it];
  const int i = item.i, j = item.j;
  const double* gx = gl;
  const double* gw = gl + 16;
  const double* ci = a.pv + 9 * i;
  const double* cj = a.pv + 9 * j;
  const double* ni = a.pn + 3 * i;
  const double* nj = a.pn + 3 * j;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  double k6[6];
  const int n2 = n * n, n3 = n2 * n, n4 = n3 * n;
  const double nn = ni[0] * nj[0] + ni[1] * nj[1] + ni[2] * nj[2];
  if (CLS == C_IDENT) {
    double e1[3], e2[3];
    for (int d = 0; d < 3; ++d) {
      e1[d] = ci[3 + d] - ci[d];
      e2[d] = ci[6 + d] - ci[3 + d];
    }
    // hexagon sectors (P_s, Q_s)
    const int HP[6][2] = {{1, 0}, {1, 1}, {0, 1}, {-1, 0}, {-1, -1}, {0, -1}};
    const int HQ[6][2] = {{1, 1}, {0, 1}, {-1, 0}, {-1, -1}, {0, -1}, {1, 0}};
    const double* tab = gl + QT_RAD + (C_IDENT - 1) * RAD_STRIDE;
    double e12[3];
    for (int d = 0; d < 3; ++d) e12[d] = e1[d] + e2[d];
    // z = xi ((1 - t) P_s + t Q_s): |R_hat| <= max over the hexagon's corners
    const int K = radial_order(tab, a.kappa * fmax(fmax(norm3(e1), norm3(e2)), norm3(e12)));
    if (K >= 0) {
      // lanes over (sector, t), NRAY rays per lane; xi by the radial table
      const int nr = 6 * n;
      // (a uniform loop: lanes past the end take the last ray with weight 0,
      // so the series loop inside keeps scalar counters and addresses)
      for (int b0 = 0; b0 < nr; b0 += 64 * NRAY) {
        double R[NRAY][3], W[NRAY];
#pragma unroll
        for (int r = 0; r < NRAY; ++r) {
          const int p0 = b0 + 64 * r + lane;
          const int p = p0 < nr ? p0 : nr - 1;
          const int s = p / n, ib = p - s * n;
          const double t = gx[ib];
          const double z1 = (1.0 - t) * HP[s][0] + t * HQ[s][0];
          const double z2 = (1.0 - t) * HP[s][1] + t * HQ[s][1];
          for (int d = 0; d < 3; ++d) R[r][d] = -(z1 * e1[d] + z2 * e2[d]);
          W[r] = p0 < nr ? gw[ib] : 0.0;
        }
        radial_rays<NRAY>(R, W, ni, ni, nn, a.kappa, tab, K, acc);
      }
    } else
    for (int p = lane; p < 6 * n2; p += 64) {
      const int s = p / n2, rem = p - s * n2, ia = rem / n, ib = rem - ia * n;
      const double xi = gx[ia], t = gx[ib];
      const double w = gw[ia] * gw[ib] * 0.5 * (1.0 - xi) * (1.0 - xi) * xi;
      const double z1 = xi * ((1.0 - t) * HP[s][0] + t * HQ[s][0]);
      const double z2 = xi * ((1.0 - t) * HP[s][1] + t * HQ[s][1]);
      kernel6(-(z1 * e1[0] + z2 * e2[0]), -(z1 * e1[1] + z2 * e2[1]), -(z1 * e1[2] + z2 * e2[2]), ni, ni,
              a.kappa, k6);
      for (int m = 0; m < 6; ++m) acc[m] += w * k6[m];
    }
  } else if (CLS == C_EDGE) {
    // shared vertices P, Q in the order they appear in triangle i
    int pid[2], np_ = 0, ri = 0, rj = 0;
    for (int p = 0; p < 3; ++p) {
      const int v = a.ptri[3 * i + p];
      const bool sh = v == a.ptri[3 * j] || v == a.ptri[3 * j + 1] || v == a.ptri[3 * j + 2];
      if (sh) pid[np_++] = p; else ri = p;
    }
    for (int p = 0; p < 3; ++p) {
      const int v = a.ptri[3 * j + p];
      const bool sh = v == a.ptri[3 * i] || v == a.ptri[3 * i + 1] || v == a.ptri[3 * i + 2];
      if (!sh) rj = p;
    }
    double e[3], av[3], bv[3];
    for (int d = 0; d < 3; ++d) {
      const double P = ci[3 * pid[0] + d], Q = ci[3 * pid[1] + d];
      e[d] = Q - P;
      av[d] = ci[3 * ri + d] - Q;
      bv[d] = cj[3 * rj + d] - Q;
    }
    const double* tab = gl + QT_RAD + (C_EDGE - 1) * RAD_STRIDE;
    // (z1, x2, y2) / xi lie in [-1, 1] x [0, 1] x [0, 1]
    const int K = radial_order(tab, a.kappa * (norm3(e) + norm3(av) + norm3(bv)));
    if (K >= 0) {
      // lanes over (piece, w1, w2), NRAY rays per lane; xi by the radial table
      const int nr = 4 * n2;
      for (int b0 = 0; b0 < nr; b0 += 64 * NRAY) {   // uniform, as above
        double R[NRAY][3], W[NRAY];
#pragma unroll
        for (int r = 0; r < NRAY; ++r) {
          // the ray's (z1, x2, y2) / xi and weight from the table (consecutive
          // lanes, consecutive rays)
          const int i0 = b0 + 64 * r + lane;
          const int it = i0 < nr ? i0 : nr - 1;
          const double4 ry = reinterpret_cast<const double4*>(gl + qt_edge_rays(n))[it];
          for (int d = 0; d < 3; ++d) R[r][d] = -ry.x * e[d] + ry.y * av[d] - ry.z * bv[d];
          W[r] = i0 < nr ? ry.w : 0.0;
        }
        radial_rays<NRAY>(R, W, ni, nj, nn, a.kappa, tab, K, acc);
      }
    } else
    // lanes over (piece, xi, w1); the innermost variable w2 enters the
    // separation linearly, r = R0 + w2 R1
    for (int it = lane; it < 4 * n2; it += 64) {
      const int piece = it / n2, rem = it - piece * n2;
      const int ia = rem / n, ib = rem - ia * n;
      const double xi = gx[ia], w1 = gx[ib];
      double wb = gw[ia] * gw[ib] * (1.0 - xi) * xi * xi;
      // (z1, x2, y2) = (z1_0, x2_0, y2_0) + w2 (z1_1, x2_1, y2_1)
      double z0, z1c, x0, x1, y0, y1;
      if (piece == 0) {
        z0 = xi * w1; z1c = 0; x0 = xi * (1 - w1); x1 = 0; y0 = 0; y1 = xi;
      } else if (piece == 1) {
        z0 = xi * w1; z1c = -xi * w1; x0 = 0; x1 = xi * w1; y0 = xi; y1 = 0; wb *= w1;
      } else if (piece == 2) {
        z0 = -xi * w1; z1c = xi * w1; x0 = xi; x1 = 0; y0 = 0; y1 = xi * w1; wb *= w1;
      } else {
        z0 = -xi * w1; z1c = 0; x0 = 0; x1 = xi; y0 = xi * (1 - w1); y1 = 0;
      }
      double R0[3], R1[3];
      for (int d = 0; d < 3; ++d) {
        R0[d] = -z0 * e[d] + x0 * av[d] - y0 * bv[d];
        R1[d] = -z1c * e[d] + x1 * av[d] - y1 * bv[d];
      }
      const LinSep L = lin_sep(R0, R1, ni, nj);
      for (int ic = 0; ic < n; ++ic) {
        const double w2 = gx[ic], w = wb * gw[ic];
        kernel6s(fma(w2, fma(w2, L.c, L.b), L.a), fma(w2, L.p1, L.p0), fma(w2, L.q1, L.q0), nn, a.kappa, k6);
        for (int m = 0; m < 6; ++m) acc[m] += w * k6[m];
      }
    }
  } else if (CLS == C_VERTEX) {
    int si = 0, sj = 0;
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q)
        if (a.ptri[3 * i + p] == a.ptri[3 * j + q]) { si = p; sj = q; }
    // the other two vertices in order of appearance
    const int vi = si == 0 ? 1 : 0, wi = si == 2 ? 1 : 2;
    const int vj = sj == 0 ? 1 : 0, wj = sj == 2 ? 1 : 2;
    double S[3], A0[3], A1[3], B0[3], B1[3];
    for (int d = 0; d < 3; ++d) {
      S[d] = ci[3 * si + d];
      A0[d] = ci[3 * vi + d] - S[d];
      A1[d] = ci[3 * wi + d] - ci[3 * vi + d];
      B0[d] = cj[3 * vj + d] - S[d];
      B1[d] = cj[3 * wj + d] - cj[3 * vj + d];
    }
    const double* tab = gl + QT_RAD + (C_VERTEX - 1) * RAD_STRIDE;
    double A01[3], B01[3];
    for (int d = 0; d < 3; ++d) {
      A01[d] = A0[d] + A1[d];
      B01[d] = B0[d] + B1[d];
    }
    const int K = radial_order(tab, a.kappa * (fmax(norm3(A0), norm3(A01)) + fmax(norm3(B0), norm3(B01))));
    if (K >= 0) {
      // lanes over (piece, eta, t1, t2), NRAY rays per lane; xi by the radial table
      const int nr = 2 * n3;
      for (int b0 = 0; b0 < nr; b0 += 64 * NRAY) {   // uniform, as above
        double R[NRAY][3], W[NRAY];
#pragma unroll
        for (int r = 0; r < NRAY; ++r) {
          // the ray's s_a, s_a t1, s_b, s_b t2 and weight from the table
          const int i0 = b0 + 64 * r + lane;
          const int it = i0 < nr ? i0 : nr - 1;
          const double* ry = gl + QT_RAY + 6 * it;
          const double2 r01 = *reinterpret_cast<const double2*>(ry);
          const double2 r23 = *reinterpret_cast<const double2*>(ry + 2);
          for (int d = 0; d < 3; ++d) R[r][d] = (r01.x * A0[d] + r01.y * A1[d]) - (r23.x * B0[d] + r23.y * B1[d]);
          W[r] = i0 < nr ? ry[4] : 0.0;
        }
        radial_rays<NRAY>(R, W, ni, nj, nn, a.kappa, tab, K, acc);
      }
    } else
    // lanes over (piece, xi, eta, t1); the innermost t2 enters linearly
    for (int it = lane; it < 2 * n3; it += 64) {
      const int piece = it / n3, rem = it - piece * n3;
      const int ia = rem / n2, ib = (rem / n) % n, ic = rem % n;
      const double xi = gx[ia], eta = gx[ib], t1 = gx[ic];
      const double wb = gw[ia] * gw[ib] * gw[ic] * xi * xi * xi * eta;
      const double sa = piece == 0 ? xi : xi * eta;
      const double sb = piece == 0 ? xi * eta : xi;
      double R0[3], R1[3];
      for (int d = 0; d < 3; ++d) {
        R0[d] = sa * (A0[d] + t1 * A1[d]) - sb * B0[d];
        R1[d] = -sb * B1[d];
      }
      const LinSep L = lin_sep(R0, R1, ni, nj);
      for (int id = 0; id < n; ++id) {
        const double t2 = gx[id], w = wb * gw[id];
        kernel6s(fma(t2, fma(t2, L.c, L.b), L.a), fma(t2, L.p1, L.p0), fma(t2, L.q1, L.q0), nn, a.kappa, k6);
        for (int m = 0; m < 6; ++m) acc[m] += w * k6[m];
      }
    }
  } else {  // CLOSE
    const double tai = 2.0 * a.pa[i], taj = 2.0 * a.pa[j];
    // lanes over (s1, t1, s2) from the order's table (a uniform loop: lanes
    // past the end take the last point with weight 0); the innermost t2
    // enters linearly
    const double4* cp = reinterpret_cast<const double4*>(gl + qt_close_pts(n));
    for (int b0 = 0; b0 < n3; b0 += 64) {
      const int it0 = b0 + lane;
      const double4 o = cp[it0 < n3 ? it0 : n3 - 1];
      const double s1 = o.x, s1t1 = o.y, s2 = o.z;
      const double wb = it0 < n3 ? tai * taj * o.w : 0.0;
      double R0[3], R1[3];
      for (int d = 0; d < 3; ++d) {
        const double x = ci[d] + s1 * (ci[3 + d] - ci[d]) + s1t1 * (ci[6 + d] - ci[3 + d]);
        R0[d] = x - (cj[d] + s2 * (cj[3 + d] - cj[d]));
        R1[d] = -s2 * (cj[6 + d] - cj[3 + d]);
      }
      const LinSep L = lin_sep(R0, R1, ni, nj);
      for (int id = 0; id < n; ++id) {
        const double t2 = gx[id], w = wb * gw[id];
        kernel6s(fma(t2, fma(t2, L.c, L.b), L.a), fma(t2, L.p1, L.p0), fma(t2, L.q1, L.q0), nn, a.kappa, k6);
        for (int m = 0; m < 6; ++m) acc[m] += w * k6[m];
      }
    }
  }
  for (int m = 0; m < 6; ++m) acc[m] = wave_sum(acc[m]);
  if (lane == 0) {
    double scale = 1.0;
    if (CLS == C_IDENT) scale = 4.0 * a.pa[i] * a.pa[i];
    else if (CLS == C_EDGE || CLS == C_VERTEX) scale = 4.0 * a.pa[i] * a.pa[j];
    for (int m = 0; m < 6; ++m) acc[m] *= scale;
    if (CLS == C_IDENT) {
      acc[1] = acc[2] = acc[3] = acc[4] = 0.0;   // r.n = 0 on a flat panel
    }
    if (raw)
      for (int m = 0; m < 6; ++m) raw[6 * it + m] = acc[m];
    else
      write_pair(a, CLS, i, j, item.ent, acc, ent);
  }
}

__global__ void k_to_f32(const double4* __restrict__ src, float4* __restrict__ dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double4 v = src[e];
    dst[e] = make_float4((float)v.x, (float)v.y, (float)v.z, (float)v.w);
  }
}

NearArgs near_args(fagbi_handle* h) {
  NearArgs a;
  a.pv = h->d_pv.as<double>();
  a.pn = h->d_pn.as<double>();
  a.pa = h->d_pa.as<double>();
  a.ptri = h->d_ptri.as<int32_t>();
  a.pc = h->d_pc.as<double4>();
  a.leaf_start = h->d_leaf_start.as<int32_t>();
  a.leaf_cnt = h->d_leaf_cnt.as<int32_t>();
  a.src_off = h->d_src_off.as<int64_t>();
  a.ent_off = h->d_ent_off.as<int64_t>();
  a.src_tree = h->d_src_tree.as<int32_t>();
  a.perm = h->d_perm.as<int32_t>();
  a.leaf_of = h->d_leaf_of.as<int32_t>();
  a.lnbr_off = h->d_lnbr_off.as<int32_t>();
  a.lnbr = h->d_lnbr.as<int32_t>();
  a.lnbr_col = h->d_lnbr_col.as<int32_t>();
  a.kappa = h->prm.kappa;
  a.eps = h->prm.eps_out / h->prm.eps_in;
  a.near_ratio = h->prm.near_ratio;
  return a;
}

int run_singular(fagbi_handle* h, int cls_index, const uint8_t* skip, double* raw, hipStream_t s) {
  NearArgs a = near_args(h);
  const int64_t m = h->wl_n[cls_index];
  if (m == 0) return 0;
  const unsigned g = (unsigned)((m + 3) / 4);
  const int n = h->prm.quad_duffy;
  const double* gl = h->d_gl.as<double>();
  double4* E = h->d_E64.as<double4>();
  const Item* it = h->d_wl[cls_index].as<Item>();
  switch (cls_index) {
    case 0: k_near_singular<C_IDENT><<<g, 256, 0, s>>>(a, it, m, gl, n, E, skip, raw); break;
    case 1: k_near_singular<C_EDGE><<<g, 256, 0, s>>>(a, it, m, gl, n, E, skip, raw); break;
    case 2: k_near_singular<C_VERTEX><<<g, 256, 0, s>>>(a, it, m, gl, n, E, skip, raw); break;
    default: k_near_singular<C_CLOSE><<<g, 256, 0, s>>>(a, it, m, gl, n, E, skip, raw); break;
  }
  FAGBI_HIP(hipGetLastError());
  return 0;
}

int assemble_nearfield(fagbi_handle* h, hipStream_t s) {
  const int nl = h->lev[h->L].n;
  NearArgs a = near_args(h);
  // (hat functions: the entries by vertex pairs are allocated by their assembly)
  if (!h->hat()) {
    FAGBI_TRY(h->alloc(h->d_E64, (size_t)h->n_ent * sizeof(double4)));
    FAGBI_TRY(h->alloc(h->d_E32, (size_t)h->n_ent * sizeof(float4)));
  }
  StageTimer t_cls(h, s, &h->prof.ms_classify);
  // per-leaf class counts, one scan over the flattened [class][leaf] array,
  // then the worklists at the scanned offsets
  Tmp cnt, off, part;
  const int64_t m = 4 * (int64_t)nl;
  FAGBI_TRY(cnt.alloc(m * 8));
  FAGBI_TRY(off.alloc((m + 1) * 8));
  FAGBI_TRY(part.alloc(scan_part_size(m) * 8));
  k_near_classify<0><<<nl, 256, 0, s>>>(a, cnt.as<int64_t>(), nl, nullptr, nullptr, nullptr, nullptr, nullptr);
  FAGBI_HIP(hipGetLastError());
  FAGBI_TRY((device_scan<int64_t, int64_t>(cnt.as<int64_t>(), m, off.as<int64_t>(), part.as<int64_t>(), s)));
  int64_t bnd[5];
  for (int k = 0; k < 5; ++k)
    FAGBI_HIP(hipMemcpyAsync(&bnd[k], off.as<int64_t>() + (int64_t)k * nl, 8, hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipStreamSynchronize(s));
  for (int k = 0; k < 4; ++k) {
    const int64_t c = bnd[k + 1] - bnd[k];
    h->singular_count[k] = c;
    h->wl_n[k] = c;
    FAGBI_TRY(h->alloc(h->d_wl[k], (size_t)std::max<int64_t>(c, 1) * sizeof(Item)));
  }
  k_near_classify<1><<<nl, 256, 0, s>>>(a, off.as<int64_t>(), nl, h->d_wl[0].as<Item>(), h->d_wl[1].as<Item>(),
                                        h->d_wl[2].as<Item>(), h->d_wl[3].as<Item>(),
                                        h->hat() ? nullptr : h->d_E64.as<double4>());
  FAGBI_HIP(hipGetLastError());
  t_cls.stop();
  if (h->hat()) {
    h->prof.ms_surrogate = 0;
    h->mlp_gated_pairs = 0;
    {
      StageTimer t_sing(h, s, &h->prof.ms_singular);
      FAGBI_TRY(hat_assemble(h, s));
    }
    k_to_f32<<<2048, 256, 0, s>>>(h->d_E64.as<double4>(), h->d_E32.as<float4>(), h->n_vb_ent);
    FAGBI_HIP(hipGetLastError());
    FAGBI_HIP(hipStreamSynchronize(s));
    h->precond_ready = false;
    return 0;
  }
  h->prof.ms_surrogate = 0;
  StageTimer t_sing(h, s, &h->prof.ms_singular);
  // identical pairs: always the FP64 singular cubature
  FAGBI_TRY(run_singular(h, 0, nullptr, nullptr, s));
  const bool use_mlp = h->prm.mlp_mode != FAGBI_MLP_OFF && h->mlp_ready;
  h->mlp_gated_pairs = 0;
  if (use_mlp) {
    // the surrogate writes its entries for every near-singular pair and flags
    // the ones whose calibrated error passes the gate
    {
      StageTimer t_mlp(h, s, &h->prof.ms_surrogate);
      FAGBI_TRY(mlp_assembly_stage(h, s));
    }
    if (h->prm.mlp_mode == FAGBI_MLP_PRECOND) {
      // preconditioner from the surrogate's entries, operator from cubature
      FAGBI_TRY(precond_setup(h, s));
      for (int k = 1; k < 4; ++k) FAGBI_TRY(run_singular(h, k, nullptr, nullptr, s));
    } else {
      for (int k = 1; k < 4; ++k) FAGBI_TRY(run_singular(h, k, h->d_mlp_skip[k].as<uint8_t>(), nullptr, s));
    }
  } else {
    for (int k = 1; k < 4; ++k) FAGBI_TRY(run_singular(h, k, nullptr, nullptr, s));
  }
  k_to_f32<<<2048, 256, 0, s>>>(h->d_E64.as<double4>(), h->d_E32.as<float4>(), h->n_ent);
  FAGBI_HIP(hipGetLastError());
  FAGBI_HIP(hipStreamSynchronize(s));
  if (h->profiling) {
    t_sing.stop();   // singular stage without the surrogate's share
    h->prof.ms_singular -= h->prof.ms_surrogate;
  }
  h->precond_ready = use_mlp && h->prm.mlp_mode == FAGBI_MLP_PRECOND;
  return 0;
}

// ---------------------------------------------------------------------------
// block-diagonal preconditioner (Sec. 2.6): for each leaf c the 2n_c x 2n_c
// block of A between its own panels, ordered [phi_c; dphi_c], inverted by
// Gauss-Jordan elimination with partial pivoting (one wavefront per leaf,
// matrix in LDS).  The inverse is stored transposed for coalesced apply.
// ---------------------------------------------------------------------------
// Blocks of the preconditioner: groups of consecutive leaves (one leaf per
// group for FAGBI_PRECOND_BLOCK; consecutive leaves up to 32 panels for
// FAGBI_PRECOND_GROUP).  Group g covers leaves [gl[g], gl[g+1]) and panels
// [gp[g], gp[g+1]); its block is ordered [phi of the group's panels; dphi of
// them] and holds every stored near-field entry between them (pairs of
// leaves that are not neighbours have none: they are far field).
// Gauss-Jordan with partial pivoting in LDS; two wavefronts per block, each
// updating one half of every row's columns (the LDS matrix limits a CU to a
// few blocks: the second wavefront doubles the work in flight)
__global__ void __launch_bounds__(128) k_block_invert(const double4* __restrict__ ent, const int32_t* gl,
                                                     const int32_t* gp, const int32_t* leaf_start,
                                                     const int32_t* leaf_cnt, const int64_t* src_off,
                                                     const int64_t* ent_off, const int32_t* lnbr_off,
                                                     const int32_t* lnbr, const int32_t* lnbr_col,
                                                     const int64_t* inv_off, double* inv, int* bad) {
  __shared__ double A[64][65];
  __shared__ int swp[64];
  const int g = blockIdx.x;
  const int l0 = gl[g], l1 = gl[g + 1];
  const int p0 = gp[g];
  const int ng = gp[g + 1] - p0;
  const int m = 2 * ng;
  const int r = threadIdx.x & 63, hf = threadIdx.x >> 6;
  const int j0 = hf * 32, j1 = min(m, j0 + 32);   // this wavefront's columns
  for (int j = j0; j < j1; ++j)
    if (r < m) A[r][j] = 0.0;
  __syncthreads();
  for (int c1 = l0; c1 < l1; ++c1) {
    const int n1 = leaf_cnt[c1], o1 = leaf_start[c1] - p0;
    const int S = (int)(src_off[c1 + 1] - src_off[c1]);
    const int64_t eo = ent_off[c1];
    for (int q = lnbr_off[c1]; q < lnbr_off[c1 + 1]; ++q) {
      const int c2 = lnbr[q];
      if (c2 < l0 || c2 >= l1) continue;
      const int n2 = leaf_cnt[c2], o2 = leaf_start[c2] - p0, col = lnbr_col[q];
      for (int e = threadIdx.x; e < n1 * n2; e += 128) {
        const int il = e / n2, jl = e - il * n2;
        const double4 v = ent[eo + (int64_t)il * S + col + jl];
        A[o1 + il][o2 + jl] = v.x;
        A[o1 + il][ng + o2 + jl] = v.y;
        A[ng + o1 + il][o2 + jl] = v.z;
        A[ng + o1 + il][ng + o2 + jl] = v.w;
      }
    }
  }
  __syncthreads();
  // elimination with each thread's share of its row (row r, columns
  // j0 .. j0 + 31) in registers; per step only column k and the scaled pivot
  // row pass through LDS (double-buffered: two barriers per step)
  __shared__ double colk[2][64], prow[2][64];
  double a[32];
#pragma unroll
  for (int jj = 0; jj < 32; ++jj) a[jj] = (r < m && j0 + jj < m) ? A[r][j0 + jj] : 0.0;
  for (int k = 0; k < m; ++k) {
    const int bk = k & 1, kh = k >> 5, kk = k & 31;
    if (hf == kh) {   // the wavefront holding column k publishes it
      double ck = 0.0;
#pragma unroll
      for (int jj = 0; jj < 32; ++jj) ck = jj == kk ? a[jj] : ck;
      colk[bk][r] = r < m ? ck : 0.0;
    }
    __syncthreads();
    // pivot: largest |A[i][k]|, i >= k, smallest index on ties (both
    // wavefronts find the same)
    double v = (r >= k && r < m) ? fabs(colk[bk][r]) : -1.0;
    int vi = r;
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(v, o, 64);
      const int oi = __shfl_xor(vi, o, 64);
      if (ov > v || (ov == v && oi < vi)) { v = ov; vi = oi; }
    }
    if (threadIdx.x == 0) swp[k] = vi;
    if (!(v > 0.0)) {   // both wavefronts see the same column
      if (threadIdx.x == 0) atomicExch(bad, 1);
      return;
    }
    if (vi != k) {   // interchange rows k and vi (lanes k and vi of each wavefront)
#pragma unroll
      for (int jj = 0; jj < 32; ++jj) {
        const double x = a[jj];
        const double xk = __shfl(x, k, 64), xv = __shfl(x, vi, 64);
        a[jj] = r == k ? xv : (r == vi ? xk : x);
      }
    }
    const int rs = r == k ? vi : (r == vi ? k : r);   // this row's pre-interchange index
    const double d = 1.0 / colk[bk][vi];
    if (r == k) {
#pragma unroll
      for (int jj = 0; jj < 32; ++jj) {
        a[jj] = (j0 + jj == k ? 1.0 : a[jj]) * d;
        prow[bk][j0 + jj] = a[jj];
      }
    }
    __syncthreads();
    if (r < m && r != k) {
      const double f = colk[bk][rs];
#pragma unroll
      for (int jj = 0; jj < 32; ++jj) {
        const double ajj = (hf == kh && jj == kk) ? 0.0 : a[jj];
        a[jj] = ajj - f * prow[bk][j0 + jj];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int jj = 0; jj < 32; ++jj)
    if (r < m && j0 + jj < m) A[r][j0 + jj] = a[jj];
  __syncthreads();
  // undo the row interchanges as column interchanges, last first
  for (int k = m - 1; k >= 0; --k) {
    const int p = swp[k];
    if (hf == 0 && p != k && r < m) {
      const double t = A[r][k];
      A[r][k] = A[r][p];
      A[r][p] = t;
    }
    __syncthreads();
  }
  if (r < m) {
    double* out = inv + inv_off[g];
    for (int b = j0; b < j1; ++b) out[(int64_t)b * m + r] = A[r][b];
  }
}

// y = M^-1 z, one wavefront per group (inverse stored transposed; FP64, or an
// FP32 copy for the inner solves of the mixed-precision path)
template <typename T>
__global__ void __launch_bounds__(64) k_block_apply(const T* __restrict__ inv,
                                                    const int64_t* inv_off, const int32_t* gp,
                                                    const int32_t* perm, int64_t N, const double* z, double* y) {
  __shared__ double zb[64];
  const int g = blockIdx.x;
  const int p0 = gp[g];
  const int ng = gp[g + 1] - p0;
  const int m = 2 * ng;
  const int r = threadIdx.x;
  int64_t row = 0;
  if (r < m) {
    const int p = perm[p0 + (r < ng ? r : r - ng)];
    row = r < ng ? (int64_t)p : N + p;
    zb[r] = z[row];
  }
  __syncthreads();
  if (r < m) {
    const T* Ti = inv + inv_off[g];
    double acc = 0;
    for (int b = 0; b < m; ++b) acc += (double)Ti[(int64_t)b * m + r] * zb[b];
    y[row] = acc;
  }
}

__global__ void k_diag_extract(const double4* __restrict__ ent, const int32_t* leaf_start,
                               const int32_t* leaf_cnt, const int64_t* src_off, const int64_t* ent_off,
                               const int32_t* self_col, const int32_t* perm, int64_t N, double* diag) {
  const int c = blockIdx.x;
  const int nc = leaf_cnt[c];
  const int S = (int)(src_off[c + 1] - src_off[c]);
  for (int il = threadIdx.x; il < nc; il += blockDim.x) {
    const double4 e = ent[ent_off[c] + (int64_t)il * S + self_col[c] + il];
    const int p = perm[leaf_start[c] + il];
    diag[p] = e.x;
    diag[N + p] = e.w;
  }
}

__global__ void k_diag_apply(const double* diag, const double* z, double* y, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    y[e] = z[e] / diag[e];
}

__global__ void k_to_f32_1(const double* __restrict__ a, float* b, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    b[e] = (float)a[e];
}

int precond_setup(fagbi_handle* h, hipStream_t s) {
  if (h->hat()) return h->prm.precond == FAGBI_PRECOND_DIAG ? hat_diag_setup(h, s) : 0;
  const int nl = h->lev[h->L].n;
  FAGBI_TRY(h->alloc(h->d_diag, 2 * h->N * sizeof(double)));
  k_diag_extract<<<nl, 64, 0, s>>>(h->d_E64.as<double4>(), h->d_leaf_start.as<int32_t>(),
                                   h->d_leaf_cnt.as<int32_t>(), h->d_src_off.as<int64_t>(),
                                   h->d_ent_off.as<int64_t>(), h->d_self_col.as<int32_t>(),
                                   h->d_perm.as<int32_t>(), h->N, h->d_diag.as<double>());
  FAGBI_HIP(hipGetLastError());
  // groups of consecutive leaves: one leaf each, or (GROUP) as many as fit in
  // 32 panels
  const int gmax = h->prm.precond == FAGBI_PRECOND_GROUP ? 32 : 0;
  std::vector<int32_t> gl(1, 0), gp(1, 0);
  int panels = 0, cur = 0;
  for (int c = 0; c < nl; ++c) {
    const int n = h->leaf_cnt[c];
    if (c > gl.back() && (gmax == 0 || cur + n > gmax)) {
      gl.push_back(c);
      gp.push_back(panels);
      cur = 0;
    }
    cur += n;
    panels += n;
  }
  gl.push_back(nl);
  gp.push_back(panels);
  const int ng = (int)gl.size() - 1;
  h->n_groups = ng;
  std::vector<int64_t> off(ng + 1, 0);
  for (int g = 0; g < ng; ++g) off[g + 1] = off[g] + 4LL * (gp[g + 1] - gp[g]) * (gp[g + 1] - gp[g]);
  FAGBI_TRY(h->upload(h->d_grp_leaf, gl.data(), gl.size() * 4));
  FAGBI_TRY(h->upload(h->d_grp_panel, gp.data(), gp.size() * 4));
  FAGBI_TRY(h->upload(h->d_lu_off, off.data(), off.size() * 8));
  FAGBI_TRY(h->alloc(h->d_lu, (size_t)off[ng] * sizeof(double)));
  Tmp bad;
  FAGBI_TRY(bad.alloc(sizeof(int)));
  FAGBI_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
  k_block_invert<<<ng, 128, 0, s>>>(h->d_E64.as<double4>(), h->d_grp_leaf.as<int32_t>(), h->d_grp_panel.as<int32_t>(),
                                   h->d_leaf_start.as<int32_t>(), h->d_leaf_cnt.as<int32_t>(),
                                   h->d_src_off.as<int64_t>(), h->d_ent_off.as<int64_t>(),
                                   h->d_lnbr_off.as<int32_t>(), h->d_lnbr.as<int32_t>(),
                                   h->d_lnbr_col.as<int32_t>(), h->d_lu_off.as<int64_t>(), h->d_lu.as<double>(),
                                   bad.as<int>());
  FAGBI_HIP(hipGetLastError());
  FAGBI_TRY(h->alloc(h->d_lu32, (size_t)off[ng] * sizeof(float)));
  k_to_f32_1<<<1024, 256, 0, s>>>(h->d_lu.as<double>(), h->d_lu32.as<float>(), off[ng]);
  FAGBI_HIP(hipGetLastError());
  int hb = 0;
  FAGBI_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipStreamSynchronize(s));
  if (hb) return set_error(FAGBI_E_NUMERIC, "singular block in the block-diagonal preconditioner");
  return 0;
}

int precond_apply(fagbi_handle* h, const double* z, double* y, hipStream_t s, bool f32) {
  const int64_t n = 2 * h->n_unk();
  if (h->prm.precond == FAGBI_PRECOND_NONE) {
    if (z != y) FAGBI_HIP(hipMemcpyAsync(y, z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    return 0;
  }
  if (h->prm.precond == FAGBI_PRECOND_DIAG) {
    k_diag_apply<<<1024, 256, 0, s>>>(h->d_diag.as<double>(), z, y, n);
    FAGBI_HIP(hipGetLastError());
    return 0;
  }
  if (f32)
    k_block_apply<float><<<h->n_groups, 64, 0, s>>>(h->d_lu32.as<float>(), h->d_lu_off.as<int64_t>(),
                                                    h->d_grp_panel.as<int32_t>(), h->d_perm.as<int32_t>(), h->N, z,
                                                    y);
  else
    k_block_apply<double><<<h->n_groups, 64, 0, s>>>(h->d_lu.as<double>(), h->d_lu_off.as<int64_t>(),
                                                     h->d_grp_panel.as<int32_t>(), h->d_perm.as<int32_t>(), h->N, z,
                                                     y);
  FAGBI_HIP(hipGetLastError());
  return 0;
}

}  // namespace fagbi
