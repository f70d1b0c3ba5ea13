// Continuous piecewise-linear Galerkin space S^1_h (paper Sec. 2.3) on the
// box-function machinery.
//
// Unknowns are the nodal values of phi and dphi at the vertices.  On a panel
// the hat function of its corner-a vertex is the barycentric coordinate
// lambda_a, so every entry of the system is a sum over panel pairs of corner
// integrals J[a][b] = int int lambda_a(x) k(x, y) lambda_b(y).  The operator
// runs over elements, the panel corners e = 3 i + a (i in tree order):
//  * near field: for leaf c with n_c panels and S_c source panels the block
//    has 3 n_c element rows and 3 S_c element columns; the entry of (row
//    3 r + a, column 3 k + b) is at 9 ent_off[c] + (3 r + a) 3 S_c + 3 k + b
//    and holds the four operator entries of J[a][b] of the panel pair (r, k),
//    plus (1+eps)/2 and (1+1/eps)/2 times the mass A (1 + delta_ab) / 12 on
//    identical pairs.  The box-function SpMV kernel runs on this layout as is;
//  * far field: one pair of moments per corner (the 3-point rule's weights
//    times lambda_a at its points: 2/3 at point a, 1/6 at the others), so P2M,
//    the translations and LtP run unchanged over the elements;
//  * the element results are summed into the vertices (fixed order: the
//    elements of a vertex ascending).
//
// Corner integrals of the pair classes (the rules of the box-function
// assembly, evaluated point by point, with the barycentric products inside):
//  REGULAR: 3 x 3 product of the 3-point rule.
//  IDENT:   the rule over z = y - x (hexagon, six sectors, n^2 points each);
//           for fixed z the x-integral over the shrunken triangle
//           T(z) = {x : x, x + z in the reference triangle} of
//           lambda_a(x) lambda_b(x + z), a quadratic, by the 3-point rule on
//           T(z) (corners (A+B, A), (1-C, A), (1-C, 1-C-B) with A = max(0,-z2),
//           B = max(0, z2-z1), C = max(0, z1)); flat panels: I2..I5 vanish.
//  EDGE:    the rule over (z1 = y1 - x1, x2, y2) (four pyramids, n^3 points
//           each); the x1-integral over [max(x2, y2 - z1), 1 - max(0, z1)] of
//           the product, a quadratic in x1, by 2-point Gauss-Legendre.
//  VERTEX:  Duffy on each triangle and the collapsed square, 2 n^4 points.
//  CLOSE:   Duffy n x n on each triangle, n^4 points.
//  In both the innermost coordinate moves the source point along a line with
//  the target point fixed, so each lane sums lambda_b k over it first (18
//  sums) and multiplies by lambda_a once per line.
// Reference coordinates chi(x) = u + x1 (v - u) + x2 (w - v) on
// {0 <= x2 <= x1 <= 1}: lambda_u = 1 - x1, lambda_v = x1 - x2, lambda_w = x2.
// One wavefront per singular or close pair, fixed-order reductions: FP64
// results do not depend on scheduling.  Touching and close pairs are
// integrated once (for the member with the lower caller index) and mirrored:
// J_ji[b][a] = J_ij[a][b] with I2 <-> I4 and I3 <-> I5.
#include <vector>

#include "near.h"
#include "scan.h"

namespace fagbi {

// lambda at point k of the 3-point rule, of corner a
__device__ constexpr double lam3(int k, int a) { return k == a ? 2.0 / 3.0 : 1.0 / 6.0; }

// the four operator entries of corner integrals I (times scale), with the
// identity terms' mass share m (0 off identical pairs)
__device__ inline double4 hat_entry(const double* I, double scale, double eps, double m) {
  double J[6];
  for (int q = 0; q < 6; ++q) J[q] = I[q] * scale;
  double4 v = combine(J, eps);
  v.x += 0.5 * (1.0 + eps) * m;
  v.w += 0.5 * (1.0 + 1.0 / eps) * m;
  return v;
}

// regular pairs of leaf c (one block per leaf, threads over its pairs)
__global__ void __launch_bounds__(256) k_hat_regular(NearArgs a, double4* ent) {
  const int c = blockIdx.x;
  const int nc = a.leaf_cnt[c];
  const int i0 = a.leaf_start[c];
  const int64_t so = a.src_off[c];
  const int S = (int)(a.src_off[c + 1] - so);
  const int64_t base = 9 * a.ent_off[c];
  for (int e = threadIdx.x; e < nc * S; e += blockDim.x) {
    const int il = e / S, k = e - il * S;
    const int i = i0 + il, j = a.src_tree[so + k];
    if (classify(a, i, j) != C_REGULAR) continue;
    double qi[9], qj[9];
    quad_points(a.pv, i, qi);
    quad_points(a.pv, j, qj);
    const double* ni = a.pn + 3 * i;
    const double* nj = a.pn + 3 * j;
    double acc[3][3][6];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
      for (int y = 0; y < 3; ++y)
#pragma unroll
        for (int m = 0; m < 6; ++m) acc[x][y][m] = 0.0;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      // t[b] = sum_q lambda_b(y_q) k(x_p, y_q)
      double t[3][6];
#pragma unroll
      for (int y = 0; y < 3; ++y)
#pragma unroll
        for (int m = 0; m < 6; ++m) t[y][m] = 0.0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        double k6[6];
        kernel6(qi[3 * p] - qj[3 * q], qi[3 * p + 1] - qj[3 * q + 1], qi[3 * p + 2] - qj[3 * q + 2], ni, nj,
                a.kappa, k6);
#pragma unroll
        for (int y = 0; y < 3; ++y)
#pragma unroll
          for (int m = 0; m < 6; ++m) t[y][m] += lam3(q, y) * k6[m];
      }
#pragma unroll
      for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y)
#pragma unroll
          for (int m = 0; m < 6; ++m) acc[x][y][m] += lam3(p, x) * t[y][m];
    }
    const double w = (a.pa[i] / 3.0) * (a.pa[j] / 3.0);
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
      for (int y = 0; y < 3; ++y)
        ent[base + (int64_t)(3 * il + x) * (3 * S) + 3 * k + y] = hat_entry(acc[x][y], w, a.eps, 0.0);
  }
}

// barycentric coordinates of reference point (x1, x2)
__device__ inline void bary(double x1, double x2, double* l) {
  l[0] = 1.0 - x1;
  l[1] = x1 - x2;
  l[2] = x2;
}

// acc[a][b][m] += w la[a] lb[b] k[m] for the channels m in [M0, M1)
template <int M0, int M1>
__device__ inline void add_outer(double (&acc)[3][3][6], double w, const double* la, const double* lb,
                                 const double* k6) {
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    const double wa = w * la[x];
#pragma unroll
    for (int y = 0; y < 3; ++y) {
      const double wab = wa * lb[y];
#pragma unroll
      for (int m = M0; m < M1; ++m) acc[x][y][m] += wab * k6[m];
    }
  }
}

// one wavefront per singular / close pair
template <int CLS>
__global__ void __launch_bounds__(64) k_hat_singular(NearArgs a, const Item* items, int64_t n_items,
                                                     const double* gl, int n, double4* ent) {
  const int64_t it = blockIdx.x;
  const int lane = threadIdx.x;
  if (it >= n_items) return;
  const Item item = items[it];
  const int i = item.i, j = item.j;
  const double* gx = gl;
  const double* gw = gl + 16;
  const double* ci = a.pv + 9 * i;
  const double* cj = a.pv + 9 * j;
  const double* ni = a.pn + 3 * i;
  const double* nj = a.pn + 3 * j;
  double acc[3][3][6];
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int y = 0; y < 3; ++y)
#pragma unroll
      for (int m = 0; m < 6; ++m) acc[x][y][m] = 0.0;
  // triangle corner of the rule's corner a (panel i) and b (panel j)
  int oi[3] = {0, 1, 2}, oj[3] = {0, 1, 2};
  double k6[6], la[3], lb[3];
  const int n2 = n * n, n3 = n2 * n, n4 = n3 * n;
  double scale = 1.0;
  if (CLS == C_IDENT) {
    double e1[3], e2[3];
    for (int d = 0; d < 3; ++d) {
      e1[d] = ci[3 + d] - ci[d];
      e2[d] = ci[6 + d] - ci[3 + d];
    }
    const int HP[6][2] = {{1, 0}, {1, 1}, {0, 1}, {-1, 0}, {-1, -1}, {0, -1}};
    const int HQ[6][2] = {{1, 1}, {0, 1}, {-1, 0}, {-1, -1}, {0, -1}, {1, 0}};
    for (int p = lane; p < 6 * n2; p += 64) {
      const int s = p / n2, rem = p - s * n2, ia = rem / n, ib = rem - ia * n;
      const double xi = gx[ia], t = gx[ib];
      const double w = gw[ia] * gw[ib] * 0.5 * (1.0 - xi) * (1.0 - xi) * xi;
      const double z1 = xi * ((1.0 - t) * HP[s][0] + t * HQ[s][0]);
      const double z2 = xi * ((1.0 - t) * HP[s][1] + t * HQ[s][1]);
      kernel6(-(z1 * e1[0] + z2 * e2[0]), -(z1 * e1[1] + z2 * e2[1]), -(z1 * e1[2] + z2 * e2[2]), ni, ni,
              a.kappa, k6);
      // the 3-point rule on T(z), each point weighted 1/3
      const double A = fmax(0.0, -z2), B = fmax(0.0, z2 - z1), C = fmax(0.0, z1);
      const double V[3][2] = {{A + B, A}, {1.0 - C, A}, {1.0 - C, 1.0 - C - B}};
      for (int q = 0; q < 3; ++q) {
        const double x1 = (2.0 / 3.0) * V[q][0] + (1.0 / 6.0) * (V[(q + 1) % 3][0] + V[(q + 2) % 3][0]);
        const double x2 = (2.0 / 3.0) * V[q][1] + (1.0 / 6.0) * (V[(q + 1) % 3][1] + V[(q + 2) % 3][1]);
        bary(x1, x2, la);
        bary(x1 + z1, x2 + z2, lb);
        // r.n vanishes in the plane of the panel: only I1 and I6
        add_outer<0, 1>(acc, w * (1.0 / 3.0), la, lb, k6);
        add_outer<5, 6>(acc, w * (1.0 / 3.0), la, lb, k6);
      }
    }
    scale = 4.0 * a.pa[i] * a.pa[i];
  } else if (CLS == C_EDGE) {
    // P, Q: the shared vertices in their order in triangle i; R_i, R_j the
    // others (corner positions by selects: no indexed stores to the maps)
    const int ti0 = a.ptri[3 * i], ti1 = a.ptri[3 * i + 1], ti2 = a.ptri[3 * i + 2];
    const int tj0 = a.ptri[3 * j], tj1 = a.ptri[3 * j + 1], tj2 = a.ptri[3 * j + 2];
    const bool s0 = ti0 == tj0 || ti0 == tj1 || ti0 == tj2;
    const bool s1 = ti1 == tj0 || ti1 == tj1 || ti1 == tj2;
    oi[0] = s0 ? 0 : 1;
    oi[1] = (s0 && s1) ? 1 : 2;
    oi[2] = 3 - oi[0] - oi[1];
    const int vP = oi[0] == 0 ? ti0 : ti1;
    const int vQ = oi[1] == 1 ? ti1 : ti2;
    oj[0] = tj0 == vP ? 0 : (tj1 == vP ? 1 : 2);
    oj[1] = tj0 == vQ ? 0 : (tj1 == vQ ? 1 : 2);
    oj[2] = 3 - oj[0] - oj[1];
    double e[3], av[3], bv[3];
    for (int d = 0; d < 3; ++d) {
      const double P = ci[3 * oi[0] + d], Q = ci[3 * oi[1] + d];
      e[d] = Q - P;
      av[d] = ci[3 * oi[2] + d] - Q;
      bv[d] = cj[3 * oj[2] + d] - Q;
    }
    const double g0 = 0.5 - 0.5 / sqrt(3.0), g1 = 0.5 + 0.5 / sqrt(3.0);
    for (int p = lane; p < 4 * n3; p += 64) {
      const int piece = p / n3, rem = p - piece * n3;
      const int ia = rem / n2, ib = (rem / n) % n, ic = rem % n;
      const double xi = gx[ia], w1 = gx[ib], w2 = gx[ic];
      double w = gw[ia] * gw[ib] * gw[ic] * (1.0 - xi) * xi * xi;
      double z1, x2, y2;
      if (piece == 0) {
        z1 = xi * w1; x2 = xi * (1.0 - w1); y2 = xi * w2;
      } else if (piece == 1) {
        z1 = xi * w1 * (1.0 - w2); x2 = xi * w1 * w2; y2 = xi; w *= w1;
      } else if (piece == 2) {
        z1 = -xi * w1 * (1.0 - w2); x2 = xi; y2 = xi * w1 * w2; w *= w1;
      } else {
        z1 = -xi * w1; x2 = xi * w2; y2 = xi * (1.0 - w1);
      }
      kernel6(-z1 * e[0] + x2 * av[0] - y2 * bv[0], -z1 * e[1] + x2 * av[1] - y2 * bv[1],
              -z1 * e[2] + x2 * av[2] - y2 * bv[2], ni, nj, a.kappa, k6);
      const double lo = fmax(x2, y2 - z1), hi = 1.0 - fmax(0.0, z1);
      for (int q = 0; q < 2; ++q) {
        const double x1 = lo + (hi - lo) * (q == 0 ? g0 : g1);
        bary(x1, x2, la);
        bary(x1 + z1, y2, lb);
        add_outer<0, 6>(acc, 0.5 * w, la, lb, k6);
      }
    }
    scale = 4.0 * a.pa[i] * a.pa[j];
  } else if (CLS == C_VERTEX) {
    int si = 0, sj = 0;
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q)
        if (a.ptri[3 * i + p] == a.ptri[3 * j + q]) { si = p; sj = q; }
    oi[0] = si;
    oi[1] = si == 0 ? 1 : 0;
    oi[2] = si == 2 ? 1 : 2;
    oj[0] = sj;
    oj[1] = sj == 0 ? 1 : 0;
    oj[2] = sj == 2 ? 1 : 2;
    double A0[3], A1[3], B0[3], B1[3];
    for (int d = 0; d < 3; ++d) {
      const double S = ci[3 * oi[0] + d];
      A0[d] = ci[3 * oi[1] + d] - S;
      A1[d] = ci[3 * oi[2] + d] - ci[3 * oi[1] + d];
      B0[d] = cj[3 * oj[1] + d] - S;
      B1[d] = cj[3 * oj[2] + d] - cj[3 * oj[1] + d];
    }
    // lanes over (half, xi, eta, t1); the innermost t2 moves the source point
    // linearly (r = R0 + t2 R1) with the target's barycentrics fixed: its
    // products with lambda_b are summed over t2 first
    const double nn = ni[0] * nj[0] + ni[1] * nj[1] + ni[2] * nj[2];
    for (int p = lane; p < 2 * n3; p += 64) {
      const int half = p / n3, rem = p - half * n3;
      const int ia = rem / n2, ib = (rem / n) % n, ic = rem % n;
      const double xi = gx[ia], eta = gx[ib], t1 = gx[ic];
      const double wb = gw[ia] * gw[ib] * gw[ic] * xi * xi * xi * eta;
      const double x1 = half == 0 ? xi : xi * eta;
      const double y1 = half == 0 ? xi * eta : xi;
      double R0[3], R1[3];
      for (int d = 0; d < 3; ++d) {
        R0[d] = x1 * (A0[d] + t1 * A1[d]) - y1 * B0[d];
        R1[d] = -y1 * B1[d];
      }
      const LinSep L = lin_sep(R0, R1, ni, nj);
      double sb[3][6];
#pragma unroll
      for (int y = 0; y < 3; ++y)
#pragma unroll
        for (int m = 0; m < 6; ++m) sb[y][m] = 0.0;
      for (int id = 0; id < n; ++id) {
        const double t2 = gx[id], w = wb * gw[id];
        kernel6s(fma(t2, fma(t2, L.c, L.b), L.a), fma(t2, L.p1, L.p0), fma(t2, L.q1, L.q0), nn, a.kappa, k6);
        bary(y1, y1 * t2, lb);
#pragma unroll
        for (int y = 0; y < 3; ++y) {
          const double wy = w * lb[y];
#pragma unroll
          for (int m = 0; m < 6; ++m) sb[y][m] += wy * k6[m];
        }
      }
      bary(x1, x1 * t1, la);
#pragma unroll
      for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y)
#pragma unroll
          for (int m = 0; m < 6; ++m) acc[x][y][m] += la[x] * sb[y][m];
    }
    scale = 4.0 * a.pa[i] * a.pa[j];
  } else {  // CLOSE
    const double wij = 4.0 * a.pa[i] * a.pa[j];
    const double nn = ni[0] * nj[0] + ni[1] * nj[1] + ni[2] * nj[2];
    // lanes over (s1, t1, s2), the innermost t2 as in the vertex rule
    for (int p = lane; p < n3; p += 64) {
      const int ia = p / n2, ib = (p / n) % n, ic = p % n;
      const double s1 = gx[ia], t1 = gx[ib], s2 = gx[ic];
      const double wb = wij * gw[ia] * gw[ib] * s1 * gw[ic] * s2;
      double R0[3], R1[3];
      for (int d = 0; d < 3; ++d) {
        const double x = ci[d] + s1 * (ci[3 + d] - ci[d]) + s1 * t1 * (ci[6 + d] - ci[3 + d]);
        R0[d] = x - (cj[d] + s2 * (cj[3 + d] - cj[d]));
        R1[d] = -s2 * (cj[6 + d] - cj[3 + d]);
      }
      const LinSep L = lin_sep(R0, R1, ni, nj);
      double sb[3][6];
#pragma unroll
      for (int y = 0; y < 3; ++y)
#pragma unroll
        for (int m = 0; m < 6; ++m) sb[y][m] = 0.0;
      for (int id = 0; id < n; ++id) {
        const double t2 = gx[id], w = wb * gw[id];
        kernel6s(fma(t2, fma(t2, L.c, L.b), L.a), fma(t2, L.p1, L.p0), fma(t2, L.q1, L.q0), nn, a.kappa, k6);
        bary(s2, s2 * t2, lb);
#pragma unroll
        for (int y = 0; y < 3; ++y) {
          const double wy = w * lb[y];
#pragma unroll
          for (int m = 0; m < 6; ++m) sb[y][m] += wy * k6[m];
        }
      }
      bary(s1, s1 * t1, la);
#pragma unroll
      for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y)
#pragma unroll
          for (int m = 0; m < 6; ++m) acc[x][y][m] += la[x] * sb[y][m];
    }
  }
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int y = 0; y < 3; ++y)
#pragma unroll
      for (int m = 0; m < 6; ++m) acc[x][y][m] = wave_sum(acc[x][y][m]);
  if (lane != 0) return;
  // the pair's place: row of i in its leaf, column of j in that leaf's sources
  const int c1 = a.leaf_of[i];
  const int r1 = i - a.leaf_start[c1];
  const int S1 = (int)(a.src_off[c1 + 1] - a.src_off[c1]);
  const int k1 = (int)(item.ent - a.ent_off[c1]) - r1 * S1;
  const int64_t b1 = 9 * a.ent_off[c1] + (int64_t)(3 * r1) * (3 * S1) + 3 * k1;
  const double mass = a.pa[i] / 12.0;
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int y = 0; y < 3; ++y)
      ent[b1 + (int64_t)oi[x] * (3 * S1) + oj[y]] =
          hat_entry(acc[x][y], scale, a.eps, CLS == C_IDENT ? mass * (x == y ? 2.0 : 1.0) : 0.0);
  if (CLS == C_IDENT) return;
  // the mirrored pair (target j, source i)
  const int c2 = a.leaf_of[j];
  const int r2 = j - a.leaf_start[c2];
  const int S2 = (int)(a.src_off[c2 + 1] - a.src_off[c2]);
  int col = -1;
  for (int q = a.lnbr_off[c2]; q < a.lnbr_off[c2 + 1]; ++q)
    if (a.lnbr[q] == c1) col = a.lnbr_col[q] + r1;
  if (col < 0) return;
  const int64_t b2 = 9 * a.ent_off[c2] + (int64_t)(3 * r2) * (3 * S2) + 3 * col;
#pragma unroll
  for (int x = 0; x < 3; ++x)
#pragma unroll
    for (int y = 0; y < 3; ++y) {
      const double* I = acc[x][y];
      const double It[6] = {I[0], I[3], I[4], I[1], I[2], I[5]};
      ent[b2 + (int64_t)oj[y] * (3 * S2) + oi[x]] = hat_entry(It, scale, a.eps, 0.0);
    }
}

// the far field's element rows: leaf ranges, identity outputs, leaf of each
__global__ void k_hat_layout(const int32_t* __restrict__ leaf_start, const int32_t* __restrict__ leaf_cnt,
                             const int32_t* __restrict__ leaf_of, int nl, int64_t n_iota, int64_t N, int32_t* ls3,
                             int32_t* lc3, int32_t* iota, int32_t* lo3) {
  const int64_t m = max(max((int64_t)nl, n_iota), 3 * N);
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < m; g += (int64_t)gridDim.x * blockDim.x) {
    if (g < nl) {
      ls3[g] = 3 * leaf_start[g];
      lc3[g] = 3 * leaf_cnt[g];
    }
    if (g < n_iota) iota[g] = (int32_t)g;
    if (g < 3 * N) lo3[g] = leaf_of[g / 3];
  }
}

// ---------------------------------------------------------------------------
// Near field by vertex pairs.  For leaf c the corner rows (3 n_c) and the
// source corners (3 S_c) are sorted by vertex (key = vertex << 20 | local
// index, bitonic sort in LDS); each run of equal vertices is one row or one
// column, and the entry of (row r, column k) is the sum over the corners of
// run r and of run k of the corner entries, in run order.
// ---------------------------------------------------------------------------
constexpr int VB_ROWS = 128;       // >= 3 x the largest leaf (leaf_size <= 32)
constexpr int VB_SHIFT = 20;       // local corner index bits

__device__ inline void bitonic(uint64_t* k, int n) {
  for (int size = 2; size <= n; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int t = threadIdx.x; t < n / 2; t += blockDim.x) {
        const int i = 2 * t - (t & (stride - 1)), j = i + stride;
        const bool up = (i & size) == 0;
        const uint64_t a = k[i], b = k[j];
        if ((a > b) == up) {
          k[i] = b;
          k[j] = a;
        }
      }
    }
  __syncthreads();
}

__device__ inline int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// sorted keys of the leaf's corner rows (rk, n_r) and source corners (ck, n_c);
// run starts (rs, cs: run u at [rs[u], rs[u + 1])) and run counts
struct VbLeaf {
  int nr, nc, ur, uc;
};

// the first index of every run of equal vertices in key[0..n) (sorted),
// starts[runs] = n; flags per thread chunk, a block scan of their counts,
// then each thread writes its chunk's starts (blockDim.x threads, sc: as many
// ints of LDS)
__device__ inline int vb_runs(const uint64_t* key, int n, int* starts, int* sc) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int per = (n + nt - 1) / nt;
  const int t0 = min(n, tid * per), t1 = min(n, t0 + per);
  int f = 0;
  for (int t = t0; t < t1; ++t) f += (t == 0 || (key[t] >> VB_SHIFT) != (key[t - 1] >> VB_SHIFT)) ? 1 : 0;
  sc[tid] = f;
  __syncthreads();
  for (int o = 1; o < nt; o <<= 1) {   // inclusive scan
    const int v = tid >= o ? sc[tid - o] : 0;
    __syncthreads();
    sc[tid] += v;
    __syncthreads();
  }
  int u = sc[tid] - f;
  for (int t = t0; t < t1; ++t)
    if (t == 0 || (key[t] >> VB_SHIFT) != (key[t - 1] >> VB_SHIFT)) starts[u++] = t;
  const int runs = sc[nt - 1];
  if (tid == 0) starts[runs] = n;
  __syncthreads();   // starts written; sc free again
  return runs;
}

__device__ inline VbLeaf vb_sort(const NearArgs& a, int c, uint64_t* rk, uint64_t* ck, int* rs, int* cs) {
  const int nrow = a.leaf_cnt[c], i0 = a.leaf_start[c];
  const int64_t so = a.src_off[c];
  const int S = (int)(a.src_off[c + 1] - so);
  VbLeaf L{3 * nrow, 3 * S, 0, 0};
  const int pr = pow2_at_least(L.nr), pc = pow2_at_least(L.nc);
  for (int t = threadIdx.x; t < pr; t += blockDim.x)
    rk[t] = t < L.nr ? ((uint64_t)(uint32_t)a.ptri[3 * i0 + t] << VB_SHIFT) | (uint64_t)t : ~0ull;
  for (int t = threadIdx.x; t < pc; t += blockDim.x)
    ck[t] = t < L.nc ? ((uint64_t)(uint32_t)a.ptri[3 * a.src_tree[so + t / 3] + t % 3] << VB_SHIFT) | (uint64_t)t
                     : ~0ull;
  bitonic(rk, pr);
  bitonic(ck, pc);
  __shared__ int sc[256];
  L.ur = vb_runs(rk, L.nr, rs, sc);
  L.uc = vb_runs(ck, L.nc, cs, sc);
  return L;
}

// pass 0: rows, columns and entries per leaf
__global__ void __launch_bounds__(256) k_vb_count(NearArgs a, int max_pc, int64_t* nrow, int64_t* ncol,
                                                  int64_t* nent) {
  extern __shared__ uint64_t lds[];
  uint64_t* rk = lds;
  uint64_t* ck = rk + VB_ROWS;
  int* rs = reinterpret_cast<int*>(ck + max_pc);
  int* cs = rs + VB_ROWS + 1;
  const int c = blockIdx.x;
  const VbLeaf L = vb_sort(a, c, rk, ck, rs, cs);
  if (threadIdx.x == 0) {
    nrow[c] = L.ur;
    ncol[c] = L.uc;
    nent[c] = (int64_t)L.ur * L.uc;
  }
}

// pass 1: the lists, and the entries summed from the corner entries E (FP64)
__global__ void __launch_bounds__(256) k_vb_build(NearArgs a, int max_pc, const double4* __restrict__ E,
                                                  const int64_t* __restrict__ row_off,
                                                  const int64_t* __restrict__ col_off,
                                                  const int64_t* __restrict__ ent_off, int32_t* row_start,
                                                  int32_t* row_cnt, int32_t* col_elem, int32_t* col_vert,
                                                  int32_t* row_vert, int32_t* row_leaf, double4* V) {
  extern __shared__ uint64_t lds[];
  uint64_t* rk = lds;
  uint64_t* ck = rk + VB_ROWS;
  int* rs = reinterpret_cast<int*>(ck + max_pc);
  int* cs = rs + VB_ROWS + 1;
  const int c = blockIdx.x;
  const VbLeaf L = vb_sort(a, c, rk, ck, rs, cs);
  const int64_t so = a.src_off[c];
  const int S3 = L.nc;
  const uint64_t mask = (1ull << VB_SHIFT) - 1;
  const int64_t r0 = row_off[c], c0 = col_off[c], e0 = ent_off[c];
  if (threadIdx.x == 0) {
    row_start[c] = (int32_t)r0;
    row_cnt[c] = L.ur;
  }
  for (int u = threadIdx.x; u < L.uc; u += blockDim.x) {
    const int f = (int)(ck[cs[u]] & mask);
    col_elem[c0 + u] = 3 * a.src_tree[so + f / 3] + f % 3;
    col_vert[c0 + u] = (int32_t)(ck[cs[u]] >> VB_SHIFT);
  }
  for (int u = threadIdx.x; u < L.ur; u += blockDim.x) {
    row_vert[r0 + u] = (int32_t)(rk[rs[u]] >> VB_SHIFT);
    row_leaf[r0 + u] = c;
  }
  const double4* Ec = E + 9 * a.ent_off[c];
  for (int p = threadIdx.x; p < L.ur * L.uc; p += blockDim.x) {
    const int r = p / L.uc, k = p - r * L.uc;
    double4 acc = make_double4(0.0, 0.0, 0.0, 0.0);
    for (int x = rs[r]; x < rs[r + 1]; ++x) {
      const double4* row = Ec + (int64_t)(rk[x] & mask) * S3;
      for (int y = cs[k]; y < cs[k + 1]; ++y) {
        const double4 e = row[ck[y] & mask];
        acc.x += e.x;
        acc.y += e.y;
        acc.z += e.z;
        acc.w += e.w;
      }
    }
    V[e0 + p] = acc;
  }
}

// y[v] = the corner rows of vertex v (far field) plus its near rows (when
// given), both channels
__global__ void k_hat_gather(const int32_t* __restrict__ off, const int32_t* __restrict__ el,
                             const int32_t* __restrict__ poff, const int32_t* __restrict__ pr, int64_t nv,
                             int64_t n3, int64_t nr, const double* __restrict__ rows,
                             const double* __restrict__ near_rows, double* y) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double s1 = 0, s2 = 0;
  for (int k = off[v]; k < off[v + 1]; ++k) {
    const int e = el[k];
    s1 += rows[e];
    s2 += rows[n3 + e];
  }
  if (near_rows)
    for (int k = poff[v]; k < poff[v + 1]; ++k) {
      const int r = pr[k];
      s1 += near_rows[r];
      s2 += near_rows[nr + r];
    }
  y[v] = s1;
  y[nv + v] = s2;
}

// diagonal of A at vertex v: in each of its near rows, the column of v
__global__ void k_hat_diag(const double4* __restrict__ V, const int32_t* __restrict__ poff,
                           const int32_t* __restrict__ pr, const int32_t* __restrict__ row_leaf,
                           const int32_t* __restrict__ row_start, const int64_t* __restrict__ col_off,
                           const int64_t* __restrict__ ent_off, const int32_t* __restrict__ col_vert, int64_t nv,
                           double* diag) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nv) return;
  double d1 = 0, d2 = 0;
  for (int k = poff[v]; k < poff[v + 1]; ++k) {
    const int r = pr[k], c = row_leaf[r];
    const int64_t c0 = col_off[c];
    const int nc = (int)(col_off[c + 1] - c0);
    int lo = 0, hi = nc;   // columns ascending by vertex
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (col_vert[c0 + mid] < v) lo = mid + 1; else hi = mid;
    }
    if (lo < nc && col_vert[c0 + lo] == v) {
      const double4 e = V[ent_off[c] + (int64_t)(r - row_start[c]) * nc + lo];
      d1 += e.x;
      d2 += e.w;
    }
  }
  diag[v] = d1;
  diag[nv + v] = d2;
}

ElemView hat_view(fagbi_handle* h) {
  ElemView v;
  v.n = 3 * h->N;
  v.leaf_start = h->d_s1_leaf_start.as<int32_t>();
  v.leaf_cnt = h->d_s1_leaf_cnt.as<int32_t>();
  v.leaf_of = h->d_s1_leaf_of.as<int32_t>();
  v.in_idx = h->d_ptri.as<int32_t>();     // vertex of corner e = 3 i + a
  v.out_idx = h->d_s1_iota.as<int32_t>();
  v.in_stride = h->nv;
  v.xt = h->d_xt.as<double>();
  v.y = h->d_ye.as<double>();
  v.n_near = h->n_vb_rows;
  v.near_start = h->d_vb_row_start.as<int32_t>();
  v.near_cnt = h->d_vb_row_cnt.as<int32_t>();
  v.near_src = h->d_vb_col_elem.as<int32_t>();
  v.near_src_off = h->d_vb_col_off.as<int64_t>();
  v.near_ent_off = h->d_vb_ent_off.as<int64_t>();
  v.out_near = h->d_s1_iota.as<int32_t>();
  v.y_near = h->d_ye.as<double>() + 6 * h->N;
  v.zero_y = true;
  v.gather = true;
  return v;
}

int hat_gather(fagbi_handle* h, const double* rows, const double* near_rows, double* y, hipStream_t s) {
  k_hat_gather<<<(unsigned)((h->nv + 255) / 256), 256, 0, s>>>(
      h->d_vx_off.as<int32_t>(), h->d_vx_el.as<int32_t>(), h->d_vx_poff.as<int32_t>(), h->d_vx_pr.as<int32_t>(),
      h->nv, 3 * h->N, h->n_vb_rows, rows, near_rows, y);
  FAGBI_HIP(hipGetLastError());
  return 0;
}

// CSR of the items of each of nv keys, items ascending
static void key_lists(const std::vector<int32_t>& key, int64_t nv, std::vector<int32_t>& off,
                      std::vector<int32_t>& el) {
  off.assign(nv + 1, 0);
  el.resize(key.size());
  for (size_t e = 0; e < key.size(); ++e) ++off[key[e] + 1];
  for (int64_t v = 0; v < nv; ++v) off[v + 1] += off[v];
  std::vector<int32_t> pos(off.begin(), off.end() - 1);
  for (size_t e = 0; e < key.size(); ++e) el[pos[key[e]]++] = (int32_t)e;
}

// corner entries of every stored pair (the worklists of the singular and
// close pairs are built by the classification) into a temporary array, their
// sums by vertex pairs into the handle's entries (FP64 and FP32), the element
// layout and the vertex lists
int hat_assemble(fagbi_handle* h, hipStream_t s) {
  const int nl = h->lev[h->L].n;
  const int64_t N = h->N;
  NearArgs a = near_args(h);
  Tmp Ebuf;
  FAGBI_TRY(Ebuf.alloc((size_t)9 * h->n_ent * sizeof(double4)));
  double4* E = Ebuf.as<double4>();
  k_hat_regular<<<nl, 256, 0, s>>>(a, E);
  FAGBI_HIP(hipGetLastError());
  const int n = h->prm.quad_duffy;
  const double* gl = h->d_gl.as<double>();
  for (int k = 0; k < 4; ++k) {
    const int64_t m = h->wl_n[k];
    if (m == 0) continue;
    const Item* it = h->d_wl[k].as<Item>();
    switch (k) {
      case 0: k_hat_singular<C_IDENT><<<(unsigned)m, 64, 0, s>>>(a, it, m, gl, n, E); break;
      case 1: k_hat_singular<C_EDGE><<<(unsigned)m, 64, 0, s>>>(a, it, m, gl, n, E); break;
      case 2: k_hat_singular<C_VERTEX><<<(unsigned)m, 64, 0, s>>>(a, it, m, gl, n, E); break;
      default: k_hat_singular<C_CLOSE><<<(unsigned)m, 64, 0, s>>>(a, it, m, gl, n, E); break;
    }
    FAGBI_HIP(hipGetLastError());
  }
  // vertex-pair layout: the longest source list sets the sort's LDS
  std::vector<int64_t> soff(nl + 1);
  FAGBI_HIP(hipMemcpyAsync(soff.data(), h->d_src_off.p, (nl + 1) * 8, hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipStreamSynchronize(s));
  int max_s = 0;
  for (int c = 0; c < nl; ++c) max_s = std::max<int>(max_s, (int)(soff[c + 1] - soff[c]));
  int max_pc = 1;
  while (max_pc < 3 * max_s) max_pc <<= 1;
  const size_t lds = (size_t)(VB_ROWS + max_pc) * 8 + (size_t)(VB_ROWS + 1 + max_pc + 1 + 2) * 4;
  if (lds > 150 * 1024)
    return set_error(FAGBI_E_ARG, "a leaf's source list (%d panels) is too long for the hat-function layout",
                     max_s);
  FAGBI_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_vb_count),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  FAGBI_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_vb_build),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  Tmp cnt, off, part;
  FAGBI_TRY(cnt.alloc((size_t)3 * nl * 8));
  FAGBI_TRY(off.alloc((size_t)3 * (nl + 1) * 8));
  FAGBI_TRY(part.alloc((size_t)scan_part_size(nl) * 8));
  int64_t* c_row = cnt.as<int64_t>();
  int64_t *o_row = off.as<int64_t>(), *o_col = o_row + (nl + 1), *o_ent = o_col + (nl + 1);
  k_vb_count<<<nl, 256, lds, s>>>(a, max_pc, c_row, c_row + nl, c_row + 2 * nl);
  FAGBI_HIP(hipGetLastError());
  FAGBI_TRY((device_scan<int64_t, int64_t>(c_row, nl, o_row, part.as<int64_t>(), s)));
  FAGBI_TRY((device_scan<int64_t, int64_t>(c_row + nl, nl, o_col, part.as<int64_t>(), s)));
  FAGBI_TRY((device_scan<int64_t, int64_t>(c_row + 2 * nl, nl, o_ent, part.as<int64_t>(), s)));
  int64_t tot[3];
  FAGBI_HIP(hipMemcpyAsync(&tot[0], o_row + nl, 8, hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipMemcpyAsync(&tot[1], o_col + nl, 8, hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipMemcpyAsync(&tot[2], o_ent + nl, 8, hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipStreamSynchronize(s));
  h->n_vb_rows = tot[0];
  h->n_vb_ent = tot[2];
  FAGBI_TRY(h->alloc(h->d_vb_row_start, (size_t)nl * 4));
  FAGBI_TRY(h->alloc(h->d_vb_row_cnt, (size_t)nl * 4));
  FAGBI_TRY(h->alloc(h->d_vb_col_off, (size_t)(nl + 1) * 8));
  FAGBI_TRY(h->alloc(h->d_vb_ent_off, (size_t)(nl + 1) * 8));
  FAGBI_TRY(h->alloc(h->d_vb_col_elem, (size_t)std::max<int64_t>(1, tot[1]) * 4));
  FAGBI_TRY(h->alloc(h->d_vb_col_vert, (size_t)std::max<int64_t>(1, tot[1]) * 4));
  FAGBI_TRY(h->alloc(h->d_vb_row_vert, (size_t)std::max<int64_t>(1, tot[0]) * 4));
  FAGBI_TRY(h->alloc(h->d_vb_row_leaf, (size_t)std::max<int64_t>(1, tot[0]) * 4));
  FAGBI_TRY(h->alloc(h->d_E64, (size_t)std::max<int64_t>(1, tot[2]) * sizeof(double4)));
  FAGBI_TRY(h->alloc(h->d_E32, (size_t)std::max<int64_t>(1, tot[2]) * sizeof(float4)));
  FAGBI_HIP(hipMemcpyAsync(h->d_vb_col_off.p, o_col, (nl + 1) * 8, hipMemcpyDeviceToDevice, s));
  FAGBI_HIP(hipMemcpyAsync(h->d_vb_ent_off.p, o_ent, (nl + 1) * 8, hipMemcpyDeviceToDevice, s));
  k_vb_build<<<nl, 256, lds, s>>>(a, max_pc, E, o_row, o_col, o_ent, h->d_vb_row_start.as<int32_t>(),
                                  h->d_vb_row_cnt.as<int32_t>(), h->d_vb_col_elem.as<int32_t>(),
                                  h->d_vb_col_vert.as<int32_t>(), h->d_vb_row_vert.as<int32_t>(),
                                  h->d_vb_row_leaf.as<int32_t>(), h->d_E64.as<double4>());
  FAGBI_HIP(hipGetLastError());
  // the far field's element rows
  const int64_t n_iota = std::max<int64_t>(3 * N, tot[0]);
  FAGBI_TRY(h->alloc(h->d_s1_leaf_start, (size_t)nl * 4));
  FAGBI_TRY(h->alloc(h->d_s1_leaf_cnt, (size_t)nl * 4));
  FAGBI_TRY(h->alloc(h->d_s1_iota, (size_t)n_iota * 4));
  FAGBI_TRY(h->alloc(h->d_s1_leaf_of, (size_t)3 * N * 4));
  FAGBI_TRY(h->alloc(h->d_ye, (size_t)(6 * N + 2 * tot[0]) * 8));
  k_hat_layout<<<1024, 256, 0, s>>>(h->d_leaf_start.as<int32_t>(), h->d_leaf_cnt.as<int32_t>(),
                                    h->d_leaf_of.as<int32_t>(), nl, n_iota, N, h->d_s1_leaf_start.as<int32_t>(),
                                    h->d_s1_leaf_cnt.as<int32_t>(), h->d_s1_iota.as<int32_t>(),
                                    h->d_s1_leaf_of.as<int32_t>());
  FAGBI_HIP(hipGetLastError());
  // corners and near rows of each vertex, ascending (counting sorts on the host)
  std::vector<int32_t> ev(3 * N), rv(tot[0]);
  FAGBI_HIP(hipMemcpyAsync(ev.data(), h->d_ptri.p, 3 * N * 4, hipMemcpyDeviceToHost, s));
  if (tot[0] > 0) FAGBI_HIP(hipMemcpyAsync(rv.data(), h->d_vb_row_vert.p, tot[0] * 4, hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipStreamSynchronize(s));
  std::vector<int32_t> voff, vel, poff, pel;
  key_lists(ev, h->nv, voff, vel);
  key_lists(rv, h->nv, poff, pel);
  FAGBI_TRY(h->upload(h->d_vx_off, voff.data(), voff.size() * 4));
  FAGBI_TRY(h->upload(h->d_vx_el, vel.data(), vel.size() * 4));
  FAGBI_TRY(h->upload(h->d_vx_poff, poff.data(), poff.size() * 4));
  FAGBI_TRY(h->upload(h->d_vx_pr, pel.data(), std::max<size_t>(1, pel.size()) * 4));
  return 0;
}

int hat_diag_setup(fagbi_handle* h, hipStream_t s) {
  FAGBI_TRY(h->alloc(h->d_diag, 2 * h->nv * sizeof(double)));
  k_hat_diag<<<(unsigned)((h->nv + 255) / 256), 256, 0, s>>>(
      h->d_E64.as<double4>(), h->d_vx_poff.as<int32_t>(), h->d_vx_pr.as<int32_t>(), h->d_vb_row_leaf.as<int32_t>(),
      h->d_vb_row_start.as<int32_t>(), h->d_vb_col_off.as<int64_t>(), h->d_vb_ent_off.as<int64_t>(),
      h->d_vb_col_vert.as<int32_t>(), h->nv, h->d_diag.as<double>());
  FAGBI_HIP(hipGetLastError());
  return 0;
}

}  // namespace fagbi
