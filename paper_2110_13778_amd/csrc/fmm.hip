// Matrix-vector product y = A x: stored near field (block SpMV) plus the
// Cartesian Taylor FMM far field (paper Sec. 2.4: moments, MtM, MtL, LtL, LtP
// and the six-step algorithm), in FP64 or FP32 (FP64 accumulation of y).
//
// Conventions:
//  * multi-indices alpha = (a, b, c), |alpha| <= p, ordered by total degree,
//    then a descending, then b descending; orders <= p form a prefix;
//  * two expansion channels: G0 with moments M0 = m_s(dphi) - m_d(phi) and
//    Gk with Mk = -m_s(dphi) + eps m_d(phi); row 1 of the far field is
//    -(lambda0 + lambdak) tested with m_s, row 2 is -(lambda0 + lambdak/eps)
//    tested with m_d (K1..K4 of Sec. 2.2 share these expansions);
//  * MtL: lambda^a += sum_{|a|+|b| <= p} (a+b)!/(a! b!) (-1)^|b| F_{a+b}(x0)/(4 pi) M^b
//    with x0 = x_c - x_c' = (idx_c - idx_c') h_l and F the Taylor coefficients
//    of exp(-kappa r)/r; one table of F per (level, offset);
//  * MtM / LtL: binomial shifts by the child-parent centre offset
//    (+-h_{l+1}/2 per axis); variable order: a parent of order p_l gathers
//    its children's moments of order p_{l+1}, and shifted parent locals are
//    truncated to p_{l+1};
//  * leaf moments use the 3-point rule of the regular near field.
#include <cmath>

#include "internal.h"

namespace fagbi {

__host__ __device__ inline int midx(int a, int b, int c) {
  const int d = a + b + c;
  const int below = d * (d + 1) * (d + 2) / 6;
  return below + (d - a) * (d - a + 1) / 2 + (d - a - b);
}

__constant__ double c_binom[PMAX + 1][PMAX + 1];

// ---------------------------------------------------------------------------
// host: Taylor coefficients by the recurrence (derived from
// r^2 grad f = -x (f + kappa h), grad h = -kappa x f for f = exp(-kappa r)/r,
// h = exp(-kappa r), comparing coefficients after applying the Euler
// operator):
//   |k| r0^2 F_k + (2|k|-1) sum_i x0_i F_{k-e_i} + (|k|-1) sum_i F_{k-2e_i}
//       = -kappa [sum_i x0_i H_{k-e_i} + sum_i H_{k-2e_i}]
//   |k| H_k = -kappa [sum_i x0_i F_{k-e_i} + sum_i F_{k-2e_i}]
// ---------------------------------------------------------------------------
static void taylor_host(const double x0[3], double kappa, int p, double* F) {
  const int T = nterms(p);
  std::vector<double> H(T, 0.0);
  const double r2 = x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2];
  const double r0 = std::sqrt(r2);
  F[0] = std::exp(-kappa * r0) / r0;
  H[0] = std::exp(-kappa * r0);
  for (int d = 1; d <= p; ++d)
    for (int a = d; a >= 0; --a)
      for (int b = d - a; b >= 0; --b) {
        const int c = d - a - b;
        const int k[3] = {a, b, c};
        double s1f = 0, s2f = 0, s1h = 0, s2h = 0;
        for (int ax = 0; ax < 3; ++ax) {
          int m1[3] = {a, b, c}, m2[3] = {a, b, c};
          m1[ax] -= 1;
          m2[ax] -= 2;
          if (k[ax] >= 1) {
            const int id = midx(m1[0], m1[1], m1[2]);
            s1f += x0[ax] * F[id];
            s1h += x0[ax] * H[id];
          }
          if (k[ax] >= 2) {
            const int id = midx(m2[0], m2[1], m2[2]);
            s2f += F[id];
            s2h += H[id];
          }
        }
        const int id = midx(a, b, c);
        F[id] = (-kappa * (s1h + s2h) - (2 * d - 1) * s1f - (d - 1) * s2f) / (d * r2);
        H[id] = -kappa * (s1f + s2f) / d;
      }
}

static double fact(int n) {
  double f = 1;
  for (int k = 2; k <= n; ++k) f *= k;
  return f;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
struct MiTab {
  const int8_t* mi;       // [TMAX][3]
  const int16_t* gidx;    // [TMAX][TMAX] index of alpha+beta, -1 if |.| > PMAX
};

// single/double layer moments of each panel about its leaf centre
template <typename R>
__global__ void k_panel_moments(const double* __restrict__ pv, const double* __restrict__ pn,
                                const double* __restrict__ pa, const int32_t* __restrict__ leaf_of,
                                const int32_t* __restrict__ lidx, double cx, double cy, double cz,
                                double hL, int N, int T, const int8_t* __restrict__ mi, R* ms, R* md) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)N * T) return;
  const int i = (int)(g / T), t = (int)(g - (int64_t)i * T);
  const int c = leaf_of[i];
  const double ctr[3] = {cx + ((double)lidx[3 * c] + 0.5) * hL, cy + ((double)lidx[3 * c + 1] + 0.5) * hL,
                         cz + ((double)lidx[3 * c + 2] + 0.5) * hL};
  const int e[3] = {mi[3 * t], mi[3 * t + 1], mi[3 * t + 2]};
  const double* v = pv + 9 * (int64_t)i;
  const double w = pa[i] / 3.0;
  double s = 0, dsum = 0;
  for (int k = 0; k < 3; ++k) {
    double d[3];
    for (int ax = 0; ax < 3; ++ax)
      d[ax] = (2.0 / 3.0) * v[3 * k + ax] + (1.0 / 6.0) * (v[3 * ((k + 1) % 3) + ax] + v[3 * ((k + 2) % 3) + ax]) -
              ctr[ax];
    double pw[3][PMAX + 1];
    for (int ax = 0; ax < 3; ++ax) {
      pw[ax][0] = 1.0;
      for (int q = 1; q <= e[ax]; ++q) pw[ax][q] = pw[ax][q - 1] * d[ax];
    }
    s += w * pw[0][e[0]] * pw[1][e[1]] * pw[2][e[2]];
    double g2 = 0;
    if (e[0]) g2 += e[0] * pn[3 * i] * pw[0][e[0] - 1] * pw[1][e[1]] * pw[2][e[2]];
    if (e[1]) g2 += e[1] * pn[3 * i + 1] * pw[0][e[0]] * pw[1][e[1] - 1] * pw[2][e[2]];
    if (e[2]) g2 += e[2] * pn[3 * i + 2] * pw[0][e[0]] * pw[1][e[1]] * pw[2][e[2] - 1];
    dsum += w * g2;
  }
  ms[g] = (R)s;
  md[g] = (R)dsum;
}

// P2M: one block per leaf, threads over terms
template <typename R>
__global__ void k_p2m(const R* __restrict__ ms, const R* __restrict__ md, const int32_t* leaf_start,
                      const int32_t* leaf_cnt, const int32_t* __restrict__ perm, int64_t N, int T,
                      double eps, const double* __restrict__ x, R* M0, R* Mk) {
  const int c = blockIdx.x;
  const int i0 = leaf_start[c], n = leaf_cnt[c];
  for (int t = threadIdx.x; t < T; t += blockDim.x) {
    R a0 = 0, ak = 0;
    for (int i = i0; i < i0 + n; ++i) {
      const int p = perm[i];
      const R phi = (R)x[p], dphi = (R)x[N + p];
      const R s = ms[(int64_t)i * T + t], d = md[(int64_t)i * T + t];
      a0 += s * dphi - d * phi;
      ak += -s * dphi + (R)eps * d * phi;
    }
    M0[(int64_t)c * T + t] = a0;
    Mk[(int64_t)c * T + t] = ak;
  }
}

// MtM: parent^alpha = sum_children sum_{beta <= alpha, |beta| <= p_child}
//        C(alpha, beta) d^(alpha - beta) child^beta
template <typename R>
__global__ void k_m2m(const int32_t* child_start, const int32_t* child_end, const int32_t* cidx,
                      double hc, int Tp, int pc, int Tc, const int8_t* __restrict__ mi,
                      const R* __restrict__ C0, const R* __restrict__ Ck, R* P0, R* Pk) {
  const int c = blockIdx.x;
  for (int t = threadIdx.x; t < Tp; t += blockDim.x) {
    const int a[3] = {mi[3 * t], mi[3 * t + 1], mi[3 * t + 2]};
    R s0 = 0, sk = 0;
    for (int ch = child_start[c]; ch < child_end[c]; ++ch) {
      double d[3];
      for (int ax = 0; ax < 3; ++ax) d[ax] = ((cidx[3 * ch + ax] & 1) - 0.5) * hc;
      for (int b0 = 0; b0 <= a[0]; ++b0)
        for (int b1 = 0; b1 <= a[1]; ++b1)
          for (int b2 = 0; b2 <= a[2] && b0 + b1 + b2 <= pc; ++b2) {
            double coef = c_binom[a[0]][b0] * c_binom[a[1]][b1] * c_binom[a[2]][b2];
            for (int q = 0; q < a[0] - b0; ++q) coef *= d[0];
            for (int q = 0; q < a[1] - b1; ++q) coef *= d[1];
            for (int q = 0; q < a[2] - b2; ++q) coef *= d[2];
            const int bi = midx(b0, b1, b2);
            s0 += (R)coef * C0[(int64_t)ch * Tc + bi];
            sk += (R)coef * Ck[(int64_t)ch * Tc + bi];
          }
    }
    P0[(int64_t)c * Tp + t] = s0;
    Pk[(int64_t)c * Tp + t] = sk;
  }
}

// MtL: one block per target cluster, threads over alpha
template <typename R>
__global__ void k_m2l(const int32_t* __restrict__ inter_off, const int32_t* __restrict__ inter_src,
                      const int32_t* __restrict__ inter_oid, const R* __restrict__ F0,
                      const R* __restrict__ Fk, const R* __restrict__ coef, const int16_t* __restrict__ gidx,
                      const int8_t* __restrict__ mi, int p, int T, const R* __restrict__ M0,
                      const R* __restrict__ Mk, R* L0, R* Lk) {
  const int c = blockIdx.x;
  for (int t = threadIdx.x; t < T; t += blockDim.x) {
    const int da = mi[3 * t] + mi[3 * t + 1] + mi[3 * t + 2];
    const int nb = nterms(p - da);
    R l0 = 0, lk = 0;
    for (int q = inter_off[c]; q < inter_off[c + 1]; ++q) {
      const int src = inter_src[q];
      const R* f0 = F0 + (int64_t)inter_oid[q] * T;
      const R* fk = Fk + (int64_t)inter_oid[q] * T;
      const R* m0 = M0 + (int64_t)src * T;
      const R* mk = Mk + (int64_t)src * T;
      for (int b = 0; b < nb; ++b) {
        const int g = gidx[t * TMAX + b];
        const R cf = coef[t * TMAX + b];
        l0 += cf * f0[g] * m0[b];
        lk += cf * fk[g] * mk[b];
      }
    }
    L0[(int64_t)c * T + t] += l0;
    Lk[(int64_t)c * T + t] += lk;
  }
}

// LtL: child^beta += sum_{alpha >= beta, |alpha| <= p_parent} C(alpha,beta) d^(alpha-beta) parent^alpha
template <typename R>
__global__ void k_l2l(const int32_t* parent, const int32_t* cidx, double hc, int pp, int Tp, int Tc,
                      const int8_t* __restrict__ mi, const R* __restrict__ P0, const R* __restrict__ Pk,
                      R* C0, R* Ck) {
  const int c = blockIdx.x;
  const int par = parent[c];
  double d[3];
  for (int ax = 0; ax < 3; ++ax) d[ax] = ((cidx[3 * c + ax] & 1) - 0.5) * hc;
  for (int t = threadIdx.x; t < Tc; t += blockDim.x) {
    const int b[3] = {mi[3 * t], mi[3 * t + 1], mi[3 * t + 2]};
    const int db = b[0] + b[1] + b[2];
    R s0 = 0, sk = 0;
    for (int g0 = 0; g0 <= pp - db; ++g0)
      for (int g1 = 0; g0 + g1 <= pp - db; ++g1)
        for (int g2 = 0; g0 + g1 + g2 <= pp - db; ++g2) {
          double coef = c_binom[b[0] + g0][b[0]] * c_binom[b[1] + g1][b[1]] * c_binom[b[2] + g2][b[2]];
          for (int q = 0; q < g0; ++q) coef *= d[0];
          for (int q = 0; q < g1; ++q) coef *= d[1];
          for (int q = 0; q < g2; ++q) coef *= d[2];
          const int ai = midx(b[0] + g0, b[1] + g1, b[2] + g2);
          s0 += (R)coef * P0[(int64_t)par * Tp + ai];
          sk += (R)coef * Pk[(int64_t)par * Tp + ai];
        }
    C0[(int64_t)c * Tc + t] += s0;
    Ck[(int64_t)c * Tc + t] += sk;
  }
}

// LtP: far-field contribution of each panel, added to y (caller order)
template <typename R>
__global__ void k_l2p(const R* __restrict__ ms, const R* __restrict__ md, const int32_t* __restrict__ leaf_of,
                      const int32_t* __restrict__ perm, int N, int T, double eps, const R* __restrict__ L0,
                      const R* __restrict__ Lk, double* y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int c = leaf_of[i];
  const R ie = (R)(1.0 / eps);
  R y1 = 0, y2 = 0;
  for (int t = 0; t < T; ++t) {
    const R l0 = L0[(int64_t)c * T + t], lk = Lk[(int64_t)c * T + t];
    y1 += (l0 + lk) * ms[(int64_t)i * T + t];
    y2 += (l0 + lk * ie) * md[(int64_t)i * T + t];
  }
  const int p = perm[i];
  y[p] -= (double)y1;
  y[N + p] -= (double)y2;
}

// near-field block SpMV: one wavefront per target panel (tree order)
template <typename E>
__global__ void __launch_bounds__(256) k_spmv(const E* __restrict__ ent, const int32_t* __restrict__ leaf_of,
                                              const int32_t* __restrict__ leaf_start,
                                              const int64_t* __restrict__ src_off,
                                              const int64_t* __restrict__ ent_off,
                                              const int32_t* __restrict__ src_user,
                                              const int32_t* __restrict__ perm, int64_t N,
                                              const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= N) return;
  const int c = leaf_of[i];
  const int64_t so = src_off[c];
  const int S = (int)(src_off[c + 1] - so);
  const E* row = ent + ent_off[c] + (i - leaf_start[c]) * (int64_t)S;
  double a1 = 0, a2 = 0;
  for (int k = lane; k < S; k += 64) {
    const int j = src_user[so + k];
    const double xj = x[j], xn = x[N + j];
    const E e = row[k];
    a1 += (double)e.x * xj + (double)e.y * xn;
    a2 += (double)e.z * xj + (double)e.w * xn;
  }
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
  if (lane == 0) {
    const int p = perm[i];
    y[p] = a1;
    y[N + p] = a2;
  }
}

// ---------------------------------------------------------------------------
// setup: translation tables, Taylor tables per (level, offset), moments
// ---------------------------------------------------------------------------
template <typename R>
static int upload_conv(fagbi_handle* h, DBuf& b, const std::vector<double>& v) {
  std::vector<R> t(v.begin(), v.end());
  return h->upload(b, t.data(), t.size() * sizeof(R));
}

int fmm_setup(fagbi_handle* h, hipStream_t s) {
  // multi-index tables
  std::vector<int8_t> mi(3 * TMAX);
  for (int d = 0; d <= PMAX; ++d)
    for (int a = d; a >= 0; --a)
      for (int b = d - a; b >= 0; --b) {
        const int t = midx(a, b, d - a - b);
        mi[3 * t] = (int8_t)a;
        mi[3 * t + 1] = (int8_t)b;
        mi[3 * t + 2] = (int8_t)(d - a - b);
      }
  std::vector<int16_t> gidx((size_t)TMAX * TMAX, -1);
  std::vector<double> coef((size_t)TMAX * TMAX, 0.0);
  for (int t = 0; t < TMAX; ++t)
    for (int u = 0; u < TMAX; ++u) {
      const int a0 = mi[3 * t], a1 = mi[3 * t + 1], a2 = mi[3 * t + 2];
      const int b0 = mi[3 * u], b1 = mi[3 * u + 1], b2 = mi[3 * u + 2];
      if (a0 + a1 + a2 + b0 + b1 + b2 > PMAX) continue;
      gidx[(size_t)t * TMAX + u] = (int16_t)midx(a0 + b0, a1 + b1, a2 + b2);
      const double num = fact(a0 + b0) * fact(a1 + b1) * fact(a2 + b2);
      const double den = fact(a0) * fact(a1) * fact(a2) * fact(b0) * fact(b1) * fact(b2);
      const double sg = ((b0 + b1 + b2) & 1) ? -1.0 : 1.0;
      coef[(size_t)t * TMAX + u] = sg * num / den / FOUR_PI;
    }
  FAGBI_TRY(h->upload(h->d_mi, mi.data(), mi.size()));
  FAGBI_TRY(h->upload(h->d_gidx, gidx.data(), gidx.size() * 2));
  FAGBI_TRY(upload_conv<double>(h, h->d_coef64, coef));
  FAGBI_TRY(upload_conv<float>(h, h->d_coef32, coef));
  double binom[PMAX + 1][PMAX + 1] = {};
  for (int n = 0; n <= PMAX; ++n) {
    binom[n][0] = 1;
    for (int k = 1; k <= n; ++k) binom[n][k] = binom[n - 1][k - 1] + (k <= n - 1 ? binom[n - 1][k] : 0);
  }
  FAGBI_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_binom), binom, sizeof binom));
  // Taylor tables per (level, offset) for G0 and Gk
  for (int l = h->lmin; l <= h->L; ++l) {
    Level& D = h->lev[l];
    if (D.n_off == 0) continue;
    std::vector<double> f0((size_t)D.n_off * D.T), fk((size_t)D.n_off * D.T);
    for (int o = 0; o < D.n_off; ++o) {
      const double x0[3] = {D.off_xyz[3 * o] * D.h, D.off_xyz[3 * o + 1] * D.h, D.off_xyz[3 * o + 2] * D.h};
      taylor_host(x0, 0.0, D.order, f0.data() + (size_t)o * D.T);
      taylor_host(x0, h->prm.kappa, D.order, fk.data() + (size_t)o * D.T);
    }
    FAGBI_TRY(upload_conv<double>(h, D.d_F64[0], f0));
    FAGBI_TRY(upload_conv<double>(h, D.d_F64[1], fk));
    FAGBI_TRY(upload_conv<float>(h, D.d_F32[0], f0));
    FAGBI_TRY(upload_conv<float>(h, D.d_F32[1], fk));
  }
  for (int l = std::min(h->lmin, h->L); l <= h->L; ++l) {
    Level& D = h->lev[l];
    for (int ch = 0; ch < 2; ++ch) {
      FAGBI_TRY(h->alloc(D.d_M64[ch], (size_t)D.n * D.T * 8));
      FAGBI_TRY(h->alloc(D.d_L64[ch], (size_t)D.n * D.T * 8));
      FAGBI_TRY(h->alloc(D.d_M32[ch], (size_t)D.n * D.T * 4));
      FAGBI_TRY(h->alloc(D.d_L32[ch], (size_t)D.n * D.T * 4));
    }
  }
  // panel moments about the leaf centres
  const Level& LF = h->lev[h->L];
  const int T = LF.T;
  const int64_t NT = h->N * T;
  FAGBI_TRY(h->alloc(h->d_ms64, NT * 8));
  FAGBI_TRY(h->alloc(h->d_md64, NT * 8));
  FAGBI_TRY(h->alloc(h->d_ms32, NT * 4));
  FAGBI_TRY(h->alloc(h->d_md32, NT * 4));
  const unsigned grid = (unsigned)((NT + 255) / 256);
  k_panel_moments<double><<<grid, 256, 0, s>>>(h->d_pv.as<double>(), h->d_pn.as<double>(), h->d_pa.as<double>(),
                                                h->d_leaf_of.as<int32_t>(), LF.d_idx.as<int32_t>(), h->corner[0],
                                                h->corner[1], h->corner[2], LF.h, (int)h->N, T,
                                                h->d_mi.as<int8_t>(), h->d_ms64.as<double>(),
                                                h->d_md64.as<double>());
  k_panel_moments<float><<<grid, 256, 0, s>>>(h->d_pv.as<double>(), h->d_pn.as<double>(), h->d_pa.as<double>(),
                                               h->d_leaf_of.as<int32_t>(), LF.d_idx.as<int32_t>(), h->corner[0],
                                               h->corner[1], h->corner[2], LF.h, (int)h->N, T,
                                               h->d_mi.as<int8_t>(), h->d_ms32.as<float>(),
                                               h->d_md32.as<float>());
  FAGBI_HIP(hipGetLastError());
  return 0;
}

template <typename R, typename E>
static int matvec_t(fagbi_handle* h, const double* x, double* y, int parts, hipStream_t s,
                    const DBuf& ent, const DBuf& ms, const DBuf& md, bool f32) {
  const int64_t N = h->N;
  const int nl = h->lev[h->L].n;
  if (parts & FAGBI_PART_NEAR) {
    k_spmv<E><<<(unsigned)((N + 3) / 4), 256, 0, s>>>(
        ent.as<E>(), h->d_leaf_of.as<int32_t>(), h->d_leaf_start.as<int32_t>(), h->d_src_off.as<int64_t>(),
        h->d_ent_off.as<int64_t>(), h->d_src_user.as<int32_t>(), h->d_perm.as<int32_t>(), N, x, y);
  } else {
    FAGBI_HIP(hipMemsetAsync(y, 0, 2 * N * sizeof(double), s));
  }
  FAGBI_HIP(hipGetLastError());
  if (!(parts & FAGBI_PART_FAR) || h->lmin > h->L) return 0;
  const double eps = h->prm.eps_out / h->prm.eps_in;
  const int L = h->L;
  auto M = [&](Level& D, int ch) { return f32 ? D.d_M32[ch].as<R>() : D.d_M64[ch].as<R>(); };
  auto Lc = [&](Level& D, int ch) { return f32 ? D.d_L32[ch].as<R>() : D.d_L64[ch].as<R>(); };
  Level& LF = h->lev[L];
  k_p2m<R><<<nl, 64, 0, s>>>(ms.as<R>(), md.as<R>(), h->d_leaf_start.as<int32_t>(), h->d_leaf_cnt.as<int32_t>(),
                             h->d_perm.as<int32_t>(), N, LF.T, eps, x, M(LF, 0), M(LF, 1));
  for (int l = L - 1; l >= h->lmin; --l) {
    Level &P = h->lev[l], &C = h->lev[l + 1];
    k_m2m<R><<<P.n, 64, 0, s>>>(P.d_child_start.as<int32_t>(), P.d_child_end.as<int32_t>(), C.d_idx.as<int32_t>(),
                                C.h, P.T, C.order, C.T, h->d_mi.as<int8_t>(), M(C, 0), M(C, 1), M(P, 0), M(P, 1));
  }
  for (int l = h->lmin; l <= L; ++l) {
    Level& D = h->lev[l];
    FAGBI_HIP(hipMemsetAsync(Lc(D, 0), 0, (size_t)D.n * D.T * sizeof(R), s));
    FAGBI_HIP(hipMemsetAsync(Lc(D, 1), 0, (size_t)D.n * D.T * sizeof(R), s));
    if (D.n_off == 0) continue;
    const R* F0 = f32 ? D.d_F32[0].as<R>() : D.d_F64[0].as<R>();
    const R* Fk = f32 ? D.d_F32[1].as<R>() : D.d_F64[1].as<R>();
    const R* cf = f32 ? h->d_coef32.as<R>() : h->d_coef64.as<R>();
    k_m2l<R><<<D.n, 64, 0, s>>>(D.d_inter_off.as<int32_t>(), D.d_inter_src.as<int32_t>(),
                                D.d_inter_oid.as<int32_t>(), F0, Fk, cf, h->d_gidx.as<int16_t>(),
                                h->d_mi.as<int8_t>(), D.order, D.T, M(D, 0), M(D, 1), Lc(D, 0), Lc(D, 1));
  }
  for (int l = h->lmin; l < L; ++l) {
    Level &P = h->lev[l], &C = h->lev[l + 1];
    k_l2l<R><<<C.n, 64, 0, s>>>(C.d_parent.as<int32_t>(), C.d_idx.as<int32_t>(), C.h, P.order, P.T, C.T,
                                h->d_mi.as<int8_t>(), Lc(P, 0), Lc(P, 1), Lc(C, 0), Lc(C, 1));
  }
  k_l2p<R><<<(unsigned)((N + 255) / 256), 256, 0, s>>>(ms.as<R>(), md.as<R>(), h->d_leaf_of.as<int32_t>(),
                                                      h->d_perm.as<int32_t>(), (int)N, LF.T, eps, Lc(LF, 0),
                                                      Lc(LF, 1), y);
  FAGBI_HIP(hipGetLastError());
  return 0;
}

int matvec(fagbi_handle* h, const double* x, double* y, int precision, int parts, hipStream_t s) {
  if (precision == FAGBI_MIXED)
    return matvec_t<float, float4>(h, x, y, parts, s, h->d_E32, h->d_ms32, h->d_md32, true);
  return matvec_t<double, double4>(h, x, y, parts, s, h->d_E64, h->d_ms64, h->d_md64, false);
}

}  // namespace fagbi
