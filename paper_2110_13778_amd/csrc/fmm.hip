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
//
// Translation kernels work on "slots": every coupled pair (alpha, beta) of a
// translation is one slot with its coefficient held in a register; a
// 256-thread block owns one output cluster, its threads own fixed slots (so
// the triangular truncation is evenly spread), input rows are staged in LDS
// and each output coefficient is a fixed-order sum over its slots
// (deterministic in FP64).
#include <algorithm>
#include <cstring>
#include <cmath>

#include "internal.h"
#include "scan.h"

namespace fagbi {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// lane exchanges by DPP moves (no LDS traffic): within quads lane ^ 1
// (quad_perm 1,0,3,2) and lane ^ 2 (quad_perm 2,3,0,1); within 8 lanes the
// mirrored lane 7 - i = i ^ 7 (row_half_mirror); within 16 lanes 15 - i = i ^ 15
// (row_mirror)
constexpr int DPP_X1 = 0xB1, DPP_X2 = 0x4E, DPP_X7 = 0x141, DPP_X15 = 0x140;
template <int CTRL> __device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ __forceinline__ double dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// sums over aligned groups of S lanes (S = 1, 2, 4, 8 or 16) of the n values
// of two arrays, every lane of a group receiving the totals; one branch per
// exchange step
template <int n, typename R> __device__ __forceinline__ void group_sum2(R* a, R* b, int S) {
  if (S >= 2) {
#pragma unroll
    for (int t = 0; t < n; ++t) {
      a[t] += dpp<DPP_X1>(a[t]);
      b[t] += dpp<DPP_X1>(b[t]);
    }
  }
  if (S >= 4) {
#pragma unroll
    for (int t = 0; t < n; ++t) {
      a[t] += dpp<DPP_X2>(a[t]);
      b[t] += dpp<DPP_X2>(b[t]);
    }
  }
  if (S >= 8) {
#pragma unroll
    for (int t = 0; t < n; ++t) {
      a[t] += dpp<DPP_X7>(a[t]);
      b[t] += dpp<DPP_X7>(b[t]);
    }
  }
  if (S >= 16) {
#pragma unroll
    for (int t = 0; t < n; ++t) {
      a[t] += dpp<DPP_X15>(a[t]);
      b[t] += dpp<DPP_X15>(b[t]);
    }
  }
}

__host__ __device__ constexpr int midx(int a, int b, int c) {
  const int d = a + b + c;
  const int below = d * (d + 1) * (d + 2) / 6;
  return below + (d - a) * (d - a + 1) / 2 + (d - a - b);
}

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

__host__ __device__ constexpr int binom_c(int n, int k) {
  int r = 1;
  for (int q = 1; q <= k; ++q) r = r * (n - k + q) / q;
  return r;
}

static double fact(int n) {
  double f = 1;
  for (int k = 2; k <= n; ++k) f *= k;
  return f;
}

static double binom(int n, int k) { return (double)binom_c(n, k); }

struct MI {
  int a[3];
};
static MI mi_of(int t) {
  static const std::vector<MI> tab = [] {
    std::vector<MI> v(TMAX);
    for (int d = 0; d <= PMAX; ++d)
      for (int a = d; a >= 0; --a)
        for (int b = d - a; b >= 0; --b) v[midx(a, b, d - a - b)] = MI{{a, b, d - a - b}};
    return v;
  }();
  return tab[t];
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
constexpr int TB = 256;   // threads per translation block

// single/double layer moments of each panel about its leaf centre; with
// corners != 0 one set per panel corner (row e = 3 i + a), the rule's weights
// times the hat function lambda_a at its points (2/3 at point a, 1/6 at the
// others)
template <typename R>
__global__ void k_panel_moments(const double* __restrict__ pv, const double* __restrict__ pn,
                                const double* __restrict__ pa, const int32_t* __restrict__ leaf_of,
                                const int32_t* __restrict__ lidx, double cx, double cy, double cz,
                                double hL, int N, int T, const int8_t* __restrict__ mi, R* ms, R* md,
                                int corners) {
  // layout [rows][T]: moment t of a row (panel i, or corner a of panel i) at row * T + t
  const int rows = corners ? 3 * N : N;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)rows * T) return;
  const int row = (int)(g / T), t = (int)(g - (int64_t)row * T);
  const int i = corners ? row / 3 : row, a = corners ? row - 3 * (row / 3) : -1;
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
    // d^e and d^(e-1) per axis by running products (kept in registers)
    double pe[3], pm[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      pe[ax] = 1.0;
      pm[ax] = 0.0;
      for (int q = 1; q <= e[ax]; ++q) {
        pm[ax] = pe[ax];
        pe[ax] *= d[ax];
      }
    }
    const double wk = a < 0 ? w : (k == a ? (2.0 / 3.0) : (1.0 / 6.0)) * w;
    s += wk * pe[0] * pe[1] * pe[2];
    double g2 = 0;
    if (e[0]) g2 += e[0] * pn[3 * i] * pm[0] * pe[1] * pe[2];
    if (e[1]) g2 += e[1] * pn[3 * i + 1] * pe[0] * pm[1] * pe[2];
    if (e[2]) g2 += e[2] * pn[3 * i + 2] * pe[0] * pe[1] * pm[2];
    dsum += wk * g2;
  }
  ms[g] = (R)s;
  md[g] = (R)dsum;
}

// P2M: one thread per (leaf, term); panel moments [N][T]
template <typename R>
__global__ void k_p2m(const R* __restrict__ ms, const R* __restrict__ md, const int32_t* __restrict__ leaf_start,
                      const int32_t* __restrict__ leaf_cnt, int64_t N, int nl,
                      int T, double eps, const double* __restrict__ x, R* M0, R* Mk) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (int64_t)nl * T) return;
  const int c = (int)(g / T), t = (int)(g - (int64_t)c * T);
  const int i0 = leaf_start[c], n = leaf_cnt[c];
  R a0 = 0, ak = 0;
  // four panels per step, their loads issued together at clamped indices
  // (the sums keep the panel order)
  for (int i = i0; i < i0 + n; i += 4) {
    R phi[4], dphi[4], sv[4], dv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int ii = min(i + u, i0 + n - 1);
      phi[u] = (R)x[2 * ii];   // x in tree order, interleaved
      dphi[u] = (R)x[2 * ii + 1];
      sv[u] = ms[(int64_t)ii * T + t];
      dv[u] = md[(int64_t)ii * T + t];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u < i0 + n) {
        a0 += sv[u] * dphi[u] - dv[u] * phi[u];
        ak += -sv[u] * dphi[u] + (R)eps * dv[u] * phi[u];
      }
  }
  M0[g] = a0;
  Mk[g] = ak;
}

// reduce per-slot partial sums (red0/redk, nslot each, slots grouped by
// output index) into out[t] for t < Tout, fixed order
template <typename R>
__device__ inline void slot_reduce(const R* red0, const R* redk, const int32_t* __restrict__ off, int Tout,
                                   R* out0, R* outk, bool accumulate) {
  for (int t = threadIdx.x; t < Tout; t += TB) {
    R s0 = 0, sk = 0;
    for (int k = off[t]; k < off[t + 1]; ++k) {
      s0 += red0[k];
      sk += redk[k];
    }
    if (accumulate) {
      out0[t] += s0;
      outk[t] += sk;
    } else {
      out0[t] = s0;
      outk[t] = sk;
    }
  }
}

// MtL: one block per target cluster.  With D_g = g! F_g/(4 pi) (per offset
// table), Mt^b = (-1)^|b| M^b / b! and lambda^a = Lt^a / a!, the translation
// is Lt^a = sum_{|a|+|b| <= p} D_{a+b} Mt^b: one multiply-add per slot.
// slot = (g | b << 16): g the index of alpha+beta, b the index of beta; slots
// sorted by alpha (aoff).  Both channels travel together (R2 = {G0, Gk}).
template <typename R> struct Pair;
template <> struct Pair<float> { using T = float2; };
template <> struct Pair<double> { using T = double2; };

// one block's work (blk: the block's index within its level; smem_raw: the
// block's dynamic LDS); SPT slot rounds per thread, SPT * TB >= nslot
template <typename R, int SPT>
__device__ __forceinline__ void m2l_slot_block(char* smem_raw, int blk, const int32_t* __restrict__ inter_off,
                                               const int32_t* __restrict__ inter_src,
                                               const int32_t* __restrict__ inter_oid,
                                               const typename Pair<R>::T* __restrict__ Dt,
                                               const int32_t* __restrict__ slot, const R* __restrict__ mscale,
                                               const R* __restrict__ lscale, const int32_t* __restrict__ aoff,
                                               int nslot, int T, int batch, int cpb, int ncl,
                                               const R* __restrict__ M0, const R* __restrict__ Mk, R* L0, R* Lk) {
  // cpb targets per block when a translation has few slots: group g of
  // nslot threads (SPT == 1) owns target blk * cpb + g
  using R2 = typename Pair<R>::T;
  const int tid = threadIdx.x;
  const int gsz = SPT == 1 ? nslot : TB;
  const int g = SPT == 1 ? tid / nslot : 0;
  const int lt = SPT == 1 ? tid - g * nslot : tid;   // thread within the group
  const int c = blk * cpb + g;
  const bool active = g < cpb && c < ncl;
  R2* sm = reinterpret_cast<R2*>(smem_raw) + (size_t)(active ? g : 0) * batch * 2 * T;
  int sg[SPT], sb[SPT];
  R a0[SPT], ak[SPT];
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int k = lt + j * TB;
    const int v = (active && k < nslot) ? slot[k] : 0;
    sg[j] = v & 0xffff;
    sb[j] = T + (v >> 16);
    a0[j] = 0;
    ak[j] = 0;
  }
  const int q0 = active ? inter_off[c] : 0, q1 = active ? inter_off[c + 1] : 0;
  // the block iterates over the longest list among its targets
  int maxlen = 0;
  for (int gg = 0; gg < cpb; ++gg) {
    const int cc = blk * cpb + gg;
    if (cc < ncl) maxlen = max(maxlen, inter_off[cc + 1] - inter_off[cc]);
  }
  const int W = 2 * T;   // one staged source: D (T pairs) then Mt (T pairs)
  for (int b0 = 0; b0 < maxlen; b0 += batch) {
    const int qb = q0 + b0;
    const int nb = active ? max(0, min(batch, q1 - qb)) : 0;
    __syncthreads();
    for (int e = lt; e < nb * T; e += gsz) {
      const int s = e / T, t = e - s * T;
      const int q = qb + s;
      const int64_t mo = (int64_t)inter_src[q] * T + t;
      const R f = mscale[t];
      sm[s * W + t] = Dt[(int64_t)inter_oid[q] * T + t];
      R2 m;
      m.x = M0[mo] * f;
      m.y = Mk[mo] * f;
      sm[s * W + T + t] = m;
    }
    __syncthreads();
    for (int s = 0; s < nb; ++s) {
      const R2* row = sm + s * W;
#pragma unroll
      for (int j = 0; j < SPT; ++j) {
        const R2 d = row[sg[j]];
        const R2 m = row[sb[j]];
        a0[j] += d.x * m.x;
        ak[j] += d.y * m.y;
      }
    }
  }
  __syncthreads();
  R* red0 = reinterpret_cast<R*>(smem_raw) + (size_t)(active ? g : 0) * 2 * nslot;
  R* redk = red0 + nslot;
  if (active) {
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
      const int k = lt + j * TB;
      if (k < nslot) {
        red0[k] = a0[j];
        redk[k] = ak[j];
      }
    }
  }
  __syncthreads();
  if (!active) return;
  for (int t = lt; t < T; t += gsz) {
    R s0 = 0, sk = 0;
    for (int k = aoff[t]; k < aoff[t + 1]; ++k) {
      s0 += red0[k];
      sk += redk[k];
    }
    // every cluster of the level is some group's target and the MtL is the
    // first writer of the level's locals (LtL adds into them afterwards)
    L0[(int64_t)c * T + t] = s0 * lscale[t];
    Lk[(int64_t)c * T + t] = sk * lscale[t];
  }
}

// the block with the exact number of slot rounds of its level for the orders
// 7 and 8 (ceil(nslot / TB) = 7, 12) when at most SPT; SPT rounds otherwise
// (the slots past nslot read slot 0 and are not stored)
template <typename R, int SPT>
__device__ __forceinline__ void m2l_slot_dispatch(char* smem_raw, int blk, const int32_t* __restrict__ inter_off,
                                                  const int32_t* __restrict__ inter_src,
                                                  const int32_t* __restrict__ inter_oid,
                                                  const typename Pair<R>::T* __restrict__ Dt,
                                                  const int32_t* __restrict__ slot, const R* __restrict__ mscale,
                                                  const R* __restrict__ lscale, const int32_t* __restrict__ aoff,
                                                  int nslot, int T, int batch, int cpb, int ncl,
                                                  const R* __restrict__ M0, const R* __restrict__ Mk, R* L0, R* Lk) {
#define FAGBI_SLOT_BLOCK(NJ)                                                                                   \
  m2l_slot_block<R, NJ>(smem_raw, blk, inter_off, inter_src, inter_oid, Dt, slot, mscale, lscale, aoff, nslot, T, \
                        batch, cpb, ncl, M0, Mk, L0, Lk)
  const int nj = (nslot + TB - 1) / TB;   // uniform over the block
  if constexpr (SPT >= 12) if (nj == 12) { FAGBI_SLOT_BLOCK(12); return; }
  if constexpr (SPT >= 7) if (nj == 7) { FAGBI_SLOT_BLOCK(7); return; }
  FAGBI_SLOT_BLOCK(SPT);
#undef FAGBI_SLOT_BLOCK
}

template <typename R, int SPT>
__global__ void __launch_bounds__(TB) k_m2l(const int32_t* __restrict__ inter_off, const int32_t* __restrict__ inter_src,
                                            const int32_t* __restrict__ inter_oid,
                                            const typename Pair<R>::T* __restrict__ Dt,
                                            const int32_t* __restrict__ slot, const R* __restrict__ mscale,
                                            const R* __restrict__ lscale, const int32_t* __restrict__ aoff,
                                            int nslot, int T, int batch, int cpb, int ncl,
                                            const R* __restrict__ M0, const R* __restrict__ Mk, R* L0, R* Lk) {
  extern __shared__ __align__(16) char smem_raw[];
  m2l_slot_block<R, SPT>(smem_raw, (int)blockIdx.x, inter_off, inter_src, inter_oid, Dt, slot, mscale, lscale, aoff,
                         nslot, T, batch, cpb, ncl, M0, Mk, L0, Lk);
}

// Several levels' slot MtL in one launch (the levels are independent): the
// coarse levels have few clusters each, so one launch per level leaves the
// GPU mostly idle while a long chain of short launches runs.  Level i owns
// blocks [b0_i, b0_{i+1}), one target cluster per block.
constexpr int MTL_MAXL = 16;
// persistent blocks of the order-4 LDS MtL with the octant table: two per CU
// (its table leaves room for a second block's LDS; one per CU measured slower)
constexpr int MTL_OCT_BLOCKS = 512;
template <typename R>
struct MtlLevels {
  struct Lv {
    const int32_t *off, *src, *oid, *slot, *aoff;
    const typename Pair<R>::T* Dt;
    const R* msc;   // (-1)^|b| / b! for the moments, then 1 / a! for the locals
    const R *M0, *Mk;
    R *L0, *Lk;
    int nslot, T, batch, ncl, b0;
  } lv[MTL_MAXL];
  int n;
};

template <typename R, int SPT>
__global__ void __launch_bounds__(TB) k_m2l_multi(const MtlLevels<R> ls) {
  extern __shared__ __align__(16) char smem_raw[];
  const int b = (int)blockIdx.x;
  int i = 0;
  while (i + 1 < ls.n && b >= ls.lv[i + 1].b0) ++i;
  const typename MtlLevels<R>::Lv& v = ls.lv[i];
  m2l_slot_dispatch<R, SPT>(smem_raw, b - v.b0, v.off, v.src, v.oid, v.Dt, v.slot, v.msc, v.msc + v.T, v.aoff,
                            v.nslot, v.T, v.batch, 1, v.ncl, v.M0, v.Mk, v.L0, v.Lk);
}

// MtL for low orders with the whole expansion in registers: S consecutive
// lanes share one target cluster and take every S-th entry of its
// interaction list; per entry the offset's derivative table (T pairs) and the
// source moments are loaded and all (alpha, beta) with |alpha| + |beta| <= P
// are applied with compile-time indices; the S partial sums are combined by
// lane shuffles.  The locals are written, not accumulated.
template <int P>
struct TermTable {
  static constexpr int T = (P + 1) * (P + 2) * (P + 3) / 6;
  int e[T][3];       // exponents of term t
  int deg[T];
  double msc[T];     // (-1)^|b| / b!
  double lsc[T];     // 1 / a!
  constexpr TermTable() : e(), deg(), msc(), lsc() {
    for (int d = 0; d <= P; ++d)
      for (int a = d; a >= 0; --a)
        for (int b = d - a; b >= 0; --b) {
          const int c = d - a - b;
          const int t = midx(a, b, c);
          e[t][0] = a;
          e[t][1] = b;
          e[t][2] = c;
          deg[t] = d;
          double f = 1;
          for (int k = 2; k <= a; ++k) f *= k;
          for (int k = 2; k <= b; ++k) f *= k;
          for (int k = 2; k <= c; ++k) f *= k;
          lsc[t] = 1.0 / f;
          msc[t] = ((d & 1) ? -1.0 : 1.0) / f;
        }
  }
};

template <typename R, int P>
__global__ void __launch_bounds__(256) k_m2l_reg(const int32_t* __restrict__ inter_off,
                                                 const int32_t* __restrict__ inter_src,
                                                 const int32_t* __restrict__ inter_oid,
                                                 const typename Pair<R>::T* __restrict__ Dt, int ncl, int S,
                                                 const R* __restrict__ M0, const R* __restrict__ Mk, R* L0, R* Lk) {
  using R2 = typename Pair<R>::T;
  constexpr TermTable<P> tt{};
  constexpr int T = TermTable<P>::T;
  // workgroups are dealt round-robin to the 8 XCDs; give each XCD a
  // contiguous (Morton) range of targets so that their sources share its L2
  const int nbx = (int)((gridDim.x + 7) / 8);
  const int64_t blk = (int64_t)(blockIdx.x & 7) * nbx + (blockIdx.x >> 3);
  const int64_t gt = blk * blockDim.x + threadIdx.x;
  const int c = (int)(gt / S), part = (int)(gt - (int64_t)c * S);
  R l0[T], lk[T];
#pragma unroll
  for (int t = 0; t < T; ++t) l0[t] = lk[t] = 0;
  if (c < ncl) {
    const int q1 = inter_off[c + 1];
    int q = inter_off[c] + part;
    // the next pair's source and offset are loaded one step ahead
    int32_t src_n = 0, oid_n = 0;
    if (q < q1) {
      src_n = inter_src[q];
      oid_n = inter_oid[q];
    }
    for (; q < q1; q += S) {
      const int64_t src = src_n;
      const R2* dp = Dt + (int64_t)oid_n * T;
      if (q + S < q1) {
        src_n = inter_src[q + S];
        oid_n = inter_oid[q + S];
      }
      R2 d[T];
#pragma unroll
      for (int g = 0; g < T; ++g) d[g] = dp[g];
      const R* m0p = M0 + src * T;
      const R* mkp = Mk + src * T;
#pragma unroll
      for (int tb = 0; tb < T; ++tb) {
        const R m0 = m0p[tb] * (R)tt.msc[tb], mk = mkp[tb] * (R)tt.msc[tb];
        // terms are ordered by degree: |alpha| <= P - |beta| is a prefix
#pragma unroll
        for (int ta = 0; ta < nterms(P - tt.deg[tb]); ++ta) {
          const int g = midx(tt.e[ta][0] + tt.e[tb][0], tt.e[ta][1] + tt.e[tb][1], tt.e[ta][2] + tt.e[tb][2]);
          l0[ta] += d[g].x * m0;
          lk[ta] += d[g].y * mk;
        }
      }
    }
  }
  // combine the S partial sums (S <= 16 divides 64, groups are lane-aligned)
  group_sum2<T>(l0, lk, S);
  if (c < ncl && part == 0)
#pragma unroll
    for (int t = 0; t < T; ++t) {
      L0[(int64_t)c * T + t] = l0[t] * (R)tt.lsc[t];
      Lk[(int64_t)c * T + t] = lk[t] * (R)tt.lsc[t];
    }
}


// the (a, b) pairs of a shift between orders PP (a) and PC (b): a >= b
// componentwise, with the index of a - b and C(a, b)
__host__ __device__ constexpr int count_shift_pairs(int PP, int PC) {
  int n = 0;
  for (int da = 0; da <= PP; ++da)
    for (int a0 = da; a0 >= 0; --a0)
      for (int a1 = da - a0; a1 >= 0; --a1)
        for (int db = 0; db <= PC; ++db)
          for (int b0 = db; b0 >= 0; --b0)
            for (int b1 = db - b0; b1 >= 0; --b1)
              if (b0 <= a0 && b1 <= a1 && db - b0 - b1 <= da - a0 - a1) ++n;
  return n;
}

template <int PP, int PC>
struct ShiftPairs {
  static constexpr int N = count_shift_pairs(PP, PC);
  int ta[N], tb[N], g[N];
  double coef[N];
  constexpr ShiftPairs() : ta(), tb(), g(), coef() {
    int n = 0;
    for (int da = 0; da <= PP; ++da)
      for (int a0 = da; a0 >= 0; --a0)
        for (int a1 = da - a0; a1 >= 0; --a1) {
          const int a2 = da - a0 - a1;
          for (int db = 0; db <= PC; ++db)
            for (int b0 = db; b0 >= 0; --b0)
              for (int b1 = db - b0; b1 >= 0; --b1) {
                const int b2 = db - b0 - b1;
                if (!(b0 <= a0 && b1 <= a1 && b2 <= a2)) continue;
                ta[n] = midx(a0, a1, a2);
                tb[n] = midx(b0, b1, b2);
                g[n] = midx(a0 - b0, a1 - b1, a2 - b2);
                coef[n] = (double)(binom_c(a0, b0) * binom_c(a1, b1) * binom_c(a2, b2));
                ++n;
              }
        }
  }
};

// monomials (x_child - x_parent)^g for |g| <= P, with the offset
// ((idx & 1) - 1/2) h_child per axis
template <typename R, int P>
__device__ inline void shift_monomials(const int32_t* __restrict__ cidx, int c, R hc, R* mono) {
  R d[3];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) d[ax] = ((R)(cidx[3 * c + ax] & 1) - (R)0.5) * hc;
  // by degree: each monomial of degree k is a degree k-1 one times one axis
  mono[0] = 1;
#pragma unroll
  for (int k = 1; k <= P; ++k)
#pragma unroll
    for (int a = k; a >= 0; --a)
#pragma unroll
      for (int b = k - a; b >= 0; --b) {
        const int c2 = k - a - b;
        mono[midx(a, b, c2)] = a > 0 ? mono[midx(a - 1, b, c2)] * d[0]
                             : b > 0 ? mono[midx(a, b - 1, c2)] * d[1] : mono[midx(a, b, c2 - 1)] * d[2];
      }
}

// LtL with registers, one thread per child: child^b += sum_{a >= b, |a| <= PP}
// C(a, b) d^(a - b) parent^a for |b| <= PC
// A block's rows [r0, r0 + nr) of width W (one row per thread, contiguous in
// global memory) pass through LDS with an odd row stride, so that the global
// side is one coalesced span and a thread's own row has no bank conflicts.
template <int W>
struct RowStage {
  static constexpr int S = W | 1;
};
template <typename R, int W>
__device__ inline void stage_load(const R* __restrict__ g, int64_t r0, int nr, R* st) {
  const R* src = g + r0 * W;
  for (int e = threadIdx.x; e < nr * W; e += blockDim.x) {
    const int i = e / W;
    st[i * RowStage<W>::S + (e - i * W)] = src[e];
  }
}
template <typename R, int W>
__device__ inline void stage_store(R* g, int64_t r0, int nr, const R* st) {
  R* dst = g + r0 * W;
  for (int e = threadIdx.x; e < nr * W; e += blockDim.x) {
    const int i = e / W;
    dst[e] = st[i * RowStage<W>::S + (e - i * W)];
  }
}

template <typename R, int PP, int PC>
__global__ void __launch_bounds__(256) k_l2l_reg(const int32_t* __restrict__ parent, const int32_t* __restrict__ cidx,
                                                 int n, R hc, const R* __restrict__ P0, const R* __restrict__ Pk,
                                                 R* C0, R* Ck) {
  constexpr ShiftPairs<PP, PC> sp{};
  constexpr int TP = nterms(PP), TC = nterms(PC);
  constexpr int WS = RowStage<TC>::S;
  __shared__ R st[256 * WS];
  const int cb = blockIdx.x * blockDim.x;   // launched with 256 threads
  const int c = cb + threadIdx.x;
  const int nr = min((int)blockDim.x, n - cb);
  const bool active = c < n;
  R s0[TC], sk[TC];
#pragma unroll
  for (int t = 0; t < TC; ++t) s0[t] = sk[t] = 0;
  if (active) {
    const int64_t par = parent[c];
    R mono[TP], p0[TP], pk[TP];
    shift_monomials<R, PP>(cidx, c, hc, mono);
#pragma unroll
    for (int t = 0; t < TP; ++t) {
      p0[t] = P0[par * TP + t];
      pk[t] = Pk[par * TP + t];
    }
#pragma unroll
    for (int k = 0; k < ShiftPairs<PP, PC>::N; ++k) {
      const R w = (R)sp.coef[k] * mono[sp.g[k]];
      s0[sp.tb[k]] += w * p0[sp.ta[k]];
      sk[sp.tb[k]] += w * pk[sp.ta[k]];
    }
  }
  // the children's rows (the MtL results) += the shifted parent, one channel
  // at a time through LDS
#pragma unroll
  for (int chn = 0; chn < 2; ++chn) {
    R* g = chn ? Ck : C0;
    stage_load<R, TC>(g, cb, nr, st);
    __syncthreads();
    if (active)
#pragma unroll
      for (int t = 0; t < TC; ++t) st[threadIdx.x * WS + t] += chn ? sk[t] : s0[t];
    __syncthreads();
    stage_store<R, TC>(g, cb, nr, st);
    __syncthreads();
  }
}

// MtM with registers, one thread per parent: parent^a = sum_children
// sum_{b <= a, |b| <= PC} C(a, b) d^(a - b) child^b for |a| <= PP
template <typename R, int PP, int PC>
__global__ void __launch_bounds__(256) k_m2m_reg(const int32_t* __restrict__ child_start,
                                                 const int32_t* __restrict__ child_end,
                                                 const int32_t* __restrict__ cidx, int n, R hc,
                                                 const R* __restrict__ C0, const R* __restrict__ Ck, R* P0, R* Pk) {
  constexpr ShiftPairs<PP, PC> sp{};
  constexpr int TP = nterms(PP), TC = nterms(PC);
  constexpr int WS = RowStage<TP>::S;
  __shared__ R st[256 * WS];
  const int pb = blockIdx.x * blockDim.x;   // launched with 256 threads
  const int p = pb + threadIdx.x;
  const int nr = min((int)blockDim.x, n - pb);
  const bool active = p < n;
  R a0[TP], ak[TP];
#pragma unroll
  for (int t = 0; t < TP; ++t) a0[t] = ak[t] = 0;
  const int ce = active ? child_end[p] : 0;
  for (int ch = active ? child_start[p] : 0; ch < ce; ++ch) {
    R mono[TP], c0[TC], ck[TC];
    shift_monomials<R, PP>(cidx, ch, hc, mono);
#pragma unroll
    for (int t = 0; t < TC; ++t) {
      c0[t] = C0[(int64_t)ch * TC + t];
      ck[t] = Ck[(int64_t)ch * TC + t];
    }
#pragma unroll
    for (int k = 0; k < ShiftPairs<PP, PC>::N; ++k) {
      const R w = (R)sp.coef[k] * mono[sp.g[k]];
      a0[sp.ta[k]] += w * c0[sp.tb[k]];
      ak[sp.ta[k]] += w * ck[sp.tb[k]];
    }
  }
  // the parents' rows, one channel at a time through LDS
#pragma unroll
  for (int chn = 0; chn < 2; ++chn) {
    if (active)
#pragma unroll
      for (int t = 0; t < TP; ++t) st[threadIdx.x * WS + t] = chn ? ak[t] : a0[t];
    __syncthreads();
    stage_store<R, TP>(chn ? Pk : P0, pb, nr, st);
    __syncthreads();
  }
}

// Dynamic tile claims of the persistent MtL kernels.  Tiles [0, n) form 8
// contiguous ranges, one per XCD (block id mod 8), each with a claim counter
// ctr[x]; a block (or wavefront) claims the next tile of its own XCD's range
// and, once that range is used up, of the following XCDs' ranges.  A block
// whose CU is shared with other kernels simply claims fewer tiles, so the
// launch does not wait for its slowest block.  *vx is the caller's cursor over
// the ranges (0 at the start); -1 when every range is used up.  ctr[8] counts
// finished blocks and the last one clears all nine, so every launch starts
// from zero (the counters are zero when allocated).
__device__ __forceinline__ int claim_tile(int* ctr, int xcd, int* vx, int n) {
  const int per = (n + 7) / 8;
  while (*vx < 8) {
    const int x = (xcd + *vx) & 7;
    const int k = atomicAdd(&ctr[x], 1);
    if (k < per && x * per + k < n) return x * per + k;
    ++*vx;
  }
  return -1;
}
// one thread per block, after the block's last claim
__device__ __forceinline__ void claims_done(int* ctr) {
  __threadfence();
  if (atomicAdd(&ctr[8], 1) == (int)gridDim.x - 1) {
    for (int x = 0; x < 9; ++x) atomicExch(&ctr[x], 0);
    __threadfence();
  }
}

// the register-blocked MtL (k_m2l_reg) with the level's derivative table
// staged in LDS: only one of each pair of opposite offsets is stored
// (D_g(-o) = (-1)^|g| D_g(o), the kernels being even), omap[oid] = row |
// flip << 30; with OCT one offset of each class equal up to the signs of the
// components (D_g(o) = (-1)^(g . s) D_g(|o|)), omap[oid] = row | s << 29.
// Persistent blocks, each a contiguous range of targets, so only the source
// moments come from the caches.
template <typename R, int P, int NT, bool OCT = false>
__global__ void __launch_bounds__(NT) k_m2l_lds(const int32_t* __restrict__ inter_off,
                                                const int32_t* __restrict__ inter_src,
                                                const int32_t* __restrict__ inter_oid,
                                                const typename Pair<R>::T* __restrict__ Dh, int n_half,
                                                const int32_t* __restrict__ omap, int n_off, int ncl, int S,
                                                const R* __restrict__ M0, const R* __restrict__ Mk, R* L0, R* Lk) {
  using R2 = typename Pair<R>::T;
  constexpr TermTable<P> tt{};
  constexpr int T = TermTable<P>::T;
  extern __shared__ __align__(16) char smem_raw[];
  R2* dsm = reinterpret_cast<R2*>(smem_raw);
  int32_t* smap = reinterpret_cast<int32_t*>(dsm + n_half * T);
  for (int e = threadIdx.x; e < n_half * T; e += NT) dsm[e] = Dh[e];
  for (int e = threadIdx.x; e < n_off; e += NT) smap[e] = omap[e];
  __syncthreads();
  // XCD x (= block id mod 8) owns a contiguous range of tiles; its blocks
  // sweep that range together (tile it * nbx + local block), so the sources
  // in use at any time stay within the XCD's L2.  (Claimed tiles, as in the
  // leaf tile kernel, keep every block and its LDS until the last tile and
  // starved the kernels beside it: 1.03 -> 1.26 ms per FP32 matvec.)
  const int nbx = (int)((gridDim.x + 7) / 8);
  const int64_t xcd = blockIdx.x & 7, bl = blockIdx.x >> 3;
  const int64_t ntile = ((int64_t)ncl * S + NT - 1) / NT;
  const int64_t per = (ntile + (int64_t)nbx * 8 - 1) / ((int64_t)nbx * 8);
  for (int64_t it = 0; it < per; ++it) {
    const int64_t gt = ((xcd * per + it) * nbx + bl) * NT + threadIdx.x;
    const int c = (int)(gt / S), part = (int)(gt - (int64_t)c * S);
    R l0[T], lk[T];
#pragma unroll
    for (int t = 0; t < T; ++t) l0[t] = lk[t] = 0;
    if (c < ncl) {
      const int q1 = inter_off[c + 1];
      int q = inter_off[c] + part;
      // the next pair's source and offset are loaded one step ahead
      int32_t src_n = 0, oid_n = 0;
      if (q < q1) {
        src_n = inter_src[q];
        oid_n = inter_oid[q];
      }
      for (; q < q1; q += S) {
        const int64_t src = src_n;
        const uint32_t mo = (uint32_t)smap[oid_n];
        if (q + S < q1) {
          src_n = inter_src[q + S];
          oid_n = inter_oid[q + S];
        }
        R2 d[T];
        if constexpr (OCT) {
          // the sign of term g: the product of the flipped axes' signs over
          // its odd exponents (sp indexed by those axes, bit a for axis a)
          const R2* dp = dsm + (mo & 0x1fffffffu) * T;
          const R sx = (mo >> 29) & 1u ? (R)-1 : (R)1, sy = (mo >> 30) & 1u ? (R)-1 : (R)1,
                  sz = (mo >> 31) ? (R)-1 : (R)1;
          const R sp[8] = {(R)1, sx, sy, sx * sy, sz, sx * sz, sy * sz, sx * sy * sz};
#pragma unroll
          for (int g = 0; g < T; ++g) {
            d[g] = dp[g];
            const int par = (tt.e[g][0] & 1) | (tt.e[g][1] & 1) << 1 | (tt.e[g][2] & 1) << 2;
            if (par) {
              d[g].x *= sp[par];
              d[g].y *= sp[par];
            }
          }
        } else {
          const R2* dp = dsm + (mo & 0x3fffffffu) * T;
          const R sg = (mo >> 30) ? (R)-1 : (R)1;
#pragma unroll
          for (int g = 0; g < T; ++g) {
            d[g] = dp[g];
            if (tt.deg[g] & 1) {
              d[g].x *= sg;
              d[g].y *= sg;
            }
          }
        }
        const R* m0p = M0 + src * T;
        const R* mkp = Mk + src * T;
#pragma unroll
        for (int tb = 0; tb < T; ++tb) {
          const R m0 = m0p[tb] * (R)tt.msc[tb], mk = mkp[tb] * (R)tt.msc[tb];
#pragma unroll
          for (int ta = 0; ta < nterms(P - tt.deg[tb]); ++ta) {
            const int g = midx(tt.e[ta][0] + tt.e[tb][0], tt.e[ta][1] + tt.e[tb][1], tt.e[ta][2] + tt.e[tb][2]);
            l0[ta] += d[g].x * m0;
            lk[ta] += d[g].y * mk;
          }
        }
      }
    }
    group_sum2<T>(l0, lk, S);
    if (c < ncl && part == 0)
#pragma unroll
      for (int t = 0; t < T; ++t) {
        L0[(int64_t)c * T + t] = l0[t] * (R)tt.lsc[t];
        Lk[(int64_t)c * T + t] = lk[t] * (R)tt.lsc[t];
      }
  }
}

// ---------------------------------------------------------------------------
// MtL with source reuse.  Targets are taken in tiles of up to MTK consecutive
// clusters (Morton order: a tile is a compact patch of the surface, and its
// targets share most of their sources).  Per tile, the distinct sources are
// staged once in LDS as scaled moments of both channels, the half derivative
// table stays in LDS for the whole launch, and every pair reads both operands
// from LDS into registers.  The tile's pairs are split evenly over the
// block's threads (contiguous chunks, whatever their targets); a thread adds
// its partial locals into the tile's LDS accumulators whenever its chunk
// crosses into the next target.  The next tile's source rows are loaded into
// registers while the current tile computes.  A setup pass gives each tile
// its sorted distinct sources and each pair its packed index.
// ---------------------------------------------------------------------------
constexpr int MTK = 64;          // targets per tile (at most)
constexpr int MT_S = 8;          // lanes per target
constexpr int MT_NT = MTK * MT_S;   // threads per block
constexpr int MT_IPT = 7;        // staged float4 chunks per thread and channel
constexpr int MT_UMAX = 4095;    // distinct sources of one tile (12-bit slot)
constexpr int MT_BITS = 1 << 19; // source index range of one tile the setup covers (bitmap)

// setup, one block per tile (targets [tile_lo[t], tile_hi[t])): mark the
// tile's sources in an LDS bitmap over their index range, then number them in
// increasing order by prefix popcounts; PASS 0 reports the count (2^30 when
// the range exceeds the bitmap, so that the tile is split), PASS 1 writes the
// distinct sources and the packed pair indices
template <int PASS>
__global__ void __launch_bounds__(256) k_tile_setup(const int32_t* __restrict__ inter_off,
                                                    const int32_t* __restrict__ inter_src,
                                                    const int32_t* __restrict__ inter_oid,
                                                    const int32_t* __restrict__ omap,
                                                    const int32_t* __restrict__ tile_lo,
                                                    const int32_t* __restrict__ tile_hi, int32_t* tile_cnt,
                                                    const int32_t* __restrict__ tile_off, int32_t* tile_src,
                                                    uint32_t* pack) {
  extern __shared__ __align__(16) uint32_t bits[];       // [MT_BITS / 32] words, then their prefix counts
  uint32_t* wpre = bits + MT_BITS / 32;
  __shared__ int32_t red[256];
  __shared__ int32_t smin_s, smax_s;
  const int tid = threadIdx.x, tile = blockIdx.x;
  const int t0 = tile_lo[tile], t1 = tile_hi[tile];
  const int q0 = inter_off[t0], np = inter_off[t1] - q0;
  int mn = 0x7fffffff, mx = -1;
  for (int i = tid; i < np; i += 256) {
    const int v = inter_src[q0 + i];
    mn = min(mn, v);
    mx = max(mx, v);
  }
  red[tid] = mn;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] = min(red[tid], red[tid + o]);
    __syncthreads();
  }
  if (tid == 0) smin_s = red[0];
  __syncthreads();
  red[tid] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] = max(red[tid], red[tid + o]);
    __syncthreads();
  }
  if (tid == 0) smax_s = red[0];
  __syncthreads();
  const int smin = smin_s, smax = smax_s;
  if (np == 0) {
    if (PASS == 0 && tid == 0) tile_cnt[tile] = 0;
    return;
  }
  const int64_t range = (int64_t)smax - smin + 1;
  if (range > MT_BITS) {              // uniform over the block
    if (PASS == 0 && tid == 0) tile_cnt[tile] = 1 << 30;
    return;
  }
  const int W = (int)((range + 31) / 32);
  for (int w = tid; w < W; w += 256) bits[w] = 0u;
  __syncthreads();
  for (int i = tid; i < np; i += 256) {
    const int v = inter_src[q0 + i] - smin;
    atomicOr(&bits[v >> 5], 1u << (v & 31));
  }
  __syncthreads();
  // prefix counts of the words: thread chunks of consecutive words
  const int per = (W + 255) / 256;
  const int w0 = tid * per, w1 = min(W, w0 + per);
  int c = 0;
  for (int w = w0; w < w1; ++w) c += __popc(bits[w]);
  red[tid] = c;
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int k = 0; k < 256; ++k) {
      const int x = red[k];
      red[k] = acc;
      acc += x;
    }
    smin_s = acc;                    // the total, reusing the slot
  }
  __syncthreads();
  const int nu = smin_s;
  if (PASS == 0) {
    if (tid == 0) tile_cnt[tile] = nu;
    return;
  }
  int acc = red[tid];
  for (int w = w0; w < w1; ++w) {
    wpre[w] = (uint32_t)acc;
    acc += __popc(bits[w]);
  }
  __syncthreads();
  const int u0 = tile_off[tile];
  for (int w = tid; w < W; w += 256) {
    uint32_t b = bits[w];
    int k = (int)wpre[w];
    while (b) {
      const int j = __ffs(b) - 1;
      tile_src[u0 + k++] = smin + 32 * w + j;
      b &= b - 1;
    }
  }
  for (int i = tid; i < np; i += 256) {
    const int v = inter_src[q0 + i] - smin;
    const uint32_t slot = wpre[v >> 5] + (uint32_t)__popc(bits[v >> 5] & ((1u << (v & 31)) - 1u));
    const uint32_t m = (uint32_t)omap[inter_oid[q0 + i]];
    pack[q0 + i] = slot | ((m & 0x3fffffffu) << 12) | ((m >> 30) << 31);
  }
}

// the MtL itself (FP32, T(P) a multiple of 4): persistent blocks of MT_NT
// threads, one tile at a time, claimed from the block's XCD's range of tiles
// first (claim_tile)
template <int P>
__global__ void __launch_bounds__(MT_NT, 1) k_m2l_tile(const int32_t* __restrict__ inter_off,
                                                       const uint32_t* __restrict__ pack,
                                                       const int32_t* __restrict__ tile_t0,
                                                       const int32_t* __restrict__ tile_off,
                                                       const int32_t* __restrict__ tile_src, int ntile,
                                                       const float2* __restrict__ Dh, int n_half,
                                                       const float* __restrict__ M0, const float* __restrict__ Mk,
                                                       float* L0, float* Lk, int* ctr) {
  constexpr TermTable<P> tt{};
  constexpr int T = TermTable<P>::T;
  constexpr int CPR = T / 4;              // float4 chunks per moment row and channel
  static_assert(T % 4 == 0, "rows in float4 chunks");
  // LDS rows of both tables are TP = T + 2 float2 apart (a 176-byte stride
  // at order 3 starts rows on twice as many banks as 160 bytes, fewer
  // conflicts between the lanes' random rows); the last two are padding
  constexpr int TP = T + 2;
  extern __shared__ __align__(16) char smem_raw[];
  float2* dsm = reinterpret_cast<float2*>(smem_raw);
  float2* msm = dsm + (size_t)n_half * TP;
  __shared__ float msc[T], lsc[T];
  __shared__ float acc[MTK][2 * T];       // the tile's locals, both channels
  __shared__ int32_t qoff[MTK + 1];       // the tile's list offsets
  __shared__ int32_t s_tile;              // the tile claimed next
  for (int e = threadIdx.x; e < n_half * T; e += MT_NT) {
    const int rw = e / T;
    dsm[rw * TP + (e - rw * T)] = Dh[e];
  }
  if (threadIdx.x < T) {   // (-1)^|b| / b! of term b and 1 / a! of term a
    float f = 1.0f, g = 1.0f;
#pragma unroll
    for (int t = 0; t < T; ++t)
      if (t == (int)threadIdx.x) {
        f = (float)tt.msc[t];
        g = (float)tt.lsc[t];
      }
    msc[threadIdx.x] = f;
    lsc[threadIdx.x] = g;
  }
  const int xcd = (int)(blockIdx.x & 7);
  int vx = 0;   // thread 0's cursor over the XCDs' ranges
  // staged rows of a tile in registers: item i = (slot i / CPR, chunk i % CPR)
  float4 ra[MT_IPT], rb[MT_IPT];
  auto prefetch = [&](int tile) {
    const int u0 = tile_off[tile], ni = (tile_off[tile + 1] - u0) * CPR;
#pragma unroll
    for (int k = 0; k < MT_IPT; ++k) {
      const int i = threadIdx.x + k * MT_NT;
      if (i < ni) {
        const int sl = i / CPR, j = i - sl * CPR;
        const int64_t mo = (int64_t)tile_src[u0 + sl] * T + 4 * j;
        ra[k] = *reinterpret_cast<const float4*>(M0 + mo);
        rb[k] = *reinterpret_cast<const float4*>(Mk + mo);
      }
    }
  };
  if (threadIdx.x == 0) s_tile = claim_tile(ctr, xcd, &vx, ntile);
  __syncthreads();   // msc, s_tile
  int tile = s_tile;
  if (tile >= 0) prefetch(tile);
  while (tile >= 0) {
    // the previous tile's sources and locals are no longer read, and every
    // thread has read s_tile
    __syncthreads();
    const int t0 = tile_t0[tile], nt = tile_t0[tile + 1] - t0;
    {
      const int ni = (tile_off[tile + 1] - tile_off[tile]) * CPR;
#pragma unroll
      for (int k = 0; k < MT_IPT; ++k) {
        const int i = threadIdx.x + k * MT_NT;
        if (i < ni) {
          const int sl = i / CPR, j = i - sl * CPR;
          const float s0 = msc[4 * j], s1 = msc[4 * j + 1], s2 = msc[4 * j + 2], s3 = msc[4 * j + 3];
          float4* dst = reinterpret_cast<float4*>(msm + (size_t)sl * TP + 4 * j);
          dst[0] = make_float4(ra[k].x * s0, rb[k].x * s0, ra[k].y * s1, rb[k].y * s1);
          dst[1] = make_float4(ra[k].z * s2, rb[k].z * s2, ra[k].w * s3, rb[k].w * s3);
        }
      }
      for (int e = threadIdx.x; e < nt * 2 * T; e += MT_NT) (&acc[0][0])[e] = 0.0f;
      for (int e = threadIdx.x; e <= nt; e += MT_NT) qoff[e] = inter_off[t0 + e];
    }
    if (threadIdx.x == 0) s_tile = claim_tile(ctr, xcd, &vx, ntile);
    __syncthreads();
    const int next = s_tile;
    if (next >= 0) prefetch(next);
    // items: every target's list cut into runs of IL pairs (the last one
    // shorter), IL = ceil(pairs / (threads - targets)), so that the tile has
    // at most one item per thread; a thread runs its item and adds it into
    // the target's accumulators
    // MT_S consecutive lanes per target split its list
    const int c = threadIdx.x / MT_S, part = threadIdx.x - c * MT_S;
    float l0[T], lk[T];
#pragma unroll
    for (int t = 0; t < T; ++t) l0[t] = lk[t] = 0.0f;
    if (c < nt) {
      const int q1 = qoff[c + 1];
      int q = qoff[c] + part;
      uint32_t pkn = q < q1 ? pack[q] : 0u;   // the packed index, loaded one pair ahead
      for (; q < q1; q += MT_S) {
        const uint32_t pk = pkn;
        if (q + MT_S < q1) pkn = pack[q + MT_S];
        const float4* dp = reinterpret_cast<const float4*>(dsm + (size_t)((pk >> 12) & 0x7ffffu) * TP);
        const float4* mp = reinterpret_cast<const float4*>(msm + (size_t)(pk & 0xfffu) * TP);
        const float sg = (pk >> 31) ? -1.0f : 1.0f;
        float4 dr[T / 2], mr[T / 2];
#pragma unroll
        for (int k = 0; k < T / 2; ++k) {
          dr[k] = dp[k];
          mr[k] = mp[k];
        }
        float2 d[T], m[T];
#pragma unroll
        for (int k = 0; k < T / 2; ++k) {
          d[2 * k] = make_float2(dr[k].x, dr[k].y);
          d[2 * k + 1] = make_float2(dr[k].z, dr[k].w);
          m[2 * k] = make_float2(mr[k].x, mr[k].y);
          m[2 * k + 1] = make_float2(mr[k].z, mr[k].w);
        }
#pragma unroll
        for (int g = 0; g < T; ++g)
          if (tt.deg[g] & 1) {
            d[g].x *= sg;
            d[g].y *= sg;
          }
#pragma unroll
        for (int tb = 0; tb < T; ++tb) {
#pragma unroll
          for (int ta = 0; ta < nterms(P - tt.deg[tb]); ++ta) {
            const int g = midx(tt.e[ta][0] + tt.e[tb][0], tt.e[ta][1] + tt.e[tb][1], tt.e[ta][2] + tt.e[tb][2]);
            l0[ta] += d[g].x * m[tb].x;
            lk[ta] += d[g].y * m[tb].y;
          }
        }
      }
    }
    // sums over the 8 lanes of a target by DPP moves
    static_assert(MT_S == 8, "lane groups of eight");
    group_sum2<T>(l0, lk, MT_S);
    if (c < nt && part == 0)
#pragma unroll
      for (int t = 0; t < T; ++t) {
        acc[c][t] = l0[t];
        acc[c][T + t] = lk[t];
      }
    __syncthreads();
    for (int e = threadIdx.x; e < nt * 2 * T; e += MT_NT) {
      const int cc = e / (2 * T), r = e - cc * 2 * T;
      const int t = r < T ? r : r - T;
      (r < T ? L0 : Lk)[(int64_t)(t0 + cc) * T + t] = acc[cc][r] * lsc[t];
    }
    tile = next;
  }
  if (threadIdx.x == 0) claims_done(ctr);
}

// The same MtL on the matrix cores (order 3).  Per target and channel the
// pairs' derivative rows D_k and scaled source moments m_k give
//   X[g][b] = sum_k D_k[g] m_k[b],   L_a = sum over b <= g, g - b = a of X[g][b]
// (with b <= g componentwise, |a| + |b| = |g| <= 3: exactly the truncated
// translation).  One wavefront per target, four pairs per step,
// v_mfma_f32_16x16x4f32 with A[i][k] = D_k[16 t + i] (derivative tile t = 0:
// terms 0..15; t = 1: terms 16..19, rows 4..15 zero) and B[k][j] = m_k[j],
// moments 0..15.  A moment of degree 3 only meets g = b; for b = 16..19 these
// four diagonal products are summed on the vector units.  Each X entry of a
// lane is then added to its local term (xdst: tile, lane and element -> term
// a, or -1) in a per-wavefront LDS row.
template <int P>
__global__ void __launch_bounds__(MT_NT, 1) k_m2l_tile_mfma(const int32_t* __restrict__ inter_off,
                                                            const uint32_t* __restrict__ pack,
                                                            const int32_t* __restrict__ tile_t0,
                                                            const int32_t* __restrict__ tile_off,
                                                            const int32_t* __restrict__ tile_src, int ntile,
                                                            const float2* __restrict__ Dh, int n_half, int umax,
                                                            const int8_t* __restrict__ xdst,
                                                            const float* __restrict__ M0,
                                                            const float* __restrict__ Mk, float* L0, float* Lk) {
  static_assert(P == 3, "tiles of 16 derivative terms cover order 3");
  constexpr TermTable<P> tt{};
  constexpr int T = TermTable<P>::T;
  constexpr int CPR = T / 4;
  constexpr int NW = MT_NT / 64;
  constexpr int ROWB = T * 8;                 // bytes of a row (both channels)
  uint32_t odd = 0;
#pragma unroll
  for (int t = 0; t < T; ++t)
    if (tt.deg[t] & 1) odd |= 1u << t;
  // LDS: half table rows 0..n_half-1, a zero row n_half, then the staged
  // moments, slots 0..umax-1, a zero row at slot umax and one row of slack
  // (the lanes of terms 20..31 read past a row; their values are discarded);
  // pairs past the end of a list point at both zero rows
  extern __shared__ __align__(16) char smem_raw[];
  float2* dsm = reinterpret_cast<float2*>(smem_raw);
  float2* msm = dsm + (size_t)(n_half + 1) * T;
  __shared__ float msc[T], lsc[T];
  __shared__ float lred[NW][2][2 * T];   // per wavefront, alternating between its targets
  __shared__ int32_t qoff[MTK + 1];
  for (int e = threadIdx.x; e < n_half * T; e += MT_NT) dsm[e] = Dh[e];
  if (threadIdx.x < T) {
    dsm[n_half * T + threadIdx.x] = make_float2(0.0f, 0.0f);
    msm[umax * T + threadIdx.x] = make_float2(0.0f, 0.0f);
    float f = 1.0f, g = 1.0f;
#pragma unroll
    for (int t = 0; t < T; ++t)
      if (t == (int)threadIdx.x) {
        f = (float)tt.msc[t];
        g = (float)tt.lsc[t];
      }
    msc[threadIdx.x] = f;
    lsc[threadIdx.x] = g;
  }
  const int lane = (int)threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  int dst[2][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) dst[t][e] = xdst[((t * 4 + lk) * 16 + li) * 4 + e];
  // per-lane constants: byte offsets of the lane's terms, the sign-bit mask
  // of its tile-0 derivative term (odd degree flips with the offset), and
  // whether it carries one of the terms 16..19
  const uint32_t lane_off = (uint32_t)li * 8u;
  const uint32_t oddmask = ((odd >> li) & 1u) ? 0x80000000u : 0u;
  const bool hi = li < 4;
  const uint32_t dbase = (uint32_t)(reinterpret_cast<const char*>(dsm) - smem_raw);
  const uint32_t mbase = (uint32_t)(reinterpret_cast<const char*>(msm) - smem_raw);
  const uint32_t zpack = (uint32_t)umax | ((uint32_t)n_half << 12);
  const int nbx = (int)((gridDim.x + 7) / 8);
  const int xcd = (int)(blockIdx.x & 7), bl = (int)(blockIdx.x >> 3);
  const int per = (ntile + 8 * nbx - 1) / (8 * nbx);
  float4 ra[MT_IPT], rb[MT_IPT];
  auto prefetch = [&](int tile) {
    if (tile >= ntile) return;
    const int u0 = tile_off[tile], ni = (tile_off[tile + 1] - u0) * CPR;
#pragma unroll
    for (int k = 0; k < MT_IPT; ++k) {
      const int i = threadIdx.x + k * MT_NT;
      if (i < ni) {
        const int sl = i / CPR, j = i - sl * CPR;
        const int64_t mo = (int64_t)tile_src[u0 + sl] * T + 4 * j;
        ra[k] = *reinterpret_cast<const float4*>(M0 + mo);
        rb[k] = *reinterpret_cast<const float4*>(Mk + mo);
      }
    }
  };
  __syncthreads();   // msc, lsc, zero rows
  prefetch(xcd * per * nbx + bl);
  for (int it = 0; it < per; ++it) {
    const int tile = (xcd * per + it) * nbx + bl;
    __syncthreads();   // the previous tile's sources are no longer read
    if (tile >= ntile) continue;
    const int t0 = tile_t0[tile], nt = tile_t0[tile + 1] - t0;
    {
      const int ni = (tile_off[tile + 1] - tile_off[tile]) * CPR;
#pragma unroll
      for (int k = 0; k < MT_IPT; ++k) {
        const int i = threadIdx.x + k * MT_NT;
        if (i < ni) {
          const int sl = i / CPR, j = i - sl * CPR;
          const float s0 = msc[4 * j], s1 = msc[4 * j + 1], s2 = msc[4 * j + 2], s3 = msc[4 * j + 3];
          float4* dst4 = reinterpret_cast<float4*>(msm + (size_t)sl * T + 4 * j);
          dst4[0] = make_float4(ra[k].x * s0, rb[k].x * s0, ra[k].y * s1, rb[k].y * s1);
          dst4[1] = make_float4(ra[k].z * s2, rb[k].z * s2, ra[k].w * s3, rb[k].w * s3);
        }
      }
      for (int e = threadIdx.x; e <= nt; e += MT_NT) qoff[e] = inter_off[t0 + e];
    }
    __syncthreads();
    if (it + 1 < per) prefetch((xcd * per + it + 1) * nbx + bl);
    for (int c = wv; c < nt; c += NW) {      // wave-uniform
      const int q0 = qoff[c], q1 = qoff[c + 1];
      f32x4 x00 = {0.f, 0.f, 0.f, 0.f}, x01 = x00, xk0 = x00, xk1 = x00;
      float dg0 = 0.0f, dgk = 0.0f;          // the diagonal products of moments 16..19
      // packed indices of 64 pairs at a time (one coalesced load), handed to
      // the lanes of each step by ds_bpermute
      for (int base = q0; base < q1; base += 64) {
        const uint32_t pkl = base + lane < q1 ? pack[base + lane] : zpack;
        const int ns = min(16, (q1 - base + 3) / 4);   // wave-uniform
        int baddr = lk * 4;
#pragma unroll 2
        for (int s = 0; s < ns; ++s, baddr += 16) {
          const uint32_t pk = (uint32_t)__builtin_amdgcn_ds_bpermute(baddr, (int)pkl);
          const uint32_t da = dbase + ((pk >> 12) & 0x7ffffu) * (uint32_t)ROWB + lane_off;
          const uint32_t ma = mbase + (pk & 0xfffu) * (uint32_t)ROWB + lane_off;
          const float2 d0 = *reinterpret_cast<const float2*>(smem_raw + da);
          const float2 m0 = *reinterpret_cast<const float2*>(smem_raw + ma);
          const float2 d1 = *reinterpret_cast<const float2*>(smem_raw + da + 128);
          const float2 m1 = *reinterpret_cast<const float2*>(smem_raw + ma + 128);
          const uint32_t fm = pk & 0x80000000u;        // flip: odd degrees change sign
          const uint32_t f0 = fm & oddmask;
          const float a00 = __uint_as_float(__float_as_uint(d0.x) ^ f0);
          const float a0k = __uint_as_float(__float_as_uint(d0.y) ^ f0);
          const float a10 = hi ? __uint_as_float(__float_as_uint(d1.x) ^ fm) : 0.0f;
          const float a1k = hi ? __uint_as_float(__float_as_uint(d1.y) ^ fm) : 0.0f;
          const float c0 = hi ? m1.x : 0.0f, ck = hi ? m1.y : 0.0f;
          x00 = __builtin_amdgcn_mfma_f32_16x16x4f32(a00, m0.x, x00, 0, 0, 0);
          x01 = __builtin_amdgcn_mfma_f32_16x16x4f32(a10, m0.x, x01, 0, 0, 0);
          xk0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0k, m0.y, xk0, 0, 0, 0);
          xk1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1k, m0.y, xk1, 0, 0, 0);
          dg0 += a10 * c0;
          dgk += a1k * ck;
        }
      }
      // lane (li, lk) holds X[16 t + 4 lk + e][li] in element e of tile t.
      // The LDS row is private to the wavefront; between its phases the
      // wavefront waits for its own LDS operations only (lgkmcnt(0)), and
      // consecutive targets alternate rows, so the next target's zeroing
      // never meets this one's reads
      float* lr = lred[wv][(c / NW) & 1];
      if (lane < 2 * T) lr[lane] = 0.0f;
      __builtin_amdgcn_s_waitcnt(0xC07F);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (dst[0][e] >= 0) {
          atomicAdd(&lr[dst[0][e]], x00[e]);
          atomicAdd(&lr[T + dst[0][e]], xk0[e]);
        }
        if (dst[1][e] >= 0) {
          atomicAdd(&lr[dst[1][e]], x01[e]);
          atomicAdd(&lr[T + dst[1][e]], xk1[e]);
        }
      }
      if (hi) {   // X[b][b] for b = 16..19: local term 0
        atomicAdd(&lr[0], dg0);
        atomicAdd(&lr[T], dgk);
      }
      __builtin_amdgcn_s_waitcnt(0xC07F);
      __builtin_amdgcn_wave_barrier();
      if (lane < 2 * T) {
        const int t = lane < T ? lane : lane - T;
        (lane < T ? L0 : Lk)[(int64_t)(t0 + c) * T + t] = lr[lane] * lsc[t];
      }
    }
  }
}

// MtM: one block per parent; slot = (a | b << 16), a parent index, b child
// index (b <= a componentwise); coefficient rows per child octant.
template <typename R, int SPT>
__global__ void __launch_bounds__(TB) k_m2m(const int32_t* __restrict__ child_start, const int32_t* __restrict__ child_end,
                                            const int32_t* __restrict__ cidx, const int32_t* __restrict__ slot,
                                            const R* __restrict__ coef, const int32_t* __restrict__ aoff, int nslot,
                                            int Tp, int Tc, const R* __restrict__ C0, const R* __restrict__ Ck,
                                            R* P0, R* Pk) {
  extern __shared__ __align__(16) char smem_raw[];
  R* sm = reinterpret_cast<R*>(smem_raw);
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  int sb[SPT];
  R a0[SPT], ak[SPT];
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int k = tid + j * TB;
    sb[j] = k < nslot ? (slot[k] >> 16) : 0;
    a0[j] = 0;
    ak[j] = 0;
  }
  const int c0 = child_start[c], c1 = child_end[c];
  for (int e = tid; e < (c1 - c0) * Tc; e += TB) {
    const int s = e / Tc, t = e - s * Tc;
    sm[s * 2 * Tc + t] = C0[(int64_t)(c0 + s) * Tc + t];
    sm[s * 2 * Tc + Tc + t] = Ck[(int64_t)(c0 + s) * Tc + t];
  }
  __syncthreads();
  for (int ch = c0; ch < c1; ++ch) {
    const int oct = ((cidx[3 * ch] & 1) << 2) | ((cidx[3 * ch + 1] & 1) << 1) | (cidx[3 * ch + 2] & 1);
    const R* row = sm + (ch - c0) * 2 * Tc;
    const R* cr = coef + (int64_t)oct * nslot;
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
      const int k = tid + j * TB;
      const R w = k < nslot ? cr[k] : (R)0;
      a0[j] += w * row[sb[j]];
      ak[j] += w * row[Tc + sb[j]];
    }
  }
  __syncthreads();
  R* red0 = sm;
  R* redk = sm + nslot;
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int k = tid + j * TB;
    if (k < nslot) {
      red0[k] = a0[j];
      redk[k] = ak[j];
    }
  }
  __syncthreads();
  slot_reduce<R>(red0, redk, aoff, Tp, P0 + (int64_t)c * Tp, Pk + (int64_t)c * Tp, false);
}

// LtL: one block per child; slot = (a | b << 16) sorted by b (child index)
template <typename R, int SPT>
__global__ void __launch_bounds__(TB) k_l2l(const int32_t* __restrict__ parent, const int32_t* __restrict__ cidx,
                                            const int32_t* __restrict__ slot, const R* __restrict__ coef,
                                            const int32_t* __restrict__ boff, int nslot, int Tp, int Tc,
                                            const R* __restrict__ P0, const R* __restrict__ Pk, R* C0, R* Ck) {
  extern __shared__ __align__(16) char smem_raw[];
  R* sm = reinterpret_cast<R*>(smem_raw);
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  const int par = parent[c];
  const int oct = ((cidx[3 * c] & 1) << 2) | ((cidx[3 * c + 1] & 1) << 1) | (cidx[3 * c + 2] & 1);
  for (int t = tid; t < Tp; t += TB) {
    sm[t] = P0[(int64_t)par * Tp + t];
    sm[Tp + t] = Pk[(int64_t)par * Tp + t];
  }
  __syncthreads();
  const R* cr = coef + (int64_t)oct * nslot;
  R a0[SPT], ak[SPT];
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int k = tid + j * TB;
    const int a = k < nslot ? (slot[k] & 0xffff) : 0;
    const R w = k < nslot ? cr[k] : (R)0;
    a0[j] = w * sm[a];
    ak[j] = w * sm[Tp + a];
  }
  __syncthreads();
  R* red0 = sm;
  R* redk = sm + nslot;
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int k = tid + j * TB;
    if (k < nslot) {
      red0[k] = a0[j];
      redk[k] = ak[j];
    }
  }
  __syncthreads();
  slot_reduce<R>(red0, redk, boff, Tc, C0 + (int64_t)c * Tc, Ck + (int64_t)c * Tc, true);
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

// LtP for low leaf orders: whole rows in registers
template <typename R, int P>
__global__ void __launch_bounds__(256) k_l2p_reg(const R* __restrict__ ms, const R* __restrict__ md,
                                                 const int32_t* __restrict__ leaf_of, const int32_t* __restrict__ perm,
                                                 int N, double eps, const R* __restrict__ L0, const R* __restrict__ Lk,
                                                 double* y) {
  constexpr int T = nterms(P);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t c = leaf_of[i];
  const R ie = (R)(1.0 / eps);
  R y1 = 0, y2 = 0;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const R l0 = L0[c * T + t], lk = Lk[c * T + t];
    y1 += (l0 + lk) * ms[(int64_t)i * T + t];
    y2 += (l0 + lk * ie) * md[(int64_t)i * T + t];
  }
  const int p = perm[i];
  y[p] -= (double)y1;
  y[N + p] -= (double)y2;
}

// LtP with the leaf level's LtL folded in: a row's leaf local is the leaf's
// MtL part plus its parent's local shifted to the leaf centre (the products
// of k_l2l_reg in its order, so the same values), then dotted with the row's
// moments as in k_l2p_reg.  Each row repeats its leaf's shift (2 x 195
// multiply-adds from order 4 to 3, next to the row's own 2 x 20); the leaf
// level's LtL launch and its pass over the leaf locals disappear from the
// end of the matvec.
template <typename R, int PP, int P>
__global__ void __launch_bounds__(256) k_l2p_shift(const R* __restrict__ ms, const R* __restrict__ md,
                                                   const int32_t* __restrict__ leaf_of,
                                                   const int32_t* __restrict__ perm, int N, double eps,
                                                   const R* __restrict__ L0, const R* __restrict__ Lk,
                                                   const int32_t* __restrict__ parent,
                                                   const int32_t* __restrict__ cidx, R hc,
                                                   const R* __restrict__ P0, const R* __restrict__ Pk, double* y) {
  constexpr ShiftPairs<PP, P> sp{};
  constexpr int T = nterms(P), TP = nterms(PP);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int c = leaf_of[i];
  const int64_t par = parent[c];
  R mono[TP], p0[TP], pk[TP], s0[T], sk[T];
  shift_monomials<R, PP>(cidx, c, hc, mono);
#pragma unroll
  for (int t = 0; t < TP; ++t) {
    p0[t] = P0[par * TP + t];
    pk[t] = Pk[par * TP + t];
  }
#pragma unroll
  for (int t = 0; t < T; ++t) s0[t] = sk[t] = 0;
#pragma unroll
  for (int k = 0; k < ShiftPairs<PP, P>::N; ++k) {
    const R w = (R)sp.coef[k] * mono[sp.g[k]];
    s0[sp.tb[k]] += w * p0[sp.ta[k]];
    sk[sp.tb[k]] += w * pk[sp.ta[k]];
  }
  const R ie = (R)(1.0 / eps);
  R y1 = 0, y2 = 0;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const R l0 = L0[(int64_t)c * T + t] + s0[t], lk = Lk[(int64_t)c * T + t] + sk[t];
    y1 += (l0 + lk) * ms[(int64_t)i * T + t];
    y2 += (l0 + lk * ie) * md[(int64_t)i * T + t];
  }
  const int p = perm[i];
  y[p] -= (double)y1;
  y[N + p] -= (double)y2;
}

// Sum of eight per-lane values over the wavefront, scattered: recursive
// halving over lane bits 3, 2, 1 (each lane keeps the half of its values
// selected by the bit and adds the other half of its partner's, the partner
// differing in that bit), then plain sums over lane bits 0, 4, 5.  Lane 2 i
// (i < 8) ends with the total of value i.  One eighth of the exchanges of eight
// separate wavefront sums; the summation order is fixed.
__device__ inline double reduce_scatter8(const double* v, int lane) {
  const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
  double w[4], u[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = (b3 ? v[k + 4] : v[k]) + dpp<DPP_X15>(b3 ? v[k] : v[k + 4]);
#pragma unroll
  for (int k = 0; k < 2; ++k) u[k] = (b2 ? w[k + 2] : w[k]) + dpp<DPP_X7>(b2 ? w[k] : w[k + 2]);
  double z = (b1 ? u[1] : u[0]) + dpp<DPP_X2>(b1 ? u[0] : u[1]);
  z += dpp<DPP_X1>(z);
  z += __shfl_xor(z, 16, 64);
  z += __shfl_xor(z, 32, 64);
  return z;
}

// near-field block SpMV: one wavefront per leaf, lanes over the leaf's source
// panels, target rows in groups of four.  Every load of a step is issued
// unconditionally (addresses clamped into the leaf's block, the clamped
// source's contribution masked), so a lane has all of them in flight at once;
// the eight row sums of a group are one reduce-scatter.
template <typename E>
__global__ void __launch_bounds__(256) k_spmv(const E* __restrict__ ent, const int32_t* __restrict__ leaf_start,
                                              const int32_t* __restrict__ leaf_cnt,
                                              const int64_t* __restrict__ src_off,
                                              const int64_t* __restrict__ ent_off,
                                              const int32_t* __restrict__ src_tree,
                                              const int32_t* __restrict__ perm, int64_t N, int nl,
                                              const double* __restrict__ xt, double* __restrict__ y) {
  constexpr int RG = 4;
  // contiguous leaf ranges per XCD (workgroups are dealt round-robin)
  const int nbx = (int)((gridDim.x + 7) / 8);
  const int blk = (int)(blockIdx.x & 7) * nbx + (int)(blockIdx.x >> 3);
  const int c = blk * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= nl) return;
  const int nc = leaf_cnt[c], i0 = leaf_start[c];
  const int64_t so = src_off[c];
  const int S = (int)(src_off[c + 1] - so);
  const E* base = ent + ent_off[c];
  for (int r0 = 0; r0 < nc; r0 += RG) {
    const int nr = min(RG, nc - r0);
    double a[2 * RG];   // rows' first components, then second components
#pragma unroll
    for (int r = 0; r < 2 * RG; ++r) a[r] = 0.0;
    int jn = src_tree[so + min(lane, S - 1)];   // the next step's source, loaded one step ahead
    for (int k0 = 0; k0 < S; k0 += 64) {
      const int k = min(k0 + lane, S - 1);
      const int j = jn;
      if (k0 + 64 < S) jn = src_tree[so + min(k0 + 64 + lane, S - 1)];
      E e[RG];
#pragma unroll
      for (int r = 0; r < RG; ++r) e[r] = base[(int64_t)min(r0 + r, nc - 1) * S + k];
      double2 xv = reinterpret_cast<const double2*>(xt)[j];
      if (k0 + lane >= S) xv = make_double2(0.0, 0.0);
#pragma unroll
      for (int r = 0; r < RG; ++r) {
        a[r] += (double)e[r].x * xv.x + (double)e[r].y * xv.y;
        a[RG + r] += (double)e[r].z * xv.x + (double)e[r].w * xv.y;
      }
    }
    const double z = reduce_scatter8(a, lane);
    const int v = (lane >> 1) & 7, r = v & 3;
    if (lane < 16 && !(lane & 1) && r < nr) {
      const int p = perm[i0 + r0 + r];
      y[v < RG ? p : N + p] = z;
    }
  }
}

// xt = x in tree order, (phi, dphi) interleaved per row: row i takes entry
// idx[i] of both channels of x (channel stride n_x)
__global__ void k_to_tree(const double* __restrict__ x, const int32_t* __restrict__ idx, int64_t n,
                          int64_t n_x, double* xt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t p = idx[i];
  reinterpret_cast<double2*>(xt)[i] = make_double2(x[p], x[n_x + p]);
}

ElemView box_view(fagbi_handle* h) {
  ElemView v;
  v.n = v.n_near = h->N;
  v.leaf_start = v.near_start = h->d_leaf_start.as<int32_t>();
  v.leaf_cnt = v.near_cnt = h->d_leaf_cnt.as<int32_t>();
  v.leaf_of = h->d_leaf_of.as<int32_t>();
  v.near_src = h->d_src_tree.as<int32_t>();
  v.near_src_off = h->d_src_off.as<int64_t>();
  v.near_ent_off = h->d_ent_off.as<int64_t>();
  v.in_idx = v.out_idx = v.out_near = h->d_perm.as<int32_t>();
  v.in_stride = h->N;
  v.xt = h->d_xt.as<double>();
  return v;
}

// ---------------------------------------------------------------------------
// setup: slot tables, Taylor tables per (level, offset), moments
// ---------------------------------------------------------------------------
// All tables and expansion arrays of the far field live in one device
// allocation: the host side is packed into one staging buffer and copied
// with one transfer; the DBufs are views into the pool (not owned).
// Taylor coefficients of one offset by the recurrence above (one thread per
// offset and channel: kappa = 0 for G0), written as D_g = g! F_g / (4 pi)
// into the interleaved {G0, Gk} tables, FP64 and FP32
struct TaylorJob {
  const int32_t* off;
  double* dt;
  float* dt32;
  double h;
  int n_off, p, T;
};
struct TaylorJobs {
  TaylorJob j[FAGBI_MAX_LEVELS];
  int n;
};
// every level's tables in one launch: thread i -> (level, offset, channel)
__global__ void __launch_bounds__(64) k_taylor_table(TaylorJobs jobs, double kappa) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int l = 0;
  while (l < jobs.n && i >= 2 * jobs.j[l].n_off) i -= 2 * jobs.j[l].n_off, ++l;
  if (l >= jobs.n) return;
  const int32_t* __restrict__ off = jobs.j[l].off;
  const double h = jobs.j[l].h;
  const int p = jobs.j[l].p, T = jobs.j[l].T;
  double* dt = jobs.j[l].dt;
  float* dt32 = jobs.j[l].dt32;
  const int o = i >> 1, ch = i & 1;
  const double ka = ch ? kappa : 0.0;
  const double x0[3] = {off[3 * o] * h, off[3 * o + 1] * h, off[3 * o + 2] * h};
  double F[TMAX], H[TMAX];
  const double r2 = x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2];
  const double r0 = sqrt(r2);
  F[0] = exp(-ka * r0) / r0;
  H[0] = exp(-ka * r0);
  for (int d = 1; d <= p; ++d)
    for (int a = d; a >= 0; --a)
      for (int b = d - a; b >= 0; --b) {
        const int c = d - a - b;
        const int k[3] = {a, b, c};
        double s1f = 0, s2f = 0, s1h = 0, s2h = 0;
        for (int ax = 0; ax < 3; ++ax) {
          if (k[ax] >= 1) {
            const int id = midx(a - (ax == 0), b - (ax == 1), c - (ax == 2));
            s1f += x0[ax] * F[id];
            s1h += x0[ax] * H[id];
          }
          if (k[ax] >= 2) {
            const int id = midx(a - 2 * (ax == 0), b - 2 * (ax == 1), c - 2 * (ax == 2));
            s2f += F[id];
            s2h += H[id];
          }
        }
        const int id = midx(a, b, c);
        F[id] = (-ka * (s1h + s2h) - (2 * d - 1) * s1f - (d - 1) * s2f) / (d * r2);
        H[id] = -ka * (s1f + s2f) / d;
      }
  for (int d = 0; d <= p; ++d)
    for (int a = d; a >= 0; --a)
      for (int b = d - a; b >= 0; --b) {
        const int c = d - a - b, g = midx(a, b, c);
        double f = 1.0 / FOUR_PI;
        for (int q = 2; q <= a; ++q) f *= q;
        for (int q = 2; q <= b; ++q) f *= q;
        for (int q = 2; q <= c; ++q) f *= q;
        const double v = f * F[g];
        dt[2 * ((int64_t)o * T + g) + ch] = v;
        dt32[2 * ((int64_t)o * T + g) + ch] = (float)v;
      }
}

// the table rows of one offset of each opposite pair
template <typename R>
__global__ void k_half_rows(const int32_t* __restrict__ rows, int n_half, int T, const R* __restrict__ full,
                            R* half) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_half * 2 * T) return;
  const int64_t k = i / (2 * T), r = i - k * 2 * T;
  half[i] = full[(int64_t)rows[k] * 2 * T + r];
}

// the octant table: row k is D(|o|) of its class, from the representative
// offset o by D_g(|o|) = (-1)^(g . s) D_g(o); mi: the terms' exponents
__global__ void k_oct_rows(const int32_t* __restrict__ rows8, int n_oct, int T, const int8_t* __restrict__ mi,
                           const float* __restrict__ full, float* oct) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_oct * 2 * T) return;
  const int64_t k = i / (2 * T), r = i - k * 2 * T;
  const int g = (int)(r >> 1);
  const uint32_t v = (uint32_t)rows8[k], sg = v >> 29;
  const int odd = ((mi[3 * g] & 1) & (int)(sg & 1)) ^ ((mi[3 * g + 1] & 1) & (int)((sg >> 1) & 1)) ^
                  ((mi[3 * g + 2] & 1) & (int)((sg >> 2) & 1));
  const float f = full[(int64_t)(v & 0x1fffffffu) * 2 * T + r];
  oct[i] = odd ? -f : f;
}

struct Staging {
  struct Item {
    DBuf* b;
    size_t off, bytes;
  };
  std::vector<char> host;
  std::vector<Item> items;
  size_t dev_bytes = 0;   // device-only regions, after the host data
  static size_t up(size_t n) { return (n + 255) & ~(size_t)255; }
  void add(DBuf& b, const void* data, size_t bytes) {
    const size_t off = up(host.size());
    host.resize(off + bytes);
    if (bytes) memcpy(host.data() + off, data, bytes);
    items.push_back({&b, off, bytes});
  }
  template <typename R> void add_conv(DBuf& b, const std::vector<double>& v) {
    std::vector<R> t(v.begin(), v.end());
    add(b, t.data(), t.size() * sizeof(R));
  }
  void reserve(DBuf& b, size_t bytes) {
    items.push_back({&b, ~(size_t)0 - dev_bytes, bytes});   // resolved in commit
    dev_bytes += up(bytes);
  }
  int commit(fagbi_handle* h, DBuf& pool) {
    const size_t hb = up(host.size());
    FAGBI_TRY(h->alloc(pool, hb + dev_bytes));
    if (!host.empty()) FAGBI_HIP(hipMemcpy(pool.p, host.data(), host.size(), hipMemcpyHostToDevice));
    for (const Item& it : items) {
      const size_t off = it.off <= host.size() ? it.off : hb + (~(size_t)0 - it.off);
      it.b->p = static_cast<char*>(pool.p) + off;
      it.b->bytes = it.bytes;
    }
    return 0;
  }
};

// source-reuse MtL tables of level l (FP32, order 3).  Tiles start as MTK
// consecutive targets; a tile whose distinct sources do not fit the LDS left
// beside the half table is split in halves until every tile fits.  D.n_tile
// stays 0 when the level does not qualify (a single target whose sources do
// not fit).
constexpr int MT_LDS = 160 * 1024;   // a CU's LDS
constexpr size_t MT_SETUP_LDS = (size_t)2 * (MT_BITS / 32) * 4;   // setup bitmap and word prefixes
static int m2l_tile_setup(fagbi_handle* h, int l, hipStream_t s) {
  Level& D = h->lev[l];
  D.n_tile = 0;
  if (D.order != 3 || D.n_half == 0 || D.n_half >= (1 << 19) || D.n_inter == 0 || l < h->lmin) return 0;
  const int64_t row = (int64_t)(D.T + 2) * sizeof(float2);   // the tile kernel's padded LDS row
  const int64_t stat_lds = (int64_t)MTK * 2 * D.T * 4 + (MTK + 1) * 4 + D.T * 4 + 256;
  const int64_t cap = std::min<int64_t>(std::min<int64_t>(MT_UMAX, (int64_t)MT_IPT * MT_NT / (D.T / 4)),
                                        (MT_LDS - stat_lds - (int64_t)D.n_half * row) / row);
  if (cap < 64) return 0;
  for (int pass = 0; pass < 2; ++pass)
    FAGBI_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(pass ? &k_tile_setup<1> : &k_tile_setup<0>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)MT_SETUP_LDS));
  // tiles start as MTK consecutive targets; only tiles that were split are
  // counted again (their halves), the others keep their count
  std::vector<int32_t> t0;
  for (int c = 0; c < D.n; c += MTK) t0.push_back(c);
  t0.push_back(D.n);
  const int32_t *io = D.d_inter_off.as<int32_t>(), *is = D.d_inter_src.as<int32_t>(),
                *id = D.d_inter_oid.as<int32_t>(), *om = D.d_oid_map.as<int32_t>();
  std::vector<int32_t> hc(t0.size() - 1, -1);   // -1: not counted yet
  int umax = 0;
  Tmp dt0, cnt;
  for (int round = 0;; ++round) {
    // the ranges not counted yet: first targets, then last targets
    std::vector<int32_t> todo, lohi;
    for (size_t t = 0; t + 1 < t0.size(); ++t)
      if (hc[t] < 0) todo.push_back((int32_t)t);
    if (todo.empty()) break;
    if (round == 9) return 0;
    const int nq = (int)todo.size();
    for (int k = 0; k < nq; ++k) lohi.push_back(t0[todo[k]]);
    for (int k = 0; k < nq; ++k) lohi.push_back(t0[todo[k] + 1]);
    dt0.release();
    cnt.release();
    FAGBI_TRY(dt0.alloc(lohi.size() * 4));
    FAGBI_TRY(cnt.alloc((size_t)nq * 4));
    FAGBI_HIP(hipMemcpyAsync(dt0.p, lohi.data(), lohi.size() * 4, hipMemcpyHostToDevice, s));
    k_tile_setup<0><<<nq, 256, MT_SETUP_LDS, s>>>(io, is, id, om, dt0.as<int32_t>(), dt0.as<int32_t>() + nq,
                                                  cnt.as<int32_t>(), nullptr, nullptr, nullptr);
    FAGBI_HIP(hipGetLastError());
    std::vector<int32_t> got(nq);
    FAGBI_HIP(hipMemcpyAsync(got.data(), cnt.p, got.size() * 4, hipMemcpyDeviceToHost, s));
    FAGBI_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < nq; ++k) hc[todo[k]] = got[k];
    // split the tiles that do not fit
    std::vector<int32_t> nt0, nhc;
    for (size_t t = 0; t + 1 < t0.size(); ++t) {
      if (hc[t] > cap) {
        if (t0[t + 1] - t0[t] < 2) return 0;
        nt0.push_back(t0[t]);
        nt0.push_back((t0[t] + t0[t + 1]) / 2);
        nhc.push_back(-1);
        nhc.push_back(-1);
      } else {
        nt0.push_back(t0[t]);
        nhc.push_back(hc[t]);
      }
    }
    nt0.push_back(D.n);
    t0.swap(nt0);
    hc.swap(nhc);
  }
  for (int c : hc) umax = std::max(umax, c);
  const int nt = (int)t0.size() - 1;
  FAGBI_TRY(h->alloc(D.d_tile_t0, t0.size() * 4));
  FAGBI_HIP(hipMemcpyAsync(D.d_tile_t0.p, t0.data(), t0.size() * 4, hipMemcpyHostToDevice, s));
  std::vector<int32_t> off(nt + 1, 0);
  for (int t = 0; t < nt; ++t) off[t + 1] = off[t] + hc[t];
  FAGBI_TRY(h->alloc(D.d_tile_off, off.size() * 4));
  FAGBI_HIP(hipMemcpyAsync(D.d_tile_off.p, off.data(), off.size() * 4, hipMemcpyHostToDevice, s));
  FAGBI_TRY(h->alloc(D.d_tile_src, (size_t)std::max(1, off[nt]) * 4));
  FAGBI_TRY(h->alloc(D.d_pack, (size_t)D.n_inter * 4));
  k_tile_setup<1><<<nt, 256, MT_SETUP_LDS, s>>>(io, is, id, om, D.d_tile_t0.as<int32_t>(),
                                                D.d_tile_t0.as<int32_t>() + 1, nullptr, D.d_tile_off.as<int32_t>(),
                                                D.d_tile_src.as<int32_t>(), D.d_pack.as<uint32_t>());
  FAGBI_HIP(hipGetLastError());
  FAGBI_HIP(hipStreamSynchronize(s));   // the host copies above are freed on return
  D.n_tile = nt;
  D.tile_umax = umax;
  return 0;
}

static int spt_of(int nslot) {
  const int s = (nslot + TB - 1) / TB;
  return s <= 1 ? 1 : s <= 2 ? 2 : s <= 4 ? 4 : s <= 8 ? 8 : 16;
}

int fmm_setup(fagbi_handle* h, hipStream_t s) {
  Staging st;
  std::vector<int8_t> mi(3 * TMAX);
  for (int t = 0; t < TMAX; ++t) {
    const MI m = mi_of(t);
    for (int d = 0; d < 3; ++d) mi[3 * t + d] = (int8_t)m.a[d];
  }
  st.add(h->d_mi, mi.data(), mi.size());
  {
    // order-3 matrix-core MtL: X entry (derivative tile t, lane k + 16 j,
    // element e) = X[16 t + 4 j + e][k] -> local term g - b, or -1
    std::vector<int8_t> xd(2 * 4 * 16 * 4, -1);
    for (int t = 0; t < 2; ++t)
      for (int j = 0; j < 4; ++j)
        for (int k = 0; k < 16; ++k)
          for (int e = 0; e < 4; ++e) {
            const int g = 16 * t + 4 * j + e;
            if (g >= nterms(3)) continue;
            const MI G = mi_of(g), B = mi_of(k);
            if (B.a[0] > G.a[0] || B.a[1] > G.a[1] || B.a[2] > G.a[2]) continue;
            xd[((t * 4 + j) * 16 + k) * 4 + e] = (int8_t)midx(G.a[0] - B.a[0], G.a[1] - B.a[1], G.a[2] - B.a[2]);
          }
    st.add(h->d_xdst, xd.data(), xd.size());
  }
  {
    const std::vector<int32_t> zero((size_t)16 * (h->L + 1), 0);
    st.add(h->d_mtl_ctr, zero.data(), zero.size() * sizeof(int32_t));
  }
  const int lo = std::min(h->lmin, h->L);
  for (int l = lo; l <= h->L; ++l) {
    Level& D = h->lev[l];
    // MtL slots: (alpha, beta), |alpha| + |beta| <= p, grouped by alpha;
    // scale tables (-1)^|b|/b! for the moments and 1/a! for the locals
    if (l >= h->lmin) {
      std::vector<int32_t> slot, aoff(1, 0);
      std::vector<double> msc(D.T), lsc(D.T);
      for (int ta = 0; ta < D.T; ++ta) {
        const MI A = mi_of(ta);
        const int da = A.a[0] + A.a[1] + A.a[2];
        const double af = fact(A.a[0]) * fact(A.a[1]) * fact(A.a[2]);
        msc[ta] = ((da & 1) ? -1.0 : 1.0) / af;
        lsc[ta] = 1.0 / af;
        for (int tb = 0; tb < nterms(D.order - da); ++tb) {
          const MI B = mi_of(tb);
          slot.push_back(midx(A.a[0] + B.a[0], A.a[1] + B.a[1], A.a[2] + B.a[2]) | (tb << 16));
        }
        aoff.push_back((int32_t)slot.size());
      }
      D.m2l_nslot = (int)slot.size();
      st.add(D.d_m2l_slot, slot.data(), slot.size() * 4);
      st.add(D.d_m2l_aoff, aoff.data(), aoff.size() * 4);
      std::vector<double> sc(msc);
      sc.insert(sc.end(), lsc.begin(), lsc.end());
      st.add_conv<double>(D.d_m2l_c64, sc);
      st.add_conv<float>(D.d_m2l_c32, sc);
    }
    // shifts between level l (parent, order p_l) and l+1 (child, p_{l+1})
    if (l < h->L) {
      const Level& C = h->lev[l + 1];
      struct P2 {
        int a, b;
      };
      std::vector<P2> pairs;
      for (int ta = 0; ta < D.T; ++ta)
        for (int tb = 0; tb < C.T; ++tb) {
          const MI A = mi_of(ta), B = mi_of(tb);
          if (B.a[0] <= A.a[0] && B.a[1] <= A.a[1] && B.a[2] <= A.a[2]) pairs.push_back({ta, tb});
        }
      // child centre - parent centre = (bit - 1/2) h_child per axis: powers of
      // h_child/2 with the sign of odd powers taken from the octant bit
      double hp[PMAX + 1];
      hp[0] = 1.0;
      for (int k = 1; k <= PMAX; ++k) hp[k] = hp[k - 1] * (0.5 * C.h);
      auto coef = [&](const P2& q, int oct) {
        const MI A = mi_of(q.a), B = mi_of(q.b);
        double v = 1.0;
        for (int ax = 0; ax < 3; ++ax) {
          const int k = A.a[ax] - B.a[ax];
          const bool neg = !((oct >> (2 - ax)) & 1) && (k & 1);
          v *= binom(A.a[ax], B.a[ax]) * (neg ? -hp[k] : hp[k]);
        }
        return v;
      };
      // MtM: grouped by parent index a (pairs are generated in a order)
      {
        std::vector<int32_t> slot, aoff(D.T + 1, 0);
        std::vector<double> cf(8 * pairs.size());
        for (size_t k = 0; k < pairs.size(); ++k) {
          slot.push_back(pairs[k].a | (pairs[k].b << 16));
          aoff[pairs[k].a + 1] = (int32_t)(k + 1);
        }
        for (int t = 1; t <= D.T; ++t) aoff[t] = std::max(aoff[t], aoff[t - 1]);
        for (int oct = 0; oct < 8; ++oct)
          for (size_t k = 0; k < pairs.size(); ++k) cf[oct * pairs.size() + k] = coef(pairs[k], oct);
        D.up_nslot = (int)pairs.size();
        st.add(D.d_up_slot, slot.data(), slot.size() * 4);
        st.add(D.d_up_aoff, aoff.data(), aoff.size() * 4);
        st.add_conv<double>(D.d_up_c64, cf);
        st.add_conv<float>(D.d_up_c32, cf);
      }
      // LtL: grouped by child index b
      {
        std::vector<P2> byb(pairs);
        std::stable_sort(byb.begin(), byb.end(), [](const P2& x, const P2& y) { return x.b < y.b; });
        std::vector<int32_t> slot, boff(C.T + 1, 0);
        std::vector<double> cf(8 * byb.size());
        for (size_t k = 0; k < byb.size(); ++k) {
          slot.push_back(byb[k].a | (byb[k].b << 16));
          boff[byb[k].b + 1] = (int32_t)(k + 1);
        }
        for (int t = 1; t <= C.T; ++t) boff[t] = std::max(boff[t], boff[t - 1]);
        for (int oct = 0; oct < 8; ++oct)
          for (size_t k = 0; k < byb.size(); ++k) cf[oct * byb.size() + k] = coef(byb[k], oct);
        D.dn_nslot = (int)byb.size();
        st.add(D.d_dn_slot, slot.data(), slot.size() * 4);
        st.add(D.d_dn_boff, boff.data(), boff.size() * 4);
        st.add_conv<double>(D.d_dn_c64, cf);
        st.add_conv<float>(D.d_dn_c32, cf);
      }
    }
    // derivative tables per offset, D_g = g! F_g / (4 pi), channels
    // interleaved {G0, Gk}: computed on the device after the upload
    if (l >= h->lmin && D.n_off > 0) {
      st.add(D.d_off, D.off_xyz.data(), D.off_xyz.size() * 4);
      st.reserve(D.d_F64[0], (size_t)2 * D.n_off * D.T * 8);
      st.reserve(D.d_F32[0], (size_t)2 * D.n_off * D.T * 4);
      // one of each pair of opposite offsets (first non-zero component > 0)
      // for the LDS-staged kernels, and the map oid -> row | flip << 30
      std::vector<int32_t> omap(D.n_off, -1), rows;
      auto key = [&](int o, int sgn) {
        return ((int64_t)(sgn * D.off_xyz[3 * o]) + 1024) * 4194304 + ((int64_t)(sgn * D.off_xyz[3 * o + 1]) + 1024) * 2048 +
               (sgn * D.off_xyz[3 * o + 2] + 1024);
      };
      std::vector<std::pair<int64_t, int>> byk(D.n_off);
      for (int o = 0; o < D.n_off; ++o) byk[o] = {key(o, 1), o};
      std::sort(byk.begin(), byk.end());
      bool ok = true;
      for (int o = 0; o < D.n_off && ok; ++o) {
        const int x = D.off_xyz[3 * o], y = D.off_xyz[3 * o + 1], z = D.off_xyz[3 * o + 2];
        const bool canon = x > 0 || (x == 0 && (y > 0 || (y == 0 && z > 0)));
        if (!canon) continue;
        omap[o] = (int32_t)rows.size();
        rows.push_back(o);
        auto it = std::lower_bound(byk.begin(), byk.end(), std::make_pair(key(o, -1), -1));
        if (it == byk.end() || it->first != key(o, -1)) ok = false;
        else omap[it->second] = omap[o] | (1 << 30);
      }
      for (int o = 0; o < D.n_off && ok; ++o) ok = omap[o] >= 0;
      D.n_half = 0;
      if (ok) {
        st.add(D.d_rows, rows.data(), rows.size() * 4);
        st.reserve(D.d_F32[1], (size_t)2 * rows.size() * D.T * 4);
        if (D.order == 3) st.reserve(D.d_F64[1], (size_t)2 * rows.size() * D.T * 8);
        st.add(D.d_oid_map, omap.data(), omap.size() * 4);
        D.n_half = (int)rows.size();
      }
      // octant classes for the order-4 LDS kernel: the kernels are even in
      // each coordinate, D_g(o) = (-1)^(g . s) D_g(|o|) with s the signs of o
      D.n_oct = 0;
      if (D.order == 4 && D.n_off < (1 << 29)) {
        std::vector<int32_t> omap8(D.n_off), rows8;
        std::vector<std::pair<int64_t, int>> cls;   // (class key, row), sorted by key
        for (int o = 0; o < D.n_off; ++o) {
          const int x = D.off_xyz[3 * o], y = D.off_xyz[3 * o + 1], z = D.off_xyz[3 * o + 2];
          const uint32_t sg = (uint32_t)(x < 0) | (uint32_t)(y < 0) << 1 | (uint32_t)(z < 0) << 2;
          const int64_t k = ((int64_t)std::abs(x) * 2048 + std::abs(y)) * 2048 + std::abs(z);
          auto it = std::lower_bound(cls.begin(), cls.end(), std::make_pair(k, -1));
          int row;
          if (it != cls.end() && it->first == k) {
            row = it->second;
          } else {
            row = (int)rows8.size();
            cls.insert(it, {k, row});
            rows8.push_back((int32_t)((uint32_t)o | sg << 29));
          }
          omap8[o] = (int32_t)((uint32_t)row | sg << 29);
        }
        st.add(D.d_rows8, rows8.data(), rows8.size() * 4);
        st.reserve(D.d_F32o, (size_t)2 * rows8.size() * D.T * 4);
        st.add(D.d_oid_map8, omap8.data(), omap8.size() * 4);
        D.n_oct = (int)rows8.size();
      }
    }
    for (int ch = 0; ch < 2; ++ch) {
      st.reserve(D.d_M64[ch], (size_t)D.n * D.T * 8);
      st.reserve(D.d_L64[ch], (size_t)D.n * D.T * 8);
      st.reserve(D.d_M32[ch], (size_t)D.n * D.T * 4);
      st.reserve(D.d_L32[ch], (size_t)D.n * D.T * 4);
    }
  }
  // panel (or panel-corner) moments about the leaf centres
  const Level& LF = h->lev[h->L];
  const int T = LF.T;
  const int corners = h->hat() ? 1 : 0;
  const int64_t NT = (corners ? 3 : 1) * h->N * T;
  st.reserve(h->d_ms64, NT * 8);
  st.reserve(h->d_md64, NT * 8);
  st.reserve(h->d_ms32, NT * 4);
  st.reserve(h->d_md32, NT * 4);
  FAGBI_TRY(st.commit(h, h->d_fmm_pool));
  {
    TaylorJobs jobs{};
    int64_t nth = 0;
    for (int l = std::max(lo, h->lmin); l <= h->L; ++l) {
      Level& D = h->lev[l];
      if (D.n_off == 0) continue;
      jobs.j[jobs.n++] = TaylorJob{D.d_off.as<int32_t>(), D.d_F64[0].as<double>(), D.d_F32[0].as<float>(), D.h,
                                   D.n_off, D.order, D.T};
      nth += 2 * (int64_t)D.n_off;
    }
    if (jobs.n > 0) k_taylor_table<<<(unsigned)((nth + 63) / 64), 64, 0, s>>>(jobs, h->prm.kappa);
  }
  for (int l = std::max(lo, h->lmin); l <= h->L; ++l) {
    Level& D = h->lev[l];
    if (D.n_off == 0) continue;
    if (D.n_half > 0) {
      const int64_t m = (int64_t)D.n_half * 2 * D.T;
      k_half_rows<float><<<(unsigned)((m + 255) / 256), 256, 0, s>>>(D.d_rows.as<int32_t>(), D.n_half, D.T,
                                                                    D.d_F32[0].as<float>(), D.d_F32[1].as<float>());
      if (D.order == 3)
        k_half_rows<double><<<(unsigned)((m + 255) / 256), 256, 0, s>>>(D.d_rows.as<int32_t>(), D.n_half, D.T,
                                                                       D.d_F64[0].as<double>(),
                                                                       D.d_F64[1].as<double>());
    }
    if (D.n_oct > 0) {
      const int64_t m = (int64_t)D.n_oct * 2 * D.T;
      k_oct_rows<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(D.d_rows8.as<int32_t>(), D.n_oct, D.T,
                                                             h->d_mi.as<int8_t>(), D.d_F32[0].as<float>(),
                                                             D.d_F32o.as<float>());
    }
  }
  FAGBI_HIP(hipGetLastError());
  FAGBI_TRY(m2l_tile_setup(h, h->L, s));
  const unsigned grid = (unsigned)((NT + 255) / 256);
  k_panel_moments<double><<<grid, 256, 0, s>>>(h->d_pv.as<double>(), h->d_pn.as<double>(), h->d_pa.as<double>(),
                                                h->d_leaf_of.as<int32_t>(), LF.d_idx.as<int32_t>(), h->corner[0],
                                                h->corner[1], h->corner[2], LF.h, (int)h->N, T,
                                                h->d_mi.as<int8_t>(), h->d_ms64.as<double>(),
                                                h->d_md64.as<double>(), corners);
  k_panel_moments<float><<<grid, 256, 0, s>>>(h->d_pv.as<double>(), h->d_pn.as<double>(), h->d_pa.as<double>(),
                                               h->d_leaf_of.as<int32_t>(), LF.d_idx.as<int32_t>(), h->corner[0],
                                               h->corner[1], h->corner[2], LF.h, (int)h->N, T,
                                               h->d_mi.as<int8_t>(), h->d_ms32.as<float>(),
                                               h->d_md32.as<float>(), corners);
  FAGBI_HIP(hipGetLastError());
  return 0;
}

// launch helpers dispatching on slots per thread
#define FAGBI_SPT_SWITCH(spt, KER, GRID, SH, STREAM, ...)                  \
  switch (spt) {                                                            \
    case 1: KER<R, 1><<<GRID, TB, SH, STREAM>>>(__VA_ARGS__); break;        \
    case 2: KER<R, 2><<<GRID, TB, SH, STREAM>>>(__VA_ARGS__); break;        \
    case 4: KER<R, 4><<<GRID, TB, SH, STREAM>>>(__VA_ARGS__); break;        \
    case 8: KER<R, 8><<<GRID, TB, SH, STREAM>>>(__VA_ARGS__); break;        \
    default: KER<R, 16><<<GRID, TB, SH, STREAM>>>(__VA_ARGS__); break;      \
  }

template <typename R>
static R* moments_of(Level& D, int ch, bool f32) {
  return f32 ? D.d_M32[ch].as<R>() : D.d_M64[ch].as<R>();
}

// step 2: leaf moments of the two channels from the rows' values xt (tree order)
template <typename R>
static int launch_p2m(fagbi_handle* h, const ElemView& v, const R* ms, const R* md, bool f32, hipStream_t s) {
  Level& LF = h->lev[h->L];
  const int nl = LF.n;
  const double eps = h->prm.eps_out / h->prm.eps_in;
  const int64_t tot = (int64_t)nl * LF.T;
  k_p2m<R><<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(ms, md, v.leaf_start, v.leaf_cnt, v.n, nl, LF.T, eps,
                                                        v.xt, moments_of<R>(LF, 0, f32), moments_of<R>(LF, 1, f32));
  return 0;
}

// step 3 for one level: moments of level l from those of level l + 1
template <typename R>
static int launch_m2m(fagbi_handle* h, int l, bool f32, hipStream_t s) {
  Level &P = h->lev[l], &C = h->lev[l + 1];
  R *c0 = moments_of<R>(C, 0, f32), *ck = moments_of<R>(C, 1, f32);
  R *p0 = moments_of<R>(P, 0, f32), *pk = moments_of<R>(P, 1, f32);
  const unsigned gp = (unsigned)((P.n + 255) / 256);
  if (f32 && P.order == 4 && C.order == 3) {
    k_m2m_reg<R, 4, 3><<<gp, 256, 0, s>>>(P.d_child_start.as<int32_t>(), P.d_child_end.as<int32_t>(),
                                         C.d_idx.as<int32_t>(), P.n, (R)C.h, c0, ck, p0, pk);
    return 0;
  }
  if (P.order == 3 && C.order == 3) {
    k_m2m_reg<R, 3, 3><<<gp, 256, 0, s>>>(P.d_child_start.as<int32_t>(), P.d_child_end.as<int32_t>(),
                                         C.d_idx.as<int32_t>(), P.n, (R)C.h, c0, ck, p0, pk);
    return 0;
  }
  const size_t sh = std::max<size_t>((size_t)16 * C.T, (size_t)2 * P.up_nslot) * sizeof(R);
  const R* coef = f32 ? P.d_up_c32.as<R>() : P.d_up_c64.as<R>();
  FAGBI_SPT_SWITCH(spt_of(P.up_nslot), k_m2m, P.n, sh, s, P.d_child_start.as<int32_t>(),
                   P.d_child_end.as<int32_t>(), C.d_idx.as<int32_t>(), P.d_up_slot.as<int32_t>(), coef,
                   P.d_up_aoff.as<int32_t>(), P.up_nslot, P.T, C.T, c0, ck, p0, pk);
  return 0;
}

template <typename R>
static R* locals_of(Level& D, int ch, bool f32) {
  return f32 ? D.d_L32[ch].as<R>() : D.d_L64[ch].as<R>();
}

// step 5 for one level: locals of level l + 1 += LtL of those of level l
template <typename R>
static int launch_l2l(fagbi_handle* h, int l, bool f32, hipStream_t s) {
  Level &P = h->lev[l], &C = h->lev[l + 1];
  const unsigned gc = (unsigned)((C.n + 255) / 256);
  const int32_t *par = C.d_parent.as<int32_t>(), *cix = C.d_idx.as<int32_t>();
  R *p0 = locals_of<R>(P, 0, f32), *pk = locals_of<R>(P, 1, f32);
  R *c0 = locals_of<R>(C, 0, f32), *ck = locals_of<R>(C, 1, f32);
  if (P.order == 4 && C.order == 3) {
    k_l2l_reg<R, 4, 3><<<gc, 256, 0, s>>>(par, cix, C.n, (R)C.h, p0, pk, c0, ck);
    return 0;
  }
  if (P.order == 3 && C.order == 3) {
    k_l2l_reg<R, 3, 3><<<gc, 256, 0, s>>>(par, cix, C.n, (R)C.h, p0, pk, c0, ck);
    return 0;
  }
  if (f32 && P.order == 5 && C.order == 4) {
    k_l2l_reg<R, 5, 4><<<gc, 256, 0, s>>>(par, cix, C.n, (R)C.h, p0, pk, c0, ck);
    return 0;
  }
  const size_t sh = std::max<size_t>((size_t)2 * P.T, (size_t)2 * P.dn_nslot) * sizeof(R);
  const R* coef = f32 ? P.d_dn_c32.as<R>() : P.d_dn_c64.as<R>();
  FAGBI_SPT_SWITCH(spt_of(P.dn_nslot), k_l2l, C.n, sh, s, par, cix, P.d_dn_slot.as<int32_t>(), coef,
                   P.d_dn_boff.as<int32_t>(), P.dn_nslot, P.T, C.T, p0, pk, c0, ck);
  return 0;
}

template <typename R, typename E>
static int matvec_t(fagbi_handle* h, const ElemView& v, const double* x, double* y_out, int parts, hipStream_t s,
                    const DBuf& ent, const DBuf& ms, const DBuf& md, bool f32) {
  // rows: panels, or panel corners summed into the vertices at the end
  const int64_t N = v.n;
  double* y = v.y ? v.y : y_out;
  double* yn = v.y_near ? v.y_near : y;
  const int nl = h->lev[h->L].n;
  const bool prof = h->profiling;
  auto mark_on = [&](int k, hipStream_t st) -> int {
    if (prof) FAGBI_HIP(hipEventRecord(h->ev[k], st));
    return 0;
  };
  auto mark = [&](int k) { return mark_on(k, s); };
  FAGBI_TRY(mark(5));
  double* xt = v.xt;
  k_to_tree<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(x, v.in_idx, N, v.in_stride, xt);
  // the rows' results summed into the caller's outputs (hat functions)
  auto gather = [&]() -> int { return v.gather ? hat_gather(h, y, yn, y_out, s) : 0; };
  if (v.zero_y) FAGBI_HIP(hipMemsetAsync(y, 0, 2 * N * sizeof(double), s));
  const bool near = parts & FAGBI_PART_NEAR;
  const bool far = (parts & FAGBI_PART_FAR) && h->lmin <= h->L;
  // the near-field SpMV (HBM bound) runs on a second stream beside the far
  // field (cache bound); the far field joins it before LtP adds into y
  hipStream_t sn = s;
  if (near && far) {
    if (!h->s_near) {
      FAGBI_HIP(hipStreamCreateWithFlags(&h->s_near, hipStreamNonBlocking));
      FAGBI_HIP(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
      FAGBI_HIP(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    }
    FAGBI_HIP(hipEventRecord(h->ev_fork, s));
    FAGBI_HIP(hipStreamWaitEvent(h->s_near, h->ev_fork, 0));
    sn = h->s_near;
  }
  FAGBI_TRY(mark_on(0, sn));
  if (near) {
    k_spmv<E><<<(unsigned)(((nl + 3) / 4 + 7) / 8 * 8), 256, 0, sn>>>(
        ent.as<E>(), v.near_start, v.near_cnt, v.near_src_off, v.near_ent_off, v.near_src, v.out_near, v.n_near,
        nl, xt, yn);
  } else {
    FAGBI_HIP(hipMemsetAsync(yn, 0, 2 * v.n_near * sizeof(double), s));
  }
  FAGBI_HIP(hipGetLastError());
  FAGBI_TRY(mark_on(1, sn));
  if (sn != s) FAGBI_HIP(hipEventRecord(h->ev_join, sn));
  FAGBI_TRY(mark(6));
  if (!far) {
    FAGBI_TRY(mark(2));
    FAGBI_TRY(mark(3));
    FAGBI_TRY(mark(7));
    FAGBI_TRY(mark(8));
    FAGBI_TRY(gather());
    FAGBI_TRY(mark(4));
    return 0;
  }
  const double eps = h->prm.eps_out / h->prm.eps_in;
  const int L = h->L;
  auto M = [&](Level& D, int ch) { return f32 ? D.d_M32[ch].as<R>() : D.d_M64[ch].as<R>(); };
  auto Lc = [&](Level& D, int ch) { return f32 ? D.d_L32[ch].as<R>() : D.d_L64[ch].as<R>(); };
  // MtL of one level (levels are independent of each other): which kernel
  // serves level l
  enum { K_LDS64, K_TILE_MFMA, K_TILE, K_LDS32, K_REG, K_EMPTY, K_SLOT };
  // register-blocked kernels for the low orders (up to p = 4, FP32 up to 5)
  // (order 5 in registers in FP32 only: the FP64 version would spill)
  const int preg = sizeof(R) == 4 ? 5 : 4;
  // FP32 order 4 stages the octant table, the other LDS kernels the half table
  auto oct = [&](const Level& D) { return sizeof(R) == 4 && D.order == 4 && D.n_oct > 0; };
  auto dbytes_of = [&](const Level& D) {
    return (size_t)(oct(D) ? D.n_oct : D.n_half) * D.T * sizeof(typename Pair<R>::T) + (size_t)D.n_off * 4;
  };
  auto kind_of = [&](const Level& D) -> int {
    const bool small = dbytes_of(D) <= (size_t)150 * 1024;
    // FP64 at order 3: the LDS kernel with the FP64 half table (512 threads: 224 VGPRs)
    if (sizeof(R) == 8 && D.n_half > 0 && D.order == 3 && D.d_F64[1].p && small) return K_LDS64;
    if (sizeof(R) == 4 && D.n_tile > 0 && D.order == 3 && h->m2l_tiles) return h->m2l_mfma ? K_TILE_MFMA : K_TILE;
    if (sizeof(R) == 4 && (D.n_half > 0 || oct(D)) && (D.order == 3 || D.order == 4) && small) return K_LDS32;
    if (D.n_off > 0 && D.order <= preg && D.order >= 1) return K_REG;
    if (D.n_off == 0) return K_EMPTY;   // no interactions: LtL adds into zero locals
    return K_SLOT;
  };
  // the slot kernel's staging batch and LDS bytes for one target per block
  auto slot_batch = [&](const Level& D) {
    return std::max(1, std::min(16, (int)(16384 / (2 * D.T * sizeof(typename Pair<R>::T)))));
  };
  auto slot_lds = [&](const Level& D, int cpb) {
    return (size_t)cpb * std::max<size_t>((size_t)slot_batch(D) * 2 * D.T * sizeof(typename Pair<R>::T),
                                          (size_t)2 * D.m2l_nslot * sizeof(R));
  };
  auto launch_m2l = [&](int l, hipStream_t st) -> int {
    Level& D = h->lev[l];
    using R2 = typename Pair<R>::T;
    const R2* Dt = f32 ? (const R2*)D.d_F32[0].p : (const R2*)D.d_F64[0].p;
    const size_t dbytes = dbytes_of(D);
    int* ctr = h->d_mtl_ctr.as<int32_t>() + 16 * l;   // the persistent kernels' tile claims
    switch (kind_of(D)) {
      case K_LDS64:
        if constexpr (sizeof(R) == 8) {
          int S = 1;
          while (S < 16 && (int64_t)D.n * S < (int64_t)512 * 1024) S <<= 1;
          const R2* Dh = (const R2*)D.d_F64[1].p;
          FAGBI_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_m2l_lds<R, 3, 512>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)dbytes));
          k_m2l_lds<R, 3, 512><<<224, 512, dbytes, st>>>(D.d_inter_off.as<int32_t>(), D.d_inter_src.as<int32_t>(),
                                                         D.d_inter_oid.as<int32_t>(), Dh, D.n_half,
                                                         D.d_oid_map.as<int32_t>(), D.n_off, D.n, S, M(D, 0),
                                                         M(D, 1), Lc(D, 0), Lc(D, 1));
        }
        return 0;
      case K_TILE_MFMA:
        if constexpr (sizeof(R) == 4) {
          // table + zero row, staged moments + zero row, and one row of slack:
          // lanes past term 19 of a zero row read (and discard) up to 96 bytes beyond it
          const size_t lds = ((size_t)D.n_half + 1 + D.tile_umax + 2) * D.T * sizeof(float2);
          FAGBI_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_m2l_tile_mfma<3>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
          k_m2l_tile_mfma<3><<<224, MT_NT, lds, st>>>(D.d_inter_off.as<int32_t>(), D.d_pack.as<uint32_t>(),
                                                      D.d_tile_t0.as<int32_t>(), D.d_tile_off.as<int32_t>(),
                                                      D.d_tile_src.as<int32_t>(), D.n_tile,
                                                      (const float2*)D.d_F32[1].p, D.n_half, D.tile_umax,
                                                      h->d_xdst.as<int8_t>(), M(D, 0), M(D, 1), Lc(D, 0), Lc(D, 1));
        }
        return 0;
      case K_TILE:
        if constexpr (sizeof(R) == 4) {
          const size_t lds = ((size_t)D.n_half + D.tile_umax) * (D.T + 2) * sizeof(float2);
          FAGBI_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_m2l_tile<3>),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
          k_m2l_tile<3><<<224, MT_NT, lds, st>>>(D.d_inter_off.as<int32_t>(), D.d_pack.as<uint32_t>(),
                                                 D.d_tile_t0.as<int32_t>(), D.d_tile_off.as<int32_t>(),
                                                 D.d_tile_src.as<int32_t>(), D.n_tile,
                                                 (const float2*)D.d_F32[1].p, D.n_half, M(D, 0), M(D, 1),
                                                 Lc(D, 0), Lc(D, 1), ctr);
        }
        return 0;
      case K_LDS32:
        if constexpr (sizeof(R) == 4) {
          int S = 1;
          while (S < 16 && (int64_t)D.n * S < (int64_t)512 * 1024) S <<= 1;
          const R2* Dh = (const R2*)D.d_F32[1].p;
          const int32_t* om = D.d_oid_map.as<int32_t>();
          const int32_t *io = D.d_inter_off.as<int32_t>(), *is = D.d_inter_src.as<int32_t>(),
                        *id = D.d_inter_oid.as<int32_t>();
          if (D.order == 3) {
            FAGBI_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_m2l_lds<R, 3, 1024>),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)dbytes));
            // 28 of each XCD's 32 CUs: the persistent blocks hold most of a CU's
            // LDS, and the free CUs keep the main stream's coarse-level MtL from
            // waiting for the whole kernel (measured 1.24 -> 1.20 ms per FP32 matvec)
            k_m2l_lds<R, 3, 1024><<<224, 1024, dbytes, st>>>(io, is, id, Dh, D.n_half, om, D.n_off, D.n, S, M(D, 0),
                                                            M(D, 1), Lc(D, 0), Lc(D, 1));
          } else if (oct(D)) {
            FAGBI_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_m2l_lds<R, 4, 768, true>),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)dbytes));
            k_m2l_lds<R, 4, 768, true><<<MTL_OCT_BLOCKS, 768, dbytes, st>>>(
                io, is, id, (const R2*)D.d_F32o.p, D.n_oct, D.d_oid_map8.as<int32_t>(), D.n_off, D.n, S, M(D, 0),
                M(D, 1), Lc(D, 0), Lc(D, 1));
          } else {
            FAGBI_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_m2l_lds<R, 4, 768>),
                                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)dbytes));
            k_m2l_lds<R, 4, 768><<<256, 768, dbytes, st>>>(io, is, id, Dh, D.n_half, om, D.n_off, D.n, S, M(D, 0),
                                                          M(D, 1), Lc(D, 0), Lc(D, 1));
          }
        }
        return 0;
      case K_REG: {
        int S = 1;
        while (S < 16 && (int64_t)D.n * S < (int64_t)512 * 1024) S <<= 1;
        const unsigned grid = (unsigned)((((int64_t)D.n * S + 255) / 256 + 7) / 8 * 8);
        const int32_t *io = D.d_inter_off.as<int32_t>(), *is = D.d_inter_src.as<int32_t>(),
                      *id = D.d_inter_oid.as<int32_t>();
        switch (D.order) {
          case 1: k_m2l_reg<R, 1><<<grid, 256, 0, st>>>(io, is, id, Dt, D.n, S, M(D, 0), M(D, 1), Lc(D, 0), Lc(D, 1)); break;
          case 2: k_m2l_reg<R, 2><<<grid, 256, 0, st>>>(io, is, id, Dt, D.n, S, M(D, 0), M(D, 1), Lc(D, 0), Lc(D, 1)); break;
          case 3: k_m2l_reg<R, 3><<<grid, 256, 0, st>>>(io, is, id, Dt, D.n, S, M(D, 0), M(D, 1), Lc(D, 0), Lc(D, 1)); break;
          case 4: k_m2l_reg<R, 4><<<grid, 256, 0, st>>>(io, is, id, Dt, D.n, S, M(D, 0), M(D, 1), Lc(D, 0), Lc(D, 1)); break;
          default:
            if constexpr (sizeof(R) == 4)
              k_m2l_reg<R, 5><<<grid, 256, 0, st>>>(io, is, id, Dt, D.n, S, M(D, 0), M(D, 1), Lc(D, 0), Lc(D, 1));
            break;
        }
        return 0;
      }
      case K_EMPTY:
        FAGBI_HIP(hipMemsetAsync(Lc(D, 0), 0, (size_t)D.n * D.T * sizeof(R), st));
        FAGBI_HIP(hipMemsetAsync(Lc(D, 1), 0, (size_t)D.n * D.T * sizeof(R), st));
        return 0;
      default: {
        const R* sc = f32 ? D.d_m2l_c32.as<R>() : D.d_m2l_c64.as<R>();
        const int spt = spt_of(D.m2l_nslot);
        const int cpb = spt == 1 ? std::max(1, std::min(8, TB / D.m2l_nslot)) : 1;
        const unsigned grid = (unsigned)((D.n + cpb - 1) / cpb);
        FAGBI_SPT_SWITCH(spt, k_m2l, grid, slot_lds(D, cpb), st, D.d_inter_off.as<int32_t>(),
                         D.d_inter_src.as<int32_t>(), D.d_inter_oid.as<int32_t>(), Dt, D.d_m2l_slot.as<int32_t>(),
                         sc, sc + D.T, D.d_m2l_aoff.as<int32_t>(), D.m2l_nslot, D.T, slot_batch(D), cpb, D.n,
                         M(D, 0), M(D, 1), Lc(D, 0), Lc(D, 1));
        return 0;
      }
    }
  };
  // MtL of the levels [l0, l1): in FP32 the levels served by the slot kernel
  // at orders 7 and 8 (at least 8 slots per thread: the coarsest, with few
  // clusters each) in one launch, coarsest (longest lists) first, the others
  // one by one after it.  The FP32 matvec waits for this chain (measured
  // 1.057 -> 1.032 ms per matvec at 491k panels); in FP64 the finest levels'
  // MtL is the longest path, and the grouped launch only takes CUs from it
  // (2.276 -> 2.316 ms), so there every level has its own launch.
  auto launch_m2l_range = [&](int l0, int l1, hipStream_t st) -> int {
    MtlLevels<R> ls{};
    int spt = 1;
    size_t sh = 0;
    int64_t nb = 0;
    std::vector<int> rest;
    for (int l = l0; l < l1; ++l) {
      Level& D = h->lev[l];
      const int sp = kind_of(D) == K_SLOT ? spt_of(D.m2l_nslot) : 0;
      if (!f32 || sp < 8 || ls.n == MTL_MAXL) {
        rest.push_back(l);
        continue;
      }
      const R* sc = f32 ? D.d_m2l_c32.as<R>() : D.d_m2l_c64.as<R>();
      auto& v = ls.lv[ls.n++];
      v.off = D.d_inter_off.as<int32_t>();
      v.src = D.d_inter_src.as<int32_t>();
      v.oid = D.d_inter_oid.as<int32_t>();
      v.slot = D.d_m2l_slot.as<int32_t>();
      v.aoff = D.d_m2l_aoff.as<int32_t>();
      v.Dt = f32 ? (const typename Pair<R>::T*)D.d_F32[0].p : (const typename Pair<R>::T*)D.d_F64[0].p;
      v.msc = sc;
      v.M0 = M(D, 0);
      v.Mk = M(D, 1);
      v.L0 = Lc(D, 0);
      v.Lk = Lc(D, 1);
      v.nslot = D.m2l_nslot;
      v.T = D.T;
      v.batch = slot_batch(D);
      v.ncl = D.n;
      v.b0 = (int)nb;
      nb += D.n;
      spt = std::max(spt, spt_of(D.m2l_nslot));
      sh = std::max(sh, slot_lds(D, 1));
    }
    if (ls.n > 0) {
      if (nb > INT32_MAX) return set_error(FAGBI_E_ARG, "too many clusters for one MtL launch");
      if (spt == 8)
        k_m2l_multi<R, 8><<<(unsigned)nb, TB, sh, st>>>(ls);
      else
        k_m2l_multi<R, 16><<<(unsigned)nb, TB, sh, st>>>(ls);
    }
    for (int l : rest) FAGBI_TRY(launch_m2l(l, st));
    return 0;
  };
  // pipelined MtL: the two finest levels (most of the pairs) run on a second
  // stream as soon as their moments exist, beside the rest of the upward pass
  const bool pipe = L - 1 >= h->lmin;
  if (pipe && !h->s_m2l) {
    FAGBI_HIP(hipStreamCreateWithFlags(&h->s_m2l, hipStreamNonBlocking));
    FAGBI_HIP(hipEventCreateWithFlags(&h->ev_up0, hipEventDisableTiming));
    FAGBI_HIP(hipEventCreateWithFlags(&h->ev_up1, hipEventDisableTiming));
    FAGBI_HIP(hipEventCreateWithFlags(&h->ev_m2l, hipEventDisableTiming));
  }
  Level& LF = h->lev[L];
  FAGBI_TRY(launch_p2m<R>(h, v, ms.as<R>(), md.as<R>(), f32, s));
  // the leaf level's MtL, bracketed by events 7, 8 on its stream
  auto launch_m2l_leaf = [&](hipStream_t st) -> int {
    FAGBI_TRY(mark_on(7, st));
    FAGBI_TRY(launch_m2l(L, st));
    return mark_on(8, st);
  };
  if (pipe) {
    FAGBI_HIP(hipEventRecord(h->ev_up0, s));
    FAGBI_HIP(hipStreamWaitEvent(h->s_m2l, h->ev_up0, 0));
    FAGBI_TRY(launch_m2l_leaf(h->s_m2l));
  }
  for (int l = L - 1; l >= h->lmin; --l) {
    if (pipe && l == L - 2) {   // level L-1 moments are complete
      FAGBI_HIP(hipEventRecord(h->ev_up1, s));
      FAGBI_HIP(hipStreamWaitEvent(h->s_m2l, h->ev_up1, 0));
      FAGBI_TRY(launch_m2l(L - 1, h->s_m2l));
    }
    FAGBI_TRY(launch_m2m<R>(h, l, f32, s));
  }
  if (pipe && h->lmin == L - 1) {
    FAGBI_HIP(hipEventRecord(h->ev_up1, s));
    FAGBI_HIP(hipStreamWaitEvent(h->s_m2l, h->ev_up1, 0));
    FAGBI_TRY(launch_m2l(L - 1, h->s_m2l));
  }
  FAGBI_HIP(hipGetLastError());
  FAGBI_TRY(mark(2));
  // The coarse levels' MtL (few clusters at high order: latency bound) run on
  // the near-field stream once the SpMV is done, beside the main stream's
  // finest remaining level; the main stream joins both before LtL.
  const int l_hi = pipe ? L - 2 : L;
  const bool side = sn != s && l_hi > h->lmin;
  if (side) {
    if (!h->ev_upd) FAGBI_HIP(hipEventCreateWithFlags(&h->ev_upd, hipEventDisableTiming));
    FAGBI_HIP(hipEventRecord(h->ev_upd, s));
    FAGBI_HIP(hipStreamWaitEvent(sn, h->ev_upd, 0));
    FAGBI_TRY(launch_m2l_range(h->lmin, l_hi, sn));
    FAGBI_HIP(hipEventRecord(h->ev_join, sn));   // the SpMV and those levels
    FAGBI_TRY(l_hi == L ? launch_m2l_leaf(s) : launch_m2l(l_hi, s));
  } else {
    FAGBI_TRY(launch_m2l_range(h->lmin, std::min(l_hi + 1, L), s));
    if (l_hi == L) FAGBI_TRY(launch_m2l_leaf(s));
  }
  if (pipe) FAGBI_HIP(hipEventRecord(h->ev_m2l, h->s_m2l));
  FAGBI_HIP(hipGetLastError());
  FAGBI_TRY(mark(3));
  if (side) FAGBI_HIP(hipStreamWaitEvent(s, h->ev_join, 0));
  // the LtL into the leaf level is folded into the LtP for the register
  // orders (parent 4 or 3, leaves 3)
  const bool fold = L > h->lmin && LF.order == 3 && (h->lev[L - 1].order == 4 || h->lev[L - 1].order == 3);
  bool joined = false;
  for (int l = h->lmin; l < (fold ? L - 1 : L); ++l) {
    // LtL into the two finest levels adds to their MtL results
    if (pipe && l + 1 == std::max(L - 1, h->lmin + 1)) {
      FAGBI_HIP(hipStreamWaitEvent(s, h->ev_m2l, 0));
      joined = true;
    }
    FAGBI_TRY(launch_l2l<R>(h, l, f32, s));
  }
  if (pipe && !joined) FAGBI_HIP(hipStreamWaitEvent(s, h->ev_m2l, 0));
  if (sn != s && !side) FAGBI_HIP(hipStreamWaitEvent(s, h->ev_join, 0));
  if (fold) {
    Level& PL = h->lev[L - 1];
    const unsigned g = (unsigned)((N + 255) / 256);
    const R *a = ms.as<R>(), *b = md.as<R>();
    const int32_t *lo = v.leaf_of, *pm = v.out_idx, *par = LF.d_parent.as<int32_t>(), *cix = LF.d_idx.as<int32_t>();
    if (PL.order == 4)
      k_l2p_shift<R, 4, 3><<<g, 256, 0, s>>>(a, b, lo, pm, (int)N, eps, Lc(LF, 0), Lc(LF, 1), par, cix, (R)LF.h,
                                              Lc(PL, 0), Lc(PL, 1), y);
    else
      k_l2p_shift<R, 3, 3><<<g, 256, 0, s>>>(a, b, lo, pm, (int)N, eps, Lc(LF, 0), Lc(LF, 1), par, cix, (R)LF.h,
                                              Lc(PL, 0), Lc(PL, 1), y);
  } else {
    const unsigned g = (unsigned)((N + 255) / 256);
    const R *a = ms.as<R>(), *b = md.as<R>();
    const int32_t *lo = v.leaf_of, *pm = v.out_idx;
    switch (LF.order) {
      case 2: k_l2p_reg<R, 2><<<g, 256, 0, s>>>(a, b, lo, pm, (int)N, eps, Lc(LF, 0), Lc(LF, 1), y); break;
      case 3: k_l2p_reg<R, 3><<<g, 256, 0, s>>>(a, b, lo, pm, (int)N, eps, Lc(LF, 0), Lc(LF, 1), y); break;
      case 4: k_l2p_reg<R, 4><<<g, 256, 0, s>>>(a, b, lo, pm, (int)N, eps, Lc(LF, 0), Lc(LF, 1), y); break;
      default:
        k_l2p<R><<<g, 256, 0, s>>>(a, b, lo, pm, (int)N, LF.T, eps, Lc(LF, 0), Lc(LF, 1), y);
        break;
    }
  }
  FAGBI_HIP(hipGetLastError());
  FAGBI_TRY(gather());
  FAGBI_TRY(mark(4));
  return 0;
}

int matvec(fagbi_handle* h, const double* x, double* y, int precision, int parts, hipStream_t s) {
  if (h->profiling && !h->ev[0])
    for (int k = 0; k < 9; ++k) FAGBI_HIP(hipEventCreate(&h->ev[k]));
  const ElemView v = h->hat() ? hat_view(h) : box_view(h);
  int r = precision == FAGBI_MIXED
              ? matvec_t<float, float4>(h, v, x, y, parts, s, h->d_E32, h->d_ms32, h->d_md32, true)
              : matvec_t<double, double4>(h, v, x, y, parts, s, h->d_E64, h->d_ms64, h->d_md64, false);
  if (r < 0 || !h->profiling) return r;
  FAGBI_HIP(hipEventSynchronize(h->ev[4]));
  float t[4], tot;
  FAGBI_HIP(hipEventSynchronize(h->ev[1]));
  FAGBI_HIP(hipEventElapsedTime(&t[0], h->ev[0], h->ev[1]));
  FAGBI_HIP(hipEventElapsedTime(&t[1], h->ev[6], h->ev[2]));
  FAGBI_HIP(hipEventElapsedTime(&t[2], h->ev[2], h->ev[3]));
  FAGBI_HIP(hipEventElapsedTime(&t[3], h->ev[3], h->ev[4]));
  FAGBI_HIP(hipEventElapsedTime(&tot, h->ev[5], h->ev[4]));
  float tleaf;
  FAGBI_HIP(hipEventSynchronize(h->ev[8]));
  FAGBI_HIP(hipEventElapsedTime(&tleaf, h->ev[7], h->ev[8]));
  const int p = precision == FAGBI_MIXED ? 1 : 0;
  fagbi_profile& P = h->prof;
  P.matvecs[p] += 1;
  P.ms_near[p] += t[0];
  P.ms_up[p] += t[1];
  P.ms_m2l[p] += t[2];
  P.ms_down[p] += t[3];
  P.ms_total[p] += tot;
  P.ms_m2l_leaf[p] += tleaf;
  return 0;
}

// ---------------------------------------------------------------------------
// Cartesian treecode for the solvation energy (Sec. 2.5): every charge visits
// the clusters level by level from l0 = min(l_min, L).  A cluster with
// rho_l / R <= theta adds its particle-cluster term, the MtL row alpha = 0 at
// the charge from the FMM moments of the same x:
//   V += sum_|b|<=p_l (-1)^|b| [F_b(x_n - x_c; 0) M0_b + F_b(x_n - x_c; kappa) Mk_b] / 4 pi,
// a cluster that fails passes its children on, and a leaf that fails is
// summed directly with the 3-point rule.  All charges advance together: the
// frontier of a level is a list of (charge, cluster) pairs; one thread per
// pair takes the decision (and sums a failing leaf), the accepted pairs are
// compacted and evaluated by lane groups, the children of the others are
// appended in pair order by a scan.  Contributions meet in device atomics,
// so the summation order (not the value beyond rounding) varies between runs.
// ---------------------------------------------------------------------------
// pairs of one level, at most
constexpr int64_t TC_MAX_PAIRS = (int64_t)1 << 26;
// coefficient storage of one wavefront: 64 / g groups of T(p) terms,
// at most 4 T(4), 2 T(6) or T(8)
constexpr int TC_TG = 2 * nterms(6);

struct TcLevels {
  const int32_t* idx[FAGBI_MAX_LEVELS];
  const int32_t* cs[FAGBI_MAX_LEVELS];
  const int32_t* ce[FAGBI_MAX_LEVELS];
  const double* m0[FAGBI_MAX_LEVELS];
  const double* mk[FAGBI_MAX_LEVELS];
  double* lam[FAGBI_MAX_LEVELS];       // Coulomb locals (right-hand side mode)
  double h[FAGBI_MAX_LEVELS], rho2[FAGBI_MAX_LEVELS];
  // clusters, expansion order p_l, terms T(p_l) (row length of moments and
  // locals), and the order the treecode evaluates, min(p_l, p_max)
  int n[FAGBI_MAX_LEVELS], order[FAGBI_MAX_LEVELS], T[FAGBI_MAX_LEVELS], pt[FAGBI_MAX_LEVELS];
};

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Taylor coefficients F_k (Coulomb), F_k and H_k (screened) of one offset d by
// the recurrence of the MtL tables, degree by degree with the lanes of a
// group over the terms of a degree, contracted with the cluster's moments
// (staged in LDS first) on the fly.  The wavefront runs 64 / g groups of g
// lanes, each on its own accepted cluster (g >= the terms of the top degree).
// Returns this lane's part of the particle-cluster terms (times 4 pi).
// In the right-hand side mode (RHS) the coefficients at x_c - x_n = -d,
// (-1)^|a| F_a(d), times qs are added to the cluster's Coulomb locals lam
// instead (kappa = 0, no moments).
template <bool RHS>
__device__ double tc_far(bool has, double dx, double dy, double dz, double kappa, int p, int T, int g,
                         const double* __restrict__ m0, const double* __restrict__ mk, double* lam, double qs,
                         double* F0, double* FK, double* HK, double* S0, double* SK, int gl) {
  double v = 0, ir = 0, ir2 = 0, E = 0, em1;
  if (has) {
    if (!RHS)
      for (int t = gl; t < T; t += g) {
        S0[t] = m0[t];
        SK[t] = mk[t];
      }
    const double r2 = (dx * dx + dy * dy) + dz * dz;
    ir = inv_sqrt(r2);
    ir2 = ir * ir;
    if (!RHS) exp_expm1(-kappa * (r2 * ir), E, em1);
    if (gl == 0) {
      F0[0] = ir;
      if (!RHS) {
        FK[0] = E * ir;
        HK[0] = E;
      }
    }
  }
  wave_sync();
  if (has && gl == 0) {
    if (RHS) unsafeAtomicAdd(lam, qs * ir);
    else v = ir * S0[0] + E * ir * SK[0];
  }
  const double x0[3] = {dx, dy, dz};
  for (int d = 1; d <= p; ++d) {
    const int below = d * (d + 1) * (d + 2) / 6, nd = (d + 1) * (d + 2) / 2;
    if (has && gl < nd) {
      int m = 0;
      while ((m + 1) * (m + 2) / 2 <= gl) ++m;
      const int sidx = gl - m * (m + 1) / 2;
      const int e[3] = {d - m, m - sidx, sidx};
      // every read is issued (a missing term reads entry 0 with weight 0), so
      // none waits for another
      // (the right-hand side needs the Coulomb coefficients only)
      double a1[3], a2[3], f1[3], k1[3], h1[3], f2[3], k2[3], h2[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int j1 = e[i] >= 1 ? midx(e[0] - (i == 0), e[1] - (i == 1), e[2] - (i == 2)) : 0;
        const int j2 = e[i] >= 2 ? midx(e[0] - 2 * (i == 0), e[1] - 2 * (i == 1), e[2] - 2 * (i == 2)) : 0;
        a1[i] = e[i] >= 1 ? x0[i] : 0.0;
        a2[i] = e[i] >= 2 ? 1.0 : 0.0;
        f1[i] = F0[j1];
        f2[i] = F0[j2];
        if (!RHS) {
          k1[i] = FK[j1];
          h1[i] = HK[j1];
          k2[i] = FK[j2];
          h2[i] = HK[j2];
        }
      }
      double s1f = 0, s2f = 0, s1k = 0, s2k = 0, s1h = 0, s2h = 0;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        s1f += a1[i] * f1[i];
        s2f += a2[i] * f2[i];
        if (!RHS) {
          s1k += a1[i] * k1[i];
          s1h += a1[i] * h1[i];
          s2k += a2[i] * k2[i];
          s2h += a2[i] * h2[i];
        }
      }
      const double id = 1.0 / d;
      const double f0 = (-(2 * d - 1) * s1f - (d - 1) * s2f) * ir2 * id;
      const int t = below + gl;
      F0[t] = f0;
      double fk = 0;
      if (!RHS) {
        fk = (-kappa * (s1h + s2h) - (2 * d - 1) * s1k - (d - 1) * s2k) * ir2 * id;
        FK[t] = fk;
        HK[t] = -kappa * (s1k + s2k) * id;
      }
      if (RHS) {
        unsafeAtomicAdd(lam + t, (d & 1) ? -qs * f0 : qs * f0);
      } else {
        const double c = f0 * S0[t] + fk * SK[t];
        v += (d & 1) ? -c : c;
      }
    }
    wave_sync();
  }
  return v;
}

// cube centre corner + (idx + 1/2) h of cluster c and d = x - centre, in the
// oracle's rounding
__device__ inline void tc_offset(const TcLevels& lv, int l, int c, double3 corner, double4 xq, double& dx,
                                 double& dy, double& dz) {
  const int32_t* ix = lv.idx[l] + 3 * (int64_t)c;
  const double h = lv.h[l];
  dx = __dsub_rn(xq.x, __dadd_rn(corner.x, __dmul_rn((double)ix[0] + 0.5, h)));
  dy = __dsub_rn(xq.y, __dadd_rn(corner.y, __dmul_rn((double)ix[1] + 0.5, h)));
  dz = __dsub_rn(xq.z, __dadd_rn(corner.z, __dmul_rn((double)ix[2] + 0.5, h)));
}

// the first frontier: every (charge, cluster of level l0) pair
__global__ void k_tc_init(int64_t M, int n0, int32_t* pn, int32_t* pc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  pn[i] = (int32_t)(i / n0);
  pc[i] = (int32_t)(i % n0);
}

// one thread per (charge, cluster) pair of level l: acc[i] = 1 when the
// criterion holds, nch[i] = children to visit; a leaf that fails is summed
// directly here (energy: into V[n] times 4 pi / q; right-hand side: into b)
template <bool RHS>
__global__ void __launch_bounds__(256) k_tc_classify(TcLevels lv, int l, int L, double th2, double kappa, double eps,
                                                     double3 corner, const double4* __restrict__ chg, int64_t M,
                                                     const int32_t* __restrict__ pn, const int32_t* __restrict__ pc,
                                                     const double* __restrict__ pv, const double* __restrict__ pnrm,
                                                     const double* __restrict__ pa, const int32_t* __restrict__ perm,
                                                     const int32_t* __restrict__ leaf_start,
                                                     const int32_t* __restrict__ leaf_cnt, int64_t N,
                                                     const double* __restrict__ x, double* V, double* b, int32_t* acc,
                                                     int32_t* nch, const int32_t* __restrict__ ptri, int64_t nv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int n = pn[i], c = pc[i];
  const double4 xq = chg[n];
  double dx, dy, dz;
  tc_offset(lv, l, c, corner, xq, dx, dy, dz);
  const double R2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
  const bool a = lv.rho2[l] <= __dmul_rn(th2, R2);
  acc[i] = a;
  nch[i] = (!a && l < L) ? lv.ce[l][c] - lv.cs[l][c] : 0;
  if (a || l < L) return;
  // direct sum over the leaf's panels (tree order).  Hat functions (ptri set):
  // the values at the rule's points interpolate the nodal values of the
  // panel's vertices (x: channel stride nv), and the source terms go to the
  // panel's corners e = 3 i + a with lambda_a (b: corner rows, stride 3N)
  const int i0 = leaf_start[c], i1 = i0 + leaf_cnt[c];
  double v = 0;
  for (int ii = i0; ii < i1; ++ii) {
    double qp[9];
    quad_points(pv, ii, qp);
    const double nx = pnrm[3 * (int64_t)ii], ny = pnrm[3 * (int64_t)ii + 1], nz = pnrm[3 * (int64_t)ii + 2];
    const int p = perm[ii];
    const double w = pa[ii] / 3.0;
    if (RHS) {
      // b1 += qs sum_q w / r, b2 += -qs sum_q w (y_q - x_n) . n / r^3
      double a1 = 0, a2 = 0, g1[3], g2[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double rx = qp[3 * q] - xq.x, ry = qp[3 * q + 1] - xq.y, rz = qp[3 * q + 2] - xq.z;
        const double ir = inv_sqrt(rx * rx + ry * ry + rz * rz);
        g1[q] = ir;
        g2[q] = -(rx * nx + ry * ny + rz * nz) * (ir * ir * ir);
        a1 += g1[q];
        a2 += g2[q];
      }
      if (ptri) {
        const int64_t N3 = 3 * N;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          double c1 = 0, c2 = 0;
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const double l = q == k ? 2.0 / 3.0 : 1.0 / 6.0;
            c1 += l * g1[q];
            c2 += l * g2[q];
          }
          unsafeAtomicAdd(b + 3 * (int64_t)ii + k, xq.w * w * c1);
          unsafeAtomicAdd(b + N3 + 3 * (int64_t)ii + k, xq.w * w * c2);
        }
      } else {
        unsafeAtomicAdd(b + p, xq.w * w * a1);
        unsafeAtomicAdd(b + N + p, xq.w * w * a2);
      }
    } else {
      double ph[3], dph[3];
      if (ptri) {
        double hu[3], hv[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int64_t vx = ptri[3 * (int64_t)ii + k];
          hu[k] = x[vx];
          hv[k] = x[nv + vx];
        }
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          ph[q] = dph[q] = 0.0;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const double l = q == k ? 2.0 / 3.0 : 1.0 / 6.0;
            ph[q] += l * hu[k];
            dph[q] += l * hv[k];
          }
        }
      } else {
        ph[0] = ph[1] = ph[2] = x[p];
        dph[0] = dph[1] = dph[2] = x[N + p];
      }
      double s = 0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double rx = xq.x - qp[3 * q], ry = xq.y - qp[3 * q + 1], rz = xq.z - qp[3 * q + 2];
        const double rr2 = rx * rx + ry * ry + rz * rz;
        const double ir = inv_sqrt(rr2);
        const double u = kappa * (rr2 * ir);
        double E, em1;
        exp_expm1(-u, E, em1);
        const double rny = rx * nx + ry * ny + rz * nz;
        s += ir * (-em1 * dph[q] + (eps * E * (1.0 + u) - 1.0) * rny * (ir * ir) * ph[q]);
      }
      v += w * s;
    }
  }
  if (!RHS) unsafeAtomicAdd(V + n, v);
}

// pair list of the accepted pairs (in pair order)
__global__ void k_tc_compact(int64_t M, const int32_t* __restrict__ acc, const int64_t* __restrict__ off,
                             int64_t* list) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M && acc[i]) list[off[i]] = i;
}

// particle-cluster terms of the accepted pairs: 64 / g groups of g lanes per
// wavefront, one pair each
template <bool RHS>
__global__ void __launch_bounds__(64) k_tc_far(TcLevels lv, int l, double kappa, double3 corner,
                                               const double4* __restrict__ chg, const int64_t* __restrict__ list,
                                               int64_t nacc, const int32_t* __restrict__ pn,
                                               const int32_t* __restrict__ pc, double* V) {
  __shared__ double F0[TC_TG], FK[TC_TG], HK[TC_TG], S0[TC_TG], SK[TC_TG];
  const int lane = threadIdx.x;
  const int p = lv.pt[l], T = nterms(p);
  const int g = p <= 4 ? 16 : p <= 6 ? 32 : 64, ng = 64 / g, gi = lane / g, gl = lane % g;
  const int64_t k = (int64_t)blockIdx.x * ng + gi;
  const bool has = k < nacc;
  int n = 0, c = 0;
  double dx = 0, dy = 0, dz = 0;
  double4 xq = make_double4(0, 0, 0, 0);
  if (has) {
    const int64_t i = list[k];
    n = pn[i];
    c = pc[i];
    xq = chg[n];
    tc_offset(lv, l, c, corner, xq, dx, dy, dz);
  }
  const int64_t off = (int64_t)c * lv.T[l];
  double v = tc_far<RHS>(has, dx, dy, dz, kappa, p, T, g, RHS ? nullptr : lv.m0[l] + off,
                         RHS ? nullptr : lv.mk[l] + off, RHS ? lv.lam[l] + off : nullptr, xq.w, F0 + gi * T,
                         FK + gi * T, HK + gi * T, S0 + gi * T, SK + gi * T, gl);
  if (RHS) return;
  for (int o = g >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (has && gl == 0) unsafeAtomicAdd(V + n, v);
}

// The same particle-to-local terms (right-hand side) for a level with few
// clusters: many charges share each cluster, so instead of one global atomic
// per term each block accumulates into an LDS copy of the level's evaluated
// locals ([n][T(p)], then one Coulomb coefficient row per group) and adds the
// copy to global memory once.  Wavefronts stride over the accepted pairs.
__global__ void __launch_bounds__(1024) k_tc_far_rhs_lds(TcLevels lv, int l, double3 corner,
                                                        const double4* __restrict__ chg,
                                                        const int64_t* __restrict__ list, int64_t nacc,
                                                        const int32_t* __restrict__ pn,
                                                        const int32_t* __restrict__ pc) {
  extern __shared__ __align__(16) double sl[];
  const int p = lv.pt[l], Tp = nterms(p), ncl = lv.n[l];
  const int g = p <= 4 ? 16 : p <= 6 ? 32 : 64, ng = 64 / g;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, gi = lane / g, gl = lane % g;
  const int nwb = blockDim.x >> 6;
  double* F0 = sl + (size_t)ncl * Tp + (size_t)wave * TC_TG;
  for (int e = threadIdx.x; e < ncl * Tp; e += blockDim.x) sl[e] = 0.0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * nwb * ng;
  for (int64_t wb = ((int64_t)blockIdx.x * nwb + wave) * ng; wb < nacc; wb += stride) {
    const int64_t k = wb + gi;
    const bool has = k < nacc;
    int c = 0;
    double dx = 0, dy = 0, dz = 0;
    double4 xq = make_double4(0, 0, 0, 0);
    if (has) {
      const int64_t i = list[k];
      c = pc[i];
      xq = chg[pn[i]];
      tc_offset(lv, l, c, corner, xq, dx, dy, dz);
    }
    tc_far<true>(has, dx, dy, dz, 0.0, p, Tp, g, nullptr, nullptr, sl + (size_t)c * Tp, xq.w, F0 + gi * Tp,
                 nullptr, nullptr, nullptr, nullptr, gl);
  }
  __syncthreads();
  double* lam = lv.lam[l];
  const int TL = lv.T[l];
  for (int e = threadIdx.x; e < ncl * Tp; e += blockDim.x) {
    const double v = sl[e];
    if (v != 0.0) {
      const int c = e / Tp;
      unsafeAtomicAdd(lam + (int64_t)c * TL + (e - c * Tp), v);
    }
  }
}

// children of the pairs that failed, appended in pair order
__global__ void k_tc_expand(TcLevels lv, int l, int64_t M, const int32_t* __restrict__ pn,
                            const int32_t* __restrict__ pc, const int32_t* __restrict__ nch,
                            const int64_t* __restrict__ off, int32_t* npn, int32_t* npc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M || !nch[i]) return;
  const int n = pn[i], c0 = lv.cs[l][pc[i]];
  const int64_t o = off[i];
  for (int j = 0; j < nch[i]; ++j) {
    npn[o + j] = n;
    npc[o + j] = c0 + j;
  }
}

// q_n V_n / 4 pi
__global__ void k_tc_qv(const double4* __restrict__ chg, const double* __restrict__ V, int64_t nc, double* qv) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < nc) qv[n] = chg[n].w * V[n] * (1.0 / FOUR_PI);
}

// right-hand side, step 6 of the far field: b += locals tested with the
// panel's single- and double-layer moments (tree order -> caller order)
__global__ void __launch_bounds__(256) k_l2p_rhs(const double* __restrict__ ms, const double* __restrict__ md,
                                                 const int32_t* __restrict__ leaf_of,
                                                 const int32_t* __restrict__ perm, int64_t N, int T,
                                                 const double* __restrict__ lam, double* b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t c = leaf_of[i];
  double s1 = 0, s2 = 0;
  for (int t = 0; t < T; ++t) {
    const double l = lam[c * T + t];
    s1 += l * ms[i * T + t];
    s2 += l * md[i * T + t];
  }
  const int p = perm[i];
  b[p] += s1;
  b[N + p] += s2;
}

static int tc_levels(fagbi_handle* h, int l0, int p_max, TcLevels& lv) {
  lv = TcLevels{};
  for (int l = l0; l <= h->L; ++l) {
    Level& D = h->lev[l];
    if (D.order > 8) return set_error(FAGBI_E_ARG, "treecode: expansion order above 8");
    lv.idx[l] = D.d_idx.as<int32_t>();
    lv.cs[l] = D.d_child_start.as<int32_t>();
    lv.ce[l] = D.d_child_end.as<int32_t>();
    lv.m0[l] = D.d_M64[0].as<double>();
    lv.mk[l] = D.d_M64[1].as<double>();
    lv.lam[l] = D.d_L64[0].as<double>();
    lv.h[l] = D.h;
    lv.rho2[l] = D.rho * D.rho;
    lv.n[l] = D.n;
    lv.order[l] = D.order;
    lv.T[l] = D.T;
    lv.pt[l] = std::min(D.order, p_max);
  }
  return 0;
}

// the level-by-level visit shared by the energy (RHS = false: V[n] += the
// charge's potential times 4 pi) and the right-hand side (RHS = true: b and
// the Coulomb locals)
// a work list of at least `bytes` (reallocated only while it holds nothing live)
static int tc_grow(fagbi::Tmp& t, size_t bytes) {
  if (t.bytes >= bytes) return 0;
  FAGBI_HIP(hipDeviceSynchronize());   // no kernel still reads the old list
  t.release();
  return t.alloc(bytes + bytes / 2);
}

template <bool RHS>
static int tc_visit(fagbi_handle* h, const TcLevels& lv, int l0, const double* chg, int64_t nc, double theta,
                    const double* x, double* V, double* b, hipStream_t s) {
  const int L = h->L;
  const double3 corner = make_double3(h->corner[0], h->corner[1], h->corner[2]);
  const double eps = h->prm.eps_out / h->prm.eps_in, kappa = RHS ? 0.0 : h->prm.kappa;
  const double4* q4 = reinterpret_cast<const double4*>(chg);
  Tmp* W = h->tc_ws;   // pn[2], pc[2], acc, nch, aoff, koff, part, list
  int64_t M = nc * (int64_t)lv.n[l0];
  if (M > TC_MAX_PAIRS) return set_error(FAGBI_E_ARG, "treecode: too many (charge, cluster) pairs on one level");
  int cur = 0;
  FAGBI_TRY(tc_grow(W[0], (size_t)M * 4));
  FAGBI_TRY(tc_grow(W[2], (size_t)M * 4));
  k_tc_init<<<(unsigned)((M + 255) / 256), 256, 0, s>>>(M, lv.n[l0], W[0].as<int32_t>(), W[2].as<int32_t>());
  for (int l = l0; l <= L && M > 0; ++l) {
    FAGBI_TRY(tc_grow(W[4], (size_t)M * 4));
    FAGBI_TRY(tc_grow(W[5], (size_t)M * 4));
    FAGBI_TRY(tc_grow(W[6], (size_t)(M + 1) * 8));
    FAGBI_TRY(tc_grow(W[7], (size_t)(M + 1) * 8));
    FAGBI_TRY(tc_grow(W[8], (size_t)scan_part_size(M) * 8));
    int32_t *pn = W[cur].as<int32_t>(), *pc = W[2 + cur].as<int32_t>();
    int32_t *acc = W[4].as<int32_t>(), *nch = W[5].as<int32_t>();
    int64_t *aoff = W[6].as<int64_t>(), *koff = W[7].as<int64_t>(), *part = W[8].as<int64_t>();
    const unsigned gm = (unsigned)((M + 255) / 256);
    k_tc_classify<RHS><<<gm, 256, 0, s>>>(lv, l, L, theta * theta, kappa, eps, corner, q4, M, pn, pc,
                                          h->d_pv.as<double>(), h->d_pn.as<double>(), h->d_pa.as<double>(),
                                          h->d_perm.as<int32_t>(), h->d_leaf_start.as<int32_t>(),
                                          h->d_leaf_cnt.as<int32_t>(), h->N, x, V, b, acc, nch,
                                          h->hat() ? h->d_ptri.as<int32_t>() : nullptr, h->nv);
    FAGBI_TRY((device_scan<int32_t, int64_t>(acc, M, aoff, part, s)));
    FAGBI_TRY((device_scan<int32_t, int64_t>(nch, M, koff, part, s)));
    int64_t tot[2];
    FAGBI_HIP(hipMemcpyAsync(&tot[0], aoff + M, 8, hipMemcpyDeviceToHost, s));
    FAGBI_HIP(hipMemcpyAsync(&tot[1], koff + M, 8, hipMemcpyDeviceToHost, s));
    FAGBI_HIP(hipStreamSynchronize(s));
    const int64_t nacc = tot[0], Mn = tot[1];
    if (nacc > 0) {
      FAGBI_TRY(tc_grow(W[9], (size_t)nacc * 8));
      int64_t* list = W[9].as<int64_t>();
      k_tc_compact<<<gm, 256, 0, s>>>(M, acc, aoff, list);
      const int p = lv.pt[l], ng = p <= 4 ? 4 : p <= 6 ? 2 : 1;
      const size_t lds = ((size_t)lv.n[l] * nterms(p) + (size_t)16 * TC_TG) * sizeof(double);
      if (RHS && (size_t)lv.n[l] * nterms(p) * sizeof(double) <= (size_t)120 * 1024) {
        FAGBI_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tc_far_rhs_lds),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        const int64_t per_block = (int64_t)16 * ng;
        const unsigned grid = (unsigned)std::min<int64_t>(256, (nacc + per_block - 1) / per_block);
        k_tc_far_rhs_lds<<<grid, 1024, lds, s>>>(lv, l, corner, q4, list, nacc, pn, pc);
      } else {
        k_tc_far<RHS><<<(unsigned)((nacc + ng - 1) / ng), 64, 0, s>>>(lv, l, kappa, corner, q4, list, nacc, pn,
                                                                      pc, V);
      }
    }
    if (Mn > TC_MAX_PAIRS)
      return set_error(FAGBI_E_ARG, "treecode: too many (charge, cluster) pairs on one level (theta too small)");
    if (Mn > 0) {
      // the other pair buffers hold nothing live now
      FAGBI_TRY(tc_grow(W[1 - cur], (size_t)Mn * 4));
      FAGBI_TRY(tc_grow(W[3 - cur], (size_t)Mn * 4));
      k_tc_expand<<<gm, 256, 0, s>>>(lv, l, M, pn, pc, nch, koff, W[1 - cur].as<int32_t>(),
                                     W[3 - cur].as<int32_t>());
    }
    FAGBI_HIP(hipGetLastError());
    cur = 1 - cur;
    M = Mn;
  }
  return 0;
}

int treecode_potentials(fagbi_handle* h, const double* x, const double* chg, int64_t nc, double theta, int p_max,
                        double* qv, hipStream_t s) {
  const int L = h->L, l0 = std::min(h->lmin, h->L);
  // moments of x: leaf moments (from panel or corner moments) and the upward pass, FP64
  const ElemView v = h->hat() ? hat_view(h) : box_view(h);
  k_to_tree<<<(unsigned)((v.n + 255) / 256), 256, 0, s>>>(x, v.in_idx, v.n, v.in_stride, v.xt);
  FAGBI_TRY(launch_p2m<double>(h, v, h->d_ms64.as<double>(), h->d_md64.as<double>(), false, s));
  for (int l = L - 1; l >= l0; --l) FAGBI_TRY(launch_m2m<double>(h, l, false, s));
  TcLevels lv;
  FAGBI_TRY(tc_levels(h, l0, p_max, lv));
  Tmp V;
  FAGBI_TRY(V.alloc((size_t)nc * 8));
  FAGBI_HIP(hipMemsetAsync(V.p, 0, (size_t)nc * 8, s));
  FAGBI_TRY(tc_visit<false>(h, lv, l0, chg, nc, theta, x, V.as<double>(), nullptr, s));
  k_tc_qv<<<(unsigned)((nc + 255) / 256), 256, 0, s>>>(reinterpret_cast<const double4*>(chg), V.as<double>(), nc,
                                                        qv);
  FAGBI_HIP(hipGetLastError());
  FAGBI_HIP(hipStreamSynchronize(s));
  return 0;
}

// b (caller order, f64[2n]) by the reverse treecode; chg holds x, y, z and
// q / (4 pi eps_in) per charge
int treecode_rhs(fagbi_handle* h, const double* chg, int64_t nc, double theta, int p_max, double* b, hipStream_t s) {
  const int L = h->L, l0 = std::min(h->lmin, h->L);
  TcLevels lv;
  FAGBI_TRY(tc_levels(h, l0, p_max, lv));
  // rows: the panels (caller order, b itself), or the panel corners (the
  // matvec's corner rows, summed into the vertices of b at the end)
  const bool hat = h->hat();
  const int64_t nrow = hat ? 3 * h->N : h->N;
  double* rows = hat ? h->d_ye.as<double>() : b;
  FAGBI_HIP(hipMemsetAsync(rows, 0, (size_t)2 * nrow * sizeof(double), s));
  for (int l = l0; l <= L; ++l) {
    Level& D = h->lev[l];
    for (int ch = 0; ch < 2; ++ch)
      FAGBI_HIP(hipMemsetAsync(D.d_L64[ch].p, 0, (size_t)D.n * D.T * sizeof(double), s));
  }
  FAGBI_TRY(tc_visit<true>(h, lv, l0, chg, nc, theta, nullptr, nullptr, rows, s));
  for (int l = l0; l < L; ++l) FAGBI_TRY(launch_l2l<double>(h, l, false, s));
  Level& LF = h->lev[L];
  const int32_t* lo = hat ? h->d_s1_leaf_of.as<int32_t>() : h->d_leaf_of.as<int32_t>();
  const int32_t* pm = hat ? h->d_s1_iota.as<int32_t>() : h->d_perm.as<int32_t>();
  k_l2p_rhs<<<(unsigned)((nrow + 255) / 256), 256, 0, s>>>(h->d_ms64.as<double>(), h->d_md64.as<double>(), lo, pm,
                                                          nrow, LF.T, LF.d_L64[0].as<double>(), rows);
  FAGBI_HIP(hipGetLastError());
  if (hat) FAGBI_TRY(hat_gather(h, rows, nullptr, b, s));
  FAGBI_HIP(hipStreamSynchronize(s));
  return 0;
}

}  // namespace fagbi
