// Cluster tree of panel centroids built on the GPU (paper Sec. 2.4: level-0
// cube, cube refinement, clusters as the panels whose centroids lie in a
// cube, separation ratio, neighbour lists N(c) and interaction lists I(c)).
//
// Choices the paper leaves open:
//  * level-0 cube centred on the vertex bounding box, side = largest extent
//    times (1 + 1e-12);
//  * uniform depth: L = smallest level whose fullest cube holds <= leaf_size
//    centroids; empty cubes are dropped;
//  * cube index of a centroid on level l: floor((c - corner)/h_l) clamped to
//    [0, 2^l - 1] (computed once on level 20 and shifted, which is exact);
//  * panels ordered by (leaf cube Morton key, input index);
//  * cluster centre = cube centre, one radius per level (the farthest
//    3-point-rule quadrature point of a member panel from its cube centre:
//    the far field only ever evaluates that rule), so the separation ratio
//    2 rho_l / |x_c - x_c'| depends on the index offset alone and every level
//    has a fixed stencil of interaction offsets;
//  * c' in N(c) iff c' is a child of a neighbour of c's parent and the ratio
//    exceeds eta0; the remaining such children form I(c); both lists keep
//    the order (parent's neighbour list, then child order).
//
// All decisions (cube indices, radii, separation tests) are the IEEE results
// of the written expressions: this file is compiled without FP contraction.
// Mesh checks: every undirected edge is shared by exactly two triangles, once
// in each direction; no degenerate triangle; positive enclosed volume.
#pragma clang fp contract(off)

#include <algorithm>
#include <climits>
#include <cmath>
#include <memory>

#include "internal.h"
#include "scan.h"

namespace fagbi {
namespace {

constexpr int DEEP = 20;                 // key resolution: 2^20 cubes per axis
constexpr unsigned long long EMPTY = ~0ull;
using scan_detail::TB;
using scan_detail::IPT;
using scan_detail::TILE;
using scan_detail::block_exclusive_scan;
using scan_detail::k_scan_reduce;
using scan_detail::k_scan_part;
using scan_detail::k_scan_down;

__host__ __device__ inline uint64_t spread3(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | x << 32) & 0x1f00000000ffffull;
  x = (x | x << 16) & 0x1f0000ff0000ffull;
  x = (x | x << 8) & 0x100f00f00f00f00full;
  x = (x | x << 4) & 0x10c30c30c30c30c3ull;
  x = (x | x << 2) & 0x1249249249249249ull;
  return x;
}

__host__ __device__ inline uint32_t compact3(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
  x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
  x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
  x = (x ^ (x >> 32)) & 0x1fffffull;
  return (uint32_t)x;
}

__device__ inline int64_t cube_coord(double c, double corner, double h, int64_t nmax) {
  double k = floor((c - corner) / h);
  if (k < 0) k = 0;
  if (k > (double)(nmax - 1)) k = (double)(nmax - 1);
  return (int64_t)k;
}

__device__ inline uint64_t edge_hash(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// ---------------------------------------------------------------------------
// stable LSD radix sort of (64-bit key, 32-bit value), 4 bits per pass
// ---------------------------------------------------------------------------
constexpr int RBITS = 4, RBINS = 1 << RBITS;

__global__ void __launch_bounds__(TB) k_radix_hist(const uint64_t* __restrict__ key, int64_t n, int shift,
                                                   int nb, int* hist) {
  __shared__ int cnt[RBINS];
  if (threadIdx.x < RBINS) cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * TILE;
  for (int j = threadIdx.x; j < TILE; j += TB)
    if (base + j < n) atomicAdd(&cnt[(key[base + j] >> shift) & (RBINS - 1)], 1);
  __syncthreads();
  if (threadIdx.x < RBINS) hist[threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(TB) k_radix_scatter(const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin,
                                                      uint64_t* kout, int32_t* vout, int64_t n, int shift, int nb,
                                                      const int* __restrict__ offs) {
  __shared__ int cnt[RBINS * TB];   // [digit][thread]
  __shared__ int lds[TB / 64];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * TILE + t * IPT;
  uint64_t k[IPT];
  int32_t v[IPT];
  int d[IPT];
#pragma unroll
  for (int b = 0; b < RBINS; ++b) cnt[b * TB + t] = 0;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    const bool ok = base + j < n;
    k[j] = ok ? kin[base + j] : 0;
    v[j] = ok ? vin[base + j] : 0;
    d[j] = ok ? (int)((k[j] >> shift) & (RBINS - 1)) : -1;
    if (ok) cnt[d[j] * TB + t] += 1;
  }
  __syncthreads();
  // exclusive scan over the flattened [digit][thread] counters: digit-major
  // order with threads in position order keeps the sort stable
  constexpr int PER = RBINS * TB / TB;
  int loc[PER];
  int s = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    loc[i] = cnt[t * PER + i];
    s += loc[i];
  }
  int tot;
  int run = block_exclusive_scan<int>(s, lds, tot);
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    cnt[t * PER + i] = run;
    run += loc[i];
  }
  __syncthreads();
  // cnt[b][t] now holds the block-local rank of thread t's first digit-b
  // item; subtract the block-local start of digit b to get the rank within
  // the digit, then add the global start of (digit b, this block)
  __shared__ int dstart[RBINS];
  if (t < RBINS) dstart[t] = cnt[t * TB] - offs[t * nb + blockIdx.x];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    if (d[j] < 0) continue;
    const int b = d[j];
    const int r = cnt[b * TB + t] - dstart[b];
    cnt[b * TB + t] += 1;
    kout[r] = k[j];
    vout[r] = v[j];
  }
}

// ---------------------------------------------------------------------------
// mesh checks and geometry
// ---------------------------------------------------------------------------
struct Check {
  int open_tri, orient_tri, degen_tri, pad;
  double vol6, lo[3], hi[3];
};

__global__ void k_edge_insert(const int32_t* __restrict__ tri, int64_t nt, unsigned long long* tab, int* cnt,
                              uint64_t mask) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * nt) return;
  const int64_t t = e / 3;
  const int k = (int)(e - 3 * t);
  const uint64_t a = (uint32_t)tri[3 * t + k], b = (uint32_t)tri[3 * t + (k + 1) % 3];
  const unsigned long long key = (a << 32) | b;
  uint64_t s = edge_hash(key) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long prev = atomicCAS(&tab[s], EMPTY, key);
    if (prev == EMPTY || prev == key) {
      atomicAdd(&cnt[s], 1);
      return;
    }
    s = (s + 1) & mask;
  }
}

__device__ inline int edge_count(const unsigned long long* tab, const int* cnt, uint64_t mask, uint64_t a,
                                 uint64_t b) {
  const unsigned long long key = (a << 32) | b;
  uint64_t s = edge_hash(key) & mask;
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long v = tab[s];
    if (v == key) return cnt[s];
    if (v == EMPTY) return 0;
    s = (s + 1) & mask;
  }
  return 0;
}

__global__ void k_edge_check(const int32_t* __restrict__ tri, int64_t nt, const unsigned long long* __restrict__ tab,
                             const int* __restrict__ cnt, uint64_t mask, Check* chk) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 3 * nt) return;
  const int64_t t = e / 3;
  const int k = (int)(e - 3 * t);
  const uint64_t a = (uint32_t)tri[3 * t + k], b = (uint32_t)tri[3 * t + (k + 1) % 3];
  const int ab = edge_count(tab, cnt, mask, a, b), ba = edge_count(tab, cnt, mask, b, a);
  if (ab + ba != 2)
    atomicMin(&chk->open_tri, (int)t);
  else if (ab != 1)
    atomicMin(&chk->orient_tri, (int)t);
}

// per-panel corners, centroid, unit normal, area; per-block partial volume
// and bounding box of the referenced vertices
__global__ void __launch_bounds__(TB) k_geometry(const double* __restrict__ v, const int32_t* __restrict__ tri,
                                                 int64_t nt, double* cor, double* cen, double* nrm, double* area,
                                                 double* part, Check* chk) {
  __shared__ double red[7][TB];
  const int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x;
  double vol = 0, lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (t < nt) {
    const double* u = v + 3 * (int64_t)tri[3 * t];
    const double* p = v + 3 * (int64_t)tri[3 * t + 1];
    const double* w = v + 3 * (int64_t)tri[3 * t + 2];
    double e1[3], e2[3], cr[3];
    for (int d = 0; d < 3; ++d) {
      e1[d] = p[d] - u[d];
      e2[d] = w[d] - u[d];
      cen[3 * t + d] = (u[d] + p[d] + w[d]) / 3.0;
      cor[9 * t + d] = u[d];
      cor[9 * t + 3 + d] = p[d];
      cor[9 * t + 6 + d] = w[d];
      lo[d] = fmin(u[d], fmin(p[d], w[d]));
      hi[d] = fmax(u[d], fmax(p[d], w[d]));
    }
    cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
    cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
    cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
    const double two_a = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    if (!(two_a > 0) || !isfinite(two_a)) atomicMin(&chk->degen_tri, (int)t);
    area[t] = 0.5 * two_a;
    for (int d = 0; d < 3; ++d) nrm[3 * t + d] = cr[d] / two_a;
    vol = u[0] * (p[1] * w[2] - p[2] * w[1]) - u[1] * (p[0] * w[2] - p[2] * w[0]) +
          u[2] * (p[0] * w[1] - p[1] * w[0]);
  }
  red[0][threadIdx.x] = vol;
  for (int d = 0; d < 3; ++d) {
    red[1 + d][threadIdx.x] = lo[d];
    red[4 + d][threadIdx.x] = hi[d];
  }
  __syncthreads();
  for (int s = TB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      for (int d = 0; d < 3; ++d) {
        red[1 + d][threadIdx.x] = fmin(red[1 + d][threadIdx.x], red[1 + d][threadIdx.x + s]);
        red[4 + d][threadIdx.x] = fmax(red[4 + d][threadIdx.x], red[4 + d][threadIdx.x + s]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 7) part[7 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(TB) k_geometry_final(const double* __restrict__ part, int nb, Check* chk) {
  __shared__ double red[7][TB];
  double a[7] = {0, INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nb; b += TB) {
    a[0] += part[7 * b];
    for (int d = 0; d < 3; ++d) {
      a[1 + d] = fmin(a[1 + d], part[7 * b + 1 + d]);
      a[4 + d] = fmax(a[4 + d], part[7 * b + 4 + d]);
    }
  }
  for (int k = 0; k < 7; ++k) red[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int s = TB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      for (int d = 0; d < 3; ++d) {
        red[1 + d][threadIdx.x] = fmin(red[1 + d][threadIdx.x], red[1 + d][threadIdx.x + s]);
        red[4 + d][threadIdx.x] = fmax(red[4 + d][threadIdx.x], red[4 + d][threadIdx.x + s]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    chk->vol6 = red[0][0];
    for (int d = 0; d < 3; ++d) {
      chk->lo[d] = red[1 + d][0];
      chk->hi[d] = red[4 + d][0];
    }
  }
}

__global__ void k_keys(const double* __restrict__ cen, int64_t n, double c0, double c1, double c2, double h,
                       uint64_t* key, int32_t* val) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t nmax = (int64_t)1 << DEEP;
  const int64_t x = cube_coord(cen[3 * t], c0, h, nmax);
  const int64_t y = cube_coord(cen[3 * t + 1], c1, h, nmax);
  const int64_t z = cube_coord(cen[3 * t + 2], c2, h, nmax);
  key[t] = (spread3((uint64_t)x) << 2) | (spread3((uint64_t)y) << 1) | spread3((uint64_t)z);
  val[t] = (int32_t)t;
}

// deepest level on which key[k] and key[k + leaf] share a cube, plus one: the
// keys are sorted, so a cube holding more than `leaf` centroids contains such
// a window
__global__ void k_leaf_level(const uint64_t* __restrict__ key, int64_t n, int leaf, int* L) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k + leaf >= n) return;
  const uint64_t x = key[k] ^ key[k + leaf];
  const int shared = x == 0 ? DEEP : DEEP - 1 - (63 - __clzll((long long)x)) / 3;
  atomicMax(L, shared + 1);
}

// final order: by leaf key, ties by input index (a leaf holds <= leaf items)
__global__ void k_leaf_order(const uint64_t* __restrict__ key, const int32_t* __restrict__ val, int64_t n, int sh,
                             int leaf, int32_t* perm, uint64_t* keyL) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint64_t kl = key[k] >> sh;
  int64_t s = k, e = k + 1;
  while (s > 0 && k - s < leaf && (key[s - 1] >> sh) == kl) --s;
  while (e < n && e - k <= leaf && (key[e] >> sh) == kl) ++e;
  const int32_t me = val[k];
  int r = 0;
  for (int64_t j = s; j < e; ++j) r += val[j] < me;
  perm[s + r] = me;
  keyL[k] = kl;
}

// tree-order panel arrays; pc = (centroid, sqrt(area)) for the near-field
// classification
__global__ void k_permute(const int32_t* __restrict__ perm, int64_t n, const double* __restrict__ cor,
                          const double* __restrict__ nrm, const double* __restrict__ area,
                          const int32_t* __restrict__ tri, double* pv, double* pn, double* pa, int32_t* ptri,
                          double4* pc) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t t = perm[k];
  for (int d = 0; d < 9; ++d) pv[9 * k + d] = cor[9 * t + d];
  for (int d = 0; d < 3; ++d) {
    pn[3 * k + d] = nrm[3 * t + d];
    ptri[3 * k + d] = tri[3 * t + d];
  }
  pa[k] = area[t];
  const double* c = cor + 9 * t;
  pc[k] = make_double4((c[0] + c[3] + c[6]) / 3.0, (c[1] + c[4] + c[7]) / 3.0, (c[2] + c[5] + c[8]) / 3.0,
                       sqrt(area[t]));
}

// ---------------------------------------------------------------------------
// levels
// ---------------------------------------------------------------------------
__global__ void k_level_flags(const uint64_t* __restrict__ keyL, int64_t n, int sh, int32_t* flag) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  flag[k] = (k == 0 || (keyL[k] >> sh) != (keyL[k - 1] >> sh)) ? 1 : 0;
}

// owner (cluster of each panel), cluster start/end and cube index
__global__ void k_level_fill(const uint64_t* __restrict__ keyL, const int32_t* __restrict__ flag,
                             const int32_t* __restrict__ excl, int64_t n, int sh, int32_t* owner, int32_t* idx,
                             int32_t* start, int32_t* end) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t c = excl[k] + flag[k] - 1;
  owner[k] = c;
  if (flag[k]) {
    const uint64_t m = keyL[k] >> sh;
    idx[3 * c] = (int32_t)compact3(m >> 2);
    idx[3 * c + 1] = (int32_t)compact3(m >> 1);
    idx[3 * c + 2] = (int32_t)compact3(m);
    start[c] = (int32_t)k;
    if (c > 0) end[c - 1] = (int32_t)k;
  }
  if (k == n - 1) end[c] = (int32_t)n;
}

// farthest quadrature point (2/3 of one corner, 1/6 of each other) of a
// member panel from its cube centre; distances are non-negative, so their
// bit patterns order like the values
__global__ void __launch_bounds__(TB) k_level_rho(const double* __restrict__ pv, const int32_t* __restrict__ owner,
                                                  const int32_t* __restrict__ idx, int64_t n, double c0, double c1,
                                                  double c2, double h, unsigned long long* rho_bits) {
  __shared__ double red[TB];
  const int64_t k = (int64_t)blockIdx.x * TB + threadIdx.x;
  double rho = 0;
  if (k < n) {
    const int32_t c = owner[k];
    const double* cv = pv + 9 * k;
    const double corner[3] = {c0, c1, c2};
    for (int v = 0; v < 3; ++v) {
      double s[3];
      for (int d = 0; d < 3; ++d) {
        const double ctr = corner[d] + ((double)idx[3 * c + d] + 0.5) * h;
        const double qp = (2.0 / 3.0) * cv[3 * v + d] +
                          (1.0 / 6.0) * (cv[3 * ((v + 1) % 3) + d] + cv[3 * ((v + 2) % 3) + d]);
        s[d] = qp - ctr;
      }
      const double dist = sqrt((s[0] * s[0] + s[1] * s[1]) + s[2] * s[2]);
      rho = fmax(rho, dist);
    }
  }
  red[threadIdx.x] = rho;
  __syncthreads();
  for (int s = TB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(rho_bits, (unsigned long long)__double_as_longlong(red[0]));
}

// farthest vertex of a member panel from its cube centre, per cluster (the
// ball of radius rho_c around the centre holds the cluster's panels whole);
// one wavefront per cluster, lanes over its panels (contiguous in tree order);
// the square root is monotone and correctly rounded, so the root of the
// largest squared distance is the largest distance
__global__ void __launch_bounds__(256) k_cluster_rho(const double* __restrict__ pv,
                                                     const int32_t* __restrict__ start,
                                                     const int32_t* __restrict__ end,
                                                     const int32_t* __restrict__ idx, int ncl, double c0,
                                                     double c1, double c2, double h, double* rho_c) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= ncl) return;
  const double ctr[3] = {c0 + ((double)idx[3 * c] + 0.5) * h, c1 + ((double)idx[3 * c + 1] + 0.5) * h,
                         c2 + ((double)idx[3 * c + 2] + 0.5) * h};
  double r2 = 0;
  for (int k = start[c] + lane; k < end[c]; k += 64) {
    const double* cv = pv + 9 * (int64_t)k;
    for (int v = 0; v < 3; ++v) {
      const double s0 = cv[3 * v] - ctr[0], s1 = cv[3 * v + 1] - ctr[1], s2 = cv[3 * v + 2] - ctr[2];
      r2 = fmax(r2, (s0 * s0 + s1 * s1) + s2 * s2);
    }
  }
  for (int o = 32; o > 0; o >>= 1) r2 = fmax(r2, __shfl_xor(r2, o, 64));
  if (lane == 0) rho_c[c] = sqrt(r2);
}

__global__ void k_parents(const int32_t* __restrict__ start, int n, const int32_t* __restrict__ owner_up,
                          int32_t* parent) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) parent[c] = owner_up[start[c]];
}

__global__ void k_children(const int32_t* __restrict__ parent, int n, int32_t* child_start, int32_t* child_end) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int p = parent[c];
  if (c == 0 || parent[c - 1] != p) child_start[p] = c;
  if (c == n - 1 || parent[c + 1] != p) child_end[p] = c + 1;
}

// ---------------------------------------------------------------------------
// neighbour / interaction lists of one level from the parent level's
// neighbour lists; PASS 0 counts (and records the largest neighbour offset),
// PASS 1 fills at the scanned offsets
// ---------------------------------------------------------------------------
struct ListArgs {
  const int32_t* idx;          // this level
  const int32_t* parent;
  const int32_t* pnbr_off;     // parent level
  const int32_t* pnbr;
  const int32_t* pchild_start;
  const int32_t* pchild_end;
  int n;
  double c0, c1, c2, h, rho, eta0;
  int W, span;
  const double* rho_c;         // per-cluster radii, or null for rho on every cluster
};

template <int PASS>
__global__ void k_lists(ListArgs a, int32_t* ncnt, int32_t* icnt, int* reach, const int32_t* __restrict__ nbr_off,
                        const int32_t* __restrict__ inter_off, int32_t* nbr, int32_t* inter_src, int32_t* ikey) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.n) return;
  const int p = a.parent[c];
  const int ix = a.idx[3 * c], iy = a.idx[3 * c + 1], iz = a.idx[3 * c + 2];
  const double xc0 = a.c0 + ((double)ix + 0.5) * a.h;
  const double xc1 = a.c1 + ((double)iy + 0.5) * a.h;
  const double xc2 = a.c2 + ((double)iz + 0.5) * a.h;
  int nn = 0, ni = 0, rmax = 0;
  int32_t pn = PASS ? nbr_off[c] : 0, pi = PASS ? inter_off[c] : 0;
  for (int q = a.pnbr_off[p]; q < a.pnbr_off[p + 1]; ++q) {
    const int pq = a.pnbr[q];
    for (int c2 = a.pchild_start[pq]; c2 < a.pchild_end[pq]; ++c2) {
      const int jx = a.idx[3 * c2], jy = a.idx[3 * c2 + 1], jz = a.idx[3 * c2 + 2];
      const double s0 = xc0 - (a.c0 + ((double)jx + 0.5) * a.h);
      const double s1 = xc1 - (a.c1 + ((double)jy + 0.5) * a.h);
      const double s2 = xc2 - (a.c2 + ((double)jz + 0.5) * a.h);
      const double dist = sqrt((s0 * s0 + s1 * s1) + s2 * s2);
      const double num = a.rho_c ? a.rho_c[c] + a.rho_c[c2] : a.rho + a.rho;
      const double eta = num / dist;   // +inf for c2 == c
      const int o0 = ix - jx, o1 = iy - jy, o2 = iz - jz;
      if (eta > a.eta0) {
        if (PASS == 0) {
          ++nn;
          rmax = max(rmax, max(abs(o0), max(abs(o1), abs(o2))));
        } else {
          nbr[pn++] = c2;
        }
      } else {
        if (PASS == 0) {
          ++ni;
        } else {
          inter_src[pi] = c2;
          ikey[pi++] = ((o0 + a.W) * a.span + (o1 + a.W)) * a.span + (o2 + a.W);
        }
      }
    }
  }
  if (PASS == 0) {
    ncnt[c] = nn;
    icnt[c] = ni;
    if (rmax > 0) atomicMax(reach, rmax);
  }
}

__global__ void k_mark(const int32_t* __restrict__ ikey, int64_t n, int32_t* used) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) used[ikey[k]] = 1;
}

__global__ void k_offsets(const int32_t* __restrict__ used, const int32_t* __restrict__ id, int64_t nkeys, int W,
                          int span, int32_t* off_xyz) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nkeys || !used[k]) return;
  const int32_t o = id[k];
  off_xyz[3 * o] = (int32_t)(k / ((int64_t)span * span)) - W;
  off_xyz[3 * o + 1] = (int32_t)((k / span) % span) - W;
  off_xyz[3 * o + 2] = (int32_t)(k % span) - W;
}

__global__ void k_map_ids(const int32_t* __restrict__ ikey, int64_t n, const int32_t* __restrict__ id, int32_t* oid) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) oid[k] = id[ikey[k]];
}

// ---------------------------------------------------------------------------
// leaf-level near-field layout: per leaf c, the source panels of every
// c' in N(c) in list order, and n_c x S_c entries stored row by row
// ---------------------------------------------------------------------------
// one wavefront per leaf (launched with 256 threads), lanes over its
// neighbour leaves: each neighbour's column is the exclusive prefix sum of the
// neighbours' panel counts in list order
__global__ void __launch_bounds__(256) k_leaf_count(const int32_t* __restrict__ nbr_off,
                                                   const int32_t* __restrict__ nbr,
                                                   const int32_t* __restrict__ start,
                                                   const int32_t* __restrict__ end, int nl, int32_t* cnt,
                                                   int64_t* nsrc, int64_t* nent, int32_t* self_col,
                                                   int32_t* col) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= nl) return;
  const int q0 = nbr_off[c], q1 = nbr_off[c + 1];
  int base = 0, sc = -1;
  for (int qb = q0; qb < q1; qb += 64) {
    const int q = qb + lane;
    const int c2 = q < q1 ? nbr[q] : -1;
    const int m = q < q1 ? end[c2] - start[c2] : 0;
    int x = m;   // inclusive scan over the lanes
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (q < q1) {
      col[q] = base + x - m;
      if (c2 == c) sc = base + x - m;
    }
    base += __shfl(x, 63, 64);
  }
  for (int o = 32; o > 0; o >>= 1) sc = max(sc, __shfl_xor(sc, o, 64));
  if (lane == 0) {
    const int nc = end[c] - start[c];
    cnt[c] = nc;
    nsrc[c] = base;
    nent[c] = (int64_t)base * nc;
    self_col[c] = sc;
  }
}

// one wavefront per leaf (256 threads), lanes over its neighbour leaves, each
// writing that neighbour's run of panels into the leaf's source list
__global__ void __launch_bounds__(256) k_leaf_sources(const int32_t* __restrict__ nbr_off,
                                                     const int32_t* __restrict__ nbr,
                                                     const int32_t* __restrict__ start,
                                                     const int32_t* __restrict__ end,
                                                     const int64_t* __restrict__ src_off,
                                                     const int32_t* __restrict__ col, int nl,
                                                     int32_t* src_tree, int32_t* leaf_of) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= nl) return;
  const int64_t so = src_off[c];
  for (int q = nbr_off[c] + lane; q < nbr_off[c + 1]; q += 64) {
    const int c2 = nbr[q];
    const int j0 = start[c2], n2 = end[c2] - j0;
    const int64_t b = so + col[q];
    for (int j = 0; j < n2; ++j) src_tree[b + j] = j0 + j;
  }
  for (int i = start[c] + lane; i < end[c]; i += 64) leaf_of[i] = c;
}

inline unsigned grid_of(int64_t n, int tb = TB) { return (unsigned)std::max<int64_t>(1, (n + tb - 1) / tb); }

// scratch memory for one build: bump allocation from a few large chunks,
// all freed when the build returns
struct Arena {
  std::vector<std::unique_ptr<Tmp>> chunks;
  size_t used = 0, cap = 0;
  template <class T> int get(T*& p, size_t count) {
    const size_t bytes = (std::max<size_t>(1, count) * sizeof(T) + 255) & ~(size_t)255;
    if (chunks.empty() || used + bytes > cap) {
      cap = std::max<size_t>(bytes, (size_t)64 << 20);
      chunks.emplace_back(new Tmp());
      FAGBI_TRY(chunks.back()->alloc(cap));
      used = 0;
    }
    p = reinterpret_cast<T*>(static_cast<char*>(chunks.back()->p) + used);
    used += bytes;
    return 0;
  }
};

// exclusive scan in[0..n) -> out[0..n], out[n] = total
template <typename TI, typename TO>
int scan(Arena& A, const TI* in, int64_t n, TO* out, hipStream_t s) {
  TO* part;
  FAGBI_TRY(A.get(part, scan_part_size(n)));
  return device_scan<TI, TO>(in, n, out, part, s);
}

int scan_ii(Arena& A, const int32_t* in, int64_t n, int32_t* out, hipStream_t s) {
  return scan<int32_t, int32_t>(A, in, n, out, s);
}
int scan_ll(Arena& A, const int64_t* in, int64_t n, int64_t* out, hipStream_t s) {
  return scan<int64_t, int64_t>(A, in, n, out, s);
}

// sorts (key, val) by the low `bits` bits of key, stably; the result ends in
// k0/v0
int radix_sort(Arena& A, uint64_t* k0, int32_t* v0, int64_t n, int bits, hipStream_t s) {
  uint64_t* k1;
  int32_t* v1;
  int* hist;
  int* offs;
  const int nb = (int)std::max<int64_t>(1, (n + TILE - 1) / TILE);
  FAGBI_TRY(A.get(k1, n));
  FAGBI_TRY(A.get(v1, n));
  FAGBI_TRY(A.get(hist, (size_t)RBINS * nb));
  FAGBI_TRY(A.get(offs, (size_t)RBINS * nb + 1));
  const int passes = (bits + RBITS - 1) / RBITS;
  const int64_t nh = (int64_t)RBINS * nb, nbh = (nh + TILE - 1) / TILE;
  int* part;
  FAGBI_TRY(A.get(part, nbh + 1));
  uint64_t *ka = k0, *kb = k1;
  int32_t *va = v0, *vb = v1;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * RBITS;
    k_radix_hist<<<nb, TB, 0, s>>>(ka, n, shift, nb, hist);
    k_scan_reduce<int, int><<<(unsigned)nbh, TB, 0, s>>>(hist, nh, part);
    k_scan_part<int><<<1, TB, 0, s>>>(part, nbh);
    k_scan_down<int, int><<<(unsigned)nbh, TB, 0, s>>>(hist, nh, part, nbh, offs);
    k_radix_scatter<<<nb, TB, 0, s>>>(ka, va, kb, vb, n, shift, nb, offs);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  FAGBI_HIP(hipGetLastError());
  if (ka != k0) {
    FAGBI_HIP(hipMemcpyAsync(k0, ka, n * 8, hipMemcpyDeviceToDevice, s));
    FAGBI_HIP(hipMemcpyAsync(v0, va, n * 4, hipMemcpyDeviceToDevice, s));
  }
  return 0;
}

template <class T> int to_host(std::vector<T>& v, const T* d, size_t n) {
  v.resize(n);
  if (n) FAGBI_HIP(hipMemcpy(v.data(), d, n * sizeof(T), hipMemcpyDeviceToHost));
  return 0;
}

}  // namespace

int build_tree(fagbi_handle* h, const double* verts, int64_t nv, const int32_t* tris, int64_t nt) {
  const int leaf = h->prm.leaf_size;
  const double eta0 = h->prm.eta0;
  if (nt <= 0 || nv <= 2) return set_error(FAGBI_E_ARG, "build_tree: empty mesh");
  // index checks on the host: every later kernel indexes vertices through
  // the triangles
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t* tr = tris + 3 * t;
    for (int k = 0; k < 3; ++k)
      if (tr[k] < 0 || tr[k] >= nv)
        return set_error(FAGBI_E_ARG, "build_tree: triangle %lld has vertex index %d out of [0,%lld)",
                         (long long)t, tr[k], (long long)nv);
    if (tr[0] == tr[1] || tr[1] == tr[2] || tr[0] == tr[2])
      return set_error(FAGBI_E_MESH, "build_tree: triangle %lld repeats a vertex", (long long)t);
  }
  if (h->hat()) {   // every vertex carries a hat function: it must lie on a triangle
    std::vector<char> used(nv, 0);
    for (int64_t k = 0; k < 3 * nt; ++k) used[tris[k]] = 1;
    for (int64_t v = 0; v < nv; ++v)
      if (!used[v])
        return set_error(FAGBI_E_MESH, "build_tree: vertex %lld belongs to no triangle", (long long)v);
  }
  hipStream_t s = 0;
  const int64_t N = nt;
  Arena A;
  double* dv;
  int32_t* dt;
  FAGBI_TRY(A.get(dv, 3 * nv));
  FAGBI_TRY(A.get(dt, 3 * N));
  FAGBI_HIP(hipMemcpyAsync(dv, verts, 3 * nv * 8, hipMemcpyHostToDevice, s));
  FAGBI_HIP(hipMemcpyAsync(dt, tris, 3 * N * 4, hipMemcpyHostToDevice, s));
  // ---- edge checks (hash set of directed edges with multiplicities) -------
  Check* chk;
  FAGBI_TRY(A.get(chk, 1));
  {
    Check c0{};
    c0.open_tri = c0.orient_tri = c0.degen_tri = INT_MAX;
    FAGBI_HIP(hipMemcpy(chk, &c0, sizeof c0, hipMemcpyHostToDevice));
  }
  uint64_t hs = 1;
  while (hs < (uint64_t)(6 * N)) hs <<= 1;
  unsigned long long* tab;
  int* tcnt;
  FAGBI_TRY(A.get(tab, hs));
  FAGBI_TRY(A.get(tcnt, hs));
  FAGBI_HIP(hipMemsetAsync(tab, 0xff, hs * 8, s));
  FAGBI_HIP(hipMemsetAsync(tcnt, 0, hs * 4, s));
  k_edge_insert<<<grid_of(3 * N), TB, 0, s>>>(dt, N, tab, tcnt, hs - 1);
  k_edge_check<<<grid_of(3 * N), TB, 0, s>>>(dt, N, tab, tcnt, hs - 1, chk);
  // ---- geometry ---------------------------------------------------------------
  double *cor, *cen, *nrm, *area, *part;
  const int nbg = (int)grid_of(N);
  FAGBI_TRY(A.get(cor, 9 * N));
  FAGBI_TRY(A.get(cen, 3 * N));
  FAGBI_TRY(A.get(nrm, 3 * N));
  FAGBI_TRY(A.get(area, N));
  FAGBI_TRY(A.get(part, 7 * (size_t)nbg));
  k_geometry<<<nbg, TB, 0, s>>>(dv, dt, N, cor, cen, nrm, area, part, chk);
  k_geometry_final<<<1, TB, 0, s>>>(part, nbg, chk);
  FAGBI_HIP(hipGetLastError());
  Check hc;
  FAGBI_HIP(hipMemcpy(&hc, chk, sizeof hc, hipMemcpyDeviceToHost));
  if (hc.open_tri != INT_MAX)
    return set_error(FAGBI_E_MESH,
                     "build_tree: mesh is open or non-manifold (an edge of triangle %d is not shared by exactly "
                     "two triangles)", hc.open_tri);
  if (hc.orient_tri != INT_MAX)
    return set_error(FAGBI_E_MESH, "build_tree: inconsistent triangle orientation (at triangle %d)", hc.orient_tri);
  if (hc.degen_tri != INT_MAX)
    return set_error(FAGBI_E_MESH, "build_tree: triangle %d is degenerate", hc.degen_tri);
  if (!(hc.vol6 > 0))
    return set_error(FAGBI_E_MESH,
                     "build_tree: mesh encloses negative volume (triangles must be counter-clockwise seen from "
                     "outside)");
  // ---- level-0 cube, keys, sort ------------------------------------------------
  const double ext = std::max(hc.hi[0] - hc.lo[0], std::max(hc.hi[1] - hc.lo[1], hc.hi[2] - hc.lo[2]));
  const double side = ext * (1.0 + 1e-12);
  double corner[3];
  for (int d = 0; d < 3; ++d) corner[d] = 0.5 * (hc.lo[d] + hc.hi[d]) - 0.5 * side;
  const double h20 = side / (double)(1 << DEEP);
  uint64_t* key;
  int32_t* val;
  FAGBI_TRY(A.get(key, N));
  FAGBI_TRY(A.get(val, N));
  k_keys<<<grid_of(N), TB, 0, s>>>(cen, N, corner[0], corner[1], corner[2], h20, key, val);
  FAGBI_TRY(radix_sort(A, key, val, N, 3 * DEEP, s));
  int* dL;
  FAGBI_TRY(A.get(dL, 1));
  FAGBI_HIP(hipMemsetAsync(dL, 0, 4, s));
  k_leaf_level<<<grid_of(N), TB, 0, s>>>(key, N, leaf, dL);
  int L = 0;
  FAGBI_HIP(hipMemcpy(&L, dL, 4, hipMemcpyDeviceToHost));
  if (L > DEEP) return set_error(FAGBI_E_MESH, "build_tree: leaf_size not reached within 20 levels (coincident centroids?)");
  // ---- a new mesh replaces every device buffer ------------------------------
  h->near_ready = false;
  h->tree_ready = false;
  FAGBI_HIP(hipDeviceSynchronize());
  h->free_all();
  {
    std::vector<double> gl(qt_size(h->prm.quad_duffy));
    quad_table(h->prm.quad_duffy, gl.data());
    FAGBI_TRY(h->upload(h->d_gl, gl.data(), gl.size() * sizeof(double)));
  }
  h->N = N;
  h->nv = nv;
  h->L = L;
  h->side = side;
  for (int d = 0; d < 3; ++d) h->corner[d] = corner[d];
  uint64_t* keyL;
  FAGBI_TRY(A.get(keyL, N));
  FAGBI_TRY(h->alloc(h->d_perm, N * 4));
  FAGBI_TRY(h->alloc(h->d_pv, 9 * N * 8));
  FAGBI_TRY(h->alloc(h->d_pn, 3 * N * 8));
  FAGBI_TRY(h->alloc(h->d_pa, N * 8));
  FAGBI_TRY(h->alloc(h->d_ptri, 3 * N * 4));
  FAGBI_TRY(h->alloc(h->d_pc, N * sizeof(double4)));
  FAGBI_TRY(h->alloc(h->d_xt, (h->hat() ? 6 : 2) * N * sizeof(double)));   // rows: panels or corners
  int32_t* perm = h->d_perm.as<int32_t>();
  k_leaf_order<<<grid_of(N), TB, 0, s>>>(key, val, N, 3 * (DEEP - L), leaf, perm, keyL);
  k_permute<<<grid_of(N), TB, 0, s>>>(perm, N, cor, nrm, area, dt, h->d_pv.as<double>(), h->d_pn.as<double>(),
                                      h->d_pa.as<double>(), h->d_ptri.as<int32_t>(), h->d_pc.as<double4>());
  // ---- levels: clusters, cube indices, radii ---------------------------------
  std::vector<int32_t*> owner(L + 1), start(L + 1), end(L + 1);
  std::vector<int32_t*> excl(L + 1), flag(L + 1);
  for (int l = 0; l <= L; ++l) {
    FAGBI_TRY(A.get(flag[l], N));
    FAGBI_TRY(A.get(excl[l], N + 1));
    k_level_flags<<<grid_of(N), TB, 0, s>>>(keyL, N, 3 * (L - l), flag[l]);
    FAGBI_TRY(scan_ii(A, flag[l], N, excl[l], s));
  }
  h->lev.assign(L + 1, Level());
  std::vector<int32_t> ncl(L + 1);
  for (int l = 0; l <= L; ++l) FAGBI_HIP(hipMemcpyAsync(&ncl[l], excl[l] + N, 4, hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipStreamSynchronize(s));
  unsigned long long* rho_bits;
  FAGBI_TRY(A.get(rho_bits, L + 1));
  FAGBI_HIP(hipMemsetAsync(rho_bits, 0, (L + 1) * 8, s));
  for (int l = 0; l <= L; ++l) {
    Level& D = h->lev[l];
    D.n = ncl[l];
    D.h = side / (double)(1 << l);
    D.order = h->prm.adaptive ? std::min(h->prm.p_leaf + L - l, h->prm.p_max) : h->prm.p_leaf;
    D.T = nterms(D.order);
    FAGBI_TRY(h->alloc(D.d_idx, 3 * (size_t)D.n * 4));
    FAGBI_TRY(h->alloc(D.d_parent, (size_t)D.n * 4));
    FAGBI_TRY(h->alloc(D.d_child_start, (size_t)D.n * 4));
    FAGBI_TRY(h->alloc(D.d_child_end, (size_t)D.n * 4));
    FAGBI_HIP(hipMemsetAsync(D.d_child_start.p, 0, (size_t)D.n * 4, s));
    FAGBI_HIP(hipMemsetAsync(D.d_child_end.p, 0, (size_t)D.n * 4, s));
    FAGBI_TRY(A.get(owner[l], N));
    FAGBI_TRY(A.get(start[l], D.n));
    FAGBI_TRY(A.get(end[l], D.n));
    k_level_fill<<<grid_of(N), TB, 0, s>>>(keyL, flag[l], excl[l], N, 3 * (L - l), owner[l],
                                           D.d_idx.as<int32_t>(), start[l], end[l]);
    k_level_rho<<<grid_of(N), TB, 0, s>>>(h->d_pv.as<double>(), owner[l], D.d_idx.as<int32_t>(), N, corner[0],
                                          corner[1], corner[2], D.h, rho_bits + l);
    if (h->prm.radii == FAGBI_RADII_CLUSTER) {
      FAGBI_TRY(h->alloc(D.d_rho_c, (size_t)D.n * 8));
      k_cluster_rho<<<(unsigned)((D.n + 3) / 4), 256, 0, s>>>(h->d_pv.as<double>(), start[l], end[l],
                                                              D.d_idx.as<int32_t>(), D.n, corner[0], corner[1],
                                                              corner[2], D.h, D.d_rho_c.as<double>());
    }
  }
  {
    const int32_t m1 = -1;
    FAGBI_HIP(hipMemcpy(h->lev[0].d_parent.p, &m1, 4, hipMemcpyHostToDevice));
  }
  for (int l = 1; l <= L; ++l) {
    Level &C = h->lev[l], &P = h->lev[l - 1];
    k_parents<<<grid_of(C.n), TB, 0, s>>>(start[l], C.n, owner[l - 1], C.d_parent.as<int32_t>());
    k_children<<<grid_of(C.n), TB, 0, s>>>(C.d_parent.as<int32_t>(), C.n, P.d_child_start.as<int32_t>(),
                                           P.d_child_end.as<int32_t>());
  }
  FAGBI_HIP(hipGetLastError());
  {
    std::vector<double> rho(L + 1);
    FAGBI_HIP(hipMemcpy(rho.data(), rho_bits, (L + 1) * 8, hipMemcpyDeviceToHost));
    for (int l = 0; l <= L; ++l) h->lev[l].rho = rho[l];
  }
  // ---- neighbour and interaction lists ------------------------------------------
  std::vector<int32_t*> nbr_off(L + 1), nbr(L + 1);
  FAGBI_TRY(A.get(nbr_off[0], 2));
  FAGBI_TRY(A.get(nbr[0], 1));
  {
    const int32_t no[2] = {0, 1}, nb0 = 0, io[2] = {0, 0};
    FAGBI_HIP(hipMemcpy(nbr_off[0], no, 8, hipMemcpyHostToDevice));
    FAGBI_HIP(hipMemcpy(nbr[0], &nb0, 4, hipMemcpyHostToDevice));
    FAGBI_TRY(h->alloc(h->lev[0].d_inter_off, 8));
    FAGBI_HIP(hipMemcpy(h->lev[0].d_inter_off.p, io, 8, hipMemcpyHostToDevice));
  }
  int lmin = L + 1;
  int reach = 0;   // largest |offset component| among neighbours on level l-1
  int* dreach;
  FAGBI_TRY(A.get(dreach, 1));
  for (int l = 1; l <= L; ++l) {
    Level &C = h->lev[l], &P = h->lev[l - 1];
    const int W = 2 * reach + 1;
    const int span = 2 * W + 1;
    if ((double)span * span * span > (double)(1 << 28))
      return set_error(FAGBI_E_MESH, "build_tree: neighbour stencil too wide on level %d (reach %d)", l, reach);
    ListArgs a{C.d_idx.as<int32_t>(), C.d_parent.as<int32_t>(), nbr_off[l - 1], nbr[l - 1],
               P.d_child_start.as<int32_t>(), P.d_child_end.as<int32_t>(), C.n, corner[0], corner[1], corner[2],
               C.h, C.rho, eta0, W, span, C.d_rho_c.p ? C.d_rho_c.as<double>() : nullptr};
    int32_t *ncnt, *icnt;
    FAGBI_TRY(A.get(ncnt, C.n));
    FAGBI_TRY(A.get(icnt, C.n));
    FAGBI_TRY(A.get(nbr_off[l], C.n + 1));
    FAGBI_TRY(h->alloc(C.d_inter_off, ((size_t)C.n + 1) * 4));
    FAGBI_HIP(hipMemsetAsync(dreach, 0, 4, s));
    k_lists<0><<<grid_of(C.n), TB, 0, s>>>(a, ncnt, icnt, dreach, nullptr, nullptr, nullptr, nullptr, nullptr);
    FAGBI_TRY(scan_ii(A, ncnt, C.n, nbr_off[l], s));
    FAGBI_TRY(scan_ii(A, icnt, C.n, C.d_inter_off.as<int32_t>(), s));
    int32_t tot[3];
    FAGBI_HIP(hipMemcpyAsync(&tot[0], nbr_off[l] + C.n, 4, hipMemcpyDeviceToHost, s));
    FAGBI_HIP(hipMemcpyAsync(&tot[1], C.d_inter_off.as<int32_t>() + C.n, 4, hipMemcpyDeviceToHost, s));
    FAGBI_HIP(hipMemcpyAsync(&tot[2], dreach, 4, hipMemcpyDeviceToHost, s));
    FAGBI_HIP(hipStreamSynchronize(s));
    const int64_t nnb = tot[0], nin = tot[1];
    int32_t* ikey;
    FAGBI_TRY(A.get(nbr[l], nnb));
    FAGBI_TRY(A.get(ikey, nin));
    FAGBI_TRY(h->alloc(C.d_inter_src, (size_t)std::max<int64_t>(1, nin) * 4));
    FAGBI_TRY(h->alloc(C.d_inter_oid, (size_t)std::max<int64_t>(1, nin) * 4));
    k_lists<1><<<grid_of(C.n), TB, 0, s>>>(a, nullptr, nullptr, nullptr, nbr_off[l], C.d_inter_off.as<int32_t>(),
                                           nbr[l], C.d_inter_src.as<int32_t>(), ikey);
    C.n_inter = nin;
    if (nin > 0) {
      // distinct offsets numbered in increasing key order
      const int64_t nkeys = (int64_t)span * span * span;
      int32_t *used, *id, *offs;
      FAGBI_TRY(A.get(used, nkeys));
      FAGBI_TRY(A.get(id, nkeys + 1));
      FAGBI_HIP(hipMemsetAsync(used, 0, nkeys * 4, s));
      k_mark<<<grid_of(nin), TB, 0, s>>>(ikey, nin, used);
      FAGBI_TRY(scan_ii(A, used, nkeys, id, s));
      int32_t noff = 0;
      FAGBI_HIP(hipMemcpy(&noff, id + nkeys, 4, hipMemcpyDeviceToHost));
      FAGBI_TRY(A.get(offs, 3 * (size_t)noff));
      k_offsets<<<grid_of(nkeys), TB, 0, s>>>(used, id, nkeys, W, span, offs);
      k_map_ids<<<grid_of(nin), TB, 0, s>>>(ikey, nin, id, C.d_inter_oid.as<int32_t>());
      FAGBI_HIP(hipGetLastError());
      FAGBI_TRY(to_host(C.off_xyz, offs, 3 * (size_t)noff));
      C.n_off = noff;
      if (lmin > L) lmin = l;
    }
    reach = tot[2];
  }
  h->lmin = lmin;
  // ---- leaf-level near-field layout ----------------------------------------------
  const Level& LF = h->lev[L];
  const int nl = LF.n;
  int32_t *col, *cnt;
  int64_t *nsrc, *nent;
  int32_t nq = 0;
  FAGBI_HIP(hipMemcpy(&nq, nbr_off[L] + nl, 4, hipMemcpyDeviceToHost));
  FAGBI_TRY(A.get(cnt, nl));
  FAGBI_TRY(A.get(nsrc, nl));
  FAGBI_TRY(A.get(nent, nl));
  FAGBI_TRY(h->alloc(h->d_self_col, (size_t)nl * 4));
  FAGBI_TRY(h->alloc(h->d_lnbr_off, ((size_t)nl + 1) * 4));
  FAGBI_TRY(h->alloc(h->d_lnbr, (size_t)std::max(1, nq) * 4));
  FAGBI_TRY(h->alloc(h->d_lnbr_col, (size_t)std::max(1, nq) * 4));
  col = h->d_lnbr_col.as<int32_t>();
  FAGBI_HIP(hipMemcpyAsync(h->d_lnbr_off.p, nbr_off[L], ((size_t)nl + 1) * 4, hipMemcpyDeviceToDevice, s));
  FAGBI_HIP(hipMemcpyAsync(h->d_lnbr.p, nbr[L], (size_t)nq * 4, hipMemcpyDeviceToDevice, s));
  FAGBI_TRY(h->alloc(h->d_leaf_start, (size_t)nl * 4));
  FAGBI_TRY(h->alloc(h->d_leaf_cnt, (size_t)nl * 4));
  FAGBI_HIP(hipMemcpyAsync(h->d_leaf_start.p, start[L], (size_t)nl * 4, hipMemcpyDeviceToDevice, s));
  k_leaf_count<<<(unsigned)((nl + 3) / 4), 256, 0, s>>>(nbr_off[L], nbr[L], start[L], end[L], nl,
                                                        h->d_leaf_cnt.as<int32_t>(), nsrc, nent,
                                                        h->d_self_col.as<int32_t>(), col);
  FAGBI_TRY(h->alloc(h->d_src_off, ((size_t)nl + 1) * 8));
  FAGBI_TRY(h->alloc(h->d_ent_off, ((size_t)nl + 1) * 8));
  FAGBI_TRY(scan_ll(A, nsrc, nl, h->d_src_off.as<int64_t>(), s));
  FAGBI_TRY(scan_ll(A, nent, nl, h->d_ent_off.as<int64_t>(), s));
  FAGBI_HIP(hipMemcpy(&h->n_src, h->d_src_off.as<int64_t>() + nl, 8, hipMemcpyDeviceToHost));
  FAGBI_HIP(hipMemcpy(&h->n_ent, h->d_ent_off.as<int64_t>() + nl, 8, hipMemcpyDeviceToHost));
  FAGBI_TRY(h->alloc(h->d_src_tree, (size_t)std::max<int64_t>(1, h->n_src) * 4));
  FAGBI_TRY(h->alloc(h->d_leaf_of, (size_t)N * 4));
  k_leaf_sources<<<(unsigned)((nl + 3) / 4), 256, 0, s>>>(nbr_off[L], nbr[L], start[L], end[L],
                                                          h->d_src_off.as<int64_t>(), col, nl,
                                                          h->d_src_tree.as<int32_t>(), h->d_leaf_of.as<int32_t>());
  FAGBI_HIP(hipGetLastError());
  FAGBI_TRY(to_host(h->leaf_cnt, h->d_leaf_cnt.as<int32_t>(), nl));
  h->max_leaf = 0;
  for (int c = 0; c < nl; ++c) h->max_leaf = std::max(h->max_leaf, h->leaf_cnt[c]);
  FAGBI_HIP(hipStreamSynchronize(s));
  h->tree_ready = true;
  return 0;
}

}  // namespace fagbi
