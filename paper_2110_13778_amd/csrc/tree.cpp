// Cluster tree of panel centroids (paper Sec. 2.4: level-0 cube, cube
// refinement, clusters as the panels whose centroids lie in a cube, separation
// ratio, neighbour lists N(c) and interaction lists I(c)).
//
// Choices the paper leaves open:
//  * level-0 cube centred on the vertex bounding box, side = largest extent
//    times (1 + 1e-12);
//  * uniform depth: L = smallest level whose fullest cube holds <= leaf_size
//    centroids; empty cubes are dropped;
//  * cube index of a centroid on level l: floor((c - corner)/h_l) clamped to
//    [0, 2^l - 1] (computed once on level 20 and shifted, which is exact);
//  * cluster centre = cube centre, one radius per level (the farthest
//    3-point-rule quadrature point of a member panel from its cube centre:
//    the far field only ever evaluates that rule), so the separation ratio
//    2 rho_l / |x_c - x_c'| depends on the index offset alone and every level
//    has a fixed stencil of interaction offsets;
//  * c' in N(c) iff c' is a child of a neighbour of c's parent and the ratio
//    exceeds eta0; the remaining such children form I(c).
#include "tree.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <thread>

#include "../../include/fagbi.h"

namespace fagbi {

static int host_threads(int64_t work) {
  unsigned hc = std::thread::hardware_concurrency();
  int n = (int)std::min<unsigned>(hc ? hc : 1, 16);
  return (int)std::max<int64_t>(1, std::min<int64_t>(n, work / 4096 + 1));
}

// fn(thread, begin, end) over [0, n) split into nth contiguous chunks
template <class F>
static void parallel_chunks(int64_t n, int nth, F fn) {
  std::vector<std::thread> th;
  for (int t = 0; t < nth; ++t) {
    const int64_t lo = n * t / nth, hi = n * (t + 1) / nth;
    th.emplace_back([=, &fn] { fn(t, lo, hi); });
  }
  for (auto& x : th) x.join();
}

static uint64_t spread3(uint64_t v) {
  uint64_t out = 0;
  for (int b = 0; b < 21; ++b) out |= ((v >> b) & 1ull) << (3 * b);
  return out;
}

static uint64_t morton(int64_t x, int64_t y, int64_t z) {
  return (spread3((uint64_t)x) << 2) | (spread3((uint64_t)y) << 1) | spread3((uint64_t)z);
}

static int64_t cube_coord(double c, double corner, double h, int64_t nmax) {
  double k = std::floor((c - corner) / h);
  if (k < 0) k = 0;
  if (k > (double)(nmax - 1)) k = (double)(nmax - 1);
  return (int64_t)k;
}

int build_tree_host(const double* verts, int64_t nv, const int32_t* tris, int64_t nt,
                    int leaf_size, double eta0, TreeOut& out, std::string& err) {
  char buf[256];
  if (nt <= 0 || nv <= 2 || leaf_size <= 0 || !(eta0 >= 0)) {
    err = "build_tree: empty mesh or bad leaf_size/eta0";
    return FAGBI_E_ARG;
  }
  for (int64_t t = 0; t < 3 * nt; ++t)
    if (tris[t] < 0 || tris[t] >= nv) {
      snprintf(buf, sizeof buf, "build_tree: triangle %lld has vertex index %d out of [0,%lld)",
               (long long)(t / 3), tris[t], (long long)nv);
      err = buf;
      return FAGBI_E_ARG;
    }
  // ---- closed, consistently oriented 2-manifold check -------------------
  // every undirected edge must occur exactly twice, once in each direction
  {
    std::vector<uint64_t> und(3 * nt);
    for (int64_t t = 0; t < nt; ++t)
      for (int e = 0; e < 3; ++e) {
        uint64_t a = (uint64_t)tris[3 * t + e], b = (uint64_t)tris[3 * t + (e + 1) % 3];
        if (a == b) {
          snprintf(buf, sizeof buf, "build_tree: triangle %lld repeats a vertex", (long long)t);
          err = buf;
          return FAGBI_E_MESH;
        }
        und[3 * t + e] = ((std::min(a, b) * (uint64_t)nv + std::max(a, b)) << 1) | (a < b ? 1u : 0u);
      }
    std::sort(und.begin(), und.end());
    for (size_t k = 0; k < und.size(); k += 2) {
      if (k + 1 >= und.size() || (und[k] >> 1) != (und[k + 1] >> 1) ||
          (k + 2 < und.size() && (und[k + 2] >> 1) == (und[k] >> 1))) {
        err = "build_tree: mesh is open or non-manifold (an edge is not shared by exactly two triangles)";
        return FAGBI_E_MESH;
      }
      if ((und[k] & 1) == (und[k + 1] & 1)) {
        err = "build_tree: inconsistent triangle orientation";
        return FAGBI_E_MESH;
      }
    }
  }
  // ---- per-panel geometry --------------------------------------------------
  const int64_t N = nt;
  std::vector<double> cen(3 * N), cor(9 * N), nrm(3 * N), area(N);
  double vol6 = 0;
  for (int64_t t = 0; t < N; ++t) {
    const double* u = verts + 3 * tris[3 * t];
    const double* v = verts + 3 * tris[3 * t + 1];
    const double* w = verts + 3 * tris[3 * t + 2];
    double e1[3], e2[3], cr[3];
    for (int d = 0; d < 3; ++d) {
      e1[d] = v[d] - u[d];
      e2[d] = w[d] - u[d];
      cen[3 * t + d] = (u[d] + v[d] + w[d]) / 3.0;
      cor[9 * t + d] = u[d];
      cor[9 * t + 3 + d] = v[d];
      cor[9 * t + 6 + d] = w[d];
    }
    cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
    cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
    cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double two_a = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    if (!(two_a > 0) || !std::isfinite(two_a)) {
      snprintf(buf, sizeof buf, "build_tree: triangle %lld is degenerate", (long long)t);
      err = buf;
      return FAGBI_E_MESH;
    }
    area[t] = 0.5 * two_a;
    for (int d = 0; d < 3; ++d) nrm[3 * t + d] = cr[d] / two_a;
    vol6 += u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0]) +
            u[2] * (v[0] * w[1] - v[1] * w[0]);
  }
  if (!(vol6 > 0)) {
    err = "build_tree: mesh encloses negative volume (triangles must be counter-clockwise seen from outside)";
    return FAGBI_E_MESH;
  }
  // ---- level-0 cube ----------------------------------------------------------
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t t = 0; t < 3 * N; ++t) {
    const double* p = verts + 3 * tris[t];
    for (int d = 0; d < 3; ++d) {
      lo[d] = std::min(lo[d], p[d]);
      hi[d] = std::max(hi[d], p[d]);
    }
  }
  double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
  double side = ext * (1.0 + 1e-12);
  for (int d = 0; d < 3; ++d) out.corner[d] = 0.5 * (lo[d] + hi[d]) - 0.5 * side;
  out.side = side;
  const int DEEP = 20;
  const double h20 = side / (double)(1 << DEEP);
  std::vector<int64_t> ix(3 * N);
  std::vector<uint64_t> key20(N);
  for (int64_t t = 0; t < N; ++t) {
    for (int d = 0; d < 3; ++d)
      ix[3 * t + d] = cube_coord(cen[3 * t + d], out.corner[d], h20, (int64_t)1 << DEEP);
    key20[t] = morton(ix[3 * t], ix[3 * t + 1], ix[3 * t + 2]);
  }
  // ---- leaf level -------------------------------------------------------------
  std::vector<uint64_t> sk(key20);
  std::sort(sk.begin(), sk.end());
  int L = -1;
  for (int l = 0; l <= DEEP; ++l) {
    int sh = 3 * (DEEP - l);
    int64_t best = 0;
    for (int64_t a = 0; a < N;) {
      int64_t b = a;
      uint64_t k = sk[a] >> sh;
      while (b < N && (sk[b] >> sh) == k) ++b;
      best = std::max(best, b - a);
      a = b;
    }
    if (best <= leaf_size) {
      L = l;
      break;
    }
  }
  if (L < 0) {
    err = "build_tree: leaf_size not reached within 20 levels (coincident centroids?)";
    return FAGBI_E_MESH;
  }
  out.L = L;
  const int shL = 3 * (DEEP - L);
  std::vector<std::pair<uint64_t, int32_t>> ord(N);
  for (int64_t t = 0; t < N; ++t) ord[t] = {key20[t] >> shL, (int32_t)t};
  std::sort(ord.begin(), ord.end());
  out.perm.resize(N);
  for (int64_t k = 0; k < N; ++k) out.perm[k] = ord[k].second;
  out.corners.resize(9 * N);
  out.normal.resize(3 * N);
  out.area.resize(N);
  out.tri.resize(3 * N);
  for (int64_t k = 0; k < N; ++k) {
    int64_t t = out.perm[k];
    for (int d = 0; d < 9; ++d) out.corners[9 * k + d] = cor[9 * t + d];
    for (int d = 0; d < 3; ++d) {
      out.normal[3 * k + d] = nrm[3 * t + d];
      out.tri[3 * k + d] = tris[3 * t + d];
    }
    out.area[k] = area[t];
  }
  // ---- levels ---------------------------------------------------------------
  out.lev.assign(L + 1, TreeLevel());
  for (int l = 0; l <= L; ++l) {
    TreeLevel& T = out.lev[l];
    int sh = 3 * (L - l);
    T.h = side / (double)(1 << l);
    std::vector<int32_t> owner(N);
    for (int64_t a = 0; a < N;) {
      int64_t b = a;
      uint64_t k = ord[a].first >> sh;
      while (b < N && (ord[b].first >> sh) == k) ++b;
      int64_t t0 = ord[a].second;
      for (int d = 0; d < 3; ++d)
        T.idx.push_back((int32_t)(ix[3 * t0 + d] >> (DEEP - l)));
      T.start.push_back((int32_t)a);
      T.end.push_back((int32_t)b);
      for (int64_t m = a; m < b; ++m) owner[m] = T.n;
      ++T.n;
      a = b;
    }
    // radius: farthest quadrature point (3-point rule: 2/3 of one corner and
    // 1/6 of the other two) of a member panel from its cube centre; the far
    // field only ever evaluates the rule at these points
    const int nth = host_threads(N);
    std::vector<double> part(nth, 0.0);
    parallel_chunks(N, nth, [&](int t, int64_t lo, int64_t hi) {
      double rho = 0;
      for (int64_t k = lo; k < hi; ++k) {
        const int32_t c = owner[k];
        const double* cv = &out.corners[9 * k];
        for (int v = 0; v < 3; ++v) {
          double s[3];
          for (int d = 0; d < 3; ++d) {
            double ctr = out.corner[d] + ((double)T.idx[3 * c + d] + 0.5) * T.h;
            double qp = (2.0 / 3.0) * cv[3 * v + d] +
                        (1.0 / 6.0) * (cv[3 * ((v + 1) % 3) + d] + cv[3 * ((v + 2) % 3) + d]);
            s[d] = qp - ctr;
          }
          double dist = std::sqrt((s[0] * s[0] + s[1] * s[1]) + s[2] * s[2]);
          rho = std::max(rho, dist);
        }
      }
      part[t] = rho;
    });
    double rho = 0;
    for (double v : part) rho = std::max(rho, v);
    T.rho = rho;
  }
  // parents / children
  out.lev[0].parent.assign(1, -1);
  for (int l = 1; l <= L; ++l) {
    TreeLevel &C = out.lev[l], &P = out.lev[l - 1];
    C.parent.resize(C.n);
    P.child_start.assign(P.n, 0);
    P.child_end.assign(P.n, 0);
    int p = 0;
    for (int c = 0; c < C.n; ++c) {
      while (!(C.start[c] >= P.start[p] && C.start[c] < P.end[p])) ++p;
      C.parent[c] = p;
    }
    for (int c = C.n - 1; c >= 0; --c) P.child_start[C.parent[c]] = c;
    for (int c = 0; c < C.n; ++c) P.child_end[C.parent[c]] = c + 1;
  }
  out.lev[L].child_start.assign(out.lev[L].n, 0);
  out.lev[L].child_end.assign(out.lev[L].n, 0);
  // neighbour and interaction lists (clusters split over host threads; the
  // per-thread pieces are concatenated in cluster order)
  {
    TreeLevel& R = out.lev[0];
    R.nbr_off = {0, 1};
    R.nbr = {0};
    R.inter_off = {0, 0};
  }
  out.lmin = L + 1;
  int reach = 0;   // largest |offset component| among neighbours on level l-1
  for (int l = 1; l <= L; ++l) {
    TreeLevel &C = out.lev[l], &P = out.lev[l - 1];
    const int W = 2 * reach + 1;            // bound on |offset| on this level
    const int span = 2 * W + 1;
    // pass 1: counts per cluster; pass 2: fill at the prefix-sum offsets
    const int nth = host_threads(C.n);
    std::vector<int32_t> ncnt(C.n), icnt(C.n);
    std::vector<int> reach_t(nth, 0);
    auto visit = [&](int64_t c, auto&& on_nbr, auto&& on_int) {
      const int p = C.parent[c];
      double xc[3];
      for (int d = 0; d < 3; ++d) xc[d] = out.corner[d] + ((double)C.idx[3 * c + d] + 0.5) * C.h;
      for (int q = P.nbr_off[p]; q < P.nbr_off[p + 1]; ++q) {
        const int pq = P.nbr[q];
        for (int c2 = P.child_start[pq]; c2 < P.child_end[pq]; ++c2) {
          double s[3];
          for (int d = 0; d < 3; ++d)
            s[d] = xc[d] - (out.corner[d] + ((double)C.idx[3 * c2 + d] + 0.5) * C.h);
          double dist = std::sqrt((s[0] * s[0] + s[1] * s[1]) + s[2] * s[2]);
          double eta = (C.rho + C.rho) / dist;   // +inf for c2 == c
          int o[3];
          for (int d = 0; d < 3; ++d) o[d] = C.idx[3 * c + d] - C.idx[3 * c2 + d];
          if (eta > eta0)
            on_nbr(c2, o);
          else
            on_int(c2, o);
        }
      }
    };
    parallel_chunks(C.n, nth, [&](int t, int64_t lo, int64_t hi) {
      int rmax = 0;
      for (int64_t c = lo; c < hi; ++c) {
        int nn = 0, ni = 0;
        visit(c, [&](int, const int* o) {
          ++nn;
          for (int d = 0; d < 3; ++d) rmax = std::max(rmax, std::abs(o[d]));
        }, [&](int, const int*) { ++ni; });
        ncnt[c] = nn;
        icnt[c] = ni;
      }
      reach_t[t] = rmax;
    });
    C.nbr_off.assign(C.n + 1, 0);
    C.inter_off.assign(C.n + 1, 0);
    for (int c = 0; c < C.n; ++c) {
      C.nbr_off[c + 1] = C.nbr_off[c] + ncnt[c];
      C.inter_off[c + 1] = C.inter_off[c] + icnt[c];
    }
    C.nbr.resize(C.nbr_off[C.n]);
    C.inter_src.resize(C.inter_off[C.n]);
    std::vector<int32_t> ikey(C.inter_off[C.n]);
    parallel_chunks(C.n, nth, [&](int, int64_t lo, int64_t hi) {
      for (int64_t c = lo; c < hi; ++c) {
        int32_t pn = C.nbr_off[c], pi = C.inter_off[c];
        visit(c, [&](int c2, const int*) { C.nbr[pn++] = c2; },
              [&](int c2, const int* o) {
                C.inter_src[pi] = c2;
                ikey[pi++] = ((o[0] + W) * span + (o[1] + W)) * span + (o[2] + W);
              });
      }
    });
    // distinct offsets, numbered in increasing key order (independent of the
    // traversal and of the thread count)
    std::vector<int32_t> id((size_t)span * span * span, -1);
    for (int32_t k : ikey) id[k] = 0;
    int32_t nid = 0;
    for (size_t k = 0; k < id.size(); ++k)
      if (id[k] == 0) {
        id[k] = nid++;
        C.off_xyz.push_back((int)(k / ((size_t)span * span)) - W);
        C.off_xyz.push_back((int)((k / span) % span) - W);
        C.off_xyz.push_back((int)(k % span) - W);
      }
    C.inter_oid.resize(ikey.size());
    parallel_chunks((int64_t)ikey.size(), nth, [&](int, int64_t lo, int64_t hi) {
      for (int64_t k = lo; k < hi; ++k) C.inter_oid[k] = id[ikey[k]];
    });
    int newreach = 0;
    for (int v : reach_t) newreach = std::max(newreach, v);
    reach = newreach;
    if (!C.inter_src.empty() && out.lmin > L) out.lmin = l;
  }
  return 0;
}

}  // namespace fagbi
