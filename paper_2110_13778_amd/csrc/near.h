// Near-field pair machinery shared by the assembly and the surrogate network
// (internal): pair classes, per-pair arguments, classification, the 3x3
// regular rule and the mapping of the six integrals to operator entries.
#pragma once
#include "internal.h"

namespace fagbi {

enum { C_REGULAR = 0, C_IDENT = 1, C_EDGE = 2, C_VERTEX = 3, C_CLOSE = 4 };

struct Item {
  int32_t i, j;       // tree-order panels (target, source)
  int64_t ent;        // entry index
};

struct NearArgs {
  const double* pv;     // corners [N][9]
  const double* pn;     // normals [N][3]
  const double* pa;     // areas [N]
  const double4* pc;    // centroid and sqrt(area) [N]
  const int32_t* ptri;  // vertex ids [N][3]
  const int32_t* leaf_start;
  const int32_t* leaf_cnt;
  const int64_t* src_off;
  const int64_t* ent_off;
  const int32_t* src_tree;
  const int32_t* perm;       // tree position -> caller index
  const int32_t* leaf_of;
  const int32_t* lnbr_off;   // leaf neighbour lists and the column where
  const int32_t* lnbr;       // each neighbour's panels start in the leaf's
  const int32_t* lnbr_col;   // source list
  double kappa, eps, near_ratio;
};

__device__ inline int classify(const NearArgs& a, int i, int j) {
  if (i == j) return C_IDENT;
  int shared = 0;
  for (int p = 0; p < 3; ++p) {
    const int vi = a.ptri[3 * i + p];
    shared += (vi == a.ptri[3 * j]) + (vi == a.ptri[3 * j + 1]) + (vi == a.ptri[3 * j + 2]);
  }
  if (shared == 2) return C_EDGE;
  if (shared == 1) return C_VERTEX;
  // centroid distance, evaluated without contraction so the test is the
  // IEEE result of the written expression
  const double4 pi = a.pc[i], pj = a.pc[j];
  const double s0 = __dadd_rn(pi.x, -pj.x), s1 = __dadd_rn(pi.y, -pj.y), s2 = __dadd_rn(pi.z, -pj.z);
  const double dist = sqrt(__dadd_rn(__dadd_rn(__dmul_rn(s0, s0), __dmul_rn(s1, s1)), __dmul_rn(s2, s2)));
  return dist < __dmul_rn(a.near_ratio, fmax(pi.w, pj.w)) ? C_CLOSE : C_REGULAR;
}

__device__ inline void regular_pair(const NearArgs& a, int i, int j, double* I) {
  double qi[9], qj[9];
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) {
      qi[3 * k + d] = (2.0 / 3.0) * a.pv[9 * i + 3 * k + d] +
                      (1.0 / 6.0) * (a.pv[9 * i + 3 * ((k + 1) % 3) + d] + a.pv[9 * i + 3 * ((k + 2) % 3) + d]);
      qj[3 * k + d] = (2.0 / 3.0) * a.pv[9 * j + 3 * k + d] +
                      (1.0 / 6.0) * (a.pv[9 * j + 3 * ((k + 1) % 3) + d] + a.pv[9 * j + 3 * ((k + 2) % 3) + d]);
    }
  const double* ni = a.pn + 3 * i;
  const double* nj = a.pn + 3 * j;
  for (int m = 0; m < 6; ++m) I[m] = 0;
  double k6[6];
  for (int p = 0; p < 3; ++p)
    for (int q = 0; q < 3; ++q) {
      kernel6(qi[3 * p] - qj[3 * q], qi[3 * p + 1] - qj[3 * q + 1], qi[3 * p + 2] - qj[3 * q + 2], ni, nj,
              a.kappa, k6);
      for (int m = 0; m < 6; ++m) I[m] += k6[m];
    }
  const double w = (a.pa[i] / 3.0) * (a.pa[j] / 3.0);
  for (int m = 0; m < 6; ++m) I[m] *= w;
}

__device__ inline double4 combine(const double* I, double eps) {
  return make_double4(-(eps * I[2] - I[1]), -I[0], -I[5], -(I[3] - I[4] / eps));
}

// write the entry of (target i, source j) and, for mirrored classes, of
// (target j, source i): I1, I6 symmetric, I2 <-> I4, I3 <-> I5
__device__ inline void write_pair(const NearArgs& a, int cls, int i, int j, int64_t ent_ij, const double* I,
                                  double4* ent) {
  double4 v = combine(I, a.eps);
  if (cls == C_IDENT) {
    v.x += 0.5 * (1.0 + a.eps) * a.pa[i];
    v.w += 0.5 * (1.0 + 1.0 / a.eps) * a.pa[i];
  }
  ent[ent_ij] = v;
  if (cls == C_IDENT) return;
  const int ci = a.leaf_of[i], cj = a.leaf_of[j];
  int col = -1;
  for (int q = a.lnbr_off[cj]; q < a.lnbr_off[cj + 1]; ++q)
    if (a.lnbr[q] == ci) col = a.lnbr_col[q] + (i - a.leaf_start[ci]);
  if (col >= 0) {
    const int S = (int)(a.src_off[cj + 1] - a.src_off[cj]);
    const double It[6] = {I[0], I[3], I[4], I[1], I[2], I[5]};
    ent[a.ent_off[cj] + (int64_t)(j - a.leaf_start[cj]) * S + col] = combine(It, a.eps);
  }
}

NearArgs near_args(fagbi_handle* h);

}  // namespace fagbi
