// Host-side cluster tree construction (plain C++, built with FP contraction
// off so that cube indices, radii and separation tests are exactly the IEEE
// results of the written expressions).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace fagbi {

struct TreeLevel {
  int n = 0;
  double h = 0, rho = 0;
  std::vector<int32_t> idx;                 // 3n
  std::vector<int32_t> start, end;          // panel ranges (tree order)
  std::vector<int32_t> parent;              // n (-1 on level 0)
  std::vector<int32_t> child_start, child_end;
  std::vector<int32_t> nbr_off, nbr;
  std::vector<int32_t> inter_off, inter_src, inter_oid;
  std::vector<int32_t> off_xyz;             // distinct offsets idx_c - idx_c'
};

struct TreeOut {
  int L = 0, lmin = 0;
  double corner[3], side;
  std::vector<int32_t> perm;                // tree position -> input panel
  std::vector<TreeLevel> lev;
  // per panel, tree order
  std::vector<double> corners;              // 9N: u, v, w
  std::vector<double> normal, area;         // 3N, N
  std::vector<int32_t> tri;                 // 3N vertex ids
};

// Returns 0 or a negative fagbi error code with a message in `err`.
int build_tree_host(const double* verts, int64_t nv, const int32_t* tris, int64_t nt,
                    int leaf_size, double eta0, TreeOut& out, std::string& err);

}  // namespace fagbi
