// Internal state and device helpers of the fagbi library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/fagbi.h"
#include "fmath.h"

namespace fagbi {

constexpr int PMAX = 10;                       // highest supported expansion order
constexpr int TMAX = (PMAX + 1) * (PMAX + 2) * (PMAX + 3) / 6;   // 286 terms
constexpr double FOUR_PI = 12.566370614359172953850573533118;
constexpr double UNIT_KCAL = 4.0 * 3.14159265358979323846264338327950288 * 332.0716;

__host__ __device__ constexpr int nterms(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

int set_error(int code, const char* fmt, ...);

#define FAGBI_HIP(call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::fagbi::set_error(FAGBI_E_HIP, "%s failed: %s (%s:%d)", #call,         \
                                hipGetErrorString(e_), __FILE__, __LINE__);          \
  } while (0)

#define FAGBI_TRY(call)                  \
  do {                                   \
    int r_ = (call);                     \
    if (r_ < 0) return r_;               \
  } while (0)

// device allocation owned by the handle
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// device memory through a process-wide cache: freed blocks are kept per
// device and size class and handed out again (after a device
// synchronisation, so no kernel still uses them); the cache returns its
// blocks to HIP when it holds more than a cap or an allocation fails
int dev_alloc(void** p, size_t bytes);
void dev_free(void* p);

// scratch device memory owned by a scope (freed on destruction)
struct Tmp {
  void* p = nullptr;
  size_t bytes = 0;
  Tmp() = default;
  Tmp(const Tmp&) = delete;
  Tmp& operator=(const Tmp&) = delete;
  ~Tmp() { release(); }
  void release() {
    if (p) dev_free(p);
    p = nullptr;
    bytes = 0;
  }
  int alloc(size_t n);
  template <class T> T* as() const { return static_cast<T*>(p); }
};

struct Level {
  int n = 0;          // clusters on this level
  int order = 0;      // expansion order p_l
  int T = 0;          // terms of order p_l
  double h = 0, rho = 0;
  DBuf d_rho_c;                      // per-cluster radii (FAGBI_RADII_CLUSTER only)
  int64_t n_inter = 0;               // interaction pairs (c, c' in I(c))
  std::vector<int32_t> off_xyz;      // 3 * n_off distinct offsets (c - c')
  int n_off = 0;
  // device: cube indices [n][3], parent [n] (-1 on level 0), children on
  // level+1 [child_start, child_end), CSR interaction lists with offset ids
  DBuf d_idx, d_parent, d_child_start, d_child_end, d_inter_off, d_inter_src, d_inter_oid;
  // derivative tables per offset [n_off][T] as {G0, Gk} pairs (index 0); FP32
  // table of one offset of each opposite pair [n_half][T] (index 1) with the
  // map oid -> row | flip << 30
  DBuf d_F64[2], d_F32[2], d_oid_map;
  DBuf d_off, d_rows;   // offsets [n_off][3] and the half table's rows, for the table kernels
  int n_half = 0;
  // octant table (FP32, order 4): one row per class of offsets equal up to
  // the signs of their components, (|x|, |y|, |z|); rows8[k] = representative
  // oid | its signs << 29, oid_map8[oid] = row | signs << 29 (bit 29 + a: the
  // component a is negative)
  DBuf d_F32o, d_rows8, d_oid_map8;
  int n_oct = 0;
  DBuf d_M64[2], d_L64[2];           // moments / locals [n][T], channel 0 (G0), 1 (Gk)
  DBuf d_M32[2], d_L32[2];
  // slot tables (one slot per coupled pair of multi-indices) of the
  // translations that start on this level: MtL (|a|+|b| <= p_l), and for the
  // shifts to the children MtM (sorted by parent index a) and LtL (sorted by
  // child index b), with one coefficient row per child octant
  int m2l_nslot = 0, up_nslot = 0, dn_nslot = 0;
  DBuf d_m2l_slot, d_m2l_aoff, d_m2l_c64, d_m2l_c32;
  DBuf d_up_slot, d_up_aoff, d_up_c64, d_up_c32;
  DBuf d_dn_slot, d_dn_boff, d_dn_c64, d_dn_c32;
  // MtL with source reuse: targets in tiles of consecutive clusters; per tile
  // its distinct sources [tile_off[t], tile_off[t + 1]) of tile_src (sorted),
  // per interaction pair the packed index (slot of its source in the tile |
  // half-table row << 12 | flip << 31); n_tile = 0 when not set up
  DBuf d_tile_t0, d_tile_off, d_tile_src, d_pack;   // tile t: targets [tile_t0[t], tile_t0[t + 1])
  int n_tile = 0, tile_umax = 0;
};

}  // namespace fagbi

struct fagbi_handle {
  fagbi_params prm;
  int device = 0;
  // ---- mesh / tree (host copies) ----
  int64_t N = 0, nv = 0;
  int L = -1, lmin = 0;
  double corner[3] = {0, 0, 0}, side = 0;
  std::vector<fagbi::Level> lev;      // 0..L
  // leaf-level near field layout (panels per leaf; device arrays below)
  std::vector<int32_t> leaf_cnt;
  int64_t n_src = 0, n_ent = 0;
  int max_leaf = 0;
  bool tree_ready = false, near_ready = false;
  int64_t singular_count[4] = {0, 0, 0, 0};
  // ---- device buffers ----
  // tree position -> caller panel index; per panel in tree order: corners
  // [9], unit normal [3], area, vertex ids [3]; leaf of each panel
  fagbi::DBuf d_perm, d_pv, d_pn, d_pa, d_ptri, d_leaf_of;
  fagbi::DBuf d_pc;                   // per panel: centroid, sqrt(area)
  fagbi::DBuf d_xt;                   // matvec input in tree order [2N]
  // treecode work lists, grown as needed and kept: (charge, cluster) pairs
  // of a level [2 x 2], decisions, child counts, their scans, scan scratch,
  // accepted pair list
  fagbi::Tmp tc_ws[10];
  fagbi::DBuf d_fmm_pool;             // one allocation behind all far-field tables and expansions
  fagbi::DBuf d_leaf_start, d_leaf_cnt, d_src_off, d_ent_off, d_src_tree, d_self_col;
  fagbi::DBuf d_lnbr_off, d_lnbr, d_lnbr_col;  // leaf neighbour lists, column of each block
  fagbi::DBuf d_E64, d_E32;           // near-field entries (double4 / float4)
  fagbi::DBuf d_ms64, d_md64, d_ms32, d_md32;  // panel moments [N][T(p_L)]
  fagbi::DBuf d_mi;                   // multi-index table [TMAX][3]
  fagbi::DBuf d_xdst;                 // matrix-core MtL: X entry -> local term
  fagbi::DBuf d_mtl_ctr;              // MtL tile claim counters, 16 ints per level (zero between launches)
  fagbi::DBuf d_lu, d_lu_off, d_piv, d_diag;    // preconditioner (block inverses, FP64)
  fagbi::DBuf d_lu32;                          // FP32 copy for the mixed path's inner solves
  fagbi::DBuf d_grp_leaf, d_grp_panel;         // its blocks: leaf and panel ranges
  int n_groups = 0;
  fagbi::DBuf d_gl;                   // Gauss-Legendre nodes/weights on [0,1]
  fagbi::DBuf d_work;                 // scratch for reductions
  // Krylov workspace
  fagbi::DBuf d_V, d_Z, d_w, d_r, d_b, d_x0, d_dots, d_t1, d_t2;
  int krylov_m = 0;
  // near-singular worklists (identical, edge, vertex, close), kept after
  // assembly for the surrogate's data generation
  fagbi::DBuf d_wl[4];
  int64_t wl_n[4] = {0, 0, 0, 0};
  bool precond_ready = false;
  // surrogate network: parameters, Adam moments, normalisation, calibration
  bool mlp_ready = false;
  int64_t mlp_gated_pairs = 0;
  fagbi::DBuf d_mlp_theta, d_mlp_m, d_mlp_v, d_mlp_norm;
  fagbi::DBuf d_mlp_skip[4];
  // hat-function basis (FAGBI_BASIS_S1): elements are the panel corners,
  // e = 3 i + a for tree-order panel i; the near field's element layout
  // (leaf ranges, source lists, entry offsets of the 3 x 3 blocks), the
  // identity map of the element outputs, the leaf of each element, the
  // elements of each vertex (CSR, ascending), the element results [2][3N]
  fagbi::DBuf d_s1_leaf_start, d_s1_leaf_cnt, d_s1_iota, d_s1_leaf_of, d_vx_off, d_vx_el, d_ye;
  // its near field by vertex pairs: per leaf the distinct vertices of its
  // panels (rows) and of its source panels (columns, each with one of its
  // corners, whose tree-order input is the vertex's value), the entry blocks
  // [rows][columns], the vertex and leaf of each row, the rows of each vertex
  // (CSR); counts of rows and entries
  fagbi::DBuf d_vb_row_start, d_vb_row_cnt, d_vb_col_off, d_vb_ent_off, d_vb_col_elem, d_vb_col_vert,
      d_vb_row_vert, d_vb_row_leaf, d_vx_poff, d_vx_pr;
  int64_t n_vb_rows = 0, n_vb_ent = 0;
  std::vector<float> mlp_blob;        // parameters | normalisation | calibration
  // FP32 leaf-level MtL by the source-reuse tile kernel (when its tables fit);
  // FAGBI_M2L_TILES=0 in the environment selects the per-pair LDS-table kernel
  bool m2l_tiles = true;
  bool m2l_mfma = false;               // leaf-level FP32 MtL on the matrix cores
  // per-phase profiling
  bool profiling = false;
  // matvec phase events: 5 start; 0, 1 around the near-field SpMV (on its
  // own stream when the far field runs beside it); 6 start of the far field,
  // 2 upward pass, 3 MtL, 4 downward pass (after joining the near field);
  // 7, 8 around the leaf level's MtL kernel on the stream it runs on
  hipEvent_t ev[9] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  hipStream_t s_near = nullptr;                 // default priority
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipStream_t s_m2l = nullptr;                  // MtL of the two finest levels, default priority
  hipEvent_t ev_up0 = nullptr, ev_up1 = nullptr, ev_m2l = nullptr;
  hipEvent_t ev_upd = nullptr;                  // upward pass complete (coarse MtL on the near stream)
  double* hpin = nullptr;                       // pinned host copy of a GMRES Hessenberg column
  size_t hpin_n = 0;
  hipEvent_t ev_col = nullptr;
  fagbi_profile prof{};
  std::vector<fagbi::DBuf*> owned;
  int alloc(fagbi::DBuf& b, size_t bytes);
  int upload(fagbi::DBuf& b, const void* host, size_t bytes);
  void free_all();
  bool hat() const { return prm.basis == FAGBI_BASIS_S1; }
  // unknowns per channel: panels (box functions) or vertices (hat functions)
  int64_t n_unk() const { return hat() ? nv : N; }
};

namespace fagbi {
// wall clock of one setup stage into *out while profiling is on (the stream
// is synchronised at both ends, so only then)
struct StageTimer {
  fagbi_handle* h;
  hipStream_t s;
  double* out;
  std::chrono::steady_clock::time_point t0;
  StageTimer(fagbi_handle* h_, hipStream_t s_, double* out_) : h(h_), s(s_), out(out_) {
    if (h->profiling) {
      (void)hipStreamSynchronize(s);
      t0 = std::chrono::steady_clock::now();
    }
  }
  void stop() {
    if (!h->profiling || !out) return;
    (void)hipStreamSynchronize(s);
    *out = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    out = nullptr;
  }
  ~StageTimer() { stop(); }
};

// The rows the near and far field run over, in tree order: the panels (box
// functions) or the panel corners (hat functions).  The matvec gathers
// xt[e] = (x[in_idx[e]], x[in_stride + in_idx[e]]), runs the SpMV, P2M and
// LtP over the rows (row results at y[out_idx[e]] and y[n + out_idx[e]]) and,
// with a gather list, sums the rows of each output into the caller's y.
// The near field may run over rows of its own (the hat functions' vertex
// pairs): its leaf ranges, source lists (indices into xt), entry offsets and
// row outputs y_near[out_near[r]], y_near[n_near + ...]; zero_y clears the far
// field's rows first (the SpMV then does not write them).
struct ElemView {
  int64_t n = 0;
  const int32_t *leaf_start = nullptr, *leaf_cnt = nullptr, *leaf_of = nullptr;
  const int32_t *in_idx = nullptr, *out_idx = nullptr;
  int64_t in_stride = 0;
  double* xt = nullptr;        // [n] (phi, dphi) pairs
  double* y = nullptr;         // row results [2n]; nullptr: the caller's y
  int64_t n_near = 0;
  const int32_t *near_start = nullptr, *near_cnt = nullptr, *near_src = nullptr, *out_near = nullptr;
  const int64_t *near_src_off = nullptr, *near_ent_off = nullptr;
  double* y_near = nullptr;    // near rows [2 n_near]; nullptr: as y
  bool zero_y = false;
  bool gather = false;         // sum the rows into the vertices (hat functions)
};
ElemView box_view(fagbi_handle* h);
ElemView hat_view(fagbi_handle* h);

// stages implemented in the .hip files
int build_tree(fagbi_handle* h, const double* verts, int64_t nv, const int32_t* tris, int64_t nt);
int assemble_nearfield(fagbi_handle* h, hipStream_t s);
int fmm_setup(fagbi_handle* h, hipStream_t s);
int matvec(fagbi_handle* h, const double* x, double* y, int precision, int parts,
           hipStream_t s);
int precond_setup(fagbi_handle* h, hipStream_t s);
int run_singular(fagbi_handle* h, int cls_index, const uint8_t* skip, double* raw, hipStream_t s);
int mlp_assembly_stage(fagbi_handle* h, hipStream_t s);
int precond_apply(fagbi_handle* h, const double* z, double* y, hipStream_t s, bool f32 = false);
int rhs(fagbi_handle* h, const double* xq, const double* q, int64_t nc, double* b,
        hipStream_t s);
int energy_scratch_init(int device);
int energy_noalloc(fagbi_handle* h, const double* x, const double* chg, int64_t nc, double* E, hipStream_t s);
int energy(fagbi_handle* h, const double* x, const double* xq, const double* q,
           int64_t nc, double* E, hipStream_t s);
int energy_treecode(fagbi_handle* h, const double* x, const double* xq, const double* q, int64_t nc,
                    double theta, int p_max, double* E, hipStream_t s);
int treecode_potentials(fagbi_handle* h, const double* x, const double* chg, int64_t nc, double theta,
                        int p_max, double* qv, hipStream_t s);
int rhs_treecode(fagbi_handle* h, const double* xq, const double* q, int64_t nc, double theta, int p_max,
                 double* b, hipStream_t s);
int treecode_rhs(fagbi_handle* h, const double* chg, int64_t nc, double theta, int p_max, double* b,
                 hipStream_t s);
int solve(fagbi_handle* h, const double* xq, const double* q, int64_t nc, double* x,
          fagbi_solve_info* info, hipStream_t s);
void gauss_legendre01(int n, double* x, double* w);
// hat-function basis: near field (entries, element layout, vertex lists),
// diagonal preconditioner, and the element-to-vertex sum
int hat_assemble(fagbi_handle* h, hipStream_t s);
int hat_diag_setup(fagbi_handle* h, hipStream_t s);
int hat_gather(fagbi_handle* h, const double* rows, const double* near_rows, double* y, hipStream_t s);

// The quadrature table of the singular and close rules (device d_gl):
// [0, 16) Gauss-Legendre nodes on [0, 1], [16, 32) weights, then one radial
// table per touching class (identical, edge, vertex; RAD_STRIDE doubles each):
// the xi-rule of that class's transform applied to the kernels' functions of
// u = kappa * xi * rho as power series in v = kappa * rho,
//   [4 k + f], k = 0..RAD_KMAX, f = T0 (em1), T2 (e^-u (1 + u)), T5a (c1), T5b (c2)
//   [RAD_T1]   the Laplace double-layer factor (xi-rule of the Jacobian / xi^2)
//   [RAD_VK + K] the largest v for which the terms above degree K stay below
//              2^-56 of each series' leading term
constexpr int RAD_KMAX = 24;
constexpr int RAD_T1 = 4 * (RAD_KMAX + 1);
constexpr int RAD_VK = RAD_T1 + 1;
constexpr int RAD_STRIDE = 128;
constexpr int QT_RAD = 32;
// then the per-ray data of the vertex rule ([2 n^3][6]: s_a, s_a t1, s_b,
// s_b t2, weight, 0) and of the edge rule ([4 n^2][4]: z1, x2, y2, weight),
// the coordinates of a ray divided by its radial coordinate
constexpr int QT_RAY = QT_RAD + 3 * RAD_STRIDE;
__host__ __device__ inline int qt_edge_rays(int n) { return QT_RAY + 12 * n * n * n; }
// and the outer points of the close rule ([n^3][4]: s1, s1 t1, s2, weight
// without the areas)
__host__ __device__ inline int qt_close_pts(int n) { return qt_edge_rays(n) + 16 * n * n; }
__host__ __device__ inline int qt_size(int n) { return qt_close_pts(n) + 4 * n * n * n; }
void quad_table(int n, double* t);   // t: qt_size(n) doubles
}  // namespace fagbi

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
namespace fagbi {

// the three quadrature points of panel i (barycentric (2/3, 1/6, 1/6) and
// permutations, weight A/3 each) from its corners pv[9 i ..]
__device__ inline void quad_points(const double* __restrict__ pv, int64_t i, double* qp) {
  const double* v = pv + 9 * i;
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d)
      qp[3 * k + d] = (2.0 / 3.0) * v[3 * k + d] + (1.0 / 6.0) * (v[3 * ((k + 1) % 3) + d] + v[3 * ((k + 2) % 3) + d]);
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// the six pair integrands at separation r = x - y with normals nx (target),
// ny (source): G0-Gk, dG0/dny, dGk/dny, dG0/dnx, dGk/dnx, d2(Gk-G0)/dnx dny
// the six kernels from r^2, r.n_x, r.n_y and n_x.n_y (the innermost loops of
// the cubature, where r = R0 + t R1, form these as polynomials in t)
__device__ inline void kernel6s(double r2, double rnx, double rny, double nn, double kappa, double* k) {
  const double ir = inv_sqrt(r2);
  const double u = kappa * (r2 * ir);
  double E, em1;
  exp_expm1(-u, E, em1);
  const double i4pr = ir * (1.0 / FOUR_PI);
  const double ir2 = ir * ir;
  const double i4pr3 = i4pr * ir2;
  const double e1u = E * (1.0 + u);
  k[0] = -em1 * i4pr;
  k[1] = rny * i4pr3;
  k[2] = e1u * rny * i4pr3;
  k[3] = -rnx * i4pr3;
  k[4] = -e1u * rnx * i4pr3;
  const double c1 = em1 + u * E;
  const double c2 = 3.0 * em1 + 3.0 * u * E + u * u * E;
  k[5] = (c1 * nn - c2 * rnx * rny * ir2) * i4pr3;
}

// r = R0 + t R1 on the innermost cubature axis: r^2 = a + t (b + t c),
// r.n_x = p0 + t p1, r.n_y = q0 + t q1
struct LinSep {
  double a, b, c, p0, p1, q0, q1;
};
__device__ inline LinSep lin_sep(const double* R0, const double* R1, const double* nx, const double* ny) {
  LinSep L;
  L.a = R0[0] * R0[0] + R0[1] * R0[1] + R0[2] * R0[2];
  L.b = 2.0 * (R0[0] * R1[0] + R0[1] * R1[1] + R0[2] * R1[2]);
  L.c = R1[0] * R1[0] + R1[1] * R1[1] + R1[2] * R1[2];
  L.p0 = R0[0] * nx[0] + R0[1] * nx[1] + R0[2] * nx[2];
  L.p1 = R1[0] * nx[0] + R1[1] * nx[1] + R1[2] * nx[2];
  L.q0 = R0[0] * ny[0] + R0[1] * ny[1] + R0[2] * ny[2];
  L.q1 = R1[0] * ny[0] + R1[1] * ny[1] + R1[2] * ny[2];
  return L;
}

__device__ inline void kernel6(double rx, double ry, double rz, const double* nx,
                               const double* ny, double kappa, double* k) {
  const double r2 = rx * rx + ry * ry + rz * rz;
  const double ir = inv_sqrt(r2);
  const double u = kappa * (r2 * ir);
  double E, em1;
  exp_expm1(-u, E, em1);
  const double i4pr = ir * (1.0 / FOUR_PI);
  const double ir2 = ir * ir;
  const double i4pr3 = i4pr * ir2;
  const double rny = rx * ny[0] + ry * ny[1] + rz * ny[2];
  const double rnx = rx * nx[0] + ry * nx[1] + rz * nx[2];
  const double nn = nx[0] * ny[0] + nx[1] * ny[1] + nx[2] * ny[2];
  const double e1u = E * (1.0 + u);
  k[0] = -em1 * i4pr;
  k[1] = rny * i4pr3;
  k[2] = e1u * rny * i4pr3;
  k[3] = -rnx * i4pr3;
  k[4] = -e1u * rnx * i4pr3;
  const double c1 = em1 + u * E;
  const double c2 = 3.0 * em1 + 3.0 * u * E + u * u * E;
  k[5] = (c1 * nn - c2 * rnx * rny * ir2) * i4pr3;
}

}  // namespace fagbi
