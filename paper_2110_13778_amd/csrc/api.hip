// C ABI entry points, handle lifetime, error reporting and tree upload.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <unordered_map>
#include <utility>
#include <vector>

#include "internal.h"

namespace fagbi {

static thread_local std::string g_err;

int set_error(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

// Gauss-Legendre rule on [0,1] by Newton iteration on P_n from the Chebyshev
// initial guesses (three-term recurrence for P_n and P_n').
void gauss_legendre01(int n, double* x, double* w) {
  const double pi = 3.14159265358979323846264338327950288;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 1;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      dp = n * (z * p1 - p0) / (z * z - 1);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      dp = n * (z * p1 - p0) / (z * z - 1);
    }
    x[n - 1 - i] = 0.5 * (z + 1.0);
    w[n - 1 - i] = 1.0 / ((1 - z * z) * dp * dp);   // (2/((1-z^2)P'^2)) / 2
  }
}

// Radial table of one touching class.  Its transform writes the separation as
// r = xi * rho_hat with Jacobian factor g(xi) (identical: (1 - xi)^2 xi / 2,
// edge: (1 - xi) xi^2, vertex: xi^3), so with v = kappa * |rho_hat| the
// xi-rule of each kernel is a fixed power series in v:
//   T0  = sum_i w_i g(x_i) em1(v x_i) / x_i      em1(u) = e^-u - 1
//   T1  = sum_i w_i g(x_i) / x_i^2
//   T2  = sum_i w_i g(x_i) e1u(v x_i) / x_i^2     e1u(u) = e^-u (1 + u)
//   T5a = sum_i w_i g(x_i) c1(v x_i) / x_i^3      c1 = e1u - 1
//   T5b = sum_i w_i g(x_i) c2(v x_i) / x_i^3      c2 = 3 c1 + u^2 e^-u
// with Taylor coefficients (-1)^k / k!, (-1)^k (1 - k) / k!, and
// (-1)^k (k - 1)(k - 3) / k! of em1, e1u (and c1 from k = 2) and c2, times
// the moments G_j = sum_i w_i g(x_i) x_i^j.
static void radial_table(int n, const double* x, const double* w, int cls, double* t) {
  constexpr int KX = RAD_KMAX + 40;
  std::vector<double> G(KX + 3);   // G[j + 2], j = -2 .. KX
  for (int j = -2; j <= KX; ++j) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      const double xi = x[i];
      const double g = cls == 0 ? 0.5 * (1.0 - xi) * (1.0 - xi) * xi
                     : cls == 1 ? (1.0 - xi) * xi * xi : xi * xi * xi;
      s += w[i] * g * std::pow(xi, j);
    }
    G[j + 2] = s;
  }
  std::vector<double> c(4 * (KX + 1), 0.0);
  double fact = 1.0;
  for (int k = 0; k <= KX; ++k) {
    if (k > 0) fact *= k;
    const double sg = (k & 1) ? -1.0 : 1.0;
    if (k >= 1) c[4 * k] = sg / fact * G[k + 1];
    c[4 * k + 1] = sg * (1.0 - k) / fact * G[k];
    if (k >= 2) {
      c[4 * k + 2] = sg * (1.0 - k) / fact * G[k - 1];
      c[4 * k + 3] = sg * (k - 1.0) * (k - 3.0) / fact * G[k - 1];
    }
  }
  for (int k = 0; k <= RAD_KMAX; ++k)
    for (int f = 0; f < 4; ++f) t[4 * k + f] = c[4 * k + f];
  t[RAD_T1] = G[0];
  // truncation: the largest v at which the tail above degree K is <= 2^-56
  // of the leading term of every series (leading degrees 1, 0, 2, 2)
  const int lead[4] = {1, 0, 2, 2};
  auto ratio = [&](int K, double v) {
    double r = 0.0;
    for (int f = 0; f < 4; ++f) {
      double tail = 0.0;
      for (int k = KX; k > K; --k) tail = tail * v + std::fabs(c[4 * k + f]);
      tail *= std::pow(v, K + 1 - lead[f]);
      r = std::max(r, tail / std::fabs(c[4 * lead[f] + f]));
    }
    return r;
  };
  for (int K = 0; K <= RAD_KMAX; ++K) {
    double lo = 0.0, hi = 16.0;
    if (K >= 2)
      for (int it = 0; it < 48; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (ratio(K, mid) <= 0x1p-56) lo = mid; else hi = mid;
      }
    t[RAD_VK + K] = lo;
  }
}

// the table depends on n only: built once per process and order
void quad_table(int n, double* t) {
  static std::mutex mu;
  static std::map<int, std::vector<double>> cache;
  std::lock_guard<std::mutex> lock(mu);
  std::vector<double>& c = cache[n];
  if (c.empty()) {
    c.assign(qt_size(n), 0.0);
    const double *x = c.data(), *w = c.data() + 16;
    gauss_legendre01(n, c.data(), c.data() + 16);
    for (int cls = 0; cls < 3; ++cls)
      radial_table(n, x, w, cls, c.data() + QT_RAD + cls * RAD_STRIDE);
    // vertex rays (piece, eta, t1, t2): R / xi = s_a (A0 + t1 A1) - s_b (B0 + t2 B1)
    const int n2 = n * n, n3 = n2 * n;
    for (int it = 0; it < 2 * n3; ++it) {
      const int piece = it / n3, rem = it - piece * n3;
      const int ib = rem / n2, ic = (rem / n) % n, id = rem % n;
      const double eta = x[ib], sa = piece == 0 ? 1.0 : eta, sb = piece == 0 ? eta : 1.0;
      double* r = c.data() + QT_RAY + 6 * it;
      r[0] = sa;
      r[1] = sa * x[ic];
      r[2] = sb;
      r[3] = sb * x[id];
      r[4] = w[ib] * w[ic] * w[id] * eta;
    }
    // edge rays (piece, w1, w2): R / xi = -z1 e + x2 a - y2 b
    for (int it = 0; it < 4 * n2; ++it) {
      const int piece = it / n2, rem = it - piece * n2;
      const int ib = rem / n, ic = rem - ib * n;
      const double w1 = x[ib], w2 = x[ic];
      double z, xx, y, W = w[ib] * w[ic];
      if (piece == 0) {
        z = w1; xx = 1.0 - w1; y = w2;
      } else if (piece == 1) {
        z = w1 * (1.0 - w2); xx = w1 * w2; y = 1.0; W *= w1;
      } else if (piece == 2) {
        z = -w1 * (1.0 - w2); xx = 1.0; y = w1 * w2; W *= w1;
      } else {
        z = -w1; xx = w2; y = 1.0 - w1;
      }
      double* r = c.data() + qt_edge_rays(n) + 4 * it;
      r[0] = z;
      r[1] = xx;
      r[2] = y;
      r[3] = W;
    }
    // close rule, outer points (s1, t1, s2) of the Duffy-collapsed product
    for (int it = 0; it < n3; ++it) {
      const int ia = it / n2, ib = (it / n) % n, ic = it % n;
      double* r = c.data() + qt_close_pts(n) + 4 * it;
      r[0] = x[ia];
      r[1] = x[ia] * x[ib];
      r[2] = x[ic];
      r[3] = x[ia] * w[ia] * w[ib] * x[ic] * w[ic];
    }
  }
  std::copy(c.begin(), c.end(), t);
}

}  // namespace fagbi

using namespace fagbi;

namespace fagbi {
namespace {

// size class: multiples of 2 MiB from 2 MiB on, powers of two (>= 256 B) below
size_t size_class(size_t n) {
  constexpr size_t big = (size_t)2 << 20;
  if (n >= big) return (n + big - 1) / big * big;
  size_t c = 256;
  while (c < n) c <<= 1;
  return c;
}

struct DevCache {
  std::mutex mu;
  std::map<std::pair<int, size_t>, std::vector<void*>> free_blocks;   // (device, class) -> blocks
  std::unordered_map<void*, std::pair<int, size_t>> live;             // block -> (device, class)
  size_t cached = 0;
  // caller holds mu; returns every cached block of this device to HIP
  void trim(int dev) {
    for (auto it = free_blocks.begin(); it != free_blocks.end();) {
      if (it->first.first != dev) {
        ++it;
        continue;
      }
      for (void* b : it->second) {
        (void)hipFree(b);
        cached -= it->first.second;
      }
      it = free_blocks.erase(it);
    }
  }
};

// never destroyed: blocks still cached at exit go back with the process
DevCache& cache() {
  static DevCache* c = new DevCache();
  return *c;
}

constexpr size_t kCacheCap = (size_t)64 << 30;   // cached bytes kept, at most

}  // namespace

int dev_alloc(void** p, size_t n) {
  *p = nullptr;
  if (n == 0) return 0;
  int dev = 0;
  FAGBI_HIP(hipGetDevice(&dev));
  const size_t c = size_class(n);
  DevCache& C = cache();
  std::lock_guard<std::mutex> lock(C.mu);
  auto it = C.free_blocks.find({dev, c});
  if (it != C.free_blocks.end() && !it->second.empty()) {
    FAGBI_HIP(hipDeviceSynchronize());   // every earlier use of the block has finished
    *p = it->second.back();
    it->second.pop_back();
    C.cached -= c;
    C.live[*p] = {dev, c};
    return 0;
  }
  hipError_t e = hipMalloc(p, c);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    FAGBI_HIP(hipDeviceSynchronize());
    C.trim(dev);
    e = hipMalloc(p, c);
  }
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return set_error(FAGBI_E_OOM, "device allocation of %zu bytes failed: %s", n, hipGetErrorString(e));
  }
  C.live[*p] = {dev, c};
  return 0;
}

void dev_free(void* p) {
  if (!p) return;
  DevCache& C = cache();
  std::lock_guard<std::mutex> lock(C.mu);
  auto it = C.live.find(p);
  if (it == C.live.end()) return;
  const auto key = it->second;
  C.live.erase(it);
  C.free_blocks[key].push_back(p);
  C.cached += key.second;
  if (C.cached > kCacheCap) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(key.first);
    (void)hipDeviceSynchronize();
    C.trim(key.first);
    (void)hipSetDevice(cur);
  }
}

}  // namespace fagbi

int Tmp::alloc(size_t n) {
  release();
  if (n == 0) return 0;
  FAGBI_TRY(dev_alloc(&p, n));
  bytes = n;
  return 0;
}

// (re)allocate a handle-owned buffer; every DBuf passed here is a member of
// the handle (or of one of its levels), registered once for free_all()
int fagbi_handle::alloc(DBuf& b, size_t bytes) {
  if (b.p) {
    dev_free(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  bool known = false;
  for (DBuf* o : owned) known |= (o == &b);
  if (!known) owned.push_back(&b);
  if (bytes == 0) return 0;
  FAGBI_TRY(dev_alloc(&b.p, bytes));
  b.bytes = bytes;
  return 0;
}

int fagbi_handle::upload(DBuf& b, const void* host, size_t bytes) {
  FAGBI_TRY(alloc(b, bytes));
  if (bytes) FAGBI_HIP(hipMemcpy(b.p, host, bytes, hipMemcpyHostToDevice));
  return 0;
}

void fagbi_handle::free_all() {
  for (DBuf* b : owned) {
    if (b->p) dev_free(b->p);
    b->p = nullptr;
    b->bytes = 0;
  }
  owned.clear();
}

extern "C" {

const char* fagbi_last_error(void) { return g_err.c_str(); }

int fagbi_default_params(fagbi_params* p) {
  if (!p) return set_error(FAGBI_E_ARG, "null params");
  memset(p, 0, sizeof *p);
  p->eps_in = 1.0;
  p->eps_out = 80.0;
  p->kappa = 0.1257;
  p->eta0 = 0.8;
  p->leaf_size = 32;
  p->p_leaf = 4;
  p->adaptive = 0;
  p->p_max = 8;
  p->quad_duffy = 7;
  p->near_ratio = 2.0;
  p->precision = FAGBI_FP64;
  p->precond = FAGBI_PRECOND_BLOCK;
  p->tol = 1e-6;
  p->max_iter = 200;
  p->max_outer = 5;
  p->inner_tol = 5e-7;
  p->mlp_mode = FAGBI_MLP_OFF;
  p->mlp_gate_tol = 1e-3;
  p->rhs_pmax = 8;
  return 0;
}

static int check_params(const fagbi_params* p) {
  if (!(p->eps_in > 0) || !(p->eps_out > 0) || !(p->kappa >= 0))
    return set_error(FAGBI_E_ARG, "eps_in, eps_out must be > 0 and kappa >= 0");
  if (!(p->eta0 >= 0) || p->leaf_size < 1)
    return set_error(FAGBI_E_ARG, "eta0 must be >= 0 and leaf_size >= 1");
  if (p->leaf_size > 32)
    return set_error(FAGBI_E_ARG, "leaf_size must be <= 32 (preconditioner blocks <= 64)");
  if (p->p_leaf < 0 || p->p_max < p->p_leaf || p->p_max > 8)
    return set_error(FAGBI_E_ARG, "need 0 <= p_leaf <= p_max <= 8");
  if (p->quad_duffy < 1 || p->quad_duffy > 16)
    return set_error(FAGBI_E_ARG, "quad_duffy must be in [1, 16]");
  if (!(p->near_ratio >= 0)) return set_error(FAGBI_E_ARG, "near_ratio must be >= 0");
  if (p->precision != FAGBI_FP64 && p->precision != FAGBI_MIXED)
    return set_error(FAGBI_E_ARG, "precision must be FAGBI_FP64 or FAGBI_MIXED");
  if (p->precond < 0 || p->precond > 3) return set_error(FAGBI_E_ARG, "bad precond");
  if (!(p->tol > 0) || p->max_iter < 1 || p->max_iter > 2000 || p->max_outer < 1 ||
      !(p->inner_tol > 0))
    return set_error(FAGBI_E_ARG, "bad solver tolerances/iteration limits");
  if (p->mlp_mode < 0 || p->mlp_mode > 2) return set_error(FAGBI_E_ARG, "bad mlp_mode");
  if (!(p->rhs_theta >= 0 && p->rhs_theta < 1)) return set_error(FAGBI_E_ARG, "rhs_theta must be in [0, 1)");
  if (p->rhs_pmax < 0) return set_error(FAGBI_E_ARG, "rhs_pmax must be >= 0");
  if (p->radii != FAGBI_RADII_LEVEL && p->radii != FAGBI_RADII_CLUSTER)
    return set_error(FAGBI_E_ARG, "radii must be FAGBI_RADII_LEVEL or FAGBI_RADII_CLUSTER");
  if (p->basis != FAGBI_BASIS_S0 && p->basis != FAGBI_BASIS_S1)
    return set_error(FAGBI_E_ARG, "basis must be FAGBI_BASIS_S0 or FAGBI_BASIS_S1");
  if (p->basis == FAGBI_BASIS_S1) {
    if (p->mlp_mode != FAGBI_MLP_OFF) return set_error(FAGBI_E_ARG, "the hat-function basis needs mlp_mode OFF");
    if (p->precond != FAGBI_PRECOND_NONE && p->precond != FAGBI_PRECOND_DIAG)
      return set_error(FAGBI_E_ARG, "the hat-function basis takes precond NONE or DIAG");
  }
  return 0;
}

int fagbi_create(const fagbi_params* p, fagbi_handle** out) {
  if (!p || !out) return set_error(FAGBI_E_ARG, "null argument");
  *out = nullptr;
  FAGBI_TRY(check_params(p));
  fagbi_handle* h = new (std::nothrow) fagbi_handle();
  if (!h) return set_error(FAGBI_E_OOM, "host allocation failed");
  h->prm = *p;
  if (const char* e = std::getenv("FAGBI_M2L_TILES")) h->m2l_tiles = std::atoi(e) != 0;
  if (const char* e = std::getenv("FAGBI_M2L_MFMA")) h->m2l_mfma = std::atoi(e) != 0;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return set_error(FAGBI_E_HIP, "no HIP device");
  }
  // Gauss-Legendre nodes and weights of the singular/close rules
  std::vector<double> gl(qt_size(p->quad_duffy));
  quad_table(p->quad_duffy, gl.data());
  int r = h->upload(h->d_gl, gl.data(), gl.size() * sizeof(double));
  // this device's address of the allocation-free energy sum's scratch array
  if (r == 0) r = fagbi::energy_scratch_init(h->device);
  if (r < 0) {
    h->free_all();
    delete h;
    return r;
  }
  *out = h;
  return 0;
}

void fagbi_destroy(fagbi_handle* h) {
  if (!h) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  h->free_all();
  for (auto& t : h->tc_ws) t.release();
  for (auto& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  if (h->s_near) (void)hipStreamDestroy(h->s_near);
  if (h->hpin) (void)hipHostFree(h->hpin);
  for (hipEvent_t e : {h->ev_up0, h->ev_up1, h->ev_m2l, h->ev_upd, h->ev_col})
    if (e) (void)hipEventDestroy(e);
  if (h->s_m2l) (void)hipStreamDestroy(h->s_m2l);
  (void)hipSetDevice(cur);
  delete h;
}

int fagbi_build_tree(fagbi_handle* h, const double* verts, int64_t nv, const int32_t* tris,
                     int64_t nt) {
  if (!h || !verts || !tris) return set_error(FAGBI_E_ARG, "null argument");
  if (nt > (int64_t)1 << 30) return set_error(FAGBI_E_ARG, "too many panels");
  StageTimer tm(h, 0, &h->prof.ms_tree);
  return fagbi::build_tree(h, verts, nv, tris, nt);
}

int fagbi_assemble_nearfield(fagbi_handle* h, void* stream) {
  if (!h) return set_error(FAGBI_E_ARG, "null handle");
  if (!h->tree_ready) return set_error(FAGBI_E_STATE, "assemble_nearfield before build_tree");
  hipStream_t s = (hipStream_t)stream;
  h->near_ready = false;
  FAGBI_TRY(fagbi::assemble_nearfield(h, s));
  {
    StageTimer tm(h, s, &h->prof.ms_fmm_setup);
    FAGBI_TRY(fagbi::fmm_setup(h, s));
  }
  if (!h->precond_ready) {
    StageTimer tm(h, s, &h->prof.ms_precond);
    FAGBI_TRY(fagbi::precond_setup(h, s));
  }
  FAGBI_HIP(hipStreamSynchronize(s));
  h->near_ready = true;
  return 0;
}

int fagbi_matvec_parts(fagbi_handle* h, const double* x, double* y, int32_t precision,
                       int32_t parts, void* stream) {
  if (!h || !x || !y) return set_error(FAGBI_E_ARG, "null argument");
  if (!h->near_ready) return set_error(FAGBI_E_STATE, "matvec before assemble_nearfield");
  if (precision != FAGBI_FP64 && precision != FAGBI_MIXED)
    return set_error(FAGBI_E_ARG, "bad precision");
  if (x == y) return set_error(FAGBI_E_ARG, "x and y must not alias");
  return fagbi::matvec(h, x, y, precision, parts & FAGBI_PART_ALL, (hipStream_t)stream);
}

int fagbi_matvec(fagbi_handle* h, const double* x, double* y, int32_t precision,
                 void* stream) {
  return fagbi_matvec_parts(h, x, y, precision, FAGBI_PART_ALL, stream);
}

int fagbi_precond_apply(fagbi_handle* h, const double* z, double* y, void* stream) {
  if (!h || !z || !y) return set_error(FAGBI_E_ARG, "null argument");
  if (!h->near_ready) return set_error(FAGBI_E_STATE, "precond_apply before assemble_nearfield");
  return fagbi::precond_apply(h, z, y, (hipStream_t)stream);
}

int fagbi_rhs(fagbi_handle* h, const double* xq, const double* q, int64_t nc, double* b,
              void* stream) {
  if (!h || !xq || !q || !b || nc < 1) return set_error(FAGBI_E_ARG, "bad argument");
  if (!h->tree_ready) return set_error(FAGBI_E_STATE, "rhs before build_tree");
  return fagbi::rhs(h, xq, q, nc, b, (hipStream_t)stream);
}

int fagbi_solve(fagbi_handle* h, const double* xq, const double* q, int64_t nc, double* x,
                fagbi_solve_info* info, void* stream) {
  if (!h || !xq || !q || !x || nc < 1) return set_error(FAGBI_E_ARG, "bad argument");
  if (!h->near_ready) return set_error(FAGBI_E_STATE, "solve before assemble_nearfield");
  return fagbi::solve(h, xq, q, nc, x, info, (hipStream_t)stream);
}

int fagbi_solvation_energy(fagbi_handle* h, const double* x, const double* xq, const double* q,
                           int64_t nc, double* E_kcal, void* stream) {
  if (!h || !x || !xq || !q || !E_kcal || nc < 1) return set_error(FAGBI_E_ARG, "bad argument");
  if (!h->tree_ready) return set_error(FAGBI_E_STATE, "energy before build_tree");
  return fagbi::energy(h, x, xq, q, nc, E_kcal, (hipStream_t)stream);
}

int fagbi_solvation_energy_noalloc(fagbi_handle* h, const double* x, const double* chg, int64_t nc,
                                   double* E_kcal, void* stream) {
  if (!h || !x || !chg || !E_kcal || nc < 1) return set_error(FAGBI_E_ARG, "bad argument");
  if (reinterpret_cast<uintptr_t>(chg) % 32) return set_error(FAGBI_E_ARG, "chg must be 32-byte aligned");
  if (h->hat()) return set_error(FAGBI_E_ARG, "not available with the hat-function basis");
  if (!h->tree_ready) return set_error(FAGBI_E_STATE, "energy before build_tree");
  return fagbi::energy_noalloc(h, x, chg, nc, E_kcal, (hipStream_t)stream);
}

int fagbi_rhs_treecode(fagbi_handle* h, const double* xq, const double* q, int64_t nc, double theta,
                       int32_t p_max, double* b, void* stream) {
  if (!h || !xq || !q || !b || nc < 1) return set_error(FAGBI_E_ARG, "bad argument");
  if (!(theta >= 0.0 && theta < 1.0)) return set_error(FAGBI_E_ARG, "theta outside [0, 1)");
  if (p_max < 0) return set_error(FAGBI_E_ARG, "p_max must be >= 0");
  if (!h->near_ready) return set_error(FAGBI_E_STATE, "treecode right-hand side before assemble_nearfield");
  return fagbi::rhs_treecode(h, xq, q, nc, theta, p_max, b, (hipStream_t)stream);
}

int fagbi_solvation_energy_treecode(fagbi_handle* h, const double* x, const double* xq, const double* q,
                                    int64_t nc, double theta, int32_t p_max, double* E_kcal, void* stream) {
  if (!h || !x || !xq || !q || !E_kcal || nc < 1) return set_error(FAGBI_E_ARG, "bad argument");
  if (!(theta >= 0.0 && theta < 1.0)) return set_error(FAGBI_E_ARG, "theta outside [0, 1)");
  if (p_max < 0) return set_error(FAGBI_E_ARG, "p_max must be >= 0");
  if (!h->near_ready) return set_error(FAGBI_E_STATE, "treecode energy before assemble_nearfield");
  return fagbi::energy_treecode(h, x, xq, q, nc, theta, p_max, E_kcal, (hipStream_t)stream);
}

int fagbi_get_tree_info(fagbi_handle* h, fagbi_tree_info* info) {
  if (!h || !info) return set_error(FAGBI_E_ARG, "null argument");
  if (!h->tree_ready) return set_error(FAGBI_E_STATE, "no tree");
  memset(info, 0, sizeof *info);
  info->n_panels = h->N;
  info->n_leaves = h->lev[h->L].n;
  info->levels = h->L;
  info->lmin = h->lmin;
  info->near_pairs = h->n_ent;
  int64_t pairs = 0, macs = 0;
  for (int l = 0; l <= h->L; ++l) {
    const Level& D = h->lev[l];
    const int64_t np = D.n_inter;
    pairs += np;
    int64_t per = 0;   // sum over alpha of T(p - |alpha|)
    for (int d = 0; d <= D.order; ++d) per += (int64_t)((d + 1) * (d + 2) / 2) * nterms(D.order - d);
    macs += 2 * np * per;
    if (l < FAGBI_MAX_LEVELS) {
      info->lev_clusters[l] = D.n;
      info->lev_order[l] = D.order;
      info->lev_offsets[l] = D.n_off;
      info->lev_pairs[l] = np;
    }
  }
  info->m2l_pairs = pairs;
  info->m2l_flops_fp = macs;
  for (int k = 0; k < 4; ++k) info->singular_pairs[k] = h->singular_count[k];
  info->order_leaf = h->lev[h->L].order;
  info->order_root = h->lev[0].order;
  info->rho_leaf = h->lev[h->L].rho;
  info->h_leaf = h->lev[h->L].h;
  int64_t bytes = 0;
  for (const DBuf* b : h->owned) bytes += (int64_t)b->bytes;
  for (const Tmp& t : h->tc_ws) bytes += (int64_t)t.bytes;
  info->device_bytes = bytes;
  if (h->hat()) {
    info->hat_rows = h->n_vb_rows;
    info->hat_entries = h->n_vb_ent;
  }
  return 0;
}

int fagbi_set_profiling(fagbi_handle* h, int32_t on) {
  if (!h) return set_error(FAGBI_E_ARG, "null handle");
  h->profiling = on != 0;
  if (h->profiling) h->prof = fagbi_profile{};
  return 0;
}

int fagbi_get_profile(fagbi_handle* h, fagbi_profile* out) {
  if (!h || !out) return set_error(FAGBI_E_ARG, "null argument");
  *out = h->prof;
  return 0;
}

int fagbi_get_permutation(fagbi_handle* h, int32_t* perm) {
  if (!h || !perm) return set_error(FAGBI_E_ARG, "null argument");
  if (!h->tree_ready) return set_error(FAGBI_E_STATE, "no tree");
  FAGBI_HIP(hipMemcpy(perm, h->d_perm.p, h->N * 4, hipMemcpyDeviceToHost));
  return 0;
}

}  // extern "C"
