// Right-hand side and solvation energy (paper Sec. 2.2 source terms and
// Sec. 2.3 discrete energy, unit factor of Sec. 3), and the Krylov solvers:
// right-preconditioned GMRES in FP64 (Sec. 2.3 closing paragraph), and for
// FAGBI_MIXED a flexible GMRES on the FP64 operator whose preconditioner is an
// inner GMRES on the FP32 operator (inner solves to inner_tol); Arnoldi
// (classical Gram-Schmidt, applied twice), Givens rotations, the small
// least-squares solve and the energy sum stay in FP64.
#include <chrono>
#include <cmath>
#include <functional>
#include <mutex>

#include "fmath.h"
#include "internal.h"

namespace fagbi {

constexpr int RB = 256;   // reduction block

// Both direct sums run one thread per panel over its three quadrature points
// (quad_points) with the charges staged through LDS; charges carry q / (4 pi).
// FP64 throughout.

// b1 = (1/eps_in) sum_q w_q sum_k q_k G0(x_q, y_k); b2 likewise with dG0/dn_x.
// HAT: per panel corner a, the same sums with lambda_a(x_q) inside, written to
// the element rows b[e], b[3N + e] (e = 3 i + a) for the sum into the vertices
template <bool HAT = false>
__global__ void __launch_bounds__(256) k_rhs(const double* __restrict__ pv, const double* __restrict__ pn,
                                             const double* __restrict__ pa, const int32_t* __restrict__ perm,
                                             int N, const double4* __restrict__ chg, int nc, double inv_eps_in,
                                             double* b) {
  __shared__ double4 tile[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < N;
  double qp[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, n[3] = {0, 0, 0}, w = 0;
  if (valid) {
    quad_points(pv, i, qp);
    for (int d = 0; d < 3; ++d) n[d] = pn[3 * i + d];
    w = pa[i] / 3.0;
  }
  double s1 = 0, s2 = 0;
  double h1[3] = {0, 0, 0}, h2[3] = {0, 0, 0};   // per point (HAT)
  for (int t0 = 0; t0 < nc; t0 += 256) {
    __syncthreads();
    if (t0 + (int)threadIdx.x < nc) {
      double4 c = chg[t0 + threadIdx.x];
      c.w *= 1.0 / FOUR_PI;
      tile[threadIdx.x] = c;
    }
    __syncthreads();
    const int m = min(256, nc - t0);
    if (valid)
      for (int k = 0; k < m; ++k) {
        const double4 c = tile[k];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const double rx = qp[3 * q] - c.x, ry = qp[3 * q + 1] - c.y, rz = qp[3 * q + 2] - c.z;
          const double ir = inv_sqrt(rx * rx + ry * ry + rz * rz);
          const double g = c.w * ir;
          if constexpr (HAT) {
            h1[q] += g;
            h2[q] -= g * (rx * n[0] + ry * n[1] + rz * n[2]) * (ir * ir);
          } else {
            s1 += g;
            s2 -= g * (rx * n[0] + ry * n[1] + rz * n[2]) * (ir * ir);
          }
        }
      }
  }
  if (!valid) return;
  if constexpr (HAT) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double c1 = 0, c2 = 0;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double l = q == a ? 2.0 / 3.0 : 1.0 / 6.0;
        c1 += l * h1[q];
        c2 += l * h2[q];
      }
      b[3 * i + a] = w * c1 * inv_eps_in;
      b[3 * (int64_t)N + 3 * i + a] = w * c2 * inv_eps_in;
    }
  } else {
    const int p = perm[i];
    b[p] = w * s1 * inv_eps_in;
    b[N + p] = w * s2 * inv_eps_in;
  }
}

// per-block partial sums of sum_i w_i sum_q sum_n q_n [K1 dphi_i + K2 phi_i]
// with K1 = (G0 - Gk)(x_n, y), K2 = d/dn_y (eps Gk - G0)(x_n, y), y on the
// panel.  HAT: phi and dphi at point q interpolated from the nodal values,
// sum_a lambda_a(x_q) x[v_a] (perm then holds the panels' vertices [N][3] and
// N_x the vertex count)
template <bool HAT = false>
__global__ void __launch_bounds__(256) k_energy(const double* __restrict__ pv, const double* __restrict__ pn,
                                                const double* __restrict__ pa, const int32_t* __restrict__ perm,
                                                int N, const double4* __restrict__ chg, int nc, double eps,
                                                double kappa, const double* __restrict__ x, double* partial,
                                                int64_t N_x = 0) {
  __shared__ double4 tile[256];
  __shared__ double red[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < N;
  double qp[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, n[3] = {0, 0, 0}, w = 0, phi = 0, dphi = 0;
  double hu[3] = {0, 0, 0}, hv[3] = {0, 0, 0};   // HAT: nodal values at the corners
  if (valid) {
    quad_points(pv, i, qp);
    for (int d = 0; d < 3; ++d) n[d] = pn[3 * i + d];
    w = pa[i] / 3.0;
    if constexpr (HAT) {
      for (int a = 0; a < 3; ++a) {
        const int64_t v = perm[3 * i + a];
        hu[a] = x[v];
        hv[a] = x[N_x + v];
      }
    } else {
      const int p = perm[i];
      phi = x[p];
      dphi = x[N + p];
    }
  }
  double a1 = 0, a2 = 0;   // sum q K1, sum q K2
  double b1[3] = {0, 0, 0}, b2[3] = {0, 0, 0};   // per point (HAT)
  for (int t0 = 0; t0 < nc; t0 += 256) {
    __syncthreads();
    if (t0 + (int)threadIdx.x < nc) {
      double4 c = chg[t0 + threadIdx.x];
      c.w *= 1.0 / FOUR_PI;
      tile[threadIdx.x] = c;
    }
    __syncthreads();
    const int m = min(256, nc - t0);
    if (valid)
      for (int k = 0; k < m; ++k) {
        const double4 c = tile[k];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const double rx = c.x - qp[3 * q], ry = c.y - qp[3 * q + 1], rz = c.z - qp[3 * q + 2];
          const double r2 = rx * rx + ry * ry + rz * rz;
          const double ir = inv_sqrt(r2);
          const double u = kappa * (r2 * ir);
          double E, em1;
          exp_expm1(-u, E, em1);
          const double rny = rx * n[0] + ry * n[1] + rz * n[2];
          const double g = c.w * ir;
          if constexpr (HAT) {
            b1[q] -= g * em1;
            b2[q] += g * (eps * E * (1.0 + u) - 1.0) * rny * (ir * ir);
          } else {
            a1 -= g * em1;
            a2 += g * (eps * E * (1.0 + u) - 1.0) * rny * (ir * ir);
          }
        }
      }
  }
  double tot = w * (a1 * dphi + a2 * phi);
  if constexpr (HAT) {
    tot = 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double u = 0, v = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double l = q == a ? 2.0 / 3.0 : 1.0 / 6.0;
        u += l * hu[a];
        v += l * hv[a];
      }
      tot += b1[q] * v + b2[q] * u;
    }
    tot *= w;
  }
  red[threadIdx.x] = valid ? tot : 0.0;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// scale times the sum of n doubles, by one block in a fixed order
__global__ void k_sum(const double* __restrict__ v, int n, double scale, double* out) {
  __shared__ double red[RB];
  double a = 0;
  for (int k = threadIdx.x; k < n; k += RB) a += v[k];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int o = RB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0] * scale;
}

// partial[i][blk] = V_i[chunk] . w[chunk]   (grid: NB x nvec)
__global__ void __launch_bounds__(RB) k_multidot(const double* __restrict__ V, int64_t ld, const double* __restrict__ w,
                                                 int64_t n, int NB, double* partial) {
  __shared__ double red[RB];
  const int vi = blockIdx.y;
  const double* v = V + vi * ld;
  double a = 0;
  for (int64_t e = (int64_t)blockIdx.x * RB + threadIdx.x; e < n; e += (int64_t)NB * RB) a += v[e] * w[e];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int o = RB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)vi * NB + blockIdx.x] = red[0];
}

// out[i] (+)= sum_blk partial[i][blk]
__global__ void k_reduce_rows(const double* __restrict__ partial, int NB, double* out, int accumulate) {
  __shared__ double red[RB];
  const int vi = blockIdx.x;
  double a = 0;
  for (int k = threadIdx.x; k < NB; k += RB) a += partial[(int64_t)vi * NB + k];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int o = RB / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[vi] = accumulate ? out[vi] + red[0] : red[0];
}

// w -= sum_i h_i V_i   (or x += sum_i h_i V_i with sign = +1)
__global__ void k_combine(const double* __restrict__ V, int64_t ld, const double* __restrict__ hcoef, int nv,
                          double sign, int64_t n, double* w) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    double a = 0;
    for (int i = 0; i < nv; ++i) a += hcoef[i] * V[i * ld + e];
    w[e] += sign * a;
  }
}

// y = alpha * x  (alpha read from device: 1/norm), or y = a*x + b*y
__global__ void k_scale_dev(const double* __restrict__ x, const double* __restrict__ nrm, int64_t n, double* y) {
  const double s = 1.0 / sqrt(*nrm);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = x[e] * s;
}
__global__ void k_axpby(double a, const double* __restrict__ x, double b, double* y, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    y[e] = a * x[e] + b * y[e];
}

static int upload_charges(Tmp& buf, const double* xq, const double* q, int64_t nc) {
  std::vector<double> c(4 * nc);
  for (int64_t k = 0; k < nc; ++k) {
    c[4 * k] = xq[3 * k];
    c[4 * k + 1] = xq[3 * k + 1];
    c[4 * k + 2] = xq[3 * k + 2];
    c[4 * k + 3] = q[k];
  }
  FAGBI_TRY(buf.alloc(c.size() * 8));
  FAGBI_HIP(hipMemcpy(buf.p, c.data(), c.size() * 8, hipMemcpyHostToDevice));
  return 0;
}

int rhs(fagbi_handle* h, const double* xq, const double* q, int64_t nc, double* b, hipStream_t s) {
  if (nc > (1 << 30)) return set_error(FAGBI_E_ARG, "too many charges");
  if (h->hat() && !h->d_vx_off.p)
    return set_error(FAGBI_E_STATE, "hat-function right-hand side before assemble_nearfield");
  Tmp chg;
  FAGBI_TRY(upload_charges(chg, xq, q, nc));
  if (h->hat()) {
    // corner sums into the element rows, then into the vertices
    double* rows = h->d_ye.as<double>();
    k_rhs<true><<<(unsigned)((h->N + 255) / 256), 256, 0, s>>>(h->d_pv.as<double>(), h->d_pn.as<double>(),
                                                               h->d_pa.as<double>(), nullptr, (int)h->N,
                                                               chg.as<double4>(), (int)nc, 1.0 / h->prm.eps_in,
                                                               rows);
    FAGBI_HIP(hipGetLastError());
    FAGBI_TRY(hat_gather(h, rows, nullptr, b, s));
  } else {
    k_rhs<<<(unsigned)((h->N + 255) / 256), 256, 0, s>>>(h->d_pv.as<double>(), h->d_pn.as<double>(),
                                                          h->d_pa.as<double>(), h->d_perm.as<int32_t>(), (int)h->N,
                                                          chg.as<double4>(), (int)nc, 1.0 / h->prm.eps_in, b);
  }
  FAGBI_HIP(hipGetLastError());
  FAGBI_HIP(hipStreamSynchronize(s));   // the charge buffer is freed on return
  return 0;
}

int energy(fagbi_handle* h, const double* x, const double* xq, const double* q, int64_t nc, double* E,
           hipStream_t s) {
  Tmp chg, part, out;
  FAGBI_TRY(upload_charges(chg, xq, q, nc));
  const int nb = (int)((h->N + 255) / 256);
  FAGBI_TRY(part.alloc(nb * 8));
  FAGBI_TRY(out.alloc(8));
  if (h->hat())
    k_energy<true><<<nb, 256, 0, s>>>(h->d_pv.as<double>(), h->d_pn.as<double>(), h->d_pa.as<double>(),
                                      h->d_ptri.as<int32_t>(), (int)h->N, chg.as<double4>(), (int)nc,
                                      h->prm.eps_out / h->prm.eps_in, h->prm.kappa, x, part.as<double>(), h->nv);
  else
    k_energy<<<nb, 256, 0, s>>>(h->d_pv.as<double>(), h->d_pn.as<double>(), h->d_pa.as<double>(),
                                h->d_perm.as<int32_t>(), (int)h->N, chg.as<double4>(), (int)nc,
                                h->prm.eps_out / h->prm.eps_in, h->prm.kappa, x, part.as<double>());
  k_sum<<<1, RB, 0, s>>>(part.as<double>(), nb, 1.0, out.as<double>());
  FAGBI_HIP(hipGetLastError());
  double tot = 0;
  FAGBI_HIP(hipMemcpyAsync(&tot, out.p, 8, hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipStreamSynchronize(s));
  *E = 0.5 * UNIT_KCAL * tot;
  if (!std::isfinite(*E)) return set_error(FAGBI_E_NUMERIC, "non-finite energy");
  return 0;
}

// ---------------------------------------------------------------------------
// Allocation-free direct energy sum.  The per-block partial sums live in a
// file-scope device array: one copy per GPU, kept until the process ends.
// Host code never passes the array's name to a kernel (in host code it is a
// stand-in, not a device address): each device's address is looked up once,
// with that device current, and kept in g_scratch.
// ---------------------------------------------------------------------------
constexpr int ENERGY_SCRATCH = 1 << 16;   // partial sums of 256 panels each: N <= 2^24
static __device__ __align__(256) double scratch[ENERGY_SCRATCH];
constexpr int SCRATCH_MAX_DEV = 64;
static double* g_scratch[SCRATCH_MAX_DEV];
static std::mutex g_scratch_mu;

int energy_scratch_init(int device) {
  if (device < 0 || device >= SCRATCH_MAX_DEV)
    return set_error(FAGBI_E_ARG, "device %d beyond the %d devices of the scratch table", device,
                     SCRATCH_MAX_DEV);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return 0;
  double* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return set_error(FAGBI_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  g_scratch[device] = ptr;
  return 0;
}

int energy_noalloc(fagbi_handle* h, const double* x, const double* chg, int64_t nc, double* E, hipStream_t s) {
  const int64_t nb = (h->N + 255) / 256;
  if (nb > ENERGY_SCRATCH)
    return set_error(FAGBI_E_ARG, "%lld panels exceed the allocation-free limit of %d", (long long)h->N,
                     ENERGY_SCRATCH * 256);
  if (nc > (1 << 30)) return set_error(FAGBI_E_ARG, "too many charges");
  double* part = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    part = g_scratch[h->device];
  }
  if (!part) return set_error(FAGBI_E_STATE, "scratch array not set up on device %d", h->device);
  k_energy<<<(unsigned)nb, 256, 0, s>>>(h->d_pv.as<double>(), h->d_pn.as<double>(), h->d_pa.as<double>(),
                                        h->d_perm.as<int32_t>(), (int)h->N, reinterpret_cast<const double4*>(chg),
                                        (int)nc, h->prm.eps_out / h->prm.eps_in, h->prm.kappa, x, part);
  k_sum<<<1, RB, 0, s>>>(part, (int)nb, 0.5 * UNIT_KCAL, E);
  FAGBI_HIP(hipGetLastError());
  return 0;
}

// b by the reverse treecode (the charges carry q / (4 pi eps_in))
int rhs_treecode(fagbi_handle* h, const double* xq, const double* q, int64_t nc, double theta, int p_max,
                 double* b, hipStream_t s) {
  if (nc > (1 << 30)) return set_error(FAGBI_E_ARG, "too many charges");
  std::vector<double> qs(nc);
  for (int64_t k = 0; k < nc; ++k) qs[k] = q[k] / (FOUR_PI * h->prm.eps_in);
  Tmp chg;
  FAGBI_TRY(upload_charges(chg, xq, qs.data(), nc));
  return treecode_rhs(h, chg.as<double>(), nc, theta, p_max, b, s);
}

// E by the Cartesian treecode: per-charge terms q_n V_n on the GPU, then the
// fixed-order sum
int energy_treecode(fagbi_handle* h, const double* x, const double* xq, const double* q, int64_t nc, double theta,
                    int p_max, double* E, hipStream_t s) {
  if (nc > (1 << 30)) return set_error(FAGBI_E_ARG, "too many charges");
  Tmp chg, qv, out;
  FAGBI_TRY(upload_charges(chg, xq, q, nc));
  FAGBI_TRY(qv.alloc((size_t)nc * 8));
  FAGBI_TRY(out.alloc(8));
  FAGBI_TRY(treecode_potentials(h, x, chg.as<double>(), nc, theta, p_max, qv.as<double>(), s));
  k_sum<<<1, RB, 0, s>>>(qv.as<double>(), (int)nc, 1.0, out.as<double>());
  FAGBI_HIP(hipGetLastError());
  double tot = 0;
  FAGBI_HIP(hipMemcpyAsync(&tot, out.p, 8, hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipStreamSynchronize(s));
  *E = 0.5 * UNIT_KCAL * tot;
  if (!std::isfinite(*E)) return set_error(FAGBI_E_NUMERIC, "non-finite energy");
  return 0;
}

// ---------------------------------------------------------------------------
// GMRES / flexible GMRES
// ---------------------------------------------------------------------------
struct Krylov {
  int m = 0;
  int64_t n = 0;
  Tmp V, Z, w, partial, hcol;
  int NB = 0;
};

static int krylov_alloc(Krylov& K, int m, int64_t n) {
  K.m = m;
  K.n = n;
  K.NB = (int)std::min<int64_t>(256, (n + RB - 1) / RB);
  FAGBI_TRY(K.V.alloc((size_t)(m + 1) * n * 8));
  FAGBI_TRY(K.Z.alloc((size_t)m * n * 8));
  FAGBI_TRY(K.w.alloc((size_t)n * 8));
  FAGBI_TRY(K.partial.alloc((size_t)(m + 2) * K.NB * 8));
  FAGBI_TRY(K.hcol.alloc((size_t)2 * (m + 2) * 8));
  return 0;
}

// hcol[0..nv) (+)= V[0..nv)^T w
static void multidot(Krylov& K, const double* V, int nv, const double* w, double* out, int acc, hipStream_t s) {
  dim3 g(K.NB, nv);
  k_multidot<<<g, RB, 0, s>>>(V, K.n, w, K.n, K.NB, K.partial.as<double>());
  k_reduce_rows<<<nv, RB, 0, s>>>(K.partial.as<double>(), K.NB, out, acc);
}

using Op = std::function<int(const double*, double*)>;

// pinned host buffer for one Hessenberg column pair of a basis of m vectors
static int pinned_column(fagbi_handle* h, int m) {
  const size_t need = 2 * (size_t)(m + 2);
  if (h->hpin_n >= need) return 0;
  if (h->hpin) FAGBI_HIP(hipHostFree(h->hpin));
  h->hpin = nullptr;
  h->hpin_n = 0;
  FAGBI_HIP(hipHostMalloc(reinterpret_cast<void**>(&h->hpin), need * 8, hipHostMallocDefault));
  h->hpin_n = need;
  return 0;
}

// Solve A x = b, right preconditioned (flexible: P may change per step).
// x holds x0 on entry.  Returns 0 (converged) or FAGBI_W_NOT_CONVERGED.
static int gmres(fagbi_handle* h, Krylov& K, const Op& A, const Op& P, const double* b, double* x, double tol,
                 int maxit, bool x0_zero, int* iters, double* relres, hipStream_t s) {
  const int64_t n = K.n;
  const unsigned G = 1024;
  double* V = K.V.as<double>();
  double* Z = K.Z.as<double>();
  double* w = K.w.as<double>();
  double* hc = K.hcol.as<double>();
  // r0 = b - A x0 into V_0
  if (x0_zero) {
    FAGBI_HIP(hipMemcpyAsync(V, b, n * 8, hipMemcpyDeviceToDevice, s));
  } else {
    FAGBI_TRY(A(x, V));
    k_axpby<<<G, 256, 0, s>>>(1.0, b, -1.0, V, n);
  }
  multidot(K, b, 1, b, hc, 0, s);
  multidot(K, V, 1, V, hc + 1, 0, s);
  double nb2[2];
  FAGBI_HIP(hipMemcpyAsync(nb2, hc, 16, hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipStreamSynchronize(s));
  const double bnorm = std::sqrt(nb2[0]);
  const double beta = std::sqrt(nb2[1]);
  *iters = 0;
  if (!(bnorm > 0)) {
    *relres = 0;
    FAGBI_HIP(hipMemsetAsync(x, 0, n * 8, s));
    return 0;
  }
  if (!std::isfinite(beta)) return set_error(FAGBI_E_NUMERIC, "non-finite residual");
  *relres = beta / bnorm;
  if (*relres <= tol) return 0;
  k_axpby<<<G, 256, 0, s>>>(1.0 / beta, V, 0.0, V, n);
  const int m = std::min(maxit, K.m);
  std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1, 0.0), col(m + 2);
  // the column comes back through pinned memory, waited for by polling an
  // event (a copy into pageable memory and a stream synchronisation left the
  // GPU idle for ~65 us per iteration); solve() sizes the buffer for both
  // levels of the flexible solve, so the inner solves never replace it
  FAGBI_TRY(pinned_column(h, K.m));
  if (!h->ev_col) FAGBI_HIP(hipEventCreateWithFlags(&h->ev_col, hipEventDisableTiming));
  g[0] = beta;
  int k = 0;
  for (; k < m; ++k) {
    double* vk = V + (int64_t)k * n;
    double* zk = Z + (int64_t)k * n;
    FAGBI_TRY(P(vk, zk));
    FAGBI_TRY(A(zk, w));
    double* hp = h->hpin;   // after P: an inner solve may have run
    // classical Gram-Schmidt, twice; the first pass's coefficients stay on
    // the device (hc2) until the one read-back per iteration
    double* hc2 = hc + (m + 2);
    multidot(K, V, k + 1, w, hc2, 0, s);
    k_combine<<<G, 256, 0, s>>>(V, n, hc2, k + 1, -1.0, n, w);
    multidot(K, V, k + 1, w, hc, 0, s);
    k_combine<<<G, 256, 0, s>>>(V, n, hc, k + 1, -1.0, n, w);
    multidot(K, w, 1, w, hc + k + 1, 0, s);
    FAGBI_HIP(hipMemcpyAsync(hp, hc, (k + 2) * 8, hipMemcpyDeviceToHost, s));
    FAGBI_HIP(hipMemcpyAsync(hp + (K.m + 2), hc2, (k + 1) * 8, hipMemcpyDeviceToHost, s));
    FAGBI_HIP(hipEventRecord(h->ev_col, s));
    hipError_t q;
    while ((q = hipEventQuery(h->ev_col)) == hipErrorNotReady) {
    }
    FAGBI_HIP(q);
    for (int i = 0; i <= k + 1; ++i) col[i] = hp[i];
    for (int i = 0; i <= k; ++i) col[i] += hp[K.m + 2 + i];
    const double hn = std::sqrt(col[k + 1]);
    if (!std::isfinite(hn)) return set_error(FAGBI_E_NUMERIC, "non-finite Krylov vector");
    col[k + 1] = hn;
    if (hn > 0) k_scale_dev<<<G, 256, 0, s>>>(w, hc + k + 1, n, V + (int64_t)(k + 1) * n);
    // Givens
    for (int i = 0; i < k; ++i) {
      const double t = cs[i] * col[i] + sn[i] * col[i + 1];
      col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
      col[i] = t;
    }
    const double den = std::hypot(col[k], col[k + 1]);
    cs[k] = col[k] / den;
    sn[k] = col[k + 1] / den;
    col[k] = den;
    col[k + 1] = 0;
    g[k + 1] = -sn[k] * g[k];
    g[k] = cs[k] * g[k];
    for (int i = 0; i <= k; ++i) H[(size_t)i * m + k] = col[i];
    *relres = std::fabs(g[k + 1]) / bnorm;
    if (*relres <= tol || hn == 0) {
      ++k;
      break;
    }
  }
  if (k > m) k = m;
  *iters = k;
  // back substitution and x += Z y
  std::vector<double> y(k);
  for (int i = k - 1; i >= 0; --i) {
    double a = g[i];
    for (int j = i + 1; j < k; ++j) a -= H[(size_t)i * m + j] * y[j];
    y[i] = a / H[(size_t)i * m + i];
  }
  FAGBI_HIP(hipMemcpyAsync(hc, y.data(), k * 8, hipMemcpyHostToDevice, s));
  if (x0_zero) FAGBI_HIP(hipMemsetAsync(x, 0, n * 8, s));
  k_combine<<<G, 256, 0, s>>>(Z, n, hc, k, 1.0, n, x);
  FAGBI_HIP(hipGetLastError());
  FAGBI_HIP(hipStreamSynchronize(s));
  return *relres <= tol ? 0 : FAGBI_W_NOT_CONVERGED;
}

int solve(fagbi_handle* h, const double* xq, const double* q, int64_t nc, double* x, fagbi_solve_info* info,
          hipStream_t s) {
  const int64_t n = 2 * h->n_unk();
  fagbi_solve_info inf{};
  auto t0 = std::chrono::steady_clock::now();
  Tmp b, r;
  FAGBI_TRY(b.alloc(n * 8));
  if (h->prm.rhs_theta > 0)
    FAGBI_TRY(rhs_treecode(h, xq, q, nc, h->prm.rhs_theta, h->prm.rhs_pmax, b.as<double>(), s));
  else
    FAGBI_TRY(rhs(h, xq, q, nc, b.as<double>(), s));
  FAGBI_HIP(hipStreamSynchronize(s));
  auto t1 = std::chrono::steady_clock::now();
  // is the initial guess zero?
  Krylov K;
  FAGBI_TRY(krylov_alloc(K, 1, n));
  multidot(K, x, 1, x, K.hcol.as<double>(), 0, s);
  double xx = 0;
  FAGBI_HIP(hipMemcpyAsync(&xx, K.hcol.p, 8, hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipStreamSynchronize(s));
  const bool x0_zero = xx == 0.0;
  int n64 = 0, n32 = 0, total_inner = 0;
  Op A64 = [&](const double* in, double* out) {
    ++n64;
    return matvec(h, in, out, FAGBI_FP64, FAGBI_PART_ALL, s);
  };
  Op A32 = [&](const double* in, double* out) {
    ++n32;
    return matvec(h, in, out, FAGBI_MIXED, FAGBI_PART_ALL, s);
  };
  Op M = [&](const double* in, double* out) { return precond_apply(h, in, out, s); };
  Op M32 = [&](const double* in, double* out) { return precond_apply(h, in, out, s, true); };
  int status = 0, it = 0;
  double rel = 0;
  FAGBI_TRY(pinned_column(h, std::max(h->prm.max_iter, h->prm.max_outer)));
  if (h->prm.precision == FAGBI_FP64) {
    Krylov KA;
    FAGBI_TRY(krylov_alloc(KA, h->prm.max_iter, n));
    status = gmres(h, KA, A64, M, b.as<double>(), x, h->prm.tol, h->prm.max_iter, x0_zero, &it, &rel, s);
    if (status < 0) return status;
    inf.outer_iterations = 1;
    total_inner = it;
  } else {
    Krylov KO, KI;
    FAGBI_TRY(krylov_alloc(KO, h->prm.max_outer, n));
    FAGBI_TRY(krylov_alloc(KI, h->prm.max_iter, n));
    Op inner = [&](const double* in, double* out) {
      int iti = 0;
      double rr = 0;
      int st = gmres(h, KI, A32, M32, in, out, h->prm.inner_tol, h->prm.max_iter, true, &iti, &rr, s);
      total_inner += iti;
      return st < 0 ? st : 0;
    };
    status = gmres(h, KO, A64, inner, b.as<double>(), x, h->prm.tol, h->prm.max_outer, x0_zero, &it, &rel, s);
    if (status < 0) return status;
    inf.outer_iterations = it;
  }
  // true residual in FP64
  FAGBI_TRY(r.alloc(n * 8));
  FAGBI_TRY(matvec(h, x, r.as<double>(), FAGBI_FP64, FAGBI_PART_ALL, s));
  ++n64;
  k_axpby<<<1024, 256, 0, s>>>(1.0, b.as<double>(), -1.0, r.as<double>(), n);
  Krylov KR;
  FAGBI_TRY(krylov_alloc(KR, 1, n));
  multidot(KR, r.as<double>(), 1, r.as<double>(), KR.hcol.as<double>(), 0, s);
  multidot(KR, b.as<double>(), 1, b.as<double>(), KR.hcol.as<double>() + 1, 0, s);
  double rb[2];
  FAGBI_HIP(hipMemcpyAsync(rb, KR.hcol.p, 16, hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipStreamSynchronize(s));
  auto t2 = std::chrono::steady_clock::now();
  inf.inner_iterations = total_inner;
  inf.matvecs_fp64 = n64;
  inf.matvecs_fp32 = n32;
  inf.rel_residual = rb[1] > 0 ? std::sqrt(rb[0] / rb[1]) : 0.0;
  inf.t_rhs_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  inf.t_solve_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
  if (info) *info = inf;
  if (!std::isfinite(inf.rel_residual)) return set_error(FAGBI_E_NUMERIC, "non-finite residual");
  return inf.rel_residual <= h->prm.tol ? 0 : FAGBI_W_NOT_CONVERGED;
}

}  // namespace fagbi
