// Learned near-field surrogate: a 16 -> 128 -> 128 -> 128 -> 6 tanh network
// (FP32) that maps the geometry of a near-singular panel pair (edge-adjacent,
// vertex-adjacent or close) to the correction of its six Galerkin integrals
// over the 3x3 regular rule.  Trained on the GPU by the kernels below on
// labels produced by the library's own singular cubature; used in the
// block-diagonal preconditioner (FAGBI_MLP_PRECOND) or, where its calibrated
// per-pair error passes mlp_gate_tol, in the operator's near field
// (FAGBI_MLP_GATED); the cubature is the fallback.
//
// Features (dimensionless): the pair in the target panel's frame (origin its
// centroid, z its normal, x along its first canonical edge), lengths divided
// by h = sqrt(A_target): target corners (x0, y0, x1), the three source
// corners (9), kappa*h, and the class one-hot (3).  Canonical corner order:
// edge pairs start with the shared edge (in the target's order), vertex
// pairs with the shared vertex, close pairs with the corner nearest the other
// panel's centroid (cyclic order kept).  Targets: (I_m - I3x3_m) / h^k_m with
// k = (3, 2, 2, 2, 2, 1), the scaling of I1..I6 with size at fixed kappa*h.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "near.h"
#include "scan.h"

namespace fagbi {

constexpr int NIN = 16, NH = 128, NOUT = 6, NAUX = 8;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NIN * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NH, OFF_W4 = OFF_B3 + NH,
              OFF_B4 = OFF_W4 + NH * NOUT, NPAR = OFF_B4 + NOUT;
constexpr int NNORM = 2 * NIN + 2 * 3 * NOUT;   // input mean/sd, per-class output mean/sd
constexpr int OUT_MU = 2 * NIN, OUT_SD = 2 * NIN + 3 * NOUT;
constexpr int NCLS = 3, NBIN = 8;
constexpr int NCAL = NCLS * (NBIN + 1) + NCLS * NBIN;
constexpr int NBLOB = NPAR + NNORM + NCAL;
static_assert(NPAR == 35974, "layout");

__device__ inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// canonical corner order of the pair (see file comment)
__device__ inline void canonical(const NearArgs& a, int cls, int i, int j, int* oi, int* oj) {
  const int* ti = a.ptri + 3 * i;
  const int* tj = a.ptri + 3 * j;
  if (cls == C_EDGE) {
    int n = 0, ri = 0, rj = 0;
    for (int p = 0; p < 3; ++p) {
      const bool sh = ti[p] == tj[0] || ti[p] == tj[1] || ti[p] == tj[2];
      if (sh) oi[n++] = p; else ri = p;
    }
    oi[2] = ri;
    for (int q = 0; q < 3; ++q) {
      const bool sh = tj[q] == ti[0] || tj[q] == ti[1] || tj[q] == ti[2];
      if (!sh) rj = q;
      if (tj[q] == ti[oi[0]]) oj[0] = q;
      if (tj[q] == ti[oi[1]]) oj[1] = q;
    }
    oj[2] = rj;
  } else if (cls == C_VERTEX) {
    int si = 0, sj = 0;
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q)
        if (ti[p] == tj[q]) { si = p; sj = q; }
    oi[0] = si; oi[1] = si == 0 ? 1 : 0; oi[2] = si == 2 ? 1 : 2;
    oj[0] = sj; oj[1] = sj == 0 ? 1 : 0; oj[2] = sj == 2 ? 1 : 2;
  } else {
    double ci[3], cj[3];
    for (int d = 0; d < 3; ++d) {
      ci[d] = (a.pv[9 * i + d] + a.pv[9 * i + 3 + d] + a.pv[9 * i + 6 + d]) / 3.0;
      cj[d] = (a.pv[9 * j + d] + a.pv[9 * j + 3 + d] + a.pv[9 * j + 6 + d]) / 3.0;
    }
    int bi = 0, bj = 0;
    double di = 1e300, dj = 1e300;
    for (int p = 0; p < 3; ++p) {
      double s = 0, t = 0;
      for (int d = 0; d < 3; ++d) {
        s += (a.pv[9 * i + 3 * p + d] - cj[d]) * (a.pv[9 * i + 3 * p + d] - cj[d]);
        t += (a.pv[9 * j + 3 * p + d] - ci[d]) * (a.pv[9 * j + 3 * p + d] - ci[d]);
      }
      if (s < di) { di = s; bi = p; }
      if (t < dj) { dj = t; bj = p; }
    }
    for (int p = 0; p < 3; ++p) {
      oi[p] = (bi + p) % 3;
      oj[p] = (bj + p) % 3;
    }
  }
}

// centroid distance of a pair over sqrt(h_i h_j), h = sqrt(area)
__device__ inline double pair_dratio(const NearArgs& a, int i, int j) {
  const double* P = a.pv + 9 * i;
  const double* Q = a.pv + 9 * j;
  double r[3];
  for (int d = 0; d < 3; ++d) r[d] = (P[d] + P[3 + d] + P[6 + d]) / 3.0 - (Q[d] + Q[3 + d] + Q[6 + d]) / 3.0;
  return sqrt(dot3(r, r)) / sqrt(sqrt(a.pa[i] * a.pa[j]));
}

__device__ inline void pair_features(const NearArgs& a, int cls, int i, int j, float* X, double* hout,
                                     double* dratio) {
  int oi[3], oj[3];
  canonical(a, cls, i, j, oi, oj);
  const double* P = a.pv + 9 * i;
  const double* Q = a.pv + 9 * j;
  double ci[3], cj[3];
  for (int d = 0; d < 3; ++d) {
    ci[d] = (P[d] + P[3 + d] + P[6 + d]) / 3.0;
    cj[d] = (Q[d] + Q[3 + d] + Q[6 + d]) / 3.0;
  }
  double ex[3], ey[3];
  const double* ez = a.pn + 3 * i;
  for (int d = 0; d < 3; ++d) ex[d] = P[3 * oi[1] + d] - P[3 * oi[0] + d];
  const double ln = sqrt(dot3(ex, ex));
  for (int d = 0; d < 3; ++d) ex[d] /= ln;
  ey[0] = ez[1] * ex[2] - ez[2] * ex[1];
  ey[1] = ez[2] * ex[0] - ez[0] * ex[2];
  ey[2] = ez[0] * ex[1] - ez[1] * ex[0];
  const double h = sqrt(a.pa[i]);
  double r[3];
  for (int d = 0; d < 3; ++d) r[d] = P[3 * oi[0] + d] - ci[d];
  X[0] = (float)(dot3(r, ex) / h);
  X[1] = (float)(dot3(r, ey) / h);
  for (int d = 0; d < 3; ++d) r[d] = P[3 * oi[1] + d] - ci[d];
  X[2] = (float)(dot3(r, ex) / h);
  for (int q = 0; q < 3; ++q) {
    for (int d = 0; d < 3; ++d) r[d] = Q[3 * oj[q] + d] - ci[d];
    X[3 + 3 * q] = (float)(dot3(r, ex) / h);
    X[4 + 3 * q] = (float)(dot3(r, ey) / h);
    X[5 + 3 * q] = (float)(dot3(r, ez) / h);
  }
  X[12] = (float)(a.kappa * h);
  X[13] = cls == C_EDGE ? 1.f : 0.f;
  X[14] = cls == C_VERTEX ? 1.f : 0.f;
  X[15] = cls == C_CLOSE ? 1.f : 0.f;
  *hout = h;
  (void)cj;
  *dratio = pair_dratio(a, i, j);
}

// class of a feature row from its one-hot inputs (0 edge, 1 vertex, 2 close)
__host__ __device__ inline int row_class(const float* x) { return x[14] > 0.5f ? 1 : (x[15] > 0.5f ? 2 : 0); }

__device__ inline double hpow(double h, int m) {
  return m == 0 ? h * h * h : m == 5 ? h : h * h;
}

// features, 3x3 integrals and pair data of a list of items of one class
__global__ void k_mlp_prepare(NearArgs a, int cls, const Item* __restrict__ items, int64_t n, float* X,
                              double* I3, double* hh, float* dr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const Item it = items[t];
  double h, d;
  float f[NIN];
  pair_features(a, cls, it.i, it.j, f, &h, &d);
  for (int k = 0; k < NIN; ++k) X[t * NIN + k] = f[k];
  double I[6];
  regular_pair(a, it.i, it.j, I);
  for (int m = 0; m < 6; ++m) I3[t * 6 + m] = I[m];
  hh[t] = h;
  dr[t] = (float)d;
}

// training targets and evaluation data from cubature integrals
__global__ void k_mlp_targets(int cls_index, const double* __restrict__ Iq, const double* __restrict__ I3,
                              const double* __restrict__ hh, const float* __restrict__ dr, int64_t n, float* T,
                              float* aux) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double h = hh[t];
  aux[t * NAUX] = (float)(cls_index - 1);
  aux[t * NAUX + 1] = dr[t];
  for (int m = 0; m < 6; ++m) {
    const double s = hpow(h, m);
    T[t * NOUT + m] = (float)((Iq[t * 6 + m] - I3[t * 6 + m]) / s);
    aux[t * NAUX + 2 + m] = (float)(Iq[t * 6 + m] / s);
  }
}

// ---------------------------------------------------------------------------
// dense layers on the matrix cores: C[M x N] = act(A[M x K] B[K x N] + bias),
// element (m,k) of A at A[m*sam + k*sak], (k,n) of B at B[k*sbk + n*sbn].
// 64x64 output tiles per block of four waves, each wave a 32x32 quadrant as
// 2x2 v_mfma_f32_16x16x4f32 tiles (FP32 in, FP32 accumulation); K in chunks
// of 16 staged through LDS.  Split-K over blockIdx.z writes partial sums to
// C + z*M*N (no bias/activation then).  Lane layouts of the instruction:
// A[i][k] from lane i + 16k, B[k][j] from lane j + 16k, D[i][j] in lane
// j + 16(i/4), element i % 4.
// ---------------------------------------------------------------------------
enum { ACT_NONE = 0, ACT_TANH = 1 };
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const float* __restrict__ A, int64_t sam,
                                              int64_t sak, const float* __restrict__ B, int64_t sbk, int64_t sbn,
                                              const float* __restrict__ bias, int act, float* C, int kchunk) {
  __shared__ float As[16][64 + 4];
  __shared__ float Bs[16][64 + 4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 15, kq = lane >> 4;
  const int rb = (wave >> 1) * 32, cb = (wave & 1) * 32;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int kk = e / 64, mm = e % 64;
      const int gm = m0 + mm, gk = k0 + kk;
      As[kk][mm] = (gm < M && gk < ke) ? A[gm * sam + gk * sak] : 0.f;
      const int gn = n0 + mm;
      Bs[kk][mm] = (gn < N && gk < ke) ? B[gk * sbk + gn * sbn] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      float av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = As[kk + kq][rb + 16 * t + i];
        bv[t] = Bs[kk + kq][cb + 16 * t + i];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  float* Cz = C + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int gn = n0 + cb + 16 * b + i;
      if (gn >= N) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gm = m0 + rb + 16 * a + 4 * kq + q;
        if (gm >= M) continue;
        float x = acc[a][b][q];
        if (bias) x += bias[gn];
        if (act == ACT_TANH) x = tanhf(x);
        Cz[(int64_t)gm * N + gn] = x;
      }
    }
}

// out[k] = sum_z part[z][k] (fixed order), k < n
__global__ void k_sum_parts(const float* __restrict__ part, int nz, int64_t n, float* out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  float s = 0;
  for (int z = 0; z < nz; ++z) s += part[z * n + k];
  out[k] = s;
}

// column sums of D [rows x cols] (bias gradients), one block per column
__global__ void k_colsum(const float* __restrict__ D, int rows, int cols, float* out) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  float s = 0;
  for (int r = threadIdx.x; r < rows; r += 256) s += D[(int64_t)r * cols + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

// D *= (1 - H^2)  (tanh derivative through the layer output H)
__global__ void k_tanh_back(float* D, const float* __restrict__ H, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) D[k] *= 1.f - H[k] * H[k];
}

// out[0] = sum of the n partial sums divided by div (fixed order, one block)
__global__ void k_loss_total(const double* __restrict__ part, int n, double div, double* out) {
  __shared__ double red[256];
  double a = 0;
  for (int k = threadIdx.x; k < n; k += 256) a += part[k];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0] / div;
}

// dY = 2 (Y - T) / n  and per-block partial sums of (Y - T)^2
__global__ void k_mse(const float* __restrict__ Y, const float* __restrict__ T, int64_t n, float* dY,
                      double* part) {
  __shared__ double red[256];
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double e2 = 0;
  if (k < n) {
    const float e = Y[k] - T[k];
    dY[k] = 2.f * e / (float)n;
    e2 = (double)e * e;
  }
  red[threadIdx.x] = e2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_adam(float* th, float* m, float* v, const float* __restrict__ g, int n, float lr, float b1,
                       float b2, float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  th[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + 1e-8f);
}

// rows idx of X (NIN) and T (NOUT), standardised with norm
__global__ void k_gather_std(const float* __restrict__ X, const float* __restrict__ T, const int64_t* __restrict__ idx,
                             int B, const float* __restrict__ norm, float* Xb, float* Tb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int64_t r = idx[b];
  for (int k = 0; k < NIN; ++k) Xb[b * NIN + k] = (X[r * NIN + k] - norm[k]) / norm[NIN + k];
  if (T) {
    const int c = row_class(X + r * NIN);
    for (int k = 0; k < NOUT; ++k)
      Tb[b * NOUT + k] = (T[r * NOUT + k] - norm[OUT_MU + c * NOUT + k]) / norm[OUT_SD + c * NOUT + k];
  }
}

// column mean/std of D [rows x cols] into mu[c], sd[c] (FP64 sums)
__global__ void k_colstats(const float* __restrict__ D, int64_t rows, int cols, float* mu, float* sd) {
  __shared__ double s1[256], s2[256];
  const int c = blockIdx.x;
  double a = 0, b = 0;
  for (int64_t r = threadIdx.x; r < rows; r += 256) {
    const double x = D[r * cols + c];
    a += x;
    b += x * x;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s1[threadIdx.x] += s1[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m = s1[0] / rows;
    const double var = fmax(s2[0] / rows - m * m, 0.0);
    mu[c] = (float)m;
    sd[c] = (float)fmax(sqrt(var), 1e-6 * fmax(1.0, fabs(m)));
  }
}

// surrogate entries: I = I3x3 + h^k (t * sd + mu); gate on the calibrated
// error of (class, distance bin); write entries of gated pairs (or of all
// pairs when all != 0) and flag gated pairs for the cubature to skip
// gate of a pair: its class's calibrated error estimate in the bin of its
// distance ratio is within tol
__device__ inline bool mlp_gated(const float* __restrict__ cal, int cls_index, float dr, double tol) {
  const int ci = cls_index - 1;
  const float* edges = cal + ci * (NBIN + 1);
  const float* est = cal + NCLS * (NBIN + 1) + ci * NBIN;
  int b = 0;
  while (b < NBIN - 1 && dr >= edges[b + 1]) ++b;
  return est[b] <= tol;
}

// the pairs whose prediction is used (gated, or every pair with all != 0),
// decided from the pair's class and distance ratio alone
__global__ void k_mlp_gate(NearArgs a, int cls_index, const Item* __restrict__ items, int64_t n,
                           const float* __restrict__ cal, double tol, int all, float* dr, int32_t* flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const Item it = items[t];
  const float d = (float)pair_dratio(a, it.i, it.j);
  dr[t] = d;
  flag[t] = (all || mlp_gated(cal, cls_index, d, tol)) ? 1 : 0;
}

// features, 3x3 integrals and h of the flagged pairs, packed in pair order
__global__ void k_mlp_prepare_packed(NearArgs a, int cls, const Item* __restrict__ items, int64_t n,
                                     const int32_t* __restrict__ flag, const int32_t* __restrict__ pos, float* X,
                                     double* I3, double* hh) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n || !flag[t]) return;
  const int64_t q = pos[t];
  const Item it = items[t];
  double h, d;
  float f[NIN];
  pair_features(a, cls, it.i, it.j, f, &h, &d);
  for (int k = 0; k < NIN; ++k) X[q * NIN + k] = f[k];
  double I[6];
  regular_pair(a, it.i, it.j, I);
  for (int m = 0; m < 6; ++m) I3[q * 6 + m] = I[m];
  hh[q] = h;
}

__global__ void k_mlp_apply(NearArgs a, int cls, int cls_index, const Item* __restrict__ items, int64_t n,
                            const int32_t* __restrict__ pos,
                            const float* __restrict__ tn, const float* __restrict__ norm, const double* __restrict__ I3,
                            const double* __restrict__ hh, const float* __restrict__ dr, const float* __restrict__ cal,
                            double tol, int all, double4* ent, uint8_t* skip, unsigned long long* n_gated) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool gated = false;
  if (t < n) {
    const int ci = cls_index - 1;
    gated = mlp_gated(cal, cls_index, dr[t], tol);
    const Item it = items[t];
    if (gated || all) {
      const int64_t q = pos[t];   // row of this pair among the predicted ones
      double I[6];
      for (int m = 0; m < 6; ++m)
        I[m] = I3[q * 6 + m] + hpow(hh[q], m) * ((double)tn[q * NOUT + m] * norm[OUT_SD + ci * NOUT + m] +
                                                 norm[OUT_MU + ci * NOUT + m]);
      write_pair(a, cls, it.i, it.j, it.ent, I, ent);
    }
    skip[t] = gated ? 1 : 0;
  }
  const unsigned long long mask = __ballot(gated);
  if ((threadIdx.x & 63) == 0 && mask) atomicAdd(n_gated, (unsigned long long)__popcll(mask));
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static void gemm(int M, int N, int K, const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk,
                 int64_t sbn, const float* bias, int act, float* C, hipStream_t s, int splitk = 1) {
  const int kchunk = ((K + splitk - 1) / splitk + 15) / 16 * 16;
  dim3 g((N + 63) / 64, (M + 63) / 64, splitk);
  k_gemm<<<g, 256, 0, s>>>(M, N, K, A, sam, sak, B, sbk, sbn, bias, act, C, kchunk);
}

struct Net {
  const float* th;
  int B;
  float *h1, *h2, *h3, *y;
};

static void forward(const Net& n, const float* X, hipStream_t s) {
  gemm(n.B, NH, NIN, X, NIN, 1, n.th + OFF_W1, NH, 1, n.th + OFF_B1, ACT_TANH, n.h1, s);
  gemm(n.B, NH, NH, n.h1, NH, 1, n.th + OFF_W2, NH, 1, n.th + OFF_B2, ACT_TANH, n.h2, s);
  gemm(n.B, NH, NH, n.h2, NH, 1, n.th + OFF_W3, NH, 1, n.th + OFF_B3, ACT_TANH, n.h3, s);
  gemm(n.B, NOUT, NH, n.h3, NH, 1, n.th + OFF_W4, NOUT, 1, n.th + OFF_B4, ACT_NONE, n.y, s);
}

struct Work {
  Tmp h1, h2, h3, y, d1, d2, d3, dy, part, grad, lpart;
  int B = 0, S = 0;
  int alloc(int B_) {
    B = B_;
    S = std::max(1, std::min(64, B / 256));
    FAGBI_TRY(h1.alloc((size_t)B * NH * 4));
    FAGBI_TRY(h2.alloc((size_t)B * NH * 4));
    FAGBI_TRY(h3.alloc((size_t)B * NH * 4));
    FAGBI_TRY(y.alloc((size_t)B * NOUT * 4));
    FAGBI_TRY(d1.alloc((size_t)B * NH * 4));
    FAGBI_TRY(d2.alloc((size_t)B * NH * 4));
    FAGBI_TRY(d3.alloc((size_t)B * NH * 4));
    FAGBI_TRY(dy.alloc((size_t)B * NOUT * 4));
    FAGBI_TRY(part.alloc((size_t)S * NH * NH * 4));
    FAGBI_TRY(grad.alloc((size_t)NPAR * 4));
    FAGBI_TRY(lpart.alloc((size_t)((B * NOUT + 255) / 256) * 8));
    return 0;
  }
};

// loss and gradient of the mean squared error over one batch (X, T already
// standardised); grad into w.grad
static void loss_grad(const float* th, const float* X, const float* T, Work& w, hipStream_t s) {
  Net n{th, w.B, w.h1.as<float>(), w.h2.as<float>(), w.h3.as<float>(), w.y.as<float>()};
  forward(n, X, s);
  const int64_t ny = (int64_t)w.B * NOUT;
  k_mse<<<(unsigned)((ny + 255) / 256), 256, 0, s>>>(n.y, T, ny, w.dy.as<float>(), w.lpart.as<double>());
  float* g = w.grad.as<float>();
  float* part = w.part.as<float>();
  auto wgrad = [&](const float* H, int in, const float* D, int out, int offW, int offB) {
    // dW[in x out] = H^T D, split over the batch; db = column sums of D
    gemm(in, out, w.B, H, 1, in, D, out, 1, nullptr, ACT_NONE, part, s, w.S);
    const int64_t nw = (int64_t)in * out;
    k_sum_parts<<<(unsigned)((nw + 255) / 256), 256, 0, s>>>(part, w.S, nw, g + offW);
    k_colsum<<<out, 256, 0, s>>>(D, w.B, out, g + offB);
  };
  auto dgrad = [&](const float* D, int out, int offW, int in, const float* Hprev, float* Dprev) {
    // Dprev[B x in] = D W^T, times the tanh derivative of Hprev
    gemm(w.B, in, out, D, out, 1, th + offW, 1, out, nullptr, ACT_NONE, Dprev, s);
    const int64_t nn = (int64_t)w.B * in;
    k_tanh_back<<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(Dprev, Hprev, nn);
  };
  wgrad(n.h3, NH, w.dy.as<float>(), NOUT, OFF_W4, OFF_B4);
  dgrad(w.dy.as<float>(), NOUT, OFF_W4, NH, n.h3, w.d3.as<float>());
  wgrad(n.h2, NH, w.d3.as<float>(), NH, OFF_W3, OFF_B3);
  dgrad(w.d3.as<float>(), NH, OFF_W3, NH, n.h2, w.d2.as<float>());
  wgrad(n.h1, NH, w.d2.as<float>(), NH, OFF_W2, OFF_B2);
  dgrad(w.d2.as<float>(), NH, OFF_W2, NH, n.h1, w.d1.as<float>());
  wgrad(X, NIN, w.d1.as<float>(), NH, OFF_W1, OFF_B1);
}

static uint64_t splitmix(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static double uniform01(uint64_t& x) { return (splitmix(x) >> 11) * (1.0 / 9007199254740992.0); }

static int ensure_net(fagbi_handle* h) {
  if (h->mlp_blob.size() != (size_t)NBLOB) return set_error(FAGBI_E_STATE, "surrogate network not trained or set");
  if (!h->d_mlp_theta.p) {
    FAGBI_TRY(h->upload(h->d_mlp_theta, h->mlp_blob.data(), NPAR * 4));
    FAGBI_TRY(h->upload(h->d_mlp_norm, h->mlp_blob.data() + NPAR, (NNORM + NCAL) * 4));
  }
  return 0;
}

// ---------------------------------------------------------------------------
// fused inference on the matrix cores: one block of 4 waves per 64 rows,
// each wave owns 16 rows; every layer is a sequence of
// v_mfma_f32_16x16x4f32 over K with the weights read straight from the
// (L2-resident, 140 KB) parameter vector and each wave's activations kept in
// its own LDS rows between layers, so several blocks share a CU.
// Lane layouts of the 16x16x4 FP32 instruction: A[i][k] from lane i + 16k,
// B[k][j] from lane j + 16k, D[i][j] in lane j + 16(i/4), element i % 4.
// ---------------------------------------------------------------------------
constexpr int IR = 64;               // rows per block
constexpr int AST = NH + 4;          // activation row stride (A reads: 2-way banks)

// acc[t] = bias + act[16 x K] * W[K x N] for column tiles t < ntile (W
// row-major [K][N]; columns >= N read as 0)
__device__ inline void mlp_layer(const float* act, const float* __restrict__ W, const float* __restrict__ bias,
                                 int K, int N, int ntile, int lane, f32x4* acc) {
  const int j = lane & 15, kq = lane >> 4;
  for (int t = 0; t < ntile; ++t) {
    const int col = t * 16 + j;
    const float b = col < N ? bias[col] : 0.f;
    acc[t] = f32x4{b, b, b, b};
  }
  for (int k0 = 0; k0 < K; k0 += 4) {
    const float av = act[j * AST + k0 + kq];
    const float* wr = W + (int64_t)(k0 + kq) * N + j;
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (t < ntile) {
        const float bv = (t * 16 + j) < N ? wr[t * 16] : 0.f;
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0, 0, 0);
      }
  }
}

// out[r] = network(standardised X[r]) (standardised, or in target units when
// destd is set: times the class's output sd plus its mean)
__global__ void __launch_bounds__(256) k_mlp_infer(const float* __restrict__ X, int64_t n_host,
                                                   const int32_t* __restrict__ n_dev,
                                                   const float* __restrict__ th, const float* __restrict__ norm,
                                                   int destd, float* out) {
  __shared__ float act_all[4 * 16 * AST];
  // rows: n_host, or the count in device memory (the grid covers n_host rows
  // and the blocks beyond the count leave at once)
  const int64_t n = n_dev ? (int64_t)*n_dev : n_host;
  if ((int64_t)blockIdx.x * IR >= n) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  float* act = act_all + wave * 16 * AST;
  const int64_t r0 = (int64_t)blockIdx.x * IR + wave * 16;
  // standardised inputs of this wave's rows
  for (int e = lane; e < 16 * NIN; e += 64) {
    const int r = e / NIN, k = e - r * NIN;
    const int64_t g = r0 + r;
    act[r * AST + k] = g < n ? (X[g * NIN + k] - norm[k]) / norm[NIN + k] : 0.f;
  }
  __syncthreads();
  f32x4 acc[8];
  mlp_layer(act, th + OFF_W1, th + OFF_B1, NIN, NH, 8, lane, acc);
  for (int l = 0; l < 3; ++l) {
    // every read of act by this layer is issued before the overwrite below
    // (program order within the wave); the barrier orders the writes before
    // the next layer's reads
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) act[(4 * (lane >> 4) + q) * AST + t * 16 + (lane & 15)] = tanhf(acc[t][q]);
    __syncthreads();
    if (l < 2)
      mlp_layer(act, th + (l == 0 ? OFF_W2 : OFF_W3), th + (l == 0 ? OFF_B2 : OFF_B3), NH, NH, 8, lane, acc);
    else
      mlp_layer(act, th + OFF_W4, th + OFF_B4, NH, NOUT, 1, lane, acc);
  }
  const int j = lane & 15;
  if (j < NOUT)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t g = r0 + 4 * (lane >> 4) + q;
      if (g < n) {
        float y = acc[0][q];
        if (destd) {
          const int c = row_class(X + g * NIN);
          y = y * norm[OUT_SD + c * NOUT + j] + norm[OUT_MU + c * NOUT + j];
        }
        out[g * NOUT + j] = y;
      }
    }
}

static int infer(fagbi_handle* h, const float* Xraw, int64_t n, int destd, float* out, hipStream_t s,
                 const int32_t* n_dev = nullptr) {
  if (n <= 0) return 0;
  k_mlp_infer<<<(unsigned)((n + IR - 1) / IR), 256, 0, s>>>(Xraw, n, n_dev, h->d_mlp_theta.as<float>(),
                                                             h->d_mlp_norm.as<float>(), destd, out);
  FAGBI_HIP(hipGetLastError());
  return 0;
}

int mlp_assembly_stage(fagbi_handle* h, hipStream_t s) {
  FAGBI_TRY(ensure_net(h));
  NearArgs a = near_args(h);
  const float* norm = h->d_mlp_norm.as<float>();
  const float* cal = norm + NNORM;
  Tmp cnt;
  FAGBI_TRY(cnt.alloc(8));
  FAGBI_HIP(hipMemsetAsync(cnt.p, 0, 8, s));
  const int all = h->prm.mlp_mode == FAGBI_MLP_PRECOND ? 1 : 0;
  // one set of chunk buffers for all classes; the chunks run back to back in
  // stream order.  Per chunk: the gate of every pair (class and distance
  // ratio), a scan of the flags, features and 3x3 integrals of the flagged
  // pairs only (packed), inference over the packed rows (their count read on
  // the device, so no host round trip), and the entries of the flagged pairs
  const int64_t CH = 1 << 20;
  int64_t cm = 1;
  for (int k = 1; k < 4; ++k) cm = std::max(cm, std::min<int64_t>(h->wl_n[k], CH));
  Tmp Xp, I3, hh, dr, tn, flag, pos, part;
  FAGBI_TRY(Xp.alloc((size_t)cm * NIN * 4));
  FAGBI_TRY(flag.alloc((size_t)cm * 4));
  FAGBI_TRY(pos.alloc((size_t)(cm + 1) * 4));
  FAGBI_TRY(part.alloc((size_t)scan_part_size(cm) * 4));
  FAGBI_TRY(I3.alloc((size_t)cm * 6 * 8));
  FAGBI_TRY(hh.alloc((size_t)cm * 8));
  FAGBI_TRY(dr.alloc((size_t)cm * 4));
  FAGBI_TRY(tn.alloc((size_t)cm * NOUT * 4));
  for (int k = 1; k < 4; ++k) {
    const int64_t m = h->wl_n[k];
    FAGBI_TRY(h->alloc(h->d_mlp_skip[k], (size_t)std::max<int64_t>(m, 1)));
    for (int64_t r0 = 0; r0 < m; r0 += CH) {
      const int64_t c = std::min<int64_t>(CH, m - r0);
      const Item* it = h->d_wl[k].as<Item>() + r0;
      const unsigned g = (unsigned)((c + 255) / 256);
      k_mlp_gate<<<g, 256, 0, s>>>(a, k, it, c, cal, h->prm.mlp_gate_tol, all, dr.as<float>(), flag.as<int32_t>());
      FAGBI_TRY((device_scan<int32_t, int32_t>(flag.as<int32_t>(), c, pos.as<int32_t>(), part.as<int32_t>(), s)));
      k_mlp_prepare_packed<<<g, 256, 0, s>>>(a, k + 1, it, c, flag.as<int32_t>(), pos.as<int32_t>(),
                                             Xp.as<float>(), I3.as<double>(), hh.as<double>());
      FAGBI_TRY(infer(h, Xp.as<float>(), c, 0, tn.as<float>(), s, pos.as<int32_t>() + c));
      k_mlp_apply<<<g, 256, 0, s>>>(a, k + 1, k, it, c, pos.as<int32_t>(), tn.as<float>(), norm, I3.as<double>(),
                                    hh.as<double>(),
                                    dr.as<float>(), cal, h->prm.mlp_gate_tol, all, h->d_E64.as<double4>(),
                                    h->d_mlp_skip[k].as<uint8_t>() + r0, cnt.as<unsigned long long>());
      FAGBI_HIP(hipGetLastError());
    }
  }
  unsigned long long ng = 0;
  FAGBI_HIP(hipMemcpyAsync(&ng, cnt.p, 8, hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipStreamSynchronize(s));   // also before the chunk buffers are freed
  h->mlp_gated_pairs = (int64_t)ng;
  return 0;
}

}  // namespace fagbi

using namespace fagbi;

extern "C" {

int fagbi_mlp_dataset(fagbi_handle* h, int64_t max_pairs, float* X, float* T, float* aux, int64_t* n_out,
                      void* stream) {
  if (!h || !X || !T || !aux || !n_out || max_pairs < 1) return set_error(FAGBI_E_ARG, "bad argument");
  if (!h->near_ready) return set_error(FAGBI_E_STATE, "mlp_dataset before assemble_nearfield");
  hipStream_t s = (hipStream_t)stream;
  const int64_t total = h->wl_n[1] + h->wl_n[2] + h->wl_n[3];
  const int64_t stride = std::max<int64_t>(1, (total + max_pairs - 1) / max_pairs);
  NearArgs a = near_args(h);
  int64_t off = 0;
  for (int k = 1; k < 4; ++k) {
    const int64_t m = h->wl_n[k];
    if (m == 0) continue;
    // every stride-th item of this class
    const int64_t c = std::min<int64_t>((m + stride - 1) / stride, max_pairs - off);
    if (c <= 0) break;
    std::vector<Item> all(m), sel(c);
    FAGBI_HIP(hipMemcpy(all.data(), h->d_wl[k].p, m * sizeof(Item), hipMemcpyDeviceToHost));
    for (int64_t q = 0; q < c; ++q) sel[q] = all[q * stride];
    Tmp items, Iq, I3, hh, dr;
    FAGBI_TRY(items.alloc(c * sizeof(Item)));
    FAGBI_HIP(hipMemcpy(items.p, sel.data(), c * sizeof(Item), hipMemcpyHostToDevice));
    FAGBI_TRY(Iq.alloc(c * 6 * 8));
    FAGBI_TRY(I3.alloc(c * 6 * 8));
    FAGBI_TRY(hh.alloc(c * 8));
    FAGBI_TRY(dr.alloc(c * 4));
    // cubature labels for the selected items
    DBuf saved = h->d_wl[k];
    const int64_t saved_n = h->wl_n[k];
    h->d_wl[k].p = items.p;
    h->wl_n[k] = c;
    int r = run_singular(h, k, nullptr, Iq.as<double>(), s);
    h->d_wl[k] = saved;
    h->wl_n[k] = saved_n;
    FAGBI_TRY(r);
    const unsigned g = (unsigned)((c + 255) / 256);
    k_mlp_prepare<<<g, 256, 0, s>>>(a, k + 1, items.as<Item>(), c, X + off * NIN, I3.as<double>(), hh.as<double>(),
                                    dr.as<float>());
    k_mlp_targets<<<g, 256, 0, s>>>(k, Iq.as<double>(), I3.as<double>(), hh.as<double>(), dr.as<float>(), c,
                                    T + off * NOUT, aux + off * NAUX);
    FAGBI_HIP(hipGetLastError());
    FAGBI_HIP(hipStreamSynchronize(s));
    off += c;
  }
  *n_out = off;
  return 0;
}

int fagbi_mlp_train(fagbi_handle* h, const float* X, const float* T, const float* aux, int64_t n, int32_t epochs,
                    int32_t batch, float lr, uint64_t seed, float* loss_hist, void* stream) {
  if (!h || !X || !T || !aux || n < 100 || epochs < 1 || batch < 64 || !(lr > 0))
    return set_error(FAGBI_E_ARG, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  // every tenth row is held out for the gate calibration
  std::vector<int64_t> order, vrows;
  for (int64_t r = 0; r < n; ++r) (r % 10 == 9 ? vrows : order).push_back(r);
  const int64_t nval = (int64_t)vrows.size();
  const int64_t ntr = (int64_t)order.size();
  const int B = (int)std::min<int64_t>(batch, ntr);
  // normalisation (all rows; the class one-hot inputs are left as they are)
  FAGBI_TRY(h->alloc(h->d_mlp_norm, (NNORM + NCAL) * 4));
  float* norm = h->d_mlp_norm.as<float>();
  k_colstats<<<NIN, 256, 0, s>>>(X, n, NIN, norm, norm + NIN);
  std::vector<float> xall(n * NIN), tall(n * NOUT), aall(n * NAUX);
  FAGBI_HIP(hipStreamSynchronize(s));
  FAGBI_HIP(hipMemcpy(xall.data(), X, xall.size() * 4, hipMemcpyDeviceToHost));
  FAGBI_HIP(hipMemcpy(tall.data(), T, tall.size() * 4, hipMemcpyDeviceToHost));
  FAGBI_HIP(hipMemcpy(aall.data(), aux, aall.size() * 4, hipMemcpyDeviceToHost));
  {
    // the one-hot class inputs stay as they are; targets are standardised per
    // class (their corrections differ by an order of magnitude between classes)
    std::vector<float> nm(NNORM);
    FAGBI_HIP(hipMemcpyAsync(nm.data(), norm, 2 * NIN * 4, hipMemcpyDeviceToHost, s));
    FAGBI_HIP(hipStreamSynchronize(s));
    for (int k = 13; k < 16; ++k) {
      nm[k] = 0.f;
      nm[NIN + k] = 1.f;
    }
    double s1[3][NOUT] = {}, s2[3][NOUT] = {};
    int64_t cnt[3] = {};
    for (int64_t r = 0; r < n; ++r) {
      const int c = row_class(&xall[r * NIN]);
      ++cnt[c];
      for (int m = 0; m < NOUT; ++m) {
        s1[c][m] += tall[r * NOUT + m];
        s2[c][m] += (double)tall[r * NOUT + m] * tall[r * NOUT + m];
      }
    }
    for (int c = 0; c < 3; ++c)
      for (int m = 0; m < NOUT; ++m) {
        const double mu = cnt[c] ? s1[c][m] / cnt[c] : 0.0;
        const double var = cnt[c] ? std::max(s2[c][m] / cnt[c] - mu * mu, 0.0) : 1.0;
        nm[OUT_MU + c * NOUT + m] = (float)mu;
        nm[OUT_SD + c * NOUT + m] = (float)std::max(std::sqrt(var), 1e-12);
      }
    FAGBI_HIP(hipMemcpy(norm, nm.data(), NNORM * 4, hipMemcpyHostToDevice));
  }
  // Xavier-uniform initial weights from a counter-based generator
  std::vector<float> th(NPAR, 0.f);
  uint64_t st = seed;
  auto init = [&](int off, int fin, int fout) {
    const double a = std::sqrt(6.0 / (fin + fout));
    for (int k = 0; k < fin * fout; ++k) th[off + k] = (float)((2.0 * uniform01(st) - 1.0) * a);
  };
  init(OFF_W1, NIN, NH);
  init(OFF_W2, NH, NH);
  init(OFF_W3, NH, NH);
  init(OFF_W4, NH, NOUT);
  FAGBI_TRY(h->upload(h->d_mlp_theta, th.data(), NPAR * 4));
  FAGBI_TRY(h->alloc(h->d_mlp_m, NPAR * 4));
  FAGBI_TRY(h->alloc(h->d_mlp_v, NPAR * 4));
  FAGBI_HIP(hipMemsetAsync(h->d_mlp_m.p, 0, NPAR * 4, s));
  FAGBI_HIP(hipMemsetAsync(h->d_mlp_v.p, 0, NPAR * 4, s));
  Work w;
  FAGBI_TRY(w.alloc(B));
  Tmp xb, tb, idx, bl;
  FAGBI_TRY(xb.alloc((size_t)B * NIN * 4));
  FAGBI_TRY(tb.alloc((size_t)B * NOUT * 4));
  const int nb = (int)(ntr / B);
  FAGBI_TRY(idx.alloc((size_t)std::max(nb, 1) * B * 8));
  FAGBI_TRY(bl.alloc((size_t)std::max(nb, 1) * 8));
  const int nlp = (B * NOUT + 255) / 256;
  std::vector<double> lb(std::max(nb, 1));
  int step = 0;
  // the host shuffles the rows once per epoch and uploads the order in one
  // copy; each minibatch's loss stays on the device until the epoch ends
  for (int ep = 0; ep < epochs; ++ep) {
    for (int64_t k = ntr - 1; k > 0; --k) std::swap(order[k], order[(int64_t)(uniform01(st) * (k + 1))]);
    const float lr_ep = lr * (float)(0.5 * (1.0 + std::cos(3.14159265358979 * ep / epochs)));
    FAGBI_HIP(hipStreamSynchronize(s));   // the previous epoch's kernels have read idx
    FAGBI_HIP(hipMemcpy(idx.p, order.data(), (size_t)nb * B * 8, hipMemcpyHostToDevice));
    for (int bi = 0; bi < nb; ++bi) {
      k_gather_std<<<(B + 255) / 256, 256, 0, s>>>(X, T, idx.as<int64_t>() + (int64_t)bi * B, B, norm,
                                                   xb.as<float>(), tb.as<float>());
      loss_grad(h->d_mlp_theta.as<float>(), xb.as<float>(), tb.as<float>(), w, s);
      k_loss_total<<<1, 256, 0, s>>>(w.lpart.as<double>(), nlp, (double)B * NOUT, bl.as<double>() + bi);
      ++step;
      const float c1 = 1.f - std::pow(0.9f, (float)step), c2 = 1.f - std::pow(0.999f, (float)step);
      k_adam<<<(NPAR + 255) / 256, 256, 0, s>>>(h->d_mlp_theta.as<float>(), h->d_mlp_m.as<float>(),
                                                h->d_mlp_v.as<float>(), w.grad.as<float>(), NPAR, lr_ep, 0.9f,
                                                0.999f, c1, c2);
    }
    if (loss_hist && nb > 0) {
      FAGBI_HIP(hipMemcpyAsync(lb.data(), bl.p, (size_t)nb * 8, hipMemcpyDeviceToHost, s));
      FAGBI_HIP(hipStreamSynchronize(s));
      double lsum = 0;
      for (int bi = 0; bi < nb; ++bi) lsum += lb[bi];
      loss_hist[ep] = (float)(lsum / nb);
    }
  }
  FAGBI_HIP(hipGetLastError());
  // calibration on the held-out rows: per class, 8 bins of the distance ratio
  // (quantiles), value = 95th percentile of the per-pair error
  //   e = max_m |t_pred - t| / (|i_full| + 0.1 rms(i_full))
  Tmp pv, xv;
  FAGBI_TRY(pv.alloc((size_t)nval * NOUT * 4));
  FAGBI_TRY(xv.alloc((size_t)nval * NIN * 4));
  h->mlp_blob.assign(NBLOB, 0.f);
  FAGBI_HIP(hipStreamSynchronize(s));
  FAGBI_HIP(hipMemcpy(h->mlp_blob.data(), h->d_mlp_theta.p, NPAR * 4, hipMemcpyDeviceToHost));
  FAGBI_HIP(hipMemcpy(h->mlp_blob.data() + NPAR, norm, NNORM * 4, hipMemcpyDeviceToHost));
  std::vector<float> xvh(nval * NIN), tt(nval * NOUT), ax(nval * NAUX), tp(nval * NOUT);
  for (int64_t k = 0; k < nval; ++k) {
    memcpy(&xvh[k * NIN], &xall[vrows[k] * NIN], NIN * 4);
    memcpy(&tt[k * NOUT], &tall[vrows[k] * NOUT], NOUT * 4);
    memcpy(&ax[k * NAUX], &aall[vrows[k] * NAUX], NAUX * 4);
  }
  FAGBI_HIP(hipMemcpy(xv.p, xvh.data(), xvh.size() * 4, hipMemcpyHostToDevice));
  FAGBI_TRY(infer(h, xv.as<float>(), nval, 0, pv.as<float>(), s));
  FAGBI_HIP(hipStreamSynchronize(s));
  FAGBI_HIP(hipMemcpy(tp.data(), pv.p, tp.size() * 4, hipMemcpyDeviceToHost));
  const float* nm = h->mlp_blob.data() + NPAR;
  double rms[NOUT] = {};
  for (int64_t r = 0; r < nval; ++r)
    for (int m = 0; m < NOUT; ++m) rms[m] += (double)ax[r * NAUX + 2 + m] * ax[r * NAUX + 2 + m];
  for (int m = 0; m < NOUT; ++m) rms[m] = std::sqrt(rms[m] / nval);
  float* cal = h->mlp_blob.data() + NPAR + NNORM;
  for (int c = 0; c < NCLS; ++c) {
    std::vector<std::pair<float, float>> de;   // (distance ratio, error)
    for (int64_t r = 0; r < nval; ++r) {
      if ((int)ax[r * NAUX] != c) continue;
      double e = 0;
      for (int m = 0; m < NOUT; ++m) {
        const double pred = (double)tp[r * NOUT + m] * nm[OUT_SD + c * NOUT + m] + nm[OUT_MU + c * NOUT + m];
        e = std::max(e, std::fabs(pred - tt[r * NOUT + m]) / (std::fabs(ax[r * NAUX + 2 + m]) + 0.1 * rms[m]));
      }
      de.push_back({ax[r * NAUX + 1], (float)e});
    }
    float* edges = cal + c * (NBIN + 1);
    float* est = cal + NCLS * (NBIN + 1) + c * NBIN;
    if (de.empty()) {
      for (int b = 0; b <= NBIN; ++b) edges[b] = 1e30f;
      for (int b = 0; b < NBIN; ++b) est[b] = 1e30f;   // never gated
      continue;
    }
    std::sort(de.begin(), de.end());
    for (int b = 0; b <= NBIN; ++b) edges[b] = de[std::min<size_t>(de.size() - 1, de.size() * b / NBIN)].first;
    edges[0] = 0.f;
    for (int b = 0; b < NBIN; ++b) {
      const size_t lo = de.size() * b / NBIN, hi = std::max(lo + 1, de.size() * (b + 1) / NBIN);
      std::vector<float> e;
      for (size_t k = lo; k < std::min(hi, de.size()); ++k) e.push_back(de[k].second);
      std::sort(e.begin(), e.end());
      est[b] = e[std::min(e.size() - 1, (size_t)(0.95 * e.size()))];
    }
  }
  FAGBI_HIP(hipMemcpy(norm + NNORM, cal, NCAL * 4, hipMemcpyHostToDevice));
  h->mlp_ready = true;
  return 0;
}

int fagbi_mlp_forward(fagbi_handle* h, const float* X, float* Y, int64_t n, void* stream) {
  if (!h || !X || !Y || n < 1) return set_error(FAGBI_E_ARG, "bad argument");
  FAGBI_TRY(ensure_net(h));
  hipStream_t s = (hipStream_t)stream;
  FAGBI_TRY(infer(h, X, n, 1, Y, s));
  return 0;
}

int fagbi_mlp_grad(fagbi_handle* h, const float* theta, const float* X, const float* T, int32_t n, float* loss,
                   float* grad, void* stream) {
  if (!h || !theta || !X || !T || !loss || !grad || n < 1 || n > 65536) return set_error(FAGBI_E_ARG, "bad argument");
  hipStream_t s = (hipStream_t)stream;
  Tmp th;
  FAGBI_TRY(th.alloc(NPAR * 4));
  FAGBI_HIP(hipMemcpy(th.p, theta, NPAR * 4, hipMemcpyHostToDevice));
  Work w;
  FAGBI_TRY(w.alloc(n));
  loss_grad(th.as<float>(), X, T, w, s);
  const int nlp = (n * NOUT + 255) / 256;
  std::vector<double> lp(nlp);
  FAGBI_HIP(hipMemcpyAsync(lp.data(), w.lpart.p, nlp * 8, hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipMemcpyAsync(grad, w.grad.p, NPAR * 4, hipMemcpyDeviceToHost, s));
  FAGBI_HIP(hipStreamSynchronize(s));
  double l = 0;
  for (double v : lp) l += v;
  *loss = (float)(l / ((double)n * NOUT));
  return 0;
}

int fagbi_mlp_get_weights(fagbi_handle* h, float* blob, int64_t n) {
  if (!h || !blob || n != NBLOB) return set_error(FAGBI_E_ARG, "blob must hold %d floats", NBLOB);
  if (h->mlp_blob.size() != (size_t)NBLOB) return set_error(FAGBI_E_STATE, "no trained network");
  memcpy(blob, h->mlp_blob.data(), NBLOB * 4);
  return 0;
}

int fagbi_mlp_set_weights(fagbi_handle* h, const float* blob, int64_t n) {
  if (!h || !blob || n != NBLOB) return set_error(FAGBI_E_ARG, "blob must hold %d floats", NBLOB);
  h->mlp_blob.assign(blob, blob + NBLOB);
  FAGBI_TRY(h->upload(h->d_mlp_theta, h->mlp_blob.data(), NPAR * 4));
  FAGBI_TRY(h->upload(h->d_mlp_norm, h->mlp_blob.data() + NPAR, (NNORM + NCAL) * 4));
  h->mlp_ready = true;
  return 0;
}

int fagbi_get_mlp_stats(fagbi_handle* h, int64_t* gated_pairs, int64_t* candidate_pairs) {
  if (!h || !gated_pairs || !candidate_pairs) return set_error(FAGBI_E_ARG, "null argument");
  *gated_pairs = h->mlp_gated_pairs;
  *candidate_pairs = h->wl_n[1] + h->wl_n[2] + h->wl_n[3];
  return 0;
}

}  // extern "C"
