// Device-wide exclusive prefix sums (internal): reduce per tile, scan the
// tile sums in one block, then scan each tile with its offset.  Integer
// inputs only, so the results do not depend on the launch shape.
#pragma once
#include <algorithm>

#include "internal.h"

namespace fagbi {
namespace scan_detail {

constexpr int TB = 256;                  // threads per block (4 waves)
constexpr int IPT = 8;                   // items per thread
constexpr int TILE = TB * IPT;

template <typename T>
__device__ inline T block_exclusive_scan(T v, T* lds, T& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[w] = x;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < TB / 64; ++i) {
    if (i < w) off += lds[i];
    tot += lds[i];
  }
  __syncthreads();
  total = tot;
  return off + x - v;
}

// per-tile sums of the input
template <typename TI, typename TO>
__global__ void __launch_bounds__(TB) k_scan_reduce(const TI* __restrict__ in, int64_t n, TO* part) {
  __shared__ TO lds[TB / 64];
  const int64_t base = (int64_t)blockIdx.x * TILE + threadIdx.x * IPT;
  TO s = 0;
#pragma unroll
  for (int j = 0; j < IPT; ++j)
    if (base + j < n) s += (TO)in[base + j];
  TO tot;
  block_exclusive_scan<TO>(s, lds, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// exclusive scan of the tile sums in place (one block), total at part[nb]
template <typename TO>
__global__ void __launch_bounds__(TB) k_scan_part(TO* part, int64_t nb) {
  __shared__ TO lds[TB / 64];
  TO carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += TB) {
    const int64_t i = b0 + threadIdx.x;
    const TO v = i < nb ? part[i] : (TO)0;
    TO tot;
    const TO ex = block_exclusive_scan<TO>(v, lds, tot);
    if (i < nb) part[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) part[nb] = carry;
}

// out[i] = sum of in[0..i), out[n] = total
template <typename TI, typename TO>
__global__ void __launch_bounds__(TB) k_scan_down(const TI* __restrict__ in, int64_t n, const TO* __restrict__ part,
                                                  int64_t nb, TO* out) {
  __shared__ TO lds[TB / 64];
  const int64_t base = (int64_t)blockIdx.x * TILE + threadIdx.x * IPT;
  TO v[IPT];
  TO s = 0;
#pragma unroll
  for (int j = 0; j < IPT; ++j) {
    v[j] = base + j < n ? (TO)in[base + j] : (TO)0;
    s += v[j];
  }
  TO tot;
  TO run = part[blockIdx.x] + block_exclusive_scan<TO>(s, lds, tot);
#pragma unroll
  for (int j = 0; j < IPT; ++j)
    if (base + j < n) {
      out[base + j] = run;
      run += v[j];
    }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = part[nb];
}

}  // namespace scan_detail

// tile sums needed by device_scan for n items (plus one for the total)
inline int64_t scan_part_size(int64_t n) {
  return std::max<int64_t>(1, (n + scan_detail::TILE - 1) / scan_detail::TILE) + 1;
}

// out[i] = sum of in[0..i) for i <= n (out[n] = total); part holds
// scan_part_size(n) elements of scratch
template <typename TI, typename TO>
int device_scan(const TI* in, int64_t n, TO* out, TO* part, hipStream_t s) {
  using namespace scan_detail;
  const int64_t nb = scan_part_size(n) - 1;
  k_scan_reduce<TI, TO><<<(unsigned)nb, TB, 0, s>>>(in, n, part);
  k_scan_part<TO><<<1, TB, 0, s>>>(part, nb);
  k_scan_down<TI, TO><<<(unsigned)nb, TB, 0, s>>>(in, n, part, nb, out);
  FAGBI_HIP(hipGetLastError());
  return 0;
}

}  // namespace fagbi
