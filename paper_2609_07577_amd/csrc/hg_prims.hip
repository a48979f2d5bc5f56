// Device primitives: fills, device-resident sizes, exclusive scans.
//
// The scans are reduce-then-scan over a fixed grid so that the element count
// can live in device memory (no host read-back between kernels).
#include "hg_internal.h"

namespace hg {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kScanBlocks = 256;

template <typename T>
__global__ void fill_kernel(T* __restrict__ p, T v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void set_dims_kernel(Dims* d, int64_t V, int64_t E, int64_t P) {
  d->V = V;
  d->E = E;
  d->P = P;
}

__device__ inline int64_t wave_inclusive_scan(int64_t v) {
  int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int64_t t = __shfl_up(v, d, kWave);
    if (lane >= d) v += t;
  }
  return v;
}

// Exclusive block scan of one value per thread; returns the exclusive prefix
// and writes the block total to *total.
__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t* total) {
  __shared__ int64_t wsum[kScanThreads / kWave];
  int lane = threadIdx.x & (kWave - 1);
  int wid = threadIdx.x / kWave;
  int64_t inc = wave_inclusive_scan(v);
  if (lane == kWave - 1) wsum[wid] = inc;
  __syncthreads();
  int64_t base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kScanThreads / kWave; ++k) {
    int64_t s = wsum[k];
    if (k < wid) base += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

__device__ inline void chunk_range(int64_t n, int64_t& lo, int64_t& hi) {
  int64_t per = (n + kScanBlocks - 1) / kScanBlocks;
  per = (per + kScanTile - 1) / kScanTile * kScanTile;
  lo = (int64_t)blockIdx.x * per;
  hi = lo + per;
  if (lo > n) lo = n;
  if (hi > n) hi = n;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(
    const T* __restrict__ in, const int64_t* __restrict__ count, int64_t* __restrict__ partials) {
  int64_t n = *count;
  int64_t lo, hi;
  chunk_range(n, lo, hi);
  int64_t acc = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kScanThreads) acc += (int64_t)in[i];
  int64_t tot;
  block_exclusive_scan(acc, &tot);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void scan_top_kernel(int64_t* __restrict__ partials) {
  // kScanBlocks == kScanThreads: one partial per thread
  int64_t v = partials[threadIdx.x];
  int64_t tot;
  int64_t ex = block_exclusive_scan(v, &tot);
  partials[threadIdx.x] = ex;
  if (threadIdx.x == 0) partials[kScanBlocks] = tot;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_down_kernel(
    const T* __restrict__ in, int64_t* __restrict__ out, const int64_t* __restrict__ count,
    const int64_t* __restrict__ partials) {
  int64_t n = *count;
  int64_t lo, hi;
  chunk_range(n, lo, hi);
  int64_t carry = partials[blockIdx.x];
  for (int64_t t0 = lo; t0 < hi; t0 += kScanTile) {
    int64_t v[kScanItems];
    int64_t base = t0 + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      int64_t i = base + k;
      v[k] = i < hi ? (int64_t)in[i] : 0;
      s += v[k];
    }
    int64_t tot;
    int64_t ex = block_exclusive_scan(s, &tot) + carry;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      int64_t i = base + k;
      if (i < hi) out[i] = ex;
      ex += v[k];
    }
    carry += tot;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = partials[kScanBlocks];
}

template <typename T>
void exclusive_scan_impl(const T* in, int64_t* out, const int64_t* count, int64_t max_count,
                         int64_t* partials, hipStream_t s) {
  (void)max_count;
  scan_reduce_kernel<T><<<kScanBlocks, kScanThreads, 0, s>>>(in, count, partials);
  scan_top_kernel<<<1, kScanThreads, 0, s>>>(partials);
  scan_down_kernel<T><<<kScanBlocks, kScanThreads, 0, s>>>(in, out, count, partials);
}

}  // namespace

static_assert(kScanBlocks == kScanThreads, "scan_top assumes one partial per thread");

int scan_partials_size() { return kScanBlocks + 1; }

void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  fill_kernel<int32_t><<<grid_for(n, 256 * 4, 4096), 256, 0, s>>>(p, v, n);
}
void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  fill_kernel<int64_t><<<grid_for(n, 256 * 4, 4096), 256, 0, s>>>(p, v, n);
}
void fill_u64(uint64_t* p, uint64_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  fill_kernel<uint64_t><<<grid_for(n, 256 * 4, 4096), 256, 0, s>>>(p, v, n);
}
void set_dims(Dims* d, int64_t V, int64_t E, int64_t P, hipStream_t s) {
  set_dims_kernel<<<1, 1, 0, s>>>(d, V, E, P);
}

void exclusive_scan_i32(const int32_t* in, int64_t* out, const int64_t* count,
                        int64_t max_count, int64_t* partials, hipStream_t s) {
  exclusive_scan_impl<int32_t>(in, out, count, max_count, partials, s);
}
void exclusive_scan_i64(const int64_t* in, int64_t* out, const int64_t* count,
                        int64_t max_count, int64_t* partials, hipStream_t s) {
  exclusive_scan_impl<int64_t>(in, out, count, max_count, partials, s);
}

int device_cu_count() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    return 256;
  return cus;
}

}  // namespace hg
