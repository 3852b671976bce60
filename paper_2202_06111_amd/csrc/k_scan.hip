// Device-wide exclusive prefix sums (int64 results) used for CSR offsets,
// reverse-CSR offsets and cell compaction.  Tiles of kScanBlock * kScanItems
// elements: reduce each tile, then rescan each tile with its offset.  Up to
// kDirect tiles, each block of the second launch sums the tile totals before
// its own (L2-resident, a few loads per thread); beyond that the tile totals
// are scanned recursively first.
#include "gis_internal.h"

namespace gis {

namespace {

constexpr int64_t kTileElems = (int64_t)kScanBlock * kScanItems;

__device__ __forceinline__ int64_t block_exclusive(int64_t v, int64_t* lds, int64_t& total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int64_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wid] = x;
  __syncthreads();
  int64_t before = 0;
  total = 0;
  for (int w = 0; w < kScanBlock / 64; ++w) {
    before += w < wid ? lds[w] : 0;
    total += lds[w];
  }
  __syncthreads();
  return before + x - v;
}

// Element -> summand: the element itself, or for covering-index states the
// packed pair (leaf, hole << 32).
template <typename T>
struct Plain {
  __device__ static int64_t get(T v) { return (int64_t)v; }
};
struct LeafHole {
  __device__ static int64_t get(uint8_t st) {
    return (int64_t)(st == ST_LEAF) + ((int64_t)(st == ST_HOLE) << 32);
  }
};

template <typename T, typename C = Plain<T>>
__global__ __launch_bounds__(kScanBlock) void k_tile_sums(const T* in, int64_t n, int64_t* sums) {
  __shared__ int64_t lds[kScanBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kTileElems + (int64_t)threadIdx.x * kScanItems;
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += C::get(in[base + i]);
  int64_t total;
  block_exclusive(s, lds, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

constexpr int64_t kDirect = 8192;

template <typename T, typename C = Plain<T>>
__global__ __launch_bounds__(kScanBlock) void k_tile_scan(const T* in, int64_t n,
                                                          const int64_t* offsets,
                                                          const int64_t* sums, int64_t* out,
                                                          int64_t* d_total) {
  __shared__ int64_t lds[kScanBlock / 64];
  __shared__ int64_t s_off;
  if (sums) {  // this tile's offset: the totals of the tiles before it
    int64_t part = 0;
    for (int64_t i = threadIdx.x; i < (int64_t)blockIdx.x; i += kScanBlock) part += sums[i];
    int64_t tot;
    block_exclusive(part, lds, tot);
    if (threadIdx.x == 0) s_off = tot;
    __syncthreads();
  }
  const int64_t base = (int64_t)blockIdx.x * kTileElems + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? C::get(in[base + i]) : 0;
    s += v[i];
  }
  int64_t total;
  int64_t run = block_exclusive(s, lds, total) + (offsets ? offsets[blockIdx.x] : 0) +
                (sums ? s_off : 0);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (d_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanBlock - 1) *d_total = run;
}

size_t tmp_elems(int64_t n) {
  if (n <= kTileElems) return 0;
  const int64_t nb = (n + kTileElems - 1) / kTileElems;
  return (size_t)(2 * nb) + tmp_elems(nb);
}

template <typename T, typename C = Plain<T>>
int32_t scan_impl(const T* in, int64_t* out, int64_t n, int64_t* d_total, int64_t* tmp,
                  hipStream_t s) {
  if (n <= 0) return d_total ? fill_i64(d_total, 0, 1, s) : GIS_OK;
  if (n <= kTileElems) {
    hipLaunchKernelGGL((k_tile_scan<T, C>), dim3(1), dim3(kScanBlock), 0, s, in, n,
                       (const int64_t*)nullptr, (const int64_t*)nullptr, out, d_total);
    GIS_LAUNCH_CHECK("k_tile_scan");
    return GIS_OK;
  }
  const int64_t nb = (n + kTileElems - 1) / kTileElems;
  int64_t* sums = tmp;
  int64_t* offs = tmp + nb;
  hipLaunchKernelGGL((k_tile_sums<T, C>), dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n, sums);
  GIS_LAUNCH_CHECK("k_tile_sums");
  if (nb <= kDirect) {
    hipLaunchKernelGGL((k_tile_scan<T, C>), dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n,
                       (const int64_t*)nullptr, (const int64_t*)sums, out, d_total);
    GIS_LAUNCH_CHECK("k_tile_scan");
    return GIS_OK;
  }
  int32_t rc = scan_impl<int64_t>(sums, offs, nb, nullptr, tmp + 2 * nb, s);
  if (rc != GIS_OK) return rc;
  hipLaunchKernelGGL((k_tile_scan<T, C>), dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n,
                     (const int64_t*)offs, (const int64_t*)nullptr, out, d_total);
  GIS_LAUNCH_CHECK("k_tile_scan");
  return GIS_OK;
}

}  // namespace

size_t scan_tmp_bytes(int64_t n) { return (tmp_elems(n) + 1) * sizeof(int64_t); }

int32_t scan_exclusive_i64(const int64_t* in, int64_t* out, int64_t n, int64_t* d_total, void* tmp,
                           hipStream_t s) {
  return scan_impl<int64_t>(in, out, n, d_total, (int64_t*)tmp, s);
}
int32_t scan_exclusive_u8(const uint8_t* in, int64_t* out, int64_t n, int64_t* d_total, void* tmp,
                          hipStream_t s) {
  return scan_impl<uint8_t>(in, out, n, d_total, (int64_t*)tmp, s);
}
int32_t scan_exclusive_i32(const int32_t* in, int64_t* out, int64_t n, int64_t* d_total, void* tmp,
                           hipStream_t s) {
  return scan_impl<int32_t>(in, out, n, d_total, (int64_t*)tmp, s);
}
int32_t scan_leaf_hole(const uint8_t* state, int64_t* out, int64_t n, void* tmp, hipStream_t s) {
  return scan_impl<uint8_t, LeafHole>(state, out, n, out + n, (int64_t*)tmp, s);
}

}  // namespace gis
