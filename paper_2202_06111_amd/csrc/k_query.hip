// Point queries on a pruned covering: is a state in the kept set, and which
// inputs are admissible in its cell.  A state in X maps to the finest-level
// cell floor((x - lo) / w) (the last cell for x = hi); the covering index walk
// then finds the leaf that contains it, if any.
#include "gis_launch.h"

namespace gis {

namespace {

__global__ void k_query(CoverIndex ci, GridArgs g, const uint8_t* kept, const uint64_t* mask,
                        int32_t W, const double* states, int64_t n, uint8_t* member,
                        uint64_t* adm) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t k[kMaxDim];
    bool inside = true;
    for (int d = 0; d < g.n; ++d) {
      const double v = states[i * g.n + d];
      if (!(v >= g.lo[d] && v <= g.hi[d])) {
        inside = false;
        break;
      }
      const int64_t Nd = ci.dims[ci.lmax][d];
      int64_t kd = (int64_t)floor((v - g.lo[d]) / ldexp(g.w0[d], -ci.lmax));
      k[d] = kd > Nd - 1 ? Nd - 1 : kd;
    }
    int64_t cell = -1;
    if (inside) {
      if (ci.uniform) {
        int64_t lin = 0;
        for (int d = 0; d < g.n; ++d) lin = lin * ci.dims[0][d] + k[d];
        cell = lin;
      } else {
        for (int L = 0; L <= ci.lmax; ++L) {
          const int s = ci.lmax - L;
          int64_t lin = 0;
          for (int d = 0; d < g.n; ++d) lin = lin * ci.dims[L][d] + (k[d] >> s);
          const uint8_t st = ci.state[ci.off[L] + lin];
          if (st == ST_LEAF) {
            cell = (ci.pfx[ci.off[L] + lin] & 0xffffffffll) - ci.pbase;
            break;
          }
          if (st != ST_REFINED) break;
        }
      }
    }
    const bool in = cell >= 0 && kept[cell];
    if (member) member[i] = in ? 1 : 0;
    if (adm)
      for (int w = 0; w < W; ++w) adm[i * W + w] = in ? mask[cell * W + w] : 0;
  }
}

}  // namespace

int32_t launch_query(const CoverIndex& ci, const GridArgs& g, const uint8_t* kept,
                     const uint64_t* mask, int32_t mask_words, const double* states, int64_t n,
                     uint8_t* member, uint64_t* adm, hipStream_t s) {
  if (n == 0) return GIS_OK;
  int64_t nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  hipLaunchKernelGGL(k_query, dim3((unsigned)nb), dim3(256), 0, s, ci, g, kept, mask, mask_words,
                     states, n, member, adm);
  GIS_LAUNCH_CHECK("k_query");
  return GIS_OK;
}

}  // namespace gis
