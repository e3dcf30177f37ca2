// Plan-time point preparation (Section 6, eqs. x_tilde and nfsglft_rho):
// radius reduction for rho, the map x -> x~ = (arccos gamma(r), theta, phi)
// in FP64, grid coordinates u_j = N_j x~_j / (2 pi) split into an integer base
// cell and a fractional offset, and binning of the points into tiles of base
// cells (a stable radix sort on the tile-major cell key).
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>

#include "sgl_internal.h"

namespace sgl {

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

template <class T>
__device__ inline void load_xyz(const T *xyz, int64_t i, double &x, double &y, double &z) {
  x = (double)xyz[3 * i];
  y = (double)xyz[3 * i + 1];
  z = (double)xyz[3 * i + 2];
}

__device__ inline double point_r(double x, double y, double z) { return hypot(hypot(x, y), z); }

template <class T>
__global__ __launch_bounds__(256) void k_radius(const T *__restrict__ xyz, int64_t M,
                                                double *__restrict__ partial) {
  __shared__ double smax[256];
  __shared__ double sbad[256];
  double mx = 0.0, bad = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    double x, y, z;
    load_xyz(xyz, i, x, y, z);
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
      bad += 1.0;
    } else {
      mx = fmax(mx, point_r(x, y, z));
    }
  }
  smax[threadIdx.x] = mx;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
      sbad[threadIdx.x] += sbad[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = smax[0];
    partial[2 * blockIdx.x + 1] = sbad[0];
  }
}

struct PrepGeom {
  double rho;
  int N[3];
  int L[3], T[3];
  int nlo2;  // cells l2 < nlo2 come first in a dimension-0 slab of a tile (0: plain order)
};

// x~ of eq. x_tilde; t0 = arccos((2r - rho)/rho) written as
// 2 atan2(sqrt(rho - r), sqrt(r)), which is the same angle and is well
// conditioned at both ends.  theta, phi are taken as 0 where undefined (origin,
// z axis); every term that survives there does not depend on them.
__device__ inline void angles(double x, double y, double z, double rho, double &t0, double &t1, double &t2) {
  const double rxy = hypot(x, y);
  const double r = hypot(rxy, z);
  t1 = atan2(rxy, z);
  t2 = atan2(y, x);
  if (t2 < 0.0) t2 += kTwoPi;
  t0 = 2.0 * atan2(sqrt(fmax(rho - r, 0.0)), sqrt(r));
}

template <class T, class R>
__global__ __launch_bounds__(256) void k_prep(const T *__restrict__ xyz, int64_t M, PrepGeom g,
                                              uint32_t *__restrict__ keys, int32_t *__restrict__ idx,
                                              PointRec<R> *__restrict__ rec, double *__restrict__ tout) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= M) return;
  double x, y, z;
  load_xyz(xyz, i, x, y, z);
  double t[3];
  angles(x, y, z, g.rho, t[0], t[1], t[2]);
  int b[3];
  PointRec<R> pr;
  for (int j = 0; j < 3; ++j) {
    const double u = g.N[j] * t[j] / kTwoPi;
    double fb = floor(u);
    int bj = (int)fb;
    double fr = u - fb;
    if (j < 2) {
      // angles in [0, pi]: base cells 0 .. N_j/2
      if (bj > g.N[j] / 2) { bj = g.N[j] / 2; fr = 0.0; }
      if (bj < 0) { bj = 0; fr = 0.0; }
    } else {
      if (bj >= g.N[2]) bj -= g.N[2];
      if (bj < 0) bj += g.N[2];
    }
    b[j] = bj;
    pr.frac[j] = (R)fr;
  }
  pr.cell = pack_cell(b[0], b[1], b[2]);
  const uint32_t tile = (uint32_t)(((b[0] / g.L[0]) * g.T[1] + b[1] / g.L[1]) * g.T[2] + b[2] / g.L[2]);
  // order inside a tile: dimension-0 slabs, and inside a slab the cells with
  // l2 < nlo2 before the others, each class in (l1, l2) order (a bijection
  // onto the tile's cells)
  const int l0 = b[0] % g.L[0], l1 = b[1] % g.L[1], l2 = b[2] % g.L[2];
  const int nlo = g.nlo2, nhi = g.L[2] - g.nlo2;
  const int in_slab = nlo == 0 ? l1 * g.L[2] + l2 : (l2 < nlo ? l1 * nlo + l2 : g.L[1] * nlo + l1 * nhi + (l2 - nlo));
  const uint32_t local = (uint32_t)(l0 * g.L[1] * g.L[2] + in_slab);
  keys[i] = tile * (uint32_t)(g.L[0] * g.L[1] * g.L[2]) + local;
  idx[i] = (int32_t)i;
  rec[i] = pr;
  if (tout) {
    tout[i] = t[0];
    tout[M + i] = t[1];
    tout[2 * M + i] = t[2];
  }
}

template <class R>
__global__ __launch_bounds__(256) void k_permute(const PointRec<R> *__restrict__ in, const int32_t *__restrict__ perm,
                                                 int64_t M, PointRec<R> *__restrict__ out) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k < M) out[k] = in[perm[k]];
}

// tile_start[t] = first sorted position whose key lies in tile t (lower bound).
__global__ __launch_bounds__(256) void k_tile_bounds(const uint32_t *__restrict__ keys, int64_t M, int64_t ntiles,
                                                     uint32_t cells_per_tile, int32_t *__restrict__ tile_start) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t > ntiles) return;
  if (t == ntiles) {
    tile_start[t] = (int32_t)M;
    return;
  }
  const uint64_t key = (uint64_t)t * cells_per_tile;
  int64_t lo = 0, hi = M;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if ((uint64_t)keys[mid] < key) lo = mid + 1; else hi = mid;
  }
  tile_start[t] = (int32_t)lo;
}

}  // namespace

hipError_t launch_point_radius(const Plan &p, const void *xyz, double *partial, int nblocks) {
  if (p.prec == SGL_F64)
    k_radius<double><<<nblocks, 256, 0, p.stream>>>((const double *)xyz, p.M, partial);
  else
    k_radius<float><<<nblocks, 256, 0, p.stream>>>((const float *)xyz, p.M, partial);
  return hipGetLastError();
}

hipError_t launch_point_prep(Plan &p, const void *xyz, uint32_t *keys, int32_t *idx, void *unsorted) {
  PrepGeom g;
  g.rho = p.rho;
  for (int j = 0; j < 3; ++j) {
    g.N[j] = p.N[j];
    g.L[j] = p.L[j];
    g.T[j] = p.T[j];
  }
  // The FP64 matrix-core scatter multiplies, per step of four consecutive
  // points, the column blocks below 2 (max o2 + 2q) / 16: with the points whose
  // dimension-2 offset in the tile stays at or below 16 - 2q grouped first,
  // most steps of that class need one column block fewer.
  const int thr = 16 - 2 * p.q;
  g.nlo2 = (p.mfma64 && thr >= 0 && thr + 1 < p.L[2]) ? thr + 1 : 0;
  const int nb = (int)((p.M + 255) / 256);
  double *tout = (double *)p.ptsxyz;
  if (p.prec == SGL_F64)
    k_prep<double, double><<<nb, 256, 0, p.stream>>>((const double *)xyz, p.M, g, keys, idx,
                                                     (PointRec<double> *)unsorted, tout);
  else
    k_prep<float, float><<<nb, 256, 0, p.stream>>>((const float *)xyz, p.M, g, keys, idx,
                                                   (PointRec<float> *)unsorted, tout);
  return hipGetLastError();
}

// Sort (key, index) pairs, permute the point records into sorted order and
// find the tile boundaries.  keys/idx hold 2*M entries (input and output halves).
hipError_t launch_point_sort(Plan &p, uint32_t *keys, int32_t *idx, void *unsorted) {
  const size_t M = (size_t)p.M;
  uint32_t key_bits = 1;
  const uint64_t maxkey = (uint64_t)p.ntiles * p.L[0] * p.L[1] * p.L[2];
  while (key_bits < 32 && (1ull << key_bits) < maxkey) ++key_bits;
  size_t tmp_bytes = 0;
  hipError_t e = rocprim::radix_sort_pairs(nullptr, tmp_bytes, keys, keys + M, idx, p.perm, M, 0, key_bits, p.stream);
  if (e != hipSuccess) return e;
  void *tmp = nullptr;
  e = hipMalloc(&tmp, tmp_bytes ? tmp_bytes : 16);
  if (e != hipSuccess) return e;
  e = rocprim::radix_sort_pairs(tmp, tmp_bytes, keys, keys + M, idx, p.perm, M, 0, key_bits, p.stream);
  if (e == hipSuccess) {
    const int nb = (int)((M + 255) / 256);
    if (p.prec == SGL_F64)
      k_permute<double><<<nb, 256, 0, p.stream>>>((const PointRec<double> *)unsorted, p.perm, p.M,
                                                  (PointRec<double> *)p.pts);
    else
      k_permute<float><<<nb, 256, 0, p.stream>>>((const PointRec<float> *)unsorted, p.perm, p.M,
                                                 (PointRec<float> *)p.pts);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const int nbt = (int)((p.ntiles + 1 + 255) / 256);
    k_tile_bounds<<<nbt, 256, 0, p.stream>>>(keys + M, p.M, p.ntiles, (uint32_t)(p.L[0] * p.L[1] * p.L[2]),
                                             p.tile_start);
    e = hipGetLastError();
  }
  const hipError_t es = hipStreamSynchronize(p.stream);
  hipFree(tmp);
  return e != hipSuccess ? e : es;
}

}  // namespace sgl
