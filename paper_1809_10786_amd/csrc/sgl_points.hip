// Plan-time point preparation (Section 6, eqs. x_tilde and nfsglft_rho):
// radius reduction for rho, the map x -> x~ = (arccos gamma(r), theta, phi)
// in FP64, grid coordinates u_j = N_j x~_j / (2 pi) split into an integer base
// cell and a fractional offset, and binning of the points into tiles of base
// cells (a stable radix sort on the tile-major cell key).
#include <cstring>
#include <utility>

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


// ---------------------------------------------------------------- point sort

// Stable least-significant-digit radix sort of (key, index) pairs with digits
// of at most 8 bits.  A pass counts the digits of every tile of kSortTile
// consecutive elements, scans the counts digit-major (digit 0 of every tile,
// then digit 1, ...), and moves each element to its digit's scanned offset
// for its tile plus its rank among the tile's earlier elements of the same
// digit.  Ranks and counts come from wave ballots over the lanes holding the
// same digit, so nothing is atomic: equal keys keep their input order and the
// permutation is the same on every run.
constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortItems = 16;                          // elements per thread and pass
constexpr int kSortTile = kSortThreads * kSortItems;    // elements per workgroup
constexpr int kSortRadix = 256;                         // counters per tile (8-bit digits)
constexpr int kScanChunk = 4 * kSortThreads;            // counters per workgroup of the scan
static_assert(kSortThreads == kSortRadix, "one thread per digit in the per-digit steps");

// Lanes of the wave whose element is valid and has digit d (bits wide).
__device__ inline uint64_t digit_peers(uint32_t d, bool valid, int bits) {
  uint64_t m = __ballot(valid);
  for (int b = 0; b < bits; ++b) {
    const bool set = (d >> b) & 1u;
    const uint64_t v = __ballot(set);
    m &= set ? v : ~v;
  }
  return m;
}

// counts[d * ntile + tile] = number of elements of the tile with digit d
__global__ __launch_bounds__(kSortThreads) void k_sort_count(const uint32_t *__restrict__ keys, int64_t M,
                                                             int shift, int bits, int ntile,
                                                             uint32_t *__restrict__ counts) {
  __shared__ uint32_t wc[kSortWaves][kSortRadix];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < kSortWaves * kSortRadix; e += kSortThreads) (&wc[0][0])[e] = 0;
  __syncthreads();
  const uint32_t mask = (1u << bits) - 1u;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int s = 0; s < kSortItems; ++s) {
    const int64_t i = base + (int64_t)s * kSortThreads + threadIdx.x;
    const bool valid = i < M;
    const uint32_t d = valid ? (keys[i] >> shift) & mask : 0u;
    const uint64_t m = digit_peers(d, valid, bits);
    // the highest lane of each digit group adds the group's size
    if (valid && (m >> lane) == 1ull) wc[wave][d] += (uint32_t)__popcll(m);
  }
  __syncthreads();
  uint32_t t = 0;
  for (int w = 0; w < kSortWaves; ++w) t += wc[w][threadIdx.x];
  counts[(int64_t)threadIdx.x * ntile + blockIdx.x] = t;
}

// Exclusive scan of x over the workgroup; *total gets the sum of all x.
__device__ inline uint32_t block_exclusive_scan(uint32_t x, uint32_t *wsum, uint32_t *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = x;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int w = 0; w < kSortWaves; ++w) {
    if (w < wave) before += wsum[w];
    all += wsum[w];
  }
  __syncthreads();  // wsum is free again
  *total = all;
  return before + inc - x;
}

// a[i0 .. i0 + kScanChunk) replaced by its exclusive scan plus carry; returns
// the chunk's sum
__device__ inline uint32_t scan_chunk(uint32_t *a, int64_t n, int64_t i0, uint32_t carry, uint32_t *wsum) {
  const int64_t j = i0 + 4 * (int64_t)threadIdx.x;
  uint32_t v[4], sum = 0;
  for (int u = 0; u < 4; ++u) {
    v[u] = j + u < n ? a[j + u] : 0u;
    sum += v[u];
  }
  uint32_t total;
  uint32_t run = carry + block_exclusive_scan(sum, wsum, &total);
  for (int u = 0; u < 4; ++u) {
    if (j + u < n) a[j + u] = run;
    run += v[u];
  }
  return total;
}

// each chunk of kScanChunk counters scanned on its own; its sum to sums[chunk]
__global__ __launch_bounds__(kSortThreads) void k_scan_chunks(uint32_t *__restrict__ a, int64_t n,
                                                              uint32_t *__restrict__ sums) {
  __shared__ uint32_t wsum[kSortWaves];
  const uint32_t total = scan_chunk(a, n, (int64_t)blockIdx.x * kScanChunk, 0u, wsum);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// the chunk sums scanned by one workgroup, strip by strip
__global__ __launch_bounds__(kSortThreads) void k_scan_sums(uint32_t *__restrict__ sums, int64_t nchunk) {
  __shared__ uint32_t wsum[kSortWaves];
  uint32_t carry = 0;
  for (int64_t i0 = 0; i0 < nchunk; i0 += kScanChunk) carry += scan_chunk(sums, nchunk, i0, carry, wsum);
}

// One pass: element i of tile b with digit d goes to
// offs[d * ntile + b] + sums[(d * ntile + b) / kScanChunk] + (its rank in the tile).
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(
    const uint32_t *__restrict__ kin, const int32_t *__restrict__ vin, int64_t M, int shift, int bits, int ntile,
    const uint32_t *__restrict__ offs, const uint32_t *__restrict__ sums, uint32_t *__restrict__ kout,
    int32_t *__restrict__ vout) {
  __shared__ uint32_t next[kSortRadix];            // output position of the tile's next element of each digit
  __shared__ uint32_t wc[kSortWaves][kSortRadix];  // this sweep's count per wave and digit
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  {
    const int64_t j = (int64_t)threadIdx.x * ntile + blockIdx.x;
    next[threadIdx.x] = offs[j] + sums[j / kScanChunk];
  }
  for (int e = threadIdx.x; e < kSortWaves * kSortRadix; e += kSortThreads) (&wc[0][0])[e] = 0;
  __syncthreads();
  const uint32_t mask = (1u << bits) - 1u;
  const uint64_t below = (1ull << lane) - 1ull;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int s = 0; s < kSortItems; ++s) {
    // sweep s holds the tile's elements s * kSortThreads .. + kSortThreads - 1 in thread order
    const int64_t i = base + (int64_t)s * kSortThreads + threadIdx.x;
    const bool valid = i < M;
    const uint32_t k = valid ? kin[i] : 0u;
    const int32_t v = valid ? vin[i] : 0;
    const uint32_t d = (k >> shift) & mask;
    const uint64_t m = digit_peers(d, valid, bits);
    if (valid && (m >> lane) == 1ull) wc[wave][d] = (uint32_t)__popcll(m);
    __syncthreads();
    if (valid) {
      uint32_t pos = next[d] + (uint32_t)__popcll(m & below);
      for (int w = 0; w < wave; ++w) pos += wc[w][d];
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    uint32_t t = 0;
    for (int w = 0; w < kSortWaves; ++w) {
      t += wc[w][threadIdx.x];
      wc[w][threadIdx.x] = 0;
    }
    next[threadIdx.x] += t;
    __syncthreads();
  }
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
// find the tile boundaries.  keys holds 2*M entries (input and output halves),
// idx M input indices; the sorted indices go to p.perm.
hipError_t launch_point_sort(Plan &p, uint32_t *keys, int32_t *idx, void *unsorted) {
  const int64_t M = p.M;
  int key_bits = 1;
  const uint64_t maxkey = (uint64_t)p.ntiles * p.L[0] * p.L[1] * p.L[2];
  while (key_bits < 32 && (1ull << key_bits) < maxkey) ++key_bits;
  // an odd number of passes, so that the last one writes keys + M and p.perm
  const int npass = key_bits <= 8 ? 1 : (key_bits <= 24 ? 3 : 5);
  const int bits = (key_bits + npass - 1) / npass;
  const int ntile = (int)((M + kSortTile - 1) / kSortTile);
  const int64_t ncount = (int64_t)kSortRadix * ntile;
  const int64_t nchunk = (ncount + kScanChunk - 1) / kScanChunk;
  uint32_t *counts = nullptr;
  hipError_t e = hipMalloc(&counts, (size_t)(ncount + nchunk) * sizeof(uint32_t));
  if (e != hipSuccess) return e;
  uint32_t *sums = counts + ncount;
  uint32_t *kin = keys, *kout = keys + M;
  int32_t *vin = idx, *vout = p.perm;
  for (int pass = 0; pass < npass && e == hipSuccess; ++pass) {
    const int shift = pass * bits;
    k_sort_count<<<ntile, kSortThreads, 0, p.stream>>>(kin, M, shift, bits, ntile, counts);
    k_scan_chunks<<<(unsigned)nchunk, kSortThreads, 0, p.stream>>>(counts, ncount, sums);
    k_scan_sums<<<1, kSortThreads, 0, p.stream>>>(sums, nchunk);
    k_sort_scatter<<<ntile, kSortThreads, 0, p.stream>>>(kin, vin, M, shift, bits, ntile, counts, sums, kout, vout);
    e = hipGetLastError();
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  // kin / vin now name keys + M and p.perm
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
  hipFree(counts);
  return e != hipSuccess ? e : es;
}

}  // namespace sgl
