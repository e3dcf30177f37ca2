// Internal declarations of the SGL scattered-data transform library: plan
// layout, small complex type, and the launchers each translation unit exports.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "sgl.h"

namespace sgl {

template <class R>
struct alignas(2 * sizeof(R)) cplx {
  R re, im;
};

template <class R>
__host__ __device__ inline cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R>
__host__ __device__ inline cplx<R> cadd(cplx<R> a, cplx<R> b) {
  return {a.re + b.re, a.im + b.im};
}
template <class R>
__host__ __device__ inline cplx<R> csub(cplx<R> a, cplx<R> b) {
  return {a.re - b.re, a.im - b.im};
}
template <class R>
__host__ __device__ inline cplx<R> cscale(cplx<R> a, R s) {
  return {a.re * s, a.im * s};
}
template <class R>
__host__ __device__ inline cplx<R> cconj(cplx<R> a) {
  return {a.re, -a.im};
}

// One transformed point, in tile-sorted order.  The grid coordinate of the
// point in dimension j is u_j = N_j t_j / (2 pi) = base_j + frac_j, with
// base_j = floor(u_j) packed into `cell` (11 + 10 + 11 bits: base0 | base1 << 11
// | base2 << 21 -- base0 <= N0/2 <= 1024, base1 <= N1/2 <= 512, base2 < N2 <= 1024).
template <class R>
struct PointRec {
  R frac[3];
  int32_t cell;
};

__host__ __device__ inline int cell0(int32_t c) { return c & 2047; }
__host__ __device__ inline int cell1(int32_t c) { return (c >> 11) & 1023; }
__host__ __device__ inline int cell2(int32_t c) { return (int)(((uint32_t)c >> 21) & 2047u); }
__host__ __device__ inline int32_t pack_cell(int b0, int b1, int b2) {
  return (int32_t)((uint32_t)b0 | ((uint32_t)b1 << 11) | ((uint32_t)b2 << 21));
}

constexpr int kMaxStages = 12;

// Geometry of one 1D FFT pass over a 3D array viewed as [outer][axis][inner].
// Input rows i < nin sit at FFT index (in_off + i) mod L; output rows
// o < nout take FFT index (out_off + o) mod L.  `scale_*` are optional real
// factors (deconvolution) applied along axis on input or output.
struct FftPass {
  int axis;          // grid dimension the lines run along
  int L;             // transform length
  int nstages;
  int radix[kMaxStages];
  int outer;         // number of outer indices
  int inner;         // extent of the contiguous inner dimension
  int nin, in_off;   // rows read from the input
  int nout, out_off; // rows written to the output
  int W;             // lines per workgroup
  int sign;          // +1: e^{+2 pi i k l / L} (evaluation), -1: e^{-...} (adjoint)
};

// Per-stage HIP-event timer (enabled by sgl_plan_profile).
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  std::vector<int> stage;  // stage of event pair i (events 2i, 2i+1)
  double ms[SGL_NUM_STAGES] = {};
  int64_t count[SGL_NUM_STAGES] = {};
};

// The plan (opaque to callers).
// Table operand and tile list of one conversion product (sgl_conv_products.hip).
struct ConvGroup {
  int32_t Mpad, Kpad;  // padded rows (16) and columns (32) of the table operand
  int64_t plane_off;   // first half of the hi plane; the lo plane follows (Mpad * Kpad halves)
  int32_t rexp_off;    // first row exponent
  int32_t pad_;
};
struct ConvTab {
  void *groups = nullptr, *planes = nullptr, *rexp = nullptr, *tiles = nullptr;
  int ntiles = 0;
};

struct Plan {
  // parameters
  int B = 0, sigma = 2, q = 6, prec = SGL_F64;
  uint32_t flags = 0;
  int64_t M = 0;
  double rho = 0.0, lambda = 0.0;
  hipStream_t stream = nullptr;
  int device = 0;
  // grids: reduced trigonometric grid n, FFT grid N = sigma n,
  // stored (pruned) grid E with first stored index lo
  int n[3], N[3], E[3], lo[3];
  bool pruned[3];
  // point bins (gather tiles) over base cells: edge L, count T, base range NB
  int L[3], T[3], NB[3], X[3];
  int64_t ntiles = 0;
  int gather_mode = 0;  // 0: LDS tiles, 1: box streamed in slabs and cell-owned scatter
  // tiled gather in 256-thread workgroups, leaving room on each CU for the
  // workgroups of a concurrent scatter
  bool gather_narrow = false;
  int mfma = 0;         // FP32, 8^3 tiles, q <= 8: matrix-core gather and spread
  int mfma64 = 0;       // FP64, 8^3 tiles, box edge <= 24: FP64 matrix-core spread
  // scatter output blocks over stored cells
  int Lo[3], To[3];
  int64_t nblocks = 0;
  // conversion table offsets (in reals)
  std::vector<int64_t> krad_off, kpol_off, beta_off;
  int64_t krad_size = 0, kpol_size = 0, beta_size = 0;
  // device memory
  void *pts = nullptr;       // PointRec<R>[M], sorted
  int32_t *perm = nullptr;   // sorted position -> caller's index
  int32_t *tile_start = nullptr;  // ntiles + 1
  int32_t *chunks = nullptr;      // gather/spread work list: {tile, start, count} triples
  int64_t nchunks = 0;
  int32_t *tile_chunk = nullptr;  // ntiles + 1: first chunk of every tile
  void *staging = nullptr;        // nchunks window boxes (tiled scatter)
  // cell-owned scatter: work items {block, first candidate, count, slot},
  // folds {block, first slot, slots} and the partial blocks of the slots
  int32_t *own_work = nullptr, *own_fold = nullptr;
  int64_t nown = 0, nown_fold = 0, nown_slots = 0;
  void *own_stage = nullptr;
  int F[3] = {8, 8, 8};           // fold block edges (stored cells)
  void *krad = nullptr, *kpol = nullptr;  // conversion matrices (always FP64)
  ConvTab conv[4];                       // conversion products: FP64 or FP16 hi/lo table operands
  void *deconv = nullptr;                 // n0 + n1 + n2 reals
  void *twiddle = nullptr;                // per dimension: N_j complex double
  int64_t tw_off[3] = {0, 0, 0};
  void *beta = nullptr;   // radial output / adjoint input, complex double
  void *zeta = nullptr;   // polar output in compact form, complex double
  void *eta = nullptr;    // dense eta on the reduced grid (complex double in both precisions)
  void *bufX = nullptr;   // FFT scratch T1 and the stored grid G (aliased)
  void *bufY = nullptr;   // FFT scratch (first pass output)
  void *bufZ = nullptr;   // FFT scratch (second pass output)
  void *ptsxyz = nullptr; // for the exact NDFT: transformed points t (double, 3 x M)
  size_t bytes = 0;
  FftPass passA, passB, passC;      // forward passes (evaluation sign)
  FftPass passAh, passBh, passCh;   // adjoint passes
  Profiler prof;
};

// ---- launchers (all enqueue on p.stream; return hipError_t) ----
hipError_t launch_point_radius(const Plan &p, const void *xyz, double *partial, int nblocks);
hipError_t launch_point_prep(Plan &p, const void *xyz, uint32_t *keys, int32_t *idx, void *unsorted);
hipError_t launch_point_sort(Plan &p, uint32_t *keys, int32_t *idx, void *unsorted);
hipError_t launch_conv_product(const Plan &p, int mode, const void *in, void *out);
hipError_t launch_grad_points(const Plan &p, const void *grid, const void *xyz, const void *g, void *grad);
// Learned density-compensation weights (sgl_learn.hip).
int mlp_num_params();
hipError_t launch_point_features(const Plan &p, const void *xyz, float *feat);
hipError_t launch_mlp_forward(const float *params, const float *feat, int64_t M, float *c, hipStream_t s);
hipError_t launch_mlp_backward(const float *params, const float *feat, const float *dc, int64_t M, float *grad,
                               hipStream_t s);
hipError_t launch_mlp_backward_noalloc(const float *params, const float *feat, const float *dc, int64_t M,
                                       float *grad, hipStream_t s, int device);
hipError_t launch_adam(float *params, const float *grad, float *m, float *v, int n, float lr, float b1, float b2,
                       float eps, int step, hipStream_t s);
hipError_t launch_mlp_weights(const Plan &p, const float *c, const float *feat, void *w);
hipError_t launch_weight_grad(const Plan &p, const void *y, const void *g, const void *w, double scale,
                              bool accumulate, float *dc);
hipError_t launch_scale_by(const Plan &p, void *out, const void *a, const void *w, int64_t n);
hipError_t launch_sub_from(const Plan &p, void *a, const void *b, int64_t n);
hipError_t launch_norm2(const Plan &p, const void *a, int64_t n, double *out_dev);
// Weighted CGNR over the plan's transforms; fwd / adj: fhat -> f and f -> fhat.
sgl_status cgnr_run(Plan &p, const void *y_dev, const void *w_dev, void *fhat_dev, int maxiter, double tol,
                    double *info, sgl_status (*fwd)(Plan &, const void *, void *),
                    sgl_status (*adj)(Plan &, const void *, void *));
sgl_status cgne_run(Plan &p, const void *y_dev, void *fhat_dev, int maxiter, double tol, double *info,
                    sgl_status (*fwd)(Plan &, const void *, void *), sgl_status (*adj)(Plan &, const void *, void *));
hipError_t launch_conv_unfold(const Plan &p, void *eta, int eta_f64);
hipError_t launch_conv_fold_eta(const Plan &p, const void *eta, int eta_f64);
sgl_status build_conv_tables(Plan &p, const std::vector<long double> &kr, const std::vector<long double> &kp);
void free_conv_tables(Plan &p);
// One FFT pass; in_f64/out_f64 select double or float elements (float input
// with double output widens; the transform runs in the output precision).
hipError_t launch_fft_pass(const Plan &p, const FftPass &fp, const void *in, void *out, int tw_index, int dcmode,
                           int in_f64, int out_f64);
hipError_t launch_gather(const Plan &p, const void *grid, void *f);
hipError_t launch_scatter(const Plan &p, const void *f, void *grid);
// work list of the cell-owned scatter from the host copy of tile_start
void owned_work_list(const Plan &p, const std::vector<int32_t> &ts, std::vector<int32_t> &work,
                     std::vector<int32_t> &fold, int64_t &nslots);
hipError_t launch_fold(const Plan &p, void *grid);  // sums in FP64, writes the grid in the plan's precision
hipError_t launch_ndft_forward(const Plan &p, const void *eta, void *f);
hipError_t launch_ndft_adjoint(const Plan &p, const void *f, void *eta);

// host table builders (long double), sgl_tables.cpp
void build_radial_table(int B, double rho, std::vector<long double> &out, std::vector<int64_t> &off);
void build_polar_table(int B, std::vector<long double> &out, std::vector<int64_t> &off);
void build_deconv(const Plan &p, std::vector<long double> &out);
void build_twiddles(int L, int sign, std::vector<long double> &re, std::vector<long double> &im);

}  // namespace sgl
