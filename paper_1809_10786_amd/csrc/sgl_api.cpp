// C-ABI entry points (include/sgl.h): argument checks, plan construction
// (points, bins, tables, workspace), and the composition of the forward and
// adjoint transforms out of the stage kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "sgl_internal.h"

using namespace sgl;

struct sgl_plan_s {
  Plan p;
  // sgl_forward_adjoint: the adjoint runs on a second stream with scratch of
  // its own (a copy of p sharing every read-only array), set up on first use
  bool paired = false;
  sgl::Plan adj;
  hipEvent_t fork = nullptr, join = nullptr;
};

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr size_t kLdsBudget = 64 * 1024;

thread_local char g_last_error[256] = "";

sgl_status from_hip(hipError_t e) {
  if (e == hipSuccess) return SGL_OK;
  snprintf(g_last_error, sizeof g_last_error, "%s: %s", hipGetErrorName(e), hipGetErrorString(e));
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SGL_E_NOMEM;
  return SGL_E_DEVICE;
}

#define SGL_TRY(expr)                       \
  do {                                      \
    const hipError_t e_ = (expr);           \
    if (e_ != hipSuccess) return from_hip(e_); \
  } while (0)

bool radices_of(int L, FftPass &fp) {
  fp.L = L;
  fp.nstages = 0;
  int r = L;
  for (int f : {8, 4, 2, 3, 5})
    while (r % f == 0) {
      if (fp.nstages == kMaxStages) return false;
      fp.radix[fp.nstages++] = f;
      r /= f;
    }
  return r == 1;
}

// Lines per FFT workgroup: two LDS buffers of L x W elements plus the L
// twiddles must fit the LDS budget.
int lines_per_group(int L, size_t elem) {
  int W = 1;
  while (W < 32 && (2 * (size_t)L * (W * 2) + L) * elem <= kLdsBudget) W *= 2;
  return W;
}

void free_plan(Plan &p) {
  void *bufs[] = {p.pts,  p.perm, p.tile_start, p.chunks, p.krad,    p.kpol,       p.deconv,   p.twiddle,
                  p.beta, p.zeta, p.eta,        p.bufX,   p.bufY,    p.bufZ,       p.ptsxyz,   p.tile_chunk,
                  p.staging, p.own_work, p.own_fold, p.own_stage};
  for (void *b : bufs)
    if (b) hipFree(b);
  free_conv_tables(p);
}

template <class T>
hipError_t dev_alloc(Plan &p, T **ptr, size_t bytes) {
  void *v = nullptr;
  const hipError_t e = hipMalloc(&v, bytes ? bytes : 16);
  if (e == hipSuccess) {
    *ptr = (T *)v;
    p.bytes += bytes;
  }
  return e;
}

// The scratch one transform direction writes: beta, compact zeta, eta and the
// two FFT buffers (double values on the adjoint side in both precisions).
hipError_t alloc_scratch(Plan &p) {
  const int B = p.B;
  const size_t nbeta = (size_t)(2 * B - 1) * B * B;  // sum_m (B - |m|) (2B - 1) = B^2 (2B - 1)
  const size_t neta = (size_t)p.n[0] * p.n[1] * p.n[2];
  const size_t n01 = (size_t)p.n[0] * p.E[1] * p.n[2];  // after the dimension-1 pass
  const size_t nEE = (size_t)p.E[0] * p.E[1] * p.n[2];  // after dimensions 0 and 1 (or 2, adjoint)
  const size_t nG = (size_t)p.E[0] * p.E[1] * p.E[2];
  hipError_t e = dev_alloc(p, &p.beta, nbeta * 16);
  if (e == hipSuccess) e = dev_alloc(p, &p.zeta, (size_t)(2 * B - 1) * B * (2 * B - 1) * 16);
  if (e == hipSuccess) e = dev_alloc(p, &p.eta, neta * 16);
  if (e == hipSuccess) e = dev_alloc(p, &p.bufX, nG * 16);
  if (e == hipSuccess) e = dev_alloc(p, &p.bufY, std::max(n01, nEE) * 16);
  if (e == hipSuccess) e = dev_alloc(p, &p.bufZ, std::max(n01, nEE) * 16);
  return e;
}

void free_scratch(Plan &p) {
  void *bufs[] = {p.beta, p.zeta, p.eta, p.bufX, p.bufY, p.bufZ};
  for (void *b : bufs)
    if (b) hipFree(b);
  p.beta = p.zeta = p.eta = p.bufX = p.bufY = p.bufZ = nullptr;
}

template <class R>
hipError_t upload_real(Plan &p, void **dst, const std::vector<long double> &v) {
  std::vector<R> h(v.size());
  for (size_t i = 0; i < v.size(); ++i) h[i] = (R)v[i];
  hipError_t e = dev_alloc(p, dst, h.size() * sizeof(R));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, h.data(), h.size() * sizeof(R), hipMemcpyHostToDevice);
}

hipError_t upload_twiddles(Plan &p) {
  std::vector<double> h;
  for (int j = 0; j < 3; ++j) {
    std::vector<long double> re, im;
    build_twiddles(p.N[j], +1, re, im);
    p.tw_off[j] = (int64_t)h.size() / 2;
    for (int t = 0; t < p.N[j]; ++t) {
      h.push_back((double)re[t]);
      h.push_back((double)im[t]);
    }
  }
  hipError_t e = dev_alloc(p, &p.twiddle, h.size() * sizeof(double));
  if (e != hipSuccess) return e;
  return hipMemcpy(p.twiddle, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice);
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
  const char *x = (const char *)a, *y = (const char *)b;
  return x < y + nb && y < x + na;
}

size_t cbytes(const Plan &p) { return p.prec == SGL_F64 ? 16 : 8; }

// Geometry of grids, bins and blocks (host only).
sgl_status setup_geometry(Plan &p) {
  const int B = p.B;
  p.n[0] = 4 * B;
  p.n[1] = 2 * B;
  p.n[2] = 2 * B;
  // FFT lengths: sigma n_j when it factors into 2, 3 and 5, else the next even
  // length that does (the effective oversampling N_j / n_j then exceeds sigma;
  // the window keeps the lambda of sigma, so its error bound still holds)
  FftPass tmp;
  for (int j = 0; j < 3; ++j) {
    int N = p.sigma * p.n[j];
    while (N <= 2048 && !radices_of(N, tmp)) N += 2;
    p.N[j] = N;
  }
  if (p.N[0] > 2048 || p.N[1] > 1024 || p.N[2] > 1024) return SGL_E_UNSUPPORTED;
  p.lambda = p.sigma * (double)p.q / ((2.0 * p.sigma - 1.0) * kPi);
  for (int j = 0; j < 3; ++j) {
    if (j < 2 && p.N[j] / 2 + 2 * p.q < p.N[j]) {
      p.pruned[j] = true;
      p.E[j] = p.N[j] / 2 + 2 * p.q;
      p.lo[j] = 1 - p.q;
    } else {
      p.pruned[j] = false;
      p.E[j] = p.N[j];
      p.lo[j] = 0;
    }
    p.NB[j] = (j < 2) ? p.N[j] / 2 + 1 : p.N[j];
  }
  // gather tiles: the largest edges (<= 8) whose window box fits in LDS: 120 KB
  // for FP64 boxes (a workgroup may hold 160 KB on gfx950), 64 KB for FP32 ones
  // (the matrix-core kernels stage their own FP16 planes)
  const size_t cb = cbytes(p);
  const size_t kBoxBudget = (p.prec == SGL_F64 ? 120 : 64) * 1024;
  int L[3] = {8, 8, 8};
  auto box = [&](const int *l) { return (size_t)(l[0] + 2 * p.q - 1) * (l[1] + 2 * p.q - 1) * (l[2] + 2 * p.q - 1) * cb; };
  while (box(L) > kBoxBudget && (L[0] > 4 || L[1] > 4 || L[2] > 4)) {
    int j = (L[0] >= L[1] && L[0] >= L[2]) ? 0 : (L[1] >= L[2] ? 1 : 2);
    L[j] /= 2;
  }
  p.gather_mode = box(L) <= kBoxBudget ? 0 : 1;
  // the row-register spreading of the tiled scatter needs one thread per box
  // row (at most 512) and a box edge of 4 or 8 base cells along dimension 2
  if ((size_t)(L[0] + 2 * p.q - 1) * (L[1] + 2 * p.q - 1) > 512 || p.q > 8 || (L[2] != 4 && L[2] != 8))
    p.gather_mode = 1;
  if (p.gather_mode == 1) {
    // wide windows: tiles of 8^3 base cells, the box streamed through LDS in
    // slabs of four dimension-0 planes (k_gather_slab; four planes of the box
    // fit the budget for every q <= 16)
    L[0] = L[1] = L[2] = 8;
  }
  p.ntiles = 1;
  for (int j = 0; j < 3; ++j) {
    p.L[j] = std::min(L[j], p.NB[j]);
    p.T[j] = (p.NB[j] + p.L[j] - 1) / p.L[j];
    p.X[j] = p.L[j] + 2 * p.q - 1;
    p.ntiles *= p.T[j];
  }
  if ((uint64_t)p.ntiles * p.L[0] * p.L[1] * p.L[2] >= (1ull << 32)) return SGL_E_UNSUPPORTED;
  p.mfma = (p.prec == SGL_F32 && p.gather_mode == 0 && p.q <= 8 && p.L[0] == 8 && p.L[1] == 8 && p.L[2] == 8);
  // FP64 boxes of 8^3 tiles fit the LDS budget up to q = 6
  p.mfma64 = (p.prec == SGL_F64 && p.gather_mode == 0 && p.q <= 6 && p.L[0] == 8 && p.L[1] == 8 &&
              p.L[2] == 8);
  // blocks of 16^3 stored cells of the cell-owned scatter (the last block of
  // a dimension may be partial)
  p.nblocks = 1;
  for (int j = 0; j < 3; ++j) {
    p.Lo[j] = 16;
    p.To[j] = (p.E[j] + p.Lo[j] - 1) / p.Lo[j];
    p.nblocks *= p.To[j];
  }
  // worst-case number of bin rows a block visits must fit the kernel's table
  // (768 slots: bins in dimensions 0 and 1 times at most 3 dimension-2 intervals)
  int64_t rows = 3;
  for (int j = 0; j < 2; ++j) {
    const int span = p.Lo[j] + 2 * p.q - 1;
    rows *= std::min<int64_t>(p.T[j], span / p.L[j] + 2 + (p.pruned[j] ? 0 : 2));
  }
  if (rows > 768) return SGL_E_UNSUPPORTED;
  // FFT passes: [outer][axis][inner] views; every pass computes in FP64.  The
  // forward runs dimension 1 (n1 -> E1 rows), 0 (n0 -> E0) and last 2, the one
  // that doubles (n2 -> N2), so both intermediates stay near the size of eta;
  // the adjoint runs the mirror order (2, 0, 1).
  auto pass = [&](FftPass &fp, int j, int outer, int inner, int nin, int in_off, int nout, int out_off, int sign) {
    fp.axis = j;
    radices_of(p.N[j], fp);
    fp.outer = outer;
    fp.inner = inner;
    fp.nin = nin;
    fp.in_off = in_off;
    fp.nout = nout;
    fp.out_off = out_off;
    fp.sign = sign;
    fp.W = lines_per_group(p.N[j], 16);
  };
  const int n0 = p.n[0], n1 = p.n[1], n2 = p.n[2];
  const int E0 = p.E[0], E1 = p.E[1];
  pass(p.passA, 1, n0, n2, n1, -n1 / 2, E1, p.lo[1], +1);             // eta [n0][n1][n2] -> [n0][E1][n2]
  pass(p.passB, 0, 1, E1 * n2, n0, -n0 / 2, E0, p.lo[0], +1);         // -> [E0][E1][n2]
  pass(p.passC, 2, E0 * E1, 1, n2, -n2 / 2, p.N[2], 0, +1);           // -> grid [E0][E1][N2]
  pass(p.passCh, 2, E0 * E1, 1, p.N[2], 0, n2, -n2 / 2, -1);          // grid -> [E0][E1][n2]
  pass(p.passBh, 0, 1, E1 * n2, E0, p.lo[0], n0, -n0 / 2, -1);        // -> [n0][E1][n2]
  pass(p.passAh, 1, n0, n2, E1, p.lo[1], n1, -n1 / 2, -1);            // -> eta [n0][n1][n2]
  return SGL_OK;
}

template <class R>
sgl_status build_tables(Plan &p) {
  std::vector<long double> kr, kp, dc;
  build_radial_table(p.B, p.rho, kr, p.krad_off);
  build_polar_table(p.B, kp, p.kpol_off);
  build_deconv(p, dc);
  SGL_TRY(upload_real<double>(p, &p.krad, kr));
  SGL_TRY(upload_real<double>(p, &p.kpol, kp));
  {
    const sgl_status st = build_conv_tables(p, kr, kp);
    if (st != SGL_OK) return st;
  }
  SGL_TRY(upload_real<double>(p, &p.deconv, dc));
  SGL_TRY(upload_twiddles(p));
  return SGL_OK;
}

sgl_status make_plan(Plan &p, const void *points) {
  // 1. radius reduction: rho and finiteness (eq. nfsglft_rho)
  const int nrb = (int)std::min<int64_t>(1024, (p.M + 255) / 256);
  double *partial = nullptr;
  SGL_TRY(hipMalloc(&partial, 2 * nrb * sizeof(double)));
  hipError_t e = launch_point_radius(p, points, partial, nrb);
  std::vector<double> hp(2 * nrb);
  if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), partial, hp.size() * sizeof(double), hipMemcpyDeviceToHost, p.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
  hipFree(partial);
  SGL_TRY(e);
  double maxr = 0.0, bad = 0.0;
  for (int b = 0; b < nrb; ++b) {
    maxr = std::max(maxr, hp[2 * b]);
    bad += hp[2 * b + 1];
  }
  if (bad > 0) return SGL_E_INVAL;
  if (p.rho > 0.0) {
    if (p.rho < maxr) return SGL_E_RANGE;
  } else {
    p.rho = maxr > 0.0 ? maxr : 1.0;
  }
  // 2. geometry: set up by sgl_plan before any device work
  // 3. points: transform, key, sort into tiles
  const size_t M = (size_t)p.M;
  const size_t rec = p.prec == SGL_F64 ? sizeof(PointRec<double>) : sizeof(PointRec<float>);
  SGL_TRY(dev_alloc(p, &p.pts, M * rec));
  SGL_TRY(dev_alloc(p, &p.perm, M * sizeof(int32_t)));
  SGL_TRY(dev_alloc(p, &p.tile_start, (p.ntiles + 1) * sizeof(int32_t)));
  if (p.flags & SGL_FLAG_EXACT_NDFT) SGL_TRY(dev_alloc(p, &p.ptsxyz, 3 * M * sizeof(double)));
  uint32_t *keys = nullptr;
  int32_t *idx = nullptr;
  void *unsorted = nullptr;
  e = hipMalloc(&keys, 2 * M * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMalloc(&idx, M * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&unsorted, M * rec);
  if (e == hipSuccess) e = launch_point_prep(p, points, keys, idx, unsorted);
  if (e == hipSuccess) e = launch_point_sort(p, keys, idx, unsorted);
  if (keys) hipFree(keys);
  if (idx) hipFree(idx);
  if (unsorted) hipFree(unsorted);
  SGL_TRY(e);
  // 4. gather work list: chunks of at most kChunk points of one tile
  std::vector<int32_t> ts(p.ntiles + 1);
  SGL_TRY(hipMemcpy(ts.data(), p.tile_start, ts.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
  const int kChunk = 2048;
  std::vector<int32_t> ch, tc(p.ntiles + 1);
  for (int64_t t = 0; t < p.ntiles; ++t) {
    tc[t] = (int32_t)(ch.size() / 3);
    for (int s = ts[t]; s < ts[t + 1]; s += kChunk) {
      ch.push_back((int32_t)t);
      ch.push_back(s);
      ch.push_back(std::min(kChunk, ts[t + 1] - s));
    }
  }
  tc[p.ntiles] = (int32_t)(ch.size() / 3);
  p.nchunks = (int64_t)ch.size() / 3;
  SGL_TRY(dev_alloc(p, &p.chunks, ch.size() * sizeof(int32_t)));
  if (!ch.empty()) SGL_TRY(hipMemcpy(p.chunks, ch.data(), ch.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  SGL_TRY(dev_alloc(p, &p.tile_chunk, tc.size() * sizeof(int32_t)));
  SGL_TRY(hipMemcpy(p.tile_chunk, tc.data(), tc.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  if (p.gather_mode == 0)
    SGL_TRY(dev_alloc(p, &p.staging, (size_t)p.nchunks * p.X[0] * p.X[1] * p.X[2] * cbytes(p)));
  if (p.gather_mode == 1) {
    // work items of the cell-owned scatter: dense blocks split into segments
    std::vector<int32_t> work, fold;
    owned_work_list(p, ts, work, fold, p.nown_slots);
    p.nown = (int64_t)work.size() / 4;
    p.nown_fold = (int64_t)fold.size() / 3;
    SGL_TRY(dev_alloc(p, &p.own_work, work.size() * sizeof(int32_t)));
    SGL_TRY(hipMemcpy(p.own_work, work.data(), work.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if (!fold.empty()) {
      SGL_TRY(dev_alloc(p, &p.own_fold, fold.size() * sizeof(int32_t)));
      SGL_TRY(hipMemcpy(p.own_fold, fold.data(), fold.size() * sizeof(int32_t), hipMemcpyHostToDevice));
      SGL_TRY(dev_alloc(p, &p.own_stage, (size_t)p.nown_slots * 16 * 16 * 16 * cbytes(p)));
    }
  }
  // 5. tables
  const sgl_status st = p.prec == SGL_F64 ? build_tables<double>(p) : build_tables<float>(p);
  if (st != SGL_OK) return st;
  // 6. workspace
  SGL_TRY(alloc_scratch(p));
  SGL_TRY(hipStreamSynchronize(p.stream));
  return SGL_OK;
}

sgl_status check_plan(sgl_plan_t plan) { return plan ? SGL_OK : SGL_E_INVAL; }

// ---- per-stage event timing ----
void prof_collect(Plan &p) {
  Profiler &pr = p.prof;
  for (size_t i = 0; i < pr.stage.size(); ++i) {
    float ms = 0.0f;
    if (hipEventSynchronize(pr.pool[2 * i + 1]) == hipSuccess &&
        hipEventElapsedTime(&ms, pr.pool[2 * i], pr.pool[2 * i + 1]) == hipSuccess) {
      pr.ms[pr.stage[i]] += ms;
      pr.count[pr.stage[i]] += 1;
    }
  }
  pr.stage.clear();
  pr.next = 0;
}

struct Stage {
  Plan &p;
  bool on;
  Stage(Plan &p_, int stage) : p(p_), on(p_.prof.on) {
    if (!on) return;
    if (p.prof.next + 2 > p.prof.pool.size()) prof_collect(p);
    hipEventRecord(p.prof.pool[p.prof.next++], p.stream);
    p.prof.stage.push_back(stage);
  }
  ~Stage() {
    if (on) hipEventRecord(p.prof.pool[p.prof.next++], p.stream);
  }
};

#define SGL_STAGE(id, expr)      \
  do {                           \
    Stage st_(p, id);            \
    SGL_TRY(expr);               \
  } while (0)

// eta_f64: element type of the eta output (the products themselves run in FP64).
// The four products run as batched matrix-core tiles (FP64, or FP16 hi/lo
// with SGL_FLAG_CONV_SPLIT16); unfold and fold map the compact zeta to and
// from eta.
sgl_status conv_fwd(Plan &p, const void *fhat, void *eta, int eta_f64) {
  SGL_STAGE(SGL_STAGE_CONV_RADIAL, launch_conv_product(p, 0, fhat, p.beta));
  SGL_STAGE(SGL_STAGE_CONV_POLAR, launch_conv_product(p, 1, p.beta, p.zeta));
  SGL_STAGE(SGL_STAGE_CONV_POLAR, launch_conv_unfold(p, eta, eta_f64));
  return SGL_OK;
}

sgl_status conv_adj(Plan &p, const void *eta, int eta_f64, void *fhat) {
  SGL_STAGE(SGL_STAGE_CONV_POLAR_ADJ, launch_conv_fold_eta(p, eta, eta_f64));
  SGL_STAGE(SGL_STAGE_CONV_POLAR_ADJ, launch_conv_product(p, 2, p.zeta, p.beta));
  SGL_STAGE(SGL_STAGE_CONV_RADIAL_ADJ, launch_conv_product(p, 3, p.beta, fhat));
  return SGL_OK;
}

// eta_f64: element type of the eta input.  The three FFT passes run in FP64 in
// both modes; the last one writes the grid in the plan's precision for the
// gather.  An FP32 FFT would leave every grid value with an absolute error of
// ~6e-8 of the largest ones, and the polynomial grows steeply towards r = rho:
// points at small r, where |f| is far below its maximum, would lose their
// relative accuracy.  Rounding the finished grid to FP32 keeps each value's
// error relative to itself.
sgl_status nfft_fwd(Plan &p, const void *eta, int eta_f64, void *f) {
  if (p.flags & SGL_FLAG_EXACT_NDFT) {
    if (eta_f64 != (p.prec == SGL_F64)) return SGL_E_INVAL;
    SGL_STAGE(SGL_STAGE_NDFT, launch_ndft_forward(p, eta, f));
    return SGL_OK;
  }
  const int grid_f64 = p.prec == SGL_F64;
  SGL_STAGE(SGL_STAGE_FFT_A, launch_fft_pass(p, p.passA, eta, p.bufY, 1, 1, eta_f64, 1));
  SGL_STAGE(SGL_STAGE_FFT_B, launch_fft_pass(p, p.passB, p.bufY, p.bufZ, 0, 0, 1, 1));
  SGL_STAGE(SGL_STAGE_FFT_C, launch_fft_pass(p, p.passC, p.bufZ, p.bufX, 2, 0, 1, grid_f64));
  SGL_STAGE(SGL_STAGE_GATHER, launch_gather(p, p.bufX, f));
  return SGL_OK;
}

// eta_f64: element type of the eta output (the adjoint FFT itself runs in FP64).
sgl_status nfft_adj(Plan &p, const void *f, void *eta, int eta_f64) {
  if (p.flags & SGL_FLAG_EXACT_NDFT) {
    if (eta_f64 != (p.prec == SGL_F64)) return SGL_E_INVAL;
    SGL_STAGE(SGL_STAGE_NDFT_ADJ, launch_ndft_adjoint(p, f, eta));
    return SGL_OK;
  }
  SGL_STAGE(SGL_STAGE_SCATTER, launch_scatter(p, f, p.bufX));
  if (p.gather_mode == 0) SGL_STAGE(SGL_STAGE_FOLD, launch_fold(p, p.bufX));
  // the folded grid is double; the direct scatter writes the plan's precision
  const int grid_f64 = p.prec == SGL_F64;
  SGL_STAGE(SGL_STAGE_FFT_CH, launch_fft_pass(p, p.passCh, p.bufX, p.bufY, 2, 0, grid_f64, 1));
  SGL_STAGE(SGL_STAGE_FFT_BH, launch_fft_pass(p, p.passBh, p.bufY, p.bufZ, 0, 0, 1, 1));
  SGL_STAGE(SGL_STAGE_FFT_AH, launch_fft_pass(p, p.passAh, p.bufZ, eta, 1, 2, 1, eta_f64));
  return SGL_OK;
}

void prof_release(Plan &p) {
  if (!p.prof.pool.empty()) {
    hipStreamSynchronize(p.stream);
    for (hipEvent_t e : p.prof.pool) hipEventDestroy(e);
  }
  p.prof.pool.clear();
  p.prof.stage.clear();
  p.prof.next = 0;
  p.prof.on = false;
}

}  // namespace

extern "C" {

int64_t sgl_num_coeffs(int32_t B) {
  if (B < 1) return -1;
  return (int64_t)B * (B + 1) * (2 * B + 1) / 6;
}

int64_t sgl_coeff_index(int32_t n, int32_t l, int32_t m) {
  if (n < 1 || l < 0 || l >= n || m < -l || m > l) return -1;
  return (int64_t)n * (n - 1) * (2 * n - 1) / 6 + (int64_t)l * (l + 1) + m;
}

sgl_status sgl_eta_dims(int32_t B, int32_t dims[3]) {
  if (!dims || B < 2 || B > 256) return SGL_E_INVAL;
  dims[0] = 4 * B;
  dims[1] = 2 * B;
  dims[2] = 2 * B;
  return SGL_OK;
}

sgl_status sgl_plan(sgl_plan_t *out, const sgl_params *prm, int64_t M, const void *points_dev, void *hip_stream) {
  if (!out) return SGL_E_INVAL;
  *out = nullptr;
  if (!prm || !points_dev) return SGL_E_INVAL;
  if (prm->B < 2 || prm->B > 256) return SGL_E_INVAL;
  if (prm->sigma < 2 || prm->sigma > 4) return SGL_E_INVAL;
  if (prm->q < 1 || prm->q > 16 || 2 * prm->q > prm->sigma * 2 * prm->B) return SGL_E_INVAL;
  if (prm->precision != SGL_F64 && prm->precision != SGL_F32) return SGL_E_INVAL;
  if (prm->flags & ~(uint32_t)(SGL_FLAG_EXACT_NDFT | SGL_FLAG_CONV_SPLIT16)) return SGL_E_INVAL;
  if (!std::isfinite(prm->rho)) return SGL_E_INVAL;
  if (M < 1 || M > 0x7fffffffLL) return SGL_E_INVAL;
  if ((prm->flags & SGL_FLAG_CONV_SPLIT16) && prm->B > SGL_CONV_SPLIT16_MAX_B) return SGL_E_UNSUPPORTED;
  sgl_plan_s *h = new (std::nothrow) sgl_plan_s;
  if (!h) return SGL_E_NOMEM;
  Plan &p = h->p;
  p.B = prm->B;
  p.sigma = prm->sigma;
  p.q = prm->q;
  p.prec = prm->precision;
  p.flags = prm->flags;
  p.M = M;
  p.rho = prm->rho > 0 ? prm->rho : 0.0;
  p.stream = (hipStream_t)hip_stream;
  // host-only geometry checks (FFT lengths, tile tables) come before any device call
  const sgl_status sg = setup_geometry(p);
  if (sg != SGL_OK) {
    delete h;
    return sg;
  }
  if (hipGetDevice(&p.device) != hipSuccess) {
    delete h;
    return SGL_E_DEVICE;
  }
  const sgl_status st = make_plan(p, points_dev);
  if (st != SGL_OK) {
    hipStreamSynchronize(p.stream);
    free_plan(p);
    delete h;
    return st;
  }
  *out = h;
  return SGL_OK;
}

sgl_status sgl_conv_forward(sgl_plan_t plan, const void *fhat_dev, void *eta_dev) {
  if (check_plan(plan) != SGL_OK || !fhat_dev || !eta_dev) return SGL_E_INVAL;
  Plan &p = plan->p;
  const size_t cb = cbytes(p);
  if (overlaps(fhat_dev, sgl_num_coeffs(p.B) * cb, eta_dev, (size_t)p.n[0] * p.n[1] * p.n[2] * cb)) return SGL_E_INVAL;
  return conv_fwd(p, fhat_dev, eta_dev, p.prec == SGL_F64);
}

sgl_status sgl_conv_adjoint(sgl_plan_t plan, const void *eta_dev, void *fhat_dev) {
  if (check_plan(plan) != SGL_OK || !fhat_dev || !eta_dev) return SGL_E_INVAL;
  Plan &p = plan->p;
  const size_t cb = cbytes(p);
  if (overlaps(fhat_dev, sgl_num_coeffs(p.B) * cb, eta_dev, (size_t)p.n[0] * p.n[1] * p.n[2] * cb)) return SGL_E_INVAL;
  return conv_adj(p, eta_dev, p.prec == SGL_F64, fhat_dev);
}

sgl_status sgl_nfft_forward(sgl_plan_t plan, const void *eta_dev, void *f_dev) {
  if (check_plan(plan) != SGL_OK || !eta_dev || !f_dev) return SGL_E_INVAL;
  Plan &p = plan->p;
  const size_t cb = cbytes(p);
  if (overlaps(eta_dev, (size_t)p.n[0] * p.n[1] * p.n[2] * cb, f_dev, (size_t)p.M * cb)) return SGL_E_INVAL;
  return nfft_fwd(p, eta_dev, p.prec == SGL_F64, f_dev);
}

sgl_status sgl_nfft_adjoint(sgl_plan_t plan, const void *f_dev, void *eta_dev) {
  if (check_plan(plan) != SGL_OK || !eta_dev || !f_dev) return SGL_E_INVAL;
  Plan &p = plan->p;
  const size_t cb = cbytes(p);
  if (overlaps(eta_dev, (size_t)p.n[0] * p.n[1] * p.n[2] * cb, f_dev, (size_t)p.M * cb)) return SGL_E_INVAL;
  return nfft_adj(p, f_dev, eta_dev, p.prec == SGL_F64);
}

sgl_status sgl_grad_points(sgl_plan_t plan, const void *fhat_dev, const void *points_dev, const void *g_dev,
                           void *grad_dev) {
  if (check_plan(plan) != SGL_OK || !fhat_dev || !points_dev || !g_dev || !grad_dev) return SGL_E_INVAL;
  Plan &p = plan->p;
  if (p.flags & SGL_FLAG_EXACT_NDFT) return SGL_E_UNSUPPORTED;
  const size_t cb = cbytes(p), rb = cb / 2;
  const size_t nf = sgl_num_coeffs(p.B) * cb, np = (size_t)p.M * 3 * rb, ng = (size_t)p.M * cb;
  if (overlaps(grad_dev, np, fhat_dev, nf) || overlaps(grad_dev, np, points_dev, np) ||
      overlaps(grad_dev, np, g_dev, ng))
    return SGL_E_INVAL;
  // the forward grid (conversion and FFT as in sgl_forward), then the gradient gather
  const sgl_status st = conv_fwd(p, fhat_dev, p.eta, 1);
  if (st != SGL_OK) return st;
  SGL_STAGE(SGL_STAGE_FFT_A, launch_fft_pass(p, p.passA, p.eta, p.bufY, 1, 1, 1, 1));
  SGL_STAGE(SGL_STAGE_FFT_B, launch_fft_pass(p, p.passB, p.bufY, p.bufZ, 0, 0, 1, 1));
  SGL_STAGE(SGL_STAGE_FFT_C, launch_fft_pass(p, p.passC, p.bufZ, p.bufX, 2, 0, 1, p.prec == SGL_F64));
  SGL_STAGE(SGL_STAGE_GATHER, launch_grad_points(p, p.bufX, points_dev, g_dev, grad_dev));
  return SGL_OK;
}

// The whole transforms without argument checks.  The fast path hands FP64 eta
// between the conversion and the FFT in both modes.
static sgl_status plan_forward(Plan &p, const void *fhat_dev, void *f_dev) {
  const int eta_f64 = (p.flags & SGL_FLAG_EXACT_NDFT) ? (p.prec == SGL_F64) : 1;
  const sgl_status st = conv_fwd(p, fhat_dev, p.eta, eta_f64);
  if (st != SGL_OK) return st;
  return nfft_fwd(p, p.eta, eta_f64, f_dev);
}

static sgl_status plan_adjoint(Plan &p, const void *f_dev, void *fhat_dev) {
  const int eta_f64 = (p.flags & SGL_FLAG_EXACT_NDFT) ? (p.prec == SGL_F64) : 1;
  const sgl_status st = nfft_adj(p, f_dev, p.eta, eta_f64);
  if (st != SGL_OK) return st;
  return conv_adj(p, p.eta, eta_f64, fhat_dev);
}

sgl_status sgl_cgnr(sgl_plan_t plan, const void *y_dev, const void *w_dev, void *fhat_dev, int32_t maxiter,
                    double tol, double *info) {
  if (check_plan(plan) != SGL_OK || !y_dev || !fhat_dev || maxiter < 0 || !(tol >= 0.0) || !std::isfinite(tol))
    return SGL_E_INVAL;
  Plan &p = plan->p;
  const size_t cb = cbytes(p);
  const size_t nf = sgl_num_coeffs(p.B) * cb, ny = (size_t)p.M * cb, nw = (size_t)p.M * (cb / 2);
  if (overlaps(fhat_dev, nf, y_dev, ny) || (w_dev && overlaps(fhat_dev, nf, w_dev, nw))) return SGL_E_INVAL;
  return cgnr_run(p, y_dev, w_dev, fhat_dev, maxiter, tol, info, plan_forward, plan_adjoint);
}

sgl_status sgl_cgne(sgl_plan_t plan, const void *y_dev, void *fhat_dev, int32_t maxiter, double tol, double *info) {
  if (check_plan(plan) != SGL_OK || !y_dev || !fhat_dev || maxiter < 0 || !(tol >= 0.0) || !std::isfinite(tol))
    return SGL_E_INVAL;
  Plan &p = plan->p;
  const size_t cb = cbytes(p);
  if (overlaps(fhat_dev, sgl_num_coeffs(p.B) * cb, y_dev, (size_t)p.M * cb)) return SGL_E_INVAL;
  return cgne_run(p, y_dev, fhat_dev, maxiter, tol, info, plan_forward, plan_adjoint);
}

// ---------------------------------------------------------------- batches

}  // extern "C"

struct sgl_batch_s {
  hipStream_t stream = nullptr;   // the caller's stream: sgl_batch_run launches here
  hipStream_t capture = nullptr;  // the stream the graph was captured from
  std::vector<hipStream_t> side;  // fork branches
  std::vector<hipEvent_t> events;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void batch_free(sgl_batch_s *b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  for (hipEvent_t e : b->events) hipEventDestroy(e);
  for (hipStream_t t : b->side) hipStreamDestroy(t);
  if (b->capture) hipStreamDestroy(b->capture);
  delete b;
}

// Captures every plan's forward and/or adjoint on the side streams (plan j on
// branch j mod nstreams) between a fork and a join on the capture stream.
static sgl_status batch_capture(sgl_batch_s *b, const sgl_plan_t *plans, int n, const void *const *fhat,
                                void *const *f, const void *const *y, void *const *ghat) {
  const int ns = (int)b->side.size();
  SGL_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
  sgl_status st = SGL_OK;
  hipError_t e = hipEventRecord(b->events[0], b->capture);
  for (int k = 0; k < ns && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->side[k], b->events[0], 0);
  for (int j = 0; j < n && e == hipSuccess && st == SGL_OK; ++j) {
    Plan &p = plans[j]->p;
    const hipStream_t keep = p.stream;
    p.stream = b->side[j % ns];
    if (fhat) st = plan_forward(p, fhat[j], f[j]);
    if (st == SGL_OK && y) st = plan_adjoint(p, y[j], ghat[j]);
    p.stream = keep;
  }
  for (int k = 0; k < ns && e == hipSuccess; ++k) {
    e = hipEventRecord(b->events[1 + k], b->side[k]);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->capture, b->events[1 + k], 0);
  }
  const hipError_t ee = hipStreamEndCapture(b->capture, &b->graph);
  if (st != SGL_OK) return st;
  SGL_TRY(e);
  SGL_TRY(ee);
  SGL_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return SGL_OK;
}

extern "C" {

sgl_status sgl_batch_create(sgl_batch_t *out, const sgl_plan_t *plans, int32_t n, const void *const *fhat_dev,
                            void *const *f_dev, const void *const *y_dev, void *const *ghat_dev, int32_t nstreams,
                            void *stream) {
  if (!out) return SGL_E_INVAL;
  *out = nullptr;
  if (!plans || n < 1 || n > 4096 || nstreams < 1 || nstreams > 16) return SGL_E_INVAL;
  if (!fhat_dev != !f_dev || !y_dev != !ghat_dev || (!fhat_dev && !y_dev)) return SGL_E_INVAL;
  int dev = -1;
  for (int j = 0; j < n; ++j) {
    if (check_plan(plans[j]) != SGL_OK) return SGL_E_INVAL;
    const Plan &p = plans[j]->p;
    if (p.prof.on) return SGL_E_INVAL;
    if (j == 0) dev = p.device;
    if (p.device != dev) return SGL_E_INVAL;
    for (int i = 0; i < j; ++i)
      if (plans[i] == plans[j]) return SGL_E_INVAL;
    const size_t cb = cbytes(p), nf = sgl_num_coeffs(p.B) * cb, ny = (size_t)p.M * cb;
    if (fhat_dev && (!fhat_dev[j] || !f_dev[j] || overlaps(fhat_dev[j], nf, f_dev[j], ny))) return SGL_E_INVAL;
    if (y_dev && (!y_dev[j] || !ghat_dev[j] || overlaps(ghat_dev[j], nf, y_dev[j], ny))) return SGL_E_INVAL;
  }
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != dev) return SGL_E_INVAL;
  sgl_batch_s *b = new (std::nothrow) sgl_batch_s;
  if (!b) return SGL_E_NOMEM;
  b->stream = (hipStream_t)stream;
  hipError_t e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
  for (int k = 0; k < nstreams && e == hipSuccess; ++k) {
    hipStream_t t = nullptr;
    e = hipStreamCreateWithFlags(&t, hipStreamNonBlocking);
    if (e == hipSuccess) b->side.push_back(t);
  }
  for (int k = 0; k <= nstreams && e == hipSuccess; ++k) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->events.push_back(ev);
  }
  sgl_status st = from_hip(e);
  if (st == SGL_OK) st = batch_capture(b, plans, n, fhat_dev, f_dev, y_dev, ghat_dev);
  if (st != SGL_OK) {
    batch_free(b);
    return st;
  }
  *out = b;
  return SGL_OK;
}

sgl_status sgl_batch_run(sgl_batch_t batch) {
  if (!batch) return SGL_E_INVAL;
  return from_hip(hipGraphLaunch(batch->exec, batch->stream));
}

sgl_status sgl_batch_destroy(sgl_batch_t batch) {
  if (!batch) return SGL_E_INVAL;
  hipStreamSynchronize(batch->stream);
  batch_free(batch);
  return SGL_OK;
}

// ---------------------------------------------------------------- learned weights

int32_t sgl_mlp_num_params(void) { return mlp_num_params(); }

sgl_status sgl_point_features(sgl_plan_t plan, const void *points_dev, float *feat_dev) {
  if (check_plan(plan) != SGL_OK || !points_dev || !feat_dev) return SGL_E_INVAL;
  return from_hip(launch_point_features(plan->p, points_dev, feat_dev));
}

sgl_status sgl_mlp_forward(sgl_plan_t plan, const float *params_dev, const float *feat_dev, float *c_dev) {
  if (check_plan(plan) != SGL_OK || !params_dev || !feat_dev || !c_dev) return SGL_E_INVAL;
  return from_hip(launch_mlp_forward(params_dev, feat_dev, plan->p.M, c_dev, plan->p.stream));
}

sgl_status sgl_mlp_backward(sgl_plan_t plan, const float *params_dev, const float *feat_dev, const float *dc_dev,
                            float *grad_dev) {
  if (check_plan(plan) != SGL_OK || !params_dev || !feat_dev || !dc_dev || !grad_dev) return SGL_E_INVAL;
  return from_hip(launch_mlp_backward(params_dev, feat_dev, dc_dev, plan->p.M, grad_dev, plan->p.stream));
}

sgl_status sgl_mlp_backward_noalloc(sgl_plan_t plan, const float *params_dev, const float *feat_dev,
                                    const float *dc_dev, float *grad_dev) {
  if (check_plan(plan) != SGL_OK || !params_dev || !feat_dev || !dc_dev || !grad_dev) return SGL_E_INVAL;
  if (plan->p.M > SGL_MLP_NOALLOC_MAX_POINTS) return SGL_E_UNSUPPORTED;
  return from_hip(launch_mlp_backward_noalloc(params_dev, feat_dev, dc_dev, plan->p.M, grad_dev, plan->p.stream,
                                              plan->p.device));
}

sgl_status sgl_mlp_adam(sgl_plan_t plan, float *params_dev, const float *grad_dev, float *m_dev, float *v_dev,
                        float lr, float beta1, float beta2, float eps, int32_t step) {
  if (check_plan(plan) != SGL_OK || !params_dev || !grad_dev || !m_dev || !v_dev || step < 1 || !(lr > 0.0f) ||
      !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return SGL_E_INVAL;
  return from_hip(launch_adam(params_dev, grad_dev, m_dev, v_dev, mlp_num_params(), lr, beta1, beta2, eps, step,
                              plan->p.stream));
}

sgl_status sgl_mlp_weights(sgl_plan_t plan, const float *c_dev, const float *feat_dev, void *w_dev) {
  if (check_plan(plan) != SGL_OK || !feat_dev || !w_dev) return SGL_E_INVAL;
  return from_hip(launch_mlp_weights(plan->p, c_dev, feat_dev, w_dev));
}

sgl_status sgl_mlp_weight_grad(sgl_plan_t plan, const void *y_dev, const void *g_dev, const void *w_dev,
                               double scale, float *dc_dev) {
  if (check_plan(plan) != SGL_OK || !y_dev || !g_dev || !w_dev || !dc_dev || !std::isfinite(scale))
    return SGL_E_INVAL;
  return from_hip(launch_weight_grad(plan->p, y_dev, g_dev, w_dev, scale, false, dc_dev));
}

// One training step of the weight network on coefficient vectors drawn by the
// caller: y = Lambda fhat_b, w = weights(MLP(feat)), e_b = Lambda^H (w y) - fhat_b,
// loss = mean_b |e_b|^2 / |fhat_b|^2; dL/dc from g = Lambda e_b; backward; Adam.
struct TrainLayout {  // byte offsets into the training workspace, each 256-aligned
  size_t y, t, e, w, c, dc, grad, norms, bytes;
  explicit TrainLayout(const Plan &p) {
    const size_t M = (size_t)p.M, nc = (size_t)sgl_num_coeffs(p.B), cb = cbytes(p);
    size_t o = 0;
    auto take = [&o](size_t n) {
      const size_t at = o;
      o += (n + 255) & ~(size_t)255;
      return at;
    };
    y = take(M * cb);
    t = take(M * cb);
    e = take(nc * cb);
    w = take(M * cb / 2);
    c = take(M * sizeof(float));
    dc = take(M * sizeof(float));
    grad = take((size_t)mlp_num_params() * sizeof(float));
    norms = take(2 * sizeof(double));
    bytes = o;
  }
};

static sgl_status train_step(Plan &p, float *params, float *m, float *v, const float *feat, const char *fhat,
                             int nbatch, float lr, int step, double *loss, char *ws) {
  const int64_t M = p.M, nc = sgl_num_coeffs(p.B);
  const size_t cb = cbytes(p);
  const TrainLayout L(p);
  char *y = ws + L.y, *t = ws + L.t, *e = ws + L.e, *w = ws + L.w;
  float *c = (float *)(ws + L.c), *dc = (float *)(ws + L.dc), *grad = (float *)(ws + L.grad);
  double *norms = (double *)(ws + L.norms);
  hipStream_t s = p.stream;
  SGL_TRY(launch_mlp_forward(params, feat, M, c, s));
  SGL_TRY(launch_mlp_weights(p, c, feat, w));
  double total = 0.0;
  for (int b = 0; b < nbatch; ++b) {
    const char *fh = fhat + (size_t)b * nc * cb;
    sgl_status st = plan_forward(p, fh, y);
    if (st != SGL_OK) return st;
    SGL_TRY(launch_scale_by(p, t, y, w, M));
    if ((st = plan_adjoint(p, t, e)) != SGL_OK) return st;
    SGL_TRY(launch_sub_from(p, e, fh, nc));
    SGL_TRY(launch_norm2(p, e, nc, norms));
    SGL_TRY(launch_norm2(p, fh, nc, norms + 1));
    double hn[2];
    SGL_TRY(hipMemcpyAsync(hn, norms, sizeof hn, hipMemcpyDeviceToHost, s));
    SGL_TRY(hipStreamSynchronize(s));
    if (!(hn[1] > 0.0)) return SGL_E_INVAL;  // a zero coefficient vector
    total += hn[0] / hn[1];
    if ((st = plan_forward(p, e, t)) != SGL_OK) return st;
    SGL_TRY(launch_weight_grad(p, y, t, w, 1.0 / (nbatch * hn[1]), b > 0, dc));
  }
  SGL_TRY(launch_mlp_backward(params, feat, dc, M, grad, s));
  SGL_TRY(launch_adam(params, grad, m, v, mlp_num_params(), lr, 0.9f, 0.999f, 1e-8f, step, s));
  SGL_TRY(hipStreamSynchronize(s));
  *loss = total / nbatch;
  return SGL_OK;
}

sgl_status sgl_mlp_train_step(sgl_plan_t plan, float *params_dev, float *m_dev, float *v_dev, const float *feat_dev,
                              const void *fhat_dev, int32_t nbatch, float lr, int32_t step, double *loss) {
  if (check_plan(plan) != SGL_OK || !params_dev || !m_dev || !v_dev || !feat_dev || !fhat_dev || !loss ||
      nbatch < 1 || step < 1 || !(lr > 0.0f))
    return SGL_E_INVAL;
  Plan &p = plan->p;
  void *ws = nullptr;
  if (hipMalloc(&ws, TrainLayout(p).bytes) != hipSuccess) return SGL_E_NOMEM;
  const sgl_status st = train_step(p, params_dev, m_dev, v_dev, feat_dev, (const char *)fhat_dev, nbatch, lr, step,
                                   loss, (char *)ws);
  hipStreamSynchronize(p.stream);
  hipFree(ws);
  return st;
}

sgl_status sgl_forward(sgl_plan_t plan, const void *fhat_dev, void *f_dev) {
  if (check_plan(plan) != SGL_OK || !fhat_dev || !f_dev) return SGL_E_INVAL;
  Plan &p = plan->p;
  const size_t cb = cbytes(p);
  if (overlaps(fhat_dev, sgl_num_coeffs(p.B) * cb, f_dev, (size_t)p.M * cb)) return SGL_E_INVAL;
  return plan_forward(p, fhat_dev, f_dev);
}

sgl_status sgl_adjoint(sgl_plan_t plan, const void *f_dev, void *fhat_dev) {
  if (check_plan(plan) != SGL_OK || !fhat_dev || !f_dev) return SGL_E_INVAL;
  Plan &p = plan->p;
  const size_t cb = cbytes(p);
  if (overlaps(fhat_dev, sgl_num_coeffs(p.B) * cb, f_dev, (size_t)p.M * cb)) return SGL_E_INVAL;
  return plan_adjoint(p, f_dev, fhat_dev);
}

// Second scratch set and stream for sgl_forward_adjoint.
static sgl_status pair_setup(sgl_plan_s *h) {
  if (h->paired) return SGL_OK;
  Plan a = h->p;  // shares every read-only array of the plan
  a.prof = Profiler();
  a.beta = a.zeta = a.eta = a.bufX = a.bufY = a.bufZ = nullptr;
  a.stream = nullptr;
  hipError_t e = alloc_scratch(a);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&a.stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->join, hipEventDisableTiming);
  if (e != hipSuccess) {
    free_scratch(a);
    if (a.stream) hipStreamDestroy(a.stream);
    if (h->fork) hipEventDestroy(h->fork);
    if (h->join) hipEventDestroy(h->join);
    h->fork = h->join = nullptr;
    return from_hip(e);
  }
  h->adj = a;
  h->paired = true;
  return SGL_OK;
}

sgl_status sgl_forward_adjoint(sgl_plan_t plan, const void *fhat_dev, void *f_dev, const void *y_dev,
                               void *ghat_dev) {
  if (check_plan(plan) != SGL_OK || !fhat_dev || !f_dev || !y_dev || !ghat_dev) return SGL_E_INVAL;
  Plan &p = plan->p;
  const size_t cb = cbytes(p), nf = sgl_num_coeffs(p.B) * cb, ny = (size_t)p.M * cb;
  if (overlaps(fhat_dev, nf, f_dev, ny) || overlaps(ghat_dev, nf, y_dev, ny) || overlaps(f_dev, ny, y_dev, ny) ||
      overlaps(f_dev, ny, ghat_dev, nf) || overlaps(fhat_dev, nf, ghat_dev, nf))
    return SGL_E_INVAL;
  if (p.prof.on) {  // one stream, so that every stage is timed on its own
    const sgl_status st = plan_forward(p, fhat_dev, f_dev);
    return st != SGL_OK ? st : plan_adjoint(p, y_dev, ghat_dev);
  }
  sgl_status st = pair_setup(plan);
  if (st != SGL_OK) return st;
  Plan &a = plan->adj;
  SGL_TRY(hipEventRecord(plan->fork, p.stream));
  SGL_TRY(hipStreamWaitEvent(a.stream, plan->fork, 0));
  // the adjoint's scatter shares the CUs: the narrow gather leaves it registers
  // (the FP64 matrix-core scatter needs a CU's LDS to itself, so there the
  // wide gather is kept)
  p.gather_narrow = !p.mfma64;
  st = plan_forward(p, fhat_dev, f_dev);
  p.gather_narrow = false;
  const sgl_status sa = plan_adjoint(a, y_dev, ghat_dev);
  // the caller's stream waits for the adjoint, whatever happened on either side
  const hipError_t e1 = hipEventRecord(plan->join, a.stream);
  const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(p.stream, plan->join, 0) : e1;
  if (st != SGL_OK) return st;
  if (sa != SGL_OK) return sa;
  return from_hip(e2);
}

sgl_status sgl_plan_rho(sgl_plan_t plan, double *rho) {
  if (check_plan(plan) != SGL_OK || !rho) return SGL_E_INVAL;
  *rho = plan->p.rho;
  return SGL_OK;
}

sgl_status sgl_plan_info(sgl_plan_t plan, int64_t info[12]) {
  if (check_plan(plan) != SGL_OK || !info) return SGL_E_INVAL;
  const Plan &p = plan->p;
  const int64_t v[12] = {p.M, p.N[0], p.N[1], p.N[2], p.E[0], p.E[1], p.E[2],
                         p.L[0], p.L[1], p.L[2], (int64_t)p.bytes, p.mfma ? 2 : (p.mfma64 ? 3 : p.gather_mode)};
  std::memcpy(info, v, sizeof(v));
  return SGL_OK;
}

sgl_status sgl_plan_profile(sgl_plan_t plan, int32_t enable) {
  if (check_plan(plan) != SGL_OK) return SGL_E_INVAL;
  Plan &p = plan->p;
  if (!enable) {
    prof_collect(p);
    p.prof.on = false;
    return SGL_OK;
  }
  if (p.prof.pool.empty()) {
    p.prof.pool.resize(8192);
    for (auto &e : p.prof.pool) {
      const hipError_t err = hipEventCreate(&e);
      if (err != hipSuccess) {
        e = nullptr;
        for (auto &x : p.prof.pool)
          if (x) hipEventDestroy(x);
        p.prof.pool.clear();
        return from_hip(err);
      }
    }
  }
  p.prof.on = true;
  return SGL_OK;
}

sgl_status sgl_plan_stage_times(sgl_plan_t plan, double ms[SGL_NUM_STAGES], int64_t counts[SGL_NUM_STAGES],
                                int32_t reset) {
  if (check_plan(plan) != SGL_OK || !ms || !counts) return SGL_E_INVAL;
  Plan &p = plan->p;
  prof_collect(p);
  for (int i = 0; i < SGL_NUM_STAGES; ++i) {
    ms[i] = p.prof.ms[i];
    counts[i] = p.prof.count[i];
    if (reset) {
      p.prof.ms[i] = 0.0;
      p.prof.count[i] = 0;
    }
  }
  return SGL_OK;
}

sgl_status sgl_destroy(sgl_plan_t plan) {
  if (!plan) return SGL_E_INVAL;
  prof_release(plan->p);
  hipStreamSynchronize(plan->p.stream);
  if (plan->paired) {
    hipStreamSynchronize(plan->adj.stream);
    free_scratch(plan->adj);
    hipStreamDestroy(plan->adj.stream);
    hipEventDestroy(plan->fork);
    hipEventDestroy(plan->join);
  }
  free_plan(plan->p);
  delete plan;
  return SGL_OK;
}

const char *sgl_last_error(void) { return g_last_error; }

const char *sgl_status_string(sgl_status s) {
  switch (s) {
    case SGL_OK: return "ok";
    case SGL_E_INVAL: return "invalid argument";
    case SGL_E_RANGE: return "rho smaller than the largest point radius";
    case SGL_E_NOMEM: return "out of memory";
    case SGL_E_DEVICE: return "HIP device or launch error";
    case SGL_E_UNSUPPORTED: return "unsupported configuration";
  }
  return "unknown status";
}

}  // extern "C"
