// Windowed gather (the evaluation of s(t) of Section 2) and its adjoint
// scatter, with the Gaussian window of Def. 2.5 truncated as in eq. nfft_psi.
// With u_j = N_j t_j / (2 pi), the 2q taps per dimension are the integers l
// with u_j - q < l <= u_j + q (base cell b = floor(u), taps b-q+1 .. b+q), and
//     s(t) = sum_taps g[l mod N] prod_j exp(-(u_j - l_j)^2 / (2 lambda)),
// where the constant (2 pi lambda)^{-3/2} has been moved into the
// deconvolution factors applied in the FFT passes.
//
// The grid g is stored pruned: in dimensions 0 and 1 (angles in [0, pi])
// only rows l in [1-q, N_j/2 + q] are kept (stored index l - lo), in
// dimension 2 the whole period (stored index l mod N).
//
//  * gather (tiled): one workgroup per chunk of points of one tile of base
//    cells; the tile's window box is staged in LDS and sixteen lanes (one LDS
//    pass group) evaluate a point together.
//  * gather (slabs): for windows too wide for the whole box in LDS, the box
//    of a chunk's tile is streamed through LDS a few dimension-0 planes at a
//    time, sixteen lanes per point, the points' partial sums kept in
//    registers.
//  * scatter (tiled): one workgroup per chunk accumulates all taps of its
//    points into the tile's window box, held as register rows, and writes the
//    box to a staging slot of its own; a fold pass then sums, for every stored
//    cell, the boxes that cover it in a fixed order.  No atomics of any kind:
//    every grid cell is written by exactly one workgroup.
//  * scatter (cell-owned): output-driven, for any cutoff (used where the
//    window box does not fit in LDS); each workgroup owns a block of stored
//    cells, every thread a row of that block in registers, and sums the taps
//    of every point whose window reaches the block in a fixed order; the
//    block is written once.
//  * FP32 plans with tiles of 8^3 cells use the matrix-core forms instead
//    (k_gather_mfma, k_spread_mfma): the dimension-2 contraction of the gather
//    and the contraction over the points of the scatter run as FP16 hi/lo
//    products with FP32 accumulation; the staging and fold are shared.  FP64
//    plans with 8^3 tiles (q <= 6) scatter on the FP64 matrix cores
//    (k_spread_mfma64), with exact FP64 products.
#include <type_traits>

#include "sgl_internal.h"

namespace sgl {

namespace {

struct Geom {
  int q;
  int N[3], E[3], lo[3], pruned[3];
  int L[3], T[3], X[3], NB[3];
  int Lo[3], To[3];
  int S01;  // plane stride of the tiled gather's LDS box, >= X1 X2
  int SR;   // row stride of the slab gather's LDS slabs, >= X2
};

__device__ inline int stored_index(int l, int j, const Geom &g) {
  if (g.pruned[j]) {
    const int s = l - g.lo[j];
    return (s >= 0 && s < g.E[j]) ? s : -1;
  }
  if (l >= 0 && l < g.N[j]) return l;
  const int s = l % g.N[j];
  return s < 0 ? s + g.N[j] : s;
}

template <class R>
__device__ inline R gauss(R d, R inv2lam) {
  return exp(-d * d * inv2lam);
}

// ---------------------------------------------------------------- gather, tiled

// Tiled gather: a workgroup copies the window box of its tile (X0 x X1 x X2
// grid values around L0 x L1 x L2 base cells) into LDS once and evaluates
// its chunk of points there.  Sixteen lanes share one point as a 4 x 4 grid
// (a, b) over the rows of the window: lane (a, b) takes the rows (t0, t1) =
// (a + 4 j0, b + 4 j1) and runs the dimension-2 sums along them, and the
// sixteen partial sums are added in a fixed butterfly.  A 16-byte LDS read is
// served sixteen lanes per pass over 64 banks, and on gfx950 the lanes of a
// pass are, within each half wave, the quads of four lanes whose quad index
// (lane % 32) / 4 has even bit parity, or those with odd parity (measured with
// the bank-conflict counter on lane pairs).  A point takes one such group, so
// that a pass reads one point's rows only; the box planes lie S01 >= X1 X2
// values apart, with S01 chosen on the host so that those sixteen rows fall in
// sixteen distinct groups of four banks (a value is 16 bytes in FP64).  The
// gather is bound by LDS bandwidth, and rows of different points meeting in a
// pass cost it a quarter more in bank conflicts.
// The window values of a point are computed once, by its sixteen lanes (at
// most three exponentials each), into an LDS slot of the point that all
// sixteen lanes then read; the box fill divides by the box edges in single
// precision, which is exact here.
// 1,024-thread workgroups run 16 waves per CU; the narrow form (256 threads)
// leaves registers for a scatter running beside it on the same CU, with the
// same sums and so the same bits.
template <int Q2>
struct GatherTiled {
  static constexpr int threads = Q2 <= 12 ? 1024 : Q2 <= 16 ? 512 : 256;
  static constexpr int J = (Q2 + 3) / 4;  // rows per lane along dimensions 0 and 1
  // values of a point slot: w2 at t = 0 .. Q2 - 1, then w0 and w1 at the
  // rows a + 4 j (b + 4 j) of the four lanes a (b), j < J
  static constexpr int nwv = Q2 + 8 * J;
  // slot stride: 16 modulo 32 values, so that the two points of a 32-lane
  // pass of 8-byte reads meet opposite halves of the banks
  static constexpr int ws = nwv <= 16 ? 16 : (nwv + 15) / 32 * 32 + 16;
  template <class R>
  static constexpr size_t slot_bytes(int nthreads) {
    return (size_t)(nthreads / 16) * ws * sizeof(R);
  }
};
constexpr int kGatherLanes = 16;
// largest box the tiled gather takes: the fill's single-precision division is
// exact for element indices below 2^14
constexpr int kGatherBoxMax = 1 << 14;

template <class R, int Q2>
__global__ __launch_bounds__(GatherTiled<Q2>::threads) void k_gather_tiled(const cplx<R> *__restrict__ grid,
                                                      const PointRec<R> *__restrict__ pts,
                                                      const int32_t *__restrict__ perm,
                                                      const int32_t *__restrict__ chunks, Geom g, R inv2lam,
                                                      cplx<R> *__restrict__ f) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  constexpr int q = Q2 / 2;
  constexpr int J = GatherTiled<Q2>::J, NWV = GatherTiled<Q2>::nwv, WS = GatherTiled<Q2>::ws;
  const int tidx = chunks[3 * blockIdx.x];
  const int start = chunks[3 * blockIdx.x + 1];
  const int count = chunks[3 * blockIdx.x + 2];
  const int c2 = tidx % g.T[2];
  const int c1 = (tidx / g.T[2]) % g.T[1];
  const int c0 = tidx / (g.T[2] * g.T[1]);
  const int X0 = g.X[0], X1 = g.X[1], X2 = g.X[2], S01 = g.S01;
  cplx<R> *tile = (cplx<R> *)smem;
  R *wslots = (R *)(smem + (size_t)X0 * S01 * sizeof(cplx<R>));
  const int wb0 = c0 * g.L[0] - q + 1, wb1 = c1 * g.L[1] - q + 1, wb2 = c2 * g.L[2] - q + 1;
  // e = (i0 X1 + i1) X2 + i2 < 2^14: (e + 1/2) / X2 lies at least 1 / (2 X2)
  // from an integer, and the single-precision product is within 2^-10 of it
  const float rX2 = 1.0f / (float)X2, rX1 = 1.0f / (float)X1;
  for (int e = threadIdx.x; e < X0 * X1 * X2; e += blockDim.x) {
    const int r = (int)(((float)e + 0.5f) * rX2), i2 = e - r * X2;
    const int i0 = (int)(((float)r + 0.5f) * rX1), i1 = r - i0 * X1;
    const int s0 = stored_index(wb0 + i0, 0, g), s1 = stored_index(wb1 + i1, 1, g),
              s2 = stored_index(wb2 + i2, 2, g);
    // two scalars rather than a conditionally assigned pair, which the
    // compiler kept in scratch memory for FP64
    R vr = 0, vi = 0;
    if (s0 >= 0 && s1 >= 0 && s2 >= 0) {
      const cplx<R> v = grid[((size_t)s0 * g.E[1] + s1) * g.E[2] + s2];
      vr = v.re;
      vi = v.im;
    }
    tile[i0 * S01 + i1 * X2 + i2] = cplx<R>{vr, vi};
  }
  __syncthreads();
  // lane -> (point slot, a, b): quad qd = (lane % 32) / 4 of the half wave,
  // group = bit parity of qd; the quads of one group, in order, are a = qd / 2
  // (0, 3, 5, 6 for even parity; 1, 2, 4, 7 for odd), and b = lane % 4.  The
  // sixteen lanes of a point share k, so they are active or inactive together
  // around the exchanges, which stay inside the group (lane xor 1, 2, 12, 20).
  const int lane = threadIdx.x % 64, qd = (lane % 32) / 4;
  const int a = qd >> 1, b = lane % 4, sub = 4 * a + b;
  const int slot = ((int)threadIdx.x / 64) * 4 + (lane / 32) * 2 + (__popc(qd) & 1);
  const bool lead = (lane % 32) == (__popc(qd) & 1) * 4;  // a = 0, b = 0
  R *ws = wslots + slot * WS;
  for (int k = start + slot; k < start + count; k += (int)blockDim.x / kGatherLanes) {
    const PointRec<R> pr = pts[k];
    const int o0 = cell0(pr.cell) - c0 * g.L[0];
    const int o1 = cell1(pr.cell) - c1 * g.L[1];
    const int o2 = cell2(pr.cell) - c2 * g.L[2];
    // the point's window values into its slot, value v by lane v % 16: the
    // value at window offset t is gauss(frac + q - 1 - t), zero past the
    // window (rows a + 4 j >= Q2 of the last j)
#pragma unroll
    for (int m = 0; m < (NWV + 15) / 16; ++m) {
      const int v = sub + 16 * m;
      if (v < NWV) {
        int t;
        R fr;
        if (v < Q2) {
          t = v;
          fr = pr.frac[2];
        } else if (v < Q2 + 4 * J) {
          t = (v - Q2) / J + 4 * ((v - Q2) % J);
          fr = pr.frac[0];
        } else {
          t = (v - Q2 - 4 * J) / J + 4 * ((v - Q2 - 4 * J) % J);
          fr = pr.frac[1];
        }
        ws[v] = t < Q2 ? gauss<R>(fr + (R)(q - 1 - t), inv2lam) : (R)0;
      }
    }
    // the slot's writers and readers are lanes of this wave: LDS operations
    // of a wave complete in order, the fences keep the compiler's order
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    R w0[J], w1[J], w2[Q2];
#pragma unroll
    for (int t = 0; t < Q2; ++t) w2[t] = ws[t];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      w0[j] = ws[Q2 + a * J + j];
      w1[j] = ws[Q2 + 4 * J + b * J + j];
    }
    const cplx<R> *base = tile + (o0 * S01 + o1 * X2 + o2);
    R ar = 0, ai = 0;
#pragma unroll
    for (int j0 = 0; j0 < J; ++j0) {
      // rows past the window read its last row (inside the box) with weight 0
      const cplx<R> *plane = base + min(a + 4 * j0, Q2 - 1) * S01;
      R br = 0, bi = 0;
#pragma unroll
      for (int j1 = 0; j1 < J; ++j1) {
        const cplx<R> *row = plane + min(b + 4 * j1, Q2 - 1) * X2;
        // the reads of half a row are issued before their products, so their
        // LDS latencies overlap (the compiler otherwise keeps one to three in
        // flight; a whole row in flight needs more registers than 16 waves have)
        constexpr int H2 = (Q2 + 1) / 2;
        R cr = 0, ci = 0;
#pragma unroll
        for (int h = 0; h < Q2; h += H2) {
          cplx<R> v[H2];
#pragma unroll
          for (int u = 0; u < H2; ++u) v[u] = h + u < Q2 ? row[h + u] : cplx<R>{0, 0};
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 0; u < H2; ++u) {
            if (h + u < Q2) {
              cr += w2[h + u] * v[u].re;
              ci += w2[h + u] * v[u].im;
            }
          }
        }
        br += w1[j1] * cr;
        bi += w1[j1] * ci;
      }
      ar += w0[j0] * br;
      ai += w0[j0] * bi;
    }
    // butterfly over the group: every lane ends with the same sum
    constexpr int kXor[4] = {1, 2, 12, 20};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      ar += __shfl_xor(ar, kXor[m], 64);
      ai += __shfl_xor(ai, kXor[m], 64);
    }
    if (lead) f[perm[k]] = cplx<R>{ar, ai};
    // the slot is read before the next point's values overwrite it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// ---------------------------------------------------------------- gather, MFMA

// FP32 gather with the dimension-2 contraction on the matrix cores (tiles of
// 8^3 cells).  For one chunk of one tile, the window box G[i0][i1][i2] is
// staged in LDS as four FP16 planes (re/im x hi/lo with hi = fp16(s G),
// lo = fp16(s G - hi), s a power of two that puts the box maximum into
// [2^13, 2^14)).  Rows are (i0, i1) with i1 padded to a multiple of 4, so the
// four D rows of a lane share one i0.  For every group of 16 points,
// T[(i0, i1), p] = sum_i2 G[(i0, i1), i2] w2_p[i2] is a rows x 16 x 32 product
// done as hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_f16 (FP32 accumulation;
// the dropped lo*lo term is ~2^-22 relative), and the remaining sum
// f_p = sum_(i0,i1) w0_p[i0] w1_p[i1] T[(i0, i1), p] runs on the vector units.
// Each wave takes passes of two groups, so every A fragment read from LDS
// serves 32 points.  Weights are box-shifted: w_p[i] = gauss(frac + q - 1 -
// (i - o_p)) for 0 <= i - o_p < 2q, zero elsewhere (also past the box).
typedef _Float16 sgl_half8 __attribute__((ext_vector_type(8)));
typedef _Float16 sgl_half2 __attribute__((ext_vector_type(2)));
typedef _Float16 sgl_half4 __attribute__((ext_vector_type(4)));
typedef float sgl_float4 __attribute__((ext_vector_type(4)));
typedef float sgl_float2 __attribute__((ext_vector_type(2)));
typedef double sgl_double4 __attribute__((ext_vector_type(4)));

constexpr int kPlaneK = 24;  // i2 slots an MFMA row reads; K slots 24..31 meet zero weights
constexpr int kLdsMax = 160 * 1024;

template <int Q2>
struct GatherShape {
  static constexpr int X = 7 + Q2;          // box edge
  static constexpr int X1p = (X + 3) & ~3;  // padded i1 extent of a row group
  static constexpr int nrow = X * X1p;
  static constexpr int nrb = (nrow + 15) / 16;
  static constexpr int NR = nrb * 16;
  // Row stride of the planes in halves.  An MFMA row reads kPlaneK slots; the
  // slots past X belong to the next row (or the pad after the last plane), and
  // they meet zero weights.  20 halves (40 bytes) puts the 16 rows of one read
  // on distinct banks for lanes 0..15; the lanes gfx950 serves together in one
  // pass of 16-byte reads (quads of even or odd index parity) still meet in a
  // few banks (about 0.9 conflict cycles per LDS instruction, measured).
  static constexpr int KS = X <= 20 ? 20 : 24;
  static constexpr int S = ((X1p / 4) % 2 == 0) ? X1p + 4 : X1p;  // w1 floats per point: odd multiple of 4
  // Planes hold nrow rows each.  The last row block reads NR - nrow rows past a
  // plane's end, which lie in the next plane (or in the zeroed tail after the
  // last one); they meet w0 = 0 (i0 past the box), so any finite value serves.
  static constexpr int PS = nrow * KS;  // halves per plane
  static constexpr int tail = (NR - nrow) * KS + 8;
  static constexpr size_t plane_bytes = ((size_t)4 * PS + tail) * sizeof(_Float16);
  static constexpr size_t tab_bytes(int waves) { return (size_t)waves * 32 * S * sizeof(float); }
  static constexpr size_t static_bytes(int waves) { return 4 * waves + 3 * 32 * 4; }  // red, sidx
  static constexpr size_t need(int waves) { return plane_bytes + tab_bytes(waves) + static_bytes(waves); }
  // Two blocks per CU when LDS allows (one block's box staging then overlaps
  // the other's products), else one block of as many waves as fit.
  static constexpr int waves2 = need(8) <= kLdsMax / 2 ? 8 : need(6) <= kLdsMax / 2 ? 6 : need(4) <= kLdsMax / 2 ? 4 : 0;
  static constexpr int waves = waves2 ? waves2 : need(16) <= kLdsMax ? 16 : need(12) <= kLdsMax ? 12 : 8;
  static constexpr int threads = 64 * waves;
  static constexpr int items = nrow * (KS / 2);  // staged pairs of i2 slots
  static constexpr int KB = (items + threads - 1) / threads;
  static constexpr size_t lds = plane_bytes + tab_bytes(waves);
};

// eight halves at p (8-byte aligned)
__device__ inline sgl_half8 ld_half8(const _Float16 *p) {
  const sgl_half4 a = *(const sgl_half4 *)p, b = *(const sgl_half4 *)(p + 4);
  return __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7);
}

template <int Q2>
__global__ __launch_bounds__(GatherShape<Q2>::threads) void k_gather_mfma(const cplx<float> *__restrict__ grid,
                                                                          const PointRec<float> *__restrict__ pts,
                                                                          const int32_t *__restrict__ perm,
                                                                          const int32_t *__restrict__ chunks,
                                                                          Geom g, float inv2lam,
                                                                          cplx<float> *__restrict__ f) {
  using Sh = GatherShape<Q2>;
  constexpr int q = Q2 / 2, X = Sh::X, X1p = Sh::X1p, NR = Sh::NR, S = Sh::S, KS = Sh::KS;
  constexpr int NW = Sh::waves, NT = Sh::threads;
  constexpr int PS = Sh::PS;            // halves per plane
  constexpr int UR = (Q2 >= 10 && Q2 < 16) ? 2 : 1;  // row blocks in flight per wave (as registers allow)
  static_assert(X <= KS && KS <= kPlaneK, "box too long along dimension 2");
  static_assert(Sh::need(Sh::waves) <= kLdsMax, "LDS budget");
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  _Float16 *plane = (_Float16 *)smem;              // [4][nrow][KS] + tail: re_hi, re_lo, im_hi, im_lo
  float *wtab = (float *)(plane + 4 * PS + Sh::tail);  // [NW][32 points][S]: w1 at [0, X1p)
  __shared__ float red[NW];
  __shared__ int sidx[3][32];

  const int tidx = chunks[3 * blockIdx.x];
  const int start = chunks[3 * blockIdx.x + 1];
  const int count = chunks[3 * blockIdx.x + 2];
  const int c0 = tidx / (g.T[2] * g.T[1]), c1 = (tidx / g.T[2]) % g.T[1], c2 = tidx % g.T[2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

  // 1. stored grid index of every box coordinate (-1: outside the stored grid)
  if (threadIdx.x < 96) {
    const int d = threadIdx.x / 32, i = threadIdx.x % 32;
    const int cd = d == 0 ? c0 : (d == 1 ? c1 : c2);
    sidx[d][i] = i < X ? stored_index(cd * 8 - q + 1 + i, d, g) : -1;
  } else if (threadIdx.x < 96 + Sh::tail) {
    plane[4 * PS + threadIdx.x - 96] = (_Float16)0.0f;  // the tail the last row block's reads run into
  }
  __syncthreads();
  // 2. the box (with its zero padding) in registers, pairs of i2 slots per item
  cplx<float> v[Sh::KB][2];
  float mx = 0.0f;
#pragma unroll
  for (int u = 0; u < Sh::KB; ++u) {
    const int e = threadIdx.x + u * NT;
    v[u][0] = v[u][1] = cplx<float>{0.0f, 0.0f};
    if (e < Sh::items) {
      const int r = e / (KS / 2), kp = e % (KS / 2);
      const int i0 = r / X1p, i1 = r % X1p;
      if (i0 < X && i1 < X) {
        const int s0 = sidx[0][i0], s1 = sidx[1][i1];
        if (s0 >= 0 && s1 >= 0) {
          const size_t base = ((size_t)s0 * g.E[1] + s1) * g.E[2];
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const int k = 2 * kp + c;
            const int s2 = k < X ? sidx[2][k] : -1;
            if (s2 >= 0) v[u][c] = grid[base + s2];
          }
        }
      }
      mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v[u][0].re), fabsf(v[u][0].im)), fmaxf(fabsf(v[u][1].re), fabsf(v[u][1].im))));
    }
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  if (lane == 0) red[wave] = mx;
  __syncthreads();
  float bmx = 0.0f;
  for (int w = 0; w < NW; ++w) bmx = fmaxf(bmx, red[w]);
  int ex = 0;
  if (bmx > 0.0f) frexpf(bmx, &ex);     // bmx = m 2^ex, m in [0.5, 1)
  // scaled maximum in [2^13, 2^14) (the FP32 range caps the scale for denormal boxes)
  const float sc = ldexpf(1.0f, min(14 - ex, 126));
  // 3. FP16 hi/lo planes
#pragma unroll
  for (int u = 0; u < Sh::KB; ++u) {
    const int e = threadIdx.x + u * NT;
    if (e < Sh::items) {
      const int o = (e / (KS / 2)) * KS + 2 * (e % (KS / 2));
      const sgl_float2 re = {v[u][0].re * sc, v[u][1].re * sc}, im = {v[u][0].im * sc, v[u][1].im * sc};
      const sgl_half2 rh = __builtin_convertvector(re, sgl_half2), ih = __builtin_convertvector(im, sgl_half2);
      const sgl_half2 rl = __builtin_convertvector(sgl_float2{re[0] - (float)rh[0], re[1] - (float)rh[1]}, sgl_half2);
      const sgl_half2 il = __builtin_convertvector(sgl_float2{im[0] - (float)ih[0], im[1] - (float)ih[1]}, sgl_half2);
      *(sgl_half2 *)(plane + o) = rh;
      *(sgl_half2 *)(plane + PS + o) = rl;
      *(sgl_half2 *)(plane + 2 * PS + o) = ih;
      *(sgl_half2 *)(plane + 3 * PS + o) = il;
    }
  }
  __syncthreads();

  // 4. every wave takes passes of 32 points (two groups of 16)
  const int pl = lane & 15, h = lane >> 4;
  const int ha = h < 3 ? h : 2;  // lanes h = 3 meet the zero K rows 24..31 of B; any finite A serves
  const float kexp = -inv2lam * 1.4426950408889634f;
  const float inv = 1.0f / sc;
  const int npass = (count + 31) / 32;
  float *tb0 = wtab + (size_t)(wave * 32 + pl) * S, *tb1 = tb0 + 16 * S;
  // the point records of the wave's next pass are loaded while it works on the current one
  PointRec<float> nxt[2];
  auto fetch = [&](int ps) {
#pragma unroll
    for (int gi = 0; gi < 2; ++gi) {
      const int idx = ps * 32 + gi * 16 + pl;
      if (ps < npass && idx < count) nxt[gi] = pts[start + idx];
    }
  };
  fetch(wave);
  for (int ps = wave; ps < npass; ps += NW) {
    sgl_half8 bh[2], bl[2];
    int kk[2], o0[2];
    float d0[2];  // w0 at i0 is gauss(d0 - i0) inside the window
    bool valid[2];
    const PointRec<float> cur[2] = {nxt[0], nxt[1]};
    fetch(ps + NW);
#pragma unroll
    for (int gi = 0; gi < 2; ++gi) {
      const int idx = ps * 32 + gi * 16 + pl;
      valid[gi] = idx < count;
      kk[gi] = start + idx;
      float fr0 = 0.0f, fr1 = 0.0f, fr2 = 0.0f;
      int o1 = 1 << 20, o2 = 1 << 20;  // outside every box when invalid
      o0[gi] = 1 << 20;
      if (valid[gi]) {
        const PointRec<float> pr = cur[gi];
        fr0 = pr.frac[0];
        fr1 = pr.frac[1];
        fr2 = pr.frac[2];
        o0[gi] = cell0(pr.cell) - c0 * 8;
        o1 = cell1(pr.cell) - c1 * 8;
        o2 = cell2(pr.cell) - c2 * 8;
      }
      d0[gi] = fr0 + (float)(q - 1 + o0[gi]);
      float *tb = gi ? tb1 : tb0;
#pragma unroll
      for (int i1 = 0; i1 < X1p; i1 += 4) {
        const int t = i1 + h - o1;
        const float d = fr1 + (float)(q - 1 - t);
        tb[i1 + h] = ((unsigned)t < (unsigned)Q2) ? __builtin_amdgcn_exp2f(d * d * kexp) : 0.0f;
      }
      float w[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int t = 8 * h + j - o2;
        const float d = fr2 + (float)(q - 1 - t);
        w[j] = (h < 3 && (unsigned)t < (unsigned)Q2) ? __builtin_amdgcn_exp2f(d * d * kexp) : 0.0f;
      }
#pragma unroll
      for (int j = 0; j < 8; j += 2) {
        const sgl_half2 hh = __builtin_convertvector(sgl_float2{w[j], w[j + 1]}, sgl_half2);
        const sgl_half2 ll =
            __builtin_convertvector(sgl_float2{w[j] - (float)hh[0], w[j + 1] - (float)hh[1]}, sgl_half2);
        bh[gi][j] = hh[0];
        bh[gi][j + 1] = hh[1];
        bl[gi][j] = ll[0];
        bl[gi][j + 1] = ll[1];
      }
    }
    // rows of box i0 outside every window of the pass have w0 = 0 for all its
    // points: only the row blocks that meet [min o0, max o0 + Q2) contribute
    int lo = min(valid[0] ? o0[0] : X, valid[1] ? o0[1] : X);
    int hi = max(valid[0] ? o0[0] : 0, valid[1] ? o0[1] : 0);
    for (int o = 1; o < 16; o <<= 1) {
      lo = min(lo, __shfl_xor(lo, o));
      hi = max(hi, __shfl_xor(hi, o));
    }
    const int rb_lo = __builtin_amdgcn_readfirstlane((lo * X1p) / 16);
    const int rb_hi = __builtin_amdgcn_readfirstlane(min(Sh::nrb, ((hi + Q2) * X1p + 15) / 16));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float ar[2] = {0.0f, 0.0f}, ai[2] = {0.0f, 0.0f};
#pragma unroll UR
    for (int rb = rb_lo; rb < rb_hi; ++rb) {
      const _Float16 *ap = plane + (rb * 16 + pl) * KS + 8 * ha;
      const sgl_half8 a0 = ld_half8(ap);
      const sgl_half8 a1 = ld_half8(ap + PS);
      const sgl_half8 a2 = ld_half8(ap + 2 * PS);
      const sgl_half8 a3 = ld_half8(ap + 3 * PS);
      // rows 4h .. 4h+3 of the block: one i0, i1 = i1b .. i1b+3
      const int r4 = rb * 16 + 4 * h;
      const int i0 = r4 / X1p, i1b = r4 - (r4 / X1p) * X1p;
      // four independent accumulation chains, interleaved
      sgl_float4 dr0 = {0, 0, 0, 0}, di0 = {0, 0, 0, 0}, dr1 = {0, 0, 0, 0}, di1 = {0, 0, 0, 0};
      dr0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a0, bh[0], dr0, 0, 0, 0);
      di0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2, bh[0], di0, 0, 0, 0);
      dr1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a0, bh[1], dr1, 0, 0, 0);
      di1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2, bh[1], di1, 0, 0, 0);
      dr0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a0, bl[0], dr0, 0, 0, 0);
      di0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2, bl[0], di0, 0, 0, 0);
      dr1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a0, bl[1], dr1, 0, 0, 0);
      di1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a2, bl[1], di1, 0, 0, 0);
      dr0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, bh[0], dr0, 0, 0, 0);
      di0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a3, bh[0], di0, 0, 0, 0);
      dr1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a1, bh[1], dr1, 0, 0, 0);
      di1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(a3, bh[1], di1, 0, 0, 0);
      // w0 of the lane's row group (zero outside the window, e.g. rows past the box)
      const int t00 = i0 - o0[0], t01 = i0 - o0[1];
      const float e0 = d0[0] - (float)i0, e1 = d0[1] - (float)i0;
      const float w00 = ((unsigned)t00 < (unsigned)Q2) ? __builtin_amdgcn_exp2f(e0 * e0 * kexp) : 0.0f;
      const float w01 = ((unsigned)t01 < (unsigned)Q2) ? __builtin_amdgcn_exp2f(e1 * e1 * kexp) : 0.0f;
      const sgl_float4 w10 = *(const sgl_float4 *)(tb0 + i1b);
      const sgl_float4 w11 = *(const sgl_float4 *)(tb1 + i1b);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float cw0 = w00 * w10[j], cw1 = w01 * w11[j];
        ar[0] += cw0 * dr0[j];
        ai[0] += cw0 * di0[j];
        ar[1] += cw1 * dr1[j];
        ai[1] += cw1 * di1[j];
      }
    }
#pragma unroll
    for (int gi = 0; gi < 2; ++gi) {
      // the four lanes of a point hold disjoint rows: sum them
      ar[gi] += __shfl_xor(ar[gi], 16);
      ai[gi] += __shfl_xor(ai[gi], 16);
      ar[gi] += __shfl_xor(ar[gi], 32);
      ai[gi] += __shfl_xor(ai[gi], 32);
      if (valid[gi] && h == 0) f[perm[kk[gi]]] = cplx<float>{ar[gi] * inv, ai[gi] * inv};
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// ---------------------------------------------------------------- gather, slabs

// Gather for windows too wide for the whole box of a tile in LDS (large q):
// one workgroup per chunk streams the box through LDS in slabs of kSlab
// dimension-0 planes.  The chunk's points are taken 64 at a time, sixteen
// lanes per point in one LDS pass group (as in the tiled gather): lane
// (r, h), r < 8, h < 2, sums the rows t1 = r + 8 m of every plane of the
// point's window that the slab holds, over the taps t2 = 2 j + h.  Slab rows
// lie SR values apart with SR = 2 (mod 4), chosen on the host, so the sixteen
// values read together (r SR + h) fall in sixteen distinct groups of banks,
// and a lane keeps only its half of the point's dimension-2 window in
// registers.  The point's window values along all three dimensions are
// computed once per point, by its sixteen lanes, into an LDS slot; the
// partial sums stay in registers across the slabs and the sixteen lanes add
// them in a fixed butterfly.
constexpr int kSlab = 4;
constexpr int kSlabThreads = 1024;
template <int Q2>
struct GatherSlab {
  static constexpr int M = (Q2 + 7) / 8;  // rows per lane and plane
  static constexpr int H = Q2 / 2;        // taps per lane and row
  // slot: w0 and w1 at window offsets 0 .. Q2 - 1, then w2 at the even and
  // at the odd offsets; stride 16 modulo 32 values
  static constexpr int nwv = 3 * Q2;
  static constexpr int ws = nwv <= 16 ? 16 : (nwv + 15) / 32 * 32 + 16;
  template <class R>
  static constexpr size_t slot_bytes() {
    return (size_t)(kSlabThreads / 16) * ws * sizeof(R);
  }
};

template <class R, int Q2>
__global__ __launch_bounds__(kSlabThreads) void k_gather_slab(const cplx<R> *__restrict__ grid,
                                                              const PointRec<R> *__restrict__ pts,
                                                              const int32_t *__restrict__ perm,
                                                              const int32_t *__restrict__ chunks, Geom g,
                                                              R inv2lam, cplx<R> *__restrict__ f) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  constexpr int q = Q2 / 2;
  constexpr int M = GatherSlab<Q2>::M, H = GatherSlab<Q2>::H;
  constexpr int NWV = GatherSlab<Q2>::nwv, WS = GatherSlab<Q2>::ws;
  const int tidx = chunks[3 * blockIdx.x];
  const int start = chunks[3 * blockIdx.x + 1];
  const int count = chunks[3 * blockIdx.x + 2];
  const int c2 = tidx % g.T[2];
  const int c1 = (tidx / g.T[2]) % g.T[1];
  const int c0 = tidx / (g.T[2] * g.T[1]);
  const int X0 = g.X[0], X1 = g.X[1], X2 = g.X[2], SR = g.SR;
  cplx<R> *slab = (cplx<R> *)smem;  // [kSlab][X1][SR]
  R *wslots = (R *)(smem + (size_t)kSlab * X1 * SR * sizeof(cplx<R>));
  const int wb0 = c0 * g.L[0] - q + 1, wb1 = c1 * g.L[1] - q + 1, wb2 = c2 * g.L[2] - q + 1;
  // lane -> (point slot, sub) by LDS pass group, as in the tiled gather
  const int lane = threadIdx.x % 64, qd = (lane % 32) / 4;
  const int sub = 4 * (qd >> 1) + lane % 4, rr = sub >> 1, hh = sub & 1;
  const int slot = ((int)threadIdx.x / 64) * 4 + (lane / 32) * 2 + (__popc(qd) & 1);
  const bool lead = (lane % 32) == (__popc(qd) & 1) * 4;  // sub = 0
  R *ws = wslots + slot * WS;
  // slab element e = (ip X1 + i1) X2 + i2 < 2^14: exact single-precision division
  const float rX2 = 1.0f / (float)X2, rX1 = 1.0f / (float)X1;
  for (int pass = 0; pass < count; pass += kSlabThreads / 16) {
    const int idx = pass + slot;
    const bool valid = idx < count;
    PointRec<R> pr;
    pr.frac[0] = pr.frac[1] = pr.frac[2] = 0;
    pr.cell = 0;
    int o0 = 1 << 20, o1 = 0, o2 = 0;  // no plane of any slab when invalid
    if (valid) {
      pr = pts[start + idx];
      o0 = cell0(pr.cell) - c0 * g.L[0];
      o1 = cell1(pr.cell) - c1 * g.L[1];
      o2 = cell2(pr.cell) - c2 * g.L[2];
    }
    // the point's window values, value v by lane v % 16: v = d Q2 + t for
    // d = 0, 1; w2 at offset t in 2 Q2 + (t % 2) H + t / 2
#pragma unroll
    for (int m = 0; m < (NWV + 15) / 16; ++m) {
      const int v = sub + 16 * m;
      if (v < NWV) {
        const int d = v / Q2, u = v - d * Q2;
        const int t = d < 2 ? u : (u < H ? 2 * u : 2 * (u - H) + 1);
        const R fr = d == 0 ? pr.frac[0] : (d == 1 ? pr.frac[1] : pr.frac[2]);
        ws[v] = gauss<R>(fr + (R)(q - 1 - t), inv2lam);
      }
    }
    // writers and readers of the slot are lanes of this wave
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    R w2[H], w1[M];
#pragma unroll
    for (int j = 0; j < H; ++j) w2[j] = ws[2 * Q2 + hh * H + j];
    // rows past the window read its last row (inside the box) with weight 0
#pragma unroll
    for (int m = 0; m < M; ++m) w1[m] = rr + 8 * m < Q2 ? ws[Q2 + rr + 8 * m] : (R)0;
    R ar = 0, ai = 0;
    for (int s0 = 0; s0 < X0; s0 += kSlab) {
      const int np = min(kSlab, X0 - s0);
      __syncthreads();  // the previous slab is consumed
      for (int e = threadIdx.x; e < np * X1 * X2; e += kSlabThreads) {
        const int r = (int)(((float)e + 0.5f) * rX2), i2 = e - r * X2;
        const int ip = (int)(((float)r + 0.5f) * rX1), i1 = r - ip * X1;
        const int sa = stored_index(wb0 + s0 + ip, 0, g), sb = stored_index(wb1 + i1, 1, g),
                  sc = stored_index(wb2 + i2, 2, g);
        R vr = 0, vi = 0;
        if (sa >= 0 && sb >= 0 && sc >= 0) {
          const cplx<R> v = grid[((size_t)sa * g.E[1] + sb) * g.E[2] + sc];
          vr = v.re;
          vi = v.im;
        }
        slab[r * SR + i2] = cplx<R>{vr, vi};
      }
      __syncthreads();
      // planes of this slab inside the point's window
      const int p_lo = max(s0, o0), p_hi = min(s0 + np, o0 + Q2);
      for (int i0 = p_lo; i0 < p_hi; ++i0) {
        const R w0 = ws[i0 - o0];
        const cplx<R> *plane = slab + (size_t)(i0 - s0) * X1 * SR + o2 + hh;
        R br = 0, bi = 0;
#pragma unroll
        for (int m = 0; m < M; ++m) {
          const cplx<R> *row = plane + (size_t)(o1 + min(rr + 8 * m, Q2 - 1)) * SR;
          R cr = 0, ci = 0;
#pragma unroll
          for (int j = 0; j < H; ++j) {
            const cplx<R> v = row[2 * j];
            cr += w2[j] * v.re;
            ci += w2[j] * v.im;
            if (j % 4 == 3) __builtin_amdgcn_sched_barrier(0);
          }
          br += w1[m] * cr;
          bi += w1[m] * ci;
          // bounds how far the scheduler hoists the row reads (registers)
          __builtin_amdgcn_sched_barrier(0);
        }
        ar += w0 * br;
        ai += w0 * bi;
      }
    }
    // butterfly over the group: every lane ends with the same sum
    constexpr int kXor[4] = {1, 2, 12, 20};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      ar += __shfl_xor(ar, kXor[m], 64);
      ai += __shfl_xor(ai, kXor[m], 64);
    }
    if (valid && lead) f[perm[start + idx]] = cplx<R>{ar, ai};
    // the slot is read before the next pass's values overwrite it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// ---------------------------------------------------------------- gradient in x

// For the gradient of f = Lambda fhat with respect to the point positions
// (rho fixed): the NFFT sum f = sum_l alpha_l prod_j w(u_j - l_j) differentiates
// through the window, d w(d) / d u = -(d / lambda) w(d), and u_j = N_j x~_j / 2 pi
// with x~ = (2 atan2(sqrt(rho - r), sqrt(r)), theta, phi) (eq. x_tilde):
//   d x~_0 / d x = -x / (r sqrt(r (rho - r))),
//   d theta / d x = (x z, y z, -rxy^2) / (r^2 rxy),   d phi / d x = (-y, x, 0) / rxy^2.
// Output: grad_ic = Re(conj(g_i) d f_i / d x_ic), the gradient of a real loss
// whose gradient with respect to f is g (conjugate Wirtinger convention).
// At r = rho (x~_0 = 0, the outermost point of a plan whose rho is max r) the
// factor d x~_0 / d r is unbounded while d f / d x~_0 vanishes: f depends on
// x~_0 only through cos x~_0 = (2r - rho)/rho, so with F(cos t) = f(t),
// d f / d r = (2/rho) F'(1) = -(2/rho) d^2 f / d x~_0^2 at t = 0.  That limit
// is taken for rho - r <= 1e-14 rho (t <= 2e-7, where its O((2B t)^2)
// relative error is below 1e-9).  Undefined (NaN) on the z axis, at the
// origin and at r > rho.
template <class R, int Q2>
__global__ __launch_bounds__(256) void k_grad_points(const cplx<R> *__restrict__ grid,
                                                     const PointRec<R> *__restrict__ pts,
                                                     const int32_t *__restrict__ perm, int64_t M, Geom g,
                                                     double lam, double rho, const R *__restrict__ xyz,
                                                     const cplx<R> *__restrict__ gin, R *__restrict__ grad) {
  constexpr int q = Q2 / 2;
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= M) return;
  const PointRec<R> pr = pts[k];
  const int i = perm[k];
  const int b0 = cell0(pr.cell), b1 = cell1(pr.cell), b2 = cell2(pr.cell);
  const R inv2lam = (R)(0.5 / lam), invlam = (R)(1.0 / lam);
  R w2[Q2], d2[Q2];
  int i2[Q2];
#pragma unroll
  for (int t = 0; t < Q2; ++t) {
    const R d = pr.frac[2] + (R)(q - 1 - t);
    w2[t] = gauss<R>(d, inv2lam);
    d2[t] = -d * invlam * w2[t];
    i2[t] = stored_index(b2 - q + 1 + t, 2, g);
  }
  // dimension-1 window, its derivative and stored rows: in FP64 with windows of
  // up to 12 taps computed once up front (kept in registers, the loop over them
  // unrolled; B = 64, M = 4e6: 12.1 -> 9.7 ms per differentiation step), else
  // inside the loop over t0 (in FP32 the extra registers cost more than the
  // exponentials save: 2.9 -> 3.6 ms at B = 48, M = 2e6)
  constexpr bool kHoist1 = Q2 <= 12 && sizeof(R) == sizeof(double);
  R w1h[kHoist1 ? Q2 : 1], dw1h[kHoist1 ? Q2 : 1];
  int s1h[kHoist1 ? Q2 : 1];
  if constexpr (kHoist1) {
#pragma unroll
    for (int t1 = 0; t1 < Q2; ++t1) {
      const R e1 = pr.frac[1] + (R)(q - 1 - t1);
      w1h[t1] = gauss<R>(e1, inv2lam);
      dw1h[t1] = -e1 * invlam * w1h[t1];
      s1h[t1] = stored_index(b1 - q + 1 + t1, 1, g);
    }
  }
  cplx<R> f0 = {0, 0}, f1 = {0, 0}, f2 = {0, 0};  // d f / d u_0, u_1, u_2
  cplx<R> f00 = {0, 0};                             // d^2 f / d u_0^2
  for (int t0 = 0; t0 < Q2; ++t0) {
    const int s0 = stored_index(b0 - q + 1 + t0, 0, g);
    const R e0 = pr.frac[0] + (R)(q - 1 - t0);
    const R w0 = gauss<R>(e0, inv2lam), dw0 = -e0 * invlam * w0;
    const R ddw0 = (e0 * e0 * invlam - (R)1) * invlam * w0;
    cplx<R> a = {0, 0}, a1 = {0, 0}, a2 = {0, 0};
#pragma unroll(kHoist1 ? Q2 : 1)
    for (int t1 = 0; t1 < Q2; ++t1) {
      int s1;
      R w1, dw1;
      if constexpr (kHoist1) {
        s1 = s1h[t1];
        w1 = w1h[t1];
        dw1 = dw1h[t1];
      } else {
        s1 = stored_index(b1 - q + 1 + t1, 1, g);
        const R e1 = pr.frac[1] + (R)(q - 1 - t1);
        w1 = gauss<R>(e1, inv2lam);
        dw1 = -e1 * invlam * w1;
      }
      const cplx<R> *row = grid + ((size_t)s0 * g.E[1] + s1) * g.E[2];
      cplx<R> c = {0, 0}, cd = {0, 0};
#pragma unroll
      for (int t2 = 0; t2 < Q2; ++t2) {
        const cplx<R> v = row[i2[t2]];
        c.re += w2[t2] * v.re;
        c.im += w2[t2] * v.im;
        cd.re += d2[t2] * v.re;
        cd.im += d2[t2] * v.im;
      }
      a.re += w1 * c.re;
      a.im += w1 * c.im;
      a1.re += dw1 * c.re;
      a1.im += dw1 * c.im;
      a2.re += w1 * cd.re;
      a2.im += w1 * cd.im;
    }
    f0.re += dw0 * a.re;
    f0.im += dw0 * a.im;
    f00.re += ddw0 * a.re;
    f00.im += ddw0 * a.im;
    f1.re += w0 * a1.re;
    f1.im += w0 * a1.im;
    f2.re += w0 * a2.re;
    f2.im += w0 * a2.im;
  }
  // chain rule in double
  const double x = (double)xyz[3 * (size_t)i], y = (double)xyz[3 * (size_t)i + 1], z = (double)xyz[3 * (size_t)i + 2];
  const double rxy = hypot(x, y), r = hypot(rxy, z);
  const cplx<R> gv = gin[i];
  // Re(conj(g) df/du_j) times du_j / d x~_j = N_j / 2 pi
  const double inv2pi = 0.15915494309189533576888376337251436;
  const double c0 = ((double)gv.re * f0.re + (double)gv.im * f0.im) * g.N[0] * inv2pi;
  const double c1 = ((double)gv.re * f1.re + (double)gv.im * f1.im) * g.N[1] * inv2pi;
  const double c2 = ((double)gv.re * f2.re + (double)gv.im * f2.im) * g.N[2] * inv2pi;
  double gx = NAN, gy = NAN, gz = NAN;
  if (rxy > 0.0 && r <= rho) {
    // Re(conj(g) d f / d r): the chain rule through d x~_0 / d r = -1 / sqrt(r (rho - r)),
    // or its limit at x~_0 = 0
    double drad;
    if (rho - r > 1e-14 * rho) {
      drad = -c0 / sqrt(r * (rho - r));
    } else {
      const double s0 = g.N[0] * inv2pi;
      drad = -2.0 / rho * ((double)gv.re * f00.re + (double)gv.im * f00.im) * s0 * s0;
    }
    const double r2 = r * r, rxy2 = rxy * rxy;
    gx = drad * x / r + c1 * x * z / (r2 * rxy) - c2 * y / rxy2;
    gy = drad * y / r + c1 * y * z / (r2 * rxy) + c2 * x / rxy2;
    gz = drad * z / r - c1 * rxy / r2;
  }
  grad[3 * (size_t)i] = (R)gx;
  grad[3 * (size_t)i + 1] = (R)gy;
  grad[3 * (size_t)i + 2] = (R)gz;
}

// ---------------------------------------------------------------- scatter


// Bins (tiles of base cells) in dimension j whose points can touch stored
// cells [S, S + ext): merged disjoint bin intervals [first, last].
__host__ __device__ inline int bin_ranges(int S, int ext, int j, const Geom &g, int *first, int *last) {
  const int q = g.q, L = g.L[j], NB = g.NB[j];
  int cand_lo[3], cand_hi[3], nc = 0;
  if (g.pruned[j]) {
    // stored s = b + t, t in [0, 2q)
    const int lo = max(0, S - 2 * q + 1), hi = min(NB - 1, S + ext - 1);
    if (lo <= hi) {
      cand_lo[nc] = lo;
      cand_hi[nc] = hi;
      ++nc;
    }
  } else {
    const int N = g.N[j];
    const int blo = S - q, bhi = S + ext - 1 + q - 1;  // bases, modulo N
    if (bhi - blo + 1 >= N) {
      cand_lo[nc] = 0;
      cand_hi[nc] = NB - 1;
      ++nc;
    } else {
      for (int w = -1; w <= 1; ++w) {
        const int lo = max(0, blo + w * N), hi = min(NB - 1, bhi + w * N);
        if (lo <= hi) {
          cand_lo[nc] = lo;
          cand_hi[nc] = hi;
          ++nc;
        }
      }
    }
  }
  // to bins, then merge (candidates are increasing in base)
  int n = 0;
  for (int c = 0; c < nc; ++c) {
    const int f0 = cand_lo[c] / L, l0 = cand_hi[c] / L;
    if (n > 0 && f0 <= last[n - 1] + 0) {
      if (l0 > last[n - 1]) last[n - 1] = l0;
    } else {
      first[n] = f0;
      last[n] = l0;
      ++n;
    }
  }
  return n;
}

// FP64 matrix-core form of the tiled spreading (FP64 data, tiles of 8^3
// cells): for the points of one chunk the window box is the product
//   D[(i0, i1)][(i2, c)] = sum_p (w0_p[i0] w1_p[i1]) (y_p^c w2_p[i2]),
// c = re, im, on v_mfma_f64_16x16x4f64 with K = 4 points per step: A[row][p]
// = w0 w1, B[p][col] with the real and imaginary parts interleaved along the
// columns (col = 2 i2 + c, 2X columns in three blocks of 16 for X <= 24), so
// every product is an exact FP64 multiply-add.  The workgroup's waves split
// into two roles over double-buffered LDS tables of kSB64 points: while
// kSpread64Prod waves multiply batch b out of one buffer, the other waves load
// batch b + 1 and build its w0 and w1 tables and B in the other buffer (one
// thread per point and dimension; each thread clears the entries it wrote
// into that buffer two batches before, so the tables are zero outside the
// windows without a clearing pass), and one barrier per batch hands the
// buffers over.  Product wave w owns the row blocks w, w + kSpread64Prod, ...
// of the box for the whole chunk (accumulators in registers) and skips, per K
// step, the row blocks outside [min o0, max o0 + 2q) and the column blocks
// past 2 (max o2 + 2q) of its four points (A or B = 0 there).  The box goes
// to the chunk's staging slot; the fold sums the boxes.  No atomics.
constexpr int kSpread64Threads = 1024;  // 16 waves
constexpr int kSpread64Prod = 12;       // product waves; waves 12 .. 15 build tables
constexpr int kSB64 = 64;               // points per batch
constexpr int kTW64 = 33;               // doubles per w0/w1 table row (box index, padded)
constexpr int kBT64 = 50;               // doubles per B row (48 columns, padded)

template <int Q2>
__global__ __launch_bounds__(kSpread64Threads) void k_spread_mfma64(const cplx<double> *__restrict__ y,
                                                                    const PointRec<double> *__restrict__ pts,
                                                                    const int32_t *__restrict__ perm,
                                                                    const int32_t *__restrict__ chunks, Geom g,
                                                                    double inv2lam,
                                                                    cplx<double> *__restrict__ staging) {
  constexpr int q = Q2 / 2;
  constexpr int X = 8 + Q2 - 1;  // box edge in every dimension
  constexpr int nrow = X * X;
  constexpr int nrb = (nrow + 15) / 16;
  constexpr int NCB = (2 * X + 15) / 16;
  constexpr int NW = kSpread64Prod;
  constexpr int RBW = (nrb + NW - 1) / NW;
  static_assert(X <= 24 && NCB <= 3, "box edge exceeds three column blocks");
  static_assert((nrb * 16 - 1) / X < 32, "row index past the weight tables");
  static_assert(kSpread64Threads - 64 * NW >= 3 * kSB64, "one builder thread per point and dimension");
  // tw[buf][d][p][i]: w_d of point p at box index i, d = 0, 1; zero outside
  // the point's window, in particular for i >= X (rows past the box) and for
  // the invalid points of a partial batch.  bt[buf][p][col]: B, zero past 2X.
  __shared__ double tw[2][2][kSB64][kTW64];
  __shared__ double bt[2][kSB64][kBT64];
  __shared__ int srb[2][kSB64 / 4][3];  // row blocks a K step of 4 points meets, column blocks it needs

  const int tidx = chunks[3 * blockIdx.x];
  const int start = chunks[3 * blockIdx.x + 1];
  const int count = chunks[3 * blockIdx.x + 2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int pl = lane & 15, kq = lane >> 4;
  const int c0 = tidx / (g.T[2] * g.T[1]), c1 = (tidx / g.T[2]) % g.T[1], c2 = tidx % g.T[2];
  const int nbatch = (count + kSB64 - 1) / kSB64;

  // both table buffers start at zero
  for (int e = threadIdx.x; e < 2 * 2 * kSB64 * kTW64; e += kSpread64Threads) (&tw[0][0][0][0])[e] = 0.0;
  for (int e = threadIdx.x; e < 2 * kSB64 * kBT64; e += kSpread64Threads) (&bt[0][0][0])[e] = 0.0;

  // builder role: thread (bd, bp) handles dimension bd of point bp of a batch
  const bool builder = wave >= NW;
  const int tb = (int)threadIdx.x - 64 * NW;
  const int bd = tb / kSB64, bp = tb % kSB64;  // bd = 3: idle
  const int ct = bd == 0 ? c0 : (bd == 1 ? c1 : c2);
  int oprev0 = -1, oprev1 = -1;  // window start this thread wrote into buffer 0 / 1 (-1: none)
  // raw data of the thread's point of the next batch to build
  bool nval = false;
  double nfr = 0.0, nyre = 0.0, nyim = 0.0;
  int ncell = 0;
  auto fetch = [&](int b) {
    nval = builder && bd < 3 && b < nbatch && b * kSB64 + bp < count;
    if (nval) {
      const int k = start + b * kSB64 + bp;
      nfr = pts[k].frac[bd];
      ncell = pts[k].cell;
      if (bd == 2) {
        const cplx<double> v = y[perm[k]];
        nyre = v.re;
        nyim = v.im;
      }
    }
  };
  // tables of batch b into buffer buf from the fetched data, then fetch b + 1
  // (builder waves only; the thread's own entries, so no barrier inside)
  auto build = [&](int b, int buf) {
    const bool valid = nval;
    const double fr = nfr, yre = nyre, yim = nyim;
    const int cell = ncell;
    fetch(b + 1);
    if (bd >= 3) return;
    const int o = valid ? (bd == 0 ? cell0(cell) : (bd == 1 ? cell1(cell) : cell2(cell))) - ct * 8 : -1;
    const int op = buf ? oprev1 : oprev0;
    if (op >= 0) {
      for (int t = 0; t < Q2; ++t) {
        if (bd < 2) {
          tw[buf][bd][bp][op + t] = 0.0;
        } else {
          bt[buf][bp][2 * (op + t)] = 0.0;
          bt[buf][bp][2 * (op + t) + 1] = 0.0;
        }
      }
    }
    if (valid) {
      // window values by the Gaussian recurrence: with d_t = frac + q - 1 - t,
      // w_{t+1} = w_t r_t, r_t = exp((2 d_t - 1) / (2 lambda)),
      // r_{t+1} = r_t exp(-1 / lambda)
      const double cc = exp(-2.0 * inv2lam);
      const double d0 = fr + (double)(q - 1);
      double w = exp(-d0 * d0 * inv2lam), r = exp((2.0 * d0 - 1.0) * inv2lam);
      for (int t = 0; t < Q2; ++t) {
        if (bd < 2) {
          tw[buf][bd][bp][o + t] = w;
        } else {
          bt[buf][bp][2 * (o + t)] = yre * w;
          bt[buf][bp][2 * (o + t) + 1] = yim * w;
        }
        w *= r;
        r *= cc;
      }
    }
    if (buf) oprev1 = o; else oprev0 = o;
    // row blocks of a K step: rows i0 * X + i1 with i0 outside
    // [min o0, max o0 + Q2) of its points have A = 0, so the step only needs
    // the row blocks that meet that range; columns 2 i2 + c with i2 at or past
    // max o2 + Q2 have B = 0, so it only needs the column blocks below
    // 2 (max o2 + Q2).  Groups of four lanes of the dimension-0 and dimension-2
    // waves hold the four points of a step.
    if (bd == 0) {
      int lo = valid ? o : X, hi = valid ? o : 0;
      lo = min(lo, __shfl_xor(lo, 1, 64));
      hi = max(hi, __shfl_xor(hi, 1, 64));
      lo = min(lo, __shfl_xor(lo, 2, 64));
      hi = max(hi, __shfl_xor(hi, 2, 64));
      if ((bp & 3) == 0) {
        srb[buf][bp / 4][0] = lo < X ? (lo * X) / 16 : nrb;
        srb[buf][bp / 4][1] = lo < X ? min(nrb, ((hi + Q2) * X + 15) / 16) : nrb;
      }
    } else if (bd == 2) {
      int hi2 = valid ? o : 0;
      hi2 = max(hi2, __shfl_xor(hi2, 1, 64));
      hi2 = max(hi2, __shfl_xor(hi2, 2, 64));
      if ((bp & 3) == 0) srb[buf][bp / 4][2] = min(NCB, (2 * min(X, hi2 + Q2) + 15) / 16);
    }
  };

  sgl_double4 acc[RBW][NCB];
#pragma unroll
  for (int r = 0; r < RBW; ++r)
#pragma unroll
    for (int n = 0; n < NCB; ++n) acc[r][n] = sgl_double4{0.0, 0.0, 0.0, 0.0};

  fetch(0);
  __syncthreads();  // tables zeroed
  if (builder) build(0, 0);
  __syncthreads();
  for (int b = 0; b < nbatch; ++b) {
    const int buf = b & 1;
    if (!builder) {
      const int nb = min(kSB64, count - b * kSB64);
      // products over the batch, K = 4 points per step
      for (int ks = 0; ks < nb; ks += 4) {
        const int kr_lo = srb[buf][ks / 4][0], kr_hi = srb[buf][ks / 4][1], kc_hi = srb[buf][ks / 4][2];
        const int pp = ks + kq;  // this lane's point of the K step (A column, B row)
        double bf[NCB], a[RBW];
#pragma unroll
        for (int n = 0; n < NCB; ++n) bf[n] = bt[buf][pp][16 * n + pl];
        // A fragments of every owned row block, read whether or not the step
        // needs the block, so that one wait covers all of the step's LDS reads
        // (i0 clamped for blocks past the box, whose fragment goes unused)
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
          const int row = (wave + r * NW) * 16 + pl;
          const int i0 = min(row / X, kTW64 - 1), i1 = row - (row / X) * X;
          a[r] = tw[buf][0][pp][i0] * tw[buf][1][pp][i1];
        }
        // keeps the compiler from sinking the reads into the branch below
#pragma unroll
        for (int r = 0; r < RBW; ++r) __asm__ volatile("" ::"v"(a[r]));
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
          const int rb = wave + r * NW;
          if (rb < nrb && rb >= kr_lo && rb < kr_hi) {
#pragma unroll
            for (int n = 0; n < NCB; ++n)
              if (n < kc_hi) acc[r][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r], bf[n], acc[r][n], 0, 0, 0);
          }
        }
      }
    } else if (b + 1 < nbatch) {
      build(b + 1, buf ^ 1);
    }
    __syncthreads();  // batch b consumed, batch b + 1 built
  }
  if (builder) return;
  // D[kq + 4v][pl] of every (row block, column block) to the chunk's box
  double *out = (double *)(staging + (size_t)blockIdx.x * nrow * X);
#pragma unroll
  for (int r = 0; r < RBW; ++r) {
    const int rb = wave + r * NW;
    if (rb < nrb) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rb * 16 + kq + 4 * v;
        if (row < nrow) {
#pragma unroll
          for (int n = 0; n < NCB; ++n) {
            const int col = 16 * n + pl;  // 2 i2 + c
            if (col < 2 * X) out[(size_t)row * 2 * X + col] = acc[r][n][v];
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------- scatter, cell-owned

// Output-driven spreading without atomics, for any cutoff q: a workgroup owns
// a block of kOwn^3 stored cells and sums into registers the taps of the
// points whose windows reach the block.  The candidate points of a block (the
// points of the bins that can reach it, in bin order) are split at plan time
// into segments of at most kOwnSeg points, one work item each, so dense
// blocks do not serialise the launch: a block with one segment is written to
// the grid directly, the segments of a denser block write partial blocks to
// slots of their own that k_fold_owned sums in segment order.  Thread (u0, u1) owns the block's row
// of kOwn cells along dimension 2, so each cell has exactly one writer and its
// sum runs over the points in a fixed order (the candidate bins in index
// order, the points of a bin in their sorted order): the result is
// deterministic and the block is written once.
// Per batch of kOwnBatch points the workgroup stages in LDS, for every point,
// its window restricted to the block along each dimension (kOwn values per
// dimension, zero outside the 2q taps) and its sample; a thread then adds
// (y w0[u0] w1[u1]) w2[c] to its kOwn cells when its row lies in the point's
// footprint.  A wave owns four consecutive u0 rows, so a point whose window
// misses them costs the wave only the footprint test.
constexpr int kOwn = 16;
constexpr int kOwnThreads = kOwn * kOwn;
constexpr int kOwnSeg = 8192;  // candidate points per work item
constexpr int kOwnBatch = 64;
constexpr int kOwnMaxRows = 3 * 256;

template <class R, int Q2>
__global__ __launch_bounds__(kOwnThreads) void k_scatter_owned(const cplx<R> *__restrict__ y,
                                                               const PointRec<R> *__restrict__ pts,
                                                               const int32_t *__restrict__ perm,
                                                               const int32_t *__restrict__ tile_start,
                                                               const int32_t *__restrict__ work, Geom g,
                                                               R inv2lam, cplx<R> *__restrict__ grid,
                                                               cplx<R> *__restrict__ stage) {
  constexpr int q = Q2 / 2;
  __shared__ R sw[3][kOwnBatch][kOwn];
  __shared__ cplx<R> sy[kOwnBatch];
  __shared__ R sfrac[3][kOwnBatch];
  __shared__ int sbase[3][kOwnBatch];
  __shared__ int row_start[kOwnMaxRows];
  __shared__ int row_pref[kOwnMaxRows + 1];
  __shared__ int rng_f[3][3], rng_l[3][3], rng_n[3];
  // work item: block, first candidate, candidate count (-1: to the end), slot (-1: the grid)
  const int blk = work[4 * blockIdx.x], seg0 = work[4 * blockIdx.x + 1];
  const int segn = work[4 * blockIdx.x + 2], slot = work[4 * blockIdx.x + 3];
  const int C2 = blk % g.To[2];
  const int C1 = (blk / g.To[2]) % g.To[1];
  const int C0 = blk / (g.To[2] * g.To[1]);
  const int S[3] = {C0 * kOwn, C1 * kOwn, C2 * kOwn};
  const int ext0 = min(kOwn, g.E[0] - S[0]), ext1 = min(kOwn, g.E[1] - S[1]), ext2 = min(kOwn, g.E[2] - S[2]);
  // candidate bins per dimension: merged intervals [first, last]
  if (threadIdx.x < 3) {
    const int j = threadIdx.x;
    const int ext = j == 0 ? ext0 : (j == 1 ? ext1 : ext2);
    rng_n[j] = bin_ranges(S[j], ext, j, g, rng_f[j], rng_l[j]);
  }
  __syncthreads();
  // one bin row (x0, x1, a dimension-2 interval) per slot: its point range
  int nr0 = 0, nr1 = 0;
  for (int a = 0; a < rng_n[0]; ++a) nr0 += rng_l[0][a] - rng_f[0][a] + 1;
  for (int a = 0; a < rng_n[1]; ++a) nr1 += rng_l[1][a] - rng_f[1][a] + 1;
  const int n2r = rng_n[2];
  const int nslots = nr0 * nr1 * n2r;  // at most kOwnMaxRows (checked when the plan is made)
  for (int sidx = threadIdx.x; sidx < nslots; sidx += kOwnThreads) {
    const int c = sidx % n2r, pr = sidx / n2r;
    int i0 = pr / nr1, i1 = pr % nr1, x0 = 0, x1 = 0;
    for (int a = 0; a < rng_n[0]; ++a) {
      const int n = rng_l[0][a] - rng_f[0][a] + 1;
      if (i0 < n) { x0 = rng_f[0][a] + i0; break; }
      i0 -= n;
    }
    for (int a = 0; a < rng_n[1]; ++a) {
      const int n = rng_l[1][a] - rng_f[1][a] + 1;
      if (i1 < n) { x1 = rng_f[1][a] + i1; break; }
      i1 -= n;
    }
    const int t0 = (x0 * g.T[1] + x1) * g.T[2];
    const int st = tile_start[t0 + rng_f[2][c]], en = tile_start[t0 + rng_l[2][c] + 1];
    row_start[sidx] = st;
    row_pref[sidx] = en - st;  // count, turned into a prefix sum below
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int r = 0; r < nslots; ++r) {
      const int n = row_pref[r];
      row_pref[r] = tot;
      tot += n;
    }
    row_pref[nslots] = tot;
  }
  __syncthreads();
  const int total = row_pref[nslots];
  const int first = min(seg0, total), end = segn < 0 ? total : min(total, seg0 + segn);
  const int u0 = threadIdx.x / kOwn, u1 = threadIdx.x % kOwn;
  R are[kOwn], aim[kOwn];
#pragma unroll
  for (int c = 0; c < kOwn; ++c) are[c] = aim[c] = 0;
  for (int b0 = first; b0 < end; b0 += kOwnBatch) {
    const int nb = min(kOwnBatch, end - b0);
    // 1. the batch's point records and samples
    if ((int)threadIdx.x < nb) {
      const int gidx = b0 + threadIdx.x;
      int lo = 0, hi = nslots - 1;
      while (lo < hi) {  // last slot with row_pref <= gidx
        const int mid = (lo + hi + 1) / 2;
        if (row_pref[mid] <= gidx) lo = mid; else hi = mid - 1;
      }
      const int k = row_start[lo] + (gidx - row_pref[lo]);
      const PointRec<R> pr = pts[k];
      sfrac[0][threadIdx.x] = pr.frac[0];
      sfrac[1][threadIdx.x] = pr.frac[1];
      sfrac[2][threadIdx.x] = pr.frac[2];
      sbase[0][threadIdx.x] = cell0(pr.cell);
      sbase[1][threadIdx.x] = cell1(pr.cell);
      sbase[2][threadIdx.x] = cell2(pr.cell);
      sy[threadIdx.x] = y[perm[k]];
    }
    __syncthreads();
    // 2. each point's window on the block, per dimension: tap t of cell u
    //    (stored index S + u) or zero
    for (int e = threadIdx.x; e < 3 * kOwnBatch * kOwn; e += kOwnThreads) {
      const int u = e % kOwn, pp = (e / kOwn) % kOwnBatch, j = e / (kOwn * kOwnBatch);
      R w = 0;
      if (pp < nb) {
        const int s = S[j] + u;
        int t;
        if (g.pruned[j]) {
          t = s + g.lo[j] - sbase[j][pp] + q - 1;
        } else {
          t = (s - (sbase[j][pp] - q + 1)) % g.N[j];
          if (t < 0) t += g.N[j];
        }
        if (t >= 0 && t < Q2) w = gauss<R>(sfrac[j][pp] + (R)(q - 1 - t), inv2lam);
      }
      sw[j][pp][u] = w;
    }
    __syncthreads();
    // 3. taps into the thread's row, points in order
    for (int pp = 0; pp < nb; ++pp) {
      const R w01 = sw[0][pp][u0] * sw[1][pp][u1];
      if (w01 != (R)0) {
        const cplx<R> yv = sy[pp];
        const R cr = yv.re * w01, ci = yv.im * w01;
#pragma unroll
        for (int c = 0; c < kOwn; ++c) {
          const R w = sw[2][pp][c];
          are[c] += cr * w;
          aim[c] += ci * w;
        }
      }
    }
    __syncthreads();
  }
  if (slot >= 0) {
    cplx<R> *row = stage + ((size_t)slot * kOwnThreads + threadIdx.x) * kOwn;
#pragma unroll
    for (int c = 0; c < kOwn; ++c) row[c] = cplx<R>{are[c], aim[c]};
  } else if (u0 < ext0 && u1 < ext1) {
    cplx<R> *row = grid + ((size_t)(S[0] + u0) * g.E[1] + (S[1] + u1)) * g.E[2] + S[2];
#pragma unroll
    for (int c = 0; c < kOwn; ++c)
      if (c < ext2) row[c] = cplx<R>{are[c], aim[c]};
  }
}

// Sum of the partial blocks of the blocks with more than one work item, in
// segment order (FP64 sums, written in the plan's precision): fold entry b is
// {block, first slot, number of slots}.
template <class R>
__global__ __launch_bounds__(kOwnThreads) void k_fold_owned(const cplx<R> *__restrict__ stage,
                                                            const int32_t *__restrict__ fold, Geom g,
                                                            cplx<R> *__restrict__ grid) {
  const int blk = fold[3 * blockIdx.x], s0 = fold[3 * blockIdx.x + 1], ns = fold[3 * blockIdx.x + 2];
  const int C2 = blk % g.To[2];
  const int C1 = (blk / g.To[2]) % g.To[1];
  const int C0 = blk / (g.To[2] * g.To[1]);
  const int S0 = C0 * kOwn, S1 = C1 * kOwn, S2 = C2 * kOwn;
  const int ext0 = min(kOwn, g.E[0] - S0), ext1 = min(kOwn, g.E[1] - S1), ext2 = min(kOwn, g.E[2] - S2);
  const int u0 = threadIdx.x / kOwn, u1 = threadIdx.x % kOwn;
  double ar[kOwn], ai[kOwn];
#pragma unroll
  for (int c = 0; c < kOwn; ++c) ar[c] = ai[c] = 0.0;
  for (int k = 0; k < ns; ++k) {
    const cplx<R> *row = stage + ((size_t)(s0 + k) * kOwnThreads + threadIdx.x) * kOwn;
#pragma unroll
    for (int c = 0; c < kOwn; ++c) {
      const cplx<R> v = row[c];
      ar[c] += v.re;
      ai[c] += v.im;
    }
  }
  if (u0 < ext0 && u1 < ext1) {
    cplx<R> *row = grid + ((size_t)(S0 + u0) * g.E[1] + (S1 + u1)) * g.E[2] + S2;
#pragma unroll
    for (int c = 0; c < kOwn; ++c)
      if (c < ext2) row[c] = cplx<R>{(R)ar[c], (R)ai[c]};
  }
}

// ---------------------------------------------------------------- scatter, tiled

// Spreading for one chunk of points of one tile, without atomics: thread r
// owns row (i0, i1) of the tile's window box (X2 cells along dimension 2) in
// registers.  Points are taken in batches: their weights are computed once
// into LDS -- the dimension-2 weights already shifted to the point's offset
// in the box and zero elsewhere -- then every thread walks the batch and,
// when its row lies in the point's footprint, adds c * w2s[i2] to all X2 cells
// of its row with c = y w0[i0 - o0] w1[i1 - o1].  Every register index is
// static.  The box is then written to the chunk's own staging slot;
// k_fold_staging sums overlapping boxes.  The result is independent of
// scheduling.
constexpr int kSpreadBatch = 128;

template <class R, int Q2, int L2>
__global__ __launch_bounds__(512) void k_spread_rows(const cplx<R> *__restrict__ y,
                                                     const PointRec<R> *__restrict__ pts,
                                                     const int32_t *__restrict__ perm,
                                                     const int32_t *__restrict__ chunks, Geom g, R inv2lam,
                                                     cplx<R> *__restrict__ staging) {
  constexpr int q = Q2 / 2;
  constexpr int X2 = L2 + Q2 - 1;
  constexpr int X2P = (X2 + 3) & ~3;  // row stride of the shifted weights
  __shared__ R sw0[kSpreadBatch][Q2], sw1[kSpreadBatch][Q2];
  __shared__ __attribute__((aligned(16))) R sw2[kSpreadBatch][X2P];
  __shared__ int so[kSpreadBatch];
  __shared__ cplx<R> sy[kSpreadBatch];
  const int tidx = chunks[3 * blockIdx.x];
  const int start = chunks[3 * blockIdx.x + 1];
  const int count = chunks[3 * blockIdx.x + 2];
  const int c2 = tidx % g.T[2];
  const int c1 = (tidx / g.T[2]) % g.T[1];
  const int c0 = tidx / (g.T[2] * g.T[1]);
  const int X1 = g.X[1];
  const int nrow = g.X[0] * X1;
  const int i0 = threadIdx.x / X1, i1 = threadIdx.x % X1;
  const bool has_row = (int)threadIdx.x < nrow;
  R are[X2], aim[X2];
#pragma unroll
  for (int i = 0; i < X2; ++i) are[i] = aim[i] = 0;
  for (int b0 = 0; b0 < count; b0 += kSpreadBatch) {
    const int nb = min(kSpreadBatch, count - b0);
    // the workgroup may have fewer threads than a batch has points (boxes of
    // fewer than kSpreadBatch rows): stage with a stride
    for (int e = threadIdx.x; e < nb; e += blockDim.x) {
      const int k = start + b0 + e;
      const PointRec<R> pr = pts[k];
      const int o0 = cell0(pr.cell) - c0 * g.L[0];
      const int o1 = cell1(pr.cell) - c1 * g.L[1];
      const int o2 = cell2(pr.cell) - c2 * g.L[2];
      so[e] = o0 | (o1 << 8);
      sy[e] = y[perm[k]];
#pragma unroll
      for (int t = 0; t < Q2; ++t) {
        sw0[e][t] = gauss<R>(pr.frac[0] + (R)(q - 1 - t), inv2lam);
        sw1[e][t] = gauss<R>(pr.frac[1] + (R)(q - 1 - t), inv2lam);
      }
      for (int c = 0; c < X2P; ++c) {
        const int t = c - o2;
        sw2[e][c] = (t >= 0 && t < Q2) ? gauss<R>(pr.frac[2] + (R)(q - 1 - t), inv2lam) : (R)0;
      }
    }
    __syncthreads();
    if (has_row) {
      // the table reads of a point do not depend on the footprint test (the
      // indices are clamped), so that those of the next points can be issued
      // before this point's multiply-adds
#pragma unroll 4
      for (int pi = 0; pi < nb; ++pi) {
        const int o = so[pi];
        const int t0 = i0 - (o & 255), t1 = i1 - (o >> 8);
        const R w01 = sw0[pi][min(max(t0, 0), Q2 - 1)] * sw1[pi][min(max(t1, 0), Q2 - 1)];
        const cplx<R> yv = sy[pi];
        if ((unsigned)t0 < (unsigned)Q2 && (unsigned)t1 < (unsigned)Q2) {
          const R cr = yv.re * w01, ci = yv.im * w01;
#pragma unroll
          for (int c = 0; c < X2; ++c) {
            const R w = sw2[pi][c];
            are[c] += cr * w;
            aim[c] += ci * w;
          }
        }
      }
    }
    __syncthreads();
  }
  if (has_row) {
    cplx<R> *out = staging + (size_t)blockIdx.x * nrow * X2 + (size_t)threadIdx.x * X2;
#pragma unroll
    for (int i = 0; i < X2; ++i) out[i] = cplx<R>{are[i], aim[i]};
  }
}

// Matrix-core form of the tiled spreading (FP32 data, tiles of 8^3 cells).
// For the points of one chunk the window box of the tile is the product
//   D[(i0, i1)][i2] = sum_p (w0_p[i0] w1_p[i1]) (f_p w2_p[i2]),
// a contraction over the points: A[row][p] = w0 w1 (real), B[p][i2] = f_p w2
// (one matrix for the real and one for the imaginary part), K = 32 points per
// 16x16x32 FP16 product.  Both operands are split into FP16 hi + lo parts
// (A scaled by 2^12, B by a power of two that puts the largest sample seen so
// far into [2^13, 2^14); when a later batch raises it, the accumulators are
// rescaled by the exact power of two).  hi*hi + hi*lo + lo*hi with FP32
// accumulation keeps about 22 significant bits.
// Per batch of kSB points the workgroup stages the w0 and w1 tables and the
// four FP16 planes of B in LDS; each of the 4 waves then owns row blocks of 16
// box rows for the whole chunk and forms its own A fragments, so the
// accumulators stay in registers until the box is written to the staging
// area.  Two workgroups share a compute unit, so one stages its tables while
// the other multiplies, and the point records and samples of the next batch
// are loaded while the current one is multiplied.
constexpr int kSpreadThreads = 256;  // 4 waves
constexpr int kSB = 128;             // points staged at once
constexpr int kTS = kSB + 4;         // floats per weight-table row
constexpr int kBS = kSB + 8;         // halves per B-plane column (one collision per 16-byte
                                     // pass group; 144 clears it, with no measurable gain)
constexpr int kNoExp = -200;         // running exponent before the first nonzero sample


// FP16 hi + lo parts of eight FP32 values (hi rounded to nearest, lo = the
// rounded remainder)
__device__ inline void split8(const float (&v)[8], sgl_half8 &hi, sgl_half8 &lo) {
#pragma unroll
  for (int i = 0; i < 8; i += 2) {
    const sgl_half2 hh = __builtin_convertvector(sgl_float2{v[i], v[i + 1]}, sgl_half2);
    const sgl_half2 ll =
        __builtin_convertvector(sgl_float2{v[i] - (float)hh[0], v[i + 1] - (float)hh[1]}, sgl_half2);
    hi[i] = hh[0];
    hi[i + 1] = hh[1];
    lo[i] = ll[0];
    lo[i + 1] = ll[1];
  }
}

template <int Q2>
__global__ __launch_bounds__(kSpreadThreads) void k_spread_mfma(const cplx<float> *__restrict__ y,
                                                                const PointRec<float> *__restrict__ pts,
                                                                const int32_t *__restrict__ perm,
                                                                const int32_t *__restrict__ chunks, Geom g,
                                                                float inv2lam, cplx<float> *__restrict__ staging) {
  constexpr int q = Q2 / 2;
  constexpr int X = 8 + Q2 - 1;  // box edge in every dimension
  constexpr int nrow = X * X;
  constexpr int nrb = (nrow + 15) / 16;
  constexpr int NW = kSpreadThreads / 64;
  constexpr int RBW = (nrb + NW - 1) / NW;
  static_assert(X <= 32, "box edge exceeds two column blocks");
  static_assert(2 * kSB == kSpreadThreads, "two threads per point");
  // tab[d][i][p]: 64 w_d of point p at box index i, d = 0, 1; zero outside
  // the point's window, in particular for i >= X (rows past the box)
  __shared__ __attribute__((aligned(16))) float tab[2][32][kTS];
  // bpl[plane][i2][p]: FP16 parts of B (re hi, re lo, im hi, im lo)
  __shared__ __attribute__((aligned(16))) _Float16 bpl[4][32][kBS];
  __shared__ __attribute__((aligned(16))) float sfy[kSB][2];  // samples of the batch
  __shared__ float sfr2[kSB];                                 // fractional position along dimension 2
  __shared__ int so2[kSB];                                    // window start along dimension 2 in the box
  __shared__ int srb[kSB / 32][2];                            // row blocks a K step of 32 points meets
  __shared__ int red[2];                                      // exponents of the loader waves' maxima

  const int tidx = chunks[3 * blockIdx.x];
  const int start = chunks[3 * blockIdx.x + 1];
  const int count = chunks[3 * blockIdx.x + 2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int pl = lane & 15, h = lane >> 4;
  // thread roles while staging: point pp; role 0 builds w0 and the dimension-2
  // data, role 1 builds w1 and loads the sample
  const int role = threadIdx.x / kSB, pp = threadIdx.x % kSB;
  const int c0 = tidx / (g.T[2] * g.T[1]), c1 = (tidx / g.T[2]) % g.T[1], c2 = tidx % g.T[2];
  const int ct = role == 0 ? c0 : c1;
  const float kexp = -inv2lam * 1.4426950408889634f;

  // registers holding the next batch
  bool nvalid = false;
  PointRec<float> npr;
  npr.frac[0] = npr.frac[1] = npr.frac[2] = 0.0f;
  npr.cell = 0;
  cplx<float> ny = {0.0f, 0.0f};
  auto fetch = [&](int b0) {
    nvalid = b0 + pp < count;
    if (nvalid) {
      npr = pts[start + b0 + pp];
      if (role == 1) ny = y[perm[start + b0 + pp]];
    }
  };
  fetch(0);

  sgl_float4 acc[RBW][2][2];
#pragma unroll
  for (int r = 0; r < RBW; ++r)
#pragma unroll
    for (int n = 0; n < 2; ++n) acc[r][n][0] = acc[r][n][1] = sgl_float4{0.0f, 0.0f, 0.0f, 0.0f};
  int E = kNoExp;
  float sc = 1.0f;

  for (int b0 = 0; b0 < count; b0 += kSB) {
    // 1. weight tables of dimensions 0 and 1, window data of dimension 2, samples
    {
      const float fr = role == 0 ? npr.frac[0] : npr.frac[1];
      const int cell = role == 0 ? cell0(npr.cell) : cell1(npr.cell);
      const int o = cell - ct * 8;  // in [0, 8) for a valid point: it lies in this tile
#pragma unroll
      for (int i = 0; i < 32; ++i) tab[role][i][pp] = 0.0f;
      if (nvalid) {
#pragma unroll
        for (int t = 0; t < Q2; ++t) {
          const float dd = fr + (float)(q - 1 - t);
          tab[role][o + t][pp] = exp2f(dd * dd * kexp + 6.0f);
        }
      }
      if (role == 0) {
        sfr2[pp] = npr.frac[2];
        so2[pp] = nvalid ? cell2(npr.cell) - c2 * 8 : (1 << 20);
        // rows i0 * X + i1 with i0 outside [min o0, max o0 + Q2) of a K step's
        // points have A = 0 there: the step only needs the row blocks between
        int lo = nvalid ? o : X, hi = nvalid ? o : 0;
        for (int m = 1; m < 32; m <<= 1) {
          lo = min(lo, __shfl_xor(lo, m));
          hi = max(hi, __shfl_xor(hi, m));
        }
        if ((pp & 31) == 0) {
          srb[pp / 32][0] = (lo * X) / 16;
          srb[pp / 32][1] = min(nrb, ((hi + Q2) * X + 15) / 16);
        }
      } else {
        const cplx<float> v = nvalid ? ny : cplx<float>{0.0f, 0.0f};
        sfy[pp][0] = v.re;
        sfy[pp][1] = v.im;
        float mx = fmaxf(fabsf(v.re), fabsf(v.im));
        for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
        int ex = kNoExp;
        if (mx > 0.0f) frexpf(mx, &ex);
        if (lane == 0) red[wave - kSB / 64] = max(ex, kNoExp);
      }
    }
    __syncthreads();
    const int nb = min(kSB, count - b0);
    if (b0 + kSB < count) fetch(b0 + kSB);
    {
      const int eb = max(red[0], red[1]);
      if (eb > E) {
        if (E > kNoExp) {
          const float f = ldexpf(1.0f, E - eb);
#pragma unroll
          for (int r = 0; r < RBW; ++r)
#pragma unroll
            for (int n = 0; n < 2; ++n)
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                acc[r][n][0][j] *= f;
                acc[r][n][1][j] *= f;
              }
        }
        E = eb;
        sc = ldexpf(1.0f, min(14 - E, 126));
      }
    }
    // 2. B planes: work item -> column c = i2, points 8 pg .. 8 pg + 7
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int wi = threadIdx.x + it * kSpreadThreads;
      const int c = wi / (kSB / 8), pg = wi % (kSB / 8);
      float br[8], bi[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int pt = 8 * pg + i;
        const int t = c - so2[pt];
        const float dd = sfr2[pt] + (float)(q - 1 - t);
        const float w = ((unsigned)t < (unsigned)Q2) ? exp2f(dd * dd * kexp) * sc : 0.0f;
        br[i] = sfy[pt][0] * w;
        bi[i] = sfy[pt][1] * w;
      }
      sgl_half8 rh, rl, ih, il;
      split8(br, rh, rl);
      split8(bi, ih, il);
      *(sgl_half8 *)&bpl[0][c][8 * pg] = rh;
      *(sgl_half8 *)&bpl[1][c][8 * pg] = rl;
      *(sgl_half8 *)&bpl[2][c][8 * pg] = ih;
      *(sgl_half8 *)&bpl[3][c][8 * pg] = il;
    }
    __syncthreads();
    // 3. products over the batch, K = 32 points per step
    for (int ks = 0; ks < nb; ks += 32) {
      const int p0 = ks + 8 * h;  // this lane's 8 points of the K step
      const int kr_lo = srb[ks / 32][0], kr_hi = srb[ks / 32][1];
      sgl_half8 brh[2], brl[2], bih[2], bil[2];
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        const int c = 16 * n + pl;
        brh[n] = *(const sgl_half8 *)&bpl[0][c][p0];
        brl[n] = *(const sgl_half8 *)&bpl[1][c][p0];
        bih[n] = *(const sgl_half8 *)&bpl[2][c][p0];
        bil[n] = *(const sgl_half8 *)&bpl[3][c][p0];
      }
#pragma unroll
      for (int r = 0; r < RBW; ++r) {
        const int rb = wave + r * NW;
        if (rb < nrb && rb >= kr_lo && rb < kr_hi) {
          // A fragment: row rb * 16 + pl, points p0 .. p0 + 7
          const int row = rb * 16 + pl;
          const int i0 = row / X, i1 = row - (row / X) * X;  // i0 <= X + 15 / X < 32
          const float *t0 = &tab[0][i0][p0], *t1 = &tab[1][i1][p0];
          const sgl_float4 ua = *(const sgl_float4 *)t0, ub = *(const sgl_float4 *)(t0 + 4);
          const sgl_float4 va = *(const sgl_float4 *)t1, vb = *(const sgl_float4 *)(t1 + 4);
          float a[8];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            a[i] = ua[i] * va[i];
            a[i + 4] = ub[i] * vb[i];
          }
          sgl_half8 ah, al;
          split8(a, ah, al);
#pragma unroll
          for (int n = 0; n < 2; ++n) {
            acc[r][n][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, brh[n], acc[r][n][0], 0, 0, 0);
            acc[r][n][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bih[n], acc[r][n][1], 0, 0, 0);
            acc[r][n][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, brl[n], acc[r][n][0], 0, 0, 0);
            acc[r][n][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bil[n], acc[r][n][1], 0, 0, 0);
            acc[r][n][0] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, brh[n], acc[r][n][0], 0, 0, 0);
            acc[r][n][1] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bih[n], acc[r][n][1], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();  // the batch's tables are consumed
  }
  // D[4h + j][pl] of every row block to the chunk's box in the staging area;
  // 1 / (2^12 sc) applied as two normal powers of two
  const float inv = 1.0f / sc;
  cplx<float> *out = staging + (size_t)blockIdx.x * nrow * X;
#pragma unroll
  for (int r = 0; r < RBW; ++r) {
    const int rb = wave + r * NW;
    if (rb < nrb) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = rb * 16 + 4 * h + j;
        if (row < nrow) {
#pragma unroll
          for (int n = 0; n < 2; ++n) {
            const int col = 16 * n + pl;
            if (col < X)
              out[row * X + col] = cplx<float>{acc[r][n][0][j] * (1.0f / 4096.0f) * inv,
                                               acc[r][n][1][j] * (1.0f / 4096.0f) * inv};
          }
        }
      }
    }
  }
}

constexpr int kMaxCand = 256;

// Sum of the staged window boxes into the stored grid: one workgroup per
// block of F0 x F1 x F2 stored cells; every chunk whose tile's window box
// overlaps the block is added in a fixed order (tiles, then chunks), so the
// result does not depend on scheduling.  Each grid cell is summed in double
// precision and written once in the plan's precision: the sum is rounded only
// when finished, so every cell keeps its error relative to itself (as the
// forward's grid does), and the adjoint FFT that follows computes in FP64.
template <class R>
__global__ __launch_bounds__(256) void k_fold_staging(const cplx<R> *__restrict__ staging,
                                                      const int32_t *__restrict__ tile_chunk,
                                                      Geom g, int F0, int F1, int F2,
                                                      cplx<R> *__restrict__ grid) {
  __shared__ int cand[3][kMaxCand];
  __shared__ int coff[3][kMaxCand];  // region index of the block's first cell
  __shared__ int ncand[3];
  const int Tf1 = (g.E[1] + F1 - 1) / F1, Tf2 = (g.E[2] + F2 - 1) / F2;
  const int C2 = blockIdx.x % Tf2, C1 = (blockIdx.x / Tf2) % Tf1, C0 = blockIdx.x / (Tf2 * Tf1);
  const int S[3] = {C0 * F0, C1 * F1, C2 * F2};
  const int F[3] = {F0, F1, F2};
  const int q = g.q;
  if (threadIdx.x < 3) {
    const int j = threadIdx.x;
    int n = 0;
    for (int c = 0; c < g.T[j] && n < kMaxCand; ++c) {
      // stored index of the first cell of tile c's window box
      const int first = g.pruned[j] ? c * g.L[j] : c * g.L[j] - q + 1;
      int d = S[j] - first;  // region index of the block start
      bool hit;
      if (g.pruned[j]) {
        hit = d < g.X[j] && d + F[j] > 0;
      } else {
        d %= g.N[j];
        if (d < 0) d += g.N[j];
        hit = d < g.X[j] || d + F[j] > g.N[j];
      }
      if (hit) {
        cand[j][n] = c;
        coff[j][n] = d;
        ++n;
      }
    }
    ncand[j] = n;
  }
  __syncthreads();
  const int ext0 = min(F0, g.E[0] - S[0]), ext1 = min(F1, g.E[1] - S[1]), ext2 = min(F2, g.E[2] - S[2]);
  const int ncell = g.X[0] * g.X[1] * g.X[2];
  // Region index of block cell u in a box whose block-start index is d: d + u,
  // modulo N in the periodic dimension (where a box longer than the period
  // holds the same cell more than once, every copy counts).
  const int step0 = g.pruned[0] ? (1 << 30) : g.N[0];
  const int step1 = g.pruned[1] ? (1 << 30) : g.N[1];
  const int step2 = g.pruned[2] ? (1 << 30) : g.N[2];
  for (int e = threadIdx.x; e < ext0 * ext1 * ext2; e += blockDim.x) {
    const int u2 = e % ext2, r = e / ext2, u1 = r % ext1, u0 = r / ext1;
    double ar = 0, ai = 0;
    for (int a = 0; a < ncand[0]; ++a) {
      int j0 = coff[0][a] + u0;
      if (!g.pruned[0] && j0 >= g.N[0]) j0 -= g.N[0];
      for (int i0 = j0; i0 < g.X[0]; i0 += step0) {
        if (i0 < 0) continue;
        for (int b = 0; b < ncand[1]; ++b) {
          int j1 = coff[1][b] + u1;
          if (!g.pruned[1] && j1 >= g.N[1]) j1 -= g.N[1];
          for (int i1 = j1; i1 < g.X[1]; i1 += step1) {
            if (i1 < 0) continue;
            for (int c = 0; c < ncand[2]; ++c) {
              const int tile = (cand[0][a] * g.T[1] + cand[1][b]) * g.T[2] + cand[2][c];
              const int ch0 = tile_chunk[tile], ch1 = tile_chunk[tile + 1];
              if (ch0 == ch1) continue;
              int j2 = coff[2][c] + u2;
              if (!g.pruned[2] && j2 >= g.N[2]) j2 -= g.N[2];
              for (int i2 = j2; i2 < g.X[2]; i2 += step2) {
                if (i2 < 0) continue;
                const size_t off = ((size_t)i0 * g.X[1] + i1) * g.X[2] + i2;
                for (int ch = ch0; ch < ch1; ++ch) {
                  const cplx<R> v = staging[(size_t)ch * ncell + off];
                  ar += v.re;
                  ai += v.im;
                }
              }
            }
          }
        }
      }
    }
    grid[((size_t)(S[0] + u0) * g.E[1] + (S[1] + u1)) * g.E[2] + (S[2] + u2)] = cplx<R>{(R)ar, (R)ai};
  }
}

// ---------------------------------------------------------------- exact NDFT

// p(t_i) = sum_{k in I_n} eta_k e^{i <k, t_i>}, directly (Def. 2.4).
template <class R>
__global__ __launch_bounds__(256) void k_ndft(const cplx<R> *__restrict__ eta, const double *__restrict__ t, int64_t M,
                                              int n0, int n1, int n2, cplx<R> *__restrict__ f) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= M) return;
  const double t0 = t[i], t1 = t[M + i], t2 = t[2 * M + i];
  double ar = 0, ai = 0;
  for (int a = 0; a < n0; ++a) {
    double s0, c0;
    sincos((a - n0 / 2) * t0, &s0, &c0);
    double br = 0, bi = 0;
    for (int b = 0; b < n1; ++b) {
      double s1, c1;
      sincos((b - n1 / 2) * t1, &s1, &c1);
      const cplx<R> *row = eta + ((size_t)a * n1 + b) * n2;
      double cr = 0, ci = 0;
      for (int c = 0; c < n2; ++c) {
        double s2, c2;
        sincos((c - n2 / 2) * t2, &s2, &c2);
        const double er = row[c].re, ei = row[c].im;
        cr += er * c2 - ei * s2;
        ci += er * s2 + ei * c2;
      }
      br += cr * c1 - ci * s1;
      bi += cr * s1 + ci * c1;
    }
    ar += br * c0 - bi * s0;
    ai += br * s0 + bi * c0;
  }
  f[i] = cplx<R>{(R)ar, (R)ai};
}

template <class R>
__global__ __launch_bounds__(256) void k_ndft_adj(const cplx<R> *__restrict__ y, const double *__restrict__ t,
                                                  int64_t M, int n0, int n1, int n2, cplx<R> *__restrict__ eta) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)n0 * n1 * n2) return;
  const int c = (int)(e % n2), b = (int)((e / n2) % n1), a = (int)(e / ((int64_t)n1 * n2));
  const int k0 = a - n0 / 2, k1 = b - n1 / 2, k2 = c - n2 / 2;
  double ar = 0, ai = 0;
  for (int64_t i = 0; i < M; ++i) {
    double s, co;
    sincos(-(k0 * t[i] + k1 * t[M + i] + k2 * t[2 * M + i]), &s, &co);
    const double yr = y[i].re, yi = y[i].im;
    ar += yr * co - yi * s;
    ai += yr * s + yi * co;
  }
  eta[e] = cplx<R>{(R)ar, (R)ai};
}

// Plane stride of the tiled gather's LDS box: the least S >= X1 X2 (and
// within 16 of it) at which the rows a S + b X2, a, b < 4, that the sixteen
// lanes of a point read in one LDS pass fall in 16 distinct value slots modulo
// 16 (a 16-byte value covers four of the 64 banks); X1 X2 itself where no such
// stride keeps the box within the LDS of a workgroup.
int box_plane_stride(const Plan &p) {
  const int base = p.X[1] * p.X[2];
  const size_t cb = p.prec == SGL_F64 ? 16 : 8;
  for (int s = base; s < base + 16; ++s) {
    // room for the point slots of a 1,024-thread workgroup (48 values each)
    if ((size_t)p.X[0] * s * cb + 64 * 48 * cb / 2 > (size_t)kLdsMax) break;
    unsigned m16 = 0;
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) m16 |= 1u << ((a * s + b * p.X[2]) & 15);
    if (m16 == 0xffffu) return s;
  }
  return base;
}

// Row stride of the slab gather's LDS slabs: the least S >= X2 with S = 2
// (mod 4), so that the values r S + h (r < 8, h < 2) read by the sixteen lanes
// of a point fall in sixteen distinct value slots modulo 16, if the slabs and
// the point slots of a workgroup then fit in LDS; X2 otherwise.
int slab_row_stride(const Plan &p) {
  const size_t cb = p.prec == SGL_F64 ? 16 : 8;
  const int s = p.X[2] + ((2 - p.X[2] % 4) + 4) % 4;
  const size_t slots = (size_t)(kSlabThreads / 16) * (3 * 2 * p.q + 32) * (cb / 2);
  return (size_t)kSlab * p.X[1] * s * cb + slots <= (size_t)kLdsMax ? s : p.X[2];
}

Geom make_geom(const Plan &p) {
  Geom g;
  g.q = p.q;
  g.S01 = box_plane_stride(p);
  g.SR = slab_row_stride(p);
  for (int j = 0; j < 3; ++j) {
    g.N[j] = p.N[j];
    g.E[j] = p.E[j];
    g.lo[j] = p.lo[j];
    g.pruned[j] = p.pruned[j] ? 1 : 0;
    g.L[j] = p.L[j];
    g.T[j] = p.T[j];
    g.X[j] = p.X[j];
    g.NB[j] = p.NB[j];
    g.Lo[j] = p.Lo[j];
    g.To[j] = p.To[j];
  }
  return g;
}

template <class R, int Q2>
hipError_t gather_q(const Plan &p, const void *grid, void *f) {
  const Geom g = make_geom(p);
  const R inv2lam = (R)(1.0 / (2.0 * p.lambda));
  if constexpr (std::is_same<R, float>::value && Q2 <= 16) {
    if (p.mfma) {
      // gfx950 grants up to 160 KB of LDS per workgroup without an opt-in
      k_gather_mfma<Q2><<<(unsigned)p.nchunks, GatherShape<Q2>::threads, GatherShape<Q2>::lds, p.stream>>>(
          (const cplx<float> *)grid, (const PointRec<float> *)p.pts, p.perm, p.chunks, g, (float)inv2lam,
          (cplx<float> *)f);
      return hipGetLastError();
    }
  }
  if (p.gather_mode == 0) {
    if (p.X[0] * p.X[1] * p.X[2] >= kGatherBoxMax) return hipErrorInvalidValue;
    const bool narrow = p.gather_narrow || GatherTiled<Q2>::threads == 256;
    const int nthreads = narrow ? 256 : GatherTiled<Q2>::threads;
    const size_t lds =
        (size_t)p.X[0] * g.S01 * sizeof(cplx<R>) + GatherTiled<Q2>::template slot_bytes<R>(nthreads);
    k_gather_tiled<R, Q2><<<(unsigned)p.nchunks, nthreads, lds, p.stream>>>(
        (const cplx<R> *)grid, (const PointRec<R> *)p.pts, p.perm, p.chunks, g, inv2lam, (cplx<R> *)f);
  } else {
    if (kSlab * p.X[1] * p.X[2] >= kGatherBoxMax) return hipErrorInvalidValue;
    const size_t lds = (size_t)kSlab * p.X[1] * g.SR * sizeof(cplx<R>) + GatherSlab<Q2>::template slot_bytes<R>();
    k_gather_slab<R, Q2><<<(unsigned)p.nchunks, kSlabThreads, lds, p.stream>>>(
        (const cplx<R> *)grid, (const PointRec<R> *)p.pts, p.perm, p.chunks, g, inv2lam, (cplx<R> *)f);
  }
  return hipGetLastError();
}

template <class R, int Q2>
hipError_t scatter_q(const Plan &p, const void *f, void *grid) {
  const Geom g = make_geom(p);
  const R inv2lam = (R)(1.0 / (2.0 * p.lambda));
  if constexpr (std::is_same<R, float>::value && Q2 <= 16) {
    if (p.mfma) {
      k_spread_mfma<Q2><<<(unsigned)p.nchunks, kSpreadThreads, 0, p.stream>>>(
          (const cplx<float> *)f, (const PointRec<float> *)p.pts, p.perm, p.chunks, g, (float)inv2lam,
          (cplx<float> *)p.staging);
      return hipGetLastError();
    }
  }
  if constexpr (std::is_same<R, double>::value && Q2 <= 12) {
    if (p.mfma64) {
      k_spread_mfma64<Q2><<<(unsigned)p.nchunks, kSpread64Threads, 0, p.stream>>>(
          (const cplx<double> *)f, (const PointRec<double> *)p.pts, p.perm, p.chunks, g, (double)inv2lam,
          (cplx<double> *)p.staging);
      return hipGetLastError();
    }
  }
  if (p.gather_mode == 0) {
    if constexpr (Q2 <= 16) {
      const unsigned threads = (unsigned)((p.X[0] * p.X[1] + 63) / 64 * 64);
      if (p.L[2] == 8)
        k_spread_rows<R, Q2, 8><<<(unsigned)p.nchunks, threads, 0, p.stream>>>(
            (const cplx<R> *)f, (const PointRec<R> *)p.pts, p.perm, p.chunks, g, inv2lam, (cplx<R> *)p.staging);
      else
        k_spread_rows<R, Q2, 4><<<(unsigned)p.nchunks, threads, 0, p.stream>>>(
            (const cplx<R> *)f, (const PointRec<R> *)p.pts, p.perm, p.chunks, g, inv2lam, (cplx<R> *)p.staging);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  k_scatter_owned<R, Q2><<<(unsigned)p.nown, kOwnThreads, 0, p.stream>>>(
      (const cplx<R> *)f, (const PointRec<R> *)p.pts, p.perm, p.tile_start, p.own_work, g, inv2lam,
      (cplx<R> *)grid, (cplx<R> *)p.own_stage);
  if (p.nown_fold > 0)
    k_fold_owned<R><<<(unsigned)p.nown_fold, kOwnThreads, 0, p.stream>>>((const cplx<R> *)p.own_stage, p.own_fold,
                                                                         g, (cplx<R> *)grid);
  return hipGetLastError();
}

// Fold for tiles of 8^3 cells when dimensions 0 and 1 are pruned and
// dimension 2 is the full period N2 = 8 T2 >= X: the box of tile c starts at
// stored index 8c in dimensions 0 and 1 and at 8c - q + 1 (mod N2) in
// dimension 2, so stored cell s lies in the boxes of the tiles
// floor(s'/8) - k, k = 0, 1, 2, at box index (s' mod 8) + 8k < X (s' = s, or
// s + q - 1 mod N2 in dimension 2).  One thread per stored cell sums those
// boxes (all chunks of each tile, in order) in double precision and writes the
// sum in the plan's precision; a wave covers 64 consecutive cells of one row,
// whose box entries are contiguous.
template <class R>
__global__ __launch_bounds__(256) void k_fold_tiles8(const cplx<R> *__restrict__ staging,
                                                     const int32_t *__restrict__ tile_chunk, Geom g,
                                                     cplx<R> *__restrict__ grid) {
  // a thread takes the two cells s' = 2u, 2u + 1 of one row: in every box they
  // lie in the same tile, so the chunk ranges are shared and their entries are
  // adjacent
  const int64_t pair = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int half = g.E[2] / 2;
  if (pair >= (int64_t)g.E[0] * g.E[1] * half) return;
  const int X = g.X[0];
  const size_t ncell = (size_t)X * X * X;
  const int sp2 = 2 * (int)(pair % half);  // even; sp2 + 1 is in the same block of 8
  const int r = (int)(pair / half);
  const int s1 = r % g.E[1], s0 = r / g.E[1];
  double ar0 = 0.0, ai0 = 0.0, ar1 = 0.0, ai1 = 0.0;
  for (int k0 = 0; k0 < 3; ++k0) {
    const int c0 = (s0 >> 3) - k0, i0 = (s0 & 7) + 8 * k0;
    if (c0 < 0 || c0 >= g.T[0] || i0 >= X) continue;
    for (int k1 = 0; k1 < 3; ++k1) {
      const int c1 = (s1 >> 3) - k1, i1 = (s1 & 7) + 8 * k1;
      if (c1 < 0 || c1 >= g.T[1] || i1 >= X) continue;
      // the chunk ranges of the three tiles along dimension 2 are looked up
      // before any box is read (every tile index is valid)
      int cr0[3], cr1[3];
#pragma unroll
      for (int k2 = 0; k2 < 3; ++k2) {
        int c2 = (sp2 >> 3) - k2;
        if (c2 < 0) c2 += g.T[2];
        const int tile = (c0 * g.T[1] + c1) * g.T[2] + c2;
        cr0[k2] = tile_chunk[tile];
        cr1[k2] = tile_chunk[tile + 1];
      }
#pragma unroll
      for (int k2 = 0; k2 < 3; ++k2) {
        const int i2 = (sp2 & 7) + 8 * k2;  // the second cell's is i2 + 1
        if (i2 >= X) continue;
        const bool second = i2 + 1 < X;
        const int ch0 = cr0[k2], ch1 = cr1[k2];
        const size_t off = ((size_t)i0 * X + i1) * X + i2;
        for (int ch = ch0; ch < ch1; ++ch) {
          const cplx<R> *b = staging + (size_t)ch * ncell + off;
          const cplx<R> v0 = b[0];
          ar0 += v0.re;
          ai0 += v0.im;
          if (second) {
            const cplx<R> v1 = b[1];
            ar1 += v1.re;
            ai1 += v1.im;
          }
        }
      }
    }
  }
  // stored cells s = s' - q + 1 (mod N2)
  int s2 = sp2 - (g.q - 1);
  if (s2 < 0) s2 += g.N[2];
  int s2b = s2 + 1;
  if (s2b >= g.N[2]) s2b -= g.N[2];
  const size_t row = ((size_t)s0 * g.E[1] + s1) * g.E[2];
  grid[row + s2] = cplx<R>{(R)ar0, (R)ai0};
  grid[row + s2b] = cplx<R>{(R)ar1, (R)ai1};
}

template <class R, int Q2>
hipError_t grad_q(const Plan &p, const void *grid, const void *xyz, const void *g, void *grad) {
  const Geom gg = make_geom(p);
  k_grad_points<R, Q2><<<(unsigned)((p.M + 255) / 256), 256, 0, p.stream>>>(
      (const cplx<R> *)grid, (const PointRec<R> *)p.pts, p.perm, p.M, gg, p.lambda, p.rho, (const R *)xyz,
      (const cplx<R> *)g, (R *)grad);
  return hipGetLastError();
}

template <class R>
hipError_t fold_r(const Plan &p, void *grid) {
  const Geom g = make_geom(p);
  if (p.L[0] == 8 && p.L[1] == 8 && p.L[2] == 8 && p.X[0] == p.X[1] && p.X[1] == p.X[2] && p.X[0] <= 24 &&
      p.pruned[0] && p.pruned[1] && !p.pruned[2] && p.N[2] == 8 * p.T[2] && p.E[2] == p.N[2] && p.X[2] <= p.N[2]) {
    const int64_t pairs = (int64_t)p.E[0] * p.E[1] * (p.E[2] / 2);
    k_fold_tiles8<R><<<(unsigned)((pairs + 255) / 256), 256, 0, p.stream>>>((const cplx<R> *)p.staging, p.tile_chunk,
                                                                           g, (cplx<R> *)grid);
    return hipGetLastError();
  }
  const int F0 = p.F[0], F1 = p.F[1], F2 = p.F[2];
  const int64_t nb = (int64_t)((p.E[0] + F0 - 1) / F0) * ((p.E[1] + F1 - 1) / F1) * ((p.E[2] + F2 - 1) / F2);
  k_fold_staging<R><<<(unsigned)nb, 256, 0, p.stream>>>((const cplx<R> *)p.staging, p.tile_chunk, g, F0, F1, F2,
                                                        (cplx<R> *)grid);
  return hipGetLastError();
}

#define SGL_Q_CASES(F, R, ...)                 \
  switch (p.q) {                               \
    case 1: return F<R, 2>(__VA_ARGS__);       \
    case 2: return F<R, 4>(__VA_ARGS__);       \
    case 3: return F<R, 6>(__VA_ARGS__);       \
    case 4: return F<R, 8>(__VA_ARGS__);       \
    case 5: return F<R, 10>(__VA_ARGS__);      \
    case 6: return F<R, 12>(__VA_ARGS__);      \
    case 7: return F<R, 14>(__VA_ARGS__);      \
    case 8: return F<R, 16>(__VA_ARGS__);      \
    case 9: return F<R, 18>(__VA_ARGS__);      \
    case 10: return F<R, 20>(__VA_ARGS__);     \
    case 11: return F<R, 22>(__VA_ARGS__);     \
    case 12: return F<R, 24>(__VA_ARGS__);     \
    case 13: return F<R, 26>(__VA_ARGS__);     \
    case 14: return F<R, 28>(__VA_ARGS__);     \
    case 15: return F<R, 30>(__VA_ARGS__);     \
    case 16: return F<R, 32>(__VA_ARGS__);     \
    default: return hipErrorInvalidValue;      \
  }

}  // namespace

void owned_work_list(const Plan &p, const std::vector<int32_t> &ts, std::vector<int32_t> &work,
                     std::vector<int32_t> &fold, int64_t &nslots) {
  const Geom g = make_geom(p);
  work.clear();
  fold.clear();
  nslots = 0;
  for (int64_t b = 0; b < p.nblocks; ++b) {
    const int C2 = (int)(b % p.To[2]), C1 = (int)((b / p.To[2]) % p.To[1]), C0 = (int)(b / ((int64_t)p.To[2] * p.To[1]));
    const int S[3] = {C0 * kOwn, C1 * kOwn, C2 * kOwn};
    int f[3][3], l[3][3], n[3];
    for (int j = 0; j < 3; ++j) n[j] = bin_ranges(S[j], std::min(kOwn, p.E[j] - S[j]), j, g, f[j], l[j]);
    // candidate points: the kernel's slot order (x0, x1, dimension-2 interval)
    int64_t tot = 0;
    for (int a = 0; a < n[0]; ++a)
      for (int x0 = f[0][a]; x0 <= l[0][a]; ++x0)
        for (int c = 0; c < n[1]; ++c)
          for (int x1 = f[1][c]; x1 <= l[1][c]; ++x1)
            for (int e = 0; e < n[2]; ++e) {
              const int64_t t0 = ((int64_t)x0 * p.T[1] + x1) * p.T[2];
              tot += ts[t0 + l[2][e] + 1] - ts[t0 + f[2][e]];
            }
    const int nseg = (int)std::max<int64_t>(1, (tot + kOwnSeg - 1) / kOwnSeg);
    if (nseg > 1) {
      fold.push_back((int32_t)b);
      fold.push_back((int32_t)nslots);
      fold.push_back(nseg);
    }
    for (int k = 0; k < nseg; ++k) {
      work.push_back((int32_t)b);
      work.push_back(k * kOwnSeg);
      work.push_back(k + 1 < nseg ? kOwnSeg : -1);  // the last segment runs to the end
      work.push_back(nseg > 1 ? (int32_t)(nslots + k) : -1);
    }
    if (nseg > 1) nslots += nseg;
  }
}

hipError_t launch_gather(const Plan &p, const void *grid, void *f) {
  if (p.prec == SGL_F64) {
    SGL_Q_CASES(gather_q, double, p, grid, f)
  } else {
    SGL_Q_CASES(gather_q, float, p, grid, f)
  }
}

hipError_t launch_scatter(const Plan &p, const void *f, void *grid) {
  if (p.prec == SGL_F64) {
    SGL_Q_CASES(scatter_q, double, p, f, grid)
  } else {
    SGL_Q_CASES(scatter_q, float, p, f, grid)
  }
}

hipError_t launch_grad_points(const Plan &p, const void *grid, const void *xyz, const void *g, void *grad) {
  if (p.prec == SGL_F64) {
    SGL_Q_CASES(grad_q, double, p, grid, xyz, g, grad)
  } else {
    SGL_Q_CASES(grad_q, float, p, grid, xyz, g, grad)
  }
}

hipError_t launch_fold(const Plan &p, void *grid) {
  return p.prec == SGL_F64 ? fold_r<double>(p, grid) : fold_r<float>(p, grid);
}

hipError_t launch_ndft_forward(const Plan &p, const void *eta, void *f) {
  const int nb = (int)((p.M + 255) / 256);
  if (p.prec == SGL_F64)
    k_ndft<double><<<nb, 256, 0, p.stream>>>((const cplx<double> *)eta, (const double *)p.ptsxyz, p.M, p.n[0],
                                             p.n[1], p.n[2], (cplx<double> *)f);
  else
    k_ndft<float><<<nb, 256, 0, p.stream>>>((const cplx<float> *)eta, (const double *)p.ptsxyz, p.M, p.n[0],
                                            p.n[1], p.n[2], (cplx<float> *)f);
  return hipGetLastError();
}

hipError_t launch_ndft_adjoint(const Plan &p, const void *f, void *eta) {
  const int64_t ne = (int64_t)p.n[0] * p.n[1] * p.n[2];
  const int nb = (int)((ne + 255) / 256);
  if (p.prec == SGL_F64)
    k_ndft_adj<double><<<nb, 256, 0, p.stream>>>((const cplx<double> *)f, (const double *)p.ptsxyz, p.M, p.n[0],
                                                 p.n[1], p.n[2], (cplx<double> *)eta);
  else
    k_ndft_adj<float><<<nb, 256, 0, p.stream>>>((const cplx<float> *)f, (const double *)p.ptsxyz, p.M, p.n[0],
                                                p.n[1], p.n[2], (cplx<float> *)eta);
  return hipGetLastError();
}

}  // namespace sgl
