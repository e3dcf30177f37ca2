// One pass of the 3D FFT of the NFFT (Section 2: alpha_l from beta_k by the
// inverse Fourier matrix, and its conjugate transpose in the adjoint): W
// lines of length L are staged in LDS, transformed by a Stockham autosort FFT
// with radices 8, 4, 2, 3, 5 (ping-pong between two LDS buffers, one barrier
// per stage), and written back.  Input rows fill only part of each line
// (zero padding of the small grid n into sigma n) and only the needed output
// rows are stored (pruning of the grid to the region the window touches).
// Pass A of the forward transform also applies the deconvolution
// 1 / prod_j phi_j(kappa_j) (Lemma 2.6) to its input, and pass A of the
// adjoint applies it to its output.
#include "sgl_internal.h"

namespace sgl {

namespace {

// y[a] = sum_b x[b] e^{sign 2 pi i a b / RAD}
template <class R>
__device__ inline cplx<R> mul_si(cplx<R> x, int sign) {  // x * (sign * i)
  return sign > 0 ? cplx<R>{-x.im, x.re} : cplx<R>{x.im, -x.re};
}

template <class R, int RAD>
struct Dft;

template <class R>
struct Dft<R, 2> {
  __device__ static void run(cplx<R> *v, int) {
    const cplx<R> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <class R>
struct Dft<R, 4> {
  __device__ static void run(cplx<R> *v, int s) {
    const cplx<R> a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    const cplx<R> c = cadd(v[1], v[3]), d = mul_si(csub(v[1], v[3]), s);
    v[0] = cadd(a, c);
    v[2] = csub(a, c);
    v[1] = cadd(b, d);
    v[3] = csub(b, d);
  }
};

template <class R>
struct Dft<R, 8> {
  __device__ static void run(cplx<R> *v, int s) {
    cplx<R> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<R> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<R, 4>::run(e, s);
    Dft<R, 4>::run(o, s);
    const R h = (R)0.70710678118654752440084436210484903928;
    // o[k] *= e^{s i pi k / 4}
    const cplx<R> o1 = {(o[1].re - s * o[1].im) * h, (o[1].im + s * o[1].re) * h};
    const cplx<R> o2 = mul_si(o[2], s);
    const cplx<R> o3 = {(-o[3].re - s * o[3].im) * h, (-o[3].im + s * o[3].re) * h};
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

template <class R>
struct Dft<R, 3> {
  __device__ static void run(cplx<R> *v, int s) {
    const R c = (R)0.86602540378443864676372317075293618347;  // sqrt(3)/2
    const cplx<R> t = cadd(v[1], v[2]);
    const cplx<R> u = cscale(mul_si(csub(v[1], v[2]), s), c);
    const cplx<R> m = {v[0].re - t.re / 2, v[0].im - t.im / 2};
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, u);
    v[2] = csub(m, u);
  }
};

template <class R>
struct Dft<R, 5> {
  __device__ static void run(cplx<R> *v, int s) {
    const R c1 = (R)0.30901699437494742410229341718281905886;   // cos(2 pi / 5)
    const R c2 = (R)-0.80901699437494742410229341718281905886;  // cos(4 pi / 5)
    const R s1 = (R)0.95105651629515357211643933337938214340;   // sin(2 pi / 5)
    const R s2 = (R)0.58778525229247312916870595463907276860;   // sin(4 pi / 5)
    const cplx<R> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const cplx<R> d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
    const cplx<R> x0 = v[0];
    const cplx<R> a1 = {x0.re + c1 * t1.re + c2 * t2.re, x0.im + c1 * t1.im + c2 * t2.im};
    const cplx<R> a2 = {x0.re + c2 * t1.re + c1 * t2.re, x0.im + c2 * t1.im + c1 * t2.im};
    const cplx<R> b1 = mul_si(cplx<R>{s1 * d1.re + s2 * d2.re, s1 * d1.im + s2 * d2.im}, s);
    const cplx<R> b2 = mul_si(cplx<R>{s2 * d1.re - s1 * d2.re, s2 * d1.im - s1 * d2.im}, s);
    v[0] = cadd(x0, cadd(t1, t2));
    v[1] = cadd(a1, b1);
    v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2);
    v[3] = csub(a2, b2);
  }
};

// One Stockham stage: Ns = product of the radices already applied.
template <class R, int RAD>
__device__ void stage(const cplx<R> *__restrict__ src, cplx<R> *__restrict__ dst, int L, int W, int Ns,
                      const cplx<R> *__restrict__ tw, int sign) {
  const int nb = (L / RAD) * W;
  const int twstride = L / (Ns * RAD);
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const int w = b % W, j = b / W, k = j % Ns;
    cplx<R> v[RAD];
#pragma unroll
    for (int r = 0; r < RAD; ++r) v[r] = src[(j + r * (L / RAD)) * W + w];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < RAD; ++r) {
        cplx<R> t = tw[r * k * twstride];
        if (sign < 0) t.im = -t.im;
        v[r] = cmul(v[r], t);
      }
    }
    Dft<R, RAD>::run(v, sign);
    const int idxD = (j / Ns) * Ns * RAD + k;
#pragma unroll
    for (int r = 0; r < RAD; ++r) dst[(idxD + r * Ns) * W + w] = v[r];
  }
}

__device__ inline int wrap(int i, int L) {
  i %= L;
  return i < 0 ? i + L : i;
}

// Deconvolution factor dc0[k0] dc1[k1] dc2[k2] of an element of the reduced
// grid [n0][n1][n2], split for a pass along `axis` ([outer][axis][inner] view
// of that grid) into the factor of the line (outer index o, inner index ic)
// and the factor of the element's index i along the axis.
__device__ inline double dc_line(const double *dc, int axis, int o, int ic, int n0, int n1, int n2) {
  if (axis == 2) return dc[o / n1] * dc[n0 + o % n1];
  if (axis == 1) return dc[o] * dc[n0 + n1 + ic];
  return dc[n0 + ic / n2] * dc[n0 + n1 + ic % n2];
}

__device__ inline double dc_elem(const double *dc, int axis, int i, int n0, int n1) {
  return dc[axis == 0 ? i : (axis == 1 ? n0 + i : n0 + n1 + i)];
}

// dcmode: 0 none; 1 multiply the input rows by the deconvolution factor (the
// first pass of the forward reads the reduced grid); 2 the same on the output
// rows (the last pass of the adjoint writes it).
// Ri: element type read, Ro: element type written; the transform itself runs
// in FP64 (the grid's values span many orders of magnitude towards r = rho and
// an FP32 transform leaves errors of the size of the largest ones everywhere).
template <class Ri, class Ro>
__global__ __launch_bounds__(512) void k_fft(const cplx<Ri> *__restrict__ in, cplx<Ro> *__restrict__ out, FftPass fp,
                                             const cplx<double> *__restrict__ tw64, const double *__restrict__ dc,
                                             int dcmode, int n0, int n1, int n2) {
  using R = double;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int L = fp.L, W = fp.W;
  cplx<R> *buf0 = (cplx<R> *)smem;
  cplx<R> *buf1 = buf0 + (size_t)L * W;
  cplx<R> *tw = buf1 + (size_t)L * W;  // twiddles e^{2 pi i t / L} in the transform's precision
  for (int t = threadIdx.x; t < L; t += blockDim.x) tw[t] = cplx<R>{(R)tw64[t].re, (R)tw64[t].im};

  // line w of this workgroup -> (outer index o, inner index ic)
  int o_base, ic_base;
  if (fp.inner > 1) {
    const int gpo = (fp.inner + W - 1) / W;
    o_base = blockIdx.x / gpo;
    ic_base = (blockIdx.x % gpo) * W;
  } else {
    o_base = blockIdx.x * W;
    ic_base = 0;
  }

  // zero the positions no input row lands on (the input's zero padding)
  for (int e = threadIdx.x; e < (L - fp.nin) * W; e += blockDim.x)
    buf0[wrap(fp.in_off + fp.nin + e / W, L) * W + e % W] = cplx<R>{0, 0};
  __syncthreads();

  for (int e = threadIdx.x; e < fp.nin * W; e += blockDim.x) {
    int i, w;
    if (fp.inner > 1) {
      i = e / W;
      w = e % W;
    } else {
      w = e / fp.nin;
      i = e % fp.nin;
    }
    const int o = fp.inner > 1 ? o_base : o_base + w;
    const int ic = fp.inner > 1 ? ic_base + w : 0;
    if (o >= fp.outer || ic >= fp.inner) continue;
    const cplx<Ri> vi = in[((size_t)o * fp.nin + i) * fp.inner + ic];
    cplx<R> v = {(R)vi.re, (R)vi.im};
    if (dcmode == 1) v = cscale(v, (R)(dc_line(dc, fp.axis, o, ic, n0, n1, n2) * dc_elem(dc, fp.axis, i, n0, n1)));
    buf0[wrap(fp.in_off + i, L) * W + w] = v;
  }
  __syncthreads();

  cplx<R> *src = buf0, *dst = buf1;
  int Ns = 1;
  for (int s = 0; s < fp.nstages; ++s) {
    const int rad = fp.radix[s];
    switch (rad) {
      case 8: stage<R, 8>(src, dst, L, W, Ns, tw, fp.sign); break;
      case 4: stage<R, 4>(src, dst, L, W, Ns, tw, fp.sign); break;
      case 2: stage<R, 2>(src, dst, L, W, Ns, tw, fp.sign); break;
      case 3: stage<R, 3>(src, dst, L, W, Ns, tw, fp.sign); break;
      default: stage<R, 5>(src, dst, L, W, Ns, tw, fp.sign); break;
    }
    __syncthreads();
    cplx<R> *t = src;
    src = dst;
    dst = t;
    Ns *= rad;
  }

  for (int e = threadIdx.x; e < fp.nout * W; e += blockDim.x) {
    int i, w;
    if (fp.inner > 1) {
      i = e / W;
      w = e % W;
    } else {
      w = e / fp.nout;
      i = e % fp.nout;
    }
    const int o = fp.inner > 1 ? o_base : o_base + w;
    const int ic = fp.inner > 1 ? ic_base + w : 0;
    if (o >= fp.outer || ic >= fp.inner) continue;
    cplx<R> v = src[wrap(fp.out_off + i, L) * W + w];
    if (dcmode == 2) v = cscale(v, (R)(dc_line(dc, fp.axis, o, ic, n0, n1, n2) * dc_elem(dc, fp.axis, i, n0, n1)));
    out[((size_t)o * fp.nout + i) * fp.inner + ic] = cplx<Ro>{(Ro)v.re, (Ro)v.im};
  }
}

// ---------------------------------------------------------------- power-of-two lengths

// LDS row stride (elements per position) for W lines: contiguous lines
// (inner == 1) are padded by one element so that the rows of one line land
// in different banks; strided lines are read and written row by row and need
// no padding.
template <int W, bool STRIDED>
constexpr int p2_stride() {
  return STRIDED ? W : W + 1;
}

// Lines per workgroup for length L = 2^LOG2L and element type R.  A strided
// pass reads every row of its lines as one segment of W adjacent values, so
// it takes 8 lines (a 128-byte segment of FP64 values) within 78 KB of line
// buffer and twiddles (two workgroups per compute unit).  A contiguous pass
// reads whole lines, so it takes as many as fit 39 KB, which leaves room for
// four workgroups per compute unit whose loads, transforms and stores
// overlap (measured on the B = 64 FP64 passes: the contiguous ones moved
// 2.7-3.2 TB/s with 16 lines and 4.3 TB/s with 4).
template <class R, int LOG2L, bool STRIDED>
constexpr int p2_lines() {
  int w = STRIDED ? 128 / (int)sizeof(cplx<R>) : 16;
  const size_t budget = (STRIDED ? 78 : 39) * 1024;
  while (w > 1 && ((size_t)(1 << LOG2L) * (STRIDED ? w : w + 1) + (1 << LOG2L)) * sizeof(cplx<R>) > budget)
    w /= 2;
  return w;
}

// Threads per workgroup.  A strided pass gets two threads per radix-8
// butterfly of a stage (256 to 1024): with at most two workgroups per compute
// unit its row-segment loads and stores need the extra waves in flight
// (measured on the B = 64 FP64 passes: L = 512 from 49-53 us at 256 threads to
// 38-41 at 1024, L = 256 from 36-40 at 256 to 33-35 at 512).  A contiguous
// pass keeps 256, which lets more of its small workgroups share a compute
// unit (512 threads measured 2-4% slower).
template <class R, int LOG2L, bool STRIDED>
constexpr int p2_threads() {
  constexpr int nb = ((1 << LOG2L) / 8) * p2_lines<R, LOG2L, STRIDED>();  // radix-8 butterflies per stage
  if constexpr (STRIDED) return 2 * nb > 1024 ? 1024 : (2 * nb < 256 ? 256 : 2 * nb);
  return nb >= 1024 ? 512 : 256;
}

// One in-place Stockham stage of radix RAD after NS points (NS = product of
// the radices already applied): every thread reads its butterflies' inputs
// into registers, the group synchronises, and the outputs are written back
// in autosort order.  LDS element (position, line) sits at position * SW + line.
template <class R, int NT, int L, int W, int SW, int RAD, int NS>
__device__ inline void p2_stage(cplx<R> *buf, const cplx<R> *tw, int sign) {
  constexpr int NB = (L / RAD) * W;
  constexpr int PER = (NB + NT - 1) / NT;
  cplx<R> v[PER][RAD];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int b = threadIdx.x + u * NT;
    if (NB % NT == 0 || b < NB) {
      const int w = b % W, j = b / W;
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[u][r] = buf[(j + r * (L / RAD)) * SW + w];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int b = threadIdx.x + u * NT;
    if (NB % NT == 0 || b < NB) {
      const int w = b % W, j = b / W, k = j % NS;
      if (NS > 1) {
#pragma unroll
        for (int r = 1; r < RAD; ++r) {
          cplx<R> t = tw[r * k * (L / (NS * RAD))];
          if (sign < 0) t.im = -t.im;
          v[u][r] = cmul(v[u][r], t);
        }
      }
      Dft<R, RAD>::run(v[u], sign);
      const int d = (j / NS) * NS * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) buf[(d + r * NS) * SW + w] = v[u][r];
    }
  }
  __syncthreads();
}

template <class R, int NT, int L, int W, int SW, int NS>
__device__ inline void p2_stages8(cplx<R> *buf, const cplx<R> *tw, int sign) {
  if constexpr (NS < L) {
    p2_stage<R, NT, L, W, SW, 8, NS>(buf, tw, sign);
    p2_stages8<R, NT, L, W, SW, NS * 8>(buf, tw, sign);
  }
}

// The pass of k_fft for L = 2^LOG2L with compile-time geometry; STRIDED
// selects the [outer][axis][inner > 1] view (lines are adjacent inner
// indices), otherwise every line is contiguous.
template <class Ri, class Ro, int LOG2L, bool STRIDED>
__global__ __launch_bounds__((p2_threads<double, LOG2L, STRIDED>())) void k_fft_p2(
    const cplx<Ri> *__restrict__ in, cplx<Ro> *__restrict__ out, FftPass fp, const cplx<double> *__restrict__ tw64,
    const double *__restrict__ dc, int dcmode, int n0, int n1, int n2) {
  using R = double;  // the transform runs in FP64 (see k_fft)
  constexpr int L = 1 << LOG2L;
  constexpr int W = p2_lines<R, LOG2L, STRIDED>();
  constexpr int SW = p2_stride<W, STRIDED>();
  constexpr int NT = p2_threads<R, LOG2L, STRIDED>();
  constexpr int REM = LOG2L % 3 == 0 ? 1 : (LOG2L % 3 == 1 ? 2 : 4);
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  cplx<R> *buf = (cplx<R> *)smem;
  cplx<R> *tw = buf + (size_t)L * SW;  // twiddles e^{2 pi i t / L} in the transform's precision
  __shared__ double linefac[W];        // deconvolution factor of the line (dimensions other than the axis)
  for (int t = threadIdx.x; t < L; t += NT) tw[t] = cplx<R>{(R)tw64[t].re, (R)tw64[t].im};

  int o_base, ic_base;
  if constexpr (STRIDED) {
    const int gpo = (fp.inner + W - 1) / W;
    o_base = blockIdx.x / gpo;
    ic_base = (blockIdx.x % gpo) * W;
  } else {
    o_base = blockIdx.x * W;
    ic_base = 0;
  }
  if (dcmode != 0 && threadIdx.x < W) {
    const int o = STRIDED ? o_base : o_base + (int)threadIdx.x;
    const int ic = STRIDED ? ic_base + (int)threadIdx.x : 0;
    linefac[threadIdx.x] = o < fp.outer && ic < fp.inner ? dc_line(dc, fp.axis, o, ic, n0, n1, n2) : 0.0;
  }
  // zero the positions no input row lands on (the input's zero padding)
  for (int e = threadIdx.x; e < (L - fp.nin) * SW; e += NT)
    buf[((fp.in_off + fp.nin + e / SW) & (L - 1)) * SW + e % SW] = cplx<R>{0, 0};
  __syncthreads();

  for (int e = threadIdx.x; e < fp.nin * W; e += NT) {
    int i, w;
    if constexpr (STRIDED) {
      i = e / W;
      w = e % W;
    } else {
      w = e / fp.nin;
      i = e - w * fp.nin;
    }
    const int o = STRIDED ? o_base : o_base + w;
    const int ic = STRIDED ? ic_base + w : 0;
    if (o >= fp.outer || ic >= fp.inner) continue;
    const cplx<Ri> vi = in[((size_t)o * fp.nin + i) * fp.inner + ic];
    cplx<R> v = {(R)vi.re, (R)vi.im};
    if (dcmode == 1) v = cscale(v, (R)(linefac[w] * dc_elem(dc, fp.axis, i, n0, n1)));
    buf[((fp.in_off + i) & (L - 1)) * SW + w] = v;
  }
  __syncthreads();

  if constexpr (REM > 1) p2_stage<R, NT, L, W, SW, REM, 1>(buf, tw, fp.sign);
  p2_stages8<R, NT, L, W, SW, REM>(buf, tw, fp.sign);

  for (int e = threadIdx.x; e < fp.nout * W; e += NT) {
    int i, w;
    if constexpr (STRIDED) {
      i = e / W;
      w = e % W;
    } else {
      w = e / fp.nout;
      i = e - w * fp.nout;
    }
    const int o = STRIDED ? o_base : o_base + w;
    const int ic = STRIDED ? ic_base + w : 0;
    if (o >= fp.outer || ic >= fp.inner) continue;
    cplx<R> v = buf[((fp.out_off + i) & (L - 1)) * SW + w];
    if (dcmode == 2) v = cscale(v, (R)(linefac[w] * dc_elem(dc, fp.axis, i, n0, n1)));
    out[((size_t)o * fp.nout + i) * fp.inner + ic] = cplx<Ro>{(Ro)v.re, (Ro)v.im};
  }
}

template <class Ri, class Ro, int LOG2L, bool STRIDED>
hipError_t fft_p2s(const Plan &p, const FftPass &fp, const void *in, void *out, int tw_index, int dcmode) {
  constexpr int W = p2_lines<double, LOG2L, STRIDED>();
  constexpr int SW = p2_stride<W, STRIDED>();
  constexpr int NT = p2_threads<double, LOG2L, STRIDED>();
  const int groups = STRIDED ? fp.outer * ((fp.inner + W - 1) / W) : (fp.outer + W - 1) / W;
  const size_t lds = ((size_t)(1 << LOG2L) * SW + (1 << LOG2L)) * sizeof(cplx<double>);
  k_fft_p2<Ri, Ro, LOG2L, STRIDED><<<groups, NT, lds, p.stream>>>(
      (const cplx<Ri> *)in, (cplx<Ro> *)out, fp, (const cplx<double> *)p.twiddle + p.tw_off[tw_index],
      (const double *)p.deconv, dcmode, p.n[0], p.n[1], p.n[2]);
  return hipGetLastError();
}

template <class Ri, class Ro, int LOG2L>
hipError_t fft_p2(const Plan &p, const FftPass &fp, const void *in, void *out, int tw_index, int dcmode) {
  if (fp.inner > 1) return fft_p2s<Ri, Ro, LOG2L, true>(p, fp, in, out, tw_index, dcmode);
  return fft_p2s<Ri, Ro, LOG2L, false>(p, fp, in, out, tw_index, dcmode);
}

template <class Ri, class Ro>
hipError_t fft_pow2(const Plan &p, const FftPass &fp, const void *in, void *out, int tw_index, int dcmode,
                    bool *done) {
  *done = true;
  switch (fp.L) {
    case 8: return fft_p2<Ri, Ro, 3>(p, fp, in, out, tw_index, dcmode);
    case 16: return fft_p2<Ri, Ro, 4>(p, fp, in, out, tw_index, dcmode);
    case 32: return fft_p2<Ri, Ro, 5>(p, fp, in, out, tw_index, dcmode);
    case 64: return fft_p2<Ri, Ro, 6>(p, fp, in, out, tw_index, dcmode);
    case 128: return fft_p2<Ri, Ro, 7>(p, fp, in, out, tw_index, dcmode);
    case 256: return fft_p2<Ri, Ro, 8>(p, fp, in, out, tw_index, dcmode);
    case 512: return fft_p2<Ri, Ro, 9>(p, fp, in, out, tw_index, dcmode);
    case 1024: return fft_p2<Ri, Ro, 10>(p, fp, in, out, tw_index, dcmode);
    case 2048: return fft_p2<Ri, Ro, 11>(p, fp, in, out, tw_index, dcmode);
    default: *done = false; return hipSuccess;
  }
}

}  // namespace

template <class Ri, class Ro>
hipError_t fft_typed(const Plan &p, const FftPass &fp, const void *in, void *out, int tw_index, int dcmode) {
  bool done = false;
  const hipError_t e = fft_pow2<Ri, Ro>(p, fp, in, out, tw_index, dcmode, &done);
  if (done) return e;
  const int groups = fp.inner > 1 ? fp.outer * ((fp.inner + fp.W - 1) / fp.W) : (fp.outer + fp.W - 1) / fp.W;
  const size_t lds = (2 * (size_t)fp.L * fp.W + fp.L) * sizeof(cplx<double>);
  // strided passes take 512 threads, as in k_fft_p2: more waves in flight for
  // their row-segment loads and stores
  k_fft<Ri, Ro><<<groups, fp.inner > 1 ? 512 : 256, lds, p.stream>>>((const cplx<Ri> *)in, (cplx<Ro> *)out, fp,
                                                (const cplx<double> *)p.twiddle + p.tw_off[tw_index],
                                                (const double *)p.deconv, dcmode, p.n[0], p.n[1], p.n[2]);
  return hipGetLastError();
}

// in_f64 / out_f64: element types read and written; the transform runs in FP64.
hipError_t launch_fft_pass(const Plan &p, const FftPass &fp, const void *in, void *out, int tw_index, int dcmode,
                           int in_f64, int out_f64) {
  if (in_f64 && out_f64) return fft_typed<double, double>(p, fp, in, out, tw_index, dcmode);
  if (!in_f64 && out_f64) return fft_typed<float, double>(p, fp, in, out, tw_index, dcmode);
  if (in_f64 && !out_f64) return fft_typed<double, float>(p, fp, in, out, tw_index, dcmode);
  return fft_typed<float, float>(p, fp, in, out, tw_index, dcmode);
}

}  // namespace sgl
