// The four batched dense products of the conversion (Thm. 6.2, Cor. 6.3):
//   radial:         beta_m[l][a]  = sum_k K_l[a][k] fhat(l+1+k, l, m)
//   polar:          zeta_m[k1][a] = sum_l Kp_m[k1][l] beta_m[l][a]
//   polar adjoint:  beta_m[l][a]  = sum_k1 Kp_m[k1][l] zeta_m[k1][a]
//   radial adjoint: fhat(l+1+k, l, m) = sum_a K_l[a][k] beta_m[l][a]
// with Kp_{-m} = (-1)^m Kp_m, as 16 x 16 tiles on the matrix cores (one wave
// per tile, a host-built tile list per product), in two forms:
//  - FP64 (the default): v_mfma_f64_16x16x4f64 with each product's table
//    operand laid out row-major and zero padded at plan time; exact FP64
//    products and sums.
//  - split precision (SGL_FLAG_CONV_SPLIT16): v_mfma_f32_16x16x32_f16 with
//    FP16 hi + lo operands and FP32 accumulation.  The tables stay built in
//    long double: at plan time every row of the table operand is scaled by a
//    power of two that puts its largest entry into [2^13, 2^14) and split into
//    hi = fp16(s K), lo = fp16(s K - hi); the data operand is split the same
//    way per column inside the kernel.  hi*hi + hi*lo + lo*hi keeps about 22
//    significant bits of each product.  The conversion sums cancel strongly
//    when the radial functions grow towards rho, so this form is opt-in.
#include "sgl_internal.h"

namespace sgl {

namespace {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ inline int64_t mu_idx(int n, int l, int m) {
  return (int64_t)n * (n - 1) * (2 * n - 1) / 6 + (int64_t)l * (l + 1) + m;
}
__device__ inline int64_t beta_off(int B, int m) {
  int64_t c;
  if (m <= 0) c = (int64_t)(B + m - 1) * (B + m) / 2;
  else c = (int64_t)B * (B - 1) / 2 + (int64_t)m * B - (int64_t)m * (m - 1) / 2;
  return c * (2 * B - 1);
}
__device__ inline int64_t zeta_idx(int B, int m, int k1, int a) {
  return ((int64_t)(m + B - 1) * B + k1) * (2 * B - 1) + a;
}

// Data operand B[k][n] and output D[r][n] of each product.  Columns n pair the
// real (n even) and imaginary (n odd) parts of complex columns.
template <int MODE, class R>
struct Prod;

// radial, group l: rows a (2B-1), K = B - l, columns (m = -l..l) x (re, im)
template <class R>
struct Prod<0, R> {
  int B, l;
  __device__ Prod(int B_, int g) : B(B_), l(g) {}
  __device__ int M() const { return 2 * B - 1; }
  __device__ int K() const { return B - l; }
  __device__ int N() const { return 2 * (2 * l + 1); }
  __device__ double load(const void *in, int k, int n) const {
    const int m = n / 2 - l;
    return ((const R *)in)[2 * mu_idx(l + 1 + k, l, m) + (n & 1)];
  }
  __device__ void store(void *out, int r, int n, double v) const {
    const int m = n / 2 - l, am = m < 0 ? -m : m;
    ((double *)out)[2 * (beta_off(B, m) + (int64_t)(l - am) * (2 * B - 1) + r) + (n & 1)] = v;
  }
};

// polar, group m: rows k1 (B), K = B - |m| (c = l - |m|), columns (a) x (re, im)
template <class R>
struct Prod<1, R> {
  int B, m, am;
  __device__ Prod(int B_, int g) : B(B_), m(g - (B_ - 1)), am(m < 0 ? -m : m) {}
  __device__ int M() const { return B; }
  __device__ int K() const { return B - am; }
  __device__ int N() const { return 2 * (2 * B - 1); }
  __device__ double load(const void *in, int c, int n) const {
    return ((const double *)in)[2 * (beta_off(B, m) + (int64_t)c * (2 * B - 1) + n / 2) + (n & 1)];
  }
  __device__ void store(void *out, int r, int n, double v) const {
    if (m < 0 && (am & 1)) v = -v;
    ((double *)out)[2 * zeta_idx(B, m, r, n / 2) + (n & 1)] = v;
  }
};

// polar adjoint, group m: rows c = l - |m| (B - |m|), K = B (k1), columns (a) x (re, im)
template <class R>
struct Prod<2, R> {
  int B, m, am;
  __device__ Prod(int B_, int g) : B(B_), m(g - (B_ - 1)), am(m < 0 ? -m : m) {}
  __device__ int M() const { return B - am; }
  __device__ int K() const { return B; }
  __device__ int N() const { return 2 * (2 * B - 1); }
  __device__ double load(const void *in, int k1, int n) const {
    return ((const double *)in)[2 * zeta_idx(B, m, k1, n / 2) + (n & 1)];
  }
  __device__ void store(void *out, int r, int n, double v) const {
    if (m < 0 && (am & 1)) v = -v;
    ((double *)out)[2 * (beta_off(B, m) + (int64_t)r * (2 * B - 1) + n / 2) + (n & 1)] = v;
  }
};

// radial adjoint, group l: rows k (B - l), K = 2B - 1 (a), columns (m = -l..l) x (re, im)
template <class R>
struct Prod<3, R> {
  int B, l;
  __device__ Prod(int B_, int g) : B(B_), l(g) {}
  __device__ int M() const { return B - l; }
  __device__ int K() const { return 2 * B - 1; }
  __device__ int N() const { return 2 * (2 * l + 1); }
  __device__ double load(const void *in, int a, int n) const {
    const int m = n / 2 - l, am = m < 0 ? -m : m;
    return ((const double *)in)[2 * (beta_off(B, m) + (int64_t)(l - am) * (2 * B - 1) + a) + (n & 1)];
  }
  __device__ void store(void *out, int r, int n, double v) const {
    const int m = n / 2 - l;
    ((R *)out)[2 * mu_idx(l + 1 + r, l, m) + (n & 1)] = (R)v;
  }
};

// Tile list entry: product group g (l or m + B - 1), table group tg, 16-row
// block mt, 16-column block nt.
template <int MODE, class R>
__global__ __launch_bounds__(256) void k_conv_split(int B, const int32_t *__restrict__ tiles, int ntiles,
                                                    const ConvGroup *__restrict__ groups,
                                                    const _Float16 *__restrict__ planes,
                                                    const int32_t *__restrict__ rexp, const void *__restrict__ in,
                                                    void *__restrict__ out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tile = blockIdx.x * 4 + wave;
  if (tile >= ntiles) return;  // whole waves exit; no workgroup barrier follows
  const int g = tiles[4 * tile], tg = tiles[4 * tile + 1], mt = tiles[4 * tile + 2], nt = tiles[4 * tile + 3];
  const Prod<MODE, R> P(B, g);
  const ConvGroup G = groups[tg];
  const int K = P.K(), N = P.N(), M = P.M();
  const int pl = lane & 15, h = lane >> 4;
  const int n = nt * 16 + pl;
  const bool ncol = n < N;
  // column scale: largest |B[k][n]| over k (four lanes share a column)
  double cmax = 0.0;
  for (int k = 8 * h; k < G.Kpad; k += 32)
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (ncol && k + j < K) cmax = fmax(cmax, fabs(P.load(in, k + j, n)));
  cmax = fmax(cmax, __shfl_xor(cmax, 16));
  cmax = fmax(cmax, __shfl_xor(cmax, 32));
  int ec = 0;
  if (cmax > 0.0) frexp(cmax, &ec);
  ec = 14 - ec;  // column n scaled by 2^ec: largest entry in [2^13, 2^14)
  float4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
  const int row = mt * 16 + pl;
  const _Float16 *ahi = planes + G.plane_off + (int64_t)row * G.Kpad;
  const _Float16 *alo = ahi + (int64_t)G.Mpad * G.Kpad;
  for (int k0 = 0; k0 < G.Kpad; k0 += 32) {
    const half8_t a_h = *(const half8_t *)(ahi + k0 + 8 * h);
    const half8_t a_l = *(const half8_t *)(alo + k0 + 8 * h);
    half8_t b_h, b_l;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + 8 * h + j;
      const float v = (ncol && k < K) ? (float)ldexp(P.load(in, k, n), ec) : 0.0f;
      const _Float16 vh = (_Float16)v;
      b_h[j] = vh;
      b_l[j] = (_Float16)(v - (float)vh);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_h, b_h, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_h, b_l, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_l, b_h, acc, 0, 0, 0);
  }
  if (!ncol) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int r = mt * 16 + 4 * h + j;
    if (r < M) P.store(out, r, n, ldexp((double)acc[j], -(rexp[G.rexp_off + r] + ec)));
  }
}

// FP64 form: v_mfma_f64_16x16x4f64, lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] of each K = 4 step and holds D[l / 16 + 4 v][l % 16].
template <int MODE, class R>
__global__ __launch_bounds__(256) void k_conv_f64(int B, const int32_t *__restrict__ tiles, int ntiles,
                                                  const ConvGroup *__restrict__ groups,
                                                  const double *__restrict__ tab, const void *__restrict__ in,
                                                  void *__restrict__ out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tile = blockIdx.x * 4 + wave;
  if (tile >= ntiles) return;  // whole waves exit; no workgroup barrier follows
  const int g = tiles[4 * tile], tg = tiles[4 * tile + 1], mt = tiles[4 * tile + 2], nt = tiles[4 * tile + 3];
  const Prod<MODE, R> P(B, g);
  const ConvGroup G = groups[tg];
  const int K = P.K(), N = P.N(), M = P.M();
  const int c = lane & 15, kk = lane >> 4;  // column (and A row) within the tile, k within the step
  const int n = nt * 16 + c;
  const bool ncol = n < N;
  const double *arow = tab + G.plane_off + (int64_t)(mt * 16 + c) * G.Kpad;
  double4_t acc = {0.0, 0.0, 0.0, 0.0};
  // eight K steps per batch, their loads issued together (one memory latency
  // per batch instead of per step).  The table operand is zero padded to
  // Kpad, a multiple of 32, so every a is in range; b is zero past K, and the
  // padded steps add exact zeros to the same sums in the same order.
  for (int k0 = 0; k0 < K; k0 += 32) {
    double a[8], b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = k0 + 4 * u + kk;
      a[u] = arow[k];
      b[u] = (ncol && k < K) ? P.load(in, k, n) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
  }
  if (!ncol) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = mt * 16 + kk + 4 * v;
    if (r < M) P.store(out, r, n, acc[v]);
  }
}

}  // namespace

// ---------------------------------------------------------------- plan time

// Table operand of product `mode` for table group tg as a function (row, col)
// of the long-double tables; also its shape.
static void split_shape(int mode, int B, int tg, int *M, int *K) {
  const int A = 2 * B - 1;
  switch (mode) {
    case 0: *M = A; *K = B - tg; break;      // K_l[a][k], l = tg
    case 1: *M = B; *K = B - tg; break;      // Kp_m[k1][c], |m| = tg
    case 2: *M = B - tg; *K = B; break;      // Kp_m^T[c][k1]
    default: *M = B - tg; *K = A; break;     // K_l^T[k][a]
  }
}

static long double split_entry(int mode, int B, int tg, int r, int c, const std::vector<long double> &kr,
                               const std::vector<int64_t> &kro, const std::vector<long double> &kp,
                               const std::vector<int64_t> &kpo) {
  switch (mode) {
    case 0: return kr[kro[tg] + (int64_t)r * (B - tg) + c];
    case 1: return kp[kpo[tg] + (int64_t)r * (B - tg) + c];
    case 2: return kp[kpo[tg] + (int64_t)c * (B - tg) + r];
    default: return kr[kro[tg] + (int64_t)c * (B - tg) + r];
  }
}

sgl_status build_conv_tables(Plan &p, const std::vector<long double> &kr, const std::vector<long double> &kp) {
  const int B = p.B;
  const bool split = (p.flags & SGL_FLAG_CONV_SPLIT16) != 0;
  for (int mode = 0; mode < 4; ++mode) {
    ConvTab &T = p.conv[mode];
    std::vector<ConvGroup> groups(B);
    std::vector<_Float16> planes;
    std::vector<double> tab64;
    std::vector<int32_t> rexp;
    for (int tg = 0; tg < B; ++tg) {
      int M, K;
      split_shape(mode, B, tg, &M, &K);
      ConvGroup &G = groups[tg];
      G.Mpad = (M + 15) / 16 * 16;
      G.Kpad = (K + 31) / 32 * 32;
      G.rexp_off = (int32_t)rexp.size();
      if (!split) {
        // FP64 form: the table operand row-major [Mpad][Kpad], zero padded
        G.plane_off = (int64_t)tab64.size();
        const size_t base = tab64.size();
        tab64.resize(base + (size_t)G.Mpad * G.Kpad, 0.0);
        for (int r = 0; r < M; ++r)
          for (int c = 0; c < K; ++c)
            tab64[base + (size_t)r * G.Kpad + c] = (double)split_entry(mode, B, tg, r, c, kr, p.krad_off, kp, p.kpol_off);
        continue;
      }
      G.plane_off = (int64_t)planes.size();
      const size_t base = planes.size();
      planes.resize(base + 2 * (size_t)G.Mpad * G.Kpad, (_Float16)0.0f);
      for (int r = 0; r < G.Mpad; ++r) {
        long double mx = 0.0L;
        for (int c = 0; c < K && r < M; ++c)
          mx = std::max(mx, fabsl(split_entry(mode, B, tg, r, c, kr, p.krad_off, kp, p.kpol_off)));
        int e = 0;
        if (mx > 0.0L) frexpl(mx, &e);
        e = 14 - e;
        rexp.push_back(e);
        for (int c = 0; c < K && r < M; ++c) {
          const long double v = ldexpl(split_entry(mode, B, tg, r, c, kr, p.krad_off, kp, p.kpol_off), e);
          const _Float16 hi = (_Float16)(float)v;
          const _Float16 lo = (_Float16)(float)(v - (long double)(float)hi);
          planes[base + (size_t)r * G.Kpad + c] = hi;
          planes[base + (size_t)G.Mpad * G.Kpad + (size_t)r * G.Kpad + c] = lo;
        }
      }
    }
    // tiles: product groups (l, or m + B - 1) x row blocks x column blocks
    std::vector<int32_t> tiles;
    const int ngroups = (mode == 0 || mode == 3) ? B : 2 * B - 1;
    for (int g = 0; g < ngroups; ++g) {
      const int tg = (mode == 0 || mode == 3) ? g : std::abs(g - (B - 1));
      int M, K;
      split_shape(mode, B, tg, &M, &K);
      const int N = (mode == 0 || mode == 3) ? 2 * (2 * g + 1) : 2 * (2 * B - 1);
      for (int mt = 0; mt < (M + 15) / 16; ++mt)
        for (int nt = 0; nt < (N + 15) / 16; ++nt) {
          tiles.push_back(g);
          tiles.push_back(tg);
          tiles.push_back(mt);
          tiles.push_back(nt);
        }
    }
    T.ntiles = (int)(tiles.size() / 4);
    hipError_t e = hipMalloc(&T.groups, groups.size() * sizeof(ConvGroup));
    if (e == hipSuccess) e = hipMemcpy(T.groups, groups.data(), groups.size() * sizeof(ConvGroup), hipMemcpyHostToDevice);
    if (split) {
      if (e == hipSuccess) e = hipMalloc(&T.planes, planes.size() * sizeof(_Float16));
      if (e == hipSuccess) e = hipMemcpy(T.planes, planes.data(), planes.size() * sizeof(_Float16), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMalloc(&T.rexp, rexp.size() * sizeof(int32_t));
      if (e == hipSuccess) e = hipMemcpy(T.rexp, rexp.data(), rexp.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    } else {
      if (e == hipSuccess) e = hipMalloc(&T.planes, tab64.size() * sizeof(double));
      if (e == hipSuccess) e = hipMemcpy(T.planes, tab64.data(), tab64.size() * sizeof(double), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMalloc(&T.tiles, tiles.size() * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemcpy(T.tiles, tiles.data(), tiles.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? SGL_E_NOMEM : SGL_E_DEVICE;
  }
  return SGL_OK;
}

void free_conv_tables(Plan &p) {
  for (ConvTab &T : p.conv) {
    void *b[] = {T.groups, T.planes, T.rexp, T.tiles};
    for (void *x : b)
      if (x) hipFree(x);
    T = ConvTab{};
  }
}

template <int MODE, class R>
static hipError_t product_launch(const Plan &p, const void *in, void *out) {
  const ConvTab &T = p.conv[MODE];
  if (T.ntiles == 0) return hipSuccess;
  if (p.flags & SGL_FLAG_CONV_SPLIT16)
    k_conv_split<MODE, R><<<(unsigned)((T.ntiles + 3) / 4), 256, 0, p.stream>>>(
        p.B, (const int32_t *)T.tiles, T.ntiles, (const ConvGroup *)T.groups, (const _Float16 *)T.planes,
        (const int32_t *)T.rexp, in, out);
  else
    k_conv_f64<MODE, R><<<(unsigned)((T.ntiles + 3) / 4), 256, 0, p.stream>>>(
        p.B, (const int32_t *)T.tiles, T.ntiles, (const ConvGroup *)T.groups, (const double *)T.planes, in, out);
  return hipGetLastError();
}

// mode 0: fhat (plan precision) -> beta;  1: beta -> zeta;  2: zeta -> beta;
// 3: beta -> fhat (plan precision).
hipError_t launch_conv_product(const Plan &p, int mode, const void *in, void *out) {
  const bool f64 = p.prec == SGL_F64;
  switch (mode) {
    case 0: return f64 ? product_launch<0, double>(p, in, out) : product_launch<0, float>(p, in, out);
    case 1: return product_launch<1, double>(p, in, out);
    case 2: return product_launch<2, double>(p, in, out);
    default: return f64 ? product_launch<3, double>(p, in, out) : product_launch<3, float>(p, in, out);
  }
}

}  // namespace sgl
