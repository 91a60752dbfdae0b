// HIP kernels (gfx950) of the FFT evaluation of cDFT excess chemical
// potentials.  Method: Sec. 2.3 (functional and its chemical potentials) and
// Sec. 3.4 (convolution integrals through FFTs) of Meng, Zheng, Lin, Sushko.
//
// Spectral storage of one real n^3 field (complex, precision T):
//   main  [x][y][kz]  kz in [0, n/2)      n * n * (n/2) elements
//   nyq   [x][y]      kz = n/2            n * n elements
// and the axes are transformed in the order z (real-to-complex, contiguous),
// y, x, so after the forward passes main[kx][ky][kz] holds the DFT at
// (kx, ky, kz) and nyq[kx][ky] the DFT at (kx, ky, n/2).
//
// One evaluation = 9 passes (all 1D FFTs are unnormalised; the 1/n^3 of the
// inverse transform is applied once, in the spectral multiplies):
//   P1 z r2c of S densities            k_zfwd
//   P2 y forward                       k_ystep<FWD>
//   P3 x forward, weights, x inverse   k_xfwd      (S -> 10 weighted densities)
//   P4 y inverse                       k_ystep<INV>
//   P5 z c2r, FMT derivatives, z r2c   k_zderiv    (10 -> 10, FP64 pointwise)
//   P6 y forward                       k_ystep<FWD>
//   P7 x forward, back-convolution, pair kernels, x inverse   k_xback (10 + S -> S)
//   P8 y inverse                       k_ystep<INV>
//   P9 z c2r, + constants, exp(-mu)    k_zinv
#include <hip/hip_runtime.h>
#include <math.h>

#include "fft_core.hpp"
#include "pnp_kernels.hpp"

namespace pnp {

// ---------------------------------------------------------------------------
// launch geometry per (precision, n)
// ---------------------------------------------------------------------------
constexpr int pow2_divisor_le(long v, int cap) {
  int r = 1;
  while (r * 2 <= cap && v % (r * 2) == 0) r *= 2;
  return r;
}

template <typename T, int N> struct Geo {
  static constexpr int H = N / 2;
  static constexpr bool R3 = (N % 3 == 0);
  // z passes: complex FFT of length H, EZ elements per thread
  static constexpr int EZ = R3 ? 12 : (H >= 16 ? 16 : H);
  static constexpr int TZ = H / EZ;
  static constexpr int RZ = pow2_divisor_le((long)N * N, 256 / TZ);  // rows per block (P1, P9)
  static constexpr int RD0 = (48 * 1024) / (kFields * N * (int)sizeof(T));
  static constexpr int RD = pow2_divisor_le((long)N * N, RD0 < 1 ? 1 : (RD0 > 256 / TZ ? 256 / TZ : RD0));
  // y passes
  static constexpr int EY = R3 ? 12 : (N >= 16 ? 16 : N);
  static constexpr int TY = N / EY;
  static constexpr int PY = pow2_divisor_le(N, sizeof(T) == 4 ? 16 : 8);
  // x passes
  static constexpr int EX = R3 ? 6 : (sizeof(T) == 4 ? (N >= 8 ? 8 : N) : (N >= 4 ? 4 : N));
  static constexpr int TX = N / EX;
  static constexpr int PX = pow2_divisor_le(N, sizeof(T) == 4 ? 16 : 8);
  // tiles per instance
  static constexpr int tiles_z = (N * N) / RZ;
  static constexpr int tiles_d = (N * N) / RD;
  static constexpr int tiles_y = (N * H) / PY + N / PY;
  static constexpr int tiles_x = (N * H) / PX + N / PX;
};

// twiddle table exp(-2 pi i j / L), computed in double
template <typename T, int L>
__device__ __forceinline__ void init_twiddles(cx<T>* tw) {
  for (int j = threadIdx.x; j < L; j += blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)j / (double)L, &s, &c);
    tw[j] = mk<T>((T)c, (T)(-s));
  }
}

// Pointers read from the device-resident argument tables are generic; this
// cast tells the compiler they address global memory so that it emits
// global_load / global_store instead of flat accesses.
template <typename X>
using gp = __attribute__((address_space(1))) X*;
template <typename X>
__device__ __forceinline__ gp<X> gbl(X* p) {
  return (gp<X>)p;
}

__device__ __forceinline__ int inst_of(int tiles, int& tile) {
  const int b = blockIdx.x;
  tile = b % tiles;
  return b / tiles;
}

__device__ __forceinline__ void raise_status(uint32_t* st, uint32_t bits, uint32_t idx) {
  atomicOr(st, bits);
  atomicMin(st + 1, idx);
}

// ---------------------------------------------------------------------------
// radial tables: the analytic transforms of Sec. 2.3.1 (weights), Sec. 2.3.2
// (square well) and Sec. 2.3.4 (MSA correlation) at |k| = (2 pi / L) sqrt(m)
// for every integer m = jx^2 + jy^2 + jz^2 that occurs on the grid.
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846;

// j1(x)/x = (sin x - x cos x) / x^3, series below 0.5
__device__ double d_j1x(double x) {
  if (fabs(x) < 0.5) {
    const double x2 = x * x;
    double p = 1.0, s = 0.0, f = 1.0;  // f = (2m+1)!
    for (int m = 0; m < 8; ++m) {
      if (m > 0) f *= (double)(2 * m) * (double)(2 * m + 1);
      s += ((m & 1) ? -p : p) / (f * (double)(2 * m + 3));
      p *= x2;
    }
    return s;
  }
  double sn, cs;
  sincos(x, &sn, &cs);
  return (sn - x * cs) / (x * x * x);
}

// transform of the unit ball of radius a
__device__ double d_ball(double k, double a) { return 4.0 * kPi * a * a * a * d_j1x(k * a); }

// transform of r * theta(a - r)
__device__ double d_rball(double k, double a) {
  const double y = k * a;
  double f;
  if (fabs(y) < 1.0) {
    const double y2 = y * y;
    double p = 1.0, s = 0.0, fa = 1.0;
    for (int m = 0; m < 10; ++m) {
      if (m > 0) fa *= (double)(2 * m) * (double)(2 * m + 1);
      s += ((m & 1) ? -p : p) / (fa * (double)(2 * m + 4));
      p *= y2;
    }
    f = s;
  } else {
    double sn, cs;
    sincos(y, &sn, &cs);
    f = (2.0 * y * sn + (2.0 - y * y) * cs - 2.0) / (y * y * y * y);
  }
  return 4.0 * kPi * a * a * a * a * f;
}

// transform of theta(a - r) / r
__device__ double d_invrball(double k, double a) {
  const double y = k * a;
  double f = 0.5;
  if (y != 0.0) {
    const double s = sin(0.5 * y);
    f = 2.0 * s * s / (y * y);
  }
  return 4.0 * kPi * a * a * f;
}

template <typename T>
__global__ void __launch_bounds__(256) k_tables(const TableArgs* __restrict__ targs, int blocks_per) {
  const int inst = blockIdx.x / blocks_per;
  const TableArgs& a = targs[inst];
  const int m = (blockIdx.x % blocks_per) * blockDim.x + threadIdx.x;
  if (m >= a.M) return;
  const double k = a.kscale * sqrt((double)m);
  auto hs = gbl((T*)a.hs_tab);
  auto rs = gbl((T*)a.rsq_tab);
  gp<T> pr = a.pair_tab ? gbl((T*)a.pair_tab) : (gp<T>)nullptr;
  rs[m] = (T)(m == 0 ? 0.0 : 1.0 / sqrt((double)m));
  for (int i = 0; i < a.S; ++i) {
    const double R = a.R[i];
    const double x = k * R;
    const double j1x = d_j1x(x);
    const double j0 = (x == 0.0) ? 1.0 : sin(x) / x;
    hs[(long)m * 3 * a.S + 3 * i + 0] = (T)j0;
    hs[(long)m * 3 * a.S + 3 * i + 1] = (T)(4.0 * kPi * R * R * R * j1x);
    hs[(long)m * 3 * a.S + 3 * i + 2] = (T)(4.0 * kPi * R * R * x * j1x);
  }
  if (pr) {
    for (int p = 0; p < a.np; ++p) {
      double g = 0.0;
      const double s = a.sigma[p];
      if (a.ec_pref[p] != 0.0) {
        const double b = a.Bsig[p];
        g += a.ec_pref[p] * (2.0 * b * d_ball(k, s) - b * b * d_rball(k, s) - d_invrball(k, s));
      }
      if (a.sw_pref[p] != 0.0) g += a.sw_pref[p] * (d_ball(k, a.rout[p]) - d_ball(k, s));
      pr[(long)m * a.np + p] = (T)g;
    }
  }
}

// ---------------------------------------------------------------------------
// z direction: real <-> half spectrum along the contiguous axis
// A row of n reals a[z] is packed as c[j] = a[2j] + i a[2j+1] (j < H), C =
// DFT_H(c), and X[k] = E[k] + W^k O[k] with E = (C[k] + conj C[H-k]) / 2,
// O = (C[k] - conj C[H-k]) / (2i), W = exp(-2 pi i / n).
// ---------------------------------------------------------------------------
template <typename T, int N, typename PO>
__device__ __forceinline__ void r2c_post(cx<T>* v, int t, const cx<T>* twN, cx<T>* row, PO main_out,
                                         PO nyq_out) {
  using G = Geo<T, N>;
  constexpr int H = G::H, TZ = G::TZ, EZ = G::EZ;
#pragma unroll
  for (int m = 0; m < EZ; ++m) row[t + TZ * m] = v[m];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < EZ; ++m) {
    const int k = t + TZ * m;
    const cx<T> c = v[m];
    const cx<T> cm = cconj<T>(row[k == 0 ? 0 : H - k]);
    const cx<T> e = mk<T>((T)0.5 * (c.x + cm.x), (T)0.5 * (c.y + cm.y));
    const cx<T> d = mk<T>((T)0.5 * (c.x - cm.x), (T)0.5 * (c.y - cm.y));  // O = d / i
    const cx<T> o = cmulmi<T>(d);
    const cx<T> x = cadd<T>(e, cmul<T>(twN[k], o));
    main_out[k] = x;
    if (k == 0) *nyq_out = mk<T>(c.x - c.y, (T)0);
  }
  __syncthreads();
}

// inverse: from X[k] (k < H) and X[H] build C[k] = (X[k] + conj X[H-k]) +
// i (X[k] - conj X[H-k]) W^-k (times 2: the result of the unnormalised
// length-H inverse is n (a[2j] + i a[2j+1]))
template <typename T, int N, typename PI>
__device__ __forceinline__ void c2r_pre(cx<T>* v, int t, const cx<T>* twN, PI main_in, PI nyq_in) {
  using G = Geo<T, N>;
  constexpr int H = G::H, TZ = G::TZ, EZ = G::EZ;
#pragma unroll
  for (int m = 0; m < EZ; ++m) {
    const int k = t + TZ * m;
    cx<T> xk = main_in[k];
    cx<T> xm = (k == 0) ? *nyq_in : main_in[H - k];
    if (k == 0) { xk.y = (T)0; xm.y = (T)0; }
    const cx<T> cm = cconj<T>(xm);
    const cx<T> s = cadd<T>(xk, cm);
    const cx<T> d = csub<T>(xk, cm);
    const cx<T> o = cmulc<T>(d, twN[k]);  // d * W^-k
    v[m] = cadd<T>(s, cmuli<T>(o));
  }
}

// P1: z r2c of the S input densities (float64) into specA
template <typename T, int N>
__global__ void __launch_bounds__((Geo<T, N>::RZ * Geo<T, N>::TZ))
    k_zfwd(const EvalArgs* __restrict__ args) {
  using G = Geo<T, N>;
  constexpr int H = G::H, TZ = G::TZ, EZ = G::EZ, RZ = G::RZ;
  __shared__ cx<T> twH[H];
  __shared__ cx<T> twN[N];
  __shared__ cx<T> xch[RZ * H];
  int tile;
  const EvalArgs& a = args[inst_of(G::tiles_z, tile)];
  init_twiddles<T, H>(twH);
  init_twiddles<T, N>(twN);
  if (tile == 0 && threadIdx.x == 0) {
    gp<uint32_t> st = gbl(a.status);
    st[0] = 0u;
    st[1] = 0xffffffffu;
  }
  __syncthreads();
  const int t = threadIdx.x % TZ, r = threadIdx.x / TZ;
  const long row = (long)tile * RZ + r;
  cx<T>* lrow = xch + r * H;
  const LdsPencil<T> lp{lrow, 1};
  auto A = gbl((cx<T>*)a.specA);
  for (int s = 0; s < a.S; ++s) {
    auto src = gbl(a.rho) + (long)s * N * N * N + row * N;
    cx<T> v[EZ];
#pragma unroll
    for (int m = 0; m < EZ; ++m) {
      const cf64 p = *(gp<const cf64>)(src + 2 * (t + TZ * m));
      v[m] = mk<T>((T)p.x, (T)p.y);
    }
    fft_pencil<T, H, EZ, true>(v, t, twH, lp);
    auto f = A + (long)s * a.fstride;
    r2c_post<T, N>(v, t, twN, lrow, f + row * H, f + (long)N * N * H + row);
  }
}

// P9 (final_mode = 1): z c2r of the S chemical-potential spectra in specC,
// + constants, write beta mu_ex and exp(-beta mu_ex) in float64.
// final_mode = 0: z c2r of `nreal` spectra of `sel` into out (no constant).
template <typename T, int N>
__global__ void __launch_bounds__((Geo<T, N>::RZ * Geo<T, N>::TZ))
    k_zinv(const EvalArgs* __restrict__ args, int sel) {
  using G = Geo<T, N>;
  constexpr int H = G::H, TZ = G::TZ, EZ = G::EZ, RZ = G::RZ;
  __shared__ cx<T> twH[H];
  __shared__ cx<T> twN[N];
  __shared__ cx<T> xch[RZ * H];
  int tile;
  const EvalArgs& a = args[inst_of(G::tiles_z, tile)];
  init_twiddles<T, H>(twH);
  init_twiddles<T, N>(twN);
  __syncthreads();
  const int t = threadIdx.x % TZ, r = threadIdx.x / TZ;
  const long row = (long)tile * RZ + r;
  const LdsPencil<T> lp{xch + r * H, 1};
  auto src = gbl((const cx<T>*)(sel == 0 ? a.specA : sel == 1 ? a.specB : a.specC));
  const long n3 = (long)N * N * N;
  uint32_t bad = 0u, badidx = 0xffffffffu;
  for (int s = 0; s < a.nreal; ++s) {
    auto f = src + (long)s * a.fstride;
    cx<T> v[EZ];
    c2r_pre<T, N>(v, t, twN, f + row * H, f + (long)N * N * H + row);
    fft_pencil<T, H, EZ, false>(v, t, twH, lp);
    auto o = gbl(a.out) + (long)s * n3 + row * N;
    if (a.final_mode) {
      const double c = a.cfin[s];
      gp<double> so = a.slot ? gbl(a.slot) + (long)s * n3 + row * N : (gp<double>)nullptr;
#pragma unroll
      for (int m = 0; m < EZ; ++m) {
        const int j = t + TZ * m;
        const double m0 = (double)v[m].x + c, m1 = (double)v[m].y + c;
        *(gp<cf64>)(o + 2 * j) = cf64{m0, m1};
        if (!(isfinite(m0) && isfinite(m1))) {
          bad |= kStNonFinite;
          badidx = min(badidx, (uint32_t)(s * n3 + row * N + 2 * j));
        }
        if (so) {
          // exp(-mu) overflows a double once -mu exceeds ln(DBL_MAX)
          if (-m0 > 709.782712893384 || -m1 > 709.782712893384) {
            bad |= kStOverflow;
            badidx = min(badidx, (uint32_t)(s * n3 + row * N + 2 * j));
          }
          *(gp<cf64>)(so + 2 * j) = cf64{exp(-m0), exp(-m1)};
        }
      }
    } else {
#pragma unroll
      for (int m = 0; m < EZ; ++m) {
        const int j = t + TZ * m;
        *(gp<cf64>)(o + 2 * j) = cf64{(double)v[m].x, (double)v[m].y};
      }
    }
  }
  if (bad) raise_status(a.status, bad, badidx);
}

// P5: z c2r of the 10 weighted densities, the FMT derivatives in float64
// (Sec. 2.3.1), z r2c of the 10 derivative fields; in place on specB.
// Every thread keeps its EZD elements of all ten fields in registers, so the
// ten values at a grid point meet in one thread without an LDS round trip.
template <typename T, int N> struct GeoD {
  static constexpr int H = N / 2;
  static constexpr int EZD = (H % 3 == 0) ? 6
                                          : (H >= (sizeof(T) == 4 ? 4 : 2) ? (sizeof(T) == 4 ? 4 : 2) : H);
  static constexpr int TZD = H / EZD;
  static constexpr int RDD = pow2_divisor_le((long)N * N, 256 / TZD < 1 ? 1 : 256 / TZD);
  static constexpr int tiles = (N * N) / RDD;
};

template <typename T, int N, int F>
__device__ __forceinline__ void zd_load(cx<T>* val, int t, const cx<T>* twN,
                                        const cx<T>* twH, const LdsPencil<T>& lp, gp<cx<T>> B, long fstride,
                                        long row) {
  if constexpr (F < kFields) {
    using D = GeoD<T, N>;
    constexpr int H = D::H;
    auto fb = B + (long)F * fstride;
#pragma unroll
    for (int m = 0; m < D::EZD; ++m) {
      const int k = t + D::TZD * m;
      cx<T> xk = fb[row * H + k];
      cx<T> xm = (k == 0) ? fb[(long)N * N * H + row] : fb[row * H + H - k];
      if (k == 0) { xk.y = (T)0; xm.y = (T)0; }
      const cx<T> cm = cconj<T>(xm);
      const cx<T> sm = cadd<T>(xk, cm);
      const cx<T> d = csub<T>(xk, cm);
      const cx<T> o = cmulc<T>(d, twN[k]);
      val[F * D::EZD + m] = cadd<T>(sm, cmuli<T>(o));
    }
    fft_pencil<T, H, D::EZD, false>(val + F * D::EZD, t, twH, lp);
    __builtin_amdgcn_sched_barrier(0);  // keep the next field's loads after this FFT
    zd_load<T, N, F + 1>(val, t, twN, twH, lp, B, fstride, row);
  }
}

template <typename T, int N, int F>
__device__ __forceinline__ void zd_store(cx<T>* val, int t, const cx<T>* twN,
                                         const cx<T>* twH, const LdsPencil<T>& lp, cx<T>* lrow, gp<cx<T>> B,
                                         long fstride, long row) {
  if constexpr (F < kFields) {
    using D = GeoD<T, N>;
    constexpr int H = D::H;
    auto fb = B + (long)F * fstride;
    fft_pencil<T, H, D::EZD, true>(val + F * D::EZD, t, twH, lp);
#pragma unroll
    for (int m = 0; m < D::EZD; ++m) lrow[t + D::TZD * m] = val[F * D::EZD + m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < D::EZD; ++m) {
      const int k = t + D::TZD * m;
      const cx<T> c = val[F * D::EZD + m];
      const cx<T> cm = cconj<T>(lrow[k == 0 ? 0 : H - k]);
      const cx<T> e = mk<T>((T)0.5 * (c.x + cm.x), (T)0.5 * (c.y + cm.y));
      const cx<T> d = mk<T>((T)0.5 * (c.x - cm.x), (T)0.5 * (c.y - cm.y));
      fb[row * H + k] = cadd<T>(e, cmul<T>(twN[k], cmulmi<T>(d)));
      if (k == 0) fb[(long)N * N * H + row] = mk<T>(c.x - c.y, (T)0);
    }
    __syncthreads();
    __builtin_amdgcn_sched_barrier(0);
    zd_store<T, N, F + 1>(val, t, twN, twH, lp, lrow, B, fstride, row);
  }
}

template <typename T, int N>
__global__ void __launch_bounds__((GeoD<T, N>::RDD * GeoD<T, N>::TZD))
    k_zderiv(const EvalArgs* __restrict__ args) {
  using D = GeoD<T, N>;
  constexpr int H = D::H, TZ = D::TZD, EZ = D::EZD, RD = D::RDD;
  __shared__ cx<T> twH[H];
  __shared__ cx<T> twN[N];
  __shared__ cx<T> xch[RD * H];
  int tile;
  const EvalArgs& a = args[inst_of(D::tiles, tile)];
  if (!a.hs_on) return;  // uniform per block
  init_twiddles<T, H>(twH);
  init_twiddles<T, N>(twN);
  __syncthreads();
  const int t = threadIdx.x % TZ, r = threadIdx.x / TZ;
  const long row = (long)tile * RD + r;
  cx<T>* lrow = xch + r * H;
  const LdsPencil<T> lp{lrow, 1};
  auto B = gbl((cx<T>*)a.specB);
  cx<T> val[kFields * EZ];
  zd_load<T, N, 0>(val, t, twN, twH, lp, B, a.fstride, row);
  uint32_t bad = 0u, badidx = 0xffffffffu;
  const double inv8pi = 1.0 / (8.0 * kPi), inv12pi = 1.0 / (12.0 * kPi), inv4pi = 1.0 / (4.0 * kPi);
#pragma unroll
  for (int m = 0; m < EZ; ++m) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // the two real points z = 2j, 2j+1 of element j
      double f[kFields];
#pragma unroll
      for (int q = 0; q < kFields; ++q) f[q] = h ? (double)val[q * EZ + m].y : (double)val[q * EZ + m].x;
      const double n0 = f[0], n1 = f[1], n2 = f[2], n3 = f[3];
      const double a1x = f[4], a1y = f[5], a1z = f[6], a2x = f[7], a2y = f[8], a2z = f[9];
      if (!(n3 < 1.0)) {
        bad |= isfinite(n3) ? kStPacking : kStNonFinite;
        badidx = min(badidx, (uint32_t)(row * N + 2 * (t + TZ * m) + h));
      }
      const double inv = 1.0 / (1.0 - n3), inv2 = inv * inv, inv3 = inv2 * inv;
      const double v12 = a1x * a2x + a1y * a2y + a1z * a2z;
      const double v22 = a2x * a2x + a2y * a2y + a2z * a2z;
      const double c2 = n2 * inv2 * inv4pi;
      double d[kFields];
      d[0] = -log1p(-n3);
      d[1] = n2 * inv;
      d[2] = n1 * inv + (n2 * n2 - v22) * inv2 * inv8pi;
      d[3] = n0 * inv + (n1 * n2 - v12) * inv2 + (n2 * n2 * n2 - 3.0 * n2 * v22) * inv3 * inv12pi;
      d[4] = -a2x * inv;
      d[5] = -a2y * inv;
      d[6] = -a2z * inv;
      d[7] = -a1x * inv - c2 * a2x;
      d[8] = -a1y * inv - c2 * a2y;
      d[9] = -a1z * inv - c2 * a2z;
#pragma unroll
      for (int q = 0; q < kFields; ++q) {
        if (h) val[q * EZ + m].y = (T)d[q];
        else val[q * EZ + m].x = (T)d[q];
      }
      __builtin_amdgcn_sched_barrier(0);  // one grid point at a time: bounded live range
    }
  }
  zd_store<T, N, 0>(val, t, twN, twH, lp, lrow, B, a.fstride, row);
  if (bad) raise_status(a.status, bad, badidx);
}

// ---------------------------------------------------------------------------
// y direction: c2c along y for every (x, kz) pencil of the main array and
// every x row of the Nyquist plane; in place on `nf` fields of `sel`.
// ---------------------------------------------------------------------------
template <typename T, int N, bool FWD>
__global__ void __launch_bounds__((Geo<T, N>::PY * Geo<T, N>::TY))
    k_ystep(const EvalArgs* __restrict__ args, int sel, int nf_code) {
  using G = Geo<T, N>;
  constexpr int H = G::H, TY = G::TY, EY = G::EY, PY = G::PY;
  __shared__ cx<T> tw[N];
  __shared__ cx<T> xch[PY * N];
  int tile;
  const EvalArgs& a = args[inst_of(G::tiles_y, tile)];
  if (sel == 1 && !a.hs_on) return;  // uniform per block
  init_twiddles<T, N>(tw);
  __syncthreads();
  auto base = gbl((cx<T>*)(sel == 0 ? a.specA : sel == 1 ? a.specB : a.specC));
  const int nf = nf_code == -1 ? a.S : nf_code;
  constexpr int tiles_main = (N * H) / PY;
  long off, es;
  int t;
  LdsPencil<T> lp;
  if (tile < tiles_main) {
    const int p = threadIdx.x % PY;
    t = threadIdx.x / PY;
    const long pen = (long)tile * PY + p;  // (x, kz)
    off = (pen / H) * ((long)N * H) + (pen % H);
    es = H;
    lp = LdsPencil<T>{xch + p, PY};
  } else {
    const int p = threadIdx.x / TY;
    t = threadIdx.x % TY;
    const long x = (long)(tile - tiles_main) * PY + p;
    off = (long)N * N * H + x * N;
    es = 1;
    lp = LdsPencil<T>{xch + p * N, 1};
  }
  for (int f = 0; f < nf; ++f) {
    auto fb = base + (long)f * a.fstride + off;
    cx<T> v[EY];
#pragma unroll
    for (int m = 0; m < EY; ++m) v[m] = fb[(long)(t + TY * m) * es];
    fft_pencil<T, N, EY, FWD>(v, t, tw, lp);
#pragma unroll
    for (int m = 0; m < EY; ++m) fb[(long)(t + TY * m) * es] = v[m];
  }
}

// ---------------------------------------------------------------------------
// x direction helpers: pencil (ky, kz) of the main array or ky of the Nyquist
// plane, element kx at stride es.
// ---------------------------------------------------------------------------
template <typename T, int N>
struct XPencil {
  long off, es;
  int ky, kz;
  __device__ __forceinline__ XPencil(int tile, int p) {
    constexpr int H = N / 2;
    constexpr int PX = Geo<T, N>::PX;
    const long pen = (long)tile * PX + p;
    const long nmain = (long)N * H;
    if (pen < nmain) {
      off = pen; es = nmain; ky = (int)(pen / H); kz = (int)(pen % H);
    } else {
      const long q = pen - nmain;
      off = nmain * N + q; es = N; ky = (int)q; kz = H;
    }
  }
};

__device__ __forceinline__ int sgn_idx(int j, int n) { return j < n / 2 ? j : j - n; }

// P3: forward weights.  For every k: n^_a(k) = sum_i rho^_i(k) conj(w^_i^a(k))
// (correlation, Sec. 2.3.1); scalars w0 = j0, w1 = R j0, w2 = 4 pi R^2 j0,
// w3 = 4 pi R^3 j1(kR)/(kR); vectors conj(-i khat V) = +i khat V with
// V2 = 4 pi R^2 j1(kR), V1 = V2 / (4 pi R).
template <typename T, int N>
__global__ void __launch_bounds__((Geo<T, N>::PX * Geo<T, N>::TX))
    k_xfwd(const EvalArgs* __restrict__ args) {
  using G = Geo<T, N>;
  constexpr int H = G::H, TX = G::TX, EX = G::EX, PX = G::PX;
  __shared__ cx<T> tw[N];
  __shared__ cx<T> xch[PX * N];
  int tile;
  const EvalArgs& a = args[inst_of(G::tiles_x, tile)];
  if (!a.hs_on) return;  // uniform per block
  init_twiddles<T, N>(tw);
  __syncthreads();
  const int p = threadIdx.x % PX, t = threadIdx.x / PX;
  const XPencil<T, N> pc(tile, p);
  const LdsPencil<T> lp{xch + p, PX};
  const int S = a.S;
  const int sy = sgn_idx(pc.ky, N), sz = pc.kz;
  auto hs = gbl((const T*)a.hs_tab);
  auto rsq = gbl((const T*)a.rsq_tab);
  int mm[EX];
#pragma unroll
  for (int m = 0; m < EX; ++m) {
    const int sx = sgn_idx(t + TX * m, N);
    mm[m] = sx * sx + sy * sy + sz * sz;
  }
  cx<T> acc[6][EX];
#pragma unroll
  for (int q = 0; q < 6; ++q)
#pragma unroll
    for (int m = 0; m < EX; ++m) acc[q][m] = mk<T>((T)0, (T)0);
  auto A = gbl((const cx<T>*)a.specA);
  for (int i = 0; i < S; ++i) {
    auto src = A + (long)i * a.fstride + pc.off;
    cx<T> v[EX];
#pragma unroll
    for (int m = 0; m < EX; ++m) v[m] = src[(long)(t + TX * m) * pc.es];
    fft_pencil<T, N, EX, true>(v, t, tw, lp);
    const T R = (T)a.R[i], ar = (T)a.area[i], i4 = (T)a.inv4piR[i];
#pragma unroll
    for (int m = 0; m < EX; ++m) {
      auto w = hs + (long)mm[m] * 3 * S + 3 * i;
      const T j0 = w[0], s3 = w[1], vv = w[2];
      cfma<T>(acc[0][m], v[m], j0);
      cfma<T>(acc[1][m], v[m], j0 * R);
      cfma<T>(acc[2][m], v[m], j0 * ar);
      cfma<T>(acc[3][m], v[m], s3);
      cfma<T>(acc[4][m], v[m], vv * i4);
      cfma<T>(acc[5][m], v[m], vv);
    }
  }
  const T sc = (T)a.inv_n3;
  auto B = gbl((cx<T>*)a.specB);
  // scalar weighted densities n0..n3
#pragma unroll 1
  for (int o = 0; o < 4; ++o) {
    cx<T> v[EX];
#pragma unroll
    for (int m = 0; m < EX; ++m) {
      cx<T> s0;
      switch (o) {  // o is uniform: a scalar branch, no indexed registers
        case 0: s0 = acc[0][m]; break;
        case 1: s0 = acc[1][m]; break;
        case 2: s0 = acc[2][m]; break;
        default: s0 = acc[3][m]; break;
      }
      v[m] = cscale<T>(s0, sc);
    }
    fft_pencil<T, N, EX, false>(v, t, tw, lp);
    auto dst = B + (long)o * a.fstride + pc.off;
#pragma unroll
    for (int m = 0; m < EX; ++m) dst[(long)(t + TX * m) * pc.es] = v[m];
  }
  // vector weighted densities: n1v_c = +i khat_c V1, n2v_c = +i khat_c V2
#pragma unroll
  for (int b = 0; b < 2; ++b) {
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
      cx<T> v[EX];
#pragma unroll
      for (int m = 0; m < EX; ++m) {
        const int kx = t + TX * m;
        int s;
        if (c == 0) s = (kx == H) ? 0 : sgn_idx(kx, N);
        else if (c == 1) s = (pc.ky == H) ? 0 : sy;
        else s = (pc.kz == H) ? 0 : sz;
        const T u = (T)s * rsq[mm[m]] * sc;
        v[m] = cscale<T>(cmuli<T>(acc[4 + b][m]), u);
      }
      fft_pencil<T, N, EX, false>(v, t, tw, lp);
      auto dst = B + (long)(4 + 3 * b + c) * a.fstride + pc.off;
#pragma unroll
      for (int m = 0; m < EX; ++m) dst[(long)(t + TX * m) * pc.es] = v[m];
    }
  }
}

// P7: back-convolution (Sec. 2.3.1, convolution orientation: no conjugate)
// plus the pair kernels of Sec. 2.3.2 / 2.3.4:
//   mu^_i = j0_i (F0 + R_i F1 + 4 pi R_i^2 F2) + w3_i F3
//           - i V2_i (D1 / (4 pi R_i) + D2) + sum_j G_ij rho^_j,
// with F_a the derivative spectra and D_b = khat . (vector derivative b).
template <typename T, int N, int CH>
__global__ void __launch_bounds__((Geo<T, N>::PX * Geo<T, N>::TX))
    k_xback(const EvalArgs* __restrict__ args) {
  using G = Geo<T, N>;
  constexpr int H = G::H, TX = G::TX, EX = G::EX, PX = G::PX;
  __shared__ cx<T> tw[N];
  __shared__ cx<T> xch[PX * N];
  int tile;
  const EvalArgs& a = args[inst_of(G::tiles_x, tile)];
  init_twiddles<T, N>(tw);
  __syncthreads();
  const int p = threadIdx.x % PX, t = threadIdx.x / PX;
  const XPencil<T, N> pc(tile, p);
  const LdsPencil<T> lp{xch + p, PX};
  const int S = a.S;
  const int sy = sgn_idx(pc.ky, N), sz = pc.kz;
  auto hs = gbl((const T*)a.hs_tab);
  auto rsq = gbl((const T*)a.rsq_tab);
  auto pt = gbl((const T*)a.pair_tab);
  int mm[EX];
#pragma unroll
  for (int m = 0; m < EX; ++m) {
    const int sx = sgn_idx(t + TX * m, N);
    mm[m] = sx * sx + sy * sy + sz * sz;
  }
  cx<T> F[6][EX];
#pragma unroll
  for (int q = 0; q < 6; ++q)
#pragma unroll
    for (int m = 0; m < EX; ++m) F[q][m] = mk<T>((T)0, (T)0);
  auto B = gbl((const cx<T>*)a.specB);
  if (a.hs_on) {
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      auto src = B + (long)f * a.fstride + pc.off;
      cx<T> v[EX];
#pragma unroll
      for (int m = 0; m < EX; ++m) v[m] = src[(long)(t + TX * m) * pc.es];
      fft_pencil<T, N, EX, true>(v, t, tw, lp);
#pragma unroll
      for (int m = 0; m < EX; ++m) {
        switch (f) {  // uniform scalar branch
          case 0: F[0][m] = v[m]; break;
          case 1: F[1][m] = v[m]; break;
          case 2: F[2][m] = v[m]; break;
          default: F[3][m] = v[m]; break;
        }
      }
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll 1
      for (int c = 0; c < 3; ++c) {
        auto src = B + (long)(4 + 3 * b + c) * a.fstride + pc.off;
        cx<T> v[EX];
#pragma unroll
        for (int m = 0; m < EX; ++m) v[m] = src[(long)(t + TX * m) * pc.es];
        fft_pencil<T, N, EX, true>(v, t, tw, lp);
#pragma unroll
        for (int m = 0; m < EX; ++m) {
          const int kx = t + TX * m;
          int s;
          if (c == 0) s = (kx == H) ? 0 : sgn_idx(kx, N);
          else if (c == 1) s = (pc.ky == H) ? 0 : sy;
          else s = (pc.kz == H) ? 0 : sz;
          cfma<T>(F[4 + b][m], v[m], (T)s * rsq[mm[m]]);
        }
      }
    }
  }
  auto A = gbl((const cx<T>*)a.specA);
  auto C = gbl((cx<T>*)a.specC);
  const T sc = (T)a.inv_n3;
#pragma unroll 1
  for (int i0 = 0; i0 < S; i0 += CH) {
    cx<T> out[CH][EX];
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
      for (int m = 0; m < EX; ++m) out[c][m] = mk<T>((T)0, (T)0);
    if (a.pair_on) {
#pragma unroll 1
      for (int j = 0; j < S; ++j) {
        auto src = A + (long)j * a.fstride + pc.off;
        cx<T> v[EX];
#pragma unroll
        for (int m = 0; m < EX; ++m) v[m] = src[(long)(t + TX * m) * pc.es];
        fft_pencil<T, N, EX, true>(v, t, tw, lp);
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int i = i0 + c;
          if (i < S) {
            const int pi = a.pidx[i][j];
#pragma unroll
            for (int m = 0; m < EX; ++m) cfma<T>(out[c][m], v[m], pt[(long)mm[m] * a.np + pi]);
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int i = i0 + c;
      if (i < S) {  // uniform across the block
        cx<T> v[EX];
        const T R = (T)a.R[i], ar = (T)a.area[i], i4 = (T)a.inv4piR[i];
#pragma unroll
        for (int m = 0; m < EX; ++m) {
          cx<T> u = out[c][m];
          if (a.hs_on) {
            auto w = hs + (long)mm[m] * 3 * S + 3 * i;
            const T j0 = w[0], s3 = w[1], vv = w[2];
            cx<T> sc0 = F[0][m];
            cfma<T>(sc0, F[1][m], R);
            cfma<T>(sc0, F[2][m], ar);
            cfma<T>(u, sc0, j0);
            cfma<T>(u, F[3][m], s3);
            cx<T> dv = F[5][m];
            cfma<T>(dv, F[4][m], i4);
            cfma<T>(u, cmulmi<T>(dv), vv);
          }
          v[m] = cscale<T>(u, sc);
        }
        fft_pencil<T, N, EX, false>(v, t, tw, lp);
        auto dst = C + (long)i * a.fstride + pc.off;
#pragma unroll
        for (int m = 0; m < EX; ++m) dst[(long)(t + TX * m) * pc.es] = v[m];
      }
    }
  }
}

// plain x-direction c2c on `nf` fields of `sel` (used by the FFT test hook)
template <typename T, int N, bool FWD>
__global__ void __launch_bounds__((Geo<T, N>::PX * Geo<T, N>::TX))
    k_xplain(const EvalArgs* __restrict__ args, int sel, int nf) {
  using G = Geo<T, N>;
  constexpr int TX = G::TX, EX = G::EX, PX = G::PX;
  __shared__ cx<T> tw[N];
  __shared__ cx<T> xch[PX * N];
  int tile;
  const EvalArgs& a = args[inst_of(G::tiles_x, tile)];
  init_twiddles<T, N>(tw);
  __syncthreads();
  const int p = threadIdx.x % PX, t = threadIdx.x / PX;
  const XPencil<T, N> pc(tile, p);
  const LdsPencil<T> lp{xch + p, PX};
  auto base = gbl((cx<T>*)(sel == 0 ? a.specA : sel == 1 ? a.specB : a.specC));
  for (int f = 0; f < nf; ++f) {
    auto fb = base + (long)f * a.fstride + pc.off;
    cx<T> v[EX];
#pragma unroll
    for (int m = 0; m < EX; ++m) v[m] = fb[(long)(t + TX * m) * pc.es];
    fft_pencil<T, N, EX, FWD>(v, t, tw, lp);
#pragma unroll
    for (int m = 0; m < EX; ++m) fb[(long)(t + TX * m) * pc.es] = v[m];
  }
}

// numpy rfftn layout <-> spectral storage (test hook only)
template <typename T, int N>
__global__ void k_export(const EvalArgs* __restrict__ args, int nf, double* buf, int to_numpy) {
  constexpr int H = N / 2;
  const EvalArgs& a = args[0];
  const long total = (long)nf * N * N * (H + 1);
  auto A = gbl((cx<T>*)a.specA);
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long f = e / ((long)N * N * (H + 1));
    const long rem = e % ((long)N * N * (H + 1));
    const long kx = rem / ((long)N * (H + 1));
    const long ky = (rem / (H + 1)) % N;
    const long kz = rem % (H + 1);
    auto s = A + f * a.fstride + (kz < H ? (kx * N + ky) * H + kz : (long)N * N * H + kx * N + ky);
    if (to_numpy) {
      buf[2 * e] = (double)s->x;
      buf[2 * e + 1] = (double)s->y;
    } else {
      *s = mk<T>((T)buf[2 * e], (T)buf[2 * e + 1]);
    }
  }
}

// relaxation of the consumer stub: rho <- (1 - l) rho + l rho_b exp(mu_b - mu)
__global__ void k_relax(double* rho, const double* mu, long n3, int S, const double* rho_b_mu_b,
                        double lambda) {
  const long total = (long)S * n3;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int s = (int)(e / n3);
    const double rb = rho_b_mu_b[2 * s], mb = rho_b_mu_b[2 * s + 1];
    rho[e] = (1.0 - lambda) * rho[e] + lambda * rb * exp(mb - mu[e]);
  }
}

// per-term mode: slot = exp(-(hs + el + sh))
__global__ void k_sum_exp(const double* mu3, double* slot, long sn3, uint32_t* status) {
  uint32_t bad = 0u, badidx = 0xffffffffu;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < sn3; e += (long)gridDim.x * blockDim.x) {
    const double m = mu3[e] + mu3[sn3 + e] + mu3[2 * sn3 + e];
    if (!isfinite(m)) { bad |= kStNonFinite; badidx = min(badidx, (uint32_t)e); }
    if (-m > 709.782712893384) { bad |= kStOverflow; badidx = min(badidx, (uint32_t)e); }
    if (slot) slot[e] = exp(-m);
  }
  if (bad) raise_status(status, bad, badidx);
}

}  // namespace pnp
