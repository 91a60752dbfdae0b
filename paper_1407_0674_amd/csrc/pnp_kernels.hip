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
//   P3 x forward, weights, x inverse   k_xfwd      (S -> 8 stored fields)
//   P4 y inverse                       k_ystep<INV> (8 -> 10: vector y components)
//   P5 z c2r, FMT derivatives, z r2c   k_zderiv    (10 -> 10, FP64 pointwise)
//   P6 y forward                       k_ystep<FWD> (10 -> 8: khat . F partial sums)
//   P7 x forward, back-convolution, pair kernels, x inverse   k_xback (8 + S -> S)
// (the vector densities carry one component per axis pass; see the
// field-slot layout in pnp_kernels.hpp)
//   P8 y inverse                       k_ystep<INV>
//   P9 z c2r, + constants, exp(-mu)    k_zinv
//
// Addressing: every global access is a uniform (scalar) field base plus a
// per-lane 32-bit byte offset that is computed once per block, which maps to
// the saddr + voffset form of global_load / global_store.
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

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

// V selects the launch variant of a pass.  Bit 0, the tile shape: clear,
// the default (wide rows for full HBM bursts); set, narrow (a quarter of the
// rows or pencils per workgroup: four times the workgroups, for grids too
// small to fill the chip).  The shape only changes how many pencils a
// workgroup carries; every pencil's arithmetic is the same.  Bit 1, the FFT
// schedule: clear, the primary elements per thread of each pass family;
// set, the secondary one (half as many elements per thread, twice the
// threads per pencil, and a radix plan with smaller radices).  The schedule
// changes the order of the floating-point operations, so results of the two
// schedules agree to rounding, not bit for bit.
constexpr int narrow(int v, int V) { return (V & 1) == 0 ? v : (v / 4 > 1 ? v / 4 : 1); }

// whether a length-len pencil with ept elements per thread has a radix plan
// (every stage a radix dividing both what is left of len and ept)
constexpr bool plan_ok(int len, int ept) {
  if (ept < 2 || len % ept != 0) return false;
  for (int ns = 1; ns < len;) {
    const int r = pick_radix(len / ns, ept);
    if (r <= 1) return false;
    ns *= r;
  }
  return true;
}

// the secondary schedule of a pass family: half the primary elements per
// thread where that has a radix plan and stays within 1024 threads per
// workgroup (`per` pencils per workgroup in the wide tile shape, the larger
// one, so both shapes get the same schedule); else, where `dbl` allows it,
// twice the primary elements per thread (fewer, larger radix stages: on
// lengths with a factor 3 six elements per thread leave only radix-2 stages
// after the first); else the primary one
constexpr int alt_ept(int len, int prim, int per, bool dbl = false) {
  return (plan_ok(len, prim / 2) && per * (len / (prim / 2)) <= 1024) ? prim / 2
         : (dbl && plan_ok(len, 2 * prim))                            ? 2 * prim
                                                                       : prim;
}

template <typename T, int N, int V = 0> struct Geo {
  static constexpr int H = N / 2;
  static constexpr bool R3 = (N % 3 == 0);
  static constexpr bool SEC = (V & 2) != 0;
  // z passes (P1, P9): complex FFT of length H, EZ elements per thread
  static constexpr int EZ0 = R3 ? 12 : (H >= 16 ? 16 : H);
  static constexpr int EZ = SEC ? alt_ept(H, EZ0, 1) : EZ0;  // RZ * TZ <= 256 for any EZ
  static constexpr int TZ = H / EZ;
  static constexpr int RZ = narrow(pow2_divisor_le((long)N * N, 256 / TZ), V);  // rows per block
  // y passes
  static constexpr int PY = narrow(pow2_divisor_le(N, sizeof(T) == 4 ? 16 : 8), V);
  static constexpr int EY0 = R3 ? 12 : (N >= 16 ? 16 : N);
  static constexpr int EY = SEC ? alt_ept(N, EY0, pow2_divisor_le(N, sizeof(T) == 4 ? 16 : 8)) : EY0;
  static constexpr int TY = N / EY;
  // x passes
  static constexpr int PX = narrow(pow2_divisor_le(N, sizeof(T) == 4 ? 16 : 8), V);
  static constexpr int EX0 = R3 ? 6 : (sizeof(T) == 4 ? (N >= 8 ? 8 : N) : (N >= 4 ? 4 : N));
  static constexpr int EX = SEC ? alt_ept(N, EX0, pow2_divisor_le(N, sizeof(T) == 4 ? 16 : 8), true) : EX0;
  static constexpr int TX = N / EX;
  // tiles per instance
  static constexpr int tiles_z = (N * N) / RZ;
  static constexpr int tiles_y = (N * H) / PY + N / PY;
  static constexpr int tiles_x = (N * H) / PX + N / PX;
};

// signed wavenumber index of position j on an axis of n points
__device__ __forceinline__ int sgn_idx(int j, int n) { return j < n / 2 ? j : j - n; }

// twiddle table exp(-2 pi i j / L), computed in double
template <typename T, int L>
__device__ __forceinline__ void init_twiddles(cx<T>* tw) {
  for (int j = threadIdx.x; j < L; j += blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)j / (double)L, &s, &c);
    tw[j] = mk<T>((T)c, (T)(-s));
  }
}

// Global-memory pointers (used for the status word and the test hook).
template <typename X>
using gp = __attribute__((address_space(1))) X*;
template <typename X>
__device__ __forceinline__ gp<X> gbl(X* p) {
  return (gp<X>)p;
}

// Buffer-resource access: a scalar descriptor for one array, a per-lane
// 32-bit byte offset and a uniform 32-bit byte offset (the field).  The
// descriptor's record count is the array size, so an access past the end
// reads 0 / is dropped instead of touching other memory.
constexpr int kBufWord3 = 0x00020000;  // raw (untyped) 32-bit data on gfx9-family parts
// Cache policy of the streaming accesses of grids from 192^3 on:
// non-temporal.  Every field a pass writes is read again only by a later
// pass, after far more data than the L2 caches and the 256 MB Infinity Cache
// hold has gone by, so its lines are not worth keeping (measured: 5 % less
// time per evaluation at 256^3).  Smaller grids keep the default policy
// (measured: non-temporal stores made the batch of 32^3-128^3 instances 8 %
// slower).  Loads keep the default policy except where measured faster: the
// density input of the first pass, the derivative pass, and the field loads
// of the back pass (there the pair-table rows then stay cached for the
// gathers: 428 -> 389 us at 256^3).  Gathers of the small tables always keep
// the default policy.
constexpr int kPolicyNT = 2;
template <int N> constexpr int stream_policy() { return N >= 192 ? kPolicyNT : 0; }
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// SP: cache policy of stores and streaming loads (0 or kPolicyNT)
template <int SP>
struct BufT {
  __amdgpu_buffer_rsrc_t r;
  template <typename X>
  __device__ __forceinline__ X ld(uint32_t voff, uint32_t soff = 0) const {
    return ld_pol<X, 0>(voff, soff);
  }
  // streaming load (policy SP)
  template <typename X>
  __device__ __forceinline__ X ldnt(uint32_t voff, uint32_t soff = 0) const {
    return ld_pol<X, SP>(voff, soff);
  }
  template <typename X, int POL>
  __device__ __forceinline__ X ld_pol(uint32_t voff, uint32_t soff) const {
    if constexpr (sizeof(X) == 4) {
      return __builtin_bit_cast(X, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, POL));
    } else if constexpr (sizeof(X) == 8) {
      return __builtin_bit_cast(X, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, POL));
    } else if constexpr (sizeof(X) == 16) {
      return __builtin_bit_cast(X, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, POL));
    } else {
      static_assert(sizeof(X) == 32, "buffer access size");
      const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, POL);
      const u32x4 b = __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16, soff, POL);
      struct P { u32x4 a, b; } pr{a, b};
      return __builtin_bit_cast(X, pr);
    }
  }
  // Stores take the whole offset in the lane offset and a zero scalar
  // offset: a store wider than 64 bits reads its data registers one
  // instruction after issue, and the compiler inserts the wait that protects
  // them from an immediate overwrite only for this form of the instruction
  // (with a register scalar offset it emits none, and the low half of the
  // stored data can be replaced by the next value written to those
  // registers).  Narrow stores follow the same rule because the compiler may
  // merge adjacent ones into a wide store.
  template <typename X>
  __device__ __forceinline__ void st(X v, uint32_t voff, uint32_t soff = 0) const {
    if constexpr (sizeof(X) == 4) {
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff + soff, 0, SP);
    } else if constexpr (sizeof(X) == 8) {
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff + soff, 0, SP);
    } else if constexpr (sizeof(X) == 16) {
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff + soff, 0, SP);
    } else {
      static_assert(sizeof(X) == 32, "buffer access size");
      struct P { u32x4 a, b; };
      const P pr = __builtin_bit_cast(P, v);
      __builtin_amdgcn_raw_buffer_store_b128(pr.a, r, voff + soff, 0, SP);
      __builtin_amdgcn_raw_buffer_store_b128(pr.b, r, voff + soff + 16, 0, SP);
    }
  }
};

using Buf = BufT<0>;
template <int N> using BufN = BufT<stream_policy<N>()>;

template <int SP = 0>
__device__ __forceinline__ BufT<SP> make_buf(const void* p, uint64_t bytes) {
  const uint32_t n = bytes >= 0xffffffffull ? 0xffffffffu : (uint32_t)bytes;
  return BufT<SP>{__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)n, kBufWord3)};
}

__device__ __forceinline__ int inst_of(int tiles, int& tile) {
  const int b = blockIdx.x;
  tile = b % tiles;
  return b / tiles;
}

// Launch parts of the y and x passes: the tiles of the main array
// (kz < n/2) and those of the Nyquist plane (kz = n/2) are independent
// between two z passes, so they may run as separate launches.
enum : int { kPartAll = 0, kPartMain = 1, kPartNyquist = 2 };

// instance and tile of this block for a launch of `part` over instances with
// `main` main-array tiles and `nyq` Nyquist-plane tiles each
__device__ __forceinline__ int inst_of_part(int main, int nyq, int part, int& tile) {
  const int per = part == kPartAll ? main + nyq : part == kPartMain ? main : nyq;
  const int b = blockIdx.x;
  tile = b % per + (part == kPartNyquist ? main : 0);
  return b / per;
}

// Sum of one double per thread over the workgroup, in a fixed order (the
// result is the same on every run); valid in thread 0.  red: LDS scratch of
// one double per wavefront.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x / 64, nw = (blockDim.x + 63) / 64;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < nw; ++k) t += red[k];
  return t;
}

__device__ __forceinline__ void raise_status(uint32_t* st, uint32_t bits, uint32_t idx) {
  atomicOr(st, bits);
  atomicMin(st + 1, idx);
}

template <typename T> struct vec4;
template <> struct vec4<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct vec4<double> { typedef double type __attribute__((ext_vector_type(4))); };
template <typename T> using v4 = typename vec4<T>::type;

// ---------------------------------------------------------------------------
// radial tables: the analytic transforms of Sec. 2.3.1 (weights), Sec. 2.3.2
// (square well) and Sec. 2.3.4 (MSA correlation) at |k| = (2 pi / L) sqrt(m)
// for every integer m = jx^2 + jy^2 + jz^2 that occurs on the grid.
// ---------------------------------------------------------------------------
constexpr double kPi = 3.14159265358979323846;

// Radial profiles of the step-like kernels at y = k a, from one sin/cos pair
// of y (the caller evaluates it only where the closed forms are used):
//   j1x(y) = j1(y) / y = (sin y - y cos y) / y^3        (series below 0.5)
//   rb(y)  = (2 y sin y + (2 - y^2) cos y - 2) / y^4    (series below 1)
//   irb(y) = (1 - cos y) / y^2                          (series below 1)
// with the ball transform 4 pi a^3 j1x, the transform of r theta(a - r)
// 4 pi a^4 rb and that of theta(a - r) / r 4 pi a^2 irb.  The series are the
// Taylor expansions of the same expressions (the closed forms cancel as
// y -> 0), summed to below 1e-17 relative on their ranges.
__device__ inline double d_j1x(double y, double sn, double cs) {
  if (fabs(y) < 0.5) {
    const double y2 = y * y;
    double p = 1.0, s = 0.0, f = 1.0;  // f = (2m+1)!
    for (int m = 0; m < 8; ++m) {
      if (m > 0) f *= (double)(2 * m) * (double)(2 * m + 1);
      s += ((m & 1) ? -p : p) / (f * (double)(2 * m + 3));
      p *= y2;
    }
    return s;
  }
  return (sn - y * cs) / (y * y * y);
}

__device__ inline double d_rb(double y, double sn, double cs) {
  if (fabs(y) < 1.0) {
    const double y2 = y * y;
    double p = 1.0, s = 0.0, fa = 1.0;
    for (int m = 0; m < 10; ++m) {
      if (m > 0) fa *= (double)(2 * m) * (double)(2 * m + 1);
      s += ((m & 1) ? -p : p) / (fa * (double)(2 * m + 4));
      p *= y2;
    }
    return s;
  }
  return (2.0 * y * sn + (2.0 - y * y) * cs - 2.0) / (y * y * y * y);
}

__device__ inline double d_irb(double y, double cs) {
  if (fabs(y) < 1.0) {
    // (1 - cos y) / y^2 = sum_m (-1)^m y^(2m) / (2m + 2)!
    const double y2 = y * y;
    double p = 1.0, s = 0.0, fa = 2.0;  // fa = (2m+2)!
    for (int m = 0; m < 10; ++m) {
      if (m > 0) fa *= (double)(2 * m + 1) * (double)(2 * m + 2);
      s += ((m & 1) ? -p : p) / fa;
      p *= y2;
    }
    return s;
  }
  return (1.0 - cs) / (y * y);
}

// j1(x)/x from x alone
__device__ inline double d_j1x(double x) {
  double sn = 0.0, cs = 1.0;
  if (fabs(x) >= 0.5) sincos(x, &sn, &cs);
  return d_j1x(x, sn, cs);
}

// hs table [m][S][4] = (j0(kR), 4 pi R^3 j1(kR)/(kR), 4 pi R^2 j1(kR), 0)
// (FP64 path only); pair table [m][j][i] (row length Sp) = G_ij, the combined
// pair kernel, zero for i >= S.  One thread per (m, table entry): blockIdx.y
// picks the entry (pair-table entries first, then the hs species), blockIdx.z
// the instance.  G is symmetric, so the thread of entry (j, i) with i <= j
// writes both (j, i) and (i, j), and those with i > j have nothing to do.
template <typename T>
__global__ void __launch_bounds__(256) k_tables(const TableArgs* __restrict__ targs) {
  const TableArgs& a = targs[blockIdx.z];
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= a.M) return;
  const int item = blockIdx.y;
  const int npair = a.S * a.Sp;
  const double k = a.kscale * sqrt((double)m);
  if (item < npair) {
    if (!a.pair_tab) return;
    const int j = item / a.Sp, i = item % a.Sp;
    const Buf pr = make_buf(a.pair_tab, (uint64_t)a.M * a.S * a.Sp * sizeof(T));
    if (i >= a.S) {
      pr.template st<T>((T)0, (uint32_t)(((m * a.S + j) * a.Sp + i) * sizeof(T)));
      return;
    }
    if (i > j) return;  // written by the thread of (i, j)
    const int p = a.pidx[i][j];
    const double s = a.sigma[p];
    const double y = k * s;
    double sn = 0.0, cs = 1.0;
    if (fabs(y) >= 0.5) sincos(y, &sn, &cs);
    const double ball = 4.0 * kPi * s * s * s * d_j1x(y, sn, cs);
    double v = 0.0;
    if (a.ec_pref[p] != 0.0) {
      // MSA correlation (Sec. 2.3.4): 2 B ball - B^2 (r-ball) - (1/r-ball)
      const double b = a.Bsig[p];
      const double rball = 4.0 * kPi * s * s * s * s * d_rb(y, sn, cs);
      const double irball = 4.0 * kPi * s * s * d_irb(y, cs);
      v += a.ec_pref[p] * (2.0 * b * ball - b * b * rball - irball);
    }
    if (a.sw_pref[p] != 0.0) {
      // square well (Sec. 2.3.2): the shell between sigma and r_out
      const double ro = a.rout[p];
      v += a.sw_pref[p] * (4.0 * kPi * ro * ro * ro * d_j1x(k * ro) - ball);
    }
    pr.template st<T>((T)v, (uint32_t)(((m * a.S + j) * a.Sp + i) * sizeof(T)));
    if (i != j) pr.template st<T>((T)v, (uint32_t)(((m * a.S + i) * a.Sp + j) * sizeof(T)));
  } else if (sizeof(T) == 8 && item < npair + a.S) {  // the FP32 path evaluates these in registers
    const int i = item - npair;
    const double R = a.R[i];
    const double x = k * R;
    double sn, cs;
    sincos(x, &sn, &cs);
    const double j1x = d_j1x(x, sn, cs);
    const double j0 = (x == 0.0) ? 1.0 : sn / x;
    v4<T> w;
    w.x = (T)j0;
    w.y = (T)(4.0 * kPi * R * R * R * j1x);
    w.z = (T)(4.0 * kPi * R * R * x * j1x);
    w.w = (T)0;
    const Buf hs = make_buf(a.hs_tab, (uint64_t)a.M * a.S * 4 * sizeof(T));
    hs.template st<v4<T>>(w, (uint32_t)((m * a.S + i) * sizeof(v4<T>)));
  }
}

// ---------------------------------------------------------------------------
// z direction: real <-> half spectrum along the contiguous axis
// A row of n reals a[z] is packed as c[j] = a[2j] + i a[2j+1] (j < H), C =
// DFT_H(c), and X[k] = E[k] + W^k O[k] with E = (C[k] + conj C[H-k]) / 2,
// O = (C[k] - conj C[H-k]) / (2i), W = exp(-2 pi i / n).
// Spectral element e of a field sits at byte e * sizeof(cx<T>) + soff.
// ---------------------------------------------------------------------------
// A z-pass row is owned by TZ consecutive lanes; when TZ divides the
// wavefront every row lies inside one wavefront and its exchanges are
// wave-local.
template <int TZ> constexpr bool row_in_wave() { return TZ <= 64 && 64 % TZ == 0; }

// first element of row row_id = kx * N + ky of a spectral field's main block,
// and of the Nyquist plane
template <typename T, int N>
__device__ __forceinline__ uint32_t spec_row(uint32_t row_id) {
  return row_id * (uint32_t)(N / 2) + (row_id / (uint32_t)N) * (uint32_t)spec_pad(N, sizeof(T));
}
template <typename T, int N> constexpr uint32_t spec_nyq() { return (uint32_t)(N * spec_plane(N, sizeof(T))); }

// v holds C[k] at k = t + TZ m; writes X[k] (k < H) and X[H] of one row.
// zmul: store i s_z X instead (s_z = k below the Nyquist index, 0 at it).
template <typename T, int N, int TZ, int EZ, typename BF>
__device__ __forceinline__ void r2c_post(cx<T>* v, int t, const cx<T>* twN, cx<T>* row, const BF& f,
                                         uint32_t soff, uint32_t row_id, bool zmul = false) {
  constexpr int H = N / 2;
  constexpr uint32_t cs = sizeof(cx<T>);
#pragma unroll
  for (int m = 0; m < EZ; ++m) row[t + TZ * m] = v[m];
  lds_sync<row_in_wave<TZ>()>();
#pragma unroll
  for (int m = 0; m < EZ; ++m) {
    const int k = t + TZ * m;
    const cx<T> c = v[m];
    const cx<T> cm = cconj<T>(row[k == 0 ? 0 : H - k]);
    const cx<T> e = mk<T>((T)0.5 * (c.x + cm.x), (T)0.5 * (c.y + cm.y));
    const cx<T> d = mk<T>((T)0.5 * (c.x - cm.x), (T)0.5 * (c.y - cm.y));  // O = d / i
    cx<T> x = cadd<T>(e, cmul<T>(twN[k], cmulmi<T>(d)));
    if (zmul) x = cscale<T>(cmuli<T>(x), (T)k);
    f.template st<cx<T>>(x, (spec_row<T, N>(row_id) + k) * cs, soff);
    if (k == 0) f.template st<cx<T>>(zmul ? mk<T>((T)0, (T)0) : mk<T>(c.x - c.y, (T)0),
                            (spec_nyq<T, N>() + row_id) * cs, soff);
  }
  lds_sync<row_in_wave<TZ>()>();
}

// raw loads for the c2r pre-step of one row: X[k] and X[H-k] (X[H] from the
// Nyquist plane for k = 0) at the lane's elements k = t + TZ m (streaming
// loads: the buffer's policy)
template <typename T, int N, int TZ, int EZ, typename BF>
__device__ __forceinline__ void c2r_load(cx<T>* xk, cx<T>* xm, int t, const BF& f, uint32_t soff,
                                         uint32_t row_id) {
  constexpr int H = N / 2;
  constexpr uint32_t cs = sizeof(cx<T>);
  const uint32_t r0 = spec_row<T, N>(row_id);
#pragma unroll
  for (int m = 0; m < EZ; ++m) {
    const int k = t + TZ * m;
    xk[m] = f.template ldnt<cx<T>>((r0 + k) * cs, soff);
    xm[m] = f.template ldnt<cx<T>>((k == 0 ? spec_nyq<T, N>() + row_id : r0 + (H - k)) * cs, soff);
  }
}

// Where the mirror values X[H - k] of the c2r steps come from: on grids that
// stream their fields (192^3 on) from the row's LDS buffer after one load of
// the row (c2r_load_k, c2r_mirror; at 256^3: z_deriv 341 -> 318 us, FP64
// 192^3 z_inv 96 -> 83 us); on smaller grids, whose fields stay in the
// caches, from a second load of the row (c2r_load), which costs less there
// than the LDS round trip (128^3 z_deriv 43 against 45 us).
template <int N> constexpr bool mirror_lds() { return stream_policy<N>() != 0; }

// raw loads for the c2r pre-step with the mirror values taken from LDS: X[k]
// at the lane's elements and, in every lane, X[H] of the row (its Nyquist
// plane value); streaming loads (the buffer's policy) or default ones
template <typename T, int N, int TZ, int EZ, bool STREAM = true, typename BF>
__device__ __forceinline__ void c2r_load_k(cx<T>* xk, cx<T>& xn, int t, const BF& f, uint32_t soff,
                                           uint32_t row_id) {
  constexpr uint32_t cs = sizeof(cx<T>);
  const uint32_t r0 = spec_row<T, N>(row_id);
#pragma unroll
  for (int m = 0; m < EZ; ++m) {
    const uint32_t o = (r0 + t + TZ * m) * cs;
    xk[m] = STREAM ? f.template ldnt<cx<T>>(o, soff) : f.template ld<cx<T>>(o, soff);
  }
  const uint32_t on = (spec_nyq<T, N>() + row_id) * cs;
  xn = STREAM ? f.template ldnt<cx<T>>(on, soff) : f.template ld<cx<T>>(on, soff);
}

// X[H - k] of the lane's elements k = t + TZ m (X[H] for k = 0) through the
// row's LDS buffer, which is free again on return
template <typename T, int N, int TZ, int EZ>
__device__ __forceinline__ void c2r_mirror(cx<T>* xm, const cx<T>* xk, cx<T> xn, int t, cx<T>* row) {
  constexpr int H = N / 2;
#pragma unroll
  for (int m = 0; m < EZ; ++m) row[t + TZ * m] = xk[m];
  lds_sync<row_in_wave<TZ>()>();
#pragma unroll
  for (int m = 0; m < EZ; ++m) {
    const int k = t + TZ * m;
    xm[m] = k == 0 ? xn : row[H - k];
  }
  lds_sync<row_in_wave<TZ>()>();
}

// The c2r pre-step (inverse real transform along z): from X[k] (k < H) and
// X[H] build C[k] = (X[k] + conj X[H-k]) + i (X[k] - conj X[H-k]) W^-k; the
// unnormalised length-H inverse of C is then n (a[2j] + i a[2j+1]).
// xk0, xm0: X[k] and X[H - k] (X[H] for k = 0) at the lane's elements.
// zmul: transform i s_z X instead of X (s_z = k below the Nyquist index, 0 at it)
template <typename T, int N, int TZ, int EZ>
__device__ __forceinline__ void c2r_combine(cx<T>* v, const cx<T>* xk0, const cx<T>* xm0, int t,
                                            const cx<T>* twN, bool zmul = false) {
  constexpr int H = N / 2;
#pragma unroll
  for (int m = 0; m < EZ; ++m) {
    const int k = t + TZ * m;
    cx<T> xk = xk0[m], xm = xm0[m];
    if (k == 0) { xk.y = (T)0; xm.y = (T)0; }
    if (zmul) {
      xk = cscale<T>(cmuli<T>(xk), (T)k);
      xm = k == 0 ? mk<T>((T)0, (T)0) : cscale<T>(cmuli<T>(xm), (T)(H - k));
    }
    const cx<T> cm = cconj<T>(xm);
    const cx<T> s = cadd<T>(xk, cm);
    const cx<T> d = csub<T>(xk, cm);
    v[m] = cadd<T>(s, cmuli<T>(cmulc<T>(d, twN[k])));
  }
}

template <typename T>
__device__ __forceinline__ uint64_t spec_bytes(const EvalArgs& a, int nf) {
  return (uint64_t)nf * a.fstride * sizeof(cx<T>);
}

// P1: z r2c of the S input densities (float64) into specA
template <typename T, int N, int V = 0>
__global__ void __launch_bounds__((Geo<T, N, V>::RZ * Geo<T, N, V>::TZ))
    k_zfwd(const EvalArgs* __restrict__ args) {
  using G = Geo<T, N, V>;
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
  const uint32_t row = (uint32_t)(tile * RZ + r);
  cx<T>* lrow = xch + r * H;
  const LdsPencil<T, row_in_wave<TZ>()> lp{lrow, 1};
  const BufN<N> A = make_buf<stream_policy<N>()>(a.specA, spec_bytes<T>(a, a.S));
  if (a.ext_n == 0) {
    constexpr uint32_t n3b = (uint32_t)N * N * N * sizeof(double);
    const BufN<N> rho = make_buf<stream_policy<N>()>(a.rho, (uint64_t)a.S * n3b);
    for (int s = 0; s < a.S; ++s) {
      cx<T> v[EZ];
#pragma unroll
      for (int m = 0; m < EZ; ++m) {
        const cf64 p = rho.template ldnt<cf64>((row * H + t + TZ * m) * (uint32_t)sizeof(cf64), (uint32_t)s * n3b);
        v[m] = mk<T>((T)p.x, (T)p.y);
      }
      fft_pencil<T, H, EZ, true>(v, t, twH, lp);
      r2c_post<T, N, TZ, EZ>(v, t, twN, lrow, A, (uint32_t)(s * a.fstride * sizeof(cx<T>)), row);
    }
  } else {
    // zero extension of the (even-sized) domain: the point pair (2j, 2j+1)
    // lies inside or outside it as a whole
    const uint32_t nd = (uint32_t)a.ext_n, x = row / N, y = row % N;
    const bool row_in = x < nd && y < nd;
    const uint32_t d3b = nd * nd * nd * (uint32_t)sizeof(double);
    const BufN<N> rho = make_buf<stream_policy<N>()>(a.rho, a.ext_bulk ? 0 : (uint64_t)a.S * d3b);
    for (int s = 0; s < a.S; ++s) {
      cx<T> v[EZ];
#pragma unroll
      for (int m = 0; m < EZ; ++m) {
        const uint32_t j = t + TZ * m;
        cf64 p{0.0, 0.0};
        if (row_in && 2 * j < nd) {
          if (a.ext_bulk) p = cf64{a.ext_val[s], a.ext_val[s]};
          else p = rho.template ldnt<cf64>(((x * nd + y) * nd + 2 * j) * (uint32_t)sizeof(double), (uint32_t)s * d3b);
        }
        v[m] = mk<T>((T)p.x, (T)p.y);
      }
      fft_pencil<T, H, EZ, true>(v, t, twH, lp);
      r2c_post<T, N, TZ, EZ>(v, t, twN, lrow, A, (uint32_t)(s * a.fstride * sizeof(cx<T>)), row);
    }
  }
}

// P9 (final_mode = 1): z c2r of the S chemical-potential spectra in `sel`,
// + constants, write beta mu_ex and exp(-beta mu_ex) in float64.
// final_mode = 0: z c2r of `nreal` spectra of `sel` into out (no constant).
template <typename T, int N, int V = 0>
__global__ void __launch_bounds__((Geo<T, N, V>::RZ * Geo<T, N, V>::TZ))
    k_zinv(const EvalArgs* __restrict__ args, int sel) {
  using G = Geo<T, N, V>;
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
  const uint32_t row = (uint32_t)(tile * RZ + r);
  const LdsPencil<T, row_in_wave<TZ>()> lp{xch + r * H, 1};
  const BufN<N> src = make_buf<stream_policy<N>()>(sel == 0 ? a.specA : sel == 1 ? a.specB : a.specC, spec_bytes<T>(a, a.nreal));
  constexpr uint32_t n3 = (uint32_t)N * N * N;
  constexpr uint32_t n3b = n3 * sizeof(double);
  const BufN<N> out = make_buf<stream_policy<N>()>(a.out, (uint64_t)a.nreal * n3b);
  const BufN<N> slot = make_buf<stream_policy<N>()>(a.slot, a.slot ? (uint64_t)a.nreal * n3b : 0);
  uint32_t bad = 0u, badidx = 0xffffffffu;
  for (int s = 0; s < a.nreal; ++s) {
    cx<T> v[EZ], xk[EZ], xm[EZ];
    const uint32_t si = (uint32_t)(s * a.fstride * sizeof(cx<T>));
    if constexpr (mirror_lds<N>()) {
      cx<T> xn;
      c2r_load_k<T, N, TZ, EZ, false>(xk, xn, t, src, si, row);
      c2r_mirror<T, N, TZ, EZ>(xm, xk, xn, t, xch + r * H);
    } else {
      c2r_load<T, N, TZ, EZ>(xk, xm, t, src, si, row);  // the policy is the default one here
    }
    c2r_combine<T, N, TZ, EZ>(v, xk, xm, t, twN, (a.zmul_mask >> s) & 1u);
    fft_pencil<T, H, EZ, false>(v, t, twH, lp);
    const uint32_t so = (uint32_t)s * n3b;
    if (a.final_mode) {
      const double c = a.cfin[s];
#pragma unroll
      for (int m = 0; m < EZ; ++m) {
        const uint32_t j = row * H + t + TZ * m;  // index of the point pair (2j, 2j+1)
        const double m0 = (double)v[m].x + c, m1 = (double)v[m].y + c;
        out.template st<cf64>(cf64{m0, m1}, j * (uint32_t)sizeof(cf64), so);
        if (!(isfinite(m0) && isfinite(m1))) {
          bad |= kStNonFinite;
          badidx = min(badidx, (uint32_t)s * n3 + 2 * j);
        }
        if (a.slot) {
          // exp(-mu) overflows a double once -mu exceeds ln(DBL_MAX)
          if (-m0 > 709.782712893384 || -m1 > 709.782712893384) {
            bad |= kStOverflow;
            badidx = min(badidx, (uint32_t)s * n3 + 2 * j);
          }
          slot.template st<cf64>(cf64{exp(-m0), exp(-m1)}, j * (uint32_t)sizeof(cf64), so);
        }
      }
    } else {
#pragma unroll
      for (int m = 0; m < EZ; ++m)
        out.template st<cf64>(cf64{(double)v[m].x, (double)v[m].y}, (row * H + t + TZ * m) * (uint32_t)sizeof(cf64), so);
    }
  }
  if (bad) raise_status(a.status, bad, badidx);
}

// P5: z c2r of the 10 weighted densities, the FMT derivatives (Sec. 2.3.1),
// z r2c of the 10 derivative fields; in place on specB.  ln(1 - n3) and the
// powers of 1 / (1 - n3) (and the White Bear coefficient) are evaluated in
// float64; their products with the weighted densities in the FFT type (in
// float64 for free-energy calls).
// Every thread keeps its EZD elements of all ten fields in registers, so the
// ten values at a grid point meet in one thread without an LDS round trip.
template <typename T, int N>
constexpr int default_ezd() {
  return ((N / 2) % 3 == 0) ? 6 : ((N / 2) >= (sizeof(T) == 4 ? 4 : 2) ? (sizeof(T) == 4 ? 4 : 2) : N / 2);
}
// elements per thread of the derivative pass under launch variant V (bit 1:
// secondary schedule; RDD * TZD <= 256 for any choice)
template <typename T, int N, int V>
constexpr int ezd_of() {
  return (V & 2) ? alt_ept(N / 2, default_ezd<T, N>(), 1) : default_ezd<T, N>();
}

template <typename T, int N, int EZ = default_ezd<T, N>(), int V = 0> struct GeoD {
  static constexpr int H = N / 2;
  static constexpr int EZD = EZ;
  static constexpr int TZD = H / EZD;
  static constexpr int RDD = narrow(pow2_divisor_le((long)N * N, 256 / TZD < 1 ? 1 : 256 / TZD), V);
  static constexpr int tiles = (N * N) / RDD;
};

// The pre- and post-steps of the real transforms with the lane's constants
// P_k = (1 - i W^k) / 2 in registers (twp[m] for k = t + TZ m).  With cm the
// conjugated mirror value, the r2c step E + W^k (-i) O of r2c_post is
// cm + P_k (c - cm), and the c2r step of c2r_combine, (X_k + cm) + i conj(W^k)
// (X_k - cm), equals 2 (cm + conj(P_k) (X_k - cm)): six and eight
// instructions per element instead of fourteen and ten.
template <typename T, int N, int TZ, int EZ>
__device__ __forceinline__ void c2r_combine_p(cx<T>* v, const cx<T>* xk0, const cx<T>* xm0, int t,
                                              const cx<T>* twp, bool zmul = false) {
  constexpr int H = N / 2;
#pragma unroll
  for (int m = 0; m < EZ; ++m) {
    const int k = t + TZ * m;
    cx<T> xk = xk0[m], xm = xm0[m];
    if (k == 0) { xk.y = (T)0; xm.y = (T)0; }
    if (zmul) {
      xk = cscale<T>(cmuli<T>(xk), (T)k);
      xm = k == 0 ? mk<T>((T)0, (T)0) : cscale<T>(cmuli<T>(xm), (T)(H - k));
    }
    const T cmx = xm.x, cmy = -xm.y;  // cm = conj(xm)
    const T dx = xk.x - cmx, dy = xk.y - cmy;
    const cx<T> P = twp[m];
    // cm + conj(P) d = (cm.x + P.x dx + P.y dy, cm.y + P.x dy - P.y dx)
    const T rx = fma(P.x, dx, fma(P.y, dy, cmx));
    const T ry = fma(P.x, dy, fma(-P.y, dx, cmy));
    v[m] = mk<T>(rx + rx, ry + ry);
  }
}

template <typename T, int N, int TZ, int EZ, typename BF>
__device__ __forceinline__ void r2c_post_p(cx<T>* v, int t, const cx<T>* twp, cx<T>* row, const BF& f,
                                           uint32_t soff, uint32_t row_id, bool zmul = false) {
  constexpr int H = N / 2;
  constexpr uint32_t cs = sizeof(cx<T>);
#pragma unroll
  for (int m = 0; m < EZ; ++m) row[t + TZ * m] = v[m];
  lds_sync<row_in_wave<TZ>()>();
#pragma unroll
  for (int m = 0; m < EZ; ++m) {
    const int k = t + TZ * m;
    const cx<T> c = v[m];
    const cx<T> r = row[k == 0 ? 0 : H - k];
    const T cmx = r.x, cmy = -r.y;  // cm = conj(C[H - k])
    const T dx = c.x - cmx, dy = c.y - cmy;
    const cx<T> P = twp[m];
    cx<T> x = mk<T>(fma(P.x, dx, fma(-P.y, dy, cmx)), fma(P.x, dy, fma(P.y, dx, cmy)));
    if (zmul) x = cscale<T>(cmuli<T>(x), (T)k);
    f.template st<cx<T>>(x, (spec_row<T, N>(row_id) + k) * cs, soff);
    if (k == 0) f.template st<cx<T>>(zmul ? mk<T>((T)0, (T)0) : mk<T>(c.x - c.y, (T)0),
                            (spec_nyq<T, N>() + row_id) * cs, soff);
  }
  lds_sync<row_in_wave<TZ>()>();
}

// 1 / x in FP64: hardware reciprocal estimate refined by two Newton steps
// (error within an ulp of the quotient)
__device__ __forceinline__ double recip_f64(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, y, 1.0);
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-x, y, 1.0);
  return __builtin_fma(y, e, y);
}

// Natural logarithm in FP64 by table reduction.  Write u = m 2^e with m in
// [1/2, 1).  The top eight fraction bits of m select entry j, for the
// interval centred on c_j = 1/2 + (j + 1/2) / 512: ic_j is a double close to
// 1 / c_j and nl_j = -ln(ic_j) (both made once per workgroup by
// log_table_init).  Then r = m ic_j - 1 (one fma, so r is the correctly
// rounded value; |r| <= 2^-9) and ln u = e ln 2 + nl_j + log1p(r), with
// log1p(r) = r - r^2/2 + ... + r^7/7 (truncation below 2^-66 relative) and
// ln 2 split into a head whose products with e are exact and a tail.
// Within 2^-9 of 1 the series runs on r = u - 1 (exact) with no table, so
// ln u keeps full relative accuracy there; elsewhere the error is within a
// few units in the last place of the result (the rounding of nl_j and of
// the final sum), and a few units of 1e-16 in absolute terms where e = 1 and
// u is just above 1 + 2^-9.  Any u maps to an entry in [0, 255] (the index
// is masked), so non-positive or non-finite inputs give a meaningless value
// without touching memory outside the table.
struct LogEntry {
  double ic, nl;
};
constexpr int kLogTable = 256;

__device__ __forceinline__ void log_table_init(LogEntry* tab) {
  for (int j = threadIdx.x; j < kLogTable; j += blockDim.x) {
    const double ic = 1.0 / (0.5 + ((double)j + 0.5) / 512.0);
    tab[j] = LogEntry{ic, -log(ic)};
  }
}

__device__ __forceinline__ double log_f64(double u, const LogEntry* tab) {
  constexpr double ln2_hi = 6.93147180369123816490e-01;  // 32 significant bits
  constexpr double ln2_lo = 1.90821492927058770002e-10;
  const double m = __builtin_amdgcn_frexp_mant(u);
  const int e = __builtin_amdgcn_frexp_exp(u);
  const uint32_t hi = (uint32_t)(__builtin_bit_cast(uint64_t, m) >> 32);
  const LogEntry t = tab[(hi >> 12) & (kLogTable - 1)];
  const bool near1 = fabs(u - 1.0) < 0x1p-9;
  const double r = near1 ? u - 1.0 : __builtin_fma(m, t.ic, -1.0);
  double q = 1.0 / 7.0;
  q = __builtin_fma(q, r, -1.0 / 6.0);
  q = __builtin_fma(q, r, 1.0 / 5.0);
  q = __builtin_fma(q, r, -0.25);
  q = __builtin_fma(q, r, 1.0 / 3.0);
  q = __builtin_fma(q, r, -0.5);
  const double lp = __builtin_fma(q, r * r, r);  // log1p(r)
  const double ed = (double)e;
  const double head = __builtin_fma(ed, ln2_hi, t.nl);
  const double tail = __builtin_fma(ed, ln2_lo, lp);
  return near1 ? lp : head + tail;
}

// Coefficient of the n2^3 term of the modified (White Bear) functional,
// phi3(x) = [x + (1 - x)^2 ln(1 - x)] / (36 pi x^2 (1 - x)^2), as
// g = 36 pi phi3 and its derivative g'.  With u = 1 - x:
//   g  = 1 / (x u^2) + ln(u) / x^2,
//   g' = 2 / (x u^3) - 1 / (x^2 u^2) - 1 / (x^2 u) - 2 ln(u) / x^3.
// Both forms cancel as x -> 0; below |x| = 0.05 the power series
// g = sum_k (k+1)(k+3)/(k+2) x^k (from the series of ln(1 - x)) is used
// instead, 16 terms (truncation of g and g' below 1e-17 relative).
// inv = 1 / u and lnu = ln(u) come from the caller.
__device__ __forceinline__ void wb_coeff(double x, double inv, double lnu, double& g, double& dg) {
  constexpr int K = 16;
  double gs = (double)(K * (K + 2)) / (double)(K + 1), dgs = (double)(K - 1) * gs;
  // Horner from the top coefficient down: c_k = (k+1)(k+3)/(k+2)
#pragma unroll
  for (int k = K - 2; k >= 0; --k) {
    gs = __builtin_fma(gs, x, (double)((k + 1) * (k + 3)) / (double)(k + 2));
    if (k >= 1) dgs = __builtin_fma(dgs, x, (double)k * ((double)((k + 1) * (k + 3)) / (double)(k + 2)));
  }
  const bool small = fabs(x) < 0.05;
  const double xl = small ? 0.5 : x;
  const double ix = recip_f64(xl), ix2 = ix * ix;
  const double il = small ? 2.0 : inv, ll = small ? -0.6931471805599453 : lnu;
  const double gl = ix * il * il + ll * ix2;
  const double dgl = ix * (2.0 * il * il * il - ix * il * il - ix * il - 2.0 * ll * ix2);
  g = small ? gs : gl;
  dg = small ? dgs : dgl;
}

// PHI: also sum Phi_hs per workgroup into a.phi_part (free-energy calls)
// WB: the functional this variant evaluates (White Bear or Rosenfeld); blocks
// of instances that select the other one exit, so a launch list holding both
// runs each variant over it and every instance gets the same arithmetic as
// when evaluated alone
// The FP32 Rosenfeld variant (the hot one) is held to two waves per SIMD:
// with six elements per thread (sizes with a factor 3) the compiler would
// otherwise take a few registers past 256 and run one wave per SIMD (a
// 2.5x slower pass at 192^3), where two waves cost a spill of 16 registers.
template <typename T, int N, bool PHI = false, bool WB = false, int EZD = default_ezd<T, N>(), int V = 0>
__global__ void __launch_bounds__((GeoD<T, N, EZD, V>::RDD * GeoD<T, N, EZD, V>::TZD), (PHI || WB || sizeof(T) == 8) ? 1 : 2)
    k_zderiv(const EvalArgs* __restrict__ args) {
  using D = GeoD<T, N, EZD, V>;
  constexpr int H = D::H, TZ = D::TZD, EZ = D::EZD, RD = D::RDD;
  __shared__ cx<T> twH[H];
  __shared__ cx<T> twN[N];
  __shared__ cx<T> xch[RD * H];
  __shared__ LogEntry logt[kLogTable];
  int tile;
  const EvalArgs& a = args[inst_of(D::tiles, tile)];
  if (!a.hs_on || (a.hs_wb != 0) != WB) return;  // uniform per block
  const int t = threadIdx.x % TZ, r = threadIdx.x / TZ;
  const uint32_t row = (uint32_t)(tile * RD + r);
  cx<T>* lrow = xch + r * H;
  const LdsPencil<T, row_in_wave<TZ>()> lp{lrow, 1};
  const BufN<N> B = make_buf<stream_policy<N>()>(a.specB, spec_bytes<T>(a, kFields));
  const uint32_t fbytes = __builtin_amdgcn_readfirstlane((uint32_t)(a.fstride * sizeof(cx<T>)));
  cx<T> val[kFields * EZ];
  // The FFT twiddles of this lane and the constants P_k = (1 - i W^k) / 2 of
  // the r2c / c2r steps of its elements (c2r_combine_p, r2c_post_p; z_deriv
  // 353 -> 347 us at 256^3 against the same steps on W^k), held in registers
  // for all twenty transforms; with six elements per thread (sizes with a
  // factor 3) the registers go to the values and the twiddles are read from
  // LDS instead.
  constexpr bool kTwRegs = EZ < 6;
  typename std::conditional<kTwRegs, TwReg<T, H, EZ>, char>::type twr;
  cx<T> twp[kTwRegs ? EZ : 1];
  {
    // the raw values of fields q + 1 and q + 2 are in flight while field q is
    // transformed (z_deriv 357 -> 350 us at 256^3; three ahead gained
    // nothing more); those of fields 0 and 1 while the twiddle tables are
    // built.  With six elements per thread (sizes with a factor 3) there is
    // no room for further buffers: each field's values are loaded just before
    // its transform.
    // With the mirror values from LDS (mirror_lds) only X[k] and X[H] of a
    // row are in flight: half the load instructions and registers.
    constexpr int kAhead = kTwRegs ? 2 : 0;
    constexpr int kBufs = kAhead + 1;
    constexpr bool kLds = mirror_lds<N>();
    cx<T> kb[kBufs][EZ], mb[kLds ? 1 : kBufs][EZ], nb[kLds ? kBufs : 1];
#pragma unroll
    for (int q = 0; q < (kAhead > 0 ? kAhead : 1); ++q) {
      if constexpr (kLds) c2r_load_k<T, N, TZ, EZ>(kb[q], nb[q], t, B, (uint32_t)q * fbytes, row);
      else c2r_load<T, N, TZ, EZ>(kb[q], mb[q], t, B, (uint32_t)q * fbytes, row);
    }
    init_twiddles<T, H>(twH);
    init_twiddles<T, N>(twN);
    log_table_init(logt);
    __syncthreads();
    if constexpr (kTwRegs) {
      twr.load(t, twH);
#pragma unroll
      for (int m = 0; m < EZ; ++m) {
        const cx<T> w = twN[t + TZ * m];
        twp[m] = mk<T>((T)0.5 + (T)0.5 * w.y, (T)-0.5 * w.x);
      }
    }
#pragma unroll
    for (int q = 0; q < kFields; ++q) {
      cx<T>* kc = kb[q % kBufs];
      cx<T>* mc = mb[kLds ? 0 : q % kBufs];
      if constexpr (kAhead > 0) {
        if (q + kAhead < kFields) {
          const int qa = q + kAhead, ba = qa % kBufs;
          if constexpr (kLds) c2r_load_k<T, N, TZ, EZ>(kb[ba], nb[ba], t, B, (uint32_t)qa * fbytes, row);
          else c2r_load<T, N, TZ, EZ>(kb[ba], mb[ba], t, B, (uint32_t)qa * fbytes, row);
        }
      } else if (q > 0) {
        if constexpr (kLds) c2r_load_k<T, N, TZ, EZ>(kc, nb[0], t, B, (uint32_t)q * fbytes, row);
        else c2r_load<T, N, TZ, EZ>(kc, mc, t, B, (uint32_t)q * fbytes, row);
      }
      if constexpr (kLds) c2r_mirror<T, N, TZ, EZ>(mc, kc, nb[q % kBufs], t, lrow);
      // the z component of each vector density is i s_z Q_b, formed here
      if constexpr (kTwRegs) {
        c2r_combine_p<T, N, TZ, EZ>(val + q * EZ, kc, mc, t, twp, q == kSlotZ || q == kSlotZ + kVecStride);
        fft_pencil<T, N / 2, EZ, false>(val + q * EZ, t, twr, lp);
      } else {
        c2r_combine<T, N, TZ, EZ>(val + q * EZ, kc, mc, t, twN, q == kSlotZ || q == kSlotZ + kVecStride);
        fft_pencil<T, N / 2, EZ, false>(val + q * EZ, t, (const cx<T>*)twH, lp);
      }
    }
  }
  if (a.ext_n != 0) {
    // Aperiodic mode: Phi_hs is integrated over the domain only (Sec. 2.3.1),
    // so the derivative fields vanish outside it.  The weighted densities
    // there are replaced by zero, which makes every derivative zero (Phi and
    // its gradient vanish at n = 0) and keeps those points out of the status
    // checks.  The domain size is even: a point pair lies in it or not.
    const uint32_t nd = (uint32_t)a.ext_n;
    const bool row_in = row / N < nd && row % N < nd;
#pragma unroll
    for (int m = 0; m < EZ; ++m) {
      if (!(row_in && 2u * (uint32_t)(t + TZ * m) < nd)) {
#pragma unroll
        for (int q = 0; q < kFields; ++q) val[q * EZ + m] = mk<T>((T)0, (T)0);
      }
    }
  }
  uint32_t bad = 0u, badidx = 0xffffffffu;
  const double inv8pi = 1.0 / (8.0 * kPi), inv12pi = 1.0 / (12.0 * kPi), inv4pi = 1.0 / (4.0 * kPi);
  const double inv24pi = 1.0 / (24.0 * kPi), inv36pi = 1.0 / (36.0 * kPi);
  double phi = 0.0;  // Phi_hs summed over this thread's grid points
  // type of the products of the weighted densities with those factors: the
  // FFT type, except for free-energy calls (double throughout, Phi summed in
  // double)
  using P = typename std::conditional<PHI, double, T>::type;
#pragma unroll
  for (int m = 0; m < EZ; ++m) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // the two real points z = 2j, 2j+1 of element j
      P f[kFields];
#pragma unroll
      for (int q = 0; q < kFields; ++q) f[q] = h ? (P)val[q * EZ + m].y : (P)val[q * EZ + m].x;
      const P n0 = f[0], n1 = f[1], n2 = f[2], n3 = f[3];
      const P a1x = f[4], a1y = f[5], a1z = f[6], a2x = f[7], a2y = f[8], a2z = f[9];
      if (!(n3 < (P)1)) {
        bad |= isfinite(n3) ? kStPacking : kStNonFinite;
        badidx = min(badidx, row * N + 2 * (t + TZ * m) + h);
      }
      // the logarithm and the powers of 1 / (1 - n3) in double
      const double n3d = (double)n3, u = 1.0 - n3d;
      const double inv = recip_f64(u), inv2 = inv * inv, inv3 = inv2 * inv;
      // -ln(1 - n3): log of the rounded u plus the first-order correction for
      // the rounding of u, which equals log1p(-n3) to working precision
      const double d0 = -(log_f64(u, logt) - ((u - 1.0) + n3d) * inv);
      const P i1 = (P)inv, i2 = (P)inv2;
      const P v12 = a1x * a2x + a1y * a2y + a1z * a2z;
      const P v22 = a2x * a2x + a2y * a2y + a2z * a2z;
      P d[kFields];
      d[0] = (P)d0;
      // Phi_hs (Sec. 2.3.1): -n0 ln(1 - n3) + (n1 n2 - n1v.n2v) / (1 - n3)
      //                      + (n2^3 - 3 n2 n2v.n2v) phi3(n3)
      // with phi3 = 1 / (24 pi (1 - n3)^2) (Rosenfeld) or the modified form
      P c2;  // 6 n2 phi3: the n2v coefficient of d[7..9]
      d[1] = n2 * i1;
      if constexpr (WB) {
        double g, dg;
        wb_coeff(n3d, inv, -d0, g, dg);
        const P p3 = (P)(g * inv36pi), dp3 = (P)(dg * inv36pi);  // phi3 and its derivative
        c2 = (P)6 * n2 * p3;
        if constexpr (PHI) phi += n0 * d0 + (n1 * n2 - v12) * inv + (n2 * n2 * n2 - 3.0 * n2 * v22) * p3;
        d[2] = n1 * i1 + (P)3 * (n2 * n2 - v22) * p3;
        d[3] = n0 * i1 + (n1 * n2 - v12) * i2 + (n2 * n2 * n2 - (P)3 * n2 * v22) * dp3;
      } else {
        // Rosenfeld: 3 phi3 = 1 / (8 pi u^2), phi3' = 1 / (12 pi u^3), 6 n2 phi3 = n2 / (4 pi u^2)
        c2 = n2 * i2 * (P)inv4pi;
        if constexpr (PHI) phi += n0 * d0 + (n1 * n2 - v12) * inv + (n2 * n2 * n2 - 3.0 * n2 * v22) * inv2 * inv24pi;
        d[2] = n1 * i1 + (n2 * n2 - v22) * i2 * (P)inv8pi;
        d[3] = n0 * i1 + (n1 * n2 - v12) * i2 + (n2 * n2 * n2 - (P)3 * n2 * v22) * (P)inv3 * (P)inv12pi;
      }
      d[4] = -a2x * i1;
      d[5] = -a2y * i1;
      d[6] = -a2z * i1;
      d[7] = -a1x * i1 - c2 * a2x;
      d[8] = -a1y * i1 - c2 * a2y;
      d[9] = -a1z * i1 - c2 * a2z;
#pragma unroll
      for (int q = 0; q < kFields; ++q) {
        if (h) val[q * EZ + m].y = (T)d[q];
        else val[q * EZ + m].x = (T)d[q];
      }
      __builtin_amdgcn_sched_barrier(0);  // one grid point at a time
    }
  }
#pragma unroll
  for (int q = 0; q < kFields; ++q) {
    // the z components of the vector derivatives leave as i s_z F_z
    if constexpr (kTwRegs) {
      fft_pencil<T, N / 2, EZ, true>(val + q * EZ, t, twr, lp);
      r2c_post_p<T, N, TZ, EZ>(val + q * EZ, t, twp, lrow, B, q * fbytes, row, q == kSlotZ || q == kSlotZ + kVecStride);
    } else {
      fft_pencil<T, N / 2, EZ, true>(val + q * EZ, t, (const cx<T>*)twH, lp);
      r2c_post<T, N, TZ, EZ>(val + q * EZ, t, twN, lrow, B, q * fbytes, row, q == kSlotZ || q == kSlotZ + kVecStride);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  if (bad) raise_status(a.status, bad, badidx);
  if constexpr (PHI) {
    __shared__ double red[16];
    const double tot = block_sum(phi, red);
    if (threadIdx.x == 0) a.phi_part[tile] = tot;
  }
}

// ---------------------------------------------------------------------------
// y direction: c2c along y for every (x, kz) pencil of the main array and
// every x row of the Nyquist plane; in place on `nf` fields of `sel`
// (nf_code -1: S fields).  nf_code kVecMode: the ten FMT fields of specB
// with the vector-component bookkeeping of the field-slot layout: the
// inverse pass also writes [y] = i s_y Q_b next to Q_b; the forward pass
// writes [z] = i s_y F_y + [z] and leaves [y] unused.
// ---------------------------------------------------------------------------
constexpr int kVecMode = -2;

template <typename T, int N, int EY, int TY>
__device__ __forceinline__ void mul_isy(cx<T>* v, int t) {
#pragma unroll
  for (int m = 0; m < EY; ++m) {
    const int ky = t + TY * m;
    const T sy = ky == N / 2 ? (T)0 : (T)sgn_idx(ky, N);
    v[m] = cscale<T>(cmuli<T>(v[m]), sy);
  }
}

template <typename T, int N, bool FWD, int V = 0>
__global__ void __launch_bounds__((Geo<T, N, V>::PY * Geo<T, N, V>::TY))
    k_ystep(const EvalArgs* __restrict__ args, int sel, int nf_code, int part) {
  using G = Geo<T, N, V>;
  constexpr int H = G::H, TY = G::TY, EY = G::EY, PY = G::PY;
  __shared__ cx<T> tw[N];
  __shared__ cx<T> xch[PY * N];
  int tile;
  const EvalArgs& a = args[inst_of_part((N * H) / PY, N / PY, part, tile)];
  if (sel == 1 && !a.hs_on) return;  // uniform per block
  init_twiddles<T, N>(tw);
  __syncthreads();
  const bool vec = nf_code == kVecMode;
  const int nf = nf_code == -1 ? a.S : vec ? kFields : nf_code;
  const BufN<N> base = make_buf<stream_policy<N>()>(sel == 0 ? a.specA : sel == 1 ? a.specB : a.specC, spec_bytes<T>(a, nf));
  constexpr int tiles_main = (N * H) / PY;
  uint32_t off, es;
  int t;
  LdsPencil<T> lp;
  if (tile < tiles_main) {
    const int p = threadIdx.x % PY;
    t = threadIdx.x / PY;
    const uint32_t pen = (uint32_t)(tile * PY + p);  // (x, kz)
    off = (pen / H) * (uint32_t)spec_plane(N, sizeof(T)) + (pen % H);
    es = H;
    lp = LdsPencil<T>{xch + p, PY};
  } else {
    const int p = threadIdx.x / TY;
    t = threadIdx.x % TY;
    const uint32_t x = (uint32_t)((tile - tiles_main) * PY + p);
    off = spec_nyq<T, N>() + x * N;
    es = 1;
    lp = LdsPencil<T>{xch + p * N, 1};
  }
  uint32_t eo[EY];
#pragma unroll
  for (int m = 0; m < EY; ++m) eo[m] = (off + (uint32_t)(t + TY * m) * es) * (uint32_t)sizeof(cx<T>);
  const uint32_t fbytes = (uint32_t)(a.fstride * sizeof(cx<T>));
  for (int f = 0; f < nf; ++f) {
    if (vec && (f - kSlotX) % kVecStride != 0 && f > kSlotX) continue;  // [y], [z] below
    const uint32_t so = (uint32_t)f * fbytes;
    cx<T> v[EY];
#pragma unroll
    for (int m = 0; m < EY; ++m) v[m] = base.template ld<cx<T>>(eo[m], so);
    fft_pencil<T, N, EY, FWD>(v, t, tw, lp);
#pragma unroll
    for (int m = 0; m < EY; ++m) base.template st<cx<T>>(v[m], eo[m], so);
  }
  if (!vec) return;
#pragma unroll 1
  for (int b = 0; b < 2; ++b) {
    const uint32_t sy_off = (uint32_t)(kSlotY + kVecStride * b) * fbytes;
    const uint32_t sz_off = (uint32_t)(kSlotZ + kVecStride * b) * fbytes;
    if constexpr (!FWD) {
      // Q_b -> [y] = y-inverse of i s_y Q_b and [z] = y-inverse of Q_b
      cx<T> q[EY], w[EY];
#pragma unroll
      for (int m = 0; m < EY; ++m) q[m] = base.template ld<cx<T>>(eo[m], sz_off);
#pragma unroll
      for (int m = 0; m < EY; ++m) w[m] = q[m];
      mul_isy<T, N, EY, TY>(w, t);
      fft_pencil<T, N, EY, false>(w, t, tw, lp);
#pragma unroll
      for (int m = 0; m < EY; ++m) base.template st<cx<T>>(w[m], eo[m], sy_off);
      fft_pencil<T, N, EY, false>(q, t, tw, lp);
#pragma unroll
      for (int m = 0; m < EY; ++m) base.template st<cx<T>>(q[m], eo[m], sz_off);
    } else {
      // [z] <- i s_y (y-forward of F_y) + y-forward of [z]
      cx<T> fy[EY], g[EY];
#pragma unroll
      for (int m = 0; m < EY; ++m) fy[m] = base.template ld<cx<T>>(eo[m], sy_off);
#pragma unroll
      for (int m = 0; m < EY; ++m) g[m] = base.template ld<cx<T>>(eo[m], sz_off);
      fft_pencil<T, N, EY, true>(fy, t, tw, lp);
      mul_isy<T, N, EY, TY>(fy, t);
      fft_pencil<T, N, EY, true>(g, t, tw, lp);
#pragma unroll
      for (int m = 0; m < EY; ++m) base.template st<cx<T>>(cadd<T>(g[m], fy[m]), eo[m], sz_off);
    }
  }
}

// ---------------------------------------------------------------------------
// x direction helpers: pencil (ky, kz) of the main array or ky of the Nyquist
// plane, element kx at stride es.
// ---------------------------------------------------------------------------
template <typename T, int N, int PX>
struct XPencil {
  uint32_t off, es;  // element kx of the pencil at off + kx * es
  int ky, kz;
  __device__ __forceinline__ XPencil(int tile, int p) {
    constexpr int H = N / 2;
    const int pen = tile * PX + p;
    constexpr int nmain = N * H;
    if (pen < nmain) {
      off = (uint32_t)pen; es = (uint32_t)spec_plane(N, sizeof(T)); ky = pen / H; kz = pen % H;
    } else {
      const int q = pen - nmain;
      off = spec_nyq<T, N>() + (uint32_t)q; es = N; ky = q; kz = H;
    }
  }
};

template <int N, int PX> constexpr int x_tiles() { return (N * (N / 2)) / PX + N / PX; }


template <typename T>
__device__ __forceinline__ T inv_sqrt_m(int m) {
  if constexpr (sizeof(T) == 4) return m == 0 ? 0.0f : __builtin_amdgcn_rsqf((float)m);
  else return m == 0 ? 0.0 : 1.0 / sqrt((double)m);
}

// per-lane k-space data of the EX elements a thread owns
template <typename T, int N, int EX, int TX>
struct XKs {
  int mm[EX];   // integer |j|^2
  T ux[EX];     // unit-vector components (0 on that axis's Nyquist plane)
  T uy[EX];
  T uz[EX];
  __device__ __forceinline__ XKs(int t, int ky, int kz) {
    constexpr int H = N / 2;
    const int sy = sgn_idx(ky, N), sz = kz;
#pragma unroll
    for (int m = 0; m < EX; ++m) {
      const int kx = t + TX * m;
      const int sx = sgn_idx(kx, N);
      mm[m] = sx * sx + sy * sy + sz * sz;
      const T r = inv_sqrt_m<T>(mm[m]);
      ux[m] = kx == H ? (T)0 : (T)sx * r;
      uy[m] = ky == H ? (T)0 : (T)sy * r;
      uz[m] = kz == H ? (T)0 : (T)sz * r;
    }
  }
};

template <typename T, int N>
__device__ __forceinline__ uint64_t table_m(int /*unused*/) { return 3ull * (N / 2) * (N / 2) + 1; }

// sin and cos of x >= 0 in FP32 for the arguments k R of a grid (x up to a
// few hundred): Cody-Waite reduction by pi/2 with a three-part constant and
// fused multiply-adds, then Taylor polynomials on [-pi/4, pi/4].  Absolute
// error about 6e-8 up to x = 700.  SIGNBITS: the quadrant's sign flips as
// xors of the sign bit (fewer instructions; the back pass keeps the selects,
// with which its register allocation does not spill).
template <bool SIGNBITS = false>
__device__ __forceinline__ void sincos_f32(float x, float& sn, float& cs) {
  const float n = __builtin_rintf(x * 0.636619746685f);
  float r = __builtin_fmaf(-n, 1.57079637050628662f, x);
  r = __builtin_fmaf(-n, -4.37113882867379e-08f, r);
  r = __builtin_fmaf(-n, -1.77635683940025e-15f, r);
  const float r2 = r * r;
  float ps = __builtin_fmaf(r2, 2.75573188446e-06f, -1.98412701138e-04f);
  ps = __builtin_fmaf(r2, ps, 8.33333376795e-03f);
  ps = __builtin_fmaf(r2, ps, -0.166666671634f);
  const float s = __builtin_fmaf(r * r2, ps, r);  // sin r
  float pc = __builtin_fmaf(r2, -2.75573199815e-07f, 2.48015876423e-05f);
  pc = __builtin_fmaf(r2, pc, -1.38888892252e-03f);
  pc = __builtin_fmaf(r2, pc, 4.16666679084e-02f);
  pc = __builtin_fmaf(r2, pc, -0.5f);
  const float c = __builtin_fmaf(r2, pc, 1.0f);  // cos r
  if constexpr (SIGNBITS) {
    // odd q swaps sine and cosine; the sine's sign flips for q = 2, 3 and
    // the cosine's for q = 1, 2
    const uint32_t q = (uint32_t)(int)n;
    const bool odd = (q & 1u) != 0u;
    const float a = odd ? c : s, b = odd ? s : c;
    sn = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, a) ^ ((q & 2u) << 30));
    cs = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, b) ^ (((q + 1u) & 2u) << 30));
  } else {
    const int q = (int)n & 3;
    sn = q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
    cs = q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
  }
}

// Hard-sphere weights at |k| = k for radius R, in FP32 registers:
// j0(kR), 4 pi R^3 j1(kR)/(kR) (ball) and 4 pi R^2 j1(kR) (shell magnitude).
// j1(x)/x switches to its Taylor series below x = 1, where the closed form
// loses digits to cancellation.
template <bool SIGNBITS = false>
__device__ __forceinline__ void hs_weights_f32(float k, float R, float& j0, float& w3, float& v2) {
  const float x = k * R;
  float sn, cs;
  sincos_f32<SIGNBITS>(x, sn, cs);
  const float x2 = x * x;
  // j1(x)/x = 1/3 - x^2/30 + x^4/840 - x^6/45360 + x^8/3991680 - x^10/518918400 + ...
  const float ser =
      0.333333333333f -
      x2 * (3.33333333333e-2f - x2 * (1.19047619048e-3f - x2 * (2.20458553792e-5f - x2 * (2.50521083854e-7f -
                                                                                           x2 * 1.92708526042e-9f))));
  const float rx = __builtin_amdgcn_rcpf(x);  // 1 ulp; inf at x = 0, where both uses take their series
  const float j1x = x < 1.0f ? ser : (sn - x * cs) * rx * rx * rx;
  j0 = x < 1e-3f ? 1.0f - x2 * 0.166666667f : sn * rx;
  const float a2 = 12.5663706144f * R * R;
  w3 = a2 * R * j1x;
  v2 = a2 * x * j1x;
}

// Weights of species i at the integer class m = |j|^2: computed in registers
// for FP32, gathered from the FP64 table otherwise.
template <typename T, bool SIGNBITS = false>
__device__ __forceinline__ void hs_weights(const EvalArgs& a, const Buf& hs, int S, int i, int m, T& j0, T& w3,
                                           T& v2) {
  if constexpr (sizeof(T) == 4) {
    hs_weights_f32<SIGNBITS>((float)a.kscale * __builtin_sqrtf((float)m), (float)a.R[i], j0, w3, v2);
  } else {
    const v4<T> w = hs.template ld<v4<T>>((uint32_t)(m * S + i) * (uint32_t)sizeof(v4<T>));
    j0 = w.x;
    w3 = w.y;
    v2 = w.z;
  }
}

// FP32 weights of a thread's EX elements of one x pencil (element e at
// kx = t + TX e), shared with the mirror thread.  |k| depends on kx only
// through |sx|, and element e >= EX/2 of thread t has the |sx| of element
// EX-1-e of thread TX-t (of element EX-e of thread 0 when t = 0; element
// EX/2 of thread 0, the column kx = N/2, is its own mirror).  Each thread
// evaluates its first EX/2 elements (thread 0 also element EX/2), leaves them
// in LDS slot [e][t][p] of `buf`, and after a workgroup barrier reads the
// rest from its mirror's slots.  Callers alternate between two buffers, so
// one barrier per call suffices (a thread writes a buffer again only after
// the barrier of the call in between).
struct WTrip {
  float j0, w3, v2;
};

template <int N, int EX, int TX, int PX>
__device__ __forceinline__ void x_weights_shared(float kscale, float R, const int* mm, int t, int p, WTrip* buf,
                                                 float* j0, float* w3, float* v2) {
  constexpr int EH = EX / 2;
  static_assert(EX % 2 == 0 && TX * EX == N, "mirror map");
#pragma unroll
  for (int e = 0; e < EH; ++e) {
    WTrip w;
    hs_weights_f32<true>(kscale * __builtin_sqrtf((float)mm[e]), R, w.j0, w.w3, w.v2);
    buf[(e * TX + t) * PX + p] = w;
  }
  WTrip ny{0.0f, 0.0f, 0.0f};
  if (t == 0) hs_weights_f32<true>(kscale * __builtin_sqrtf((float)mm[EH]), R, ny.j0, ny.w3, ny.v2);
  __syncthreads();
  const int tm = t == 0 ? 0 : TX - t;
#pragma unroll
  for (int e = 0; e < EX; ++e) {
    WTrip w;
    if (e < EH) {
      w = buf[(e * TX + t) * PX + p];
    } else {
      const int em = t == 0 ? (e == EH ? 0 : EX - e) : EX - 1 - e;
      w = buf[(em * TX + tm) * PX + p];
      if (e == EH && t == 0) w = ny;
    }
    j0[e] = w.j0;
    w3[e] = w.w3;
    v2[e] = w.v2;
  }
}

// signed index of a wavenumber along one axis, 0 on the Nyquist plane
template <typename T, int N>
__device__ __forceinline__ T s_axis(int k) {
  return k == N / 2 ? (T)0 : (T)sgn_idx(k, N);
}

// unit-vector component c of k at element kx of a pencil (0 on that axis's
// Nyquist plane)
template <typename T, int N>
__device__ __forceinline__ T khat(int c, int kx, int ky, int kz, int m) {
  const T r = inv_sqrt_m<T>(m);
  if (c == 0) return kx == N / 2 ? (T)0 : (T)sgn_idx(kx, N) * r;
  if (c == 1) return ky == N / 2 ? (T)0 : (T)sgn_idx(ky, N) * r;
  return kz == N / 2 ? (T)0 : (T)kz * r;
}

// field slot of the q-th field the back pass reads (0..3, [x]1, [z]1, [x]2, [z]2)
__device__ __forceinline__ constexpr int back_field(int q) {
  return q < 4 ? q : kSlotX + (q - 4) / 2 * kVecStride + ((q - 4) % 2) * (kSlotZ - kSlotX);
}

// Per-lane addressing of an x tile: element m of the lane's pencil sits at
// byte vo + m * mstride (+ the field offset).  Both strides are uniform over
// the block, which keeps them in scalar registers.
template <typename T, int N, int EX, int PX>
struct XAddr {
  uint32_t vo, mstride;
  __device__ __forceinline__ XAddr(const XPencil<T, N, PX>& pc, int t) {
    constexpr int TX = N / EX;
    vo = (pc.off + (uint32_t)t * pc.es) * (uint32_t)sizeof(cx<T>);
    mstride = __builtin_amdgcn_readfirstlane((uint32_t)TX * pc.es * (uint32_t)sizeof(cx<T>));
  }
};

// The x passes exchange through two LDS buffers in turn (LdsPencil2): one
// workgroup barrier per FFT stage instead of two (measured at 256^3: x
// forward 257 -> 241 us, back pass 353 -> 332 us).
//
// P3: forward weights.  For every k: n^_a(k) = sum_i rho^_i(k) conj(w^_i^a(k))
// (correlation, Sec. 2.3.1); scalars w0 = j0, w1 = R j0, w2 = 4 pi R^2 j0,
// w3 = 4 pi R^3 j1(kR)/(kR); vectors conj(-i khat V) = +i khat V with
// V2 = 4 pi R^2 j1(kR), V1 = V2 / (4 pi R).
// The species pencils stream through two register buffers: the loads of
// species i + 1 are in flight while species i is transformed.
template <typename T, int N, int EX = Geo<T, N>::EX, int PX = Geo<T, N>::PX>
__global__ void __launch_bounds__((PX * (N / EX)))
    k_xfwd(const EvalArgs* __restrict__ args, int part) {
  constexpr int TX = N / EX;
  __shared__ cx<T> tw[N];
  __shared__ cx<T> xch[2 * PX * N];
  // FP32 weights.  With at most three species: every species' weights for
  // the first half of each thread's elements (and the column kx = N/2 of
  // thread 0), evaluated while the first pencil loads are in flight; an
  // element's other half is its mirror's.  With more species the first two
  // regions serve as the two buffers of x_weights_shared, one species at a
  // time.
  constexpr int EH = EX / 2;
  constexpr int kRegion = EH * TX * PX;
  __shared__ WTrip wall[sizeof(T) == 4 ? 3 * kRegion + 3 * PX : 1];
  int tile;
  const EvalArgs& a = args[inst_of_part((N * (N / 2)) / PX, N / PX, part, tile)];
  if (!a.hs_on) return;  // uniform per block
  const int p = threadIdx.x % PX, t = threadIdx.x / PX;
  const XPencil<T, N, PX> pc(tile, p);
  const LdsPencil2<T> lp{xch + p, xch + PX * N + p, PX};
  const int S = a.S;
  const Buf hs = make_buf(a.hs_tab, sizeof(T) == 8 ? table_m<T, N>(0) * S * sizeof(v4<T>) : 0);
  const BufN<N> A = make_buf<stream_policy<N>()>(a.specA, spec_bytes<T>(a, S));
  const BufN<N> B = make_buf<stream_policy<N>()>(a.specB, spec_bytes<T>(a, kFields));
  const uint32_t fbytes = __builtin_amdgcn_readfirstlane((uint32_t)(a.fstride * sizeof(cx<T>)));
  const XAddr<T, N, EX, PX> xa(pc, t);
  int mm[EX];
  {
    const int sy = sgn_idx(pc.ky, N), sz = pc.kz;
#pragma unroll
    for (int m = 0; m < EX; ++m) {
      const int sx = sgn_idx(t + TX * m, N);
      mm[m] = sx * sx + sy * sy + sz * sz;
    }
  }
  cx<T> acc[6][EX];
  cx<T> b0[EX], b1[EX];
  // the first species' pencil is in flight while the twiddle table is built
#pragma unroll
  for (int m = 0; m < EX; ++m) b0[m] = A.template ld<cx<T>>(xa.vo, m * xa.mstride);
  const bool pre = sizeof(T) == 4 && S <= 3;  // uniform
  if constexpr (sizeof(T) == 4) {
    if (pre) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (c < S) {
          const float R = (float)a.R[c];
#pragma unroll
          for (int e = 0; e < EH; ++e) {
            WTrip w;
            hs_weights_f32<true>((float)a.kscale * __builtin_sqrtf((float)mm[e]), R, w.j0, w.w3, w.v2);
            wall[c * kRegion + (e * TX + t) * PX + p] = w;
          }
          if (t == 0) {
            WTrip w;
            hs_weights_f32<true>((float)a.kscale * __builtin_sqrtf((float)mm[EH]), R, w.j0, w.w3, w.v2);
            wall[3 * kRegion + c * PX + p] = w;
          }
        }
      }
    }
  }
  init_twiddles<T, N>(tw);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kMaxSpecies; ++i) {
    if (i < S) {  // uniform
      cx<T>* cur = (i & 1) ? b1 : b0;
      cx<T>* nxt = (i & 1) ? b0 : b1;
      if (i + 1 < S) {
#pragma unroll
        for (int m = 0; m < EX; ++m) nxt[m] = A.template ld<cx<T>>(xa.vo, (uint32_t)(i + 1) * fbytes + m * xa.mstride);
      }
      fft_pencil<T, N, EX, true>(cur, t, tw, lp);
      const T R = (T)a.R[i], ar = (T)a.area[i], i4 = (T)a.inv4piR[i];
      float sj0[EX], ss3[EX], svv[EX];
      if constexpr (sizeof(T) == 4) {
        if (i < 3 && pre) {
          // own slot, the mirror's slot, or thread 0's column kx = N/2
          const int tm = t == 0 ? 0 : TX - t;
#pragma unroll
          for (int m = 0; m < EX; ++m) {
            const int em = t == 0 ? EX - m : EX - 1 - m;
            const int idx = m < EH ? i * kRegion + (m * TX + t) * PX + p
                            : (t == 0 && m == EH) ? 3 * kRegion + i * PX + p
                                                  : i * kRegion + (em * TX + tm) * PX + p;
            const WTrip w = wall[idx];
            sj0[m] = w.j0; ss3[m] = w.w3; svv[m] = w.v2;
          }
        } else {
          x_weights_shared<N, EX, TX, PX>((float)a.kscale, (float)a.R[i], mm, t, p, wall + (i & 1) * kRegion, sj0,
                                          ss3, svv);
        }
      }
#pragma unroll
      for (int m = 0; m < EX; ++m) {
        T j0, s3, vv;
        if constexpr (sizeof(T) == 4) {
          j0 = sj0[m]; s3 = ss3[m]; vv = svv[m];
        } else {
          hs_weights<T>(a, hs, S, i, mm[m], j0, s3, vv);
        }
        if (i == 0) {
          acc[0][m] = cscale<T>(cur[m], j0);
          acc[1][m] = cscale<T>(cur[m], j0 * R);
          acc[2][m] = cscale<T>(cur[m], j0 * ar);
          acc[3][m] = cscale<T>(cur[m], s3);
          acc[4][m] = cscale<T>(cur[m], vv * i4);
          acc[5][m] = cscale<T>(cur[m], vv);
        } else {
          cfma<T>(acc[0][m], cur[m], j0);
          cfma<T>(acc[1][m], cur[m], j0 * R);
          cfma<T>(acc[2][m], cur[m], j0 * ar);
          cfma<T>(acc[3][m], cur[m], s3);
          cfma<T>(acc[4][m], cur[m], vv * i4);
          cfma<T>(acc[5][m], cur[m], vv);
        }
      }
    }
  }
  const T sc = (T)a.inv_n3;
  // scalar weighted densities n0..n3
#pragma unroll
  for (int o = 0; o < 4; ++o) {
    cx<T> v[EX];
#pragma unroll
    for (int m = 0; m < EX; ++m) v[m] = cscale<T>(acc[o][m], sc);
    fft_pencil<T, N, EX, false>(v, t, tw, lp);
#pragma unroll
    for (int m = 0; m < EX; ++m) B.template st<cx<T>>(v[m], xa.vo, (uint32_t)o * fbytes + m * xa.mstride);
  }
  // vector weighted densities n_bv,c = +i khat_c A_b (A_1 = sum rho V1, A_2 =
  // sum rho V2): stored as [x] = i s_x Q_b and [z] = Q_b with Q_b = A_b / |j|
  // (the y and z components are formed by the y and z passes)
#pragma unroll
  for (int b = 0; b < 2; ++b) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      cx<T> v[EX];
#pragma unroll
      for (int m = 0; m < EX; ++m) {
        const cx<T> q = cscale<T>(acc[4 + b][m], inv_sqrt_m<T>(mm[m]) * sc);
        v[m] = c == 0 ? cmuli<T>(cscale<T>(q, s_axis<T, N>(t + TX * m))) : q;
      }
      fft_pencil<T, N, EX, false>(v, t, tw, lp);
      const int slot = (c == 0 ? kSlotX : kSlotZ) + kVecStride * b;
#pragma unroll
      for (int m = 0; m < EX; ++m) B.template st<cx<T>>(v[m], xa.vo, (uint32_t)slot * fbytes + m * xa.mstride);
    }
  }
}

// P7: back-convolution (Sec. 2.3.1, convolution orientation: no conjugate)
// plus the pair kernels of Sec. 2.3.2 / 2.3.4:
//   mu^_i = j0_i (F0 + R_i F1 + 4 pi R_i^2 F2) + w3_i F3
//           - i V2_i (D1 / (4 pi R_i) + D2) + sum_j G_ij rho^_j,
// with F_a the derivative spectra and D_b = khat . (vector derivative b).
// For S <= CH <= 4: the ten derivative pencils and then the S density pencils
// stream through two register buffers (the next pencil, and the next pair-
// table row, are in flight during each transform); the derivative spectra
// fold into the CH outputs before the density phase starts.
// Instances with more species than CH belong to the chunked kernel of the
// same launch list and are skipped here.
template <typename T, int N, int CH, int EX = Geo<T, N>::EX, int PX = Geo<T, N>::PX>
__global__ void __launch_bounds__((PX * (N / EX)))
    k_xback(const EvalArgs* __restrict__ args, int part) {
  static_assert(CH >= 1 && CH <= 4, "output chunk");
  constexpr int TX = N / EX;
  __shared__ cx<T> tw[N];
  __shared__ cx<T> xch[2 * PX * N];
  int tile;
  const EvalArgs& a = args[inst_of_part((N * (N / 2)) / PX, N / PX, part, tile)];
  // FP32 with at most three outputs: the weights of every output species for
  // the first half of each thread's elements (and the column kx = N/2 of
  // thread 0), evaluated while the first pencil loads are in flight; an
  // element's other half is its mirror's (see x_weights_shared)
  constexpr bool kPre = sizeof(T) == 4 && CH <= 3;
  constexpr int EH = EX / 2;
  __shared__ WTrip wpre[kPre ? CH * EH * TX * PX + CH * PX : 1];
  if (a.S > CH) return;  // uniform per block
  const int p = threadIdx.x % PX, t = threadIdx.x / PX;
  const XPencil<T, N, PX> pc(tile, p);
  const LdsPencil2<T> lp{xch + p, xch + PX * N + p, PX};
  const int S = a.S;
  const bool hs_on = a.hs_on, pair_on = a.pair_on;
  const Buf hs = make_buf(a.hs_tab, sizeof(T) == 8 ? table_m<T, N>(0) * S * sizeof(v4<T>) : 0);
  const Buf pt = make_buf(a.pair_tab, pair_on ? table_m<T, N>(0) * S * a.Sp * sizeof(T) : 0);
  const BufN<N> A = make_buf<stream_policy<N>()>(a.specA, spec_bytes<T>(a, S));
  const BufN<N> B = make_buf<stream_policy<N>()>(a.specB, hs_on ? spec_bytes<T>(a, kFields) : 0);
  const BufN<N> C = make_buf<stream_policy<N>()>(a.specC, spec_bytes<T>(a, S));
  const uint32_t fbytes = __builtin_amdgcn_readfirstlane((uint32_t)(a.fstride * sizeof(cx<T>)));
  const XAddr<T, N, EX, PX> xa(pc, t);
  int mm[EX];
  {
    const int sy = sgn_idx(pc.ky, N), sz = pc.kz;
#pragma unroll
    for (int m = 0; m < EX; ++m) {
      const int sx = sgn_idx(t + TX * m, N);
      mm[m] = sx * sx + sy * sy + sz * sz;
    }
  }
  cx<T> out[CH][EX];
  cx<T> b0[EX], b1[EX];
  // the first pencil of the stream is in flight while the twiddle table is built
  if (hs_on) {
#pragma unroll
    for (int m = 0; m < EX; ++m) b0[m] = B.template ldnt<cx<T>>(xa.vo, m * xa.mstride);
  } else if (pair_on) {
#pragma unroll
    for (int m = 0; m < EX; ++m) b0[m] = A.template ldnt<cx<T>>(xa.vo, m * xa.mstride);
  }
  if constexpr (kPre) {
    if (hs_on) {
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const float R = (float)a.R[c < S ? c : 0];
#pragma unroll
        for (int e = 0; e < EH; ++e) {
          WTrip w;
          hs_weights_f32<true>((float)a.kscale * __builtin_sqrtf((float)mm[e]), R, w.j0, w.w3, w.v2);
          wpre[((c * EH + e) * TX + t) * PX + p] = w;
        }
        if (t == 0) {
          WTrip w;
          hs_weights_f32<true>((float)a.kscale * __builtin_sqrtf((float)mm[EH]), R, w.j0, w.w3, w.v2);
          wpre[CH * EH * TX * PX + c * PX + p] = w;
        }
      }
    }
  }
  init_twiddles<T, N>(tw);
  __syncthreads();
  if (hs_on) {
    // F[0..3]: scalar derivative spectra; F[4 + b] = i (khat . F_bv) =
    // (i s_x F_bx + [z]) / |j| (see the field-slot layout)
    cx<T> F[6][EX];
#pragma unroll
    for (int q = 0; q < kBackFields; ++q) {
      cx<T>* cur = (q & 1) ? b1 : b0;
      cx<T>* nxt = (q & 1) ? b0 : b1;
      if (q + 1 < kBackFields) {
        const int f1 = back_field(q + 1);
#pragma unroll
        for (int m = 0; m < EX; ++m) nxt[m] = B.template ldnt<cx<T>>(xa.vo, (uint32_t)f1 * fbytes + m * xa.mstride);
      } else if (pair_on) {
        // the first density pencil is in flight during the last transform and the fold
#pragma unroll
        for (int m = 0; m < EX; ++m) nxt[m] = A.template ldnt<cx<T>>(xa.vo, m * xa.mstride);
      }
      fft_pencil<T, N, EX, true>(cur, t, tw, lp);
      const int f = back_field(q);
      if (f < 4) {
#pragma unroll
        for (int m = 0; m < EX; ++m) F[f][m] = cur[m];
      } else {
        const int b = (f - kSlotX) / kVecStride;
        const bool xs = (f - kSlotX) % kVecStride == 0;
#pragma unroll
        for (int m = 0; m < EX; ++m) {
          const T r = inv_sqrt_m<T>(mm[m]);
          if (xs) F[4 + b][m] = cscale<T>(cmuli<T>(cur[m]), s_axis<T, N>(t + TX * m) * r);
          else cfma<T>(F[4 + b][m], cur[m], r);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int i = c < S ? c : 0;
      const T R = (T)a.R[i], ar = (T)a.area[i], i4 = (T)a.inv4piR[i];
#pragma unroll
      for (int m = 0; m < EX; ++m) {
        T j0, w3, v2;
        if constexpr (kPre) {
          // own slot, the mirror's slot, or thread 0's column kx = N/2
          const int tm = t == 0 ? 0 : TX - t;
          const int em = t == 0 ? EX - m : EX - 1 - m;
          const int idx = m < EH ? ((c * EH + m) * TX + t) * PX + p
                          : (t == 0 && m == EH) ? CH * EH * TX * PX + c * PX + p
                                                : ((c * EH + em) * TX + tm) * PX + p;
          const WTrip w = wpre[idx];
          j0 = w.j0; w3 = w.w3; v2 = w.v2;
        } else {
          hs_weights<T>(a, hs, S, i, mm[m], j0, w3, v2);
        }
        cx<T> s0 = F[0][m];
        cfma<T>(s0, F[1][m], R);
        cfma<T>(s0, F[2][m], ar);
        cx<T> u = cscale<T>(s0, j0);
        cfma<T>(u, F[3][m], w3);
        // -i V2 (D1 / (4 pi R) + D2) with F[4 + b] = i D_b
        cx<T> dv = F[5][m];
        cfma<T>(dv, F[4][m], i4);
        cfma<T>(u, dv, -v2);
        out[c][m] = u;
      }
      // one species at a time: hoisting the weights of later species ahead
      // (they do not depend on F) would keep them live beside F and spill
      __builtin_amdgcn_sched_barrier(0);
    }
  } else {
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
      for (int m = 0; m < EX; ++m) out[c][m] = mk<T>((T)0, (T)0);
  }
  // the density stream starts in b0: without HS it was loaded at the start;
  // with HS after the last of the (even number of) derivative fields, into
  // the buffer that field left free
  static_assert(kBackFields % 2 == 0, "the density stream continues in b0");
  if (pair_on && sizeof(T) == 8) {
    // FP64: pair-table rows gathered after each transform (two buffers of
    // double rows would not fit the register budget)
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      if (j < S) {  // uniform
        cx<T>* cur = (j & 1) ? b1 : b0;
        cx<T>* nxt = (j & 1) ? b0 : b1;
        if (j + 1 < S) {
#pragma unroll
          for (int m = 0; m < EX; ++m) nxt[m] = A.template ldnt<cx<T>>(xa.vo, (uint32_t)(j + 1) * fbytes + m * xa.mstride);
        }
        fft_pencil<T, N, EX, true>(cur, t, tw, lp);
#pragma unroll
        for (int m = 0; m < EX; ++m) {
          const v4<T> g = pt.template ld<v4<T>>((uint32_t)((mm[m] * S + j) * a.Sp) * (uint32_t)sizeof(T));
          cfma<T>(out[0][m], cur[m], g.x);
          if constexpr (CH > 1) cfma<T>(out[1][m], cur[m], g.y);
          if constexpr (CH > 2) cfma<T>(out[2][m], cur[m], g.z);
          if constexpr (CH > 3) cfma<T>(out[3][m], cur[m], g.w);
        }
      }
    }
  } else if (pair_on) {
    // G_{0..3, j} of row [m][j][.]: one gather per element, issued before the
    // transform of the same species' pencil (its latency hides behind it)
    v4<T> g[EX];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      if (j < S) {  // uniform
        cx<T>* cur = (j & 1) ? b1 : b0;
        cx<T>* nxt = (j & 1) ? b0 : b1;
        if (j + 1 < S) {
#pragma unroll
          for (int m = 0; m < EX; ++m) nxt[m] = A.template ldnt<cx<T>>(xa.vo, (uint32_t)(j + 1) * fbytes + m * xa.mstride);
        }
#pragma unroll
        for (int m = 0; m < EX; ++m) g[m] = pt.template ld<v4<T>>((uint32_t)((mm[m] * S + j) * a.Sp) * (uint32_t)sizeof(T));
        fft_pencil<T, N, EX, true>(cur, t, tw, lp);
#pragma unroll
        for (int m = 0; m < EX; ++m) {
          cfma<T>(out[0][m], cur[m], g[m].x);
          if constexpr (CH > 1) cfma<T>(out[1][m], cur[m], g[m].y);
          if constexpr (CH > 2) cfma<T>(out[2][m], cur[m], g[m].z);
          if constexpr (CH > 3) cfma<T>(out[3][m], cur[m], g[m].w);
        }
      }
    }
  }
  const T sc = (T)a.inv_n3;
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    if (c < S) {  // uniform
      cx<T> v[EX];
#pragma unroll
      for (int m = 0; m < EX; ++m) v[m] = cscale<T>(out[c][m], sc);
      fft_pencil<T, N, EX, false>(v, t, tw, lp);
#pragma unroll
      for (int m = 0; m < EX; ++m) C.template st<cx<T>>(v[m], xa.vo, (uint32_t)c * fbytes + m * xa.mstride);
    }
  }
}

// P7 for S > 4 species: the same operator with the outputs in chunks of 4
// (the derivative spectra stay in registers; each chunk re-streams the
// density pencils).
// min_s: instances with fewer species run the streamed kernel of the same
// launch list and are skipped here (1: every instance runs here).
template <typename T, int N, int CH, int EX = Geo<T, N>::EX, int PX = Geo<T, N>::PX>
__global__ void __launch_bounds__((PX * (N / EX)))
    k_xback_chunked(const EvalArgs* __restrict__ args, int min_s, int part) {
  static_assert(CH >= 1 && CH <= 4, "output chunk");
  constexpr int TX = N / EX;
  __shared__ cx<T> tw[N];
  __shared__ cx<T> xch[2 * PX * N];
  int tile;
  const EvalArgs& a = args[inst_of_part((N * (N / 2)) / PX, N / PX, part, tile)];
  if (a.S < min_s) return;  // uniform per block
  init_twiddles<T, N>(tw);
  __syncthreads();
  const int p = threadIdx.x % PX, t = threadIdx.x / PX;
  const XPencil<T, N, PX> pc(tile, p);
  const LdsPencil2<T> lp{xch + p, xch + PX * N + p, PX};
  const int S = a.S;
  const Buf hs = make_buf(a.hs_tab, sizeof(T) == 8 ? table_m<T, N>(0) * S * sizeof(v4<T>) : 0);
  const Buf pt = make_buf(a.pair_tab, a.pair_on ? table_m<T, N>(0) * S * a.Sp * sizeof(T) : 0);
  const BufN<N> A = make_buf<stream_policy<N>()>(a.specA, spec_bytes<T>(a, S));
  const BufN<N> B = make_buf<stream_policy<N>()>(a.specB, a.hs_on ? spec_bytes<T>(a, kFields) : 0);
  const BufN<N> C = make_buf<stream_policy<N>()>(a.specC, spec_bytes<T>(a, S));
  const uint32_t fbytes = (uint32_t)(a.fstride * sizeof(cx<T>));
  const XKs<T, N, EX, TX> ks(t, pc.ky, pc.kz);
  uint32_t eo[EX];
#pragma unroll
  for (int m = 0; m < EX; ++m) eo[m] = (pc.off + (uint32_t)(t + TX * m) * pc.es) * (uint32_t)sizeof(cx<T>);
  cx<T> F[6][EX];
#pragma unroll
  for (int q = 0; q < 6; ++q)
#pragma unroll
    for (int m = 0; m < EX; ++m) F[q][m] = mk<T>((T)0, (T)0);
  if (a.hs_on) {
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      cx<T> v[EX];
#pragma unroll
      for (int m = 0; m < EX; ++m) v[m] = B.template ldnt<cx<T>>(eo[m], (uint32_t)f * fbytes);
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
    // F[4 + b] = i (khat . F_bv) = (i s_x F_bx + [z]) / |j| (field-slot layout)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        cx<T> v[EX];
        const int slot = (c == 0 ? kSlotX : kSlotZ) + kVecStride * b;
#pragma unroll
        for (int m = 0; m < EX; ++m) v[m] = B.template ldnt<cx<T>>(eo[m], (uint32_t)slot * fbytes);
        fft_pencil<T, N, EX, true>(v, t, tw, lp);
#pragma unroll
        for (int m = 0; m < EX; ++m) {
          const T r = inv_sqrt_m<T>(ks.mm[m]);
          if (c == 0) cfma<T>(F[4 + b][m], cmuli<T>(v[m]), s_axis<T, N>(t + TX * m) * r);
          else cfma<T>(F[4 + b][m], v[m], r);
        }
      }
    }
  }
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
        cx<T> v[EX];
#pragma unroll
        for (int m = 0; m < EX; ++m) v[m] = A.template ldnt<cx<T>>(eo[m], (uint32_t)j * fbytes);
        fft_pencil<T, N, EX, true>(v, t, tw, lp);
#pragma unroll
        for (int m = 0; m < EX; ++m) {
          // G_{i0..i0+3, j} in one gather: row [m][j][.] of the pair table
          const v4<T> g = pt.template ld<v4<T>>((uint32_t)((ks.mm[m] * S + j) * a.Sp + i0) * (uint32_t)sizeof(T));
          cfma<T>(out[0][m], v[m], g.x);
          if constexpr (CH > 1) cfma<T>(out[1][m], v[m], g.y);
          if constexpr (CH > 2) cfma<T>(out[2][m], v[m], g.z);
          if constexpr (CH > 3) cfma<T>(out[3][m], v[m], g.w);
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
            T j0, w3, v2;
            hs_weights<T>(a, hs, S, i, ks.mm[m], j0, w3, v2);
            cx<T> sc0 = F[0][m];
            cfma<T>(sc0, F[1][m], R);
            cfma<T>(sc0, F[2][m], ar);
            cfma<T>(u, sc0, j0);
            cfma<T>(u, F[3][m], w3);
            // -i V2 (D1 / (4 pi R) + D2) with F[4 + b] = i D_b
            cx<T> dv = F[5][m];
            cfma<T>(dv, F[4][m], i4);
            cfma<T>(u, dv, -v2);
          }
          v[m] = cscale<T>(u, sc);
        }
        fft_pencil<T, N, EX, false>(v, t, tw, lp);
#pragma unroll
        for (int m = 0; m < EX; ++m) C.template st<cx<T>>(v[m], eo[m], (uint32_t)i * fbytes);
      }
    }
  }
}

// plain x-direction c2c on `nf` fields of `sel` (used by the FFT test hook)
template <typename T, int N, bool FWD, int EX = Geo<T, N>::EX, int PX = Geo<T, N>::PX>
__global__ void __launch_bounds__((PX * (N / EX)))
    k_xplain(const EvalArgs* __restrict__ args, int sel, int nf) {
  constexpr int TX = N / EX;
  __shared__ cx<T> tw[N];
  __shared__ cx<T> xch[PX * N];
  int tile;
  const EvalArgs& a = args[inst_of(x_tiles<N, PX>(), tile)];
  init_twiddles<T, N>(tw);
  __syncthreads();
  const int p = threadIdx.x % PX, t = threadIdx.x / PX;
  const XPencil<T, N, PX> pc(tile, p);
  const LdsPencil<T> lp{xch + p, PX};
  const BufN<N> base = make_buf<stream_policy<N>()>(sel == 0 ? a.specA : sel == 1 ? a.specB : a.specC, spec_bytes<T>(a, nf));
  const uint32_t fbytes = (uint32_t)(a.fstride * sizeof(cx<T>));
  uint32_t eo[EX];
#pragma unroll
  for (int m = 0; m < EX; ++m) eo[m] = (pc.off + (uint32_t)(t + TX * m) * pc.es) * (uint32_t)sizeof(cx<T>);
  for (int f = 0; f < nf; ++f) {
    cx<T> v[EX];
#pragma unroll
    for (int m = 0; m < EX; ++m) v[m] = base.template ld<cx<T>>(eo[m], (uint32_t)f * fbytes);
    fft_pencil<T, N, EX, FWD>(v, t, tw, lp);
#pragma unroll
    for (int m = 0; m < EX; ++m) base.template st<cx<T>>(v[m], eo[m], (uint32_t)f * fbytes);
  }
}

// numpy rfftn layout <-> spectral storage (test hook only)
template <typename T, int N>
__global__ void k_export(const EvalArgs* __restrict__ args, int nf, double* buf, int to_numpy) {
  constexpr int H = N / 2;
  const EvalArgs& a = args[0];
  const long total = (long)nf * N * N * (H + 1);
  const gp<cx<T>> A = gbl((cx<T>*)a.specA);
  const gp<double> bb = gbl(buf);
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long f = e / ((long)N * N * (H + 1));
    const long rem = e % ((long)N * N * (H + 1));
    const long kx = rem / ((long)N * (H + 1));
    const long ky = (rem / (H + 1)) % N;
    const long kz = rem % (H + 1);
    const gp<cx<T>> s =
        A + f * a.fstride + (kz < H ? kx * spec_plane(N, sizeof(T)) + ky * H + kz : (long)spec_nyq<T, N>() + kx * N + ky);
    if (to_numpy) {
      bb[2 * e] = (double)s->x;
      bb[2 * e + 1] = (double)s->y;
    } else {
      *s = mk<T>((T)bb[2 * e], (T)bb[2 * e + 1]);
    }
  }
}

}  // namespace pnp
