// One translation unit of launch tables: the pass kernels of one precision
// (PNP_OPS_T: float or double), grid size (PNP_OPS_N) and FFT schedule
// (PNP_OPS_SCHED), in both tile shapes where the narrow one exists.  The
// build compiles this file once per (precision, size, schedule).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pnp_kernels.hip"
#include "pnp_launch.hpp"

#ifndef PNP_OPS_T
#error "PNP_OPS_T (float or double) must be defined"
#endif
#ifndef PNP_OPS_N
#error "PNP_OPS_N (grid size) must be defined"
#endif
#ifndef PNP_OPS_SCHED
#error "PNP_OPS_SCHED (0 primary or 1 secondary FFT schedule) must be defined"
#endif

namespace pnp {

template <typename T, int N, int V = 0> struct Launch {
  using G = Geo<T, N, V>;
  static constexpr int EZD = ezd_of<T, N, V>();
  using GD = GeoD<T, N, EZD, V>;
  // maxS: the largest species count among the launch's instances
  static void tables(const TableArgs* a, int count, int M, int maxS, hipStream_t s) {
    const int items = maxS * ((maxS + 3) / 4 * 4) + maxS;  // pair-table entries + hs species
    hipLaunchKernelGGL(k_tables<T>, dim3((M + 255) / 256, items, count), dim3(256), 0, s, a);
  }
  static void zfwd(const EvalArgs* a, int count, hipStream_t s) {
    hipLaunchKernelGGL((k_zfwd<T, N, V>), dim3(count * G::tiles_z), dim3(G::RZ * G::TZ), 0, s, a);
  }
  // part: kPartAll, kPartMain (main-array tiles) or kPartNyquist (Nyquist-plane tiles)
  static int tiles_y(int part) { return part == kPartAll ? G::tiles_y : part == kPartMain ? (N * G::H) / G::PY : N / G::PY; }
  static int tiles_x(int part) { return part == kPartAll ? G::tiles_x : part == kPartMain ? (N * G::H) / G::PX : N / G::PX; }
  static void ystep(const EvalArgs* a, int count, int sel, int nf, bool fwd, int part, hipStream_t s) {
    const dim3 g(count * tiles_y(part)), b(G::PY * G::TY);
    if (fwd)
      hipLaunchKernelGGL((k_ystep<T, N, true, V>), g, b, 0, s, a, sel, nf, part);
    else
      hipLaunchKernelGGL((k_ystep<T, N, false, V>), g, b, 0, s, a, sel, nf, part);
  }
  static void xfwd(const EvalArgs* a, int count, int part, hipStream_t s) {
    hipLaunchKernelGGL((k_xfwd<T, N, G::EX, G::PX>), dim3(count * tiles_x(part)), dim3(G::PX * G::TX), 0, s, a,
                       part);
  }
  // phi: also sum Phi_hs per workgroup (free-energy calls); fmask: the
  // hard-sphere functionals among the instances (1 Rosenfeld, 2 White Bear),
  // one launch of the matching variant each
  static void zderiv(const EvalArgs* a, int count, bool phi, int fmask, hipStream_t s) {
    const dim3 g(count * GD::tiles), b(GD::RDD * GD::TZD);
    if (fmask & 1) {
      if (phi) hipLaunchKernelGGL((k_zderiv<T, N, true, false, EZD, V>), g, b, 0, s, a);
      else hipLaunchKernelGGL((k_zderiv<T, N, false, false, EZD, V>), g, b, 0, s, a);
    }
    if (fmask & 2) {
      if (phi) hipLaunchKernelGGL((k_zderiv<T, N, true, true, EZD, V>), g, b, 0, s, a);
      else hipLaunchKernelGGL((k_zderiv<T, N, false, true, EZD, V>), g, b, 0, s, a);
    }
  }
  // smax: the largest species count among the launch's instances with at
  // most four species (0: none); large: some instance has more than four.
  // The FP32 path runs the streamed kernel for the former and the chunked one
  // for the latter (each skips the other's instances), so an instance gets
  // the arithmetic of its single call in any launch list.
  static void xback(const EvalArgs* a, int count, int smax, bool large, int part, hipStream_t s) {
    const dim3 g(count * tiles_x(part)), b(G::PX * G::TX);
    if constexpr (sizeof(T) == 8) {
      // FP64: the streamed kernel does not fit the register file; the chunked
      // one keeps every spectrum in registers without spilling
      hipLaunchKernelGGL((k_xback_chunked<T, N, 4, G::EX, G::PX>), g, b, 0, s, a, 1, part);
    } else {
      switch (smax) {
        case 1: hipLaunchKernelGGL((k_xback<T, N, 1, G::EX, G::PX>), g, b, 0, s, a, part); break;
        case 2: hipLaunchKernelGGL((k_xback<T, N, 2, G::EX, G::PX>), g, b, 0, s, a, part); break;
        case 3: hipLaunchKernelGGL((k_xback<T, N, 3, G::EX, G::PX>), g, b, 0, s, a, part); break;
        case 4: hipLaunchKernelGGL((k_xback<T, N, 4, G::EX, G::PX>), g, b, 0, s, a, part); break;
        default: break;
      }
      if (large) hipLaunchKernelGGL((k_xback_chunked<T, N, 4, G::EX, G::PX>), g, b, 0, s, a, 5, part);
    }
  }
  static void zinv(const EvalArgs* a, int count, int sel, hipStream_t s) {
    hipLaunchKernelGGL((k_zinv<T, N, V>), dim3(count * G::tiles_z), dim3(G::RZ * G::TZ), 0, s, a, sel);
  }
  static void xplain(const EvalArgs* a, int count, int nf, bool fwd, hipStream_t s) {
    if (fwd)
      hipLaunchKernelGGL((k_xplain<T, N, true, G::EX, G::PX>), dim3(count * G::tiles_x), dim3(G::PX * G::TX), 0, s,
                         a, 0, nf);
    else
      hipLaunchKernelGGL((k_xplain<T, N, false, G::EX, G::PX>), dim3(count * G::tiles_x), dim3(G::PX * G::TX), 0,
                         s, a, 0, nf);
  }
  static void xport(const EvalArgs* a, int nf, double* buf, int to_numpy, hipStream_t s) {
    const long total = (long)nf * N * N * (N / 2 + 1);
    const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL((k_export<T, N>), dim3(blocks), dim3(256), 0, s, a, nf, buf, to_numpy);
  }
  // passes whose secondary schedule differs from the primary one
  using G0 = Geo<T, N, 0>;
  using G2 = Geo<T, N, 2>;
  static constexpr uint32_t sched_alt =
      (G0::EZ != G2::EZ ? (1u << 1) | (1u << 9) : 0u) |
      (G0::EY != G2::EY ? (1u << 2) | (1u << 4) | (1u << 6) | (1u << 8) : 0u) |
      (G0::EX != G2::EX ? (1u << 3) | (1u << 7) : 0u) | (ezd_of<T, N, 0>() != ezd_of<T, N, 2>() ? 1u << 5 : 0u);
  static constexpr Ops ops{tables, zfwd, ystep, xfwd, zderiv, xback, GD::tiles, zinv, xplain, xport, sched_alt};
};

template <typename T, int N, int V> const Ops* ops_inst() { return &Launch<T, N, V>::ops; }

// PNP_OPS_SCHED (0 or 1): the FFT schedule of this translation unit
template const Ops* ops_inst<PNP_OPS_T, PNP_OPS_N, 2 * PNP_OPS_SCHED>();
#if PNP_OPS_N <= 128
template const Ops* ops_inst<PNP_OPS_T, PNP_OPS_N, 2 * PNP_OPS_SCHED + 1>();
#endif

}  // namespace pnp
