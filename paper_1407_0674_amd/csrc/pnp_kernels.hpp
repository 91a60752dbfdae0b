// Shared definitions between the HIP kernels and the host driver of the
// cDFT excess-chemical-potential evaluator.
#pragma once
#include <stdint.h>

namespace pnp {

constexpr int kMaxSpecies = 8;
constexpr int kMaxPairs = kMaxSpecies * (kMaxSpecies + 1) / 2;
constexpr int kFields = 10;  // n0, n1, n2, n3, n1v(x,y,z), n2v(x,y,z)

// Storage of the two vector weighted densities n_bv (b = 1, 2) and of their
// derivative fields.  n_bv,c(k) = i s_c Q_b(k) with Q_b = A_b / |j| the
// spectrum of a real field and s_c the signed index along axis c (0 on that
// axis's Nyquist plane), so each component is formed in the pass that
// transforms its own axis.  Field slots 4..6 hold vector 1, 7..9 vector 2:
//   after the x-forward pass:  [x] = i s_x Q_b, [z] = Q_b        ([y] unused)
//   after the y-inverse pass:  [x], [y] = i s_y Q_b, [z] = Q_b    (z multiply
//                              by i s_z is applied inside the z pass)
//   after the z derivative pass: [x] = F_x, [y] = F_y, [z] = i s_z F_z
//   after the y-forward pass:  [x] = F_x, [z] = i s_y F_y + i s_z F_z
// and the back pass forms i |j| (khat . F) = i s_x F_x + [z].
constexpr int kSlotX = 4, kSlotY = 5, kSlotZ = 6, kVecStride = 3;
constexpr int kBackFields = 8;  // fields the back pass reads: 0..3, 4, 6, 7, 9

// Spectral field layout: the main block [kx][ky][kz < n/2] with each kx
// plane (n * n/2 complex values) followed by spec_pad unused values, then the
// Nyquist plane kz = n/2 as [kx][ky].  An x-pass workgroup loads one
// 16-pencil row from every kx plane at once; with an unpadded power-of-two
// plane stride (256 KB at 256^3 in FP32) those rows share their low address
// bits and crowd a few memory channels (a plain copy with the x-pass access
// pattern at 256^3: 4.7 TB/s unpadded, 5.6 TB/s padded).  Pads of an odd
// number of 128-byte rows also speed up the y passes.  Measured per
// evaluation: 256^3 1.713 -> 1.687 ms (FP32 spectra, 48 values) and
// 3.527 -> 3.466 ms (FP64, 16 values); 192^3 0.871 -> 0.867 and
// 1.755 -> 1.733 ms; no change at 128^3, whose fields stay largely in the
// Infinity Cache.  tsize: bytes of a real component.
constexpr int64_t spec_pad(int n, int tsize) { return n >= 192 ? (tsize == 4 ? 48 : 16) : 0; }
constexpr int64_t spec_plane(int n, int tsize) { return (int64_t)n * (n / 2) + spec_pad(n, tsize); }
constexpr int64_t spec_fstride(int n, int tsize) { return n * spec_plane(n, tsize) + (int64_t)n * n; }

// status word bits (word 0); word 1 holds the smallest offending flat index
enum : uint32_t { kStPacking = 1u, kStNonFinite = 2u, kStOverflow = 4u };

// Per-instance description read by every pass kernel (device resident).
struct EvalArgs {
  int32_t n;          // grid points per axis
  int32_t S;          // species
  int32_t hs_on;      // hard-sphere term (passes x-forward, derivatives, back phase A)
  int32_t pair_on;    // EC and/or SW pair term in the back pass
  int32_t np;         // S (S + 1) / 2
  int32_t nreal;      // fields written by the real-space output pass
  int32_t final_mode; // 1: add constant, write mu and exp(-mu); 0: plain real output
  uint32_t zmul_mask; // real-output pass: fields whose z spectrum is multiplied by i s_z first
  int64_t fstride;    // complex elements per spectral field (spec_fstride)
  double inv_n3;      // 1 / n^3
  double kscale;      // 2 pi / L: |k| = kscale * sqrt(jx^2 + jy^2 + jz^2)
  double R[kMaxSpecies];
  double area[kMaxSpecies];     // 4 pi R^2
  double inv4piR[kMaxSpecies];  // 1 / (4 pi R)
  double cfin[kMaxSpecies];     // constant added to beta mu in the final pass
  int32_t Sp;         // S rounded up to a multiple of 4 (row length of the pair table)
  int32_t hs_wb;      // 1: modified (White Bear) hard-sphere functional, 0: Rosenfeld
  const double* rho;  // [S][n^3] input densities
  void* specA;        // S spectral fields (densities)
  void* specB;        // 10 spectral fields (weighted densities, then derivatives)
  void* specC;        // S spectral fields (chemical potentials)
  const void* hs_tab;    // [M][S][4]: j0(kR), 4 pi R^3 j1(kR)/(kR), 4 pi R^2 j1(kR), 0
                         // (FP64 path only; the FP32 path evaluates them in registers)
  const void* pair_tab;  // [M][S][Sp]: entry [m][j][i] = combined pair kernel G_ij
  double* out;        // real output [nreal][n^3] (mu_ex or weighted densities)
  double* slot;       // [S][n^3] exp(-mu) or null
  uint32_t* status;   // two words
  double* phi_part;   // per-workgroup sums of Phi_hs from the derivative pass, or null
  // aperiodic mode: the first pass reads an ext_n^3 domain [S][ext_n]^3 and
  // treats it as zero-extended onto the n^3 grid (domain at the corner); with
  // ext_bulk the domain holds ext_val[s] everywhere instead of rho
  int32_t ext_n;
  int32_t ext_bulk;
  double ext_val[kMaxSpecies];
};

// Per-instance arguments of the radial table builder.
struct TableArgs {
  int32_t n, S, np, M;
  double kscale;  // 2 pi / L
  double R[kMaxSpecies];
  double ec_pref[kMaxPairs];  // q_i q_j l_B (0 when EC is off)
  double sigma[kMaxPairs];    // (d_i + d_j) / 2
  double Bsig[kMaxPairs];     // B_ij / sigma_ij
  double sw_pref[kMaxPairs];  // -beta c_sw eps_ij (0 when SW is off)
  double rout[kMaxPairs];
  int8_t pidx[kMaxSpecies][kMaxSpecies];  // pair slot of (i, j)
  int32_t Sp;
  void* hs_tab;
  void* pair_tab;
};

}  // namespace pnp
