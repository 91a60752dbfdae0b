// Surface integrals over spheres by product quadrature (Sec. 3.5), as an
// alternative to the spectral delta-shell weights of the main evaluation.
//
// For a field f on the grid and a radius R, Sec. 3.5 writes
//   I(r)   = int f(r') delta(|r' - r| - R) dr'
//          = R^2 int_0^{2 pi} int_0^{pi} f(r + R n(theta, phi)) sin(phi) dphi dtheta
// and approximates the double integral by a k-by-k product rule in (theta,
// phi).  The 1D rules and the interpolation between grid points are not
// fixed by the paper; here theta_i = 2 pi i / k with weights 2 pi / k (the
// trapezoidal rule of a periodic integrand), phi_j the k Gauss-Legendre
// points of [0, pi], and f(r + R n) the trilinear interpolant of the grid
// values.  The vector integral R^2 int f(r + R n) n dOmega (the FMT n_2v of
// one species) uses the same nodes.
//
// On a uniform grid every node sits at the same displacement R n_ij / h from
// every output point, so its eight trilinear corners are the same integer
// offsets everywhere: the whole rule collapses into one fixed stencil of
// integer offsets with four weights each (scalar, x, y, z), merged on the
// host in double.  The kernel is then a 3D stencil: a workgroup stages a
// tile of f with a halo of the stencil reach in LDS and every thread sums
// the stencil for a column of TX outputs along x, so each LDS value fetched
// feeds four FMAs and each stencil record (read through the scalar cache,
// uniform across the workgroup) feeds 4 TX of them.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

namespace pnp {

constexpr int kQuadTY = 8;       // outputs per workgroup along y
constexpr int kQuadTZ = 32;      // outputs per workgroup along z (the fastest axis)
constexpr int kQuadThreads = kQuadTY * kQuadTZ;
constexpr int kQuadMaxFields = 64;
constexpr size_t kQuadFastLds = 65536;   // tiles up to this size keep several workgroups per CU
constexpr size_t kQuadMaxLds = 163840;   // the most LDS one workgroup can hold on gfx950

// One record of the merged stencil: an integer offset (its position in the
// LDS tile relative to the output point) and the weights of the scalar and
// the three vector integrals there.  A paired record also names the mirror
// offset, whose weights are the same for the scalar and opposite for the
// vector integrals.
template <typename T>
struct QuadEntry {
  int32_t lds;
  int32_t lds_mirror;  // paired records only
  T c[4];
};

struct QuadArgs {
  const double* f;        // [F][N]
  double* out;            // [F][4][N]
  const int32_t* begin;   // [2F + 1]: field f's pairs are [begin[2f], begin[2f+1]), its singles
                          // [begin[2f+1], begin[2f+2])
  const void* entries;
  int32_t nx, ny, nz;
  int32_t H;              // stencil reach (max |offset| over all fields and axes); selects
                          // the kernel, whose tile extents follow from it
  int32_t tiles_y, tiles_z;
  int32_t aperiodic;
};

__device__ __forceinline__ int quad_wrap(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Outputs per thread along x for a stencil reach H: the largest of 8, 4, 2, 1
// whose tile fits 64 KB (at least two workgroups per compute unit); for
// spheres too wide for that, the largest whose tile fits the 160 KB a
// workgroup can hold; 0 if none does.
constexpr size_t quad_tile_bytes(int tx, int H, size_t elem) {
  return (size_t)(tx + 2 * H) * (kQuadTY + 2 * H) * (kQuadTZ + 2 * H) * elem;
}
constexpr int quad_tx(int H, size_t elem) {
  for (int tx = 8; tx >= 1; tx /= 2)
    if (quad_tile_bytes(tx, H, elem) <= kQuadFastLds) return tx;
  for (int tx = 8; tx >= 1; tx /= 2)
    if (quad_tile_bytes(tx, H, elem) <= kQuadMaxLds) return tx;
  return 0;
}

// H (the stencil reach) is a template parameter so that the tile pitches are
// constants: the TX reads of one stencil offset then share one address and
// differ by immediate offsets.
template <typename T, int H>
__global__ __launch_bounds__(kQuadThreads) void k_sphere_quad(QuadArgs a) {
  constexpr int TX = quad_tx(H, sizeof(T));
  constexpr int LY = kQuadTY + 2 * H, LZ = kQuadTZ + 2 * H, LX = TX + 2 * H;
  constexpr int PLANE = LY * LZ;
  __shared__ T tile[LX * PLANE];
  const int field = blockIdx.y;
  int t = blockIdx.x;
  const int tz = t % a.tiles_z;
  t /= a.tiles_z;
  const int ty = t % a.tiles_y;
  const int tx = t / a.tiles_y;
  const int x0 = tx * TX, y0 = ty * kQuadTY, z0 = tz * kQuadTZ;
  const size_t N = (size_t)a.nx * a.ny * a.nz;
  const double* src = a.f + (size_t)field * N;

  // tile element (i, j, l) holds f at grid point (x0 - H + i, y0 - H + j, z0 - H + l):
  // its periodic image, or zero outside the grid in the aperiodic mode
  for (int e = threadIdx.x; e < LX * PLANE; e += kQuadThreads) {
    const int i = e / PLANE;
    const int rem = e - i * PLANE;
    const int j = rem / LZ;
    const int l = rem - j * LZ;
    int gx = x0 - H + i, gy = y0 - H + j, gz = z0 - H + l;
    T v = T(0);
    if (a.aperiodic) {
      if (gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny && gz >= 0 && gz < a.nz)
        v = (T)src[((size_t)gx * a.ny + gy) * a.nz + gz];
    } else {
      gx = quad_wrap(gx, a.nx);
      gy = quad_wrap(gy, a.ny);
      gz = quad_wrap(gz, a.nz);
      v = (T)src[((size_t)gx * a.ny + gy) * a.nz + gz];
    }
    tile[e] = v;
  }
  __syncthreads();

  const int yl = threadIdx.x / kQuadTZ, zl = threadIdx.x % kQuadTZ;
  const T* col = tile + (H * LY + (H + yl)) * LZ + (H + zl);
  T acc[TX][4];
#pragma unroll
  for (int x = 0; x < TX; ++x)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[x][c] = T(0);

  const QuadEntry<T>* E = reinterpret_cast<const QuadEntry<T>*>(a.entries);
  const int e0 = a.begin[2 * field], e1 = a.begin[2 * field + 1], e2 = a.begin[2 * field + 2];
  // mirror pairs d, -d: the scalar weight multiplies the sum of the two
  // values and the vector weights their difference
#pragma unroll 4
  for (int e = e0; e < e1; ++e) {
    const T c0 = E[e].c[0], c1 = E[e].c[1], c2 = E[e].c[2], c3 = E[e].c[3];
    const T* p = col + E[e].lds;
    const T* m = col + E[e].lds_mirror;
#pragma unroll
    for (int x = 0; x < TX; ++x) {
      const T vp = p[x * PLANE], vm = m[x * PLANE];
      const T sum = vp + vm, dif = vp - vm;
      acc[x][0] += c0 * sum;
      acc[x][1] += c1 * dif;
      acc[x][2] += c2 * dif;
      acc[x][3] += c3 * dif;
    }
  }
  for (int e = e1; e < e2; ++e) {
    const T c0 = E[e].c[0], c1 = E[e].c[1], c2 = E[e].c[2], c3 = E[e].c[3];
    const T* p = col + E[e].lds;
#pragma unroll
    for (int x = 0; x < TX; ++x) {
      const T v = p[x * PLANE];
      acc[x][0] += c0 * v;
      acc[x][1] += c1 * v;
      acc[x][2] += c2 * v;
      acc[x][3] += c3 * v;
    }
  }

  const int gy = y0 + yl, gz = z0 + zl;
  if (gy >= a.ny || gz >= a.nz) return;
  double* dst = a.out + (size_t)field * 4 * N;
#pragma unroll
  for (int x = 0; x < TX; ++x) {
    const int gx = x0 + x;
    if (gx < a.nx) {
      const size_t idx = ((size_t)gx * a.ny + gy) * a.nz + gz;
#pragma unroll
      for (int c = 0; c < 4; ++c) dst[(size_t)c * N + idx] = (double)acc[x][c];
    }
  }
}

// ---------------------------------------------------------------------------
// Host side: the rule, the merged stencil and the launch.

// Gauss-Legendre points and weights on [-1, 1]: Newton's method on P_k
// (three-term recurrence) from the usual cosine first guesses.
inline void gauss_legendre(int k, std::vector<double>& x, std::vector<double>& w) {
  x.assign(k, 0.0);
  w.assign(k, 0.0);
  // P_k(z) and P_{k-1}(z) by (m + 1) P_{m+1} = (2m + 1) z P_m - m P_{m-1}
  auto legendre = [k](double z, double& pk, double& pkm1) {
    double p0 = 1.0, p1 = z;
    for (int m = 1; m < k; ++m) {
      const double p2 = ((2.0 * m + 1.0) * z * p1 - m * p0) / (m + 1.0);
      p0 = p1;
      p1 = p2;
    }
    pk = p1;
    pkm1 = p0;
  };
  for (int j = 0; j < k; ++j) {
    double z = std::cos(M_PI * (j + 0.75) / (k + 0.5));
    double pk, pkm1;
    for (int it = 0; it < 100; ++it) {
      legendre(z, pk, pkm1);
      const double dp = k * (z * pk - pkm1) / (z * z - 1.0);  // P_k'(z)
      const double dz = pk / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    legendre(z, pk, pkm1);
    const double dp = k * (z * pk - pkm1) / (z * z - 1.0);
    x[j] = z;
    w[j] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

struct QuadStencil {
  // pairs: offset (dx, dy, dz) and its mirror; singles: offset alone
  std::vector<int32_t> dx, dy, dz;
  std::vector<double> c;  // 4 per record
  std::vector<char> paired;
  int reach = 0;          // max |offset|
};

// Interpolation points along one axis at fraction t of a cell (the node at
// base + t): trilinear, offsets 0 and 1 with 1 - t and t; tricubic, offsets
// -1, 0, 1, 2 with the Lagrange cubics through those points at t.  Returns
// the count; off[] and w[] receive the offsets and weights.
inline int interp_axis(double t, bool cubic, int* off, double* w) {
  if (!cubic) {
    off[0] = 0; w[0] = 1.0 - t;
    off[1] = 1; w[1] = t;
    return 2;
  }
  off[0] = -1; w[0] = -t * (t - 1.0) * (t - 2.0) / 6.0;
  off[1] = 0;  w[1] = (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0;
  off[2] = 1;  w[2] = -(t + 1.0) * t * (t - 2.0) / 2.0;
  off[3] = 2;  w[3] = (t + 1.0) * t * (t - 1.0) / 6.0;
  return 4;
}

// The k-by-k rule of one sphere of radius r (grid units) and physical radius
// R, merged over the interpolation points of every node (8 trilinear
// corners, or 64 tricubic points) into integer offsets.
inline QuadStencil build_quad_stencil(double r, double R, int k, bool cubic) {
  std::vector<double> gx, gw;
  gauss_legendre(k, gx, gw);
  const int Hc = (int)std::floor(r) + (cubic ? 2 : 1);
  const int side = 2 * Hc + 1;
  std::vector<double> acc((size_t)side * side * side * 4, 0.0);
  std::vector<char> hit((size_t)side * side * side, 0);
  for (int i = 0; i < k; ++i) {
    const double th = 2.0 * M_PI * i / k, wth = 2.0 * M_PI / k;
    for (int j = 0; j < k; ++j) {
      const double ph = 0.5 * M_PI * (gx[j] + 1.0), wph = 0.5 * M_PI * gw[j];
      const double n[3] = {std::cos(th) * std::sin(ph), std::sin(th) * std::sin(ph), std::cos(ph)};
      const double W = R * R * std::sin(ph) * wth * wph;
      int b[3], off[3][4], cnt[3];
      double wa[3][4];
      for (int a = 0; a < 3; ++a) {
        const double p = r * n[a];
        b[a] = (int)std::floor(p);
        cnt[a] = interp_axis(p - b[a], cubic, off[a], wa[a]);
      }
      for (int cx = 0; cx < cnt[0]; ++cx)
        for (int cy = 0; cy < cnt[1]; ++cy)
          for (int cz = 0; cz < cnt[2]; ++cz) {
            const double tw = wa[0][cx] * wa[1][cy] * wa[2][cz];
            if (tw == 0.0) continue;
            const int ox = b[0] + off[0][cx] + Hc, oy = b[1] + off[1][cy] + Hc, oz = b[2] + off[2][cz] + Hc;
            const size_t cell = ((size_t)ox * side + oy) * side + oz;
            hit[cell] = 1;
            acc[cell * 4 + 0] += W * tw;
            for (int a = 0; a < 3; ++a) acc[cell * 4 + 1 + a] += W * tw * n[a];
          }
    }
  }
  // A rule with even k holds every node together with its antipode, so the
  // merged weights are even in the offset for the scalar integral and odd for
  // the vector ones (in exact arithmetic; the node coordinates differ in the
  // last bits).  Offsets whose mirror agrees to 1e-14 of the largest weight
  // become one record with the mean weights; the rest stay single.
  const size_t cells = (size_t)side * side * side;
  double cmax = 0.0;
  for (size_t cell = 0; cell < cells; ++cell)
    if (hit[cell])
      for (int q = 0; q < 4; ++q) cmax = std::max(cmax, std::fabs(acc[cell * 4 + q]));
  const double tol = 1e-14 * cmax;
  QuadStencil s;
  std::vector<size_t> singles;
  auto push = [&](size_t cell, const double* c, bool paired) {
    const int ox = (int)(cell / ((size_t)side * side)), oy = (int)(cell / side % side), oz = (int)(cell % side);
    s.dx.push_back(ox - Hc);
    s.dy.push_back(oy - Hc);
    s.dz.push_back(oz - Hc);
    for (int q = 0; q < 4; ++q) s.c.push_back(c[q]);
    s.paired.push_back(paired ? 1 : 0);
    const int m = std::max(std::abs(ox - Hc), std::max(std::abs(oy - Hc), std::abs(oz - Hc)));
    s.reach = std::max(s.reach, m);
  };
  for (size_t cell = 0; cell < cells; ++cell) {
    if (!hit[cell]) continue;
    const size_t mirror = cells - 1 - cell;  // offset -d
    if (mirror == cell || !hit[mirror]) {
      singles.push_back(cell);
      continue;
    }
    if (mirror < cell) continue;  // handled with its partner
    const double* a = &acc[cell * 4];
    const double* b = &acc[mirror * 4];
    bool even = std::fabs(a[0] - b[0]) <= tol;
    for (int q = 1; q < 4; ++q) even = even && std::fabs(a[q] + b[q]) <= tol;
    if (!even) {
      singles.push_back(cell);
      singles.push_back(mirror);
      continue;
    }
    const double mean[4] = {0.5 * (a[0] + b[0]), 0.5 * (a[1] - b[1]), 0.5 * (a[2] - b[2]), 0.5 * (a[3] - b[3])};
    push(cell, mean, true);
    const int m = std::max(std::abs((int)(mirror / ((size_t)side * side)) - Hc),
                           std::max(std::abs((int)(mirror / side % side) - Hc), std::abs((int)(mirror % side) - Hc)));
    s.reach = std::max(s.reach, m);
  }
  for (size_t cell : singles) push(cell, &acc[cell * 4], false);
  return s;
}

// The packed upload: begin[2F + 1] (padded to 16 bytes), then per field its
// paired records followed by its single ones.
template <typename T>
inline std::vector<unsigned char> pack_quad(const std::vector<QuadStencil>& st, int ly, int lz,
                                            size_t& entries_at) {
  const int F = (int)st.size();
  size_t head = ((size_t)(2 * F + 1) * sizeof(int32_t) + 15) / 16 * 16;
  size_t count = 0;
  for (const auto& s : st) count += s.dx.size();
  std::vector<unsigned char> buf(head + count * sizeof(QuadEntry<T>), 0);
  int32_t* begin = reinterpret_cast<int32_t*>(buf.data());
  QuadEntry<T>* E = reinterpret_cast<QuadEntry<T>*>(buf.data() + head);
  size_t e = 0;
  for (int f = 0; f < F; ++f) {
    const QuadStencil& q = st[f];
    for (int pass = 0; pass < 2; ++pass) {
      begin[2 * f + pass] = (int32_t)e;
      for (size_t r = 0; r < q.dx.size(); ++r) {
        if ((q.paired[r] != 0) != (pass == 0)) continue;
        E[e].lds = (q.dx[r] * ly + q.dy[r]) * lz + q.dz[r];
        E[e].lds_mirror = pass == 0 ? -E[e].lds : 0;
        for (int c = 0; c < 4; ++c) E[e].c[c] = (T)q.c[r * 4 + c];
        ++e;
      }
    }
  }
  begin[2 * F] = (int32_t)e;
  entries_at = head;
  return buf;
}

template <typename T, int H>
inline void launch_sphere_quad_h(const QuadArgs& a, int F, hipStream_t s) {
  constexpr int TX = quad_tx(H, sizeof(T));
  static_assert(TX > 0, "tile does not fit the LDS budget");
  const int tiles_x = (a.nx + TX - 1) / TX;
  const dim3 grid((unsigned)(tiles_x * a.tiles_y * a.tiles_z), (unsigned)F);
  hipLaunchKernelGGL((k_sphere_quad<T, H>), grid, dim3(kQuadThreads), 0, s, a);
}

// The largest reach each precision's tile takes.
template <typename T>
constexpr int quad_max_reach() {
  int H = 1;
  while (quad_tx(H + 1, sizeof(T)) > 0) ++H;
  return H;
}

// Launch for reach a.H, 1 <= a.H <= quad_max_reach<T>() (11 in FP32, 8 in FP64).
template <typename T, int H>
inline hipError_t launch_sphere_quad_upto(const QuadArgs& a, int F, hipStream_t s) {
  if constexpr (H > quad_max_reach<T>()) {
    return hipErrorInvalidValue;
  } else {
    if (a.H == H) {
      launch_sphere_quad_h<T, H>(a, F, s);
      return hipGetLastError();
    }
    return launch_sphere_quad_upto<T, H + 1>(a, F, s);
  }
}

template <typename T>
inline hipError_t launch_sphere_quad(const QuadArgs& a, int F, hipStream_t s) {
  return launch_sphere_quad_upto<T, 1>(a, F, s);
}

}  // namespace pnp
