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
#include <string>
#include <vector>

namespace pnp {

constexpr int kQuadTY = 8;       // outputs per workgroup along y
constexpr int kQuadTZ = 32;      // outputs per workgroup along z (the fastest axis)
constexpr int kQuadThreads = kQuadTY * kQuadTZ;
constexpr int kQuadMaxFields = 64;
constexpr size_t kQuadMaxLds = 65536;

// One integer offset of the merged stencil: its position in the LDS tile
// relative to the output point and the weights of the scalar and the three
// vector integrals.
template <typename T>
struct QuadEntry {
  int32_t lds;
  int32_t pad;
  T c[4];
};

struct QuadArgs {
  const double* f;        // [F][N]
  double* out;            // [F][4][N]
  const int32_t* begin;   // [F + 1] entry ranges per field, followed by the entries
  const void* entries;
  int32_t nx, ny, nz;
  int32_t H;              // stencil reach (max |offset| over all fields and axes)
  int32_t lx, ly, lz;     // LDS tile extents
  int32_t tiles_y, tiles_z;
  int32_t aperiodic;
};

__device__ __forceinline__ int quad_wrap(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

template <typename T, int TX>
__global__ __launch_bounds__(kQuadThreads) void k_sphere_quad(QuadArgs a) {
  extern __shared__ unsigned char quad_smem[];
  T* tile = reinterpret_cast<T*>(quad_smem);
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
  const int plane = a.ly * a.lz;
  const int total = a.lx * plane;
  for (int e = threadIdx.x; e < total; e += kQuadThreads) {
    const int i = e / plane;
    const int rem = e - i * plane;
    const int j = rem / a.lz;
    const int l = rem - j * a.lz;
    int gx = x0 - a.H + i, gy = y0 - a.H + j, gz = z0 - a.H + l;
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
  const T* col = tile + (a.H * a.ly + (a.H + yl)) * a.lz + (a.H + zl);
  T acc[TX][4];
#pragma unroll
  for (int x = 0; x < TX; ++x)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[x][c] = T(0);

  const QuadEntry<T>* E = reinterpret_cast<const QuadEntry<T>*>(a.entries);
  const int e0 = a.begin[field], e1 = a.begin[field + 1];
  for (int e = e0; e < e1; ++e) {
    const int off = E[e].lds;
    const T c0 = E[e].c[0], c1 = E[e].c[1], c2 = E[e].c[2], c3 = E[e].c[3];
    const T* p = col + off;
#pragma unroll
    for (int x = 0; x < TX; ++x) {
      const T v = p[x * plane];
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
  std::vector<int32_t> dx, dy, dz;
  std::vector<double> c;  // 4 per entry
  int reach = 0;          // max |offset|
};

// The k-by-k rule of one sphere of radius r (grid units) and physical radius
// R, merged over the trilinear corners of every node into integer offsets.
inline QuadStencil build_quad_stencil(double r, double R, int k) {
  std::vector<double> gx, gw;
  gauss_legendre(k, gx, gw);
  const int Hc = (int)std::floor(r) + 1;
  const int side = 2 * Hc + 1;
  std::vector<double> acc((size_t)side * side * side * 4, 0.0);
  std::vector<char> hit((size_t)side * side * side, 0);
  for (int i = 0; i < k; ++i) {
    const double th = 2.0 * M_PI * i / k, wth = 2.0 * M_PI / k;
    for (int j = 0; j < k; ++j) {
      const double ph = 0.5 * M_PI * (gx[j] + 1.0), wph = 0.5 * M_PI * gw[j];
      const double n[3] = {std::cos(th) * std::sin(ph), std::sin(th) * std::sin(ph), std::cos(ph)};
      const double W = R * R * std::sin(ph) * wth * wph;
      int b[3];
      double fr[3];
      for (int a = 0; a < 3; ++a) {
        const double p = r * n[a];
        b[a] = (int)std::floor(p);
        fr[a] = p - b[a];
      }
      for (int cx = 0; cx < 2; ++cx)
        for (int cy = 0; cy < 2; ++cy)
          for (int cz = 0; cz < 2; ++cz) {
            const double tw = (cx ? fr[0] : 1.0 - fr[0]) * (cy ? fr[1] : 1.0 - fr[1]) *
                              (cz ? fr[2] : 1.0 - fr[2]);
            if (tw == 0.0) continue;
            const int ox = b[0] + cx + Hc, oy = b[1] + cy + Hc, oz = b[2] + cz + Hc;
            const size_t cell = ((size_t)ox * side + oy) * side + oz;
            hit[cell] = 1;
            acc[cell * 4 + 0] += W * tw;
            for (int a = 0; a < 3; ++a) acc[cell * 4 + 1 + a] += W * tw * n[a];
          }
    }
  }
  QuadStencil s;
  for (int ox = 0; ox < side; ++ox)
    for (int oy = 0; oy < side; ++oy)
      for (int oz = 0; oz < side; ++oz) {
        const size_t cell = ((size_t)ox * side + oy) * side + oz;
        if (!hit[cell]) continue;
        s.dx.push_back(ox - Hc);
        s.dy.push_back(oy - Hc);
        s.dz.push_back(oz - Hc);
        for (int q = 0; q < 4; ++q) s.c.push_back(acc[cell * 4 + q]);
        const int m = std::max(std::abs(ox - Hc), std::max(std::abs(oy - Hc), std::abs(oz - Hc)));
        s.reach = std::max(s.reach, m);
      }
  return s;
}

// Outputs per thread along x for a stencil reach H: the largest of 8, 4, 2, 1
// whose tile fits the LDS budget; 0 if none does.
inline int quad_tx(int H, size_t elem) {
  for (int tx = 8; tx >= 1; tx /= 2) {
    const size_t bytes = (size_t)(tx + 2 * H) * (kQuadTY + 2 * H) * (kQuadTZ + 2 * H) * elem;
    if (bytes <= kQuadMaxLds) return tx;
  }
  return 0;
}

// The packed upload: begin[F + 1] (padded to 16 bytes), then the entries.
template <typename T>
inline std::vector<unsigned char> pack_quad(const std::vector<QuadStencil>& st, int ly, int lz,
                                            size_t& entries_at) {
  const int F = (int)st.size();
  size_t head = ((size_t)(F + 1) * sizeof(int32_t) + 15) / 16 * 16;
  size_t count = 0;
  for (const auto& s : st) count += s.dx.size();
  std::vector<unsigned char> buf(head + count * sizeof(QuadEntry<T>), 0);
  int32_t* begin = reinterpret_cast<int32_t*>(buf.data());
  QuadEntry<T>* E = reinterpret_cast<QuadEntry<T>*>(buf.data() + head);
  size_t e = 0;
  for (int f = 0; f < F; ++f) {
    begin[f] = (int32_t)e;
    for (size_t q = 0; q < st[f].dx.size(); ++q, ++e) {
      E[e].lds = (st[f].dx[q] * ly + st[f].dy[q]) * lz + st[f].dz[q];
      E[e].pad = 0;
      for (int c = 0; c < 4; ++c) E[e].c[c] = (T)st[f].c[q * 4 + c];
    }
  }
  begin[F] = (int32_t)e;
  entries_at = head;
  return buf;
}

template <typename T>
inline hipError_t launch_sphere_quad(const QuadArgs& a, int tx, int F, hipStream_t s) {
  const int tiles_x = (a.nx + tx - 1) / tx;
  const dim3 grid((unsigned)(tiles_x * a.tiles_y * a.tiles_z), (unsigned)F);
  const size_t lds = (size_t)a.lx * a.ly * a.lz * sizeof(T);
  switch (tx) {
    case 8: hipLaunchKernelGGL((k_sphere_quad<T, 8>), grid, dim3(kQuadThreads), lds, s, a); break;
    case 4: hipLaunchKernelGGL((k_sphere_quad<T, 4>), grid, dim3(kQuadThreads), lds, s, a); break;
    case 2: hipLaunchKernelGGL((k_sphere_quad<T, 2>), grid, dim3(kQuadThreads), lds, s, a); break;
    default: hipLaunchKernelGGL((k_sphere_quad<T, 1>), grid, dim3(kQuadThreads), lds, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace pnp
