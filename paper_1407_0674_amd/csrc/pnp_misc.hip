// Kernels outside the FFT passes: the calibration copy, the density
// updates (relaxation stub, Picard step), free-energy reductions, the
// per-term Slotboom sum and the aperiodic crop.  Compiled once, in the ABI's
// translation unit (the pass templates are instantiated in their own
// translation units, one per precision and grid size).
#pragma once
#include "pnp_kernels.hip"

namespace pnp {

// plain device copy of 16-byte words (bandwidth and counter calibration)
// Streaming copy (the achievable-bandwidth reference and counter
// calibration): one 16-byte word per thread, non-temporal loads and stores,
// one short-lived workgroup per 4 KiB.  Measured on 1 GiB: 6.5 TB/s, against
// 4.5-5.2 TB/s for grid-stride loops of 2048-32768 workgroups.
__global__ void __launch_bounds__(256) k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, long words) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < words) {
    typedef unsigned int w4 __attribute__((ext_vector_type(4)));
    const w4 v = __builtin_nontemporal_load((const w4*)src + e);
    __builtin_nontemporal_store(v, (w4*)dst + e);
  }
}

// relaxation of the consumer stub: rho <- (1 - l) rho + l rho_b exp(g),
// g = mu_b - mu limited to [-clip, clip] when clip > 0
// status: the evaluation's status word, or null; a raised status leaves rho
// untouched (uniform over the grid)
// fixed: bit s set = species s is stationary (its density is not touched)
__global__ void k_relax(double* rho, const double* mu, long n3, int S, const double* rho_b_mu_b,
                        double lambda, double clip, const uint32_t* status, uint32_t fixed) {
  if (status && status[0] != 0u) return;
  const long total = (long)S * n3;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int s = (int)(e / n3);
    if ((fixed >> s) & 1u) continue;
    const double rb = rho_b_mu_b[2 * s], mb = rho_b_mu_b[2 * s + 1];
    double g = mb - mu[e];
    if (clip > 0.0) g = fmin(fmax(g, -clip), clip);
    rho[e] = (1.0 - lambda) * rho[e] + lambda * rb * exp(g);
  }
}

// Pair free energies from one per-term evaluation, per-workgroup partial sums
// (fixed order): part[2b] = sum_i sum_r (rho_i - rho_b,i)(beta mu_el,i +
// beta mu_el,i[bulk]); part[2b + 1] = sum_i sum_r rho_i beta mu_sh,i.
// rb_mb: [S][2] = (rho_b, beta mu_el[bulk]); mu3: [3][S][n3] per-term output.
__global__ void __launch_bounds__(256) k_energy_part(const double* rho, const double* mu3, long n3, int S,
                                                     const double* rb_mb, double* part) {
  __shared__ double red[4];
  const long sn3 = (long)S * n3;
  double e = 0.0, f = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < sn3; i += (long)gridDim.x * blockDim.x) {
    const int s = (int)(i / n3);
    const double r = rho[i];
    e += (r - rb_mb[2 * s]) * (mu3[sn3 + i] + rb_mb[2 * s + 1]);
    f += r * mu3[2 * sn3 + i];
  }
  const double te = block_sum(e, red);
  const double tf = block_sum(f, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = te;
    part[2 * blockIdx.x + 1] = tf;
  }
}

// out[0..3] = F_hs, F_el, F_sh, total [k_B T] from the partial sums, in a
// fixed order.  phi_scale converts the Phi sums to h^3 sum Phi.
__global__ void __launch_bounds__(256) k_energy_final(const double* phi_part, int nphi, const double* part,
                                                      int npart, double phi_scale, double el_scale,
                                                      double sh_scale, double* out) {
  __shared__ double red[4];
  double a = 0.0, e = 0.0, f = 0.0;
  for (int i = threadIdx.x; i < nphi; i += blockDim.x) a += phi_part[i];
  for (int i = threadIdx.x; i < npart; i += blockDim.x) {
    e += part[2 * i];
    f += part[2 * i + 1];
  }
  const double ta = block_sum(a, red);
  const double te = block_sum(e, red);
  const double tf = block_sum(f, red);
  if (threadIdx.x == 0) {
    const double hs = phi_scale * ta, el = el_scale * te, sh = sh_scale * tf;
    out[0] = hs;
    out[1] = el;
    out[2] = sh;
    out[3] = hs + el + sh;
  }
}

// Picard step of the equilibrium solve: rho <- (1 - l) rho + l rho_b
// exp(mu_b - mu - beta V) (beta_v may be null) and the residual
// max |rho_new - rho| / rho_b as the bit pattern of a non-negative double
// (integer max of such patterns is the max of the values: exact and
// independent of the order of the updates).  Stationary species (bit s of
// fixed) keep their densities and do not enter the residual.
__global__ void __launch_bounds__(256) k_picard(double* rho, const double* mu, const double* beta_v, long n3, int S,
                                                const double* rb_mb, double lambda, unsigned long long* res,
                                                uint32_t fixed) {
  double r = 0.0;
  const long total = (long)S * n3;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int s = (int)(e / n3);
    if ((fixed >> s) & 1u) continue;
    const double rb = rb_mb[2 * s], mb = rb_mb[2 * s + 1];
    const double g = mb - mu[e] - (beta_v ? beta_v[e] : 0.0);
    const double old = rho[e];
    const double nw = (1.0 - lambda) * old + lambda * rb * exp(g);
    rho[e] = nw;
    r = fmax(r, fabs(nw - old) / rb);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(res, (unsigned long long)__double_as_longlong(r));
}

// per-term mode: slot = exp(-(hs + el + sh))
__global__ void k_sum_exp(const double* mu3, double* slot, long sn3, uint32_t* status) {
  uint32_t bad = 0u, badidx = 0xffffffffu;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < sn3; e += (long)gridDim.x * blockDim.x) {
    const double m = mu3[e] + mu3[sn3 + e] + mu3[2 * sn3 + e];
    if (!isfinite(m)) { bad |= kStNonFinite; badidx = min(badidx, (uint32_t)e); }
    if (slot && -m > 709.782712893384) { bad |= kStOverflow; badidx = min(badidx, (uint32_t)e); }
    if (slot) slot[e] = exp(-m);
  }
  if (bad) raise_status(status, bad, badidx);
}

// Aperiodic mode: the domain part of the doubled-grid result.
//   muA  [nterm][S][(2n)^3]: the evaluation of the extended densities
//        (nterm = 3: hs, el, sh; 1: the total)
//   muB  [S][(2n)^3] or null: the EC response to the extended bulk densities,
//        subtracted from the EC term (from the total when nterm = 1)
//   out  [nterm][S][n^3]; slot [S][n^3] = exp(-total) or null
// Status as the final pass: non-finite totals, and exp(-mu) overflow when
// slot is requested.
__global__ void k_crop(const double* muA, const double* muB, int nterm, int S, int n, double* out, double* slot,
                       uint32_t* status) {
  const long n2 = 2L * n, N2 = n2 * n2 * n2, N = (long)n * n * n, total = (long)S * N;
  uint32_t bad = 0u, badidx = 0xffffffffu;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int s = (int)(e / N);
    long r = e - (long)s * N;
    const long z = r % n;
    r /= n;
    const long y = r % n, x = r / n;
    const long e2 = (long)s * N2 + (x * n2 + y) * n2 + z;
    double tot = 0.0;
    for (int t = 0; t < nterm; ++t) {
      double v = muA[(long)t * S * N2 + e2];
      if (muB && (nterm == 1 || t == 1)) v -= muB[e2];
      out[(long)t * total + e] = v;
      tot += v;
    }
    if (!isfinite(tot)) { bad |= kStNonFinite; badidx = min(badidx, (uint32_t)e); }
    if (slot) {
      if (-tot > 709.782712893384) { bad |= kStOverflow; badidx = min(badidx, (uint32_t)e); }
      slot[e] = exp(-tot);
    }
  }
  if (bad) raise_status(status, bad, badidx);
}


}  // namespace pnp
