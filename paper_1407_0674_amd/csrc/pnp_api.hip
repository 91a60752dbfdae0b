// Host driver of the C ABI declared in include/pnp_cdft.h.
//
// Responsibilities: argument validation, the physical constants and pair
// parameters of Sec. 2.3 (in double on the host), the workspace layout, the
// per-instance argument tables uploaded to a small context-owned device ring,
// the launch sequence of the nine passes, batching of equal-size requests into
// shared launches, and the device status word.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pnp_cdft.h"
#include "pnp_launch.hpp"
#include "pnp_misc.hip"
#include "sphere_quad.hip"

using namespace pnp;

struct pnp_ctx_s {
  int device = 0;
  std::string err;
  char* arena = nullptr;      // device ring for argument tables
  size_t arena_bytes = 0;
  size_t arena_pos = 0;
  // pass timing
  bool prof = false;
  uint32_t prof_mask = ~0u;                        // passes that record events
  std::vector<hipEvent_t> ev_pool;                 // free events
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_open;  // recorded, unread
  double prof_ms[PNP_NUM_PASSES] = {0};
  int32_t prof_n[PNP_NUM_PASSES] = {0};
  bool capturing = false;  // a plan is being captured: no pass events
  // autotuned tile shapes: (precision, n, count class) -> narrow-pass mask
  std::map<uint64_t, uint32_t> tune;
  // autotuned or imported FFT schedules: (precision, n) -> secondary-pass mask
  std::map<uint64_t, uint32_t> sched;
  // device address of this device's static scratch array (null if the
  // lookup failed at creation)
  void* scratch = nullptr;
  // side stream (default priority) for the Nyquist-plane tiles of the y and
  // x passes, with its fork and join events; created on first use
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool side_failed = false;
  // branch streams (default priority) on which a batch runs its grid sizes
  // below 192^3 side by side, with the fork event and one join event each;
  // created on first use
  std::vector<hipStream_t> br;
  std::vector<hipEvent_t> br_done;
  hipEvent_t br_fork = nullptr;
  bool br_failed = false;
};

// Scratch of the allocation-free evaluation (pnp_cdft_mu_ex_noalloc): one
// static device array, which every GPU the library runs on holds from the
// load of this code object until the process ends.  In host code `scratch`
// names a host-side stand-in, not a device address; the device address of
// each GPU's copy comes from hipGetSymbolAddress (pnp_create, once per
// device) and only that address is ever handed to kernels or copies.
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;  // device -> address of its scratch copy

// The address of `scratch` on the current device (looked up once per device).
void* scratch_address(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) return it->second;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();  // leave no sticky error behind
    return nullptr;
  }
  g_scratch_addr[device] = ptr;
  return ptr;
}
}  // namespace

namespace {

constexpr double kElementaryCharge = 1.602176634e-19;  // C
constexpr double kVacuumPermittivity = 8.8541878128e-12;  // F/m
constexpr double kBoltzmann = 1.380649e-23;  // J/K
constexpr double kBoltzmannEv = kBoltzmann / kElementaryCharge;  // eV/K
// e^2 / (4 pi eps0) in eV nm
const double kCoulombEvNm = kElementaryCharge / (4.0 * M_PI * kVacuumPermittivity) * 1e9;

constexpr size_t kAlign = 256;
constexpr int kEnergyBlocks = 1024;  // workgroups of the pair-energy reduction
inline size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

pnp_status fail(pnp_ctx c, pnp_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

hipEvent_t take_event(pnp_ctx c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one pass with two events on the stream when timing is on.
struct PassTimer {
  pnp_ctx c;
  hipStream_t s;
  int id = -1;
  hipEvent_t e0 = nullptr;
  void begin(int pass) {
    if (!c || !c->prof || c->capturing || !((c->prof_mask >> pass) & 1u)) return;
    id = pass;
    e0 = take_event(c);
    if (e0) hipEventRecord(e0, s);
  }
  void end() {
    if (!c || !c->prof || !e0) return;
    hipEvent_t e1 = take_event(c);
    if (e1) {
      hipEventRecord(e1, s);
      c->ev_open.push_back({id, {e0, e1}});
    } else {
      c->ev_pool.push_back(e0);
    }
    e0 = nullptr;
  }
};

bool size_ok(int n) {
  switch (n) {
    case 8: case 16: case 24: case 32: case 48: case 64: case 96: case 128: case 192: case 256:
      return true;
    default:
      return false;
  }
}

// Derived quantities of one evaluation (host, double precision).
struct Derived {
  int n = 0, S = 0, np = 0, precision = 0;
  double h = 0;
  bool hs = false, wb = false, ec = false, sw = false;  // wb: hard spheres by the White Bear form
  bool aperiodic = false;  // n is the doubled grid; n_dom the domain (n_dom = n when periodic)
  int n_dom = 0;
  double beta = 0, lB = 0, kappa = 0;
  double sigma[kMaxPairs], B[kMaxPairs], rout[kMaxPairs], eps[kMaxPairs];
  int pi[kMaxSpecies][kMaxSpecies];
  double cfin_ec[kMaxSpecies];
};

// the hard-sphere functional of one instance as a variant bit: 1 Rosenfeld,
// 2 White Bear, 0 no hard-sphere term
inline int hs_mask(const Derived& d) { return d.hs ? (d.wb ? 2 : 1) : 0; }

struct Layout {
  size_t status, energy, hs, pair, pair2, A, B, C, total;
  long fstride;
  int M;
};

inline int padded_species(int S) { return (S + 3) / 4 * 4; }

// bit i set = species i is stationary (the density updates leave it alone)
inline uint32_t fixed_mask(int S, const pnp_species* sp) {
  uint32_t m = 0u;
  for (int i = 0; i < S; ++i)
    if (!sp[i].mobile) m |= 1u << i;
  return m;
}

Layout layout_of(int n, int S, int precision, bool hs, bool pairs, bool per_term) {
  Layout L{};
  const size_t ts = precision == PNP_MIXED ? 4 : 8;
  const long H = n / 2;
  L.M = (int)(3 * H * H + 1);
  L.fstride = (long)spec_fstride(n, (int)ts);
  const size_t prow = (size_t)S * padded_species(S);
  size_t o = 0;
  L.status = o; o = up(o + 64);
  // free-energy partial sums: one per derivative-pass workgroup (at most n^2),
  // kEnergyBlocks pairs from the pair-energy pass, and the four results
  L.energy = o; o = up(o + sizeof(double) * ((size_t)n * n + 2 * kEnergyBlocks + 4));
  L.hs = o; if (precision == PNP_FP64) o = up(o + (size_t)L.M * 4 * S * ts);  // FP32 weights live in registers
  L.pair = o; if (pairs) o = up(o + (size_t)L.M * prow * ts);
  L.pair2 = o; if (pairs && per_term) o = up(o + (size_t)L.M * prow * ts);
  L.A = o; o = up(o + (size_t)S * L.fstride * 2 * ts);
  L.B = o; if (hs) o = up(o + (size_t)kFields * L.fstride * 2 * ts);
  L.C = o; o = up(o + (size_t)S * L.fstride * 2 * ts);
  L.total = o;
  return L;
}

// aperiodic_ok: the entry point accepts PNP_FLAG_APERIODIC (the evaluation
// then runs on the doubled grid, and d.n is that grid's size)
// The aperiodic mode adds, after the evaluation workspace of the doubled
// grid n2: the doubled-grid output and the doubled-grid EC response to the
// domain's bulk densities (EC only); float64 [S][n2^3], the output
// [3][S][n2^3] in per-term mode.  (The zero extension itself is read on the
// fly by the first pass.)
struct LayoutAp {
  Layout L;
  size_t muA, muB, total;
};

LayoutAp layout_aperiodic(int n2, int S, int precision, bool hs, bool pairs, bool ec, bool per_term) {
  LayoutAp A;
  A.L = layout_of(n2, S, precision, hs, pairs, per_term);
  const size_t f = sizeof(double) * (size_t)S * n2 * n2 * n2;
  size_t o = A.L.total;
  A.muA = o; o = up(o + (per_term ? 3 : 1) * f);
  A.muB = o; if (ec) o = up(o + f);
  A.total = o;
  return A;
}

pnp_status validate(pnp_ctx ctx, const pnp_grid* g, int S, const pnp_species* sp, double T,
                    const pnp_params* p, Derived& d, bool need_T, bool aperiodic_ok = false) {
  if (!ctx) return PNP_E_ARG;
  if (!g || !sp || !p) return fail(ctx, PNP_E_ARG, "null grid, species or params");
  if (g->nx != g->ny || g->ny != g->nz) return fail(ctx, PNP_E_UNSUPPORTED_SIZE, "grid must be cubic (nx = ny = nz)");
  if (p->flags & ~(uint32_t)(PNP_FLAG_ASYNC | PNP_FLAG_APERIODIC)) return fail(ctx, PNP_E_ARG, "unsupported flag");
  const bool aperiodic = p->flags & PNP_FLAG_APERIODIC;
  if (aperiodic && !aperiodic_ok) return fail(ctx, PNP_E_ARG, "PNP_FLAG_APERIODIC is not available here");
  if (aperiodic ? !(g->nx >= 4 && g->nx <= 128 && size_ok(2 * g->nx)) : !size_ok(g->nx))
    return fail(ctx, PNP_E_UNSUPPORTED_SIZE, "grid size " + std::to_string(g->nx) + " not supported" +
                                                 (aperiodic ? " in the aperiodic mode (2n must be supported)" : ""));
  if (!(g->h > 0.0) || !std::isfinite(g->h)) return fail(ctx, PNP_E_ARG, "spacing h must be > 0");
  if (S < 1 || S > kMaxSpecies) return fail(ctx, PNP_E_ARG, "species count must be in [1, 8]");
  if (p->terms == 0 || (p->terms & ~15u)) return fail(ctx, PNP_E_ARG, "terms must be a non-empty PNP_TERM_* mask");
  if ((p->terms & PNP_TERM_HS) && (p->terms & PNP_TERM_HS_WB))
    return fail(ctx, PNP_E_ARG, "PNP_TERM_HS and PNP_TERM_HS_WB are exclusive");
  if (p->precision != PNP_FP64 && p->precision != PNP_MIXED) return fail(ctx, PNP_E_ARG, "bad precision");
  if (need_T && !(T > 0.0 && std::isfinite(T))) return fail(ctx, PNP_E_ARG, "temperature must be > 0");
  for (int i = 0; i < S; ++i)
    if (!(sp[i].d > 0.0) || !std::isfinite(sp[i].q) || !std::isfinite(sp[i].rho_bulk) ||
        !std::isfinite(sp[i].mu_el_bulk))
      return fail(ctx, PNP_E_ARG, "species " + std::to_string(i) + ": bad diameter, valence or bulk density");
  d.aperiodic = aperiodic;
  d.n_dom = g->nx;
  d.n = aperiodic ? 2 * g->nx : g->nx;
  d.h = g->h; d.S = S; d.np = S * (S + 1) / 2; d.precision = p->precision;
  d.hs = p->terms & (PNP_TERM_HS | PNP_TERM_HS_WB); d.wb = p->terms & PNP_TERM_HS_WB; d.ec = p->terms & PNP_TERM_EC; d.sw = p->terms & PNP_TERM_SW;
  if (need_T) {
    if (d.ec && !(p->eps_r > 0.0)) return fail(ctx, PNP_E_ARG, "eps_r must be > 0");
    d.beta = 1.0 / (kBoltzmannEv * T);
    d.lB = d.ec ? kCoulombEvNm / p->eps_r * d.beta : 0.0;
    double k2 = 0.0;
    for (int i = 0; i < S; ++i) k2 += sp[i].rho_bulk * sp[i].q * sp[i].q;
    d.kappa = std::sqrt(std::max(0.0, 4.0 * M_PI * d.lB * k2));
  }
  int q = 0;
  for (int i = 0; i < S; ++i)
    for (int j = i; j < S; ++j, ++q) {
      d.pi[i][j] = d.pi[j][i] = q;
      const double s = 0.5 * (sp[i].d + sp[j].d);
      d.sigma[q] = s;
      const double xi = d.kappa * s;
      d.B[q] = xi == 0.0 ? 0.0 : xi / (xi + 1.0 + std::sqrt(1.0 + 2.0 * xi));
      double e = 0.0, ro = 0.0;
      if (p->sw_eps) {
        e = p->sw_eps[i * S + j];
        if (std::fabs(e - p->sw_eps[j * S + i]) > 1e-12 * std::max(1.0, std::fabs(e)))
          return fail(ctx, PNP_E_ARG, "sw_eps must be symmetric");
      }
      if (p->sw_rout) ro = p->sw_rout[i * S + j];
      if (!(ro > 0.0)) ro = (p->sw_gamma > 0.0 ? p->sw_gamma : 1.2) * s;
      d.eps[q] = e;
      d.rout[q] = ro;
    }
  for (int i = 0; i < S; ++i) {
    // the EC term's constant: its bulk value plus the k = 0 part of
    // -sum_j C_ij rho_j^bulk; nothing when the EC term is off.  In the
    // aperiodic mode the bulk densities are not uniform over the doubled grid
    // (they fill the domain only), so that part is a separate convolution.
    double c = d.ec ? sp[i].mu_el_bulk : 0.0;
    if (d.ec && !d.aperiodic)
      for (int j = 0; j < S; ++j) {
        const int pq = d.pi[i][j];
        const double s = d.sigma[pq], b = d.B[pq];
        // integral of C_ij over the ball r <= sigma (Sec. 2.3.4)
        const double c0 = -sp[i].q * sp[j].q * d.lB * M_PI * s * s * (8.0 * b / 3.0 - b * b - 2.0);
        c += c0 * sp[j].rho_bulk;
      }
    d.cfin_ec[i] = c;
  }
  return PNP_OK;
}

void fill_table_args(TableArgs& t, const Derived& d, const pnp_species* sp, double h, double sw_pref_scale,
                     bool ec, bool sw, void* hs, void* pair, int M) {
  std::memset(&t, 0, sizeof(t));
  t.n = d.n; t.S = d.S; t.np = d.np; t.M = M;
  t.kscale = 2.0 * M_PI / (d.n * h);
  for (int i = 0; i < d.S; ++i) t.R[i] = 0.5 * sp[i].d;
  int q = 0;
  for (int i = 0; i < d.S; ++i)
    for (int j = i; j < d.S; ++j, ++q) {
      t.sigma[q] = d.sigma[q];
      t.Bsig[q] = d.B[q] / d.sigma[q];
      t.ec_pref[q] = ec ? sp[i].q * sp[j].q * d.lB : 0.0;
      t.sw_pref[q] = sw ? -d.beta * sw_pref_scale * d.eps[q] : 0.0;
      t.rout[q] = d.rout[q];
    }
  for (int i = 0; i < d.S; ++i)
    for (int j = 0; j < d.S; ++j) t.pidx[i][j] = (int8_t)d.pi[i][j];
  t.Sp = padded_species(d.S);
  t.hs_tab = hs; t.pair_tab = pair;
}

void fill_eval_args(EvalArgs& e, const Derived& d, const pnp_species* sp, const Layout& L, char* ws,
                    const double* rho) {
  std::memset(&e, 0, sizeof(e));
  e.n = d.n; e.S = d.S; e.np = d.np;
  e.hs_on = d.hs; e.hs_wb = d.wb; e.pair_on = d.ec || d.sw;
  e.ext_n = d.aperiodic ? d.n_dom : 0;  // the first pass zero-extends the domain
  e.fstride = L.fstride;
  e.inv_n3 = 1.0 / ((double)d.n * d.n * d.n);
  e.kscale = 2.0 * M_PI / (d.n * d.h);
  for (int i = 0; i < d.S; ++i) {
    const double R = 0.5 * sp[i].d;
    e.R[i] = R;
    e.area[i] = 4.0 * M_PI * R * R;
    e.inv4piR[i] = 1.0 / (4.0 * M_PI * R);
    e.cfin[i] = d.cfin_ec[i];
  }
  e.Sp = padded_species(d.S);
  e.rho = rho;
  e.specA = ws + L.A;
  e.specB = ws + L.B;
  e.specC = ws + L.C;
  e.hs_tab = ws + L.hs;
  e.pair_tab = ws + L.pair;
  e.status = (uint32_t*)(ws + L.status);
  e.final_mode = 1;
  e.nreal = d.S;
}

// copy host bytes into the context's device ring (stream ordered)
void* upload(pnp_ctx c, const void* src, size_t bytes, hipStream_t s) {
  const size_t need = up(bytes);
  if (c->arena_pos + need > c->arena_bytes) {
    // the ring wraps: records written at its start may still be read by
    // launches in flight on any stream, so let the device drain first
    if (hipDeviceSynchronize() != hipSuccess) return nullptr;
    c->arena_pos = 0;
  }
  void* dst = c->arena + c->arena_pos;
  c->arena_pos += need;
  if (hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return nullptr;
  return dst;
}

// the table and evaluation records of a launch list in one copy (each copy
// of a few hundred bytes costs a blit of about 5 us on the stream); dta and
// dea are left untouched if the copy could not be enqueued
void upload_args(pnp_ctx c, const TableArgs* ta, size_t nta, const EvalArgs* ea, size_t nea, hipStream_t s,
                 const TableArgs*& dta, const EvalArgs*& dea) {
  const size_t off = up(sizeof(TableArgs) * nta);
  std::vector<char> buf(off + sizeof(EvalArgs) * nea);
  std::memcpy(buf.data(), ta, sizeof(TableArgs) * nta);
  std::memcpy(buf.data() + off, ea, sizeof(EvalArgs) * nea);
  const char* d = (const char*)upload(c, buf.data(), buf.size(), s);
  if (!d) return;
  dta = (const TableArgs*)d;
  dea = (const EvalArgs*)(d + off);
}

pnp_status device_check(pnp_ctx c, const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, PNP_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
  return PNP_OK;
}

pnp_status status_of(pnp_ctx c, const uint32_t st[2]) {
  if (st[0] == 0) return PNP_OK;
  const std::string at = " (first flat index " + std::to_string(st[1]) + ")";
  if (st[0] & kStPacking) return fail(c, PNP_E_PACKING, "weighted density n3 >= 1" + at);
  if (st[0] & kStNonFinite) return fail(c, PNP_E_NONFINITE, "non-finite value" + at);
  return fail(c, PNP_E_OVERFLOW, "exp(-beta mu_ex) overflows" + at);
}

pnp_status read_status(pnp_ctx c, const void* status_dev, hipStream_t s) {
  uint32_t st[2] = {0, 0};
  if (hipMemcpyAsync(st, status_dev, sizeof(st), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return device_check(c, "status read");
  return status_of(c, st);
}

// ---------------------------------------------------------------------------
// launchers per (precision, n): instantiated in their own translation units
// (pnp_ops.hip, one per precision and size), found here through ops_inst
// ---------------------------------------------------------------------------
template <typename T, int V>
const Ops* ops_for_n(int n) {
  if ((V & 1) && n > kNarrowMax) return nullptr;
  switch (n) {
    case 8: return ops_inst<T, 8, V>();
    case 16: return ops_inst<T, 16, V>();
    case 24: return ops_inst<T, 24, V>();
    case 32: return ops_inst<T, 32, V>();
    case 48: return ops_inst<T, 48, V>();
    case 64: return ops_inst<T, 64, V>();
    case 96: return ops_inst<T, 96, V>();
    case 128: return ops_inst<T, 128, V>();
    case 192: return (V & 1) ? nullptr : ops_inst<T, 192, V & 2>();
    case 256: return (V & 1) ? nullptr : ops_inst<T, 256, V & 2>();
    default: return nullptr;
  }
}

// variant: bit 0 narrow tile shape, bit 1 secondary FFT schedule
const Ops* ops_for(int precision, int n, int variant = 0) {
  const bool f = precision == PNP_MIXED;
  switch (variant & 3) {
    case 1: return f ? ops_for_n<float, 1>(n) : ops_for_n<double, 1>(n);
    case 2: return f ? ops_for_n<float, 2>(n) : ops_for_n<double, 2>(n);
    case 3: return f ? ops_for_n<float, 3>(n) : ops_for_n<double, 3>(n);
    default: return f ? ops_for_n<float, 0>(n) : ops_for_n<double, 0>(n);
  }
}

// The launch variant of each pass of one launch sequence: pass p runs the
// secondary FFT schedule when bit p of smask is set, and the narrow tile
// shape when bit p of mask is set and that shape exists.
struct OpsSel {
  const Ops* v[4] = {nullptr, nullptr, nullptr, nullptr};
  uint32_t mask = 0, smask = 0;
  int precision = PNP_FP64;
  const Ops* at(int pass) const {
    const int sch = ((smask >> pass) & 1u) ? 2 : 0;
    const Ops* o = ((mask >> pass) & 1u) ? v[sch | 1] : nullptr;
    return o ? o : v[sch];
  }
};

// instance-count class of a launch, part of the tile-shape key
int count_class(int count) { return count <= 1 ? 0 : count <= 3 ? 1 : count <= 15 ? 2 : 3; }

uint64_t tune_key(int precision, int n, int cls) { return ((uint64_t)precision << 40) | ((uint64_t)n << 8) | cls; }
uint64_t sched_key(int precision, int n) { return ((uint64_t)precision << 40) | (uint64_t)n; }

// The FFT schedule of (precision, n) before any tuning: the passes (numbered
// as pnp_profile_read orders them) on which the autotuner, run twice on an
// MI355X for one three-species instance with every term, chose the
// secondary schedule both times.
constexpr uint32_t passes(std::initializer_list<int> l) {
  uint32_t m = 0;
  for (int p : l) m |= 1u << p;
  return m;
}

struct SchedDefault {
  int n;
  uint32_t mixed, fp64;
};

constexpr SchedDefault kSchedDefault[] = {
    {8, passes({3, 7, 9}), passes({3, 7})},
    {16, passes({3, 4, 5, 6, 7, 8, 9}), passes({1, 3, 4, 6, 7, 9})},
    {24, passes({1, 4, 6, 9}), passes({1, 2, 4, 6, 8, 9})},
    {32, passes({1, 2, 3, 4, 5, 6, 7, 8, 9}), passes({1, 2, 3, 4, 6, 8, 9})},
    {48, passes({1, 9}), passes({1, 2, 6, 9})},
    {64, passes({1, 2, 3, 4, 5, 6, 7, 8, 9}), passes({1, 2, 4, 6, 8, 9})},
    {96, passes({1, 9}), passes({9})},
    {128, passes({1, 2, 3, 4, 6, 8, 9}), passes({1, 2, 4, 6, 8, 9})},
    {192, passes({1, 3, 7, 9}), passes({3, 9})},
    {256, passes({1, 9}), passes({1, 9})},
};

uint32_t default_sched(int precision, int n) {
  for (const SchedDefault& d : kSchedDefault)
    if (d.n == n) return precision == PNP_MIXED ? d.mixed : d.fp64;
  return 0u;
}

// The full launch sequence for `count` instances of one size and precision.
// Species counts of a launch list: the largest, and the largest among the
// instances with at most four species (0: none), which select the back-pass
// kernels.
struct SpeciesMix {
  int maxS = 1, small = 0;
  void add(int S) {
    maxS = std::max(maxS, S);
    if (S <= 4) small = std::max(small, S);
  }
};

inline SpeciesMix mix_of(int S) {
  SpeciesMix m;
  m.add(S);
  return m;
}

// Between two z passes the y and x passes of the Nyquist plane (kz = n/2)
// touch only that plane, so for large grids its tiles run as separate
// launches on the context's side stream: forked from the caller's stream
// after a z pass and joined back before the next one.  On large grids the
// main-array tiles of a y or x pass are whole rounds of the 256 compute
// units (2048 workgroups); launched together, the 16 Nyquist tiles would
// add a last, nearly empty round (measured at 256^3: the y and x passes
// 6-10 % longer), while on the side stream they run in the idle slots of
// the main launches.  The split is not used while a plan is being captured
// (every tile then runs on the capturing stream).
constexpr int kSplitMinN = 192;

struct Split {
  pnp_ctx c;
  hipStream_t s;
  bool on = false;
  Split(pnp_ctx ctx, hipStream_t stream, int n) : c(ctx), s(stream) {
    if (n < kSplitMinN || !c || c->capturing || c->side_failed) return;
    if (!c->side) {
      if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        c->side_failed = true;  // every tile stays on the caller's stream
        return;
      }
    }
    on = true;
  }
  // the side stream waits for all work enqueued on the caller's stream so far
  void fork() {
    if (!on) return;
    (void)hipEventRecord(c->ev_fork, s);
    (void)hipStreamWaitEvent(c->side, c->ev_fork, 0);
  }
  // the caller's stream waits for all work enqueued on the side stream so far
  void join() {
    if (!on) return;
    (void)hipEventRecord(c->ev_join, c->side);
    (void)hipStreamWaitEvent(s, c->ev_join, 0);
  }
  // stream of the Nyquist tiles, and the parts of the main launch
  int main_part() const { return on ? kPartMain : kPartAll; }
  hipStream_t nyq() const { return c->side; }
};

// ea: device arg tables; fmask: the hard-sphere functionals among the
// instances (1 Rosenfeld, 2 White Bear, 0 no HS term); sm: their species
// counts; n: the grid size of the launch list.
void run_sequence(pnp_ctx c, const OpsSel& op, const EvalArgs* ea, const TableArgs* ta, int count, int M,
                  int fmask, const SpeciesMix& sm, hipStream_t s, int n) {
  PassTimer pt{c, s};
  Split sp(c, s, n);
  const int mp = sp.main_part();
  // The radial tables are first read by the x passes (the forward one only in
  // FP64: the FP32 hard-sphere weights are evaluated in registers).  With the
  // side stream they are built there, beside the first y pass, and joined
  // before their first reader.  Beside the y pass (2 waves per SIMD) their
  // small workgroups fill idle register slots; beside the first z pass (4
  // waves per SIMD) they displaced its workgroups (256^3 mixed, the same
  // run: 1.657 ms per evaluation beside the y pass, 1.666 ms beside the z
  // pass).
  bool tab_pending = false;
  if (!sp.on) {
    pt.begin(0); op.at(0)->tables(ta, count, M, sm.maxS, s); pt.end();
  }
  pt.begin(1); op.at(1)->zfwd(ea, count, s); pt.end();
  sp.fork();
  if (sp.on) {
    PassTimer ps{c, sp.nyq()};
    ps.begin(0); op.at(0)->tables(ta, count, M, sm.maxS, sp.nyq()); ps.end();
    tab_pending = true;
  }
  pt.begin(2); op.at(2)->ystep(ea, count, 0, -1, true, mp, s); pt.end();
  if (sp.on) op.at(2)->ystep(ea, count, 0, -1, true, kPartNyquist, sp.nyq());
  if (fmask) {
    if (tab_pending && op.precision == PNP_FP64) {
      sp.join();
      tab_pending = false;
    }
    pt.begin(3); op.at(3)->xfwd(ea, count, mp, s); pt.end();
    if (sp.on) op.at(3)->xfwd(ea, count, kPartNyquist, sp.nyq());
    pt.begin(4); op.at(4)->ystep(ea, count, 1, kVecMode, false, mp, s); pt.end();
    if (sp.on) op.at(4)->ystep(ea, count, 1, kVecMode, false, kPartNyquist, sp.nyq());
    sp.join();
    tab_pending = false;
    pt.begin(5); op.at(5)->zderiv(ea, count, false, fmask, s); pt.end();
    sp.fork();
    pt.begin(6); op.at(6)->ystep(ea, count, 1, kVecMode, true, mp, s); pt.end();
    if (sp.on) op.at(6)->ystep(ea, count, 1, kVecMode, true, kPartNyquist, sp.nyq());
  }
  if (tab_pending) sp.join();
  pt.begin(7); op.at(7)->xback(ea, count, sm.small, sm.maxS > 4, mp, s); pt.end();
  if (sp.on) op.at(7)->xback(ea, count, sm.small, sm.maxS > 4, kPartNyquist, sp.nyq());
  pt.begin(8); op.at(8)->ystep(ea, count, 2, -1, false, mp, s); pt.end();
  if (sp.on) op.at(8)->ystep(ea, count, 2, -1, false, kPartNyquist, sp.nyq());
  sp.join();
  pt.begin(9); op.at(9)->zinv(ea, count, 2, s); pt.end();
}

// the FFT schedule of (precision, n) and the tuned tile shapes for a launch
// of `count` instances of it
OpsSel select_ops(pnp_ctx c, int precision, int n, int count) {
  OpsSel o;
  o.precision = precision;
  for (int v = 0; v < 4; ++v) o.v[v] = ops_for(precision, n, v);
  auto it = c->tune.find(tune_key(precision, n, count_class(count)));
  if (it != c->tune.end()) o.mask = it->second;
  auto is = c->sched.find(sched_key(precision, n));
  o.smask = is != c->sched.end() ? is->second : default_sched(precision, n);
  return o;
}

// One launch group of a batch: the valid requests of one (precision, n),
// with their argument records in request order.
struct Group {
  int precision = 0, n = 0;
  std::vector<int> ids;
  std::vector<TableArgs> ta;
  std::vector<EvalArgs> ea;
  int fmask = 0, M = 0;
  SpeciesMix mix;
};

// Validate every request (its status field receives the result) and build
// the argument records of the valid ones, grouped by (precision, n).
void prepare_batch(pnp_ctx ctx, int count, pnp_request* reqs, std::vector<Layout>& lay, std::vector<Group>& out) {
  std::map<std::pair<int, int>, std::vector<int>> groups;
  std::vector<Derived> der(count);
  lay.assign(count, Layout{});
  for (int r = 0; r < count; ++r) {
    pnp_request& q = reqs[r];
    q.status = PNP_OK;
    pnp_status st = validate(ctx, &q.grid, q.S, q.species, q.T, q.params, der[r], true);
    if (st == PNP_OK && (!q.rho || !q.mu_ex || !q.workspace)) st = fail(ctx, PNP_E_ARG, "null device pointer");
    if (st == PNP_OK && q.params->per_term) st = fail(ctx, PNP_E_ARG, "per_term is not available in batches");
    if (st == PNP_OK && ((uintptr_t)q.workspace % kAlign)) st = fail(ctx, PNP_E_ARG, "workspace alignment");
    if (st == PNP_OK) {
      const Derived& d = der[r];
      lay[r] = layout_of(d.n, q.S, d.precision, d.hs, d.ec || d.sw, false);
      if (q.workspace_bytes < lay[r].total) st = fail(ctx, PNP_E_NOMEM, "workspace too small");
    }
    q.status = st;
    if (st == PNP_OK) groups[{der[r].precision, der[r].n}].push_back(r);
  }
  out.clear();
  for (auto& kv : groups) {
    Group g;
    g.precision = kv.first.first;
    g.n = kv.first.second;
    g.ids = kv.second;
    const int cnt = (int)g.ids.size();
    g.ta.resize(cnt);
    g.ea.resize(cnt);
    for (int k = 0; k < cnt; ++k) {
      pnp_request& q = reqs[g.ids[k]];
      const Derived& d = der[g.ids[k]];
      const Layout& L = lay[g.ids[k]];
      char* w = (char*)q.workspace;
      const bool pairs = d.ec || d.sw;
      fill_table_args(g.ta[k], d, q.species, q.grid.h, q.params->sw_prefactor, d.ec, d.sw, w + L.hs,
                      pairs ? w + L.pair : nullptr, L.M);
      fill_eval_args(g.ea[k], d, q.species, L, w, q.rho);
      g.ea[k].out = q.mu_ex;
      g.ea[k].slot = q.slotboom;
      g.fmask |= hs_mask(d);
      g.mix.add(q.S);
      g.M = std::max(g.M, L.M);
    }
    out.push_back(std::move(g));
  }
}

}  // namespace

// A captured evaluation: argument records in a device block of its own and a
// HIP graph of every launch, replayed on any stream.
struct pnp_plan_s {
  pnp_ctx ctx = nullptr;
  int count = 0;
  std::vector<int32_t> valid;       // creation-time status of each request
  std::vector<const void*> status;  // device status word of each valid request
  void* block = nullptr;            // argument records (device)
  size_t block_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// ===========================================================================
// C ABI
// ===========================================================================
// The per-term evaluation: mu3 = [hs, el, sh] ([3][S][N]) and slot =
// exp(-(hs + el + sh)); phi_part (or null) receives the derivative pass's
// per-workgroup sums of Phi_hs.
static pnp_status enqueue_per_term(pnp_ctx ctx, const Derived& d, const pnp_grid* g, const pnp_species* sp,
                          const double* rho, const pnp_params* p, const Layout& L, char* w, double* mu,
                          double* slot, double* phi_part, hipStream_t s) {
  const int S = d.S;
  const bool pairs = d.ec || d.sw;
  const OpsSel os = select_ops(ctx, d.precision, d.n, 1);
  const double sw_c = p->sw_prefactor;
  const long n3 = (long)d.n * d.n * d.n;
  // tables: HS (+ EC pairs into pair), SW pairs into pair2
  TableArgs ta[2];
  fill_table_args(ta[0], d, sp, g->h, sw_c, d.ec, false, w + L.hs, pairs ? w + L.pair : nullptr, L.M);
  fill_table_args(ta[1], d, sp, g->h, sw_c, false, d.sw, w + L.hs, pairs ? w + L.pair2 : nullptr,
                  L.M);
  // four argument records: forward half, hs-only, el-only, sh-only
  EvalArgs ea[4];
  for (int k = 0; k < 4; ++k) {
    fill_eval_args(ea[k], d, sp, L, w, rho);
    ea[k].slot = nullptr;
    ea[k].phi_part = phi_part;
  }
  ea[0].out = mu;
  ea[1].out = mu; ea[1].pair_on = 0;
  for (int i = 0; i < S; ++i) ea[1].cfin[i] = 0.0;
  ea[2].out = mu + (long)S * n3; ea[2].hs_on = 0; ea[2].pair_on = d.ec;
  ea[3].out = mu + 2L * S * n3; ea[3].hs_on = 0; ea[3].pair_on = d.sw; ea[3].pair_tab = w + L.pair2;
  for (int i = 0; i < S; ++i) ea[3].cfin[i] = 0.0;
  if (!d.ec) for (int i = 0; i < S; ++i) ea[2].cfin[i] = 0.0;
  if (!d.hs) ea[1].hs_on = 0;
  const TableArgs* dta = nullptr;
  const EvalArgs* dea = nullptr;
  upload_args(ctx, ta, sizeof(ta) / sizeof(TableArgs), ea, sizeof(ea) / sizeof(EvalArgs), s, dta, dea);
  if (!dta || !dea) return device_check(ctx, "argument upload");
  PassTimer pt{ctx, s};
  pt.begin(0);
  os.at(0)->tables(dta, 1, L.M, S, s);
  if (d.sw) os.at(0)->tables(dta + 1, 1, L.M, S, s);
  pt.end();
  Split sq(ctx, s, d.n);
  const int mp = sq.main_part();
  pt.begin(1); os.at(1)->zfwd(dea, 1, s); pt.end();
  sq.fork();
  pt.begin(2); os.at(2)->ystep(dea, 1, 0, -1, true, mp, s); pt.end();
  if (sq.on) os.at(2)->ystep(dea, 1, 0, -1, true, kPartNyquist, sq.nyq());
  if (d.hs) {
    pt.begin(3); os.at(3)->xfwd(dea, 1, mp, s); pt.end();
    if (sq.on) os.at(3)->xfwd(dea, 1, kPartNyquist, sq.nyq());
    pt.begin(4); os.at(4)->ystep(dea, 1, 1, kVecMode, false, mp, s); pt.end();
    if (sq.on) os.at(4)->ystep(dea, 1, 1, kVecMode, false, kPartNyquist, sq.nyq());
    sq.join();
    pt.begin(5); os.at(5)->zderiv(dea, 1, phi_part != nullptr, hs_mask(d), s); pt.end();
    sq.fork();
    pt.begin(6); os.at(6)->ystep(dea, 1, 1, kVecMode, true, mp, s); pt.end();
    if (sq.on) os.at(6)->ystep(dea, 1, 1, kVecMode, true, kPartNyquist, sq.nyq());
  }
  for (int k = 1; k < 4; ++k) {
    pt.begin(7); os.at(7)->xback(dea + k, 1, S <= 4 ? S : 0, S > 4, mp, s); pt.end();
    if (sq.on) os.at(7)->xback(dea + k, 1, S <= 4 ? S : 0, S > 4, kPartNyquist, sq.nyq());
    pt.begin(8); os.at(8)->ystep(dea + k, 1, 2, -1, false, mp, s); pt.end();
    if (sq.on) os.at(8)->ystep(dea + k, 1, 2, -1, false, kPartNyquist, sq.nyq());
    sq.join();
    pt.begin(9); os.at(9)->zinv(dea + k, 1, 2, s); pt.end();
    if (k < 3) sq.fork();  // the next term's Nyquist tiles rewrite what this z pass read
  }
  const long sn3 = (long)S * n3;
  const int blocks = (int)std::min<long>((sn3 + 255) / 256, 4096);
  hipLaunchKernelGGL(k_sum_exp, dim3(blocks), dim3(256), 0, s, (const double*)mu, slot, sn3,
                     (uint32_t*)(w + L.status));
  return device_check(ctx, "launch");
}

extern "C" {

pnp_status pnp_create(int device, pnp_ctx* out) {
  if (!out) return PNP_E_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return PNP_E_DEVICE;
  pnp_ctx c = new pnp_ctx_s();
  c->device = device;
  c->arena_bytes = 4u << 20;
  if (hipSetDevice(device) != hipSuccess || hipMalloc((void**)&c->arena, c->arena_bytes) != hipSuccess) {
    delete c;
    return PNP_E_DEVICE;
  }
  c->scratch = scratch_address(device);  // with `device` current; null: the no-alloc call reports it
  *out = c;
  return PNP_OK;
}

void pnp_destroy(pnp_ctx c) {
  if (!c) return;
  hipSetDevice(c->device);
  if (c->arena) {
    hipDeviceSynchronize();
    hipFree(c->arena);
  }
  if (c->side) (void)hipStreamDestroy(c->side);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  for (hipStream_t x : c->br) (void)hipStreamDestroy(x);
  for (hipEvent_t e : c->br_done) (void)hipEventDestroy(e);
  if (c->br_fork) (void)hipEventDestroy(c->br_fork);
  for (auto& o : c->ev_open) { hipEventDestroy(o.second.first); hipEventDestroy(o.second.second); }
  for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
  delete c;
}

pnp_status pnp_profile_enable(pnp_ctx c, int32_t enable) {
  if (!c) return PNP_E_ARG;
  c->prof = enable != 0;
  return PNP_OK;
}

pnp_status pnp_profile_select(pnp_ctx c, uint32_t mask) {
  if (!c) return PNP_E_ARG;
  c->prof_mask = mask;
  return PNP_OK;
}

pnp_status pnp_profile_read(pnp_ctx c, double* ms, int32_t* launches, int32_t n, int32_t reset) {
  if (!c) return PNP_E_ARG;
  if (hipSetDevice(c->device) != hipSuccess) return device_check(c, "set device");
  for (auto& o : c->ev_open) {
    float t = 0.f;
    if (hipEventSynchronize(o.second.second) != hipSuccess ||
        hipEventElapsedTime(&t, o.second.first, o.second.second) != hipSuccess)
      return device_check(c, "event read");
    c->prof_ms[o.first] += (double)t;
    c->prof_n[o.first] += 1;
    c->ev_pool.push_back(o.second.first);
    c->ev_pool.push_back(o.second.second);
  }
  c->ev_open.clear();
  for (int i = 0; i < n && i < PNP_NUM_PASSES; ++i) {
    if (ms) ms[i] = c->prof_ms[i];
    if (launches) launches[i] = c->prof_n[i];
  }
  if (reset)
    for (int i = 0; i < PNP_NUM_PASSES; ++i) { c->prof_ms[i] = 0.0; c->prof_n[i] = 0; }
  return PNP_OK;
}

const char* pnp_last_error(pnp_ctx c) { return c ? c->err.c_str() : "null context"; }

int pnp_supported_size(int32_t n) { return size_ok(n) ? 1 : 0; }

pnp_status pnp_workspace_bytes(pnp_ctx ctx, const pnp_grid* g, int32_t S, const pnp_params* p, size_t* bytes) {
  if (!ctx || !g || !p || !bytes) return fail(ctx, PNP_E_ARG, "null argument");
  const bool aperiodic = p->flags & PNP_FLAG_APERIODIC;
  if (g->nx != g->ny || g->ny != g->nz ||
      (aperiodic ? !(g->nx >= 4 && g->nx <= 128 && size_ok(2 * g->nx)) : !size_ok(g->nx)))
    return fail(ctx, PNP_E_UNSUPPORTED_SIZE, "unsupported grid");
  if (S < 1 || S > kMaxSpecies) return fail(ctx, PNP_E_ARG, "species count must be in [1, 8]");
  if (p->precision != PNP_FP64 && p->precision != PNP_MIXED) return fail(ctx, PNP_E_ARG, "bad precision");
  const bool hs = p->terms & (PNP_TERM_HS | PNP_TERM_HS_WB), pairs = p->terms & (PNP_TERM_EC | PNP_TERM_SW);
  *bytes = aperiodic ? layout_aperiodic(2 * g->nx, S, p->precision, hs, pairs, p->terms & PNP_TERM_EC, p->per_term).total
                     : layout_of(g->nx, S, p->precision, hs, pairs, p->per_term).total;
  return PNP_OK;
}

// The aperiodic evaluation (Sec. 3.4): extend, the EC response to the
// domain's bulk densities (EC only), the evaluation of the extended densities
// on the doubled grid, and the domain part of their difference.
static pnp_status enqueue_aperiodic(pnp_ctx ctx, const Derived& d, const pnp_grid* g, const pnp_species* sp,
                                    const double* rho, const pnp_params* p, const LayoutAp& A, char* w, double* mu,
                                    double* slot, hipStream_t s) {
  const int S = d.S;
  const Layout& L = A.L;
  const bool pairs = d.ec || d.sw;
  double* muA = (double*)(w + A.muA);
  double* muB = d.ec ? (double*)(w + A.muB) : nullptr;
  const OpsSel ops = select_ops(ctx, d.precision, d.n, 1);
  if (d.ec) {
    // -sum_j C_ij (*) rho_b,j chi_domain: the EC term alone, no constant
    Derived dB = d;
    dB.hs = dB.wb = dB.sw = false;
    TableArgs ta;
    fill_table_args(ta, dB, sp, g->h, p->sw_prefactor, true, false, w + L.hs, w + L.pair, L.M);
    EvalArgs ea;
    fill_eval_args(ea, dB, sp, L, w, nullptr);
    ea.ext_bulk = 1;
    for (int i = 0; i < S; ++i) {
      ea.cfin[i] = 0.0;
      ea.ext_val[i] = sp[i].rho_bulk;
    }
    ea.out = muB;
    ea.slot = nullptr;
    const TableArgs* dta = nullptr;
    const EvalArgs* dea = nullptr;
    upload_args(ctx, &ta, 1, &ea, 1, s, dta, dea);
    if (!dta || !dea) return device_check(ctx, "argument upload");
    run_sequence(ctx, ops, dea, dta, 1, L.M, 0, mix_of(S), s, d.n);
  }
  // the extended densities (their status word starts clean here)
  if (!p->per_term) {
    TableArgs ta;
    fill_table_args(ta, d, sp, g->h, p->sw_prefactor, d.ec, d.sw, w + L.hs, pairs ? w + L.pair : nullptr, L.M);
    EvalArgs ea;
    fill_eval_args(ea, d, sp, L, w, rho);
    ea.out = muA;
    ea.slot = nullptr;
    const TableArgs* dta = nullptr;
    const EvalArgs* dea = nullptr;
    upload_args(ctx, &ta, 1, &ea, 1, s, dta, dea);
    if (!dta || !dea) return device_check(ctx, "argument upload");
    run_sequence(ctx, ops, dea, dta, 1, L.M, hs_mask(d), mix_of(S), s, d.n);
  } else {
    const pnp_status st = enqueue_per_term(ctx, d, g, sp, rho, p, L, w, muA, nullptr, nullptr, s);
    if (st != PNP_OK) return st;
  }
  const long N = (long)d.n_dom * d.n_dom * d.n_dom;
  const int cb = (int)std::min<long>((S * N + 255) / 256, 8192);
  hipLaunchKernelGGL(k_crop, dim3(cb), dim3(256), 0, s, (const double*)muA, (const double*)muB,
                     p->per_term ? 3 : 1, S, d.n_dom, mu, slot, (uint32_t*)(w + L.status));
  return device_check(ctx, "launch");
}

pnp_status pnp_cdft_mu_ex(pnp_ctx ctx, const pnp_grid* g, int32_t S, const pnp_species* sp, const double* rho,
                          double T, const pnp_params* p, double* mu, double* slot, void* ws, size_t ws_bytes,
                          void* stream) {
  Derived d;
  pnp_status st = validate(ctx, g, S, sp, T, p, d, true, true);
  if (st != PNP_OK) return st;
  if (!rho || !mu || !ws) return fail(ctx, PNP_E_ARG, "null device pointer");
  if ((uintptr_t)ws % kAlign) return fail(ctx, PNP_E_ARG, "workspace must be 256-byte aligned");
  if (d.aperiodic) {
    const LayoutAp A = layout_aperiodic(d.n, S, d.precision, d.hs, d.ec || d.sw, d.ec, p->per_term);
    if (ws_bytes < A.total) return fail(ctx, PNP_E_NOMEM, "workspace too small: need " + std::to_string(A.total));
    if (hipSetDevice(ctx->device) != hipSuccess) return device_check(ctx, "set device");
    hipStream_t s = (hipStream_t)stream;
    st = enqueue_aperiodic(ctx, d, g, sp, rho, p, A, (char*)ws, mu, slot, s);
    if (st != PNP_OK) return st;
    if (p->flags & PNP_FLAG_ASYNC) return PNP_OK;
    return read_status(ctx, (char*)ws + A.L.status, s);
  }
  const bool pairs = d.ec || d.sw;
  const Layout L = layout_of(d.n, S, d.precision, d.hs, pairs, p->per_term);
  if (ws_bytes < L.total) return fail(ctx, PNP_E_NOMEM, "workspace too small: need " + std::to_string(L.total));
  if (hipSetDevice(ctx->device) != hipSuccess) return device_check(ctx, "set device");
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  const double sw_c = p->sw_prefactor;
  if (!p->per_term) {
    TableArgs ta;
    fill_table_args(ta, d, sp, g->h, sw_c, d.ec, d.sw, w + L.hs, pairs ? w + L.pair : nullptr, L.M);
    EvalArgs ea;
    fill_eval_args(ea, d, sp, L, w, rho);
    ea.out = mu;
    ea.slot = slot;
    const TableArgs* dta = nullptr;
    const EvalArgs* dea = nullptr;
    upload_args(ctx, &ta, 1, &ea, 1, s, dta, dea);
    if (!dta || !dea) return device_check(ctx, "argument upload");
    run_sequence(ctx, select_ops(ctx, d.precision, d.n, 1), dea, dta, 1, L.M, hs_mask(d), mix_of(S), s, d.n);
  } else {
    st = enqueue_per_term(ctx, d, g, sp, rho, p, L, w, mu, slot, nullptr, s);
    if (st != PNP_OK) return st;
  }
  st = device_check(ctx, "launch");
  if (st != PNP_OK) return st;
  if (p->flags & PNP_FLAG_ASYNC) return PNP_OK;
  return read_status(ctx, w + L.status, s);
}

pnp_status pnp_cdft_mu_ex_noalloc(pnp_ctx ctx, const pnp_grid* g, int32_t S, const pnp_species* sp,
                                  const double* rho, double T, const pnp_params* p, double* mu, double* slot,
                                  void* stream) {
  if (!ctx) return PNP_E_ARG;
  if (!ctx->scratch) return fail(ctx, PNP_E_DEVICE, "the static scratch array has no device address on this device");
  size_t need = 0;
  pnp_status st = pnp_workspace_bytes(ctx, g, S, p, &need);
  if (st != PNP_OK) return st;
  if (need > kScratchBytes)
    return fail(ctx, PNP_E_NOMEM, "this evaluation needs " + std::to_string(need) + " bytes of scratch; the static "
                                  "scratch array holds " + std::to_string(kScratchBytes));
  if (hipSetDevice(ctx->device) != hipSuccess) return device_check(ctx, "set device");
  // argument records are copied from host memory at call time: a captured
  // copy would read them again at every replay
  hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing((hipStream_t)stream, &capture) != hipSuccess) return device_check(ctx, "capture query");
  if (capture != hipStreamCaptureStatusNone)
    return fail(ctx, PNP_E_ARG, "pnp_cdft_mu_ex_noalloc cannot be recorded into a graph");
  // the evaluation of pnp_cdft_mu_ex with this device's scratch as workspace;
  // every region it reads is written earlier in the same call (the status
  // words are cleared by the first pass)
  return pnp_cdft_mu_ex(ctx, g, S, sp, rho, T, p, mu, slot, ctx->scratch, kScratchBytes, stream);
}

pnp_status pnp_free_energy(pnp_ctx ctx, const pnp_grid* g, int32_t S, const pnp_species* sp, const double* rho,
                           double T, const pnp_params* p, double* energies, double* mu3, void* ws,
                           size_t ws_bytes, void* stream) {
  Derived d;
  pnp_status st = validate(ctx, g, S, sp, T, p, d, true);
  if (st != PNP_OK) return st;
  if (!rho || !mu3 || !ws || !energies) return fail(ctx, PNP_E_ARG, "null pointer");
  if ((uintptr_t)ws % kAlign) return fail(ctx, PNP_E_ARG, "workspace must be 256-byte aligned");
  const bool pairs = d.ec || d.sw;
  const Layout L = layout_of(d.n, S, d.precision, d.hs, pairs, true);
  if (ws_bytes < L.total) return fail(ctx, PNP_E_NOMEM, "workspace too small: need " + std::to_string(L.total));
  if (hipSetDevice(ctx->device) != hipSuccess) return device_check(ctx, "set device");
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  double* phi_part = (double*)(w + L.energy);
  double* part = phi_part + (size_t)d.n * d.n;
  double* res = part + 2 * kEnergyBlocks;
  st = enqueue_per_term(ctx, d, g, sp, rho, p, L, w, mu3, nullptr, d.hs ? phi_part : nullptr, s);
  if (st != PNP_OK) return st;
  const long n3 = (long)d.n * d.n * d.n;
  double rb[2 * kMaxSpecies];
  for (int i = 0; i < S; ++i) {
    rb[2 * i] = sp[i].rho_bulk;
    rb[2 * i + 1] = d.ec ? sp[i].mu_el_bulk : 0.0;
  }
  const double* drb = (const double*)upload(ctx, rb, sizeof(double) * 2 * S, s);
  if (!drb) return device_check(ctx, "argument upload");
  hipLaunchKernelGGL(k_energy_part, dim3(kEnergyBlocks), dim3(256), 0, s, rho, (const double*)mu3, n3, (int)S, drb,
                     part);
  const double h3 = g->h * g->h * g->h;
  // F_el = h^3/2 sum drho (mu_el + mu_el[bulk]); F_sh = h^3 / (2 c_sw) sum rho mu_sh (Sec. 2.3.2, 2.3.4)
  const double el_scale = d.ec ? 0.5 * h3 : 0.0;
  const double sh_scale = (d.sw && p->sw_prefactor != 0.0) ? h3 / (2.0 * p->sw_prefactor) : 0.0;
  const Ops* op = select_ops(ctx, d.precision, d.n, 1).at(5);  // the derivative pass's launch
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, s, (const double*)phi_part,
                     d.hs ? op->zderiv_tiles : 0, (const double*)part, kEnergyBlocks, h3, el_scale, sh_scale, res);
  st = device_check(ctx, "energy launch");
  if (st != PNP_OK) return st;
  if (hipMemcpyAsync(energies, res, 4 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
    return device_check(ctx, "energy read");
  return read_status(ctx, w + L.status, s);
}

pnp_status pnp_equilibrium(pnp_ctx ctx, const pnp_grid* g, int32_t S, const pnp_species* sp, double T,
                           const pnp_params* p, const double* beta_v, double* rho, double* mu, double lambda,
                           double tol, int32_t max_iter, int32_t* iters, double* residual, void* ws,
                           size_t ws_bytes, void* stream) {
  Derived d;
  pnp_status st = validate(ctx, g, S, sp, T, p, d, true);
  if (st != PNP_OK) return st;
  if (!rho || !mu || !ws || !iters || !residual) return fail(ctx, PNP_E_ARG, "null pointer");
  if (!(lambda > 0.0 && lambda <= 1.0)) return fail(ctx, PNP_E_ARG, "lambda must be in (0, 1]");
  if (!(tol >= 0.0) || max_iter < 1) return fail(ctx, PNP_E_ARG, "tol must be >= 0 and max_iter >= 1");
  if (p->per_term) return fail(ctx, PNP_E_ARG, "per_term is not available here");
  if ((uintptr_t)ws % kAlign) return fail(ctx, PNP_E_ARG, "workspace must be 256-byte aligned");
  const uint32_t fixed = fixed_mask(S, sp);
  for (int i = 0; i < S; ++i)
    if (!((fixed >> i) & 1u) && !(sp[i].rho_bulk > 0.0))
      return fail(ctx, PNP_E_ARG, "bulk densities of mobile species must be > 0");
  const bool pairs = d.ec || d.sw;
  const Layout L = layout_of(d.n, S, d.precision, d.hs, pairs, false);
  if (ws_bytes < L.total) return fail(ctx, PNP_E_NOMEM, "workspace too small: need " + std::to_string(L.total));
  double mb[kMaxSpecies];
  st = pnp_bulk_mu_ex(ctx, S, sp, T, p, mb);
  if (st != PNP_OK) return st;
  if (hipSetDevice(ctx->device) != hipSuccess) return device_check(ctx, "set device");
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)ws;
  unsigned long long* res = (unsigned long long*)(w + L.energy);
  const long n3 = (long)d.n * d.n * d.n;
  double rbmb[2 * kMaxSpecies];
  for (int i = 0; i < S; ++i) { rbmb[2 * i] = sp[i].rho_bulk; rbmb[2 * i + 1] = mb[i]; }
  TableArgs ta;
  fill_table_args(ta, d, sp, g->h, p->sw_prefactor, d.ec, d.sw, w + L.hs, pairs ? w + L.pair : nullptr, L.M);
  EvalArgs ea;
  fill_eval_args(ea, d, sp, L, w, rho);
  ea.out = mu;
  ea.slot = nullptr;
  const TableArgs* dta = nullptr;
  const EvalArgs* dea = nullptr;
  upload_args(ctx, &ta, 1, &ea, 1, s, dta, dea);
  const double* drb = (const double*)upload(ctx, rbmb, sizeof(double) * 2 * S, s);
  if (!dta || !dea || !drb) return device_check(ctx, "argument upload");
  const int blocks = (int)std::min<long>(((long)S * n3 + 255) / 256, 4096);
  *iters = 0;
  *residual = INFINITY;
  for (int it = 1; it <= max_iter; ++it) {
    run_sequence(ctx, select_ops(ctx, d.precision, d.n, 1), dea, dta, 1, L.M, hs_mask(d), mix_of(S), s, d.n);
    if (hipMemsetAsync(res, 0, sizeof(unsigned long long), s) != hipSuccess) return device_check(ctx, "reset");
    hipLaunchKernelGGL(k_picard, dim3(blocks), dim3(256), 0, s, rho, (const double*)mu, beta_v, n3, (int)S, drb,
                       lambda, res, fixed);
    st = device_check(ctx, "picard launch");
    if (st != PNP_OK) return st;
    unsigned long long rbits = 0;
    uint32_t stw[2] = {0, 0};
    if (hipMemcpyAsync(&rbits, res, sizeof(rbits), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(stw, w + L.status, sizeof(stw), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return device_check(ctx, "residual read");
    st = status_of(ctx, stw);
    *iters = it;
    std::memcpy(residual, &rbits, sizeof(double));
    if (st != PNP_OK) return st;
    if (!std::isfinite(*residual)) return fail(ctx, PNP_E_NONFINITE, "non-finite density update");
    if (*residual <= tol) break;
  }
  return PNP_OK;
}

pnp_status pnp_weighted_densities(pnp_ctx ctx, const pnp_grid* g, int32_t S, const pnp_species* sp,
                                  const double* rho, const pnp_params* p, double* n_out, void* ws,
                                  size_t ws_bytes, void* stream) {
  Derived d;
  pnp_params q = *p;
  q.terms = PNP_TERM_HS;
  q.per_term = 0;
  pnp_status st = validate(ctx, g, S, sp, 300.0, &q, d, false);
  if (st != PNP_OK) return st;
  if (!rho || !n_out || !ws) return fail(ctx, PNP_E_ARG, "null device pointer");
  if ((uintptr_t)ws % kAlign) return fail(ctx, PNP_E_ARG, "workspace must be 256-byte aligned");
  const Layout L = layout_of(d.n, S, d.precision, true, false, false);
  if (ws_bytes < L.total) return fail(ctx, PNP_E_NOMEM, "workspace too small: need " + std::to_string(L.total));
  if (hipSetDevice(ctx->device) != hipSuccess) return device_check(ctx, "set device");
  hipStream_t s = (hipStream_t)stream;
  const OpsSel os = select_ops(ctx, d.precision, d.n, 1);
  char* w = (char*)ws;
  TableArgs ta;
  fill_table_args(ta, d, sp, g->h, 0.0, false, false, w + L.hs, nullptr, L.M);
  EvalArgs ea;
  fill_eval_args(ea, d, sp, L, w, rho);
  ea.final_mode = 0;
  ea.nreal = kFields;
  ea.out = n_out;
  // the z components of the vector densities are i s_z Q_b until the z pass
  ea.zmul_mask = (1u << kSlotZ) | (1u << (kSlotZ + kVecStride));
  const TableArgs* dta = nullptr;
  const EvalArgs* dea = nullptr;
  upload_args(ctx, &ta, 1, &ea, 1, s, dta, dea);
  if (!dta || !dea) return device_check(ctx, "argument upload");
  os.at(0)->tables(dta, 1, L.M, S, s);
  os.at(1)->zfwd(dea, 1, s);
  os.at(2)->ystep(dea, 1, 0, -1, true, kPartAll, s);
  os.at(3)->xfwd(dea, 1, kPartAll, s);
  os.at(4)->ystep(dea, 1, 1, kVecMode, false, kPartAll, s);
  os.at(9)->zinv(dea, 1, 1, s);
  st = device_check(ctx, "launch");
  if (st != PNP_OK) return st;
  if (p->flags & PNP_FLAG_ASYNC) return PNP_OK;
  return read_status(ctx, w + L.status, s);
}

pnp_status pnp_sphere_quadrature(pnp_ctx ctx, const pnp_grid* g, int32_t F, const double* f,
                                 const double* radius, int32_t order, int32_t precision,
                                 uint32_t flags, double* out, void* stream) {
  if (!ctx) return PNP_E_ARG;
  if (!g || !f || !radius || !out) return fail(ctx, PNP_E_ARG, "null pointer");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(ctx, PNP_E_ARG, "grid extents must be >= 1");
  const size_t N = (size_t)g->nx * g->ny * g->nz;
  if (N > (size_t)INT32_MAX) return fail(ctx, PNP_E_UNSUPPORTED_SIZE, "grid has more than 2^31 - 1 points");
  if (!(g->h > 0.0) || !std::isfinite(g->h)) return fail(ctx, PNP_E_ARG, "grid spacing must be positive");
  if (F < 1 || F > kQuadMaxFields) return fail(ctx, PNP_E_ARG, "field count must be in [1, 64]");
  if (order < 1 || order > 64) return fail(ctx, PNP_E_ARG, "order must be in [1, 64]");
  if (precision != PNP_FP64 && precision != PNP_MIXED) return fail(ctx, PNP_E_ARG, "bad precision");
  if (flags & ~(uint32_t)(PNP_FLAG_APERIODIC | PNP_FLAG_ASYNC | PNP_FLAG_CUBIC))
    return fail(ctx, PNP_E_ARG, "unsupported flag");
  for (int i = 0; i < F; ++i)
    if (!(radius[i] > 0.0) || !std::isfinite(radius[i]) || radius[i] / g->h > 16.0)
      return fail(ctx, PNP_E_ARG, "field " + std::to_string(i) + ": radius must be in (0, 16 h]");
  std::vector<QuadStencil> st;
  int H = 0;
  for (int i = 0; i < F; ++i) {
    st.push_back(build_quad_stencil(radius[i] / g->h, radius[i], order, (flags & PNP_FLAG_CUBIC) != 0));
    H = std::max(H, st.back().reach);
  }
  H = std::max(H, 1);
  const int max_reach = precision == PNP_FP64 ? quad_max_reach<double>() : quad_max_reach<float>();
  if (H > max_reach)
    return fail(ctx, PNP_E_UNSUPPORTED_SIZE, "sphere reach " + std::to_string(H) +
                                                 " grid points does not fit the LDS tile (R / h too large)");
  QuadArgs a;
  a.f = f;
  a.out = out;
  a.nx = g->nx;
  a.ny = g->ny;
  a.nz = g->nz;
  a.H = H;
  const int ly = kQuadTY + 2 * H, lz = kQuadTZ + 2 * H;  // the kernel's tile pitches
  a.tiles_y = (g->ny + kQuadTY - 1) / kQuadTY;
  a.tiles_z = (g->nz + kQuadTZ - 1) / kQuadTZ;
  a.aperiodic = (flags & PNP_FLAG_APERIODIC) ? 1 : 0;
  size_t entries_at = 0;
  std::vector<unsigned char> buf = precision == PNP_FP64 ? pack_quad<double>(st, ly, lz, entries_at)
                                                         : pack_quad<float>(st, ly, lz, entries_at);
  if (buf.size() > ctx->arena_bytes / 2)
    return fail(ctx, PNP_E_UNSUPPORTED_SIZE, "stencils too large for one call: pass fewer fields");
  if (hipSetDevice(ctx->device) != hipSuccess) return device_check(ctx, "set device");
  hipStream_t s = (hipStream_t)stream;
  // the stencil is copied from host memory freed on return: a captured copy
  // would read it at every replay
  hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &capture) != hipSuccess) return device_check(ctx, "capture query");
  if (capture != hipStreamCaptureStatusNone)
    return fail(ctx, PNP_E_ARG, "pnp_sphere_quadrature cannot be recorded into a graph");
  const char* dev = (const char*)upload(ctx, buf.data(), buf.size(), s);
  if (!dev) return device_check(ctx, "stencil upload");
  a.begin = (const int32_t*)dev;
  a.entries = dev + entries_at;
  const hipError_t e = precision == PNP_FP64 ? launch_sphere_quad<double>(a, F, s)
                                             : launch_sphere_quad<float>(a, F, s);
  if (e != hipSuccess) return fail(ctx, PNP_E_DEVICE, std::string("sphere quadrature launch: ") + hipGetErrorString(e));
  if (flags & PNP_FLAG_ASYNC) return PNP_OK;
  if (hipStreamSynchronize(s) != hipSuccess) return device_check(ctx, "sphere quadrature");
  return PNP_OK;
}

// At least k branch streams with their join events (and the fork event);
// false (and every group stays on the caller's stream) if they cannot be made.
static bool branch_streams(pnp_ctx c, size_t k) {
  if (c->br_failed) return false;
  bool ok = c->br_fork || hipEventCreateWithFlags(&c->br_fork, hipEventDisableTiming) == hipSuccess;
  while (ok && c->br.size() < k) {
    hipStream_t x = nullptr;
    hipEvent_t e = nullptr;
    ok = hipStreamCreateWithFlags(&x, hipStreamNonBlocking) == hipSuccess;
    if (ok) ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    if (x) c->br.push_back(x);
    if (e) c->br_done.push_back(e);
    ok = ok && c->br.size() == c->br_done.size();
  }
  if (!ok) {
    (void)hipGetLastError();
    c->br_failed = true;
  }
  return ok;
}

pnp_status pnp_batch_mu_ex(pnp_ctx ctx, int32_t count, pnp_request* reqs, void* stream) {
  if (!ctx) return PNP_E_ARG;
  if (count < 0 || (count > 0 && !reqs)) return fail(ctx, PNP_E_ARG, "bad request array");
  if (hipSetDevice(ctx->device) != hipSuccess) return device_check(ctx, "set device");
  hipStream_t s = (hipStream_t)stream;
  std::vector<Layout> lay;
  std::vector<Group> groups;
  prepare_batch(ctx, count, reqs, lay, groups);
  // Grid sizes below kSplitMinN leave most of the chip idle in their
  // launches: with two or more of them each runs on a branch stream of its
  // own, forked from the caller's stream and joined back before the status
  // reads (the groups share no buffer, and every upload takes its own arena
  // slot).  Larger sizes fill the chip, use the side stream, and stay on the
  // caller's stream, beside the branches.
  size_t nsmall = 0;
  for (const Group& g : groups)
    if (g.n < kSplitMinN) ++nsmall;
  const bool fork = nsmall >= 2 && branch_streams(ctx, nsmall);
  if (fork && hipEventRecord(ctx->br_fork, s) != hipSuccess) return device_check(ctx, "batch fork");
  size_t b = 0;
  for (const Group& g : groups) {
    const int cnt = (int)g.ids.size();
    const bool branch = fork && g.n < kSplitMinN;
    hipStream_t gs = branch ? ctx->br[b] : s;
    if (branch && hipStreamWaitEvent(gs, ctx->br_fork, 0) != hipSuccess) return device_check(ctx, "batch fork");
    const TableArgs* dta = nullptr;
    const EvalArgs* dea = nullptr;
    upload_args(ctx, g.ta.data(), cnt, g.ea.data(), cnt, gs, dta, dea);
    if (!dta || !dea) return device_check(ctx, "argument upload");
    run_sequence(ctx, select_ops(ctx, g.precision, g.n, cnt), dea, dta, cnt, g.M, g.fmask, g.mix, gs, g.n);
    if (branch) {
      if (hipEventRecord(ctx->br_done[b], gs) != hipSuccess || hipStreamWaitEvent(s, ctx->br_done[b], 0) != hipSuccess)
        return device_check(ctx, "batch join");
      ++b;
    }
  }
  pnp_status st = device_check(ctx, "batch launch");
  if (st != PNP_OK) return st;
  bool async = false;
  for (int r = 0; r < count; ++r)
    if (reqs[r].status == PNP_OK && (reqs[r].params->flags & PNP_FLAG_ASYNC)) async = true;
  if (async) return PNP_OK;
  // one synchronisation for the whole batch, then each request's own status
  std::vector<uint32_t> words(2 * (size_t)count, 0u);
  for (int r = 0; r < count; ++r)
    if (reqs[r].status == PNP_OK)
      if (hipMemcpyAsync(&words[2 * r], (char*)reqs[r].workspace + lay[r].status, 8, hipMemcpyDeviceToHost, s) !=
          hipSuccess)
        return device_check(ctx, "status read");
  if (hipStreamSynchronize(s) != hipSuccess) return device_check(ctx, "batch sync");
  for (int r = 0; r < count; ++r)
    if (reqs[r].status == PNP_OK) reqs[r].status = status_of(ctx, &words[2 * r]);
  return PNP_OK;
}

pnp_status pnp_plan_create(pnp_ctx ctx, int32_t count, pnp_request* reqs, const pnp_relax_spec* relax,
                           pnp_plan* out) {
  if (!ctx) return PNP_E_ARG;
  if (!out || count < 1 || !reqs) return fail(ctx, PNP_E_ARG, "bad plan arguments");
  *out = nullptr;
  if (hipSetDevice(ctx->device) != hipSuccess) return device_check(ctx, "set device");
  std::vector<Layout> lay;
  std::vector<Group> groups;
  prepare_batch(ctx, count, reqs, lay, groups);
  if (relax)
    for (int r = 0; r < count; ++r) {
      if (reqs[r].status != PNP_OK) continue;
      const pnp_relax_spec& x = relax[r];
      if (!x.mu_bulk || !(x.lambda >= 0.0 && x.lambda <= 1.0) || std::isnan(x.clip))
        return fail(ctx, PNP_E_ARG, "relax spec " + std::to_string(r) + ": mu_bulk, lambda in [0, 1], clip");
    }
  // one device block: each group's table and evaluation records, then the
  // relax constants (rho_b, mu_b) of each request
  std::vector<size_t> ta_off(groups.size()), ea_off(groups.size()), rb_off(count, 0);
  size_t bytes = 0;
  for (size_t k = 0; k < groups.size(); ++k) {
    ta_off[k] = bytes;
    bytes = up(bytes + sizeof(TableArgs) * groups[k].ids.size());
    ea_off[k] = bytes;
    bytes = up(bytes + sizeof(EvalArgs) * groups[k].ids.size());
  }
  if (relax)
    for (int r = 0; r < count; ++r)
      if (reqs[r].status == PNP_OK) {
        rb_off[r] = bytes;
        bytes = up(bytes + sizeof(double) * 2 * reqs[r].S);
      }
  std::vector<char> host(std::max<size_t>(bytes, 1), 0);
  for (size_t k = 0; k < groups.size(); ++k) {
    std::memcpy(host.data() + ta_off[k], groups[k].ta.data(), sizeof(TableArgs) * groups[k].ids.size());
    std::memcpy(host.data() + ea_off[k], groups[k].ea.data(), sizeof(EvalArgs) * groups[k].ids.size());
  }
  if (relax)
    for (int r = 0; r < count; ++r)
      if (reqs[r].status == PNP_OK) {
        double* rb = (double*)(host.data() + rb_off[r]);
        for (int i = 0; i < reqs[r].S; ++i) {
          rb[2 * i] = reqs[r].species[i].rho_bulk;
          rb[2 * i + 1] = relax[r].mu_bulk[i];
        }
      }
  pnp_plan p = new pnp_plan_s();
  p->ctx = ctx;
  p->count = count;
  p->valid.resize(count);
  p->status.assign(count, nullptr);
  for (int r = 0; r < count; ++r) {
    p->valid[r] = reqs[r].status;
    if (reqs[r].status == PNP_OK) p->status[r] = (const char*)reqs[r].workspace + lay[r].status;
  }
  p->block_bytes = host.size();
  if (hipMalloc(&p->block, p->block_bytes) != hipSuccess ||
      hipMemcpy(p->block, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
    pnp_plan_destroy(p);
    return device_check(ctx, "plan block");
  }
  // capture every launch on a private stream of default priority
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    pnp_plan_destroy(p);
    return device_check(ctx, "capture stream");
  }
  // The size groups share nothing (every request has its own workspace and
  // outputs), so each is captured on a stream of its own, forked from the
  // capture stream and joined back: the replay runs them as parallel
  // branches, and the launches of small grids fill compute units that those
  // of the large ones leave idle.  Without these streams (creation failed,
  // or a single group) every group is captured on the capture stream.
  const size_t ng = groups.size();
  std::vector<hipStream_t> gs;
  std::vector<hipEvent_t> gev;  // [0] fork, [1 + k] group k done
  if (ng > 1) {
    gs.assign(ng, nullptr);
    gev.assign(ng + 1, nullptr);
    bool made = true;
    for (size_t k = 0; k < ng && made; ++k) made = hipStreamCreateWithFlags(&gs[k], hipStreamNonBlocking) == hipSuccess;
    for (size_t k = 0; k <= ng && made; ++k) made = hipEventCreateWithFlags(&gev[k], hipEventDisableTiming) == hipSuccess;
    if (!made) {
      (void)hipGetLastError();
      for (hipStream_t x : gs)
        if (x) (void)hipStreamDestroy(x);
      for (hipEvent_t e : gev)
        if (e) (void)hipEventDestroy(e);
      gs.clear();
      gev.clear();
    }
  }
  const bool branches = !gs.empty();
  char* blk = (char*)p->block;
  bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    ctx->capturing = true;
    if (branches) ok = hipEventRecord(gev[0], cs) == hipSuccess;
    for (size_t k = 0; k < ng && ok; ++k) {
      const Group& g = groups[k];
      hipStream_t st = branches ? gs[k] : cs;
      if (branches) ok = hipStreamWaitEvent(st, gev[0], 0) == hipSuccess;
      run_sequence(ctx, select_ops(ctx, g.precision, g.n, (int)g.ids.size()), (const EvalArgs*)(blk + ea_off[k]),
                   (const TableArgs*)(blk + ta_off[k]), (int)g.ids.size(), g.M, g.fmask, g.mix, st, g.n);
      if (branches && ok) ok = hipEventRecord(gev[1 + k], st) == hipSuccess && hipStreamWaitEvent(cs, gev[1 + k], 0) == hipSuccess;
    }
    if (relax)
      for (int r = 0; r < count; ++r) {
        if (reqs[r].status != PNP_OK) continue;
        const pnp_request& q = reqs[r];
        const long n3 = (long)q.grid.nx * q.grid.ny * q.grid.nz;
        const int blocks = (int)std::min<long>((q.S * n3 + 255) / 256, 4096);
        hipLaunchKernelGGL(k_relax, dim3(blocks), dim3(256), 0, cs, (double*)q.rho, (const double*)q.mu_ex, n3,
                           (int)q.S, (const double*)(blk + rb_off[r]), relax[r].lambda, relax[r].clip,
                           (const uint32_t*)p->status[r], fixed_mask(q.S, q.species));
      }
    ctx->capturing = false;
    // end the capture in every case (a failed fork or join above leaves ok false)
    const bool ended = hipStreamEndCapture(cs, &p->graph) == hipSuccess && p->graph;
    ok = ok && ended;
  }
  if (ok) ok = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) == hipSuccess;
  (void)hipStreamDestroy(cs);
  for (hipStream_t x : gs) (void)hipStreamDestroy(x);
  for (hipEvent_t e : gev) (void)hipEventDestroy(e);
  if (!ok) {
    pnp_plan_destroy(p);
    return device_check(ctx, "graph capture");
  }
  *out = p;
  return PNP_OK;
}

pnp_status pnp_plan_launch(pnp_plan plan, void* stream) {
  if (!plan) return PNP_E_ARG;
  if (hipSetDevice(plan->ctx->device) != hipSuccess) return device_check(plan->ctx, "set device");
  if (hipGraphLaunch(plan->exec, (hipStream_t)stream) != hipSuccess) return device_check(plan->ctx, "graph launch");
  return PNP_OK;
}

pnp_status pnp_plan_status(pnp_plan plan, void* stream, int32_t* status) {
  if (!plan || !status) return plan ? fail(plan->ctx, PNP_E_ARG, "null status array") : PNP_E_ARG;
  pnp_ctx ctx = plan->ctx;
  if (hipSetDevice(ctx->device) != hipSuccess) return device_check(ctx, "set device");
  hipStream_t s = (hipStream_t)stream;
  std::vector<uint32_t> words(2 * (size_t)plan->count, 0u);
  for (int r = 0; r < plan->count; ++r)
    if (plan->status[r] &&
        hipMemcpyAsync(&words[2 * r], plan->status[r], 8, hipMemcpyDeviceToHost, s) != hipSuccess)
      return device_check(ctx, "status read");
  if (hipStreamSynchronize(s) != hipSuccess) return device_check(ctx, "plan sync");
  for (int r = 0; r < plan->count; ++r)
    status[r] = plan->valid[r] != PNP_OK ? plan->valid[r] : status_of(ctx, &words[2 * r]);
  return PNP_OK;
}

void pnp_plan_destroy(pnp_plan plan) {
  if (!plan) return;
  (void)hipSetDevice(plan->ctx->device);
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->block) {
    (void)hipDeviceSynchronize();  // a replay in flight may still read the block
    (void)hipFree(plan->block);
  }
  delete plan;
}

pnp_status pnp_autotune(pnp_ctx ctx, int32_t count, pnp_request* reqs, int32_t reps, void* stream) {
  if (!ctx) return PNP_E_ARG;
  if (count < 1 || !reqs || reps < 1) return fail(ctx, PNP_E_ARG, "bad autotune arguments");
  if (hipSetDevice(ctx->device) != hipSuccess) return device_check(ctx, "set device");
  hipStream_t s = (hipStream_t)stream;
  std::vector<Layout> lay;
  std::vector<Group> groups;
  prepare_batch(ctx, count, reqs, lay, groups);
  // the pass timers are borrowed: keep the caller's accumulated figures
  const bool prof0 = ctx->prof;
  const uint32_t mask0 = ctx->prof_mask;
  double ms0[PNP_NUM_PASSES];
  int32_t n0[PNP_NUM_PASSES];
  pnp_status st = pnp_profile_read(ctx, ms0, n0, PNP_NUM_PASSES, 1);
  if (st != PNP_OK) return st;
  ctx->prof = true;
  ctx->prof_mask = ~0u;
  for (const Group& g : groups) {
    const int cnt = (int)g.ids.size();
    const TableArgs* dta = nullptr;
    const EvalArgs* dea = nullptr;
    upload_args(ctx, g.ta.data(), cnt, g.ea.data(), cnt, s, dta, dea);
    if (!dta || !dea) { st = device_check(ctx, "argument upload"); break; }
    OpsSel sel;
    sel.precision = g.precision;
    for (int v = 0; v < 4; ++v) sel.v[v] = ops_for(g.precision, g.n, v);
    const uint32_t alt = sel.v[0]->sched_alt;       // passes with a secondary schedule
    const uint32_t all = (1u << PNP_NUM_PASSES) - 2u;  // every pass but the tables
    // configurations: (schedule mask, tile mask); the narrow ones only where that shape exists
    const uint32_t cfg[4][2] = {{0u, 0u}, {alt, 0u}, {0u, all}, {alt, all}};
    const int ncfg = sel.v[1] ? 4 : 2;
    double t[4][PNP_NUM_PASSES] = {};
    for (int r = 0; r <= reps && st == PNP_OK; ++r)  // the first round warms up and is not counted
      for (int c = 0; c < ncfg && st == PNP_OK; ++c) {
        if (c == 1 && !alt) continue;
        if (c == 3 && !alt) continue;
        sel.smask = cfg[c][0];
        sel.mask = cfg[c][1];
        run_sequence(ctx, sel, dea, dta, cnt, g.M, g.fmask, g.mix, s, g.n);
        double ms[PNP_NUM_PASSES];
        st = pnp_profile_read(ctx, ms, nullptr, PNP_NUM_PASSES, 1);
        if (r > 0)
          for (int p = 0; p < PNP_NUM_PASSES; ++p) t[c][p] += ms[p];
      }
    if (st != PNP_OK) break;
    // per pass: under each schedule the tile shape (narrow only where it wins
    // by more than 3 %), then the secondary schedule only where its best
    // shape wins by more than 3 %
    uint32_t smask = 0, tmask = 0;
    for (int p = 1; p < PNP_NUM_PASSES; ++p) {
      bool nar[2];
      double best[2];
      for (int sc = 0; sc < 2; ++sc) {
        const double wide = t[sc][p], nw = t[2 + sc][p];
        nar[sc] = ncfg == 4 && nw < 0.97 * wide;
        best[sc] = nar[sc] ? nw : wide;
      }
      const int sc = ((alt >> p) & 1u) && best[1] < 0.97 * best[0] ? 1 : 0;
      if (sc) smask |= 1u << p;
      if (nar[sc]) tmask |= 1u << p;
    }
    // Per-pass choices need not add up (a pass's time depends on what the
    // one before left in the caches), and the default schedule of the size
    // mixes the two: the choice is timed end to end against the default
    // (its schedule, wide tiles) and kept only if its passes take more than
    // 1 % less in total.
    const uint32_t dsm = default_sched(g.precision, g.n);
    if (smask != dsm || tmask != 0u) {
      const uint32_t two[2][2] = {{dsm, 0u}, {smask, tmask}};
      double tot[2] = {0.0, 0.0};
      for (int r = 0; r <= reps && st == PNP_OK; ++r)
        for (int c = 0; c < 2 && st == PNP_OK; ++c) {
          sel.smask = two[c][0];
          sel.mask = two[c][1];
          run_sequence(ctx, sel, dea, dta, cnt, g.M, g.fmask, g.mix, s, g.n);
          double ms[PNP_NUM_PASSES];
          st = pnp_profile_read(ctx, ms, nullptr, PNP_NUM_PASSES, 1);
          if (r > 0)
            for (int p = 1; p < PNP_NUM_PASSES; ++p) tot[c] += ms[p];
        }
      if (st != PNP_OK) break;
      if (!(tot[1] < 0.99 * tot[0])) {
        smask = dsm;
        tmask = 0u;
      }
    }
    ctx->sched[sched_key(g.precision, g.n)] = smask;
    ctx->tune[tune_key(g.precision, g.n, count_class(cnt))] = tmask;
  }
  ctx->prof = prof0;
  ctx->prof_mask = mask0;
  for (int p = 0; p < PNP_NUM_PASSES; ++p) { ctx->prof_ms[p] = ms0[p]; ctx->prof_n[p] = n0[p]; }
  if (st != PNP_OK) return st;
  if (hipStreamSynchronize(s) != hipSuccess) return device_check(ctx, "autotune sync");
  return PNP_OK;
}

pnp_status pnp_tune_export(pnp_ctx ctx, char* buf, size_t cap, size_t* len) {
  if (!ctx || !len) return PNP_E_ARG;
  std::string out;
  for (const auto& kv : ctx->sched) {
    const int precision = (int)(kv.first >> 40), n = (int)(kv.first & 0xffffffffu);
    out += std::to_string(precision) + " " + std::to_string(n) + " s " + std::to_string(kv.second) + "\n";
  }
  for (const auto& kv : ctx->tune) {
    const int precision = (int)(kv.first >> 40), n = (int)((kv.first >> 8) & 0xffffffffu),
              cls = (int)(kv.first & 0xff);
    out += std::to_string(precision) + " " + std::to_string(n) + " " + std::to_string(cls) + " " +
           std::to_string(kv.second) + "\n";
  }
  *len = out.size();
  if (buf && cap > out.size()) std::memcpy(buf, out.c_str(), out.size() + 1);
  else if (buf) return fail(ctx, PNP_E_ARG, "buffer too small");
  return PNP_OK;
}

pnp_status pnp_tune_import(pnp_ctx ctx, const char* text) {
  if (!ctx || !text) return PNP_E_ARG;
  std::map<uint64_t, uint32_t> tiles, scheds;
  const char* p = text;
  while (*p) {
    int precision, n, used = 0;
    char cls[8];
    unsigned mask;
    if (std::sscanf(p, " %d %d %7s %u%n", &precision, &n, cls, &mask, &used) != 4) {
      while (*p == ' ' || *p == '\n' || *p == '\t' || *p == '\r') ++p;
      if (!*p) break;
      return fail(ctx, PNP_E_ARG, "tuning text: expected lines 'precision n class mask' or 'precision n s mask'");
    }
    const bool is_sched = std::strcmp(cls, "s") == 0;
    const bool is_tile = std::strlen(cls) == 1 && cls[0] >= '0' && cls[0] <= '3';
    if ((precision != PNP_FP64 && precision != PNP_MIXED) || !size_ok(n) || !(is_sched || is_tile) ||
        (mask & 1u) || (mask >> PNP_NUM_PASSES))
      return fail(ctx, PNP_E_ARG, "tuning text: entry out of range");
    if (is_sched) scheds[sched_key(precision, n)] = mask;
    else tiles[tune_key(precision, n, cls[0] - '0')] = mask;
    p += used;
  }
  for (const auto& kv : tiles) ctx->tune[kv.first] = kv.second;
  for (const auto& kv : scheds) ctx->sched[kv.first] = kv.second;
  return PNP_OK;
}

pnp_status pnp_read_status(pnp_ctx ctx, const void* ws, void* stream) {
  if (!ctx || !ws) return fail(ctx, PNP_E_ARG, "null argument");
  if (hipSetDevice(ctx->device) != hipSuccess) return device_check(ctx, "set device");
  return read_status(ctx, ws, (hipStream_t)stream);
}

pnp_status pnp_relax_densities(pnp_ctx ctx, const pnp_grid* g, int32_t S, const pnp_species* sp, double* rho,
                               const double* mu, const double* mu_bulk, double lambda, double clip,
                               void* stream) {
  if (!ctx) return PNP_E_ARG;
  if (!g || !sp || !rho || !mu || !mu_bulk) return fail(ctx, PNP_E_ARG, "null argument");
  if (g->nx != g->ny || g->ny != g->nz || !size_ok(g->nx)) return fail(ctx, PNP_E_UNSUPPORTED_SIZE, "bad grid");
  if (S < 1 || S > kMaxSpecies) return fail(ctx, PNP_E_ARG, "species count");
  if (!(lambda >= 0.0 && lambda <= 1.0)) return fail(ctx, PNP_E_ARG, "lambda must be in [0, 1]");
  if (std::isnan(clip)) return fail(ctx, PNP_E_ARG, "clip must be a number");
  if (hipSetDevice(ctx->device) != hipSuccess) return device_check(ctx, "set device");
  hipStream_t s = (hipStream_t)stream;
  double rb[2 * kMaxSpecies];
  for (int i = 0; i < S; ++i) { rb[2 * i] = sp[i].rho_bulk; rb[2 * i + 1] = mu_bulk[i]; }
  const double* drb = (const double*)upload(ctx, rb, sizeof(double) * 2 * S, s);
  if (!drb) return device_check(ctx, "argument upload");
  const long n3 = (long)g->nx * g->ny * g->nz;
  const int blocks = (int)std::min<long>((S * n3 + 255) / 256, 4096);
  hipLaunchKernelGGL(k_relax, dim3(blocks), dim3(256), 0, s, rho, mu, n3, (int)S, drb, lambda, clip,
                     (const uint32_t*)nullptr, fixed_mask(S, sp));
  return device_check(ctx, "relax launch");
}

pnp_status pnp_debug_rfft3(pnp_ctx ctx, const pnp_grid* g, int32_t precision, int32_t count, int32_t inverse,
                           const double* in, double* out, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return PNP_E_ARG;
  if (!g || !in || !out || !ws) return fail(ctx, PNP_E_ARG, "null argument");
  if (g->nx != g->ny || g->ny != g->nz || !size_ok(g->nx)) return fail(ctx, PNP_E_UNSUPPORTED_SIZE, "bad grid");
  if (count < 1 || count > kMaxSpecies) return fail(ctx, PNP_E_ARG, "count must be in [1, 8]");
  if (precision != PNP_FP64 && precision != PNP_MIXED) return fail(ctx, PNP_E_ARG, "bad precision");
  const int n = g->nx;
  const Layout L = layout_of(n, count, precision, false, false, false);
  if (ws_bytes < L.total) return fail(ctx, PNP_E_NOMEM, "workspace too small: need " + std::to_string(L.total));
  if (hipSetDevice(ctx->device) != hipSuccess) return device_check(ctx, "set device");
  hipStream_t s = (hipStream_t)stream;
  const Ops* op = ops_for(precision, n);
  char* w = (char*)ws;
  EvalArgs ea;
  std::memset(&ea, 0, sizeof(ea));
  ea.n = n; ea.S = count; ea.fstride = L.fstride; ea.specA = w + L.A; ea.specC = w + L.A;
  ea.status = (uint32_t*)(w + L.status); ea.rho = in; ea.out = out; ea.nreal = count; ea.final_mode = 0;
  const EvalArgs* dea = (const EvalArgs*)upload(ctx, &ea, sizeof(ea), s);
  if (!dea) return device_check(ctx, "argument upload");
  if (!inverse) {
    op->zfwd(dea, 1, s);
    op->ystep(dea, 1, 0, -1, true, kPartAll, s);
    op->xplain(dea, 1, count, true, s);
    op->xport(dea, count, out, 1, s);
  } else {
    op->xport(dea, count, (double*)in, 0, s);
    op->xplain(dea, 1, count, false, s);
    op->ystep(dea, 1, 0, -1, false, kPartAll, s);
    op->zinv(dea, 1, 0, s);
  }
  pnp_status st = device_check(ctx, "launch");
  if (st != PNP_OK) return st;
  if (hipStreamSynchronize(s) != hipSuccess) return device_check(ctx, "sync");
  return PNP_OK;
}

pnp_status pnp_bulk_mu_ex(pnp_ctx ctx, int32_t S, const pnp_species* sp, double T, const pnp_params* p,
                          double* mu) {
  pnp_ctx_s local;  // host-only call: a context is optional (it only records the error)
  if (!ctx) ctx = &local;
  if (!mu) return fail(ctx, PNP_E_ARG, "null output");
  const pnp_grid g{8, 8, 8, 1.0};  // the bulk value does not depend on the grid
  if (!p) return fail(ctx, PNP_E_ARG, "null params");
  pnp_params q = *p;
  q.flags &= ~(uint32_t)PNP_FLAG_APERIODIC;  // nor on the boundary mode
  Derived d;
  pnp_status st = validate(ctx, &g, S, sp, T, &q, d, true);
  if (st != PNP_OK) return st;
  // FMT at uniform densities: n_a = sum_i rho_i w_i^a(k = 0), the vector
  // densities vanish, and mu_i = sum_a dPhi/dn_a w_i^a(0) (Sec. 2.3.1)
  double n0 = 0, n1 = 0, n2 = 0, n3 = 0;
  for (int i = 0; i < S; ++i) {
    const double R = 0.5 * sp[i].d, rb = sp[i].rho_bulk;
    n0 += rb;
    n1 += rb * R;
    n2 += rb * 4.0 * M_PI * R * R;
    n3 += rb * 4.0 / 3.0 * M_PI * R * R * R;
  }
  if (d.hs && !(n3 < 1.0)) return fail(ctx, PNP_E_PACKING, "bulk packing fraction >= 1");
  const double u = 1.0 - n3;
  // phi3 and its derivative: the coefficient of n2^3 in Phi
  double p3 = 1.0 / (24.0 * M_PI * u * u), dp3 = 1.0 / (12.0 * M_PI * u * u * u);
  if (d.wb) {
    // 36 pi phi3 = [n3 + u^2 ln u] / (n3^2 u^2); its power series
    // sum_k (k+1)(k+3)/(k+2) n3^k below n3 = 0.05, where the closed form cancels
    double g = 0.0, dg = 0.0;
    if (n3 < 0.05) {
      for (int k = 19; k >= 0; --k) {
        const double c = (double)((k + 1) * (k + 3)) / (double)(k + 2);
        g = g * n3 + c;
        if (k >= 1) dg = dg * n3 + k * c;
      }
    } else {
      const double lu = std::log1p(-n3), ix = 1.0 / n3;
      g = ix / (u * u) + lu * ix * ix;
      dg = 2.0 * ix / (u * u * u) - ix * ix / (u * u) - ix * ix / u - 2.0 * lu * ix * ix * ix;
    }
    p3 = g / (36.0 * M_PI);
    dp3 = dg / (36.0 * M_PI);
  }
  const double d0 = -std::log1p(-n3), d1 = n2 / u, d2 = n1 / u + 3.0 * n2 * n2 * p3;
  const double d3 = n0 / u + n1 * n2 / (u * u) + n2 * n2 * n2 * dp3;
  for (int i = 0; i < S; ++i) {
    const double R = 0.5 * sp[i].d;
    double m = 0.0;
    if (d.hs) m += d0 + R * d1 + 4.0 * M_PI * R * R * d2 + 4.0 / 3.0 * M_PI * R * R * R * d3;
    // EC (Sec. 2.3.4) at uniform bulk densities: only the bulk constant
    if (d.ec) m += sp[i].mu_el_bulk;
    // mean-field square well (Sec. 2.3.2): c_sw beta sum_j rho_j u_ij(k = 0)
    if (d.sw)
      for (int j = 0; j < S; ++j) {
        const int q = d.pi[i][j];
        const double s = d.sigma[q], ro = d.rout[q];
        m += p->sw_prefactor * d.beta * sp[j].rho_bulk * (-d.eps[q]) * 4.0 / 3.0 * M_PI * (ro * ro * ro - s * s * s);
      }
    mu[i] = m;
  }
  return PNP_OK;
}

pnp_status pnp_debug_copy(pnp_ctx ctx, const void* src, void* dst, size_t bytes, void* stream) {
  if (!ctx) return PNP_E_ARG;
  if (!src || !dst) return fail(ctx, PNP_E_ARG, "null argument");
  if (bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16)
    return fail(ctx, PNP_E_ARG, "copy size and pointers must be multiples of 16 bytes");
  if (bytes == 0) return PNP_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return device_check(ctx, "set device");
  const long words = (long)(bytes / 16);
  if ((words + 255) / 256 > 0x7fffffffL) return fail(ctx, PNP_E_ARG, "copy too large");
  const int blocks = (int)((words + 255) / 256);
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const uint4*)src, (uint4*)dst, words);
  return device_check(ctx, "copy launch");
}

}  // extern "C"
