/*
 * pnp_cdft.h -- C ABI of the MI355X (gfx950) evaluator of cDFT excess chemical
 * potentials for 3D Poisson-Nernst-Planck-cDFT solvers.
 *
 * Method: Meng, Zheng, Lin, Sushko, "Numerical Solution of 3D Poisson-Nernst-
 * Planck Equations Coupled with Classical Density Functional Theory ...",
 * Sec. 2.3 (the cDFT free-energy terms and their chemical potentials) and
 * Sec. 3.4 (every cDFT integral evaluated as a convolution through FFTs).
 *
 * What one evaluation computes, for S species on a periodic n^3 grid of
 * spacing h (all outputs dimensionless, in units of k_B T):
 *   - FMT weighted densities n0..n3, n1v, n2v (Sec. 2.3.1, correlations of
 *     rho_i with the weight functions omega_i);
 *   - the ten partial derivatives of the Rosenfeld free-energy density, or
 *     of its modified White Bear form (Sec. 2.3.1), evaluated pointwise in
 *     FP64;
 *   - beta mu_hs_i by back-convolution (Sec. 2.3.1);
 *   - beta mu_el_i, the MSA electrostatic-correlation term (Sec. 2.3.4):
 *     mu_el_bulk_i - sum_j C_ij (*) (rho_j - rho_j^bulk);
 *   - beta mu_sh_i, the mean-field square-well term (Sec. 2.3.2) with the
 *     printed prefactor 1/2 (configurable);
 *   - beta mu_ex = hs + el + sh and the Slotboom factor exp(-beta mu_ex),
 *     the mu_ex part of the transformed diffusion coefficient (Sec. 2.1).
 * The Coulomb term of Sec. 2.3.3 is not part of mu_ex here: in a PNP solve it
 * is the Poisson potential.  With PNP_FLAG_APERIODIC the grid is instead the
 * domain of a non-periodic problem (Sec. 3.4: convolutions over the domain
 * only, through zero extension onto the doubled grid).
 *
 * Around the evaluation: batches of independent requests, captured replays
 * (HIP graphs), resident sessions in a device pool, free energies, the
 * equilibrium (Picard) solve, the bulk chemical potentials, a tile-shape
 * autotuner, pass timing and a calibration copy.  Beside it: the delta-shell
 * integrals by the product quadrature over spheres of Sec. 3.5
 * (pnp_sphere_quadrature), a real-space alternative to the spectral weights.
 *
 * Discrete operator: each weight / pair kernel is the inverse DFT of its
 * continuous Fourier transform sampled at the grid wave-vectors (exact bulk
 * sums, no r = 0 singularity); vector weights drop their component along an
 * axis on that axis's Nyquist plane.  Forward weighted densities are
 * correlations and back-convolutions are convolutions, as in Sec. 2.3.1.
 *
 * Units: lengths nm, energies eV, temperature K, densities nm^-3.
 *
 * Memory: every pointer marked "device" is caller-owned device memory (for
 * example allocated by PyTorch) on the context's device; the library never
 * allocates, frees or retains caller memory.  The context owns a 4 MiB
 * device ring for per-call argument records (allocated by pnp_create) and a
 * few host records; when the ring wraps (after thousands of calls) the call
 * that wraps it waits for the device to drain.  A captured plan owns a small
 * device block for its argument records (allocated by pnp_plan_create, freed
 * by pnp_plan_destroy).  Scratch space comes in through `workspace`, sized by
 * pnp_workspace_bytes().
 *
 * Errors: every function returns a pnp_status; nothing aborts or throws
 * across this boundary.  Outputs are unspecified when the return is not
 * PNP_OK.  pnp_last_error() gives a human-readable reason.
 *
 * Concurrency: a context is not thread-safe; use one per host thread.  Work
 * is enqueued on the caller's HIP stream.  From 192^3 up part of it (the
 * Nyquist-plane tiles of the y and x passes and the radial tables) runs on a
 * second stream that the context owns (default priority), forked from the
 * caller's stream after the work enqueued so far and joined back into it
 * before the call's last pass, so to the caller the work is ordered as if
 * it ran on its stream alone.  A batch with two or more grid sizes below
 * 192^3 runs each of them on a further stream of the context's (default
 * priority, one per size, created on first use), forked and joined the same
 * way.  Unless PNP_FLAG_ASYNC is set, a
 * call waits for its own work to finish so that it can return the status
 * that the kernels raised (packing fraction >= 1, non-finite values,
 * overflow of exp(-mu)).
 */
#ifndef PNP_CDFT_H
#define PNP_CDFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PNP_OK = 0,
  PNP_E_ARG = -1,              /* invalid argument (null pointer, bad count, ...) */
  PNP_E_UNSUPPORTED_SIZE = -2, /* grid size not in the supported set */
  PNP_E_NOMEM = -3,            /* workspace too small */
  PNP_E_PACKING = -4,          /* some weighted density n3 >= 1: ln(1 - n3) undefined */
  PNP_E_OVERFLOW = -5,         /* exp(-beta mu_ex) overflowed a double */
  PNP_E_NONFINITE = -6,        /* a non-finite value appeared in the evaluation */
  PNP_E_DEVICE = -7,           /* HIP runtime error */
  PNP_E_BUDGET = -8            /* request does not fit the memory budget */
} pnp_status;

/* terms of beta mu_ex.  The hard-sphere term uses Rosenfeld's free-energy
 * density (PNP_TERM_HS) or the modified White Bear form of Sec. 2.3.1
 * (PNP_TERM_HS_WB), whose n2^3 coefficient
 *   phi3(n3) = [n3 + (1 - n3)^2 ln(1 - n3)] / (36 pi n3^2 (1 - n3)^2)
 * replaces 1 / (24 pi (1 - n3)^2) and gives the Carnahan-Starling bulk
 * fluid.  The two hard-sphere bits are exclusive (PNP_E_ARG if both). */
enum { PNP_TERM_HS = 1, PNP_TERM_EC = 2, PNP_TERM_SW = 4, PNP_TERM_ALL = 7, PNP_TERM_HS_WB = 8 };

/* arithmetic of the spectral path */
enum {
  PNP_FP64 = 0,  /* FFTs, weights and pointwise work in double */
  PNP_MIXED = 1  /* FFTs, weight multiplies and the sum of the three terms
                    (taken in k-space, before the last inverse transform) in
                    float; the singular factors of the FMT derivatives
                    (log(1 - n3), 1/(1 - n3)^k, the White Bear coefficient)
                    in double, their products with the weighted densities in
                    float (in double for free energies); the bulk constants,
                    the output and exp(-beta mu) in double.  Error against
                    the FP64 path: about 1e-6 of each term's largest
                    magnitude at packing 0.45 */
};

/* flags */
enum {
  PNP_FLAG_ASYNC = 1,     /* do not wait for the status word; read it later with
                             pnp_read_status() */
  PNP_FLAG_APERIODIC = 2, /* the grid is the domain of a non-periodic problem
                             (Sec. 3.4): every convolution integrates over the
                             domain only, its integrand (rho, rho - rho_bulk
                             for the EC term, dPhi/dn_alpha for the hard-sphere
                             back-convolution) zero outside, and runs on the
                             doubled grid (2n)^3 of the same spacing with the
                             domain at its corner; results are the domain's.
                             n may be any size whose double is supported
                             (4, 8, 12, 16, 24, 32, 48, 64, 96, 128).
                             pnp_cdft_mu_ex and pnp_workspace_bytes only;
                             pnp_bulk_mu_ex ignores it; every other entry
                             point returns PNP_E_ARG. */
  PNP_FLAG_CUBIC = 4      /* pnp_sphere_quadrature only: the integrand between
                             grid points is the tricubic interpolant (Lagrange
                             cubics through the 4 x 4 x 4 surrounding points)
                             instead of the trilinear one */
};

typedef struct pnp_ctx_s* pnp_ctx;

/* Periodic grid with nx = ny = nz = n points of spacing h [nm].  Supported n:
 * 8, 16, 24, 32, 48, 64, 96, 128, 192, 256 (see pnp_supported_size). */
typedef struct {
  int32_t nx, ny, nz;
  double h;
} pnp_grid;

/* One species (Sec. 2.3: charged hard spheres).
 * mobile: nonzero for a species that moves (the ions of Sec. 2.1); 0 for a
 * stationary one, such as the fixed sites whose density Sec. 2.3.2 places at
 * given positions and couples to the mobile ions by square wells.  Every
 * species, stationary or not, enters the weighted densities and the pair
 * terms and receives its own beta mu_ex; the density updates
 * (pnp_relax_densities, session steps, plans with a density update,
 * pnp_equilibrium) leave a stationary species' density unchanged bit for
 * bit and leave it out of the equilibrium residual.  A zero-initialised
 * record is stationary: callers set mobile = 1 for ions. */
typedef struct {
  double d;           /* hard-core diameter [nm], > 0 */
  double q;           /* valence (signed) */
  double rho_bulk;    /* bulk density [nm^-3] (reference of the EC expansion, and kappa) */
  double mu_el_bulk;  /* beta mu_el_i[bulk] [k_B T]; the paper gives no formula, 0 is typical */
  int32_t mobile;     /* 1: mobile (density updated by the relaxation steps); 0: stationary */
} pnp_species;

typedef struct {
  uint32_t terms;         /* PNP_TERM_* mask */
  int32_t precision;      /* PNP_FP64 or PNP_MIXED */
  int32_t per_term;       /* 0: mu_ex is [S][N]; 1: mu_ex is [3][S][N] = (hs, el, sh) */
  uint32_t flags;         /* PNP_FLAG_* */
  double eps_r;           /* relative permittivity (Table 1 uses 16.6) */
  const double* sw_eps;   /* host, S*S row-major well depths [eV] (> 0 attractive); NULL: none */
  const double* sw_rout;  /* host, S*S outer radii [nm]; NULL or entries <= 0: gamma*sigma_ij */
  double sw_gamma;        /* well extent factor, 1.2 in Sec. 2.3.2 */
  double sw_prefactor;    /* factor in front of the mean-field integral, 1/2 as printed */
} pnp_params;

/* Create a context bound to HIP device `device` (used for every call). */
pnp_status pnp_create(int device, pnp_ctx* out);
void pnp_destroy(pnp_ctx ctx);

/* Human-readable description of the last error on this context. */
const char* pnp_last_error(pnp_ctx ctx);

/* 1 when n is a supported grid size, else 0. */
int pnp_supported_size(int32_t n);

/* Bytes of device workspace one evaluation of this shape needs. */
pnp_status pnp_workspace_bytes(pnp_ctx ctx, const pnp_grid* grid, int32_t S,
                               const pnp_params* params, size_t* bytes);

/*
 * One evaluation of beta mu_ex (Sec. 2.3) and exp(-beta mu_ex) (Sec. 2.1).
 *   rho       device, float64 [S][nx][ny][nz], z fastest; read-only
 *   T         temperature [K] > 0
 *   mu_ex     device, float64 [S][N] (per_term = 0) or [3][S][N] (per_term = 1)
 *   slotboom  device, float64 [S][N] exp(-beta mu_ex); may be NULL
 *   workspace device, >= pnp_workspace_bytes(), 256-byte aligned
 *   stream    hipStream_t (NULL = default stream)
 * Errors: PNP_E_ARG, PNP_E_UNSUPPORTED_SIZE, PNP_E_NOMEM (workspace_bytes too
 * small), PNP_E_PACKING (some n3 >= 1), PNP_E_NONFINITE, PNP_E_OVERFLOW,
 * PNP_E_DEVICE.
 */
pnp_status pnp_cdft_mu_ex(pnp_ctx ctx, const pnp_grid* grid, int32_t S,
                          const pnp_species* species, const double* rho, double T,
                          const pnp_params* params, double* mu_ex, double* slotboom,
                          void* workspace, size_t workspace_bytes, void* stream);

/*
 * pnp_cdft_mu_ex without a workspace argument and without any allocation,
 * for callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): the same evaluation, the same kernels and
 * the same results bit for bit, with the workspace taken from one static
 * device array of 64 MiB that each GPU the library runs on holds until the
 * process ends (its address is looked up once per device by pnp_create).
 * Arguments, outputs and errors as pnp_cdft_mu_ex, plus:
 *   - PNP_E_NOMEM when pnp_workspace_bytes() of the call exceeds 64 MiB
 *     (for example mixed precision up to 96^3 with S <= 4, FP64 up to 64^3
 *     with S <= 8; the aperiodic mode needs the doubled grid's workspace);
 *   - PNP_E_ARG on a stream that is capturing a graph (the argument records
 *     are copied from host memory at call time), and nothing is enqueued;
 *   - PNP_E_DEVICE when the array has no address on this device.
 * Every call on one GPU shares that GPU's array, whichever context, stream or
 * thread makes it: calls that overlap on one GPU race and give undefined
 * results.  The array keeps the last call's contents; a call writes every
 * part it reads (the status words are cleared by its first pass).  With
 * PNP_FLAG_ASYNC the status words stay in the array and are not reported.
 */
pnp_status pnp_cdft_mu_ex_noalloc(pnp_ctx ctx, const pnp_grid* grid, int32_t S,
                                  const pnp_species* species, const double* rho, double T,
                                  const pnp_params* params, double* mu_ex, double* slotboom,
                                  void* stream);

/*
 * Excess free energies [k_B T] of the densities rho (Sec. 2.3), from one
 * per-term evaluation (the same operator as pnp_cdft_mu_ex):
 *   F_hs = h^3 sum_r Phi_hs(n(r))                          (Sec. 2.3.1)
 *   F_el = h^3 sum_i sum_r drho_i (beta mu_el_i[bulk] - 1/2 (C (*) drho)_i)
 *        = h^3/2 sum_i sum_r drho_i (beta mu_el_i + beta mu_el_i[bulk])  (Sec. 2.3.4)
 *   F_sh = 1/2 beta h^3 sum_ij sum_r rho_i (u_ij (*) rho_j)
 *        = h^3 / (2 sw_prefactor) sum_i sum_r rho_i beta mu_sh_i       (Sec. 2.3.2)
 * with drho = rho - rho_bulk (the constant F_el[bulk] is dropped); terms
 * that are switched off contribute 0.  Sums run in a fixed order, so the
 * result is reproducible bit for bit.
 *   energies  host, 4 values: F_hs, F_el, F_sh, total
 *   mu3       device, float64 [3][S][N]: receives the per-term beta mu_ex
 *   workspace >= pnp_workspace_bytes() with params->per_term = 1
 * Errors: as pnp_cdft_mu_ex.  The call waits for its result.
 */
pnp_status pnp_free_energy(pnp_ctx ctx, const pnp_grid* grid, int32_t S,
                           const pnp_species* species, const double* rho, double T,
                           const pnp_params* params, double* energies, double* mu3,
                           void* workspace, size_t workspace_bytes, void* stream);

/*
 * Equilibrium densities of the grand ensemble at the bulk chemical
 * potentials (the cDFT state Sec. 3.2 solves for before the PNP iteration):
 *   rho_i(r) = rho_bulk_i exp(beta mu_b,i - beta mu_ex,i[rho](r) - beta V_i(r)),
 * with beta mu_b = pnp_bulk_mu_ex, by Picard iteration with mixing lambda
 * (the relaxation of Sec. 3.2),
 *   rho <- (1 - lambda) rho + lambda rho_bulk exp(beta mu_b - beta mu_ex[rho] - beta V),
 * until max_i max_r |rho_new - rho| / rho_bulk_i <= tol or max_iter steps.
 *   beta_v   device, float64 [S][N] external potential [k_B T], or NULL
 *   rho      device, float64 [S][N]: in the initial guess, out the last iterate
 *   mu_ex    device, float64 [S][N]: out beta mu_ex of the densities before
 *            the last update
 *   iters, residual  host out: steps taken and the last residual
 *   lambda in (0, 1], tol >= 0, max_iter >= 1; rho_bulk > 0 for every
 *   mobile species (stationary species keep their densities and are left
 *   out of the residual)
 *   workspace >= pnp_workspace_bytes() (params->per_term = 0)
 * Plain Picard iteration converges for moderate coupling; dense or strongly
 * correlated fluids need a small lambda.  Errors: as pnp_cdft_mu_ex (a
 * packing error stops the iteration and reports the step in iters).
 * The call waits for every step.
 */
pnp_status pnp_equilibrium(pnp_ctx ctx, const pnp_grid* grid, int32_t S,
                           const pnp_species* species, double T, const pnp_params* params,
                           const double* beta_v, double* rho, double* mu_ex, double lambda,
                           double tol, int32_t max_iter, int32_t* iters, double* residual,
                           void* workspace, size_t workspace_bytes, void* stream);

/*
 * The weighted densities of Sec. 2.3.1 alone, in real space.
 *   n_out  device, float64 [10][N] in the order n0, n1, n2, n3, n1v(x,y,z), n2v(x,y,z)
 * Same errors as pnp_cdft_mu_ex (no packing check).
 */
pnp_status pnp_weighted_densities(pnp_ctx ctx, const pnp_grid* grid, int32_t S,
                                  const pnp_species* species, const double* rho,
                                  const pnp_params* params, double* n_out,
                                  void* workspace, size_t workspace_bytes, void* stream);

/*
 * Surface integrals over spheres by the product quadrature of Sec. 3.5: the
 * delta-shell integrals of the FMT weights taken in real space, as an
 * alternative to the spectral weights of the evaluation above.  For each
 * field f and grid point r, with the radius R of that field,
 *   I(r)   = int f(r') delta(|r' - r| - R) dr'
 *          ~ R^2 sum_i sum_j f(r + R n_ij) sin(phi_j) w_i w~_j,
 *   I_a(r) ~ the same sum with f(r + R n_ij) n_ij,a,  a = x, y, z,
 * n_ij = (cos theta_i sin phi_j, sin theta_i sin phi_j, cos phi_j), over
 * theta_i = 2 pi i / k (weights 2 pi / k) and the k Gauss-Legendre points
 * phi_j of [0, pi]; f between grid points is the trilinear interpolant of
 * the grid values (error O(h^2)), or with PNP_FLAG_CUBIC the tricubic one
 * through the 4 x 4 x 4 surrounding points (Lagrange cubics on the offsets
 * -1, 0, 1, 2 of each axis; error O(h^4)).  The paper fixes neither the 1D
 * rules nor the interpolation; these are the readings taken.  I_a is the correlation with
 * the vector weight x/|x| delta(|x| - R) (x = r' - r), the convention of
 * pnp_weighted_densities, so with R_s = d_s / 2:
 *   n2 = sum_s I_s, n1 = sum_s I_s / (4 pi R_s), n0 = sum_s I_s / (4 pi R_s^2),
 *   n2v = sum_s I_s,a, n1v = sum_s I_s,a / (4 pi R_s).
 *   grid       nx, ny, nz >= 1 (any extents, nx ny nz < 2^31), spacing h > 0 [nm]
 *   F          number of fields, 1..64
 *   f          device, float64 [F][nx][ny][nz], z fastest; read-only
 *   radius     host, F radii [nm], 0 < R <= 16 h; the stencil reach
 *              (about R / h + 1 grid points, one more with PNP_FLAG_CUBIC)
 *              must fit the LDS tile: up to 11 points in PNP_MIXED, 8 in
 *              PNP_FP64 (else PNP_E_UNSUPPORTED_SIZE);
 *              reaches above 4 (FP64) or 7 (mixed) run with one workgroup
 *              per compute unit
 *   order      k in [1, 64] (k*k nodes per sphere)
 *   precision  PNP_FP64 (double arithmetic) or PNP_MIXED (float arithmetic,
 *              float weights; inputs and outputs stay double)
 *   flags      PNP_FLAG_APERIODIC: f is zero outside the grid (the paper's
 *              zero extension); otherwise periodic images.  PNP_FLAG_CUBIC:
 *              tricubic interpolation.  PNP_FLAG_ASYNC: do not wait for the
 *              kernel.
 *   out        device, float64 [F][4][nx][ny][nz]: (I, I_x, I_y, I_z) per field
 * The stencil (at most a few hundred offsets per field for R / h <= 4) is
 * built on the host in double and copied to the context's ring on `stream`
 * from host memory that the call frees before it returns, so the call
 * cannot be recorded into a HIP graph: on a capturing stream it returns
 * PNP_E_ARG and enqueues nothing.  Errors: PNP_E_ARG,
 * PNP_E_UNSUPPORTED_SIZE, PNP_E_DEVICE.
 */
pnp_status pnp_sphere_quadrature(pnp_ctx ctx, const pnp_grid* grid, int32_t F, const double* f,
                                 const double* radius, int32_t order, int32_t precision,
                                 uint32_t flags, double* out, void* stream);

/* One request of a batch: an independent evaluation with its own shape. */
typedef struct {
  pnp_grid grid;
  int32_t S;
  const pnp_species* species;  /* host, S entries */
  const double* rho;           /* device */
  double T;
  const pnp_params* params;    /* host */
  double* mu_ex;               /* device */
  double* slotboom;            /* device or NULL */
  void* workspace;             /* device, this request's own workspace */
  size_t workspace_bytes;
  int32_t status;              /* out: pnp_status of this request */
} pnp_request;

/*
 * Evaluate `count` independent requests of possibly different sizes,
 * temperatures and compositions.  Requests with equal grid size share every
 * kernel launch (one grid of workgroups spans all of them).  With two or
 * more grid sizes below 192^3, each of those sizes runs on a stream of the
 * context's own (default priority), forked from `stream` and joined back
 * before the call returns or, with PNP_FLAG_ASYNC, before later work on
 * `stream`; requests must not share a workspace or an output buffer.  A
 * request that fails (bad packing, overflow, ...) reports its own status and
 * does not affect the others.  Returns PNP_OK when the batch ran (check each
 * status).
 */
pnp_status pnp_batch_mu_ex(pnp_ctx ctx, int32_t count, pnp_request* reqs, void* stream);

/*
 * Captured evaluations.  A plan binds `count` requests (as pnp_batch_mu_ex:
 * same validation, same grouping by grid size and precision, the same
 * kernels and arithmetic, so a replay equals the batch call bit for bit) and
 * records every launch of their evaluation in one HIP graph; a replay costs
 * one graph launch instead of about ten kernel launches and one argument
 * upload per grid size.  This is for callers that evaluate the same buffers
 * over and over (the Gummel iterations of a PNP solve, resident sessions):
 * they rewrite rho in place and replay.
 *
 * relax: NULL, or one pnp_relax_spec per request.  With it each replay also
 * applies the density update of pnp_relax_densities to that request's rho
 * (in place: rho must then be writable) after its evaluation, skipped on the
 * device for a request whose evaluation raised a status.
 *
 * pnp_plan_create validates every request (reqs[r].status receives the
 * result; failed requests are left out of the graph), copies their argument
 * records into a device block owned by the plan (a few KiB per request),
 * and captures the graph on a private stream, each grid size on a branch of
 * its own (the replay runs the sizes side by side: requests must not share
 * a workspace or an output buffer).  The request array and the
 * host arrays it points to may be released afterwards; the device buffers
 * must stay allocated while the plan exists.  Errors: PNP_E_ARG (no valid
 * plan arguments, or a bad relax spec), PNP_E_DEVICE (capture failed).
 * pnp_plan_launch replays asynchronously on `stream` (no allocation, no
 * host work beyond the launch).  pnp_plan_status waits for `stream` and
 * writes the pnp_status of each request of the last replay into
 * status[count] (creation-time failures keep their code).  A plan is tied to
 * its context; replays of one plan on different streams must not overlap.
 */
typedef struct pnp_plan_s* pnp_plan;

typedef struct {
  const double* mu_bulk;  /* host, S values [k_B T]: beta mu_b of the update; copied */
  double lambda;          /* mixing in [0, 1] */
  double clip;            /* exponent limit (<= 0: none), as pnp_relax_densities */
} pnp_relax_spec;

pnp_status pnp_plan_create(pnp_ctx ctx, int32_t count, pnp_request* reqs,
                           const pnp_relax_spec* relax, pnp_plan* out);
pnp_status pnp_plan_launch(pnp_plan plan, void* stream);
pnp_status pnp_plan_status(pnp_plan plan, void* stream, int32_t* status);
void pnp_plan_destroy(pnp_plan plan);

/*
 * Autotuner of FFT schedules and tile shapes.  Each pass of the evaluation
 * has two FFT schedules: the primary one (16 elements per thread for the z
 * and y transforms, 12 on sizes with a factor 3; 8 for the x transforms in
 * mixed precision, 4 in FP64, 6 with a factor 3; 4, 2 or 6 for the
 * derivative pass) and a secondary one with half as many elements per
 * thread, twice the threads per pencil and smaller radices, where such a
 * radix plan exists; for the x transforms of sizes with a factor 3, twice
 * as many (12: fewer, larger radix stages); elsewhere the two are the
 * same.  Every pass also has a
 * default tile shape (workgroups carrying 16 pencils or rows, for
 * full-width HBM bursts on large grids) and, for grids up to 128^3, a
 * narrow one with a quarter of the pencils per workgroup and four times the
 * workgroups (small grids otherwise leave most of the 256 compute units
 * idle).  pnp_autotune evaluates the requests (validated and grouped as
 * pnp_batch_mu_ex; their outputs receive real results) `reps` times in each
 * (schedule, shape) combination after one warm-up round, times every pass
 * with HIP events, and keeps per pass the narrow shape where it is faster
 * by more than 3 % under a schedule, and the secondary schedule where its
 * best shape is faster than the primary's by more than 3 %.  That choice is
 * then timed end to end (`reps` more rounds) against the size's default
 * schedule with the default shapes, and kept only if its passes take more
 * than 1 % less in total; otherwise the default is stored.
 *
 * The schedule is stored in the context under (precision, n): the last
 * autotune or import for that pair sets it for every later evaluation of
 * that size (single calls, batches of any composition, plans, sessions, the
 * equilibrium solve, free energies, weighted densities), so an instance gets
 * the same arithmetic alone and in any batch.  Before any tuning the
 * schedule is a built-in table of the autotuner's choices measured on an
 * MI355X for each supported size and precision (at 256^3: the secondary
 * schedule for the two z passes; at 192^3 also for the two x passes in
 * mixed precision).  The two schedules order the floating-point
 * operations differently: results agree to rounding, not bit for bit.  The
 * tile shape is stored under (precision, n, instance-count class of the
 * launch: 1, 2-3, 4-15, >= 16); it does not change the arithmetic.  The
 * call waits for its work.  Accumulated pass timings (pnp_profile_read) are
 * left as they were.
 */
pnp_status pnp_autotune(pnp_ctx ctx, int32_t count, pnp_request* reqs, int32_t reps, void* stream);

/* The stored tuning as text, one line per key: "precision n s mask" for an
 * FFT schedule (bit p set = pass p of pnp_profile_read's order runs the
 * secondary schedule) and "precision n class mask" for a tile shape (class
 * 0-3; bit p set = pass p runs narrow).  Bit 0 (the table pass) is never
 * set.  pnp_tune_export writes it into buf (NUL-terminated; *len = its
 * length without the NUL; with buf NULL only *len is set; PNP_E_ARG if cap
 * is too small).  pnp_tune_import merges such text into the context
 * (PNP_E_ARG on malformed or out-of-range lines, and then nothing is
 * merged); a schedule bit of a pass whose two schedules are the same has no
 * effect. */
pnp_status pnp_tune_export(pnp_ctx ctx, char* buf, size_t cap, size_t* len);
pnp_status pnp_tune_import(pnp_ctx ctx, const char* text);

/* Read the status word left by an asynchronous call (after the stream has
 * finished the work).  workspace: the one passed to that call. */
pnp_status pnp_read_status(pnp_ctx ctx, const void* workspace, void* stream);

/*
 * Consumer stub of the PNP loop (not part of the evaluation): relaxes every
 * density toward the equilibrium of its current excess chemical potential,
 *   rho_i <- (1 - lambda) rho_i + lambda rho_i^bulk exp(g_i),
 *   g_i = beta mu_b,i - beta mu_ex,i, limited to [-clip, clip] when clip > 0,
 * where beta mu_b,i = mu_bulk[i].  Sec. 3.2 uses relaxation
 * rho <- lambda2 rho_new + (1 - lambda2) rho_old.  With clip > 0 every
 * density stays within max(rho_i, e^clip rho_i^bulk), which keeps a strongly
 * attractive state from running past close packing.  Stationary species
 * (mobile = 0) are left unchanged.
 *   rho      device, float64 [S][N], updated in place
 *   mu_ex    device, float64 [S][N]
 *   mu_bulk  host, S values [k_B T]
 */
pnp_status pnp_relax_densities(pnp_ctx ctx, const pnp_grid* grid, int32_t S,
                               const pnp_species* species, double* rho,
                               const double* mu_ex, const double* mu_bulk, double lambda,
                               double clip, void* stream);

/*
 * beta mu_ex of the uniform bulk state (host arithmetic, no device work):
 * every rho_i(r) = rho_bulk_i.  HS: the free-energy derivatives (Rosenfeld
 * or White Bear, as selected) at the bulk weighted densities, contracted
 * with the k = 0 weights (Sec. 2.3.1); EC: mu_el_bulk (Sec. 2.3.4, no density deviation); SW:
 * sw_prefactor * beta * sum_j rho_bulk_j u_ij(k = 0) (Sec. 2.3.2).  Equals
 * what pnp_cdft_mu_ex returns for uniform bulk densities, to rounding.
 *   ctx may be NULL (no device is used; errors are then not recorded)
 *   mu  host, S values [k_B T]
 * Errors: PNP_E_ARG, PNP_E_PACKING (bulk packing fraction >= 1).
 */
pnp_status pnp_bulk_mu_ex(pnp_ctx ctx, int32_t S, const pnp_species* species, double T,
                          const pnp_params* params, double* mu);

/*
 * Serving: resident sessions in one caller-owned device pool.
 *
 * A session holds a PNP-style state on the device: densities rho_i(r)
 * [S][N], their beta mu_ex [S][N], Slotboom factors [S][N] and the
 * evaluation workspace, sub-allocated first-fit from the pool's range
 * (256-byte aligned; freed blocks coalesce).  A step evaluates beta mu_ex
 * of every listed session in shared launches (pnp_batch_mu_ex) and then
 * relaxes each session's densities toward the equilibrium of the new
 * mu_ex (pnp_relax_densities with the session's lambda and bulk mu).
 * Pools are not thread-safe; closing a session does not wait for work in
 * flight on it, so order any reuse of its memory after that work (same
 * stream, or synchronise).
 */
typedef struct pnp_pool_s* pnp_pool;

/* Device bytes one session of this shape takes from a pool (densities,
 * mu_ex, Slotboom factors, workspace). */
pnp_status pnp_session_bytes(pnp_ctx ctx, const pnp_grid* grid, int32_t S, const pnp_params* params,
                             size_t* bytes);

/* A pool over [arena, arena + arena_bytes): device memory owned by the
 * caller, 256-byte aligned, valid until pnp_pool_destroy. */
pnp_status pnp_pool_create(pnp_ctx ctx, void* arena, size_t arena_bytes, pnp_pool* out);
void pnp_pool_destroy(pnp_pool pool);

/* Bytes held by open sessions, the largest free block, and the number of
 * open sessions. */
pnp_status pnp_pool_usage(pnp_pool pool, size_t* used, size_t* largest_free, int32_t* sessions);

/*
 * Admit a session: copies rho0 (device, float64 [S][N]) into the pool on
 * `stream`.  mu_bulk: host, S values of beta mu_ex in bulk for the update,
 * or NULL for pnp_bulk_mu_ex.  lambda in [0, 1] and clip: the update's
 * parameters (pnp_relax_densities).  params->per_term must be 0 and flags
 * are ignored.  PNP_E_BUDGET when no free block is large enough (nothing
 * is allocated).
 */
pnp_status pnp_session_open(pnp_pool pool, const pnp_grid* grid, int32_t S, const pnp_species* species,
                            double T, const pnp_params* params, const double* rho0,
                            const double* mu_bulk, double lambda, double clip, void* stream,
                            int64_t* id);

/* One step of `count` sessions; status[k] receives session k's pnp_status
 * (its densities are not updated when it is not PNP_OK). */
pnp_status pnp_session_step(pnp_pool pool, int32_t count, const int64_t* ids, int32_t* status,
                            void* stream);

/* Device pointers of a session's arrays (valid until it closes) and the
 * number of completed steps; any output pointer may be NULL. */
pnp_status pnp_session_view(pnp_pool pool, int64_t id, double** rho, double** mu_ex,
                            double** slotboom, int64_t* steps);

/* Release a session's block to the pool. */
pnp_status pnp_session_close(pnp_pool pool, int64_t id);

/* Captured session steps: keep up to max_plans step graphs (pnp_plan_*),
 * keyed by the exact id list of a step, least recently used evicted; a step
 * whose list has a graph replays it (evaluation and density update in one
 * graph launch; the update is skipped on the device for a session whose
 * evaluation raised a status).  Closing a session drops the graphs that
 * hold it.  0 (the default) steps through pnp_batch_mu_ex and
 * pnp_relax_densities instead.  Results are identical either way. */
pnp_status pnp_pool_graphs(pnp_pool pool, int32_t max_plans);

/*
 * Test hook: 3D real-to-complex DFT of `count` fields through the same
 * kernels the evaluation uses, written in numpy's rfftn layout
 * (complex128 [count][n][n][n/2+1]).  `inverse` = 1 runs the reverse
 * (unnormalised complex-to-real, numpy irfftn times N) from that layout.
 *   in/out device float64 (real fields [count][N] or interleaved complex).
 */
pnp_status pnp_debug_rfft3(pnp_ctx ctx, const pnp_grid* grid, int32_t precision,
                           int32_t count, int32_t inverse, const double* in, double* out,
                           void* workspace, size_t workspace_bytes, void* stream);

/*
 * Calibration hook: plain device-to-device copy of `bytes` bytes (a multiple
 * of 16, both pointers 16-byte aligned, buffers must not overlap) with one
 * streaming kernel.  Gives the achievable HBM bandwidth next to which the
 * passes are judged, and the reference reading of the memory counters.
 * Asynchronous on `stream`; PNP_E_ARG on a bad size or alignment.
 */
pnp_status pnp_debug_copy(pnp_ctx ctx, const void* src, void* dst, size_t bytes, void* stream);

/*
 * Pass timing.  When enabled, every evaluation records HIP events around
 * each of its passes on the caller's stream (no synchronisation is added).
 * pnp_profile_read() waits for the recorded events, adds their durations to
 * per-pass totals and returns, for pass ids 0..n-1, the summed milliseconds
 * and the number of launches since the last reset (reset = 1 clears them).
 * Pass ids: 0 radial tables, 1 z forward (densities), 2 y forward
 * (densities), 3 x forward + weights, 4 y inverse (weighted densities),
 * 5 z derivatives, 6 y forward (derivatives), 7 x back-convolution + pair
 * kernels, 8 y inverse (chemical potentials), 9 z inverse + finalize.
 */
enum { PNP_NUM_PASSES = 10 };
pnp_status pnp_profile_enable(pnp_ctx ctx, int32_t enable);
/* Record events only around the passes whose bit (1 << pass id) is set in
 * mask (default: all); fewer events disturb the timed stream less. */
pnp_status pnp_profile_select(pnp_ctx ctx, uint32_t mask);
pnp_status pnp_profile_read(pnp_ctx ctx, double* ms, int32_t* launches, int32_t n, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* PNP_CDFT_H */
