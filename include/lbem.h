/*
 * lbem.h -- C ABI of the MI355X (gfx950) lattice-Boltzmann Maxwell library.
 *
 * Two schemes from arXiv 2309.08068 are provided:
 *   LBEM_MM  Mendoza-Munoz model (Section II): 50 populations per cell, 12 face
 *            diagonal velocities in three planes plus two rest populations,
 *            lattice constants eps0 = 1, mu0 = 2 (vacuum speed 1/sqrt(2)).
 *   LBEM_HV  modified Hauser-Verhey model (Section III): 6 axis velocities, one
 *            electric and one magnetic 3-vector population each (36 scalars),
 *            with the current source term T_i = -(J.v_i) v_i / 2 of eq.
 *            (SourceTermHV); lattice constants eps0 = mu0 = 3 (speed 1/3).
 *   LBEM_MM_DIFF  the MM scheme in difference form: 24 populations per cell,
 *            d_i^{p(r)} = f_{i0}^{p(r)} - f_{i1}^{p(r)}.  D', B (eq.
 *            MacroscopicFieldsMiller) depend on the populations only through
 *            these differences, both populations of a pair move along the same
 *            v_i, and their equilibria (eq. equilibriumsMiller) differ by a
 *            term free of J, so d' = 2 d_eq - d evolves on its own and gives
 *            the E, B, D, H of LBEM_MM (equal up to FP32 rounding) at 24 / 50
 *            of its traffic.  The charge density of the sums and rest
 *            populations is not represented.
 * One time step (Appendix B) = collision with tau = 1/2 (moments, constitutive
 * relations and current, equilibria, f' = 2 f_eq - f [+ T]), imposition of hard
 * sources, advection f(x + v_q) <- f'(x).  All boundaries are periodic.
 *
 * Conventions shared by every call:
 *   - Cells are ordered x fastest: cell = x + nx * (y + ny * z); N = nx ny nz,
 *     1 <= N < 2^31.  Vector fields are [3][N] (component-major) float arrays.
 *   - "dev" pointers are device (HBM) pointers of the GPU that is current when
 *     the lattice is created; "host" pointers are ordinary host memory.
 *   - The caller owns every buffer, including the workspace; the library never
 *     allocates device memory.  A workspace must stay valid until destroy.
 *   - All work is enqueued on the stream given at create (or set_stream) and is
 *     asynchronous unless stated; outputs are valid after that stream syncs.
 *   - Functions return LBEM_OK or a negative lbem_status; lbem_last_error()
 *     gives a message for the calling thread.  Arguments are validated on the
 *     host before anything is enqueued; a failed call changes nothing.
 *   - A lattice handle must not be used from two threads at once.
 */
#ifndef LBEM_H
#define LBEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBEM_OK = 0,
    LBEM_EINVAL = -1,      /* bad argument (null, size, range, mismatched state) */
    LBEM_ENOMEM = -2,      /* workspace or buffer smaller than required */
    LBEM_EHIP = -3,        /* a HIP runtime call or kernel launch failed */
    LBEM_EUNSTABLE = -4,   /* media outside the stable range of the scheme; lbem_check: energy above the bound */
    LBEM_ESTATE = -5,      /* call not valid in the lattice's current state */
    LBEM_ENOTFINITE = -6   /* non-finite media; lbem_check: non-finite energy or detector sum */
} lbem_status;

typedef enum { LBEM_MM = 0, LBEM_HV = 1, LBEM_MM_DIFF = 2 } lbem_model;

/* Storage format of the populations.  Collision arithmetic is always FP32;
 * BF16/FP16 only change how populations are held in HBM (round to nearest
 * even on store).  FP16 multiplies by desc.storage_scale before rounding (and
 * divides after loading) so that small fields stay in the normal range.
 *
 * The *_SHIFTED formats store each population relative to an equilibrium:
 * a population leaving cell x is held as g_q = f'_q - phi_q(R_x), where R_x is
 * a per-cell record written by the same step (E, B, eps_r and 1/mu_r of x,
 * rounded to BF16, 16 bytes) and phi_q(R) is the field part of the equilibrium
 * of eqs. (equilibriumsMiller) / (equilibriumHV) evaluated on that record
 * (without the current term, which the paper's equilibria carry as v.J/16 for
 * MM and as the source term T_i for HV; rest populations unshifted).  Since
 * f' = 2 f_eq - f, g_q is the non-equilibrium part of the population, so the
 * 16-bit rounding acts on a small remainder instead of the whole value.  The
 * reader of population q at x adds phi_q(R_{x - v_q}) back.  Cost: 32 more
 * bytes per lattice update (one record written, one read) and two record
 * planes (2 x 16 B per cell) in the workspace.  Not available for batches. */
typedef enum {
    LBEM_F32 = 0,
    LBEM_BF16 = 1,
    LBEM_F16 = 2,
    LBEM_BF16_SHIFTED = 3,
    LBEM_F16_SHIFTED = 4
} lbem_storage;

typedef struct {
    int32_t model;         /* lbem_model */
    int32_t storage;       /* lbem_storage */
    int32_t nx, ny, nz;    /* lattice size, each >= 1 */
    int32_t reserved;      /* must be 0 */
    double storage_scale;  /* FP16 formats only: power of two > 0 (0 means 1); ignored otherwise */
} lbem_desc;

typedef struct lbem_lattice lbem_lattice;

/* Limits of the per-lattice tables held in the workspace. */
#define LBEM_MAX_SOURCES 65536
#define LBEM_MAX_PROBES 4096
#define LBEM_MAX_FLUX_CELLS 65536

/* Library version as major * 10000 + minor * 100 + patch. */
int32_t lbem_version(void);

/* Message describing the last failure on the calling thread ("" if none). */
const char *lbem_last_error(void);

/* Bytes of device workspace lbem_create needs for this descriptor.  The
 * workspace holds the populations (the state; see lbem_state_size for their
 * layout and padding), the record planes of the shifted formats, the media,
 * FP64 partial sums and the source, probe and monitor tables. */
lbem_status lbem_workspace_size(const lbem_desc *desc, size_t *bytes);

/* The same size as a return value: 0 if the descriptor is invalid (the reason
 * is in lbem_last_error). */
size_t lbem_workspace_bytes(const lbem_desc *desc);

/* Bytes of one population state (what save_state writes): the populations,
 * and for the shifted formats also the record plane the next step reads.  The
 * state is an opaque byte image.  Lattices whose rows take the row form of
 * the step kernel (see lbem_set_tuning) store each population plane with rows
 * a power of two of cells apart, in chunks of at most 32 KB per population
 * plane when they have more rows than one chunk holds (the last chunk
 * padded); other lattices store [Q][N].  A state is only meaningful to a
 * lattice with the same descriptor.
 * The step kernels use the padding only to finish a row's last 64-byte
 * write piece (they store values there that nothing reads), so it costs
 * almost no traffic, but it is real device memory: rows of nx cells take
 * 128, 256 or 512 cells (the next of these at or above nx), e.g. 288-cell rows
 * 512 (1.78x) and 384-cell rows 512 (1.33x: a 384^3 MM FP32 state is 15.1 GB
 * instead of 11.3 GB).  save_state / load_state copy the padded image, and
 * the adjoint keeps its checkpoints in this form. */
lbem_status lbem_state_size(const lbem_desc *desc, size_t *bytes);

/* Create a lattice.
 *   eps_r, mu_r, sigma: dev float [N] relative permittivity, relative
 *       permeability and conductivity (in the model's own units, Sections I-B
 *       and II-III); NULL means 1, 1 and 0.  They are copied into the workspace,
 *       so the caller may free them after the call returns.
 *   workspace: dev, >= lbem_workspace_size bytes, 256-byte aligned.
 *   stream: a hipStream_t (NULL = the null stream).
 * Validation (this call synchronises the stream once): every value finite
 * (else LBEM_ENOTFINITE), eps_r > 0, mu_r > 0, sigma >= 0 (else LBEM_EINVAL),
 * eps_r * mu_r >= 1 (else LBEM_EUNSTABLE: the wave would exceed the model's
 * vacuum speed, which the paper states is unstable), and for HV
 * sigma / (3 eps_r) < 2 (its explicit ohmic current is unstable beyond).
 * The populations start at zero (no field) at time level 0. */
lbem_status lbem_create(const lbem_desc *desc, const float *eps_r, const float *mu_r, const float *sigma,
                        void *workspace, size_t workspace_bytes, void *stream, lbem_lattice **out);

lbem_status lbem_destroy(lbem_lattice *lat);

/* Change the stream later work is enqueued on. */
lbem_status lbem_set_stream(lbem_lattice *lat, void *stream);

/* Initialise every cell to the equilibrium of the given fields (Appendix B,
 * first two lines): f = f_eq(E, B, J = 0), with rho_c = 0 for MM and D = eps E
 * for HV.  E, B: dev float [3][N].  Resets the time level to 0. */
lbem_status lbem_set_fields(lbem_lattice *lat, const float *E, const float *B);

/* Soft current sources (Section IV-C, Appendix B note): at time level n the
 * cells get J_src = J0[k] sin(2 pi n / period + phase), which enters the
 * current of eq. (MacorscopicCurrentMiller) for MM and the source term of eq.
 * (SourceTermHV) for HV.  Replaces every source set before.  cells: host int64
 * [n] distinct cell indices; J0: host float [n][3].  n = 0 removes all
 * sources.  n <= LBEM_MAX_SOURCES, period > 0.  Synchronises the stream.  The
 * weight sin(...) is evaluated in FP64 with whole periods removed first. */
lbem_status lbem_set_current_source(lbem_lattice *lat, int32_t n, const int64_t *cells, const float *J0,
                                    double period, double phase);

/* Add one soft point current at cell (x, y, z) with its own period and phase:
 * J_src(n) = J0 sin(2 pi n / period + phase) (Section IV-C), alongside the
 * sources already set.  J0: host float [3].  LBEM_EINVAL if the cell is outside
 * the lattice or already has a source, or the list is full.  Synchronises the
 * stream. */
lbem_status lbem_add_point_current(lbem_lattice *lat, int32_t x, int32_t y, int32_t z, const float *J0, double period,
                                   double phase);

/* Hard plane source (Appendix B "impose fields"): after the collision of step
 * n, every cell of the plane z gets f' = f_eq(E_imp, B_imp, J = 0) with
 * E_imp = E0 sin(2 pi n / period), B_imp = B0 sin(2 pi n / period).
 * E0, B0: host float [3].  z < 0 removes the source. */
lbem_status lbem_set_plane_source(lbem_lattice *lat, int32_t z, const float *E0, const float *B0, double period);

/* Probe series (the field time series at fixed points that the tests of
 * Sections IV-A to IV-C measure): every later step records E and B of the
 * state it collides (the fields reported at that time level) at the given
 * cells into
 * series[row][k][0..5] = (Ex, Ey, Ez, Bx, By, Bz), FP64, with
 * row = (n - n_set) mod cap_rows where n_set is the time level at this call.
 * cells: host int64 [n]; series: dev double [cap_rows][n][6].  n = 0 disables.
 * Synchronises the stream. */
lbem_status lbem_set_probes(lbem_lattice *lat, int32_t n, const int64_t *cells, int64_t cap_rows, double *series);

/* Energy-flux monitor for radiation patterns (Section IV-C: the largest
 * energy flux over one period at points of a sphere around a dipole): every
 * later step whose time level n (the level of the state it collides) lies in
 * [n_begin, n_end) first sets maxflux[k] = max(maxflux[k], |E x H|) with E and
 * H the fields reported at level n in cell cells[k] (FP64 product of the FP32
 * fields).  cells: host int64 [n], n <= LBEM_MAX_FLUX_CELLS, each in [0, N);
 * maxflux: dev double [n], owned by the caller, who initialises it (zeros)
 * and keeps it alive while the monitor is set; the library only folds into
 * it.  n = 0 disables.  Synchronises the stream. */
lbem_status lbem_set_flux_monitor(lbem_lattice *lat, int32_t n, const int64_t *cells, int64_t n_begin, int64_t n_end,
                                  double *maxflux);

/* Detector plane z (z < 0 disables): every later step adds the sum over the
 * plane of |E|^2 of the state it collides to an FP64 accumulator kept in the
 * workspace (deterministic order).  Setting the plane clears the accumulator.
 * This is the loss of the inverse-design problem (the energy that reaches a
 * plane); the paper measures transmitted fields at points behind the media
 * (Sections IV-A, IV-D). */
lbem_status lbem_set_detector(lbem_lattice *lat, int32_t z);
/* Write the accumulated detector sum to out (dev double [1]). */
lbem_status lbem_detector_read(lbem_lattice *lat, double *out);

/* lbem_set_detector(z), and after every later lbem_step call the accumulated
 * sum is also written to acc (dev double [1], owned by the caller, kept alive
 * while the plane is set), which this call zeroes: one small extra launch per
 * lbem_step call, not per step.  z < 0 disables (acc may then be NULL).
 * lbem_set_detector and lbem_adjoint_forward drop acc. */
lbem_status lbem_set_detector_plane(lbem_lattice *lat, int32_t z, double *acc);

/* Energy series: every later step whose time level n satisfies
 * (n - n_set) mod every == 0 writes U = 1/2 sum (E.D + B.H) of the state it
 * collides (FP64) to series[((n - n_set) / every) mod cap].  every <= 0 disables. */
lbem_status lbem_set_energy_series(lbem_lattice *lat, int32_t every, int64_t cap, double *series);

/* Advance nsteps time steps (asynchronous). */
lbem_status lbem_step(lbem_lattice *lat, int64_t nsteps);

/* Current time level. */
lbem_status lbem_get_time(lbem_lattice *lat, int64_t *t);

/* Reported fields of the current state (the pre-collision moments at the
 * current time level; MM's E is the corrected field of eq. MacroscopicEMiller
 * including the soft source at this time level).  Each of E, B, D, H is a dev
 * float [3][N] or NULL to skip.  MM: D = eps_r E, H = B / (mu0 mu_r);
 * HV: D and B are the moments, E = D / (eps0 eps_r), H = B / (mu0 mu_r). */
lbem_status lbem_get_fields(lbem_lattice *lat, float *E, float *B, float *D, float *H);

/* Field energy of Section I-B's linear media, U = 1/2 sum over cells of
 * (E.D + B.H) with D = eps_r eps0 E and H = B / (mu_r mu0), of the current
 * state -> out (dev double [1]).  FP64: per-block partials, then one
 * deterministic pass. */
lbem_status lbem_energy(lbem_lattice *lat, double *out);

/* Failure detection: computes the energy of the current state (as
 * lbem_energy) and, if a detector plane is set, its accumulated sum, waits
 * for both (synchronises the stream) and returns
 *   LBEM_ENOTFINITE if either is not finite (a NaN or infinity anywhere in
 *     the populations reaches the energy);
 *   LBEM_EUNSTABLE if max_energy > 0 and the energy exceeds it (growth: with
 *     eps_r or mu_r varying in 2-D or 3-D, both schemes have growing modes);
 *   LBEM_OK otherwise.  max_energy = 0 checks finiteness only.
 * energy: host double [1] receiving the energy, or NULL. */
lbem_status lbem_check(lbem_lattice *lat, double max_energy, double *energy);

/* Launch tuning of the step kernel, per parity (index 0 even, 1 odd time
 * level).  form[p] = kernel + 4 * order:
 *   kernel, for lattices whose x extent nx is 128, 256, 384 or 512, or
 *     fills at least 3/4 of the next of 128, 256, 384, 512 (one workgroup of that
 *     many threads per x-row, those past nx idle): 0 and 1 are the row
 *     form, whose +-1 x shifts go
 *     through LDS so that every HBM access is an aligned row, with store
 *     addresses formed before (0) or after (1, fewer registers) the
 *     collision; 2 addresses every neighbour directly; 3 does the same with
 *     each row split into workgroups of 128 threads.  Other lattices have
 *     one kernel and ignore this part.
 *   order 1 renumbers the workgroups so that each of the 8 XCDs (which
 *     receive workgroups in turn) takes groups of consecutive x-rows (one
 *     layout chunk, at least 16 rows), keeping neighbouring rows on one L2.
 * blocks_per_cu[p] caps the blocks resident per compute unit (0: no cap;
 * implemented with unused dynamic LDS).  Results are bit-identical for every
 * choice; only the speed differs.  create() sets measured defaults. */
lbem_status lbem_set_tuning(lbem_lattice *lat, const int32_t *form, const int32_t *blocks_per_cu);
lbem_status lbem_get_tuning(lbem_lattice *lat, int32_t *form, int32_t *blocks_per_cu);

/* Time every (form, cap) candidate for each parity over trial_steps launches,
 * then the four fastest again over 2 trial_steps launches in two alternating
 * rounds, and keep the fastest of those by their summed time.  backup: dev, lbem_state_size bytes; the state is
 * copied there first and restored afterwards, so the lattice is unchanged.
 * Synchronises the stream. */
lbem_status lbem_autotune(lbem_lattice *lat, int32_t trial_steps, void *backup);

/* Copy the population state to dst (dev, lbem_state_size bytes) / restore it
 * together with the time level it was saved at (get it with lbem_get_time).
 * Both are asynchronous device-to-device copies on the lattice's stream. */
lbem_status lbem_save_state(lbem_lattice *lat, void *dst);
lbem_status lbem_load_state(lbem_lattice *lat, const void *src, int64_t t);

/* ------------------------------------------------------------------------
 * Adjoint (reverse-time) differentiation of the detector loss.
 *
 * The step is affine in the populations for fixed media, f_{n+1} = S C_theta f_n
 * (S the advection, C_theta the per-cell collision of Sections II-III), so the
 * loss L = sum_{n=t0}^{t0+N-1} sum_{plane z_d} |E(f_n)|^2 has the adjoint
 *   lambda_n = C_theta^T S^T lambda_{n+1} + dl_n/df_n,   lambda_{t0+N} = 0,
 * and dL/dtheta_x accumulates mu_n(x)^T (dC_theta/dtheta_x) f_n(x) + dl_n/dtheta_x
 * with mu_n = S^T lambda_{n+1}; the first term needs only E(f_n) at x because
 * C(f) = 2 f_eq(m(f); theta) - f.  theta = (eps_r, sigma) per cell, mu_r fixed.
 * Memory: the forward stores a checkpoint every K steps; the backward
 * recomputes each segment storing E(f_n) per step (FP32 frames), then runs
 * the segment's adjoint steps in reverse (in-place AA streaming with reversed
 * velocities).  Gradients accumulate in FP32 over a segment and in FP64
 * across segments.  Every model (LBEM_MM_DIFF gives the gradients of LBEM_MM
 * at 24 / 50 of the traffic); no soft or hard sources may be set.
 * ------------------------------------------------------------------------ */

/* The adjoint needs FP32 population storage (LBEM_EINVAL otherwise): the
 * reverse kernels differentiate the unrounded FP32 step, which is the forward
 * map only when no population is rounded to 16 bits between steps. */

/* Bytes of adjoint workspace for nsteps steps with a checkpoint every K steps,
 * of which the last `keep` segments (>= 1) also hold their per-step E frames
 * (3 N floats per step) so that the reverse pass does not recompute them:
 * keep trades HBM for recomputation, keep = ceil(nsteps / K) recomputes nothing. */
lbem_status lbem_adjoint_workspace_size(const lbem_desc *desc, int64_t nsteps, int32_t K, int32_t keep,
                                        size_t *bytes);

/* The largest keep (1 <= keep <= ceil(nsteps / K)) whose adjoint workspace
 * fits in budget_bytes, written to *keep (host int32): the schedule with the
 * least recomputation a given amount of device memory allows.  Host-side
 * only, no GPU work.  LBEM_ENOMEM if even keep = 1 needs more than the
 * budget; otherwise as lbem_adjoint_workspace_size. */
lbem_status lbem_adjoint_keep(const lbem_desc *desc, int64_t nsteps, int32_t K, size_t budget_bytes,
                              int32_t *keep);

/* Run nsteps steps from the current state (time level t0) recording
 * checkpoints in ws, and write L (sum over the collided states of the plane
 * det_z of |E|^2, FP64) to loss (dev double [1]).  Leaves the lattice at
 * t0 + nsteps.  The last `keep` segments also keep E(f_n) of each of their
 * steps in ws, so the reverse pass recomputes only the earlier segments.
 * LBEM_ESTATE if sources are set. */
lbem_status lbem_adjoint_forward(lbem_lattice *lat, int64_t nsteps, int32_t K, int32_t keep, int32_t det_z,
                                 void *ws, size_t ws_bytes, double *loss);

/* Reverse pass for the last lbem_adjoint_forward with this ws: writes
 * dL/deps_r and dL/dsigma (dev double [N]) times `scale`.  If E0 and B0 (dev
 * float [3][N]) are given, the state at t0 is taken to be f_eq(E0, B0) of the
 * current media (lbem_set_fields), and its dependence on eps_r is included.
 * Leaves the lattice state as the forward left it.  The first call on a
 * lattice also times the adjoint kernel's launch variants on the workspace
 * (as lbem_autotune does for the step kernel; synchronises the stream once)
 * and keeps the fastest for later calls. */
lbem_status lbem_adjoint_backward(lbem_lattice *lat, void *ws, size_t ws_bytes, const float *E0, const float *B0,
                                  double scale, double *grad_eps, double *grad_sigma);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lbem_adjoint
 * with its workspace in a fixed device array of lbem_adjoint_static_bytes()
 * bytes (64 MiB) that the library holds on every GPU it runs on until the
 * process ends, instead of a caller buffer.  Same arguments, results and
 * errors as lbem_adjoint, except:
 *   - LBEM_ENOMEM if lbem_adjoint_workspace_size for (nsteps, K, keep)
 *     exceeds that size (nothing is enqueued);
 *   - the GPU the lattice was created on must be current (LBEM_EINVAL);
 *   - a lattice without an adjoint tuning (lbem_set_adjoint_tuning) gets
 *     form 0 and no cap instead of the timing lbem_adjoint's first reverse
 *     pass does (which creates HIP events); the gradients are the same bits.
 * It calls no allocating routine.  Every call on one GPU uses the same array:
 * calls that overlap on one GPU (several streams or threads) race and give
 * wrong gradients.  The array keeps the last call's contents; nothing in it
 * needs to start at zero. */
size_t lbem_adjoint_static_bytes(void);
lbem_status lbem_adjoint_static(lbem_lattice *lat, int64_t nsteps, int32_t K, int32_t keep, int32_t det_z,
                                const float *E0, const float *B0, double scale, double *grad_eps, double *grad_sigma,
                                double *loss);

/* Launch tuning of the adjoint kernel per parity of the reverse pass, as
 * lbem_set_tuning (form 0, 1 or 2; no split rows, no block order).  Setting it
 * skips the timing that the first lbem_adjoint_backward would do; results are
 * bit-identical for every choice.  get returns -1 before either happened. */
lbem_status lbem_set_adjoint_tuning(lbem_lattice *lat, const int32_t *form, const int32_t *blocks_per_cu);
lbem_status lbem_get_adjoint_tuning(lbem_lattice *lat, int32_t *form, int32_t *blocks_per_cu);

/* Both passes in one call: lbem_adjoint_forward(nsteps, K, keep, det_z, loss)
 * then lbem_adjoint_backward(E0, B0, scale, grad_eps, grad_sigma), with the
 * same arguments, workspace and errors. */
lbem_status lbem_adjoint(lbem_lattice *lat, int64_t nsteps, int32_t K, int32_t keep, int32_t det_z, const float *E0,
                         const float *B0, double scale, double *grad_eps, double *grad_sigma, double *loss, void *ws,
                         size_t ws_bytes);

/* ------------------------------------------------------------------------
 * Batched ragged 1-D lattices (Section IV-D generalised to many stacks).
 *
 * n independent periodic 1 x 1 x L_b lattices of one model, concatenated:
 * instance b owns cells [offsets[b], offsets[b+1]) of every per-cell array.
 * All instances share the time level.  One call of lbem_batch_step advances
 * every instance by nsteps steps in ONE persistent kernel launch: each
 * workgroup owns whole instances (longest first, to the least-loaded
 * workgroup) and separates the steps (or temporally blocked passes, see
 * lbem_batch_set_blocking) of an instance by workgroup barriers, so no
 * grid-wide synchronisation is needed.  In 1-D only the z components of
 * the velocities stream; MM's xy-plane populations and HV's +-x, +-y
 * populations stay in their cell.
 * ------------------------------------------------------------------------ */
typedef struct lbem_batch lbem_batch;

/* offsets: host int64 [n + 1], offsets[0] = 0, strictly increasing, total < 2^31. */
lbem_status lbem_batch_workspace_size(int32_t model, int32_t storage, int32_t n, const int64_t *offsets,
                                      size_t *bytes);

/* eps_r, mu_r, sigma: dev float [total] or NULL (1, 1, 0); validated as in
 * lbem_create (synchronises the stream once).  storage as lbem_storage
 * (FP16 uses no scale). */
lbem_status lbem_batch_create(int32_t model, int32_t storage, int32_t n, const int64_t *offsets, const float *eps_r,
                              const float *mu_r, const float *sigma, void *workspace, size_t workspace_bytes,
                              void *stream, lbem_batch **out);
lbem_status lbem_batch_destroy(lbem_batch *b);

/* f := f_eq(E, B, J = 0) in every cell; E, B dev float [3][total].  Time level 0. */
lbem_status lbem_batch_set_fields(lbem_batch *b, const float *E, const float *B);

/* Launch shape of the persistent kernel: threads per workgroup (64, 128, 256,
 * 512 or 1024) and workgroups per compute unit (>= 1).  Re-plans the
 * instance assignment. */
lbem_status lbem_batch_set_launch(lbem_batch *b, int32_t threads, int32_t groups_per_cu);

/* Temporal blocking of the persistent launch (0 = off, the default; else an
 * even number in [2, 64]; needs 256, 512 or 1024 threads per workgroup).  Each
 * over an instance advances it by steps_per_pass steps with its cells held in
 * registers and the z-moving populations exchanged through LDS, so HBM sees
 * one read and one write of the populations per pass instead of per step.
 * An instance of at most `threads` cells stays resident for all the steps of
 * a call; a longer one is swept in trapezoidal tiles of `threads` cells, each
 * storing the threads - 2 steps_per_pass cells it updates exactly, with the
 * overwritten halo cells kept in LDS.  The results are bit-identical to one
 * step per pass: every post-collision value is rounded to the storage format
 * between steps, as the stored form would be.  An odd first or last step of a
 * call runs one step at a time.  Costs 2 steps_per_pass / (threads - 2
 * steps_per_pass) extra collisions on long instances.  Needs a population
 * array below 2 GiB (LBEM_EINVAL otherwise). */
lbem_status lbem_batch_set_blocking(lbem_batch *b, int32_t steps_per_pass);
lbem_status lbem_batch_get_blocking(lbem_batch *b, int32_t *steps_per_pass);

/* Time each candidate launch shape over trial_steps steps (at least two
 * passes for a temporally blocked candidate; the state is saved and restored,
 * so the batch is left unchanged) and keep the fastest per step.  Candidates:
 * one step per pass at 128 to 1024 threads, and temporal blocking at 256 or
 * 1024 threads with 16 to 64 steps per pass.  Synchronises the stream.  The
 * chosen shape is written to threads / groups_per_cu (either may be NULL);
 * the chosen blocking is read with lbem_batch_get_blocking. */
lbem_status lbem_batch_autotune(lbem_batch *b, int32_t trial_steps, int32_t *threads, int32_t *groups_per_cu);

/* Advance every instance by nsteps steps: one persistent kernel launch. */
lbem_status lbem_batch_step(lbem_batch *b, int64_t nsteps);

/* The same nsteps as a HIP graph holding the persistent launch, captured on
 * first use for this (nsteps, parity) and replayed afterwards. */
lbem_status lbem_batch_step_graph(lbem_batch *b, int64_t nsteps);

/* Reference schedule: one kernel launch per instance per step. */
lbem_status lbem_batch_step_per_instance(lbem_batch *b, int64_t nsteps);

/* Reported fields (as lbem_get_fields) of every cell: dev float [3][total] or NULL. */
lbem_status lbem_batch_get_fields(lbem_batch *b, float *E, float *B);

lbem_status lbem_batch_get_time(lbem_batch *b, int64_t *t);

#ifdef __cplusplus
}
#endif

#endif /* LBEM_H */
