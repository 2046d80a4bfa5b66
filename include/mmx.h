/*
 * mmx.h -- C ABI of the MI355X (gfx950) demag + exchange + LLG hot path.
 *
 * The operations follow the paper's statement of the finite-difference
 * micromagnetic problem (Cheng, Kurokawa, Yuasa, "Magnum.np.distributed"):
 *   - the LLG equation, eq. (1), advanced by classic fixed-step RK4 and by
 *     the paper's adaptive Runge-Kutta-Fehlberg 4(5) step;
 *   - the effective field as a sum of terms (text after eq. (1));
 *   - the Heisenberg exchange field, eq. (2), with uniform A;
 *   - the DMI field, eq. (3), and the local fields the Implementation
 *     section names (uniaxial anisotropy, Slonczewski spin-transfer torque);
 *   - the Barzilai-Borwein energy minimiser of the Implementation section;
 *   - the demagnetisation field as the convolution of eq. (4) with the
 *     cell-averaged Newell tensor, done as a zero-padded FFT convolution
 *     (Implementation section and Fig. 1), on one GPU, unsharded;
 *   - the mesh (cell counts and cell size) and the material {Ms, A, alpha}
 *     of the paper's standard-problem listing.
 *
 * Units are SI: metres, A/m, J/m, seconds, gamma in m/(A s).
 *
 * Layout of every per-cell vector array (m, h, gradients): C-contiguous
 * (nx, ny, nz, 3) -- x slowest, the vector component fastest -- in the plan's
 * precision (float for MM_F32, double for MM_F64).  Per-cell scalars (Ms,
 * its gradient) are (nx, ny, nz).  Such arrays are DEVICE pointers owned by
 * the caller; the library never frees them.  A cell with Ms == 0 is vacuum:
 * it has no moment, no exchange field and is nobody's exchange neighbour.
 *
 * Error behaviour: every call returns MM_OK (0) or a negative MM_E* code, and
 * records a message retrievable with mm_last_error() (thread-local).  All
 * argument validation happens on the host before anything is enqueued, so a
 * rejected call has no device side effect.  Work is enqueued asynchronously
 * on the plan's HIP stream; a device fault surfaces as MM_EHIP at the next
 * call that synchronises.  No C++ exception crosses this boundary.
 *
 * Threading: a plan is not thread-safe; distinct plans are independent.
 *
 * Test hooks (environment, read at plan creation; every choice computes the
 * same result): MMX_XVAR=0..3 and MMX_YVAR=0..6 force an x or y pass variant
 * (see mm_plan_info), MMX_NO_CT selects the runtime-planned kernels for every
 * pass, MMX_ORDER="x:4,5,5;y:2,3,3,5" sets the radix order of runtime-planned
 * (non-power-of-two) axes, MMX_TEST_FAIL_ALLOC makes every device
 * allocation fail (MM_ENOMEM), MMX_NO_I32 keeps 64-bit cell indices in the
 * compile-time z-inverse kernels, MMX_NO_FANOUT runs a batch's launch groups of
 * one pass one after the other on its stream instead of side by side.  The
 * autotuner reads MMX_AUTOTUNE and
 * MMX_AUTOTUNE_CACHE (mm_plan_opts.autotune).
 */
#ifndef MMX_H
#define MMX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MM_OK 0
#define MM_EINVAL (-1)      /* invalid argument                              */
#define MM_ENOMEM (-2)      /* device or host allocation failed              */
#define MM_EHIP (-3)        /* HIP runtime error (includes "no GPU")         */
#define MM_ESTATE (-4)      /* call not valid in the plan's current state    */
#define MM_ENOTSUP (-5)     /* valid request this build does not support     */
#define MM_ENONFINITE (-6)  /* a synchronous result is not finite (NaN/Inf)  */

/* precision of a plan: the type of m, h, Ms and of the FFT arithmetic */
#define MM_F32 1
#define MM_F64 2

/* field terms for h_eff / h_eff_adjoint */
#define MM_DEMAG 1u
#define MM_EXCHANGE 2u

/* llg_step flags */
#define MM_NO_RENORM 1u     /* skip the end-of-step normalisation m <- m/|m| */
#define MM_NO_GRAPH 2u      /* enqueue kernels directly, no HIP graph replay */

typedef struct mm_plan mm_plan;
typedef struct mm_batch mm_batch;

/* Plan options.  Fill with mm_plan_opts_default() and change what you need. */
typedef struct mm_plan_opts {
    double far_radius;  /* P: the tensor uses Newell's closed form for offsets
                           |r|_2 <= P*max(cell) and a 27-node moment-matched
                           dipole quadrature beyond; P <= 0: Newell everywhere.
                           Default 16. */
    int64_t L[3];       /* zero-padded FFT length per axis; 0 = chosen by
                           pow2_padding.  A given L must be 7-smooth and
                           >= 2n-1 (any such L gives the same linear
                           convolution). */
    int autotune;       /* launch schedule (x and y kernel variants and tile
                           widths, radix order of the runtime-planned
                           transforms), timed on the plan's own buffers at
                           creation (by mm_batch_create per launch group):
                           0 off (default schedule); 1 cached: take the
                           winner recorded for this device, precision, pass,
                           length and size, timing the candidates only on a
                           miss; 2 search: always time them.  Winners are
                           recorded in a per-process cache; the environment
                           variable MMX_AUTOTUNE=off|cached|search overrides
                           this field and MMX_AUTOTUNE_CACHE=<file> keeps
                           the cache in a text file across processes.
                           mm_plan_schedule / mm_batch_schedule report the
                           outcome. */
    int pow2_padding;   /* for axes without an explicit L.  0: the 7-smooth
                           length (1 if n == 1, 2n if n is 7-smooth, else
                           the smallest 7-smooth length >= 2n-1); 1: the
                           smallest power of two >= 2n-1 (what
                           mm_batch_create uses without opts); 3: the
                           smallest length >= 2n-1 with compile-time
                           kernels: powers of two (x, y up to 4096; z and an
                           FP64 y up to 2048) and q * 2^k with one odd radix
                           q = 3, 5, 7 (x, y: 96, 160, 192, 224, 320, 384,
                           448, 640, 768, 896, 1280, 1536, 1792; z: the same
                           up to 896); 2 (default): that length when it
                           is at most 1.75 times the 7-smooth length, else
                           the 7-smooth length (runtime-planned kernels). */
} mm_plan_opts;

int mm_plan_opts_default(mm_plan_opts *opts);

/*
 * demag_tensor_init -- create a plan for a grid and compute its demag tensor.
 * Follows Mesh(n, dx) + DemagField() of the paper's listing; the tensor is
 * the cell-averaged kernel of eq. (4) (Newell).
 *   out        receives the plan (set to NULL on failure)
 *   grid[3]    cells per axis nx, ny, nz >= 1 (host array)
 *   cell[3]    cell size dx, dy, dz > 0 in metres (host array)
 *   precision  MM_F32 or MM_F64; the tensor is always evaluated and
 *              transformed in FP64 and rounded once to this precision
 *   hip_stream hipStream_t the plan enqueues on (NULL = default stream)
 *   opts       nullable
 * Synchronises the stream before returning.  The plan owns its device memory
 * (tensor spectrum, FFT workspace, twiddles) until mm_plan_destroy.
 * Returns MM_ENOTSUP when one padded y line of three components does not fit
 * a workgroup's 160 KiB of LDS: Ly <= 4096 for power-of-two Ly and
 * 3 (Ly+1) complex values otherwise, i.e. at most 6826 (FP32) or 3412 (FP64)
 * for other 7-smooth lengths, and at most 2048 for power-of-two Ly in FP64.
 */
int demag_tensor_init(mm_plan **out, const int64_t grid[3], const double cell[3], int precision,
                      void *hip_stream, const mm_plan_opts *opts);

int mm_plan_destroy(mm_plan *plan);

/*
 * mm_plan_bytes -- device memory a plan for this grid needs (host only; no
 * GPU call), so that the caller can own it (mm_plan_attach_memory).
 *   grid[3], precision, opts  as for demag_tensor_init (the cell size does not
 *              change the sizes)
 *   tensor_bytes    receives the size of the tensor spectrum (real octant,
 *              6 components, plan precision)
 *   workspace_bytes receives the size of everything else the forward path
 *              keeps: the two spectrum workspaces, the RK4 stage and
 *              accumulator fields, twiddle tables, descriptors and energy
 *              partials (sub-buffers start on 256-byte boundaries).
 * The scratch of the RK4-step adjoint, RKF45 and minimiser entry points is not part of
 * it: see mm_plan_scratch_bytes.
 */
int mm_plan_bytes(const int64_t grid[3], int precision, const mm_plan_opts *opts, size_t *tensor_bytes,
                  size_t *workspace_bytes);

/*
 * mm_plan_attach_memory -- move the plan onto caller-owned device memory.
 *   tensor_buf     device buffer of at least tensor_bytes (mm_plan_bytes for
 *                  the plan's grid, precision and options), 256-byte aligned;
 *                  receives the tensor spectrum
 *   workspace_buf  device buffer of at least workspace_bytes, 256-byte aligned
 * Synchronises the plan's stream, copies the spectrum into tensor_buf, frees
 * the plan's own buffers (and any captured graph or plan-owned scratch) and
 * rebuilds the plan's tables in workspace_buf; the autotuned launch shapes
 * are kept.  From then on the plan allocates no device memory of its own:
 * it uses only these buffers and the scratch attached with
 * mm_plan_attach_scratch (an entry point that needs more scratch than is
 * attached returns MM_ESTATE); the caller keeps them alive and
 * untouched until mm_plan_destroy, which does not free them.  At most once
 * per plan (MM_ESTATE otherwise).  The sizes cannot be checked: smaller
 * buffers than mm_plan_bytes reports are undefined behaviour.  On an error
 * after the copy the plan is left without a tensor and every later call
 * returns MM_ESTATE.
 */
int mm_plan_attach_memory(mm_plan *plan, void *tensor_buf, void *workspace_buf);

/*
 * mm_plan_scratch_bytes -- device scratch that the entry points beyond the
 * forward path need, per call (host only; no GPU call):
 *   bytes_out[0]  llg_step_adjoint (14 vector fields: the recomputed stages)
 *   bytes_out[1]  llg_rkf45_step (six stage derivatives and the candidate)
 *   bytes_out[2]  mm_minimize_bb (previous m, two gradients, block sums)
 * grid, precision, opts as for demag_tensor_init.  One region serves all of
 * them (each uses it only within one call, in stream order), so the largest
 * of the three covers every entry point.  h_eff, llg_step and h_eff_adjoint
 * need no scratch.
 *
 * mm_plan_attach_scratch -- use the caller's device buffer (256-byte
 * aligned, `bytes` long) as that scratch from now on.  Synchronises the
 * plan's stream and frees any scratch the plan allocated itself.  The
 * caller keeps the buffer alive until mm_plan_destroy (which does not free
 * it) or the next attach.  A plan that owns its memory (no
 * mm_plan_attach_memory) and has no attached scratch allocates the region
 * on the first call that needs it and grows it when a later call needs more.
 */
int mm_plan_scratch_bytes(const int64_t grid[3], int precision, const mm_plan_opts *opts, size_t bytes_out[3]);
int mm_plan_attach_scratch(mm_plan *plan, void *buf, size_t bytes);

/*
 * mm_plan_set_stream -- enqueue the plan's later work on hip_stream.  The new
 * stream first waits (an event, no host synchronisation) for everything
 * already enqueued on the previous one, since the plan's workspace, scratch
 * and captured graph serve every call.
 */
int mm_plan_set_stream(mm_plan *plan, void *hip_stream);

/*
 * mm_plan_set_dmi -- add the Dzyaloshinskii-Moriya field of eq. (3),
 *   h_dmi = 2D/(mu0 Ms_i) sum_k e_k^DMI x dm/dk,
 * with e^DMI = (e_y, -e_x, 0) (kind 1, interfacial) or (e_x, e_y, e_z)
 * (kind 2, bulk), to every later field evaluation of the plan (h_eff,
 * llg_step, llg_rkf45_step, mm_minimize_bb).  dm/dk are central differences
 * (m_{i+1} - m_{i-1})/(2 d_k); the paper gives no boundary condition, and a
 * neighbour outside the grid or with Ms = 0 is taken equal to the cell (its
 * difference is zero).  kind 0 or D = 0 removes the term.  D in J/m^2.
 * The energies of h_eff report demag and exchange only; the adjoint entry
 * points return MM_ENOTSUP while the term is set.  Synchronises the stream.
 */
int mm_plan_set_dmi(mm_plan *plan, int kind, double D);

/*
 * mm_plan_set_anisotropy -- add the uniaxial anisotropy field
 * 2 Ku/(mu0 Ms_i) (m_i . u) u, one of the local fields of section
 * "Implementation", to every later field evaluation of the plan (as for
 * mm_plan_set_dmi).  Ku in J/m^3 (0 removes the term); axis: host double[3],
 * any non-zero length (normalised here; ignored when Ku = 0).  The energies
 * of h_eff do not include it; the adjoint entry points return MM_ENOTSUP
 * while it is set.  Synchronises the stream.
 */
int mm_plan_set_anisotropy(mm_plan *plan, double Ku, const double axis[3]);

/*
 * mm_plan_set_stt -- add the Slonczewski spin-transfer torque, the other
 * local field of section "Implementation" (the paper times it beside demag
 * and exchange and takes its model from the cited literature), as an
 * effective field in every later field evaluation of the plan (as for
 * mm_plan_set_dmi):
 *   h_stt = beta_i [eps(m . p) (m x p) + eps_prime p],
 *   beta_i = hbar j / (mu0 e Ms_i d_layer),
 *   eps(x) = P lambda^2 / ((lambda^2 + 1) + (lambda^2 - 1) x).
 * j: current density (A/m^2, 0 removes the term); P: spin polarisation;
 * lambda > 0: the Slonczewski asymmetry parameter; eps_prime: the field-like
 * ratio; d_layer > 0: free-layer thickness (m); pol: host double[3], the
 * polarisation direction, any non-zero length (normalised here).  The other
 * arguments are ignored when j = 0.  0 in cells with Ms = 0.  The energies of
 * h_eff do not include it (the torque is not conservative); the adjoint entry
 * points return MM_ENOTSUP while it is set.  Synchronises the stream.
 */
int mm_plan_set_stt(mm_plan *plan, double j, double P, double lambda, double eps_prime, double d_layer,
                    const double pol[3]);

/* Padded lengths, device bytes held, and the launch shapes in use (each
 * nullable): tiles = {z cell columns per tile, forward x columns per tile,
 * y pass variant, forward x variant, inverse x variant}; x variants 0 and 1
 * are two tile widths, 2 the half-LDS kernel with variant 1's tiles, 3 the
 * half-LDS kernel with tiles twice as wide (lines of 1024 points or more);
 * y variants (power-of-two y lengths) 0 the LDS-resident pencil per
 * workgroup, 1 the register-resident pencil with half-line exchanges, 2 the
 * LDS-resident pencil with the waves' butterflies rotated per workgroup, 3
 * the persistent kernel with the next pencil's loads in flight, 4 the same
 * held to three waves per SIMD, 5 the persistent kernel with its twiddles
 * read from a table of the Ly roots of unity in LDS, 6 the pencil split
 * into its even and odd half-spectra, run one after the other through an LDS
 * pencil of Ly/2 positions (Ly 1024 to 4096); -W: the runtime-planned
 * kernel with W pencils per tile. */
int mm_plan_info(const mm_plan *plan, int64_t L[3], size_t *device_bytes, int tiles[5]);

/*
 * mm_plan_schedule -- the launch schedule a plan runs, as JSON text: padded
 * lengths, the x (forward, inverse), fused y and z kernels (specialised or
 * runtime-planned, variant as in mm_plan_info, tile widths) and the radix
 * order of each axis's transform.  buf: host buffer of len bytes, receives
 * a NUL-terminated string; MM_EINVAL when it does not fit.  Host only.
 */
int mm_plan_schedule(const mm_plan *plan, char *buf, size_t len);

/*
 * h_eff -- effective field h = [H_demag] + [H_exchange] in A/m (eqs. (2), (4)).
 *   m          device (nx,ny,nz,3) unit vectors
 *   Ms         device per-cell (nx,ny,nz) saturation magnetisation, or NULL
 *              to use Ms_scalar for every cell
 *   A          exchange stiffness (J/m), uniform
 *   h_out      device (nx,ny,nz,3); must not alias m
 *   terms      a subset of MM_DEMAG | MM_EXCHANGE; the plan's local terms
 *              (DMI, anisotropy, spin-transfer torque) are always added, and
 *              terms = 0 evaluates them alone (MM_EINVAL if the plan has none)
 *   energy_out host double[2] or NULL: receives (E_demag, E_exchange) in J,
 *              E = -(mu0/2) V sum Ms m.h per term, accumulated in FP64 with a
 *              fixed-order reduction; non-NULL makes the call synchronous,
 *              and a non-finite energy (from non-finite inputs) returns
 *              MM_ENONFINITE after h_out and energy_out are written.
 */
int h_eff(mm_plan *plan, const void *m, const void *Ms, double Ms_scalar, double A, void *h_out,
          unsigned terms, double *energy_out);

/*
 * mm_llg_stability -- stiffness of the explicit LLG step (host only, no GPU
 * call): omega_dt = gamma (2A/(mu0 Ms_min)) sum_a 4/d_a^2 dt, the largest
 * exchange precession rate a grid of cell size `cell` (host double[3]) can
 * carry, times the step.  Classic RK4 is stable on the imaginary axis up to
 * 2 sqrt(2) ~ 2.83; a larger value means llg_step will diverge on the
 * shortest wavelengths.  Ms_min > 0: the smallest Ms of a non-vacuum cell.
 * The Python binding warns when an llg_step call with scalar Ms exceeds the
 * bound.  MM_EINVAL for non-finite or non-positive arguments.
 */
int mm_llg_stability(const double cell[3], double Ms_min, double A, double gamma, double dt, double *omega_dt);

/*
 * llg_step -- n_steps classic RK4 steps of eq. (1) for unit m:
 *   dm/dt = -gamma/(1+alpha^2) [ m x h + alpha m x (m x h) ],
 *   h = H_demag + H_exchange (+ h_ext).  Follows llg.step(state, dt).
 *   m          device (nx,ny,nz,3), read and overwritten with m(t + n dt)
 *   Ms, Ms_scalar, A  as in h_eff
 *   alpha >= 0, gamma > 0, dt > 0, n_steps >= 0
 *   h_ext      host double[3] uniform applied field (A/m) or NULL
 *   flags      MM_NO_RENORM, MM_NO_GRAPH
 * Stage inputs are not normalised; the step ends with m <- m/|m| unless
 * MM_NO_RENORM.  The first call with a given argument set captures one step
 * in a HIP graph that later calls replay.  Asynchronous.
 */
int llg_step(mm_plan *plan, void *m, const void *Ms, double Ms_scalar, double A, double alpha,
             double gamma, double dt, int n_steps, const double h_ext[3], unsigned flags);

/*
 * llg_rkf45_step -- one attempted step of eq. (1) with the Runge-Kutta-
 * Fehlberg 4(5) method, the paper's integrator (section "Implementation":
 * the step size follows from the maximum error over the whole grid).
 *   m          device (nx,ny,nz,3); overwritten with the step's result only
 *              when the step is accepted
 *   Ms, Ms_scalar, A, alpha, gamma, h_ext  as in llg_step
 *   dt         host double: in, the step to attempt (> 0); out, the next step
 *              dt * min(5, max(0.2, 0.9 (tol/err)^(1/5))) (5 dt when err = 0),
 *              after an accepted or a rejected attempt
 *   tol        > 0: the step is accepted when err <= tol
 *   flags      MM_NO_RENORM (else the accepted result is renormalised)
 *   err_out    host double: err = max over cells and components of
 *              |y5 - y4|, the difference of the fifth- and fourth-order
 *              solutions (reduced on the device; a maximum is order-free)
 *   accepted   host int: 1 if m was advanced by dt (to the fourth-order
 *              solution, Fehlberg's pairing), else 0 (m unchanged)
 * Synchronous (the host needs err to decide).  The six stage derivatives and
 * the candidate live in the plan's scratch (mm_plan_scratch_bytes).  A
 * non-finite err returns MM_ENONFINITE with m unchanged.
 */
int llg_rkf45_step(mm_plan *plan, void *m, const void *Ms, double Ms_scalar, double A, double alpha,
                   double gamma, double *dt, double tol, const double h_ext[3], unsigned flags, double *err_out,
                   int *accepted);

/*
 * mm_minimize_bb -- relax m to a minimum of the energy (demag + exchange +
 * applied field) with Barzilai-Borwein step lengths, the paper's minimiser
 * (section "Implementation": the stopping criterion is reduced over the
 * whole grid).  Per iteration k: h = h_eff(m) + h_ext, g = m x (m x h) per
 * cell; stop when max |m x h| <= tol or k = max_iter; else
 * m <- normalise(m - tau g) with tau = (s.s)/(s.y) for odd k, (s.y)/(y.y)
 * for even k >= 2 (s, y: differences of m and g from the previous iterate,
 * sums over all cells and components in FP64), and 0.01 / max |m x h| at
 * k = 0 or when that value is not positive and finite.
 *   m          device (nx,ny,nz,3) unit vectors, overwritten with the result
 *   Ms, Ms_scalar, A, h_ext  as in llg_step
 *   tol        >= 0 (A/m); max_iter >= 0
 *   iters_out  host int: updates made; torque_out host double: max |m x h|
 *              of the returned m
 * Synchronous (one host read of four FP64 values per iteration).  Its three
 * vector fields and per-block sums live in the plan's scratch
 * (mm_plan_scratch_bytes).  A non-finite torque returns MM_ENONFINITE.
 */
int mm_minimize_bb(mm_plan *plan, void *m, const void *Ms, double Ms_scalar, double A, const double h_ext[3],
                   double tol, int max_iter, int *iters_out, double *torque_out);

/*
 * h_eff_adjoint -- vector-Jacobian product of h_eff (reverse-mode derivative
 * used for inverse problems, paper Introduction).  For the cotangent g_h:
 *   g_m  = Ms H_demag(g_h) + Lap(c g_h)          (c = 2A/(mu0 Ms))
 *   g_Ms = m . H_demag(g_h) - g_h . H_exchange(m) / Ms
 * The demag operator is self-adjoint, so it runs the same FFT pipeline and
 * tensor on g_h.  g_m: device (nx,ny,nz,3), overwritten.  g_Ms: device
 * (nx,ny,nz) or NULL, overwritten (per cell, also for a scalar Ms).  Runs
 * in the plan's workspace (no scratch).  Asynchronous.
 */
int h_eff_adjoint(mm_plan *plan, const void *m, const void *Ms, double Ms_scalar, double A,
                  const void *g_h, void *g_m, void *g_Ms, unsigned terms);

/*
 * llg_step_adjoint -- reverse of ONE llg_step (RK4 + normalisation) at state m.
 *   g        device (nx,ny,nz,3): in = cotangent of m(t+dt), out = cotangent
 *            of m(t)
 *   g_Ms     device (nx,ny,nz) accumulated (+=) with d<g, m(t+dt)>/dMs, or NULL
 * Other arguments as in llg_step.  Recomputes the four stages internally,
 * recording them in the plan's scratch (mm_plan_scratch_bytes).
 * Asynchronous.
 */
int llg_step_adjoint(mm_plan *plan, const void *m, const void *Ms, double Ms_scalar, double A,
                     double alpha, double gamma, double dt, const double h_ext[3], unsigned flags,
                     void *g, void *g_Ms);

/*
 * llg_step_adjoint_noalloc -- llg_step_adjoint for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, kernels and
 * result as llg_step_adjoint, but the 14 recorded fields live in a fixed
 * device array of MM_NOALLOC_SCRATCH_BYTES that the library brings with it
 * (one per GPU, held from the first call on that GPU until the process
 * ends) instead of the plan's scratch, and the call allocates nothing: no
 * hipMalloc, hipFree or allocating library routine.  The plan itself, its
 * workspace and the caller's m, Ms, g, g_Ms are used as by llg_step_adjoint.
 *   Errors: MM_ENOTSUP when the recorded fields need more than
 *   MM_NOALLOC_SCRATCH_BYTES (14 * 3 * nx*ny*nz * sizeof(real)); otherwise
 *   as llg_step_adjoint.  Checked on the host before anything is enqueued.
 * Every call on one GPU shares that GPU's array, whose contents persist from
 * the previous call (every recorded field is written before it is read):
 * calls that overlap on one GPU -- on different streams or from different
 * threads, for any plans -- race.  Asynchronous.
 */
#define MM_NOALLOC_SCRATCH_BYTES (128u << 20)
int llg_step_adjoint_noalloc(mm_plan *plan, const void *m, const void *Ms, double Ms_scalar, double A,
                             double alpha, double gamma, double dt, const double h_ext[3], unsigned flags,
                             void *g, void *g_Ms);

/*
 * Tensor test hooks.  host_octant is the real-space tensor N(i,j,k) for
 * 0 <= i < nx, 0 <= j < ny, 0 <= k < nz as a HOST double array
 * (nx,ny,nz,6), components xx,yy,zz,xy,xz,yz.
 *   get: evaluates the GPU's FP64 real-space tensor and copies it out.
 *   set: replaces the plan's tensor by the transform of the given octant
 *        (same FP64 transform and rounding as demag_tensor_init).
 * mm_demag_spectrum_get copies the stored, pre-scaled spectrum
 * -N^(k)/(Lx Ly Lz) for 0 <= kx <= Lx/2, 0 <= ky <= Ly/2, 0 <= kz <= Lz/2
 * into a HOST double array (Lx/2+1, Ly/2+1, Lz/2+1, 6).
 * All three synchronise.
 */
int mm_demag_tensor_get(mm_plan *plan, double *host_octant);
int mm_demag_tensor_set(mm_plan *plan, const double *host_octant);
int mm_demag_spectrum_get(mm_plan *plan, double *host_spectrum);

/*
 * Batched parameter sweep: `count` independent geometries, each with its own
 * grid, padded lengths, tensor and scalar Ms, advanced together.  Every pass
 * is a grouped launch over a ragged table of tiles -- one launch per distinct
 * padded length (geometries sharing a compile-time length run the specialised
 * kernels; all others share one runtime-planned launch) -- and one step of all
 * geometries is captured in one HIP graph.  The launch groups of one pass
 * touch disjoint geometries and run side by side: the batch forks up to three
 * internal streams of its own from the caller's stream with events and joins
 * them back before the next pass (parallel branches of the graph), so every
 * call stays ordered on the caller's stream.  opts NULL selects power-of-two
 * padding; opts->autotune times every kernel variant of each launch group
 * (forward and inverse x separately) on the batch's own buffers.  A geometry
 * whose whole three-component y pencil exceeds the LDS (FP64 y length 4096,
 * which single plans run as two half-spectra) is refused with MM_ENOTSUP.
 *   grids[count][3], cells[count][3]: host arrays
 *   m_ptrs[count]: host array of device pointers, each (nx,ny,nz,3)
 *   h_ptrs[count]: host array of device pointers for mm_batch_h_eff
 *   Ms[count]: host array of per-geometry scalar Ms
 */
int mm_batch_create(mm_batch **out, int count, const int64_t (*grids)[3], const double (*cells)[3],
                    int precision, void *hip_stream, const mm_plan_opts *opts);
int mm_batch_h_eff(mm_batch *b, void *const *m_ptrs, const double *Ms, double A, void *const *h_ptrs,
                   unsigned terms);
int mm_batch_llg_step(mm_batch *b, void *const *m_ptrs, const double *Ms, double A, double alpha,
                      double gamma, double dt, int n_steps, unsigned flags);
/*
 * mm_batch_tensor_set -- replace the tensor of one geometry of the batch by
 * the transform of a HOST real-space octant (nx,ny,nz,6) of that geometry,
 * as mm_demag_tensor_set does for a plan (the test hook that holds the
 * tensor equal in FP64 parity).  Synchronises.
 */
int mm_batch_tensor_set(mm_batch *b, int geometry, const double *host_octant);
int mm_batch_info(const mm_batch *b, int64_t *total_cells, size_t *device_bytes);
/* mm_batch_schedule -- the batch's launch groups as JSON text (pass, length,
 * kernel variant, tile width, geometries and tiles per group), as
 * mm_plan_schedule. */
int mm_batch_schedule(const mm_batch *b, char *buf, size_t len);
int mm_batch_destroy(mm_batch *b);

/*
 * Measurement hooks (used by the benchmark; no effect on results).
 * mm_plan_time_passes runs each pass of the pipeline `reps` times on the plan
 * stream between HIP events and writes the mean duration in ms of
 *   ms_out[0] z-forward (real-to-complex along z, source Ms m)
 *   ms_out[1] x-forward        ms_out[2] fused y (FFT, tensor product, IFFT)
 *   ms_out[3] x-inverse        ms_out[4] z-inverse + RK4 stage epilogue
 *   ms_out[5] z-inverse + h_eff epilogue
 * on the plan's own scratch arrays (contents irrelevant).  Synchronises.
 * mm_device_copy copies `bytes` (a multiple of 16) between device buffers with
 * a plain streaming kernel on `hip_stream` (the reference for bandwidth and
 * for hardware byte counters).
 */
int mm_plan_time_passes(mm_plan *plan, int reps, double ms_out[6]);
int mm_device_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Message for a status code (static storage). */
const char *mm_strerror(int status);
/* Detail of the last error on this thread (static thread-local storage). */
const char *mm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MMX_H */
