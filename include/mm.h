/*
 * mm.h -- C ABI of an MI355X-native finite-difference micromagnetic hot path.
 *
 * The method is the one of Bruckner, Koraltan, Abert & Suess, "magnum.np -- A
 * PyTorch based GPU enhanced Finite Difference Micromagnetic Simulation
 * Framework for High Level Development and Inverse Design" (arXiv:2302.08843):
 *   - a regular grid of nx*ny*nz cells of size dx*dy*dz (Sec. 2);
 *   - the effective field h = h_demag + h_exchange + h_anisotropy + h_zeeman
 *     (Sec. 4): demag as the zero-padded FFT convolution of M = Ms m with the
 *     cell-averaged Newell tensor in the near field and the point dipole
 *     beyond (Sec. 4.4, Eqs. convolution and dipole), the 6-neighbour
 *     exchange stencil with dm/dn = 0 (Sec. 4.2), first-order uniaxial
 *     anisotropy (Sec. 4.1) and a uniform external field;
 *   - further terms: second-order uniaxial and cubic anisotropy, per-cell
 *     exchange constants and DMI of the interface, bulk and D2d types
 *     (Sec. 4.2, 4.3), the Oersted field of a current density (Sec. 4.5);
 *   - thin layers of unequal height with the layers coupled densely per
 *     lateral frequency (the non-equidistant case of Sec. 4.4);
 *   - the LLG equation (Sec. 3, Eq. llg) integrated by an adaptive
 *     Dormand-Prince 5(4) or Runge-Kutta-Fehlberg 4(5) pair;
 *   - relaxation with high damping and no precession term (Sec. 3);
 *   - the linear-term energies (Sec. 4, Eqs. linear_energy(_discrete));
 *   - reverse-mode gradients for inverse design (Sec. 5.2) and a request
 *     server for many concurrent solves on one GPU.
 *
 * Units are SI: lengths in m, Ms and h in A/m, A in J/m, Ku in J/m^3, t in s.
 * gamma = 2.21e5 m/(A s) as printed with Eq. llg; mu0 = 4 pi 1e-7.
 *
 * Data layout.  A vector field (m, h, dm/dt) is one caller-owned DEVICE buffer
 * of 3*N values of the plan's precision (float for MM_FP32, double for
 * MM_FP64), component-major with x fastest:
 *     v[c*N + i + nx*(j + ny*k)],  c = 0,1,2 (x,y,z),  N = nx*ny*nz.
 * Scalar per-cell fields (Ms) use the same cell order with one component.
 *
 * Ownership.  The plan owns every internal buffer (spectral tensor, FFT
 * spectra, Runge-Kutta stages) and frees them in mm_plan_destroy, unless
 * they live in a caller workspace (mm_opts.workspace).  Caller
 * buffers are only read or written during the call (stream-ordered): they
 * must stay valid until the plan's stream has consumed the work.
 *
 * Ordering.  All device work of a plan runs on the plan's stream (mm_opts
 * .stream, a hipStream_t; NULL = the null stream).  mm_heff and mm_llg_rhs
 * enqueue work and return without synchronising.  mm_llg_step, mm_relax,
 * mm_energy and mm_max_torque return host values and synchronise the stream.
 *
 * Errors.  Every call returns an mm_status; no exception crosses the ABI.
 * mm_last_error() returns a thread-local message for the last failure.  On an
 * error the caller's output buffers are left unchanged, except that
 * mm_llg_step and mm_relax leave the last accepted state in m.
 *
 * Threads.  A plan is not thread-safe; distinct plans are independent.
 */
#ifndef MM_H
#define MM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mm_plan mm_plan;

typedef enum {
    MM_OK = 0,
    MM_EINVAL = -1,     /* invalid argument (sizes, cell, material, pointer) */
    MM_ENOMEM = -2,     /* device allocation failed                          */
    MM_EHIP = -3,       /* a HIP runtime call or kernel launch failed        */
    MM_ENONFINITE = -4, /* the magnetisation became NaN or infinite          */
    MM_EDTMIN = -5,     /* the adaptive step fell below dt_min               */
    MM_ENOTCONV = -6,   /* mm_relax hit max_steps before the torque criterion */
    MM_EBUSY = -7       /* resource temporarily unavailable                  */
} mm_status;

typedef enum { MM_FP32 = 0, MM_FP64 = 1 } mm_prec;

/* Field-term mask (Sec. 4). */
enum {
    MM_DEMAG = 1,
    MM_EXCH = 2,
    MM_ANIS = 4,
    MM_ZEEMAN = 8,
    MM_DMI = 16,     /* acts once mm_set_dmi gave a strength        */
    MM_OERSTED = 32, /* acts once mm_set_current gave a current     */
    MM_ALL = 63
};

/* DMI types of Sec. 4.3 (table of DMI types), by their DMI vectors
 * (e^dmi_x, e^dmi_y, e^dmi_z): interface (C_nv) (e_y, -e_x, 0), bulk (T or O)
 * (e_x, e_y, e_z), D_2d (-e_x, e_y, 0). */
enum { MM_DMI_INTERFACE = 0, MM_DMI_BULK = 1, MM_DMI_D2D = 2 };

typedef struct {
    int prec;            /* MM_FP32 (bulk arithmetic in float; tensor set up and
                            reductions in double) or MM_FP64                  */
    double ku_axis[3];   /* uniaxial easy axis; normalised by the library     */
    int demag_p;         /* Newell near-field radius in cells (Chebyshev index
                            distance, Sec. 4.4 default 20); < 0: Newell at
                            every distance                                    */
    void *stream;        /* hipStream_t for all device work; NULL = null stream */
    /* higher-order anisotropy (Sec. 4.3): second-order uniaxial ku2 along
     * ku_axis, h += 4 ku2 (e.m)^3 e / (mu0 Ms); cubic kc1, kc2 with principal
     * axes kc_axis1, kc_axis2 (orthonormalised by the library) and their
     * cross product.  Default 0.  Not linear in m: the differentiation entry
     * points reject plans that use them. */
    double ku2, kc1, kc2;
    double kc_axis1[3], kc_axis2[3];
    /* Thin layers of unequal height (Sec. 4.4, the non-equidistant case):
     * NULL for equal layers of height cell[2]; else a host array of nz
     * heights (m, positive; nz <= 16), stacked from z = 0, read during
     * mm_plan_create only.  The demag field then couples the layers densely
     * per lateral frequency (2-D FFT in x and y, O(nx ny log(nx ny) nz^2));
     * the z exchange uses 2/(dz_k (dz_k + dz_j)) in place of 1/dz^2 (the
     * flux between layer centres per layer height), the z part of DMI
     * 1/(2 dz_k) in place of 1/(2 dz), and the energies each layer's cell
     * volume.  cell[2] is ignored.  Such plans have no transposed operator
     * (mm_heff_vjp, mm_llg_rhs_vjp, mm_rk4_adjoint and the debug entry
     * points return MM_EINVAL). */
    const double *dz_layers;
    /* Caller-owned device workspace (e.g. a torch allocation) for the plan's
     * persistent buffers -- spectral kernel, FFT spectra, twiddles, reduction
     * buffers, the 10 Runge-Kutta vectors, the step controller and the error
     * norm's block partials -- laid out
     * by the library; at least mm_plan_workspace_bytes(grid, prec) bytes,
     * aligned to 256 bytes, equal layers only (MM_EINVAL otherwise).  NULL:
     * the plan allocates them itself.  The workspace must outlive the plan
     * and must not be shared by two live plans.  Set-up temporaries of
     * mm_plan_create and buffers of optional features (per-cell fields, the
     * Oersted kernel, the differentiation space) are still allocated by the
     * library. */
    void *workspace;
    size_t workspace_bytes;
} mm_opts;

/* Fill *o with defaults: MM_FP64, axis (0,0,1), demag_p 20, stream NULL,
 * no higher-order anisotropy, equal layers, no workspace. */
void mm_opts_default(mm_opts *o);

/* Device bytes of the workspace a plan of this grid and precision (MM_FP32
 * or MM_FP64, equal layers) needs for mm_opts.workspace (Sec. 2: the tensors
 * live in memory the caller provides): the folded spectral kernel
 * 6 (Pz/2+1)(Py/2+1) Hx reals, the spectra 3 nz ny Hx and 3 nz Py Hx complex
 * values, the twiddles, reduction buffers, 10 Runge-Kutta vectors of 3N
 * reals, the step controller and 2 ny nz doubles of error-norm partials,
 * each rounded up to 256 bytes (Hx = Px/2+1
 * rounded up to 128 bytes of reals).  Host-only, no device access.  0 for
 * an invalid grid or precision. */
size_t mm_plan_workspace_bytes(const int grid[3], int prec);

/* Create a plan for grid[3] = (nx, ny, nz) cells of size cell[3] = (dx, dy,
 * dz) with saturation magnetisation Ms, exchange constant A, uniaxial
 * anisotropy constant Ku and damping alpha (Sec. 2 mesh and material; Sec. 3
 * alpha).  Builds the demag kernel on the device (Newell tensor in
 * double-double arithmetic for the near field, dipole beyond, Sec. 4.4),
 * transforms it once and keeps its real spectrum resident.  Every grid
 * extent must be in [1, 512] (padded FFT length <= 1024).  Returns
 * MM_EINVAL for invalid sizes, a non-positive cell, Ms < 0, A < 0 or
 * alpha < 0; MM_ENOMEM if device memory runs out.  opt may be NULL
 * (defaults).  Synchronises the stream before returning. */
mm_status mm_plan_create(mm_plan **out, const int grid[3], const double cell[3], double Ms,
                         double A, double Ku, double alpha, const mm_opts *opt);

/* Release every device buffer of the plan (synchronises its stream first).
 * NULL is ignored. */
void mm_plan_destroy(mm_plan *p);

/* Device bytes held by the plan. */
size_t mm_plan_device_bytes(const mm_plan *p);

/* Padded FFT extents (Px, Py, Pz): 1 for a single layer, else the next power
 * of two >= 2n-1 (the zero padding of Sec. 4.4). */
void mm_plan_padded(const mm_plan *p, int P[3]);

/* Set a per-cell saturation magnetisation: Ms_cell is a device buffer of N
 * values in the plan's precision, copied into the plan (stream-ordered).
 * Ms = 0 marks a vacuum cell: its field, torque and dm/dt are zero and it is
 * left out of norms and energies; its exchange constant is taken as zero, so
 * neighbours see dm/dn = 0 there.  NULL restores the uniform Ms of
 * mm_plan_create. */
mm_status mm_set_ms(mm_plan *p, const void *Ms_cell);

/* Set a per-cell exchange constant (Sec. 4.2): A_cell is a device buffer of
 * N values (J/m, >= 0, finite; not checked) in the plan's precision, copied
 * into the plan (stream-ordered).  The coupling of neighbours i and j is the
 * harmonic mean 2 A_i A_j / (A_i + A_j) (0 when both vanish); a missing or
 * vacuum (Ms = 0) neighbour is skipped, so dm/dn = 0 there.  NULL restores
 * the uniform A of mm_plan_create.  The differentiation entry points reject
 * a plan that uses it with MM_EXCH. */
mm_status mm_set_exchange(mm_plan *p, const void *A_cell);

/* Set a per-cell first-order uniaxial anisotropy constant (Sec. 4.1, J/m^3,
 * along the plan's easy axis): Ku_cell is a device buffer of N values in the
 * plan's precision, copied into the plan (stream-ordered).  The field
 * 2 Ku_i/(mu0 Ms_i) e (e.m) and the energy density -Ku_i (e.m)^2 use it per
 * cell.  NULL restores the uniform Ku of mm_plan_create.  The
 * differentiation entry points reject a plan that uses it with MM_ANIS. */
mm_status mm_set_ku(mm_plan *p, const void *Ku_cell);

/* Set the DMI term (Sec. 4.3): h_i = 2/(mu0 Ms_i) sum_{k=+-x,+-y,+-z}
 * D~_{i,k} (e^dmi_k x m_{i+e_k}) / (2 Delta_k) with e^dmi_{-k} = -e^dmi_k and
 * the DMI vectors of `type` (MM_DMI_*).  D is a uniform strength in J/m^2;
 * if D_cell (a device buffer of N values in the plan's precision, copied into
 * the plan) is not NULL it gives per-cell strengths instead and D~ is their
 * average of Eq. D_avg: 2 D_i D_j / (D_i + D_j) for equal signs (0 when both
 * vanish), -sqrt(sqrt(-D_i D_j) |D_i + D_j| / 2) for opposite signs.  Missing
 * and vacuum neighbours are ignored (the open boundary of Sec. 4.3).
 * D = 0 with D_cell NULL removes the term.  MM_EINVAL for an unknown type or
 * a non-finite D.  The differentiation entry points reject a plan that uses
 * it with MM_DMI. */
mm_status mm_set_dmi(mm_plan *p, int type, double D, const void *D_cell);

/* Oersted field (Sec. 4.5) of a current density: h_out = sum_s j_s x G(X_t -
 * X_s) with G the cell-averaged Biot-Savart kernel (1/(4 pi V)) int_t int_s
 * (x - x')/|x - x'|^3 dx' dx within the near-field radius demag_p (closed
 * form from the antiderivative of Newell's f along the component's axis, in
 * double-double at set-up) and the singular current V D/(4 pi |D|^3) beyond
 * (Sec. 4.5: the far field of a singular current density).  j and h_out are
 * device buffers of 3N values of the plan's precision (A/m^2 in, A/m out),
 * must not alias; h_out holds the field at every cell.  The first call builds
 * and keeps the kernel spectrum, the folded octant of its imaginary part
 * (3 (Pz/2+1)(Py/2+1) Hx reals, Hx = Px/2+1 rounded up to 128 bytes), and
 * synchronises once; the convolution runs in the plan's own spectra, so later
 * calls allocate nothing and are asynchronous.  MM_EINVAL for thin-layer
 * plans. */
mm_status mm_oersted(mm_plan *p, const void *j, void *h_out);

/* Current density for the MM_OERSTED term: its Oersted field is computed now
 * (as mm_oersted) and kept; the term adds it, times sin(2 pi freq t) if freq
 * != 0 (a current of fixed shape and sinusoidal amplitude), on magnetic
 * cells.  Its energy is that of an applied field, counted in the Zeeman slot
 * of mm_energy.  j NULL removes the term.  Synchronises. */
mm_status mm_set_current(mm_plan *p, const void *j, double freq);

/* Time-dependent Zeeman drive added to the external field on masked cells:
 * H(t) += mask_i * amp * sin(2 pi freq t).  mask is a device buffer of N
 * bytes (0/1) copied into the plan; NULL removes the drive. */
mm_status mm_set_drive(mm_plan *p, const double amp[3], double freq, const unsigned char *mask);

/* Effective field h_out = sum of the terms selected by `terms` (MM_* mask)
 * at the state m and time t (t only matters for a drive).  h_ext is the
 * uniform external field in A/m (NULL = 0).  m and h_out are device buffers
 * of 3N values; they must not alias.  Asynchronous. */
mm_status mm_heff(mm_plan *p, const void *m, const double h_ext[3], unsigned terms, double t,
                  void *h_out);

/* LLG right-hand side dm/dt = -gamma/(1+alpha^2) [m x h + alpha m x (m x h)]
 * (Sec. 3, Eq. llg) with h the effective field of `terms` at (m, t).
 * Asynchronous. */
mm_status mm_llg_rhs(mm_plan *p, const void *m, const double h_ext[3], unsigned terms, double t,
                     void *dmdt_out);

typedef struct {
    double rtol, atol;  /* error tolerances of the step controller           */
    double t_end;       /* integrate until t reaches t_end ...               */
    long max_steps;     /* ... or until max_steps steps have been accepted   */
    double dt_min;      /* a step below dt_min gives MM_EDTMIN (0 -> 1e-20)  */
    int renorm;         /* renormalise |m| = 1 after each accepted step      */
    int method;         /* MM_DP45 (default) or MM_RKF45                     */
} mm_step_opts;

/* Embedded pairs of mm_llg_step: Dormand-Prince 5(4) (7 stages, the last
 * evaluated at the propagated 5th-order solution and reused as the next
 * step's first), and Runge-Kutta-Fehlberg 4(5), the paper's default (Sec. 3:
 * 6 stages, the 4th-order solution propagated, the 5th-order one used for the
 * error).  Both cost 6 right-hand sides per accepted step. */
enum { MM_DP45 = 0, MM_RKF45 = 1 };

typedef struct {
    long accepted, rejected, rhs_evals;
    double t, dt, err_last;
} mm_step_stats;

/* Adaptive integration of the LLG equation (Sec. 3) with the pair o->method
 * (Dormand-Prince 5(4) with first-same-as-last by default).  The error norm is
 * the RMS over magnetic components of e/(atol + rtol max(|y|,|y_new|)),
 * computed in double on the device; a step is accepted iff the norm <= 1 and
 * dt is rescaled by min(10, max(0.2, 0.9 err^-1/5)) (no growth right after a
 * rejection).  A trial step whose error norm is not finite (overflow) is
 * rejected with the factor 0.2; MM_ENONFINITE is returned only when the
 * current state itself holds a NaN or infinity.  *dt <= 0 selects the Hairer-Norsett-Wanner starting step.  m is
 * updated in place; *t and *dt are advanced.  st may be NULL.  Synchronises
 * once per step (8 bytes to the host).  MM_EINVAL for an unknown method. */
mm_status mm_llg_step(mm_plan *p, void *m, const double h_ext[3], unsigned terms, double *t,
                      double *dt, const mm_step_opts *o, mm_step_stats *st);

/* Relaxation (Sec. 3): integrate dm/dt = -gamma/2 m x (m x h) (alpha = 1, no
 * precession term) with renormalised Dormand-Prince steps at tolerance rtol
 * until max_i |m_i x h_i| / Ms_i < tol.  Returns MM_ENOTCONV with the last
 * accepted state in m if max_steps steps do not reach the criterion.  An
 * FP32 plan with uniform Ms, the plain stencil, equal layers and static
 * fields keeps the state in double (6N doubles allocated on first use) and
 * takes the exchange differences of the float stage input plus its rounding
 * residual, with the step decisions on the device (the host reads the
 * controller every 16 steps); other FP32 plans keep a float state, whose
 * rounding noise can hold the torque near 1e-5. */
mm_status mm_relax(mm_plan *p, void *m, const double h_ext[3], unsigned terms, double tol,
                   long max_steps, double rtol, mm_step_stats *st);

/* Energies (Sec. 4, Eq. linear_energy_discrete) in J, accumulated in double:
 * E[0] demag, E[1] exchange and E[5] DMI, each -1/2 mu0 V sum Ms m.h_t;
 * E[2] anisotropy, V times the sum of the anisotropy energy density (Sec.
 * 4.1 and 4.3: -Ku1 (e.m)^2 - Ku2 (e.m)^4 + Kc1 (cubic) + Kc2 (cubic));
 * E[3] Zeeman (with the Oersted field), -mu0 V sum Ms m.H; E[4] total of
 * the terms in `terms`.
 * Terms left out of `terms` read 0.  Synchronises. */
mm_status mm_energy(mm_plan *p, const void *m, const double h_ext[3], unsigned terms, double t,
                    double E[6]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * energies of mm_energy (same terms, same E[6], same kernels and reduction
 * order, so the same values) computed without any allocation.  The field
 * buffer (3N reals of the plan's precision) and the reduction partials and
 * results live in one static device array of MM_NOALLOC_SCRATCH_BYTES per
 * GPU, which each GPU the library runs on holds until the process ends; a
 * plan needing more than that (beyond 5.58 M cells in FP32, 2.79 M in FP64)
 * gives MM_EINVAL with the sizes in mm_last_error().  Every call on one GPU
 * uses that GPU's array and leaves its last contents there: calls that
 * overlap on one GPU (two host threads, or two streams in flight) race.
 * Synchronises the plan's stream. */
#define MM_NOALLOC_SCRATCH_BYTES (64u << 20)
mm_status mm_energy_noalloc(mm_plan *p, const void *m, const double h_ext[3], unsigned terms,
                            double t, double E[6]);

/* max_i |m_i x h_i| / Ms_i over magnetic cells.  Synchronises. */
mm_status mm_max_torque(mm_plan *p, const void *m, const double h_ext[3], unsigned terms,
                        double t, double *out);

/* ---- Differentiation (Sec. 5.2, inverse design by reverse-mode gradients) --
 * The effective field is affine in m: h = H m + h_zee(t), with H the sum of
 * the demag, exchange and anisotropy operators (Sec. 4).  These entry points
 * give the exact transposes used by reverse-mode differentiation; the Zeeman
 * term carries no m dependence and is ignored by the products.  All vectors
 * are device buffers of 3N reals of the plan's precision in the component-
 * major layout of mm_heff; grad_ms is N reals (per-cell saturation
 * magnetisation), optional (NULL) where stated.  Gradients with respect to
 * Ms treat the plan's Ms (uniform or per cell) as a per-cell field and are
 * accumulated in double on the device, then rounded to the plan's precision.
 * The first call allocates 16 work vectors of 3N reals (and N doubles),
 * released by mm_plan_destroy.  None of them synchronise except where noted. */

/* Transposed effective field: grad_m = H^T w and grad_ms = d(w . h)/dMs at
 * fixed m, for the terms in `terms` (the demag transpose reuses the resident
 * spectral tensor; the operator is symmetric as K_ab(r) = K_ba(-r)).  grad_m
 * must not alias m or w.  MM_EINVAL on null or aliased vectors. */
mm_status mm_heff_vjp(mm_plan *p, const void *m, const void *w, unsigned terms, void *grad_m,
                      void *grad_ms);

/* Vector-Jacobian product of the LLG right-hand side (Eq. llg with the
 * plan's alpha) at (m, t): grad_m = J^T w, grad_ms = d(w . dm/dt)/dMs at
 * fixed m (the field of m is recomputed first).  Same aliasing rules. */
mm_status mm_llg_rhs_vjp(mm_plan *p, const void *m, const double h_ext[3], unsigned terms,
                         double t, const void *w, void *grad_m, void *grad_ms);

/* Classical fourth-order Runge-Kutta integration with fixed step dt from t0
 * over nsteps steps (m advanced in place), with the time-averaged region loss
 *     L = (1/nsteps) sum_{n=1..nsteps} mean_{i in region} m_z,i(t_n)
 * written to *loss (0 if region is NULL or empty; loss may be NULL).  region
 * is N device bytes (nonzero = in the region).  If ckpt is not NULL it
 * receives the state before every step n with n % ckpt_every == 0:
 * ceil(nsteps / ckpt_every) vectors of 3N reals (the input of
 * mm_rk4_adjoint).  Synchronises at the end (and once to count the region). */
mm_status mm_rk4_forward(mm_plan *p, void *m, const double h_ext[3], unsigned terms, double t0,
                         double dt, long nsteps, const unsigned char *region, long ckpt_every,
                         void *ckpt, double *loss);

/* Discrete adjoint of mm_rk4_forward (reverse sweep over every RK4 stage, with
 * the LLG vector-Jacobian products above): from the checkpoints written by a
 * forward call with the same arguments, recomputes each segment of
 * ckpt_every steps, storing its 4 stage states and 4 stage fields per step
 * (a device segment of 8 ckpt_every vectors, allocated and kept by the plan),
 * and sweeps it backwards.  Writes dL/dMs (N reals, may be NULL) and dL/dm0
 * (3N reals, may be NULL), and the recomputed loss to *loss (may be NULL).
 * region must not be NULL.  Synchronises at the end. */
mm_status mm_rk4_adjoint(mm_plan *p, const void *ckpt, const double h_ext[3], unsigned terms,
                         double t0, double dt, long nsteps, const unsigned char *region,
                         long ckpt_every, void *grad_ms, void *grad_m0, double *loss);

/* ---- Serving: a request server with continuous batching ---------------------
 * Relaxations (Sec. 3: alpha = 1, no precession, renormalised steps, until
 * max_i |m_i x h_i| / Ms_i < tol) and time integrations (Eq. llg with the
 * request's alpha up to t_end) on grids of different sizes, run concurrently
 * on one GPU.  Requests of one grid class (grid, precision, near-field order
 * and cell proportions), kind, terms and tolerances share launches: a group
 * of up to `batch` of them (at most 2^17 cells together, within hbm_budget;
 * one where the x extent is 1) lives in one batch plan (spectra, Runge-Kutta
 * vectors -- in FP32 with the state in double, the float stage input's
 * rounding residual taken into the exchange differences -- and a device-side step
 * controller per request) on one of max_active streams, and every kernel of a
 * step covers all its requests.  The steps are decided on the device per
 * request (the same accept/reject and step-size rules as mm_llg_step) and
 * replayed from one HIP graph of steps_per_launch steps per group, so no step
 * waits for the host.  A request that finishes frees its slot for the next
 * request of the same group, which joins the running batch; other requests
 * start new groups first come first served as streams and device memory
 * (hbm_budget) free up, and groups overlap on the device.  Groups of one class
 * share one resident spectral kernel (the demag tensor depends on the cell
 * shape, not its size); finished groups stay resident for reuse and are
 * released, least recently used first, when memory is needed.  A request's
 * arithmetic does not depend on what else runs or which slot it takes, so its
 * result is bit-identical alone and in a mix.  Fields must be static (no
 * drive); the material is uniform per request.  The server is not
 * thread-safe: one host thread submits and polls. */
typedef struct mm_server mm_server;

typedef struct {
    size_t hbm_budget;     /* device bytes the server may hold; 0: 80 % of free memory */
    int max_active;        /* groups on the device at once (streams), 1..64 */
    int steps_per_launch;  /* device-controlled steps per graph launch, 1..64 */
    mm_prec prec;          /* arithmetic of every request */
    int demag_p;           /* near-field order as in mm_opts */
    int batch;             /* requests per group (shared launches), 1..64 */
} mm_serve_opts;
void mm_serve_opts_default(mm_serve_opts *o); /* 0, 16, 8, MM_FP32, 20, 8 */

enum { MM_SERVE_RELAX = 0, MM_SERVE_INTEGRATE = 1 };

typedef struct {
    int grid[3];
    double cell[3];
    double Ms, A, Ku, ku_axis[3], alpha; /* alpha unused by relaxations (1) */
    double h_ext[3];
    unsigned terms;
    int kind;          /* MM_SERVE_RELAX or MM_SERVE_INTEGRATE */
    double tol;        /* relaxation: torque criterion */
    double rtol, atol; /* step-size control */
    double t_end;      /* integration: end time (s) */
    long max_steps;    /* cap on accepted steps */
    void *m;           /* device, 3N reals of the server precision: start state in,
                          result out; owned by the caller, kept alive until completed */
    void *stream;      /* hipStream_t whose work so far produces m (NULL: the null
                          stream); the server reads m only after that work */
    long tag;          /* caller's identifier, returned in the completion */
} mm_request;

typedef struct {
    long tag;
    int status;        /* MM_OK, MM_ENOTCONV (relaxation hit max_steps), MM_EDTMIN,
                          MM_ENONFINITE, MM_ENOMEM (larger than the budget), MM_EHIP */
    long accepted, rejected, rhs_evals;
    double t, torque;  /* final time; final torque (relaxations; FP32: of the double
                          state, before the result is rounded to float) */
    double t_submit, t_admit, t_done; /* mm_serve_clock() seconds */
} mm_completion;

typedef struct {
    long submitted, admitted, completed, queued, active;
    long waited_memory, waited_slot; /* requests that waited at the head of the queue */
    size_t bytes_in_use, bytes_peak, budget;
    long tensors_built;
    long plans_created, plans_reused; /* admissions that built a group plan / used one */
    long graph_launches;
    long max_batch;                   /* most requests that shared one group at once */
} mm_serve_stats;

/* MM_EINVAL for options out of range; MM_ENOMEM/MM_EHIP on allocation. */
mm_status mm_serve_create(mm_server **out, const mm_serve_opts *o);
/* Queue a request (copied).  MM_EINVAL for invalid grids, materials or
 * tolerances; the request is then not queued. */
mm_status mm_serve_submit(mm_server *s, const mm_request *r);
/* Advance the server without blocking: collect finished graph launches,
 * relaunch running requests, retire finished ones, admit queued ones (an
 * admission synchronises on the new request's stream for its starting step).
 * Writes up to max_out completions (oldest first) and their count to *n_out;
 * more stay for the next call. */
mm_status mm_serve_poll(mm_server *s, mm_completion *out, int max_out, int *n_out);
mm_status mm_serve_get_stats(const mm_server *s, mm_serve_stats *st);
/* Waits for the device work of active requests, then frees everything. */
void mm_serve_destroy(mm_server *s);
/* Host monotonic clock (seconds) of the completion timestamps. */
double mm_serve_clock(void);

/* Per-pass timing with HIP events recorded on the plan's stream around every
 * launch of the field pipeline (diagnostics for roofline measurements).
 * Passes: x forward transform, y forward transform, last-axis transform with
 * the spectral product (the hottest pass), y inverse transform, x inverse
 * transform with the local terms, and the Runge-Kutta vector kernels.
 * mm_profile(p, 1) clears the totals and starts recording; mm_profile(p, 0)
 * stops.  mm_profile_read synchronises and returns the summed milliseconds
 * and launch counts per pass (arrays of MM_NPASS). */
enum { MM_PASS_X_FWD = 0, MM_PASS_Y_FWD = 1, MM_PASS_MID = 2, MM_PASS_Y_INV = 3,
       MM_PASS_X_INV_LOCAL = 4, MM_PASS_RK = 5, MM_NPASS = 6 };
mm_status mm_profile(mm_plan *p, int enable);
mm_status mm_profile_read(mm_plan *p, double ms[], long count[]);

/* Diagnostics for bit-level tests.  mm_debug_kernel writes the real-space
 * demag kernel K (h = sum K M) of component s (0..5 = xx,yy,zz,xy,xz,yz) as
 * placed in the zero-padded grid, Px*Py*Pz doubles with x fastest, into the
 * device buffer out.  mm_debug_spectrum writes the resident folded spectrum
 * of component s, (Pz/2+1)*(Py/2+1)*(Px/2+1) doubles with kx fastest,
 * including the 1/(Px Py Pz) normalisation of the inverse transform. */
mm_status mm_debug_kernel(mm_plan *p, int s, void *out);
mm_status mm_debug_spectrum(mm_plan *p, int s, void *out);

/* Thread-local message describing the last failure of this thread. */
const char *mm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MM_H */
