/*
 * bbdg.h — C ABI of libbbdg: Bernstein-Bezier discontinuous Galerkin solver
 * for the first-order acoustic wave equation on affine tetrahedral meshes,
 * running on AMD Instinct MI355X (gfx950).
 *
 * What is computed.  The PDE (1/kappa) p_t + div u = 0, rho u_t + grad p = 0
 * with rho = 1 and kappa = c^2 constant per element (paper, Section 2), in
 * the upwind DG discretisation of Section 2 (fluxes with tau_p = 1/{{rho c}},
 * tau_u = {{rho c}}, {{.}} the arithmetic mean) written in strong form with
 * the inverse mass matrix applied (the ODE system of Section 3).  The
 * unknowns are the Bernstein-Bezier coefficients of p, u, v, w on every
 * element (Section 3.1).  One right-hand-side evaluation is
 *   volume term:  the sparse barycentric derivative operators of Lemma 1
 *                 (Section 3.1.1, Appendix A.1) and the chain rule;
 *   surface term: upwind flux on the face control points, the face operator
 *                 L_0 and the lift reduction E_L of the factorisation
 *                 L^f = E_L^f L_0 (Section 3.1.2, Appendix A.3), E_L applied
 *                 one degree reduction at a time;
 * and a time step is the five-stage low-storage RK4 of Carpenter and Kennedy
 * cited in Section 4.2 (volume, surface and update fused in one kernel per
 * stage).
 *
 * Conventions shared by every entry point.
 *   Orders:      1 <= N <= 9.  Np = (N+1)(N+2)(N+3)/6 coefficients per element
 *                and field, Nfp = (N+1)(N+2)/2 per face.
 *   Coefficient order: alpha = (a0,a1,a2,a3), |alpha| = N, a3 slowest, then a2,
 *                then a1 fastest (a0 = N-a1-a2-a3); bbdg_alpha_table lists it.
 *                Barycentric coordinate lambda_i belongs to local vertex i of the
 *                element; B_alpha = N!/alpha! lambda^alpha.
 *   Faces:       local face f is the face opposite local vertex f.
 *   Fields:      device arrays of shape (K, 4, Np), row-major: element-major,
 *                each element's coefficients of p, u, v, w (in that order) in
 *                one contiguous block of 4 Np values, so that an element's
 *                state is read and written as one coalesced run.  Element type
 *                is double (BBDG_F64) or float (BBDG_F32) as chosen at create
 *                time.
 *   Geometry:    host array geo of shape (K, 10) double: d(lambda_i)/dx,
 *                d(lambda_i)/dy, d(lambda_i)/dz for i = 1, 2, 3 (9 values), then
 *                J = 3 V / 4 (V the element volume; J > 0 required).
 *   Connectivity: host arrays (K, 4): EToE = neighbour element across face f or
 *                -1 on the domain boundary; EToF = the neighbour's local face;
 *                EToO = orientation code 0..5 of the shared face: with
 *                (a0<a1<a2) the own face's local vertices and (b0<b1<b2) the
 *                neighbour's, own vertex a_m is neighbour vertex b_pi(m), and
 *                EToO is the index of (pi(0),pi(1),pi(2)) in the list
 *                (0,1,2) (0,2,1) (1,0,2) (1,2,0) (2,0,1) (2,1,0).
 *   Streams:     `stream` is a hipStream_t passed as void* (NULL = default
 *                stream).  Every device call is stream-ordered and asynchronous;
 *                only bbdg_destroy synchronises.
 *   Ownership:   the caller owns every field, work and output buffer; the
 *                library owns only the device copies of geometry, connectivity
 *                and operator index tables, allocated in bbdg_create and freed
 *                in bbdg_destroy, and, on every device it runs on, the static
 *                work array of bbdg_run_noalloc (held until the process ends).
 *   Errors:      every int-returning call returns BBDG_OK (0) or a negative
 *                BBDG_E_* code; nothing throws across the ABI.  Arguments are
 *                validated before the device is touched.  A handle is not
 *                thread-safe; use one handle per stream.
 */
#ifndef BBDG_H
#define BBDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BBDG_OK 0
#define BBDG_E_ARG (-1)       /* null pointer, size or count out of range */
#define BBDG_E_ORDER (-2)     /* N outside 1..9 */
#define BBDG_E_MESH (-3)      /* bad vertex id, J <= 0, non-conforming or asymmetric connectivity */
#define BBDG_E_NONFINITE (-4) /* NaN or Inf in geometry, wavespeed or time-step arguments */
#define BBDG_E_DTYPE (-5)     /* unknown element type */
#define BBDG_E_BC (-6)        /* unknown boundary condition */
#define BBDG_E_DEVICE (-7)    /* HIP runtime error: device selection, allocation, copy */
#define BBDG_E_LAUNCH (-8)    /* kernel launch failed */
#define BBDG_E_MODE (-9)      /* unknown right-hand-side mode */
#define BBDG_E_OUTSIDE (-10)  /* a point lies in no element of the mesh */
#define BBDG_E_RESIDENT (-11) /* a persistent grid that cannot be co-resident on the device */
#define BBDG_E_TIMEOUT (-12)  /* a grid-wide barrier of a persistent launch timed out (see bbdg_status) */
#define BBDG_E_TOOBIG (-13)   /* the problem needs more work space than bbdg_run_noalloc holds */

enum { BBDG_F64 = 0, BBDG_F32 = 1 };

/* Domain-boundary exterior states (face of an element with EToE = -1):
 *   RIGID:            p+ = p-,  u+ = u- - 2 (n.u-) n   (wall with u.n = 0)
 *   PRESSURE_RELEASE: p+ = -p-, u+ = u-                (the mirror condition of Section 2)
 * with c+ = c- on the boundary. */
enum { BBDG_BC_RIGID = 0, BBDG_BC_PRESSURE_RELEASE = 1 };

/* What bbdg_rhs evaluates: the whole right-hand side, or only its volume
 * (derivative) or surface (flux + lift) part. */
enum { BBDG_RHS_FULL = 0, BBDG_RHS_VOLUME = 1, BBDG_RHS_SURFACE = 2 };

typedef struct bbdg_solver bbdg_solver;

/* Np for order N, or BBDG_E_ORDER. */
int bbdg_np(int N);

/* Fills alpha (host, Np x 4 int32, caller-allocated) with the multi-index
 * (a0,a1,a2,a3) of every coefficient in storage order (Section 3.1 defines
 * B_ijkl; the order is this library's). */
int bbdg_alpha_table(int N, int32_t* alpha);

/* Geometric factors and face connectivity of an affine tetrahedral mesh
 * (Section 3: affine maps, geometric factors, Jacobians; faces are matched
 * through their global vertex sets).  Inputs (host): VX (Nv x 3 double)
 * vertex coordinates, EToV (K x 4 int32) vertex ids of each element.
 * Outputs (host, caller-allocated): geo (K x 10), EToE, EToF, EToO (K x 4),
 * in the layouts above.  Fails with BBDG_E_MESH on an out-of-range vertex id,
 * J <= 0, or a face shared by more than two elements. */
int bbdg_mesh_geometry(int64_t K, int64_t Nv, const double* VX, const int32_t* EToV,
                       double* geo, int32_t* EToE, int8_t* EToF, int8_t* EToO);

/* Creates a solver for order N, element type dtype (BBDG_F64 / BBDG_F32),
 * K elements with the given connectivity (host), geometry (host, K x 10) and
 * wavespeed c (host, K doubles, c > 0; rho = 1, kappa = c^2), boundary
 * condition bc, on HIP device `device`; 4 K Np must stay below 2^31 (fields
 * are addressed with 32-bit offsets).  Everything is validated first:
 * connectivity must be symmetric (EToE[EToE[k][f]][EToF[k][f]] == k, with
 * EToF of that entry equal to f and a consistent inverse orientation). */
int bbdg_create(bbdg_solver** out, int N, int dtype, int64_t K,
                const int32_t* EToE, const int8_t* EToF, const int8_t* EToO,
                const double* geo, const double* c, int bc, int device);

/* Dense nodal comparator (not the Bernstein-Bezier method): the same DG
 * scheme (Section 2 flux, strong form of Section 3) in the Lagrange basis of
 * the equispaced lattice (the BB control-point positions), with dense
 * operators applied by MFMA (Section 4.2 describes the paper's nodal
 * comparators).  Same arguments and validation as bbdg_create; the fields of
 * such a solver are nodal values at the lattice points, in the coefficient
 * order of bbdg_alpha_table.  bbdg_rhs, bbdg_run, bbdg_work_bytes and
 * bbdg_destroy accept both kinds of handle. */
int bbdg_nodal_create(bbdg_solver** out, int N, int dtype, int64_t K,
                      const int32_t* EToE, const int8_t* EToF, const int8_t* EToO,
                      const double* geo, const double* c, int bc, int device);

/* Second dense nodal comparator, element per thread (Section 4.2 describes
 * the paper's blocked "element-per-thread" nodal kernels): the same scheme,
 * operators and field layout as bbdg_nodal_create, applied with vector FMAs by
 * one thread per element, in blocks of output rows whose operator entries are
 * shared by a wavefront of elements, after a flux kernel that writes the
 * upwind flux of every face node to a buffer the handle owns (4 x K x 4 Nfp
 * elements of the element type, allocated here).  Same arguments and validation as
 * bbdg_create; bbdg_rhs, bbdg_run, bbdg_run_noalloc, bbdg_work_bytes and
 * bbdg_destroy accept it; bbdg_basis returns 2. */
int bbdg_nodal_ept_create(bbdg_solver** out, int N, int dtype, int64_t K,
                          const int32_t* EToE, const int8_t* EToF, const int8_t* EToO,
                          const double* geo, const double* c, int bc, int device);

/* The comparator's dense operators of order N, as built at create time (host,
 * caller-allocated): dr (3 x Np x Np) with Dr_i = V (D^i - D^0) V^{-1}, so that
 * grad f = sum_i grad(lambda_i) Dr_i f, and lift (Np x 4 Nfp), the face lifts
 * V L^f Vf^{-1} of the four faces side by side (face f, face-local node g in
 * column f Nfp + g).  V, Vf: Bernstein-Vandermonde matrices of the volume and
 * face lattices. */
int bbdg_nodal_operators(int N, double* dr, double* lift);

/* 0 for a Bernstein-Bezier solver, 1 for the MFMA nodal comparator, 2 for the
 * element-per-thread nodal comparator, BBDG_E_ARG for NULL. */
int bbdg_basis(const bbdg_solver* s);

/* Order, element type and element count of a solver. */
int bbdg_info(const bbdg_solver* s, int* N, int* dtype, int64_t* K, int* Np);

/* One right-hand-side evaluation: rhs = A(q) (mode BBDG_RHS_FULL), or only
 * its volume or surface part.  q and rhs are device (K, 4, Np) arrays of the
 * solver's element type; they must not overlap. */
int bbdg_rhs(bbdg_solver* s, const void* q, void* rhs, int mode, void* stream);

/* Bytes of device work space that bbdg_run needs: the LSRK residual and a
 * second field buffer, 2 * 4 * K * Np elements. */
size_t bbdg_work_bytes(const bbdg_solver* s);

/* Advances q (device (K, 4, Np), in/out) by `steps` LSRK4 steps of size dt
 * from time t0.  work: device, >= bbdg_work_bytes(s), 256-byte aligned; its
 * contents on entry are ignored.  steps >= 0, dt finite. */
int bbdg_run(bbdg_solver* s, void* q, void* work, double t0, double dt, int64_t steps,
             void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): bbdg_run with the
 * work space taken from a static device array of BBDG_NOALLOC_WORK_BYTES
 * (64 MiB) that the library holds on every device it runs on until the
 * process ends, so that the call itself allocates nothing (no hipMalloc,
 * hipFree or allocating library routine).  Same arguments, kernels and
 * results as bbdg_run without `work`: q is the caller's device (K, 4, Np)
 * field, in/out.  Fails with BBDG_E_TOOBIG, before touching the device, when
 * bbdg_work_bytes(s) exceeds BBDG_NOALLOC_WORK_BYTES (e.g. FP64 with
 * 4 K Np > 1,048,576), and with BBDG_E_DEVICE if the array's address could
 * not be looked up when the first solver on the device was created.  The
 * array's contents on entry are ignored (nothing in it needs to start at
 * zero).  Every call on one device shares that device's array: calls that
 * overlap in time on one device (several streams or threads, any handles)
 * race and give undefined results; serialise them. */
#define BBDG_NOALLOC_WORK_BYTES ((size_t)64 << 20)
int bbdg_run_noalloc(bbdg_solver* s, void* q, double t0, double dt, int64_t steps, void* stream);

/* Output stores of the FP64 stage kernel that bbdg_run launches (a
 * performance choice; the arithmetic and results are identical):
 *   AUTO:        non-temporal stores (and residual loads) when the state,
 *                residual and second buffer, 3 x 4 K Np doubles, exceed the
 *                256 MB last-level cache of the MI355X, plain otherwise;
 *   PLAIN:       always plain stores;
 *   NONTEMPORAL: always non-temporal.
 * FP32 solvers, nodal comparators and batched runs always use plain stores.
 * The default is AUTO.  bbdg_set_store_policy fails with BBDG_E_ARG for an
 * unknown policy; bbdg_nontemporal_stores returns 1 if bbdg_run on this
 * handle uses the non-temporal variant, else 0 (BBDG_E_ARG for NULL). */
enum { BBDG_STORES_AUTO = 0, BBDG_STORES_PLAIN = 1, BBDG_STORES_NONTEMPORAL = 2 };
int bbdg_set_store_policy(bbdg_solver* s, int policy);
int bbdg_nontemporal_stores(const bbdg_solver* s);

/* ---- Batched shots: point sources and receivers ---------------------------
 * The paper's experiments have no forcing (f = 0 in Section 2); the batched
 * path adds the standard seismic source term to the pressure equation,
 *   (1/kappa) p_t + div u = w(t) delta(x - x_s),
 * discretised by the same Galerkin projection that defines the DG scheme
 * (the delta tested against every basis function of the element holding
 * x_s), and records receivers p(x_r, t) = sum_alpha p_alpha B_alpha(lambda(x_r))
 * (the Bernstein expansion of Section 3.1).  The wavelet is the Ricker
 * w(t) = (1 - 2 pi^2 f0^2 (t - ts)^2) exp(-pi^2 f0^2 (t - ts)^2). */

/* Point location (host).  For each of n points xyz (n x 3 double), elem[i]
 * is the lowest-numbered element whose barycentric coordinates of the point
 * are all >= -1e-10, and bary (n x 4 double) holds those coordinates with
 * negative values set to 0 and renormalised to sum 1.  VX, EToV as in
 * bbdg_mesh_geometry.  Returns BBDG_E_OUTSIDE when a point lies in no element
 * (its elem entry is -1; the other points are still filled). */
int bbdg_locate_points(int64_t K, int64_t Nv, const double* VX, const int32_t* EToV,
                       int64_t n, const double* xyz, int32_t* elem, double* bary);

/* Bernstein polynomials of order N at n barycentric points (host): out
 * (n x Np double) holds B_alpha(bary_i) = N!/alpha! prod_j lambda_j^alpha_j
 * (Section 3.1) in coefficient order.  Receiver weights are these values. */
int bbdg_bernstein_eval(int N, int64_t n, const double* bary, double* out);

/* Point-source vectors (host).  coef (n x Np double): for a point with
 * barycentric coordinates bary[i] in element elem[i],
 *   kappa_k (M^k)^{-1} B(lambda),   M^k = V_k m,
 *   m_ab = (N!)^2/(a! b!) 3! (a+b)!/(2N+3)!,
 * the element mass matrix of the Bernstein basis (exact simplex integral;
 * V_k = 4 J_k / 3 the element volume), so that adding w(t) coef to the
 * pressure right-hand side of element k is the projected source term above.
 * Fails with BBDG_E_ARG for an element id outside 0..K-1. */
int bbdg_source_coeffs(const bbdg_solver* s, int64_t n, const int32_t* elem, const double* bary,
                       double* coef);

/* Bytes of device work space that bbdg_run_batched needs for `shots` shots:
 * the LSRK residual and a second field buffer, 2 * shots * 4 * K * Np
 * elements, then the wavelet values at the stage times of one launch (5120
 * doubles). */
size_t bbdg_batched_work_bytes(const bbdg_solver* s, int64_t shots);

/* Advances `shots` independent states on the solver's mesh and wavespeed by
 * `steps` LSRK4 steps of size dt from time t0, in persistent cooperative
 * kernel launches of up to 1024 steps each (grid-wide barriers between the
 * stages), each preceded by a small kernel that tabulates the wavelet at its
 * stage times.
 *   q:        device (shots, K, 4, Np), in/out (shot-major; each shot is a
 *             (K, 4, Np) field as above).
 *   src_elem: device int32 (shots): source element of each shot, or -1 for a
 *             shot without source; NULL = no sources at all.
 *   src_coef: device (shots x Np) of the solver's element type: the
 *             bbdg_source_coeffs vector of each shot's source.
 *   f0, ts:   Ricker peak frequency (> 0) and delay; the wavelet is evaluated
 *             at each stage time t + c_s dt.
 *   R, rec_elem, rec_coef: R >= 0 receivers shared by all shots: device int32
 *             element ids (R) and device (R x Np) weights B_alpha(lambda_r).  A
 *             receiver whose element id is outside 0..K-1 records NaN.
 *   traces:   device (steps, shots, R) of the element type: the pressure at
 *             every receiver after every step.  May be NULL when R = 0.
 *   work:     device, >= bbdg_batched_work_bytes(s, shots), 256-byte aligned.
 *   wpb:      wavefronts per workgroup, 2, 4 or 8; 0 = the value
 *             bbdg_tune_batched chose for this shot count (4 if not tuned).
 * shots * ceil(K / E) must stay below 2^32 (E = elements per wavefront).
 * Fails with BBDG_E_RESIDENT, before anything runs, if the grid cannot be
 * co-resident.  Runs asynchronously on `stream`; a grid barrier that timed
 * out while it ran (q and traces are then NaN) is reported by bbdg_status.
 * Calls on one handle must not overlap (they share its barrier words). */
int bbdg_run_batched(bbdg_solver* s, void* q, int64_t shots, const int32_t* src_elem,
                     const void* src_coef, double f0, double ts, int R, const int32_t* rec_elem,
                     const void* rec_coef, void* traces, void* work, double t0, double dt,
                     int64_t steps, int wpb, void* stream);

/* Autotuner of the batched launch shape: times two-step batched runs of
 * `shots` zero states for every wavefronts-per-workgroup candidate (2, 4, 8),
 * which sets the elements per workgroup (one element group of 64/Np
 * elements, at least one, per wave, or one workgroup team where the order
 * has one of that size), stores the fastest in the handle (used by
 * bbdg_run_batched with wpb = 0) and returns it in *wpb.  A candidate whose grid barrier times out (see
 * bbdg_status) or that cannot be co-resident is skipped.  Returns
 * BBDG_E_TIMEOUT, without tuning, if an earlier run of the handle left a
 * timeout unreported.  scratch: device, >= bbdg_batched_work_bytes(s,
 * shots) + shots * 4 * K * Np elements, 256-byte aligned; its contents are
 * overwritten.  Synchronises the device. */
int bbdg_tune_batched(bbdg_solver* s, int64_t shots, void* scratch, int* wpb, void* stream);

/* Co-residency of the persistent batched kernel for this handle's order and
 * element type with wpb (2, 4, 8) waves per workgroup; record != 0 asks for
 * the instantiation that also records stages for the misfit gradient.
 * out (host, 6 int32): workgroups per CU that the runtime's occupancy query
 * reports; the bound derived from the kernel's own resources, which the
 * cooperative launches use (VGPRs: 512 per SIMD lane in granules of 8, at
 * most 8 waves per SIMD, two-wave workgroups counted as sharing two SIMDs;
 * LDS: 160 KiB per CU in 2 KiB granules; 0 for a kernel that uses scratch
 * memory; at most 8 and at most the query's count); VGPRs per lane; static
 * LDS bytes per workgroup; scratch bytes per lane; CUs of the device.
 * A shape whose bound is 0 is refused by bbdg_run_batched (BBDG_E_RESIDENT)
 * and skipped by bbdg_tune_batched; the misfit calls use the tuned shape when
 * both of its instantiations have a bound of at least 1, else the first of
 * 4, 2, 8 that has (BBDG_E_RESIDENT if none). */
int bbdg_batched_occupancy(const bbdg_solver* s, int wpb, int record, int32_t* out);

/* ---- Receiver misfit and its gradient ---------------------------------------
 * For the batched forward run above (shots, sources, receivers, t0, dt,
 * steps) with traces d (steps x shots x R) and observations d_obs of the same
 * shape, the misfit is J = 1/2 sum (d - d_obs)^2, and its gradient is taken
 * with respect to m = c^2 (= kappa, rho = 1) of every element.  The
 * gradient is the exact derivative of the discrete forward map (discrete
 * adjoint): every stage of the scheme is reversed with the transposed
 * operators (transposed barycentric derivatives of Lemma 1, L^{fT} =
 * L_0 (E_L^f)^T of Section 3.1.2 evaluated by degree raising, transposed
 * upwind flux of Section 2), and includes the dependence of the flux
 * weights tau_p = 2/(c- + c+), tau_u = (c- + c+)/2 and of the source vector
 * on m.  States use the solver's element type; gradient sums are FP64.
 * The forward states are kept at checkpoints every ckpt_every steps (0 = only
 * the initial state).  The work space holds the stage records of
 * rec_segments segments (>= 1; values above the segment count hold all of
 * them): the forward run records its last rec_segments segments, and every
 * other segment is recomputed once from its checkpoint, recording its stages,
 * during the reverse sweep.  A record slot takes 5 * ckpt_every * shots *
 * (K Np + 2 F Nfp) elements, F the number of distinct faces (an interior
 * face counts once: the pressure record of each element and the jumps of
 * each face), so the caller trades device memory for recomputed steps. */

/* Replaces the wavespeed (host, K doubles, c > 0) of a solver; the mesh is
 * unchanged.  Source vectors scale with kappa of their element: recompute
 * them with bbdg_source_coeffs afterwards.  Synchronises the device. */
int bbdg_set_wavespeed(bbdg_solver* s, const double* c);

/* Bytes of device work space for bbdg_misfit / bbdg_misfit_gradient with
 * these sizes (0 for invalid sizes, rec_segments < 1 included). */
size_t bbdg_misfit_work_bytes(const bbdg_solver* s, int64_t shots, int R, int64_t steps, int64_t ckpt_every,
                              int64_t rec_segments);

/* Runs the batched forward problem from q0 (device (shots, K, 4, Np), or NULL
 * for zero initial states), keeps checkpoints and traces in work (device,
 * >= bbdg_misfit_work_bytes, 256-byte aligned) and writes J (device, one
 * double).  Arguments as bbdg_run_batched; obs: device (steps, shots, R) of
 * the element type; R >= 1, steps >= 1, rec_segments >= 1 (else
 * BBDG_E_ARG) and the same as for bbdg_misfit_work_bytes. */
int bbdg_misfit(bbdg_solver* s, int64_t shots, const void* q0, const int32_t* src_elem,
                const void* src_coef, double f0, double ts, int R, const int32_t* rec_elem,
                const void* rec_coef, const void* obs, double t0, double dt, int64_t steps,
                int64_t ckpt_every, int64_t rec_segments, double* J, void* work, void* stream);

/* Gradient dJ/dm (device, K doubles) of the misfit of the last bbdg_misfit
 * call on the same work space, with the same arguments (its checkpoints and
 * traces are reused). */
int bbdg_misfit_gradient(bbdg_solver* s, int64_t shots, const void* q0, const int32_t* src_elem,
                         const void* src_coef, double f0, double ts, int R, const int32_t* rec_elem,
                         const void* rec_coef, const void* obs, double t0, double dt, int64_t steps,
                         int64_t ckpt_every, int64_t rec_segments, double* grad, void* work,
                         void* stream);

/* Measurement aid, not part of the method: copies `bytes` (a multiple of 16,
 * both pointers 16-byte aligned, no overlap) from device buffer src to dst
 * with a plain streaming kernel on the current device.  Used to measure the
 * bandwidth a simple copy reaches and to calibrate hardware byte counters. */
int bbdg_copy_probe(const void* src, void* dst, size_t bytes, void* stream);

/* Synchronises the solver's device and frees its tables.  Accepts NULL. */
int bbdg_destroy(bbdg_solver* s);

/* Status of the persistent (batched) launches of this handle: waits for the
 * device to finish its work, then returns BBDG_E_TIMEOUT (and clears the
 * flag) if a grid-wide barrier of any such launch since the last call timed
 * out, else BBDG_OK.  Those barriers bound their wait (2 s unless
 * bbdg_set_barrier_timeout says otherwise): a grid that the device does not
 * keep co-resident ends every workgroup instead of hanging, and the run's
 * outputs (q and traces of bbdg_run_batched, J and the gradient of the
 * misfit calls) are filled with NaN. */
int bbdg_status(bbdg_solver* s);

/* Longest wait at a grid barrier of the handle's persistent launches, in
 * seconds (0 .. 3600; default 2).  Fails with BBDG_E_ARG outside that range. */
int bbdg_set_barrier_timeout(bbdg_solver* s, double seconds);

/* The HIP error code (hipError_t) behind the last BBDG_E_LAUNCH or
 * BBDG_E_RESIDENT returned on this thread (0 if none): a diagnostic. */
int bbdg_last_hip_error(void);

/* Static description of an error code. */
const char* bbdg_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* BBDG_H */
