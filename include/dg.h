/*
 * dg.h -- C interface of libdgmoist: the explicit discontinuous Galerkin
 * right-hand side of the moist compressible Euler equations with implicit
 * condensation and optional Kessler warm rain, on MI355X (gfx950).
 *
 * The operations follow the paper's statement of the problem
 * (Hittmeir, Lederer, Schoeberl, von Wahl, arXiv 2305.13847):
 *   - unknowns U = (rho_d', rho_m', [rho_r'], m_1..m_d, E'), perturbations from
 *     a hydrostatic background that depends on height only (Section 2.3,
 *     perturbation formulation; Section 3, balance-law form);
 *   - rho_v, rho_c and T are recovered pointwise from the implicit
 *     condensation system (Section 2.2) before every right-hand side
 *     evaluation (Section 3.4);
 *   - DG weak form with the Lax-Friedrichs flux and the moist wave-speed bound,
 *     periodic or slip-wall boundaries (Section 3.2);
 *   - diagonal mass matrix and the SSPRK(4,3) time step (Section 3.3).
 * The spatial basis is nodal: tensor-product Gauss-Lobatto points on
 * structured boxes, which double as quadrature points (lumped, diagonal
 * mass); the L2 projection of Section 3.4 is then the identity.  The
 * paper's own Legendre basis with Gauss quadrature is selectable
 * (dg_params.basis).
 *
 * Memory and ownership
 *   All state arrays passed to the hot calls are DEVICE pointers owned by the
 *   caller.  The library never frees them.  The handle owns tables, background
 *   profiles, stage buffers and status words; these are allocated in
 *   dg_create / dg_create_batch and released in dg_destroy.  Hot calls
 *   (dg_rhs, dg_saturation_split, dg_rk_step, the *_vjp calls) allocate
 *   nothing and only enqueue work on the given stream.  Calls on one handle
 *   must not overlap in time (they share the handle's stage buffers).
 *
 * Layout
 *   U is structure-of-arrays U[v][e][n]: variable v in the order above,
 *   element e = ex + nx (ey + ny ez) (2D: e = ex + nx ez; the last axis is
 *   vertical), node n = i + (k+1) (j + (k+1) l) with i along x.  dtype is
 *   double (DG_FP64) or float (DG_FP32_BULK).  For a batch the members'
 *   elements are concatenated: member m owns elements
 *   [dg_member_offset(m), dg_member_offset(m) + ne_m) of every variable.
 *   Background arrays are per vertical node index iz = ez (k+1) + l.
 *
 * Errors
 *   Every call returns a dg_status; DG_OK is 0.  On any other status
 *   dg_last_error() returns a message (thread-local).  Argument errors are
 *   reported before anything is enqueued.  Problems found on the device
 *   (a Newton solve that did not converge, non-finite values, a state with no
 *   temperature above 50 K) never abort: they set status words that
 *   dg_get_stats reads.
 */
#ifndef DG_H
#define DG_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_handle dg_handle;

typedef enum {
  DG_OK = 0,
  DG_EINVAL = -1,        /* bad argument (sizes, orders, pointers)            */
  DG_ENOMEM = -2,        /* device allocation failed in dg_create*            */
  DG_EHIP = -3,          /* a HIP runtime call failed                          */
  DG_ENOCONV = -4,       /* dg_get_stats: some Newton solve did not converge  */
  DG_ENONFINITE = -5,    /* dg_get_stats: non-finite or invalid state seen    */
  DG_EUNSUPPORTED = -6   /* valid request this build does not implement       */
} dg_status;

enum { DG_PERIODIC = 0, DG_SLIPWALL = 1 };       /* boundary type per axis     */
enum { DG_FP64 = 0, DG_FP32_BULK = 1 };          /* precision of U and flux    */
enum { DG_SSPRK43 = 0, DG_SSPRK33 = 1 };          /* time integrator           */
enum { DG_VR_CONST = 0, DG_VR_COSMO = 1 };       /* terminal rain speed model  */
enum { DG_BASIS_LOBATTO = 0, DG_BASIS_GAUSS = 1 }; /* spatial basis (dg_params) */

/* Structured box mesh; axis dim-1 is vertical (gravity along -e_z).  bc[a]
 * applies to both ends of axis a. */
typedef struct {
  int dim;            /* 2 or 3                                  */
  int n[3];           /* elements per axis (n[a] >= 1)           */
  double lo[3], hi[3];
  int bc[3];          /* DG_PERIODIC or DG_SLIPWALL              */
} dg_mesh;

/* Model parameters.  Thermodynamic constants: the paper's appendix table;
 * g is not in the table (9.81).  Kessler/COSMO rain closure: Section 2.1. */
typedef struct {
  double g, cvd, cvv, cl, cpd, cpv, Rd, Rv, Lref, Tref, eref, pref;
  int rain;                   /* 0: nvars = 3 + dim; 1: nvars = 4 + dim       */
  int vr_mode;                /* DG_VR_CONST or DG_VR_COSMO                    */
  double vr_const;            /* m/s, for DG_VR_CONST                          */
  double rho_w, N0r, v0r;     /* COSMO terminal-speed parameters               */
  double q_au;                /* autoconversion threshold (0 in the paper)     */
  int precision;              /* DG_FP64 or DG_FP32_BULK                       */
  int rk;                     /* DG_SSPRK43 (default) or DG_SSPRK33            */
  double newton_rtol;         /* split stops when |dT| <= rtol * T (1e-14)     */
  int newton_maxit;           /* iteration cap (30); counted as non-converged  */
  /* Rayleigh sponge layer (Section 3.6): at the end of
   * every RK step, (rho_m', rho_r', m, E') <- (1 - delta(z)) (rho_m', rho_r',
   * m, E') with delta(z) = alpha/2 (1 - cos(pi (z - zD)/(zT - zD))) above zD
   * (zT the member's top, far-field velocity 0), and the moist mass removed
   * is added to rho_d' at the same node.  alpha = 0 (default) switches it
   * off; 0 < alpha <= 1 and zD below every member's top otherwise. */
  double sponge_zD;           /* m, bottom of the sponge layer                 */
  double sponge_alpha;        /* strength in [0, 1]                             */
  /* Spatial basis of Q^k.  DG_BASIS_LOBATTO (default): nodes at the k+1
   * Gauss-Lobatto points per axis, which double as quadrature points (lumped
   * mass).  DG_BASIS_GAUSS: the paper's own discretisation (Section 3.1,
   * Legendre modes with their exact diagonal mass, Gauss-Legendre quadrature
   * of k+1 points per axis; Section 3.4, split at the quadrature points and
   * L2 projection of T and rho_v), held by its values at the Gauss points:
   * U[v][e][n] and the background arrays are then values at the Gauss
   * points, and face fluxes use the traces of U', T and rho_v along each
   * normal line.  With DG_BASIS_GAUSS the adjoint calls dg_rhs_vjp and
   * dg_rk_step_vjp return DG_EUNSUPPORTED. */
  int basis;                  /* DG_BASIS_LOBATTO or DG_BASIS_GAUSS             */
  /* Artificial diffusion (Section 3.5), Lobatto basis only: the symmetric
   * interior penalty form on interior faces, with penalty
   * sip_sigma k^2 / h_n (the printed h^2/k is read as the usual k^2/h),
   * acting on the perturbation unknowns.  The viscosity is
   * sip_gamma 0.5 h^(1-d/2) ||u||_{0,K} per element (||u - v_r e_z||_{0,K}
   * for rho_r), h = |K|^(1/d), evaluated from every stage state, and carried
   * to a continuous Q1 field by vertex means.  Slip walls carry no
   * diffusive terms.  sip_gamma = 0 (default) switches it off.  With it
   * on, the adjoint calls return DG_EUNSUPPORTED, and so does dg_create*
   * with DG_BASIS_GAUSS. */
  double sip_gamma;           /* >= 0                                           */
  double sip_sigma;           /* > 0 (default 10)                               */
} dg_params;

typedef struct {
  long long splits;           /* node splits performed since the last reset    */
  long long nonconverged;     /* splits that hit newton_maxit                  */
  int max_iters;              /* largest Newton iteration count seen           */
  int nonfinite;              /* 1 if a non-finite or invalid state was seen   */
} dg_stats;

/* Fill *p with the paper's constants, no rain, FP64, SSPRK(4,3), no sponge. */
void dg_default_params(dg_params* p);

/* Create a handle for one mesh (Section 3.1 space on the box, Section 3.2
 * discretisation, with the model of Sections 2.1-2.3 in *p).  order k in 1..7
 * in 2D and 1..4 in 3D (a 3D element of order 5 or more has more nodes than a
 * thread block; one thread owns one node), nvars = 3 + dim (rain = 0) or
 * 4 + dim (rain = 1), otherwise DG_EINVAL.  A handle holds fewer than 2^29
 * nodes in FP64 and 2^30 in FP32 bulk (each variable's array stays below
 * 4 GiB), otherwise DG_EINVAL.  Device memory for tables, stage buffers and status
 * words is allocated here (DG_ENOMEM on failure).  *out receives the
 * handle; release it with dg_destroy. */
dg_status dg_create(const dg_mesh* mesh, int order, int nvars, const dg_params* p,
                    dg_handle** out);

/* Create a handle for an ensemble of nmembers meshes of the same order,
 * dimension and variable set; each member advances with its own dt. */
dg_status dg_create_batch(const dg_mesh* meshes, int nmembers, int order, int nvars,
                          const dg_params* p, dg_handle** out);

/* Background state of ensemble member `member` (0 for a single mesh): the
 * hydrostatic state the unknowns are perturbations of (Section 2.3).  HOST
 * arrays of n_z (k+1) doubles at the node heights, copied.  rho_r may be NULL
 * (taken as 0).  The background pressure is computed on the device as the
 * equation of state of the split background state.  Must be called for every
 * member before the first hot call; synchronises the device.  DG_EINVAL for a
 * bad member, a null array, a non-finite value or a state with no valid
 * temperature. */
dg_status dg_set_background(dg_handle* h, const double* rho_d, const double* rho_m,
                            const double* rho_r, const double* E, int member);

/* Element offset and element count of member m in the concatenated layout. */
dg_status dg_member_offset(const dg_handle* h, int member, long long* elem_offset,
                           long long* nelem);

/* Total number of values in one state array (nvars x elements x nodes). */
long long dg_state_size(const dg_handle* h);

/* dUdt = M^{-1} (volume + face + source terms) of the Section 3.2 weak form
 * with the diagonal mass of Section 3.3, after the pointwise split of
 * Section 3.4 (fluxes and sources of the Section 2.3 perturbation system,
 * Kessler sources of Section 2.1 when rain is on).  U and dUdt: caller-owned
 * device arrays in the state layout and precision; they must not alias
 * (DG_EINVAL).  Uses the handle's split buffers. */
dg_status dg_rhs(dg_handle* h, const void* U, void* dUdt, hipStream_t stream);

/* dg_rhs for callers that cannot allocate device memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels, with the split's per-node scratch (T and rho_vs(T), 16 bytes per
 * node) in a static device array of 32 MiB that the library holds on every
 * GPU it runs on until the process ends, instead of the handle's buffers.
 * The call allocates nothing.  Limits: at most 2^21 nodes (elements x nodes
 * per element) per handle, otherwise DG_EINVAL; Lobatto basis without
 * artificial diffusion, otherwise DG_EUNSUPPORTED.  All calls on one GPU
 * share the array: calls that overlap in time on one GPU race, so the caller
 * orders them (one stream, or events).  Arguments and results as dg_rhs. */
dg_status dg_rhs_noalloc(dg_handle* h, const void* U, void* dUdt, hipStream_t stream);

/* Implicit condensation split of Section 2.2 at every node of U (the
 * reconstruction of Section 3.4): T, rho_v = min(rho_vs(T), rho_m) and
 * rho_c = rho_m - rho_v with rho e = E - |m|^2 / (2 rho).  T, rho_v, rho_c
 * are caller-owned device double arrays of one value per node (elements x
 * nodes, node order of U).  T is in/out: if use_guess != 0 its contents seed
 * Newton (warm start; a guess outside (lower bound, 600 K) is ignored),
 * otherwise it is output only.  rho_v or rho_c may be NULL.  DG_EINVAL for a
 * null U or T; a solve that hits newton_maxit or a state with no valid
 * temperature is reported by dg_get_stats. */
dg_status dg_saturation_split(dg_handle* h, const void* U, double* T, int use_guess,
                              double* rho_v, double* rho_c, hipStream_t stream);

/* nsteps steps of the SSP Runge-Kutta scheme of Section 3.3 (SSPRK(4,3),
 * or SSPRK(3,3) by dg_params.rk) in place on U, each stage the right-hand
 * side of dg_rhs (split, volume, faces, sources, diagonal mass) followed by
 * the Shu-Osher update; with the sponge on, Section 3.6's relaxation closes
 * every step.  U: caller-owned device array in the state layout.  dt: HOST
 * array of 1 value (single mesh) or nmembers values (batch), each positive
 * and finite, otherwise DG_EINVAL.  Uses the handle's stage buffers. */
dg_status dg_rk_step(dg_handle* h, void* U, const double* dt, int nsteps, hipStream_t stream);

/* Vector-Jacobian product of dg_rhs: U_bar = (d rhs / d U)^T dUdt_bar, the
 * transpose of the linearised Section 3.2 operator, with the derivative of
 * the Section 2.2 split taken by the implicit-function theorem on its
 * active branch.  Arrays in the state layout and precision, device,
 * caller-owned; U_bar is overwritten and must not alias U or dUdt_bar
 * (DG_EINVAL).  Lobatto basis without diffusion only (DG_EUNSUPPORTED). */
dg_status dg_rhs_vjp(dg_handle* h, const void* U, const void* dUdt_bar, void* U_bar,
                     hipStream_t stream);

/* Vector-Jacobian product of the Section 2.2 split: U_bar =
 * (d(T, rho_v, rho_c)/dU)^T (T_bar, rho_v_bar, rho_c_bar), by the
 * implicit-function theorem.  The bar arrays are device doubles per node
 * (any may be NULL); U_bar is overwritten and must not alias U. */
dg_status dg_saturation_split_vjp(dg_handle* h, const void* U, const double* T_bar,
                                  const double* rho_v_bar, const double* rho_c_bar,
                                  void* U_bar, hipStream_t stream);

/* Vector-Jacobian product of one Section 3.3 RK step (with the sponge's
 * transpose when it is on): U_n_bar = (d U_{n+1}/d U_n)^T U_np1_bar.  The
 * stages are recomputed from U_n into the handle's buffers.  dt as in
 * dg_rk_step; arrays as in dg_rhs_vjp (U_n_bar must not alias the others).
 * Lobatto basis without diffusion only (DG_EUNSUPPORTED). */
dg_status dg_rk_step_vjp(dg_handle* h, const void* U_n, const void* U_np1_bar, void* U_n_bar,
                         const double* dt, hipStream_t stream);

/* Conservation diagnostics of the state U (all members), in FP64 with a
 * fixed-order reduction over the quadrature of the basis:
 *   out3[0] = sum w J rho_d'             (dry mass; conserved),
 *   out3[1] = sum w J (rho_m' + rho_r')   (total water; changes only by the
 *             rain that sediments through the slip walls, Section 2.1 rain
 *             flux with the wall treatment of Section 3.2),
 *   out3[2] = the instantaneous rain mass flux out through the slip walls,
 *             sum over wall face points of w_f J_f rho_r v_r (out at the floor,
 *             in at the lid); with the Gauss basis rho_r is the face trace.
 * U is a device array in the state layout; out3 is a HOST array of 3
 * doubles, written when the call returns (it synchronises the stream).
 * DG_EINVAL for null pointers or a handle without background. */
dg_status dg_reduce_mass(dg_handle* h, const void* U, double* out3, hipStream_t stream);

/* dg_reduce_mass restricted to ensemble member `member` (DG_EINVAL if it does
 * not exist). */
dg_status dg_reduce_mass_member(dg_handle* h, const void* U, double* out3, int member,
                                hipStream_t stream);

/* Read the device status words (synchronises the device).  Returns DG_OK,
 * DG_ENOCONV or DG_ENONFINITE. */
dg_status dg_get_stats(dg_handle* h, dg_stats* out);
dg_status dg_reset_stats(dg_handle* h);

dg_status dg_destroy(dg_handle* h);

/* Launch geometry: elements per block (1 .. 256 / (k+1)^dim) and persistent
 * blocks per compute unit (0: one block per work item; n > 0: a grid of
 * n x CUs blocks that walk the work items).  Persistence applies to the
 * Lobatto-basis stage kernel of dg_rk_step only; every other kernel takes
 * one block per work item.  Not a hot call: synchronises. */
dg_status dg_set_launch(dg_handle* h, int elems_per_block, int persist_per_cu);
dg_status dg_get_launch(const dg_handle* h, int* elems_per_block, int* persist_per_cu);

/* Order of the work items (3D handles; 2D items are always in element
 * order): 0 y-bands of rows with z inside a band, so the elements above and
 * below an item were visited shortly before it; 1 plain element order; 2
 * (default) and 3 y-bands twice and four times as wide.  Results do not depend
 * on it.  Not a hot call: synchronises.  DG_EINVAL for another value. */
dg_status dg_set_item_order(dg_handle* h, int order);
dg_status dg_get_item_order(const dg_handle* h, int* order);

/* Autotuner: times nsteps RK steps of a copy of U (device) for every
 * candidate geometry (elements per block {max, max/2, max/4} x persistent
 * blocks per CU {0, 1, 2, 4} x item order {0, 1, 2, 3} in 3D), keeps the
 * fastest and reports it (any output pointer may be NULL; best_ms is per
 * step; the order is read back with dg_get_item_order).  U is not modified. */
dg_status dg_autotune(dg_handle* h, const void* U, const double* dt, int nsteps, int* best_epb,
                      int* best_persist, double* best_ms);

/* dg_rk_step (Section 3.3) replayed from a captured hipGraph: the first call
 * for a given (U, nsteps, launch geometry) captures every kernel of the
 * nsteps steps, later calls replay it; dt is uploaded before each replay.
 * Arguments as dg_rk_step.  Kernel timing must be disabled (DG_EINVAL). */
dg_status dg_rk_step_graph(dg_handle* h, void* U, const double* dt, int nsteps, hipStream_t stream);

/* Kernel timing (instrumentation).  While enabled, every kernel the library
 * launches is bracketed by HIP events on its stream; dg_timing_read
 * synchronises and returns the accumulated device time and launch count of a
 * kernel class since it was enabled.  Classes: DG_K_SPLIT (the split),
 * DG_K_STAGE (right-hand side / fused stage), DG_K_ADJOINT (the *_vjp
 * kernels), DG_K_OTHER.  Enabling allocates events; not for captured graphs. */
enum { DG_K_SPLIT = 0, DG_K_STAGE = 1, DG_K_ADJOINT = 2, DG_K_OTHER = 3 };
dg_status dg_timing_enable(dg_handle* h, int enable);
dg_status dg_timing_read(dg_handle* h, int kclass, double* total_ms, long long* launches);

/* Message for the last non-OK status returned on this thread. */
const char* dg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DG_H */
