/*
 * dg_tri.h -- C interface of libdgmoist on triangulations: the moist DG
 * right-hand side, split and SSP Runge-Kutta step of dg.h on a conforming
 * triangulation of the vertical (x, z) plane, with the space P^k of the
 * paper's Section 3.1 (simplicial meshes).
 *
 * The discretisation (arXiv 2305.13847):
 *   - U_h in [P^k(T_h)]^{4+d}, d = 2, held by its coefficients in the
 *     orthonormal Dubiner basis of the unit triangle {r, s >= 0, r + s <= 1}:
 *       psi_pq(r, s) = N_pq t^p P_p((2r - t)/t) P_q^{(2p+1,0)}(2s - 1),
 *       t = 1 - s, N_pq^2 = 2 (2p+1) (p+q+1),
 *     so the element mass matrix is (det A) I (Section 3.1; diagonal mass).
 *     Mode m runs over p = 0..k and, for each p, q = 0..k-p.  Element e is
 *     the affine image x = V0 + A (r, s) of the unit triangle, A = [V1 - V0,
 *     V2 - V0], with counter-clockwise vertices (det A > 0).
 *   - Volume integrals use the product of Gauss-Legendre rules of the
 *     footnote in Section 3.4, carried onto the triangle by the Duffy map:
 *     k+1 points a_i across, k+2 points b_j up, s = (1 + b_j)/2,
 *     r = (1 + a_i)(1 - s)/2, weight w_i w_j (1 - s)/4, point q = j (k+1) + i
 *     (exact for total degree 2k+1).  Faces use the (k+1)-point
 *     Gauss-Legendre rule; face f joins V_f and V_{f+1 mod 3}.
 *   - The split of Section 2.2 runs at the volume points; T and rho_v are
 *     L2-projected onto P^k (Section 3.4), and fluxes and sources are
 *     assembled from the projections at every quadrature point.
 *   - Lax-Friedrichs flux along the outward unit normal with
 *     Lambda = max over both sides of |u.n| + |v_r n_z| + c_m; slip walls
 *     take m+ = m- - 2 (m-.n) n (Section 3.2).  A face's neighbour is the
 *     element the mesh names; the two elements run along their shared edge in
 *     opposite directions, so face point i meets the neighbour's point k - i.
 *   - SSPRK(4,3) or SSPRK(3,3) (Section 3.3).
 *   - The background depends on height only: n_z layers of height dz from
 *     z0, its fields given at the k+1 Gauss heights of every layer.  An
 *     element takes the degree-k interpolant of the layer holding its
 *     centroid, at all of its points; the background pressure is the
 *     equation of state of the split background.
 *
 * Memory and ownership
 *   Coefficient arrays passed to the hot calls are DEVICE pointers owned by
 *   the caller, layout C[v][e][m] (variable, element, mode), in double
 *   (DG_FP64) or float (DG_FP32_BULK).  The handle owns tables, mesh tables,
 *   background and stage buffers (allocated in dg_tri_create, released in
 *   dg_tri_destroy).  Hot calls (dg_tri_rhs, dg_tri_split, dg_tri_rk_step)
 *   allocate nothing; calls on one handle must not overlap in time.
 *
 * Errors
 *   As in dg.h: every call returns a dg_status, dg_last_error() describes the
 *   last failure on the calling thread, and device-side problems (a Newton
 *   solve at the iteration cap, a state with no valid temperature) set status
 *   words read by dg_tri_get_stats.
 */
#ifndef DG_TRI_H
#define DG_TRI_H

#include "dg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_tri dg_tri;

/* A conforming triangulation (Section 3.1).  All arrays are HOST arrays,
 * copied by dg_tri_create. */
typedef struct {
  int ne;             /* triangles, 1 <= ne < 2^29                              */
  const double* xy;   /* ne x 3 x 2: counter-clockwise vertices (x, z)          */
  const int* nb;      /* ne x 3: element across face f (V_f to V_f+1); -1: slip
                         wall.  Periodic pairs are listed like interior faces  */
  const int* nbf;     /* ne x 3: the neighbour's face index (0..2)             */
  double z0, dz;      /* background layers: n_z layers of height dz from z0     */
  int nz;
} dg_tri_mesh;

/* Create a handle.  order k in 1..4; nvars = 5 (rain = 0) or 6 (rain = 1);
 * p as in dg.h (precision, rain closure, rk scheme, Newton settings); the
 * sponge and the artificial diffusion are not available on triangles
 * (DG_EUNSUPPORTED), p->basis is ignored.  DG_EINVAL for a bad order, a
 * triangle with det A <= 0, or neighbour tables that are not symmetric
 * (nb[nb[e][f]][nbf[e][f]] must be e).  DG_ENOMEM if device allocation fails. */
dg_status dg_tri_create(const dg_tri_mesh* mesh, int order, int nvars, const dg_params* p,
                        dg_tri** out);

/* Background (Section 2.3 perturbation form): HOST arrays of n_z (k+1)
 * doubles at the Gauss heights of the layers (lowest layer first), copied;
 * rho_r may be NULL (0).  The background pressure is computed on the device
 * from the split background.  Must be called before the first hot call;
 * synchronises.  DG_EINVAL for null or non-finite values or a state with no
 * valid temperature. */
dg_status dg_tri_set_background(dg_tri* h, const double* rho_d, const double* rho_m,
                                const double* rho_r, const double* E);

/* Physical coordinates of the volume quadrature points: HOST array xz of
 * ne x (k+1)(k+2) x 2 doubles, point order as above. */
dg_status dg_tri_points(const dg_tri* h, double* xz);

/* Number of values of one coefficient array (nvars x ne x (k+1)(k+2)/2) and
 * of the volume points (ne x (k+1)(k+2)). */
long long dg_tri_state_size(const dg_tri* h);
long long dg_tri_npoints(const dg_tri* h);

/* L2 projection onto P^k (Section 3.4) of nfields fields given at the volume
 * points: vals is a DEVICE double array [f][e][q], C a DEVICE array [f][e][m]
 * in the handle's precision.  c_m = sum_q w_q psi_m(x_q) vals_q (the basis is
 * orthonormal, det A cancels). */
dg_status dg_tri_project(dg_tri* h, const double* vals, int nfields, void* C, hipStream_t stream);

/* Reconstruction of Section 3.4: the split of Section 2.2 at every volume
 * point of C and the L2 projections of T and rho_v, written as coefficient
 * arrays Tc and Rvc (DEVICE doubles, [e][m]). */
dg_status dg_tri_split(dg_tri* h, const void* C, double* Tc, double* Rvc, hipStream_t stream);

/* dC/dt of the Section 3.2 weak form with the diagonal mass of Section 3.3,
 * after the reconstruction of Section 3.4.  C and dCdt: caller-owned device
 * arrays in the coefficient layout; they must not alias (DG_EINVAL). */
dg_status dg_tri_rhs(dg_tri* h, const void* C, void* dCdt, hipStream_t stream);

/* nsteps steps of the SSP Runge-Kutta scheme of Section 3.3 in place on C;
 * each stage is one fused kernel (right-hand side, update, and the split of
 * the updated state for the next stage).  dt > 0 and finite. */
dg_status dg_tri_rk_step(dg_tri* h, void* C, double dt, int nsteps, hipStream_t stream);

/* Status words (synchronises): DG_OK, DG_ENOCONV or DG_ENONFINITE. */
dg_status dg_tri_get_stats(dg_tri* h, dg_stats* out);
dg_status dg_tri_reset_stats(dg_tri* h);

/* Kernel timing: as dg_timing_enable / dg_timing_read of dg.h, classes
 * DG_K_SPLIT (split kernels), DG_K_STAGE (right-hand side / fused stage),
 * DG_K_OTHER (projection). */
dg_status dg_tri_timing_enable(dg_tri* h, int enable);
dg_status dg_tri_timing_read(dg_tri* h, int kclass, double* total_ms, long long* launches);

dg_status dg_tri_destroy(dg_tri* h);

#ifdef __cplusplus
}
#endif
#endif /* DG_TRI_H */
