/*
 * lbmrv: lattice Boltzmann schemes with relative velocities on AMD MI355X (gfx950).
 *
 * C ABI of the HIP library liblbmrv.so.  Plain pointers and sizes only.
 *
 * The scheme (Dubois, Fevrier, Graille, "Lattice Boltzmann schemes with relative
 * velocities", section 1): at every node the populations f are mapped to the
 * moments of a polynomial basis P_k evaluated at v_j - u~ (eq. (MatMu)), relaxed
 * diagonally towards equilibrium in that moving frame (eq. (relaxationu)),
 * mapped back and transported along the lattice velocities (eq. (transport)).
 * u~ = 0 is the d'Humieres MRT scheme; u~ = u = q / rho with the Geier basis is
 * the cascaded scheme (Prop. th:cascd2q9).
 *
 * Conventions shared by every call
 * --------------------------------
 * Lattice units.  The node spacing is dx = 1 and the velocities are
 * v_j = lambda c_j with integer directions c_j (eq. (lambda): dt = dx / lambda).
 * Velocities passed in or returned (u, u~) are in the same units as v_j.
 *
 * Direction order (the index j of the population arrays):
 *   D2Q9  (section 1.3): (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1)
 *   D3Q19: (0,0,0); (1,0,0) (-1,0,0) (0,1,0) (0,-1,0) (0,0,1) (0,0,-1);
 *          (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1) (1,0,-1) (-1,0,1)
 *          (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
 *   D3Q27: the 19 above, then (1,1,1) (-1,-1,-1) (1,1,-1) (-1,-1,1) (1,-1,1)
 *          (-1,1,-1) (-1,1,1) (1,-1,-1)
 *
 * Moment bases (index k of the rates s_k):
 *   LBMRV_BASIS_DEFAULT, D2Q9: eq. (mom) of the paper, in its order
 *     1, X, Y, (3|X|^2-4l^2)/l^2, (X^2-Y^2)/l^2, XY/l^2, X(3|X|^2-5l^2)/l^3,
 *     Y(3|X|^2-5l^2)/l^3, (9/2|X|^4 - 21/2 l^2|X|^2 + 4 l^4)/l^4
 *   LBMRV_BASIS_GEIER, D2Q9: eq. (polgeier): 1, X, Y, X^2+Y^2, X^2-Y^2, XY, XY^2, X^2Y, X^2Y^2
 *   LBMRV_BASIS_DEFAULT, D3Q19: 1; X, Y, Z; |X|^2, 2X^2-Y^2-Z^2, Y^2-Z^2, XY, YZ, XZ;
 *     XY^2, XZ^2, X^2Y, YZ^2, X^2Z, Y^2Z; X^2Y^2, X^2Z^2, Y^2Z^2
 *   LBMRV_BASIS_DEFAULT, D3Q27: the D3Q19 list with XYZ inserted after Y^2Z, then
 *     X^2Y^2, X^2Z^2, Y^2Z^2, X^2YZ, XY^2Z, XYZ^2, X^2Y^2Z, X^2YZ^2, XY^2Z^2, X^2Y^2Z^2
 *   Equilibrium: f^eq_j = w_j rho (1 + v_j.u/cs2 + (v_j.u)^2/(2 cs2^2) - |u|^2/(2 cs2)),
 *   cs2 = lambda^2/3, standard weights; independent of u~ (section 1.2).
 *
 * Population arrays are structure-of-arrays: element (j, x, y, z) sits at
 *   f[j * N + (z * ny + y) * nx + x],   N = nx * ny * nz  (nz = 1 in 2-D),
 * with element type by storage:
 *   LBMRV_F64     double, f itself
 *   LBMRV_F32     float,  f itself
 *   LBMRV_F32DEV  float,  the deviation f_j - w_j rho0
 *   LBMRV_F16DEV  IEEE binary16, the deviation f_j - w_j rho0 (rounded to
 *                 nearest-even on store, subnormals kept); arithmetic in FP32
 * Arithmetic is FP64 for LBMRV_F64 and FP32 otherwise.  Every axis is periodic.
 *
 * Memory and streams.  All arrays passed to lbmrv_step / lbmrv_moments /
 * lbmrv_conservation are device pointers owned by the caller, aligned to their
 * element size, on the device that is current when the call is made (an
 * LBMRV_F16DEV D3Q19 state that is also 4-byte aligned, with an even nx, takes
 * a faster path in the in-place form; results are the same bits).  A
 * `hip_stream` argument is a hipStream_t (NULL = the null stream); work is
 * enqueued on it asynchronously unless stated otherwise.  The context owns only
 * its parameters, (after the first lbmrv_conservation call) a small device
 * buffer for partial sums and, for a run-time basis, a small device table.
 *
 * Concurrency.  A context is not thread-safe: calls on one context must not
 * run concurrently from several host threads.  lbmrv_conservation and
 * lbmrv_deviation_norm share the context's partial-sum buffer; they are
 * blocking, so successive calls never overlap on the device.  Different
 * contexts are independent.
 *
 * Errors.  Every int-returning call returns LBMRV_OK (0) or a negative code.
 * Arguments are validated on the host before any HIP call, so an invalid call
 * has no device-side effect.  lbmrv_strerror gives a message.
 */
#ifndef LBMRV_H
#define LBMRV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBMRV_OK 0
#define LBMRV_ERR_INVALID_ARG (-1)   /* a pointer, size, enum or rate is invalid    */
#define LBMRV_ERR_UNSUPPORTED (-2)   /* valid request the library does not serve    */
#define LBMRV_ERR_HIP (-4)           /* a HIP runtime call failed                   */
#define LBMRV_ERR_NONFINITE (-5)     /* lbmrv_conservation found a NaN or infinity  */
#define LBMRV_ERR_ALIGNMENT (-6)     /* a pointer is not aligned to its element     */

enum lbmrv_lattice { LBMRV_D2Q9 = 0, LBMRV_D3Q19 = 1, LBMRV_D3Q27 = 2 };
enum lbmrv_basis { LBMRV_BASIS_DEFAULT = 0, LBMRV_BASIS_GEIER = 1, LBMRV_BASIS_CUSTOM = 2 };
enum lbmrv_storage { LBMRV_F64 = 0, LBMRV_F32 = 1, LBMRV_F32DEV = 2, LBMRV_F16DEV = 3 };
enum lbmrv_utmode { LBMRV_UT_ZERO = 0, LBMRV_UT_FLUID = 1, LBMRV_UT_FIELD = 2 };
enum lbmrv_streaming { LBMRV_STREAM_PULL = 0, LBMRV_STREAM_PUSH = 1, LBMRV_STREAM_AA = 2 };
enum lbmrv_equilibrium { LBMRV_EQ_POLYNOMIAL = 0, LBMRV_EQ_MAXWELLIAN = 1 };
enum lbmrv_block_order { LBMRV_ORDER_AUTO = 0, LBMRV_ORDER_NATURAL = 1, LBMRV_ORDER_XCD = 2 };

typedef struct lbmrv_ctx lbmrv_ctx;

/*
 * Create a context for one lattice, basis, scale, rate vector, grid and storage.
 *   out      receives the context (set to NULL on error)
 *   lattice  enum lbmrv_lattice
 *   basis    enum lbmrv_basis (GEIER only with D2Q9)
 *   lambda   velocity scale of eq. (lambda), finite and > 0
 *   s        q relaxation rates, one per basis element in the order above;
 *            s_k for the conserved moments (k = 0..d) must be exactly 0
 *            (section 1.1), the others in [0, 2]
 *   dims     d extents (nx, ny[, nz]), each >= 1, nx <= 65535*4096,
 *            ny, nz <= 65535, and nx*ny*nz <= 2^32 - 256 nodes (node indices
 *            are 32-bit; element offsets j*N + n are 64-bit, so q*N may
 *            exceed 2^32)
 *   storage  enum lbmrv_storage
 *   rho0     reference density of the deviation storages (finite; ignored
 *            for LBMRV_F64 and LBMRV_F32)
 * Makes no HIP call.  Errors: INVALID_ARG.
 */
int lbmrv_create(lbmrv_ctx **out, int lattice, int basis, double lambda, const double *s,
                 const int64_t *dims, int storage, double rho0);

/*
 * A moment basis given at run time: q polynomials P_0 .. P_{q-1} in the
 * dimensionless variable xi = X / lambda (X = v_j - u~, section 1.2), each a
 * sum of terms coef * xi_x^ex * xi_y^ey * xi_z^ez.  Term t belongs to
 * polynomial poly_of_term[t] and has exponents exps[3t .. 3t+2] and
 * coefficient coef[t]; terms of one polynomial with the same exponents add up.
 */
typedef struct {
  int32_t nterms;               /* number of terms, 1 .. 4096            */
  const int32_t *poly_of_term;  /* [nterms], each in 0 .. q-1            */
  const int32_t *exps;          /* [nterms][3], each exponent in 0 .. 8  */
  const double *coef;           /* [nterms], finite                      */
} lbmrv_poly_basis;

/*
 * lbmrv_create with a run-time moment basis (section 1.2 allows any
 * polynomial basis; the rates s_k then act on its moments).  Requirements,
 * checked on the host:
 *   - P_0 = 1 and P_{1+a} = xi_a (a < d) exactly: the conserved moments come
 *     first, as rho and the momentum (s_k = 0 for them, section 1.1);
 *   - the span of P equals the span of one of the built-in bases of the
 *     lattice (D2Q9: the span of eq. (mom) or of eq. (polgeier); D3Q19/D3Q27:
 *     the span of the monomials listed for LBMRV_BASIS_DEFAULT), to 1e-12
 *     relative.  These spans are closed under differentiation, so the shift
 *     T(u~) is the exact product of Prop. th:csd2q9; in 2-D no term may
 *     carry xi_z;
 *   - P = R W with W that built-in basis and R well conditioned (condition
 *     number below 1e10).
 * The kernels shift in the built-in basis W and relax through the dense
 * matrix R^{-1} S R of the non-conserved block, computed in FP64 on the host.
 * The context owns a small device table (at most 19 KB) allocated on the
 * current device by this call, filled by a blocking copy, and refreshed the
 * same way by lbmrv_set_rates; the context must then be used on that device.
 * lbmrv_moments returns m0_k = sum_j P_k(c_j) f_j (in xi units).  The
 * in-place streaming form is not available (lbmrv_step returns UNSUPPORTED).
 * Errors: INVALID_ARG (arguments, or a basis that fails a requirement above),
 * HIP (the allocation or copy failed).
 */
int lbmrv_create_custom(lbmrv_ctx **out, int lattice, const lbmrv_poly_basis *basis, double lambda,
                        const double *s, const int64_t *dims, int storage, double rho0);

/* Replace the q relaxation rates (same rules as lbmrv_create).  No HIP call,
 * except for a context with a run-time basis (see lbmrv_create_custom). */
int lbmrv_set_rates(lbmrv_ctx *c, const double *s);

/*
 * Select the streaming form used by lbmrv_step.  All give the same f(t + n dt)
 * bit for bit:
 *   LBMRV_STREAM_PULL (default): each node gathers f*_j(x - c_j); two arrays,
 *     post-collision values kept between fused passes;
 *   LBMRV_STREAM_PUSH: each node scatters to x + c_j; two arrays;
 *   LBMRV_STREAM_AA: one array updated in place (half the memory): even steps
 *     store each post-collision population in its opposite slot at the node,
 *     odd steps gather from the opposite slots upstream and scatter downstream;
 *     an odd step count ends with one swap pass.  lbmrv_step then accepts
 *     f_in == f_out (otherwise f_in is first copied to f_out).
 * No HIP call.
 */
int lbmrv_set_streaming(lbmrv_ctx *c, int kind);

/*
 * Equilibrium moments the relaxation aims at:
 *   LBMRV_EQ_POLYNOMIAL (default): m^eq(u~) = M(u~) f^eq with the second-order
 *     polynomial f^eq documented above (section 1.2);
 *   LBMRV_EQ_MAXWELLIAN: m^eq(u~)_k = rho E[P_k(xi - u~)] for xi distributed as
 *     the continuous Maxwellian of density rho, velocity u and temperature cs2
 *     (the equilibria of Geier's cascaded scheme, mentioned in the paper's
 *     introduction).  Conserved moments are unchanged.
 * lbmrv_adjoint differentiates either form.  No HIP call.
 */
int lbmrv_set_equilibrium(lbmrv_ctx *c, int kind);

/*
 * Half-way bounce-back walls on domain faces (the paper's analysis is for the
 * whole space; walls are the usual closure).  Bit 2a + side of wall_mask makes
 * the low (side 0) or high (side 1) face of axis a (0 = x, 1 = y, 2 = z) a
 * wall placed half a node outside the last layer; other faces stay periodic.
 * A population that would come from beyond a wall is the node's own
 * post-collision opposite population plus 2 w_j rho_w (v_j . u_w) / cs2 for a
 * wall moving at u_w (wall_u [6][3], physical units, face index 2a + side,
 * NULL = all at rest); at an edge the first crossed wall face in axis order
 * gives u_w.  The pull form supports any wall_mask.  The in-place form
 * supports walls placed on both faces of an axis (with a wall on one face
 * only, lbmrv_step returns UNSUPPORTED): there a population bounced at step n
 * is kept in the node's own opposite slot; its results equal the pull form's
 * bit for bit in FP64 and FP32 storage (FP16: the moving-wall term is added
 * before instead of after one storage rounding).  The push form returns
 * UNSUPPORTED, and so does lbmrv_adjoint for any wall.  No HIP call.
 */
int lbmrv_set_walls(lbmrv_ctx *c, uint32_t wall_mask, const double *wall_u, double rho_w);

/*
 * Order in which the step kernels' workgroups take their tiles.  The GPU
 * deals workgroups to its eight XCDs (each with its own L2) round-robin:
 *   LBMRV_ORDER_NATURAL: tiles in grid order, so the eight XCDs work on
 *     neighbouring addresses at any moment;
 *   LBMRV_ORDER_XCD: each XCD takes one contiguous range of tiles, so tiles
 *     that are neighbours along x (sharing the cache lines at their common
 *     edge) meet in one L2;
 *   LBMRV_ORDER_AUTO (default): XCD while the population array (q N
 *     elements) fits in 256 MiB, NATURAL beyond (the faster choice measured
 *     on both sides of that size).
 * Results are identical bit for bit in every order.  No HIP call.
 */
int lbmrv_set_block_order(lbmrv_ctx *c, int order);

/* Query: q, d, N (nodes), bytes per stored population. */
int lbmrv_info(const lbmrv_ctx *c, int64_t *q, int64_t *d, int64_t *nodes, int64_t *bytes_per_pop);

/*
 * Advance nsteps full time steps (relaxation then transport, section 1.2):
 * f_out <- f(t + nsteps dt) given f_in = f(t), both pre-collision.
 *   f_in, f_out  device arrays of q*N elements of the storage type, distinct
 *                except in the in-place form (LBMRV_STREAM_AA).  f_in is the
 *                ping-pong partner and is overwritten (its contents are
 *                unspecified on return when nsteps >= 1).  nsteps = 0 copies
 *                f_in to f_out.
 *   ut_mode      LBMRV_UT_ZERO (u~ = 0), LBMRV_UT_FLUID (u~ = ut_alpha * u at
 *                every node and step; ut_alpha = 1 is the cascaded choice) or
 *                LBMRV_UT_FIELD (u~(x) read from ut_field, fixed over the call)
 *   ut_alpha     finite
 *   ut_field     FIELD mode: device float array [d][N] (SoA, same node order),
 *                otherwise ignored (may be NULL)
 *   nsteps       >= 0
 * Errors: INVALID_ARG, UNSUPPORTED (walls with the push form or one-sided
 * walls in place; the in-place form with a run-time basis), ALIGNMENT, HIP.
 */
int lbmrv_step(lbmrv_ctx *c, void *f_in, void *f_out, int ut_mode, double ut_alpha,
               const float *ut_field, int64_t nsteps, void *hip_stream);

/*
 * The two half-steps of section 1.2 on their own, for checks of non-conserved
 * moments and for external drivers:
 *   lbmrv_collide:  f_out(x) <- f*(x), the relaxation at every node (f_out may
 *                   equal f_in: the update is node-local)
 *   lbmrv_transport: f_out_j(x) <- f_in_j(x - c_j) (eq. (transport)); f_out != f_in
 */
int lbmrv_collide(lbmrv_ctx *c, const void *f_in, void *f_out, int ut_mode, double ut_alpha,
                  const float *ut_field, void *hip_stream);
int lbmrv_transport(lbmrv_ctx *c, const void *f_in, void *f_out, void *hip_stream);

/*
 * Per-node macroscopic fields of f (eq. (rhoq)):
 *   rho  [N], u [d][N] (u = q / rho, physical units), and, if m0 is not NULL,
 *   m0 [q][N] = M(0) f, the fixed-frame moments of the user basis.
 * Output element type: double for LBMRV_F64, float otherwise.  Errors: as step.
 */
int lbmrv_moments(lbmrv_ctx *c, const void *f, void *rho, void *u, void *m0, void *hip_stream);

/*
 * Global sums in FP64: out[0] = sum_x rho, out[1 .. d] = sum_x q^alpha
 * (physical units), out[d+1 .. 3] = 0.  Synchronises hip_stream.  Returns
 * LBMRV_ERR_NONFINITE (with out filled) if any population is NaN or infinite.
 */
int lbmrv_conservation(lbmrv_ctx *c, const void *f, double out[4], void *hip_stream);

/*
 * lbmrv_conservation for callers that cannot allocate device memory: code
 * being captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc.  It computes the same sums with the same kernels (results equal
 * lbmrv_conservation's bit for bit), but writes them to device memory and
 * returns without waiting:
 *   out_dev  device array of 5 doubles, caller-owned, 8-byte aligned:
 *            [0] sum_x rho, [1 .. d] sum_x q^alpha (physical units),
 *            [d+1 .. 3] = 0, [4] the number of NaN or infinite populations
 * The partial sums live in a library-owned device array of 1024 x 5 doubles
 * (40 KB, one per GPU, taken at the first call on that GPU and held until the
 * process ends); its size does not depend on the grid, so every grid that
 * lbmrv_create accepts is served.  The call makes no allocation (no hipMalloc,
 * no allocating library routine) and no synchronisation.  All calls on one
 * GPU share that array: calls that overlap on one GPU (different streams, or
 * host threads without ordering) race and must be serialised by the caller.
 * Each call overwrites every partial sum before reading it, so nothing is
 * cleared between calls.
 * Errors: INVALID_ARG, ALIGNMENT, UNSUPPORTED (device index >= 64), HIP.
 */
int lbmrv_conservation_noalloc(lbmrv_ctx *c, const void *f, double *out_dev, void *hip_stream);

/*
 * Distance of a state from a uniform reference state, for the growth rate of
 * small perturbations (linear stability of the scheme about a uniform flow;
 * the paper names stability as the question its schemes leave open).
 *   f_ref  host array of q doubles: the reference populations (f itself, not
 *          the stored deviations), e.g. one node of a uniform equilibrium
 * lbmrv_deviation_norm: out[0] = sum over nodes and j of (f_j - f_ref_j)^2,
 *   accumulated in FP64 in a fixed order (deterministic).  Blocking: returns
 *   after the work queued on hip_stream is done.  Returns NONFINITE (out[0]
 *   still written) when some population is NaN or infinite.
 * lbmrv_deviation_scale: f_j <- f_ref_j + factor (f_j - f_ref_j) at every
 *   node, in FP64 and then the storage's arithmetic type and rounding;
 *   asynchronous on hip_stream.
 * Errors: INVALID_ARG (null or misaligned f, null or non-finite f_ref,
 * non-finite factor), HIP.
 */
int lbmrv_deviation_norm(lbmrv_ctx *c, const void *f, const double *f_ref, double *out, void *hip_stream);
int lbmrv_deviation_scale(lbmrv_ctx *c, void *f, const double *f_ref, double factor, void *hip_stream);

/*
 * Initial state (K5): f_out <- f^eq(rho, u) + noise_amp * noise, computed in
 * FP64 and stored in the context's storage type (minus w_j rho0 for the
 * deviation storages, rounded to nearest-even).
 *   rho [N], u [d][N] (physical units), noise [q][N] or NULL: device doubles.
 */
int lbmrv_init_equilibrium(lbmrv_ctx *c, const double *rho, const double *u, const double *noise,
                           double noise_amp, void *f_out, void *hip_stream);

/*
 * Storage conversion.  lbmrv_import: out <- rn(f - w_j rho0) in the storage
 * type from FP64 populations f [q][N]; lbmrv_export: f <- in + w_j rho0 in FP64.
 * Device arrays.  For LBMRV_F64 both are copies.
 */
int lbmrv_import(lbmrv_ctx *c, const double *f, void *out, void *hip_stream);
int lbmrv_export(lbmrv_ctx *c, const void *in, double *f, void *hip_stream);

/*
 * Host tables of a lattice: cdirs [q][3] integer directions in the order
 * documented above, w [q] equilibrium weights.  No HIP call.
 */
int lbmrv_lattice_tables(int lattice, int32_t *cdirs, double *w);

/*
 * Discrete adjoint of nsteps time steps (the transpose of the linearised
 * relaxation of eq. (relaxationu) and of the transport of eq. (transport)),
 * for u~ = 0, u~ = ut_alpha * u(f) (differentiated through u = q / rho), or a
 * given field u~(x) held fixed over the steps.  Given the
 * cotangent cot_fN = dJ/df_N of an objective J(f_N), with f_N the state after
 * nsteps steps from f0, it returns
 *   grad_f0 [q][N] = dJ/df0 (derivative with respect to the populations; for a
 *                    deviation storage this is also dJ/d(stored value)),
 *   grad_s  [q]    = dJ/ds_k, accumulated in FP64 (0 for k <= d),
 *   grad_ut [d][N] = dJ/du~(x), accumulated in FP64 (FIELD mode only),
 *   f_N            = the forward state (optional, may be NULL).
 * The forward states are recomputed from snapshots taken every K steps.
 *   ut_mode     LBMRV_UT_ZERO, LBMRV_UT_FLUID or LBMRV_UT_FIELD; ut_alpha as in
 *               lbmrv_step (finite)
 *   f0, f_N     storage type [q][N]; cot_fN, grad_f0: double for LBMRV_F64,
 *               float otherwise; grad_s, grad_ut: double; all device arrays
 *   workspace   device memory of at least lbmrv_adjoint_workspace_bytes(c,
 *               nsteps, K) bytes, 256-byte aligned, owned by the caller
 * Either equilibrium (lbmrv_set_equilibrium) and a run-time basis are
 * differentiated; walls are not (UNSUPPORTED).
 * Asynchronous on hip_stream.  With more than one segment of K steps, the
 * segments are recomputed on a second stream that the context creates at its
 * first such call (default priority, on the device current then; a later
 * call on another device returns INVALID_ARG) and orders against hip_stream
 * with events: all of that work is complete before anything enqueued on
 * hip_stream after the call runs.  Errors: INVALID_ARG, UNSUPPORTED,
 * ALIGNMENT, HIP.
 */
size_t lbmrv_adjoint_workspace_bytes(const lbmrv_ctx *c, int64_t nsteps, int64_t K);
int lbmrv_adjoint(lbmrv_ctx *c, const void *f0, int ut_mode, double ut_alpha, const float *ut_field,
                  int64_t nsteps, int64_t K, const void *cot_fN, void *workspace, size_t workspace_bytes,
                  void *f_N, void *grad_f0, double *grad_s, double *grad_ut, void *hip_stream);

void lbmrv_destroy(lbmrv_ctx *c);
const char *lbmrv_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* LBMRV_H */
