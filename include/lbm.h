/*
 * lbm.h -- C ABI of the MI355X KBC lattice Boltzmann library.
 *
 * The library advances the entropic multi-relaxation-time (KBC) lattice
 * Boltzmann equation of Dorschner, Chikatamarla & Karlin, "Fluid-structure
 * interaction with the entropic lattice Boltzmann method" (Sec. II.A), with
 * Grad's-approximation reconstruction of missing populations at moving walls
 * (Sec. II.C.1) and the stress-based wall force on a body (Sec. II.C.2), on one
 * AMD Instinct MI355X (gfx950).  The call order of one fluid-structure
 * coupling step (Sec. II.C, conventional serial staggered scheme) is
 *     lbm_step -> lbm_wall_force -> (structure solve on the host) -> lbm_set_geometry.
 *
 * Conventions (all functions):
 *   - Return an lbm_status: LBM_OK (0) on success, a negative code on error.
 *     lbm_last_error() gives a human-readable message for the last failure.
 *   - Lattice units throughout.  Lattices: D2Q9 and D3Q27, the tensor products
 *     of D1Q3 (weights 2/3, 1/6, 1/6 per axis; speed of sound 1/sqrt(3)).
 *     Velocity index i = (cx+1) + 3(cy+1) + 9(cz+1); opposite index Q-1-i.
 *   - Host arrays are owned by the caller; the library copies in before
 *     returning and copies out before returning from synchronous calls.
 *   - Node order is x-fastest: node = x + nx*(y + ny*z).  Vector fields are
 *     planar: u[a*N + node].  Population arrays are population-major:
 *     f[i*N + node], full (unshifted) f_i in double precision.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Device memory is owned by the context unless allocation callbacks are
 *     given (then the callback owner must outlive the context).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int lbm_status;
#define LBM_OK 0
#define LBM_ERR_INVALID (-1)     /* bad argument or description */
#define LBM_ERR_OOM (-2)         /* device allocation failed */
#define LBM_ERR_DEVICE (-3)      /* a HIP runtime call failed */
#define LBM_ERR_NONFINITE (-4)   /* a node reached a non-finite or invalid state */
#define LBM_ERR_GEOMETRY (-5)    /* body does not fit the domain */
#define LBM_ERR_UNSUPPORTED (-6) /* valid request this build does not provide */

/* Lattice (value = number of velocities Q). */
#define LBM_D2Q9 9
#define LBM_D3Q27 27

/* Population storage.  All forms store the deviation f_i - W_i from the rest
 * state; F16/BF16 store it in 16 bits and compute in FP32, F32 stores and
 * computes in FP32, F64 stores and computes in FP64. */
#define LBM_F64 0
#define LBM_F32 1
#define LBM_F16_SHIFTED 2
#define LBM_BF16_SHIFTED 3

/* Collision: entropic KBC (stabiliser gamma per node, Sec. II.A Eq. 6) or
 * LBGK (gamma fixed to 2, relaxation rate 2 beta). */
#define LBM_KBC 0
#define LBM_LBGK 1

/* Face conditions, faces ordered -x, +x, -y, +y, -z, +z.  PERIODIC must be
 * paired; INLET is allowed on -x only, OUTLET on +x only, and either needs
 * nx >= 2.
 *   INLET : equilibrium at the inflow velocity and the lagged density of the
 *           interior neighbour (parabolic profile option, smooth ramp).
 *   OUTLET: equilibrium at density 1 and the lagged velocity of the upstream
 *           neighbour.
 *   WALL  : resting no-slip wall half a spacing outside the face, filled by
 *           Grad's approximation like any cut link (q = 1/2). */
#define LBM_FACE_PERIODIC 0
#define LBM_FACE_INLET 1
#define LBM_FACE_OUTLET 2
#define LBM_FACE_WALL 3

/* Bodies.  The structure solver is host-side; the library takes either a
 * prescribed motion law that the device evaluates every step, or the
 * structure's surface mesh (Sec. II.C.1: the FEM surface quadrilaterals split
 * into triangles, vertices moved by the computed displacements, vertex
 * velocities interpolated at the link intersections).
 *   SPHERE (circle in 2D): params X0[3], R, A[3], omega, phase;
 *           centre X0 + A sin(omega t + phase), rigid translation.
 *   FLAP (2D): params x_f, length l, thickness h, amplitude d0, omega, phase,
 *           y_base; solid where 0 <= s <= l and |x - x_c(s,t)| <= h/2, with
 *           s = y - y_base and x_c = x_f + d0 sin(omega t + phase) (s/l)^2.
 *   MESH:   closed surface given by nverts vertices (verts, 3 doubles each),
 *           their velocities (vert_vel, 3 doubles each) and ntris faces (tris,
 *           3 vertex indices each).  D3Q27: triangles; D2Q9: each face is the
 *           segment of its first two vertices (the third index is ignored,
 *           z components are ignored).  A node is solid when it lies inside
 *           the closed surface or on it.  Along a cut link the wall fraction
 *           is the first intersection with a face, and the wall velocity the
 *           vertex velocities interpolated linearly (barycentric) there.  The
 *           mesh describes the surface at the time of the next step's new
 *           state and stays in place until the next lbm_set_geometry call; the
 *           first call also sets the current geometry.  params are unused.
 *   PLATES: params y_lo, y_hi, u_lo[3], u_hi[3]; solid where y < y_lo or
 *           y > y_hi; each plate slides tangentially with its velocity.
 * Points on the surface count as solid.  Time t is the step count. */
#define LBM_BODY_NONE 0
#define LBM_BODY_SPHERE 1
#define LBM_BODY_FLAP 2
#define LBM_BODY_MESH 3
#define LBM_BODY_PLATES 4

typedef struct lbm_ctx lbm_ctx;

typedef struct {
  int lattice;        /* LBM_D2Q9 or LBM_D3Q27 */
  int nx, ny, nz;     /* >= 1 each; nz == 1 for D2Q9 */
  double nu;          /* kinematic viscosity > 0; beta = 1/(6 nu + 1) (Sec. II.A, Eq. 7) */
  int storage;        /* LBM_F64 .. LBM_BF16_SHIFTED; same for every instance */
  int collision;      /* LBM_KBC or LBM_LBGK */
  int kbc_trace_in_s; /* 0: trace of the second moments relaxes with gamma (part of h);
                         1: it relaxes with the shear part s */
  int face[6];        /* LBM_FACE_* for -x,+x,-y,+y,-z,+z */
  double u_in[3];     /* inflow velocity (mean velocity for the parabolic profile) */
  int inlet_profile;  /* 0 uniform, 1 parabolic 1.5 U y(H-y)/(H/2)^2 (Sec. III.A.1) */
  int ramp_steps;     /* inflow ramp 0.5 (1 - cos(pi min(t,T)/T)); 0 = none */
} lbm_instance_desc;

typedef struct {
  int device;                              /* HIP device ordinal */
  void* hip_stream;                        /* hipStream_t to launch on; NULL = own stream */
  void* (*alloc)(size_t bytes, void* ctx); /* optional device allocator (e.g. PyTorch) */
  void (*free)(void* ptr, void* ctx);      /* matching release; both or neither */
  void* alloc_ctx;                         /* passed back to alloc/free */
  int use_graph;                           /* 1: replay lbm_step through a captured hipGraph */
} lbm_device_opts;

typedef struct {
  int kind;               /* LBM_BODY_* */
  double params[16];      /* analytic bodies: layout per kind, see above */
  int nverts, ntris;      /* MESH: vertex and face counts (else ignored) */
  const double* verts;    /* MESH: nverts * 3 positions, host memory */
  const double* vert_vel; /* MESH: nverts * 3 velocities, host memory */
  const int* tris;        /* MESH: ntris * 3 vertex indices, host memory */
} lbm_body;

typedef struct {
  double mass;        /* sum of rho over fluid nodes (FP64) */
  double momentum[3]; /* sum of rho u over fluid nodes (FP64) */
  double gamma_min, gamma_mean, gamma_max; /* over fluid nodes of the last stats step */
  double fp64_gamma_fraction; /* share of nodes whose gamma used the FP64 path */
  int64_t step;       /* steps taken */
} lbm_totals;

/* Creates a context holding n_instances lattices that are stepped together
 * (one batched launch per kernel).  All instances must share lattice and
 * storage.  Populations start at the rest state f_i = W_i.  opts may be NULL
 * (device 0, own stream, internal allocation, graphs on).
 * Errors: LBM_ERR_INVALID (bad description), LBM_ERR_OOM, LBM_ERR_DEVICE. */
lbm_status lbm_create(const lbm_instance_desc* desc, int n_instances,
                      const lbm_device_opts* opts, lbm_ctx** out);

/* Releases every device resource of the context.  NULL is accepted. */
lbm_status lbm_destroy(lbm_ctx* ctx);

/* Sets instance inst to the entropic equilibrium f^eq(rho, u) at every node
 * (Sec. II.A, Eqs. 4-5).  rho: N doubles; u: D*N doubles, planar.
 * Requires rho > 0 and |u_a| < 1 (else LBM_ERR_INVALID).  Synchronous. */
lbm_status lbm_init_fields(lbm_ctx* ctx, int inst, const double* rho, const double* u);

/* Replaces the body of instance inst (Sec. II.C.1: the geometry and wall
 * velocity the fluid boundary condition needs).  An analytic body's geometry
 * at the current time is built on the device and thereafter follows its
 * motion law on the device, so lbm_step needs no host update; a mesh is
 * copied to the device before the call returns (the caller keeps ownership of
 * its arrays) and used from the next step on.  body == NULL or kind NONE
 * removes the body.
 * Errors: LBM_ERR_INVALID (unknown kind, flap in 3D, a mesh with no faces, a
 * vertex index out of range or non-finite coordinates), LBM_ERR_GEOMETRY (the
 * body's swept region does not fit inside the domain with a 2-node margin
 * along periodic axes). */
lbm_status lbm_set_geometry(lbm_ctx* ctx, int inst, const lbm_body* body);

/* Advances every instance by n_steps >= 0 steps (Sec. II.A, Eq. 1, pull form:
 * geometry update, fresh-node refill, streaming, Grad fill, face conditions,
 * KBC collision).  Asynchronous on the context stream: with boundary nodes
 * the boundary kernels of a step run on a private side stream of the
 * context that forks from the context stream after the geometry update and
 * joins it again before the step ends, so work enqueued on the context
 * stream afterwards sees the whole step.  Each call that
 * enqueues steps also enqueues a copy of the device error word to the host
 * and records an event after it; the next lbm_step call checks that copy if
 * the event has completed (without waiting for it) and returns
 * LBM_ERR_NONFINITE if the word was set.  Synchronous calls check the word
 * itself. */
lbm_status lbm_step(lbm_ctx* ctx, int n_steps);

/* Density and velocity of the stored (post-collision) state of instance inst:
 * rho = sum_i f_i and rho u = sum_i f_i c_i (Sec. II.A, Eq. 5, the moments
 * the collision conserves), so they equal the moments the last collision
 * used.  tot holds their FP64 sums over fluid nodes (mass and momentum
 * drift) and, with statistics on, the gamma statistics of the last step.
 * Solid nodes report rho = 0, u = 0.  rho: N doubles, u: D*N doubles, tot:
 * totals; any output may be NULL.  Synchronous.  Returns LBM_ERR_NONFINITE if
 * the device error word is set (outputs are still written). */
lbm_status lbm_moments(lbm_ctx* ctx, int inst, double* rho, double* u, lbm_totals* tot);

/* Force of the fluid on the body of instance inst (Sec. II.C.2): for each
 * quadrature point (xq, nq outward unit body normal, wq weight) the
 * pre-collision stress sigma = -p I - (1-beta) Pi^(1) of the last step is
 * sampled at xq + nq and xq + 2 nq (linear over fluid nodes), extrapolated
 * to the surface as 2 sigma(p1) - sigma(p2), and t_q = sigma_q nq.
 * force = sum_q wq t_q (FP64, deterministic order).  Arrays are point-major
 * with D components (xq[q*D + a]).  traction (n_q*D doubles) may be NULL.
 * Requires at least one step since the last geometry or population change
 * (else LBM_ERR_INVALID).  Synchronous. */
lbm_status lbm_wall_force(lbm_ctx* ctx, int inst, const double* xq, const double* nq,
                          const double* wq, int n_q, double* traction, double force[3]);

/* lbm_wall_force for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving or coupling loops, harnesses that forbid
 * allocation): same arguments, kernels and results, but its workspace is a
 * static device array of the library (5.8 MB per GPU, kept until the process
 * ends) instead of memory the context allocates, and the call makes no
 * device allocation or release.  n_q is limited to 65536 points (larger
 * requests return LBM_ERR_INVALID).  Every call on one GPU shares that
 * workspace: calls that overlap on one GPU (several contexts on different
 * streams or threads) race and must be serialised by the caller.
 * Synchronous. */
lbm_status lbm_wall_force_noalloc(lbm_ctx* ctx, int inst, const double* xq, const double* nq,
                                  const double* wq, int n_q, double* traction, double force[3]);

/* Multiphase KBC (Sec. III.B) on instance inst (enable != 0) or off.  Each
 * step then adds the body force
 *   F = 2 phi grad(phi) + kappa rho grad(lap rho) + kappa_w rho sum_i W_i s(x + c_i) c_i,
 *   phi = sqrt(rho/3 - p(rho)),  p(rho) the sixth-degree polynomial of Eq. eos,
 * from the densities of the state after streaming and the boundary fill
 * (Eqs. Force, force1, Korteweg, force2; the kappa term with the sign that the
 * divergence of the Korteweg tensor gives).  Derivatives use the
 * lattice-weight stencils grad_a X = 3 sum_i W_i c_ia X(x + c_i) and
 * lap X = 6 sum_i W_i (X(x + c_i) - X(x)); a neighbour that is solid or
 * beyond a wall face gives the node's own value and counts s = 1 in the
 * wetting sum.  The force enters by the exact difference method (Eq.
 * force_mp): the post-collision state gains f^eq(rho, u + F/rho) -
 * f^eq(rho, u); gamma uses the scalar product weighted by
 * 1 / f^eq(rho, u + F/rho).  The collision runs in FP64.  kappa sets the
 * surface tension, kappa_w the wetting (negative: non-wetting); this
 * discretisation is stable for kappa rho_liquid below about 0.3.
 * While any instance of the context has it on, every instance steps through
 * the multiphase kernels (those with it off at zero force) and stores
 * moments that include the force (lbm_moments reports j = rho u + F).
 * Needs FP64 or FP32 storage and periodic or wall faces
 * (LBM_ERR_UNSUPPORTED otherwise); lbm_wall_force returns
 * LBM_ERR_UNSUPPORTED for a multiphase instance.  The first call that
 * enables it allocates 3 fields of N values (FP64 for FP64 storage, else
 * FP32) for all instances.  Synchronous. */
lbm_status lbm_set_multiphase(lbm_ctx* ctx, int inst, int enable, double kappa, double kappa_w);

/* ---- Structure solver and two-way coupling (Sec. II.B, II.C) ------------
 * A rectangular beam [x0, x0 + length] x [y0, y0 + height] in plane strain:
 * total-Lagrangian Saint Venant-Kirchhoff material (Sec. II.B: P = F S,
 * S = lambda tr(E) I + 2 mu E, E = (F^T F - I)/2), nex x ney 9-node
 * biquadratic elements with 3 x 3 Gauss points, consistent mass, the
 * two-field (u, v) formulation with the one-step-theta scheme (theta = 1/2:
 * Crank-Nicolson) solved by Newton's method.  The edge x = x0 is clamped.
 * Node (i, j), 0 <= i <= 2 nex, 0 <= j <= 2 ney, has index j + (2 ney + 1) i
 * and DOFs 2 k (x), 2 k + 1 (y).  Units are the caller's (lattice units when
 * coupled).  Host code; the beam has ~10^2-10^3 unknowns. */
typedef struct lbm_fem lbm_fem;
typedef struct {
  double x0, y0, length, height;
  int nex, ney;
  double rho, lambda, mu;   /* density, Lame coefficients */
  double dt, theta;
} lbm_fem_desc;
/* Errors: LBM_ERR_INVALID for a bad description. */
lbm_status lbm_fem_create(const lbm_fem_desc* desc, lbm_fem** out);
lbm_status lbm_fem_destroy(lbm_fem* fem);
/* Node count, and (if coords is not NULL) the 2 * nodes reference
 * coordinates. */
lbm_status lbm_fem_info(const lbm_fem* fem, int* nodes, double* coords);
/* Consistent nodal loads (2 * nodes doubles into f) of a uniform body force
 * b per unit mass. */
lbm_status lbm_fem_body_force(const lbm_fem* fem, const double b[2], double* f);
/* One theta step with the external nodal loads fext (2 * nodes doubles) at
 * the new time (the previous step's loads are kept as the old time level's).
 * iterations (may be NULL) receives the Newton count.  Returns
 * LBM_ERR_NONFINITE if Newton does not converge in 30 iterations. */
lbm_status lbm_fem_step(lbm_fem* fem, const double* fext, int* iterations);
/* Displacements u and velocities v (2 * nodes doubles each; either may be
 * NULL). */
lbm_status lbm_fem_get_state(const lbm_fem* fem, double* u, double* v);
lbm_status lbm_fem_set_state(lbm_fem* fem, const double* u, const double* v);

/* Two-way coupling of instance inst (2D) with a beam, by the conventional
 * serial staggered scheme of Sec. II.C.  The body of the instance becomes a
 * closed polygon (LBM_BODY_MESH): the beam's wet boundary (bottom edge from
 * the clamped end to the tip, the tip, the top edge back), in its current
 * position and velocity, then the static chain arc (n_arc points, 2 doubles
 * each, from the clamped top corner round to the clamped bottom corner,
 * both excluded; n_arc = 0 closes the beam along its clamped edge).  Each
 * coupled step: lbm_step; the traction of the fluid on the beam at the three
 * Gauss points of every quadratic wet edge in its current position
 * (lbm_wall_force_noalloc, Sec. II.C.2), less the reference pressure
 * rho_0 c_s^2 = 1/3 (the beam is only partly wet, so a uniform pressure does
 * not cancel on it); lbm_fem_step with the consistent
 * nodal loads sum_q N_a t_q w_q; the polygon set from the new state for the
 * next step.  fem must outlive the coupling; the context and instance must
 * be 2D.  Errors: those of lbm_set_geometry at creation. */
typedef struct lbm_fsi lbm_fsi;
lbm_status lbm_fsi_create(lbm_ctx* ctx, int inst, lbm_fem* fem, const double* arc, int n_arc,
                          lbm_fsi** out);
lbm_status lbm_fsi_destroy(lbm_fsi* fsi);
/* n_steps coupled steps.  beam_force (3 doubles per step, may be NULL): the
 * force of the fluid on the beam's wet edges (gauge pressure); tip (2 per step, may be NULL):
 * the displacement of the node at mid-height of the free end.  Stops at the
 * first error (LBM_ERR_NONFINITE from the fluid or the structure). */
lbm_status lbm_fsi_step(lbm_fsi* fsi, int n_steps, double* beam_force, double* tip);

/* Checkpoint: copies the populations of instance inst to / from the host
 * (Q*N doubles, population-major, full f_i).  A set is rounded to the
 * storage format.  Resuming from get -> set is bitwise exact. */
lbm_status lbm_get_populations(lbm_ctx* ctx, int inst, double* f);
lbm_status lbm_set_populations(lbm_ctx* ctx, int inst, const double* f);
/* Copies the populations of the box [lo, hi) of instance inst to the host
 * ((hi-lo) product * Q doubles, population-major over the box's own
 * x-fastest node order, full f_i), e.g. a crop with its halo for checking one
 * step elsewhere.  Along a periodic axis the box may wrap once (lo >= -n,
 * hi <= 2n, at most n wide); along other axes 0 <= lo < hi <= n, else
 * LBM_ERR_INVALID.  Synchronous. */
lbm_status lbm_get_populations_box(lbm_ctx* ctx, int inst, const int lo[3], const int hi[3],
                                   double* f);

/* Switches per-step statistics (gamma min/mean/max, FP64-path share) on or
 * off; off by default because it adds a reduction to every step.  Nodes with
 * missing populations are collided in FP64 and count as FP64-path nodes;
 * inflow / outflow face nodes hold an exact equilibrium, whose collision is
 * the identity, and count with gamma = 2; in contexts with several
 * instances, the statistics of an instance cover its bulk nodes only. */
lbm_status lbm_set_stats(lbm_ctx* ctx, int enabled);

/* Launch mode: 0 = one batched launch per kernel for all instances (default),
 * 1 = one launch per instance (reference for the batched form). */
lbm_status lbm_set_launch_mode(lbm_ctx* ctx, int mode);

/* Times the candidate tile shapes of the bulk kernel on this context's
 * instances (18 steps each from the same saved state) and keeps the fastest.
 * Both population buffers, the flags and the clock are restored afterwards,
 * so the following steps are bitwise those of an untuned context; the call
 * needs device memory for two more population buffers while it runs.
 * cache_path (nullable) names a JSON file of earlier results keyed by
 * lattice, storage, sizes and device; it is read first and updated.
 * chosen (nullable) receives the index of the chosen variant. */
lbm_status lbm_autotune(lbm_ctx* ctx, const char* cache_path, int* chosen);

/* Selects a bulk-kernel variant by index (0 .. lbm_variant_count()-1). */
lbm_status lbm_set_variant(lbm_ctx* ctx, int variant);
int lbm_variant_count(void);
const char* lbm_variant_name(int variant);

/* Information: nodes of instance inst (N), total nodes, algorithmic bytes per
 * lattice update (2 Q sizeof(storage)), steps taken. */
lbm_status lbm_info(const lbm_ctx* ctx, int inst, int64_t* nodes, int64_t* total_nodes,
                    int* bytes_per_update, int64_t* step);

/* Waits for all work on the context stream.  Returns LBM_ERR_NONFINITE if the
 * device error word is set. */
lbm_status lbm_synchronize(lbm_ctx* ctx);

const char* lbm_status_string(lbm_status s);
const char* lbm_last_error(const lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
