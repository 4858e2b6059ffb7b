/*
 * lbm.h - C ABI of the MI355X (gfx950) two-component Shan-Chen D3Q19 lattice
 * Boltzmann step coupled to triangulated Skalak capsules through an
 * immersed boundary.
 *
 * The problem follows Wouters, Aouane, Krueger, Harting, "Mesoscale
 * simulation of soft particles with tunable contact angle in multi-component
 * fluids" (arXiv:1904.11386):
 *   - fluid: D3Q19 BGK (Sec. II.A, eqs. method:boltzmann, lbm:equilibrium,
 *     lbm:weights), force as an equilibrium-velocity shift (Sec. II.A), two
 *     components with the Shan-Chen interaction (Sec. II.D,
 *     eq. method:shanchen), pseudo-potential psi = rho or 1 - exp(-rho);
 *   - capsules: Skalak membrane energy (Sec. II.B, eq. method:strain) and
 *     volume penalty (Sec. II.B, eq. method:volume), node forces by virtual
 *     work, forward-Euler node motion (Sec. II.B);
 *   - wettability: a virtual density offset on the preferred component
 *     (Sec. II.D) with particle colour Delta rho = cos(theta)
 *     (Sec. III.D, eq. results:anglescaling), spread over the membrane with
 *     the same delta and scaled by wet_scale;
 *   - planar half-way bounce-back walls that may move (Sec. II.C,
 *     eq. method:SBB), or on-site velocity boundaries (Zou and He, in the
 *     D3Q19 form of Hecht and Harting), the boundaries of the paper's
 *     shear-flow case (Sec. III.A), forward runs only;
 *   - optionally, Helfrich bending of the membranes (Sec. II.B) and the
 *     short-range particle-particle repulsion between boundary nodes of
 *     different capsules (Sec. III.E);
 *   - observables: component masses, capsule centre of mass and height
 *     above the interface (Sec. III.D, eq. interface:contactangle), Taylor
 *     deformation (Sec. III.A, eq. results:taylorparameter).
 * The fluid-structure coupling is an immersed boundary with Peskin's
 * 4-point delta (the method the paper cites as prior art in Sec. I) instead
 * of the paper's bounce-back coupling.
 *
 * Conventions for every call
 *   - Returns 0 (LBM_OK) or one of the LBM_E* codes below; no exception
 *     crosses the ABI.  The message of the last error of a context is
 *     returned by lbm_last_error(ctx); lbm_last_error(NULL) gives the last
 *     error of a failed lbm_init / lbm_workspace_bytes on this thread.
 *   - Ownership: the caller owns all device memory (one workspace block,
 *     which must outlive the context) and all host arrays; host inputs are
 *     copied, never retained.  The library owns only the host context,
 *     freed by lbm_destroy.
 *   - Streams: all device work is enqueued on the HIP stream given to
 *     lbm_init (NULL = the null stream).  lbm_observables, lbm_get_*,
 *     lbm_debug_*, lbm_step_timed and the adjoint calls marked so
 *     synchronise that stream.
 *   - Lattice arrays are [z][y][x] with x fastest; nodes are (x, y, z)
 *     triples in lattice units; angles are degrees.
 *   - D3Q19 direction order: 0 rest; 1..6 = +x -x +y -y +z -z; 7..18 =
 *     (+-1,+-1,0), (+-1,0,+-1), (0,+-1,+-1) with opposites adjacent.
 *   - Calls on one context are not thread-safe; different contexts are
 *     independent.
 */
#ifndef LBM_CAPSULES_LBM_H
#define LBM_CAPSULES_LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBM_OK = 0,
    LBM_EINVAL = 1,     /* bad argument; nothing was enqueued            */
    LBM_ENOMEM = 2,     /* workspace smaller than lbm_workspace_bytes     */
    LBM_EHIP = 3,       /* a HIP runtime call failed                      */
    LBM_ESTATE = 4,     /* call out of order (e.g. capsules after a step) */
    LBM_EUNSTABLE = 5   /* FP64 mass check found non-finite or drifting mass */
};

enum { LBM_FP32 = 0, LBM_FP16 = 1 };

enum { LBM_OBJ_COM_Z = 0, LBM_OBJ_TAYLOR_D = 1 };

typedef struct lbm_params {
    int32_t nx, ny, nz;     /* lattice size, each >= 4, nx*ny*nz <= 2^30        */
    int32_t precision;      /* LBM_FP32, or LBM_FP16 population storage         */
    int32_t walls;          /* 0 periodic; 1 solid rows y = 0 and y = ny - 1
                               (half-way bounce-back, ny >= 5); 2 on-site
                               velocity boundaries on the fluid rows y = 0
                               and y = ny - 1 (ring_len 0).  Both move
                               at wall_u_lo / wall_u_hi; capsules keep their
                               stencils off the boundary rows.  On-site
                               boundaries exchange mass with the outside:
                               the FP16 form then runs without mass
                               compensation and the mass check tests
                               finiteness only                              */
    int32_t n_slots;        /* checkpoint slots carved from the workspace       */
    int32_t check_every;    /* FP64 mass check period in steps, 0 = never       */
    int32_t use_graphs;     /* 1: lbm_step replays captured two-step HIP graphs
                               when the stream is not the null stream          */
    double tau[2];          /* BGK relaxation times of A and B, each > 0.5      */
    double G;               /* Shan-Chen coupling G^{AB} = G^{BA} >= 0          */
    double rho_maj, rho_min;/* densities that scale the colour (Sec. II.D)      */
    double wall_u_lo[3];    /* velocity of the wall row y = 0                   */
    double wall_u_hi[3];    /* velocity of the wall row y = ny - 1              */
    double z_interface;     /* plane from which capsule heights are measured    */
    double mass_tol;        /* relative mass drift rejected by the check        */
    double wet_scale;       /* >= 0; virtual density rho_v = 2 cos(theta)
                               (rho_maj - rho_min) wet_scale; 1 = the colour law
                               of Sec. II.D as written                           */
    int32_t ring_len;       /* > 0: room for the adjoint (FP32 only), with a
                               recompute ring of ring_len states                 */
    int32_t stream_policy;  /* cache policy of the population streams:
                               0 chosen by size (1 up to 512 MiB of populations,
                               else 2); 1 non-temporal loads, cached stores;
                               2 cached loads, non-temporal stores. Results do
                               not depend on it.                                 */
    int32_t zchunk;         /* z planes marched per lattice block: 0 chosen by
                               storage form and grid size, else a multiple of 8
                               up to 64. Results do not depend on it.            */
    int32_t psi_kind;       /* Shan-Chen pseudo-potential: 0 psi = rho; 1 psi =
                               1 - exp(-rho) (Sec. II.D, rho0 = 1). The virtual
                               density of the wettability term is added to psi
                               either way.                                       */
    double rep_eps;         /* particle-particle repulsion (Sec. III.E): node
                               pairs of different capsules at separation
                               d < rep_d0 repel along their separation with
                               rep_eps (rep_d0 - d)^{3/2}; 0 = off (the paper
                               uses 0.5). Finite, >= 0; the adjoint
                               differentiates it.                                */
    double rep_d0;          /* its cut-off, in (0, 2] when rep_eps > 0 (the
                               paper uses 1.25)                                  */
    int32_t coupling;       /* fluid-structure coupling: 0 the immersed boundary
                               (Peskin 4-point delta, massless nodes); 1 the
                               paper's own: half-way bounce-back of the
                               populations that cross a membrane, with the
                               moving-element term and the momentum exchange
                               (Sec. II.C, eqs. method:SBB and
                               method:momentumtransfer), the Shan-Chen sum
                               across it from densities interpolated on the
                               viewer's side plus the colour offset (Sec. II.D,
                               eq. method:interpolateshanchen), fresh nodes
                               with the adaptive mass correction (Sec. II.E,
                               eqs. method:freshnodes, method:masscorrection)
                               and inertial nodes.  1 needs FP32 storage,
                               walls 0, n_slots 0, ring_len 0 and rep_eps 0   */
    double node_mass;       /* coupling 1: mass of a boundary node (> 0; the
                               paper uses 5, Sec. III)                          */
    double mass_c0;         /* coupling 1: strength C0 of the adaptive mass
                               correction (>= 0; the paper uses 2500)           */
    int32_t deterministic;  /* 0 or 1, coupling 0 only.  1: the immersed
                               boundary's sums run in a fixed order (capsule
                               volumes per capsule, each bin's nodes by id, the
                               lattice force and virtual-density fields
                               gathered per cell instead of added with
                               atomics), so a step is the same bit for bit
                               from run to run and across a state save and
                               load; 0 differs from it by rounding order only.
                               A debugging mode: its gather costs more than
                               the atomic spreading.  The adjoint's own sums
                               keep their atomics.                            */
    int32_t mass_fix;       /* 0 or 1, FP32 storage with check_every > 0 and
                               walls 0 or 1.  1: at each mass check every
                               population of a component is scaled so that the
                               component's FP64 mass is the intended one: the
                               initial mass (the FP64 sum of the densities
                               given to lbm_init) plus, with coupling 1, the
                               coupling's own change (lbm_obs.mass_ledger).
                               FP32 rounding otherwise drifts the masses by a
                               few 1e-9 per step in flows with interfaces; the
                               FP16 form compensates every step by itself. The
                               check then tests the drift from the intended
                               mass.                                          */
    int32_t lattice_passes; /* passes over the lattice per step, results equal
                               bit for bit either way: 2 a density pass and the
                               collide (Sec. II.A then Sec. II.D); 1 the collide
                               forms the densities of its block and halo from
                               the pulled populations itself, with the
                               immersed boundary's tiles given a density pass
                               of their own for the wettability reaction
                               (needs FP32 storage, walls 0, coupling 0 and
                               ring_len 0, else LBM_EINVAL); 0 chosen by the
                               library: 1 where allowed and the populations
                               exceed 512 MiB, else 2.                        */
} lbm_params;

typedef struct lbm_obs {
    double mass[2];         /* sum over fluid nodes of the post-collision populations */
    double momentum[3];     /* sum over fluid nodes and components of f* c           */
    int64_t step;           /* completed time steps                                   */
    double particle_momentum[3]; /* coupling 1: sum over boundary nodes of m V (else 0) */
    double pending_momentum[3];  /* coupling 1: half of the last step's exchanged
                                    momentum, which the nodes receive with the next
                                    step (Sec. II.C); fluid + particle + pending
                                    momentum is conserved (else 0)              */
    double mass_ledger[2];  /* coupling 1: the mass per component that the
                               moving-element bounce-back terms and the
                               fresh-node refills changed since init, summed in
                               FP64 as stored: the Delta rho^c the adaptive
                               correction reads (eq. method:masscorrection);
                               mass - initial mass - this is the FP32
                               storage's rounding (else 0)                     */
} lbm_obs;

typedef struct lbm_capsule_obs {
    double com[3];          /* mean node position (equal node masses)                */
    double volume, area;    /* enclosed volume and surface area                      */
    double axes[3];         /* ellipsoid half-axes, ascending, same volume moments   */
    double taylor_D;        /* (a_max - a_min) / (a_max + a_min)                     */
    double height;          /* com[2] - z_interface                                  */
} lbm_capsule_obs;

typedef struct lbm_ctx lbm_ctx;

/* Size query (no passage of the paper: the library's own memory contract,
 * one caller-owned device block holding the whole state).  *bytes receives
 * the device workspace size for a lattice p with room for max_nodes
 * membrane nodes and max_faces triangles in total (each in [0, 2^29]: node
 * and face ids are 32-bit).  Host-only, no device work.  LBM_EINVAL on a bad
 * p or sizes out of range. */
int lbm_workspace_bytes(const lbm_params* p, int64_t max_nodes, int64_t max_faces,
                        int64_t* bytes);

/* Create a context: the two-component fluid of Sec. II.A (D3Q19 BGK,
 * eqs. method:boltzmann, lbm:equilibrium, lbm:weights, relaxation times
 * tau[2]) and Sec. II.D (Shan-Chen coupling G, eq. method:shanchen, and
 * the pseudo-potential psi_kind), in a periodic box or between the walls of
 * Sec. II.C (eq. method:SBB) / Sec. III.A.  rhoA, rhoB: host float arrays of
 * nx*ny*nz initial densities (> 0 on fluid nodes).  The populations start as
 * the rest equilibrium w_i rho (u = 0) and are streamed by the first step.
 * workspace: device pointer of at least ws_bytes bytes, 256-byte aligned,
 * ws_bytes >= lbm_workspace_bytes(p, max_nodes, max_faces).
 * hip_stream: a hipStream_t or NULL.  max_nodes, max_faces in [0, 2^29].
 * Validates p (tau > 0.5, sizes >= 4, G >= 0, finite wall velocities,
 * precision in {FP32, FP16}) and the sizes before any device work; *out is
 * NULL after any failure; errors: LBM_EINVAL, LBM_ENOMEM, LBM_EHIP. */
int lbm_init(const lbm_params* p, const float* rhoA, const float* rhoB,
             void* workspace, int64_t ws_bytes, int64_t max_nodes, int64_t max_faces,
             void* hip_stream, lbm_ctx** out);

/* Append n_caps capsules: triangulated membranes with the Skalak energy
 * (Sec. II.B, eq. method:strain; kS, C) and the volume penalty (Sec. II.B,
 * eq. method:volume; kV), wetting the fluid with the particle colour
 * Delta rho = cos(theta) (Sec. II.D; Sec. III.D, eq. results:anglescaling).
 * Host arrays: nodes_per_cap[n_caps],
 * faces_per_cap[n_caps]; xyz_rest[sum nodes][3] absolute rest positions,
 * which are also the initial positions; tri[sum faces][3] capsule-local node
 * indices, counter-clockwise seen from outside; kS (> 0), C (> -1/2),
 * kV (>= 0) and theta_deg (in [0, 180]) per capsule.  Each capsule is stored
 * as an integer anchor (its rest centroid rounded) plus FP32 offsets; the
 * reference metric, rest areas and rest volume are computed in FP64.  Only
 * before any step has been enqueued (else LBM_ESTATE, also after a state is
 * loaded back to step 0: the captured graphs and tile lists were built for
 * the capsules present then); LBM_ENOMEM beyond the sizes
 * given to lbm_init.  Under the bounce-back coupling (coupling 1) a capsule
 * must fit the box in which its labels are found (1.5 times its extent plus
 * 9 lattice units, within the smallest lattice edge), and no more than 32
 * capsules may lie within one such box of each other (they are told apart by
 * one parity bit each); else LBM_EINVAL.  *first_id (may be NULL) receives
 * the index of the first new capsule. */
int lbm_capsules_add(lbm_ctx* ctx, int32_t n_caps, const int32_t* nodes_per_cap,
                     const int32_t* faces_per_cap, const double* xyz_rest,
                     const int32_t* tri, const double* kS, const double* C,
                     const double* kV, const double* theta_deg, int32_t* first_id);

/* Boundary-node velocities of the capsules first_id .. first_id + n_caps - 1
 * under the bounce-back coupling (coupling 1; Sec. II.B, forward Euler of
 * inertial nodes): every node of capsule k takes the velocity v[k][3]
 * (finite, |v_k| < 0.5; 0 at the start); with prescribed != 0 the nodes keep
 * it, whatever the forces (the rigid translation of Sec. II.E's
 * mass-conservation test, Fig. mass-conservation), with prescribed = 0 they
 * move under the forces from there.  Before the first step or between steps
 * (it takes effect from the next step, e.g. to hold capsules still while the
 * fluid relaxes and then release them); synchronises.  LBM_EINVAL under the
 * immersed boundary (coupling 0, whose nodes are massless) or for a range
 * outside the capsules added. */
int lbm_capsules_velocity(lbm_ctx* ctx, int32_t first_id, int32_t n_caps, const double* v, int32_t prescribed);

/* Helfrich bending (Sec. II.B, eqs. method:curvature and surf_dens, zero
 * spontaneous curvature): bending moduli kB[n_caps] (finite, >= 0; 0 = none,
 * the default) of the capsules first_id .. first_id + n_caps - 1.  Each node
 * of a capsule with kB > 0 gets F = 2 kB [2 H (H^2 - K) + Lap_s H] n A, with
 * the mean curvature H, Gaussian curvature K, Laplace-Beltrami operator,
 * outward normal n and mixed area A of the discrete operators of Meyer et
 * al. (2003) on the current mesh.  Only before the first lbm_step (else
 * LBM_ESTATE); LBM_EINVAL for a range outside the capsules added, a bad kB,
 * or kB > 0 on a context with the adjoint (ring_len > 0), which does not
 * differentiate it.  Like lbm_capsules_add, refused (LBM_ESTATE) once any
 * step has been enqueued, also after a state is loaded back to step 0. */
int lbm_capsules_bending(lbm_ctx* ctx, int32_t first_id, int32_t n_caps, const double* kB);

/* The LBM-free reference model (Sec. III.B, eq. emulatetension): nsteps of
 * membrane-only relaxation of every capsule, without the fluid.  Each node
 * moves by mobility * F (the nodes are massless, so the relaxation is
 * overdamped), with F its Skalak, volume and bending forces plus the
 * emulated surface tension: every element gets gamma A / w, A the part of
 * its area between the planes z_interface -+ w/2, directed horizontally and
 * radially away from the vertical axis through its capsule's centre of mass
 * at the start of the call, shared evenly by its three nodes.  The lattice
 * state is not touched, nor are the wettability and repulsion terms used.
 * Asynchronous on the stream.  LBM_EINVAL for nsteps < 0, gamma < 0, w <= 0,
 * mobility <= 0 or non-finite values.  (Stability of the explicit update
 * needs mobility below about 2 / the stiffest elastic mode; 0.05 is stable
 * for kV = 20 at R = 5.) */
int lbm_reference_relax(lbm_ctx* ctx, int32_t nsteps, double gamma, double w, double z_interface,
                        double mobility);

/* Advance nsteps >= 0 time steps (Sec. II.A eq. method:boltzmann: pull
 * streaming and BGK collision with the force as an equilibrium-velocity
 * shift; Sec. II.D eq. method:shanchen: the inter-component force with the
 * wettability offset; Sec. II.B: membrane forces by virtual work and the
 * forward-Euler node update), asynchronously on the stream.  With
 * use_graphs, pairs of steps are replayed from HIP graphs captured on the
 * first call (kernels only, no memory-set nodes).  With
 * check_every > 0 the FP64 mass check runs every check_every steps and
 * synchronises; it returns LBM_EUNSTABLE when a component mass is not
 * finite or (except with walls = 2) has drifted by more than mass_tol
 * relative to its start.  Under the bounce-back coupling (coupling 1) the
 * call also reads the coupling's list flags at its end (and at each check),
 * synchronising, and returns LBM_EUNSTABLE when a list overflowed, a capsule
 * outgrew its label box, a membrane is not closed, or the label boxes of two
 * capsules of one parity colour met; its steps after the first are replayed
 * in pairs from graphs as well. */
int lbm_step(lbm_ctx* ctx, int32_t nsteps);

/* Kernel groups of one step, in launch order (for lbm_step_timed).  Under
 * the bounce-back coupling (coupling 1) LBM_K_CLEAR holds the step's head
 * (labels, link list, fresh nodes, the bounce-back of the crossing
 * populations and the tile flags), LBM_K_SPREAD the Shan-Chen sum across
 * the membranes and LBM_K_INTERP the node update; the bin and spreading
 * groups are empty.  In one lattice pass (lattice_passes) LBM_K_DENSITY
 * launches nothing (the collide forms the densities) and LBM_K_SPREAD
 * begins with the densities of the immersed boundary's tiles. */
enum {
    LBM_K_CLEAR = 0,    /* zero last step's immersed-boundary tiles        */
    LBM_K_DENSITY = 1,  /* density pass over the lattice                   */
    LBM_K_VOLUME = 2,   /* FP64 capsule volumes                            */
    LBM_K_FACES = 3,    /* Skalak + volume forces per triangle             */
    LBM_K_NODES = 4,    /* node force gather and home-bin counts           */
    LBM_K_SCAN = 5,     /* scan of the tile bins                           */
    LBM_K_SCATTER = 6,  /* counting-sort scatter                           */
    LBM_K_REPULSE = 7,  /* particle-particle repulsion (rep_eps > 0)       */
    LBM_K_BEND = 8,     /* Helfrich bending forces (some kB > 0)           */
    LBM_K_SPREAD = 9,   /* wettability reaction and LDS-binned spreading   */
    LBM_K_COLLIDE = 10, /* fused pull + force + collide over the lattice,
                           and the on-site boundary closure (walls = 2)    */
    LBM_K_INTERP = 11,  /* interpolation and node advection                */
    LBM_NK = 12
};

/* Measurement (no passage of the paper, which reports no timings).
 * As lbm_step (without the mass check), and synchronises: HIP events are
 * recorded on the stream before each kernel group, and kernel_ms[LBM_NK]
 * receives the summed elapsed milliseconds of each group over the nsteps
 * (>= 1) steps.  A group that launches nothing in these steps reads 0; every
 * other group's time includes the cost of its pair of events (about 5 us
 * per step, what an empty group measures), which dominates the membrane
 * groups of a few us. */
int lbm_step_timed(lbm_ctx* ctx, int32_t nsteps, double* kernel_ms);

/* FP64 observables of the current state: the component masses whose drift
 * Sec. II.E measures (Fig. mass-conservation), the total momentum, and per
 * capsule the centre of mass and its height above the interface (Sec. III.D,
 * eq. interface:contactangle), volume, area and the Taylor deformation from
 * the volume's second moments (Sec. III.A, eq. results:taylorparameter).
 * Synchronises.  caps may be NULL, else it must hold one entry per capsule. */
int lbm_observables(lbm_ctx* ctx, lbm_obs* out, lbm_capsule_obs* caps);

/* lbm_observables for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid it):
 * the same results, bit for bit, with the FP64 reduction partials and the
 * per-capsule moments kept in a fixed device array of the library (about
 * 576 KiB per device, resolved at lbm_init and held until the process ends)
 * instead of the context's workspace.  It calls no hipMalloc, hipFree or
 * allocating routine; host-side partial sums go through fixed stack
 * buffers.  At most 4096 capsules when caps is not NULL (else LBM_EINVAL).
 * Every context on one device shares the array: calls that overlap on one
 * device (other threads, or streams not ordered with each other) race.
 * Synchronises. */
int lbm_observables_noalloc(lbm_ctx* ctx, lbm_obs* out, lbm_capsule_obs* caps);

/* The moments of Sec. II.A (rho = sum f, rho u = sum f c + F / 2) of the
 * most recent collision (time level step - 1):
 * rhoA, rhoB [N] and u [3][N] (x, y, z planes of the physical velocity with
 * the half-force term).  Host buffers, any may be NULL.  LBM_ESTATE before
 * the first step.  Synchronises. */
int lbm_get_fields(lbm_ctx* ctx, float* rhoA, float* rhoB, float* u);

/* Current absolute boundary-node positions (Sec. II.B), anchor + offset,
 * [nodes][3].  Synchronises. */
int lbm_get_nodes(lbm_ctx* ctx, double* xyz);

/* Node forces F_b = -dE/dx_b (Sec. II.B, virtual work) [nodes][3] used by the
 * most recent step: elastic, volume, the wettability reaction (the momentum
 * balance of Sec. II.D) and the optional bending and repulsion.
 * Synchronises; LBM_ESTATE before the first step. */
int lbm_get_node_forces(lbm_ctx* ctx, float* F);

/* Spread fields of the most recent step (the immersed-boundary coupling,
 * which the paper names as prior art in Sec. I and does not define):
 * F_ib [3][N] and the virtual densities phi [2][N] (A, B) of the colour of
 * Sec. II.D.  Synchronises; LBM_ESTATE before a step. */
int lbm_get_spread(lbm_ctx* ctx, float* Fib, float* phi);

/* Labels of the bounce-back coupling (coupling 1; the inside and outside of
 * each membrane that Sec. II.C and II.D separate): labels[N] receives, per
 * lattice node ([z][y][x], x fastest), the index of the capsule whose closed
 * surface holds it, or -1, for the membranes at the current node positions
 * (those the next step streams across).  Recomputed on the device from the
 * positions.  LBM_EINVAL under coupling 0.  Synchronises. */
int lbm_debug_labels(lbm_ctx* ctx, int32_t* labels);

/* Boundary-node velocities V [nodes][3] (coupling 1; Sec. II.B), zero under
 * the immersed boundary's massless nodes.  Synchronises. */
int lbm_get_node_velocities(lbm_ctx* ctx, float* V);

/* Debugging (no passage of the paper: the spreading's own bookkeeping).
 * Binning of the current node positions: tile_of_node[nodes] is the index
 * of the 4x4x4 spreading bin holding the node floor(X) (bins numbered x
 * fastest),
 * base_idx[nodes][3] the unwrapped stencil base floor(X) - 1.  Recomputed
 * from the positions on the device.  Synchronises. */
int lbm_debug_bins(lbm_ctx* ctx, int32_t* tile_of_node, int32_t* base_idx);

/* Checkpoint and resume (no passage of the paper: the adjoint's
 * checkpoints).  Copy the full state (populations, density buffers, node
 * positions, step counter) to / from slot 0 <= slot < n_slots inside the
 * workspace.  Asynchronous on the stream. */
int lbm_state_save(lbm_ctx* ctx, int32_t slot);
int lbm_state_load(lbm_ctx* ctx, int32_t slot);

/* Discrete adjoint of the coupled step (no passage of the paper, which
 * computes no gradients; the objectives are its observables, below) (FP32
 * storage, ring_len > 0, at least
 * one capsule).  J is a capsule objective at the end of a run: LBM_OBJ_COM_Z
 * the node-mean height above z_interface (Sec. III.D, eq.
 * interface:contactangle) or LBM_OBJ_TAYLOR_D (Sec. III.A, eq.
 * results:taylorparameter), of capsule `capsule`.
 *
 * lbm_adjoint_forward advances nsteps from the current state, keeping a
 * checkpoint in slot s at every multiple s * every of the run (needs
 * every <= ring_len and n_slots >= ceil(nsteps / every)), and returns J in
 * *J (FP64, synchronises).
 *
 * lbm_adjoint_backward then seeds lambda_X = dJ/dX at the final positions
 * and sweeps the segments in reverse: each segment is recomputed from its
 * checkpoint into the ring, and each step's adjoint is applied in reverse
 * order.  grads[3] receives dJ/dtheta (per radian, every capsule's angle
 * shifted together), dJ/dkS (every capsule's shear modulus shifted
 * together) and dJ/dG.  At theta = 90 degrees the one-sided derivative of
 * the preferred-component choice made at set-up is returned.  Immersed-
 * boundary stencils must stay two nodes away from solid rows.  The state
 * afterwards is the one at the start of the run.  Synchronises. */
int lbm_adjoint_forward(lbm_ctx* ctx, int32_t nsteps, int32_t every, int32_t objective, int32_t capsule,
                        double* J);
int lbm_adjoint_backward(lbm_ctx* ctx, double* grads);

/* The same reverse sweep, one call per stage, for a caller that drives it
 * (lbm_adjoint_backward is seed, then per segment in reverse lbm_state_load,
 * lbm_adjoint_record and lbm_adjoint_step for the recorded steps, last
 * first, then lbm_adjoint_grads).  Same preconditions as above (FP32 storage,
 * ring_len > 0, capsules); no passage of the paper.
 *
 * lbm_adjoint_seed: lambda_X = dJ/dX at the current node positions for
 * objective (LBM_OBJ_COM_Z, Sec. III.D eq. interface:contactangle, or
 * LBM_OBJ_TAYLOR_D, Sec. III.A eq. results:taylorparameter) of capsule
 * `capsule`; every other adjoint field and the parameter gradients are
 * zeroed.  Synchronises.  LBM_EINVAL for an unknown objective or capsule.
 *
 * lbm_adjoint_record: ring entry 0 = the current state, entries 1 ..
 * nsteps - 1 the states after each of the next nsteps - 1 recomputed steps
 * (1 <= nsteps <= ring_len, else LBM_EINVAL).  The step counter and the
 * population and density buffers are left as they were; the node positions
 * are those after the recomputed steps.  Asynchronous.
 *
 * lbm_adjoint_step: applies the adjoint of recorded step ring_index to the
 * adjoint state and adds its parameter derivatives.  The indices of one
 * recording must come in reverse order, nsteps - 1 first (else
 * LBM_ESTATE); LBM_ESTATE before lbm_adjoint_seed or lbm_adjoint_record.
 * Leaves the node positions at those of entry ring_index.  Asynchronous.
 *
 * lbm_adjoint_grads: grads[3] = dJ/dtheta (per radian), dJ/dkS, dJ/dG
 * accumulated since the seed, as for lbm_adjoint_backward.  Synchronises. */
int lbm_adjoint_seed(lbm_ctx* ctx, int32_t objective, int32_t capsule);
int lbm_adjoint_record(lbm_ctx* ctx, int32_t nsteps);
int lbm_adjoint_step(lbm_ctx* ctx, int32_t ring_index);
int lbm_adjoint_grads(lbm_ctx* ctx, double* grads);

/* Teardown (no passage of the paper).  Free the host context (not the
 * workspace).  NULL is ignored. */
void lbm_destroy(lbm_ctx* ctx);

/* Error reporting (no passage of the paper).  Last error message of ctx,
 * or of this thread's failed init when NULL. */
const char* lbm_last_error(const lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_CAPSULES_LBM_H */
