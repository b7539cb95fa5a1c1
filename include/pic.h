/* pic.h -- C-ABI of the particle-mesh hot path of an electrostatic IFE-PIC
 * step on one AMD Instinct MI355X (gfx950).
 *
 * The library performs, for every macro-particle, the particle half of the PIC
 * loop (§2.1): trilinear gather of the node electric field ("gather"),
 * leapfrog push ("particle-push"), removal at the outer boundary (§3.1.3: the
 * particle is absorbed and removed) or at the object / terrain (§5.2.2: the
 * particle is collected and its charge accumulated for surface charging), and
 * trilinear weighting of the charge back to the mesh nodes ("scatter"), whose
 * result is the source term rho of eq. (2.1). The field solve of the loop (the
 * IFE discretisation, PCG and domain decomposition of §2.3) is not part of the
 * library: the node field is an input (pic_set_node_E).
 *
 * Units and mesh. The PIC mesh is globally uniform (§2.2) with nx*ny*nz cubic
 * cells of edge h starting at `origin`; nodes are numbered
 * node(i,j,k) = i + (nx+1)*(j + (ny+1)*k), x fastest. The domain is the
 * half-open box [0, n*h) per axis. Normalised units as in §3.1.1 / §5.2.1.
 *
 * Step definition (one call of pic_step advances every particle by dt):
 *   1. gather   E_p = sum_n W_n E[node_n], trilinear weights of the cell
 *   2. kick     v  += (q/m) dt E_p          (v stored at half steps)
 *   3. drift    x  += v dt
 *   4. box      a particle outside the box is removed, counted per face
 *               (faces 0..5 = x-, x+, y-, y+, z-, z+; first axis in x, y, z
 *               order, lower face first). With the crater terrain, z < 0 is a
 *               collection, not an escape.
 *   5. object   sphere: |x - c| <= R; crater: z < 0, or z <= z_flat and the
 *               point lies outside the bowl sphere of radius
 *               Rc = (a^2 + d^2) / (2d) centred at height z_flat - d + Rc on the
 *               crater axis (a flat plane at z_flat with a spherical bowl of
 *               radius a and depth d, a height function z = z(x, y) as in
 *               §5.2.1). A collected particle is removed and counted in its bin
 *               (sphere: one bin; crater: the surface column
 *               (clamp(floor x), clamp(floor y)), bin = ix + nx*iy).
 *   6. deposit  rho is zeroed, then every remaining particle adds q*w*W_n to
 *               its 8 cell nodes at its new position; rho = sum / h^3.
 * Fixed-point deposit: each contribution is rounded half-to-even to an int64 at
 * scale 2^32, corner 7 receiving llrint(q*w*2^32) minus the other seven, so the
 * total is conserved exactly and the result is independent of summation order.
 *
 * Conventions.
 *   - Every call validates its arguments before changing any state; on error the
 *     state is unchanged and pic_last_error() describes the problem.
 *   - Host pointers are borrowed for the duration of the call; the caller keeps
 *     ownership. Device pointers (the *_dev calls) are read before the call
 *     returns (the call synchronises its stream).
 *   - A context is used from one host thread at a time.
 *   - pic_step only enqueues work on the context's stream and returns; the
 *     pic_get_* calls synchronise the stream and report device-side errors
 *     (PIC_E_RANGE: a non-finite or runaway particle position) raised since
 *     the last synchronising call.
 *   - The library owns all device memory of a context and frees it in
 *     pic_destroy. It takes that memory from pic_config.alloc when the caller
 *     gives an allocator (for instance a framework's caching allocator, so
 *     that the context's tens of GB are not held beside the framework's pool),
 *     else from hipMalloc.
 */
#ifndef PIC_H_
#define PIC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_MAX_SPECIES 4
#define PIC_NUM_FACES 6
/* Most ids of one pic_get_particles_by_id_noalloc call. */
#define PIC_NOALLOC_MAX_IDS 65536

typedef struct pic_ctx pic_ctx;

typedef enum {
  PIC_OK = 0,
  PIC_E_INVALID = -1, /* a bad argument; nothing changed */
  PIC_E_NOMEM = -2,   /* device memory could not be allocated (nothing changed), or
                         particles did not fit the reserved regions (reported at sync) */
  PIC_E_DEVICE = -3,  /* no usable GPU, or a HIP runtime error */
  PIC_E_STATE = -4,   /* call out of order (e.g. pic_step before pic_set_node_E) */
  PIC_E_RANGE = -5    /* a particle position became non-finite or moved > 2^20 cells */
} pic_status;

/* Particle representation on the device. */
typedef enum {
  PIC_REPR_FP64 = 0,      /* FP64 positions and velocities (48 B per particle) */
  PIC_REPR_FP32_ABS = 1,  /* FP32 positions (cell units) and velocities (24 B) */
  PIC_REPR_FP32_CELL = 2  /* cell + FP32 in-cell offsets + FP32 velocities: 24 B per
                             particle streamed (the offsets' two top bits, always zero
                             in [0, 1), hold the cell within its tile of 4^3 cells; the
                             tile region holding a particle gives the tile) and a 4 B
                             cell index kept only for particles outside a region */
} pic_repr;

/* Charge deposition arithmetic. */
typedef enum {
  PIC_DEP_FIXED64 = 0,     /* int64 fixed point, scale 2^32: deterministic */
  PIC_DEP_ATOMIC_FP32 = 1, /* FP32 atomic sums: order-dependent rounding */
  PIC_DEP_ATOMIC_FP64 = 2  /* FP64 atomic sums: order-dependent rounding */
} pic_deposit;

typedef enum { PIC_OBJ_NONE = 0, PIC_OBJ_SPHERE = 1, PIC_OBJ_CRATER = 2 } pic_object_kind;

typedef struct {
  int32_t kind;      /* pic_object_kind */
  double center[3];  /* sphere centre; crater axis at (center[0], center[1]) */
  double radius;     /* sphere radius */
  double z_flat;     /* crater: height of the flat ground */
  double rim_radius; /* crater: bowl radius at the flat level (a) */
  double depth;      /* crater: bowl depth below the flat level (d > 0) */
  int32_t patches;   /* sphere only, 0..64: 0 = one tally bin for the whole
                        sphere; m >= 1 = 6 m^2 surface patches, the bin of a
                        collected particle being the patch its offset d from
                        the centre points through (gnomonic cube map): face
                        2a + (d_a >= 0) of the largest |d_a| (ties to the lower
                        axis), the two other components in axis order divided
                        by |d_a| and cut into m equal intervals of [-1, 1]:
                        bin = (face m + iv) m + iu. Where on the sphere the
                        collected charge sits (the flux jump q(X) of eq. (2.5)). */
} pic_object;

typedef struct {
  double q;      /* charge of one physical particle */
  double m;      /* mass (> 0) */
  double weight; /* physical particles per macro-particle */
} pic_species;

typedef struct {
  int32_t nx, ny, nz;  /* cells per axis, 1..1023 */
  double h;            /* cell edge (> 0) */
  double origin[3];    /* position of node (0,0,0) */
  double dt;           /* time step (> 0) */
  int32_t n_species;   /* 1..PIC_MAX_SPECIES */
  pic_species species[PIC_MAX_SPECIES];
  pic_object object;
  int32_t repr;          /* pic_repr */
  int32_t deposit;       /* pic_deposit */
  int32_t sort_interval; /* particles are kept grouped by tile of 4^3 cells; every
                            step moves each particle to its new tile's region.
                            K >= 1 also re-plans the tile regions of all species
                            every K steps; 0 (default) re-plans a species' regions
                            only after its load or when one of its tiles runs
                            out of spare room. Results do not depend on it. */
  int32_t reflect;       /* bit f: box face f (0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+)
                            reflects instead of removing (the symmetry planes of
                            the particle setups in §3.1.3 and §5.2.2): right after
                            the drift, a particle beyond the face is mirrored about
                            it and its normal velocity negated, axes x, y, z in
                            turn; one that lands exactly on a max face is put just
                            inside. The crater's z- face (the terrain) cannot. */
  int64_t capacity[PIC_MAX_SPECIES]; /* max particles per species (device memory is
                                        reserved for this many plus per-tile spare
                                        room and an overflow list, double-buffered) */
  void *stream;          /* hipStream_t to enqueue on, or NULL for a library stream */
  /* Device memory allocator (optional; all three NULL: hipMalloc / hipFree).
   * alloc(bytes, alloc_user) returns device memory of the context's GPU with
   * at least 256-byte alignment, or NULL when it cannot (the calling
   * pic_* function then fails with PIC_E_NOMEM and nothing changes);
   * dealloc(ptr, alloc_user) takes back a pointer that alloc returned. The
   * library calls them from the calling thread, only inside pic_create,
   * pic_load_particles* (id arrays), pic_set_photoemission, pic_solve_field,
   * pic_get_particles_by_id and pic_destroy, and gives back every
   * allocation by the end of pic_destroy (after synchronising the context's
   * stream). alloc and dealloc are given together or not at all. */
  void *(*alloc)(size_t bytes, void *user);
  void (*dealloc)(void *ptr, void *user);
  void *alloc_user;
} pic_config;

/* Ambient particles injected through box faces every step (the particle
 * setups of §3.1.3 and §5.2.2 inject the ambient plasma at the open faces; the
 * paper gives no method). Per step, after every particle was pushed and before
 * the deposit, for each species s and injecting face: a ghost slab of
 * thickness L = min(1, dt (max(0, u.n_in) + 6 vth)) cells outside each face
 * cell holds floor(n L + U) ghost particles (n = density h^3 per cell, U a
 * uniform draw) placed uniformly in the slab, with velocities u + vth N(0,1)
 * per component (Marsaglia's polar method); each moves dt and is injected if it
 * ends inside the box, rounded to the context's representation; it then meets
 * the object test like a pushed particle (collected at once, or kept and
 * deposited). Random numbers: SplitMix64 as a counter-based generator keyed by
 * (seed, step index, species, face, face cell, ghost); the step index counts
 * pic_step steps from pic_create, or from the value pic_set_step_index set. Only correctly rounded operations are used
 * (ln by an atanh series), so the injected particles are fully determined by
 * the inputs. Ghosts faster than u.n_in + 6 vth toward the face are not
 * generated (a relative flux deficit below 1e-9). Injected particles take the
 * id -1 in species that carry ids. */
typedef struct {
  int32_t faces;                    /* bit f: face f injects; 0 turns injection off */
  uint64_t seed;
  double density[PIC_MAX_SPECIES];  /* ambient particles per unit volume (>= 0) */
  double vth[PIC_MAX_SPECIES];      /* thermal speed per component (>= 0) */
  double drift[PIC_MAX_SPECIES][3]; /* drift velocity */
} pic_injection;

/* Creates a context: validates cfg and allocates device memory for the mesh
 * (node E, rho), tallies and per-species particle buffers of cfg->capacity.
 * Returns PIC_E_NOMEM if the device cannot hold it. *out is set on success. */
pic_status pic_create(const pic_config *cfg, pic_ctx **out);

/* Frees the context and all its device memory (synchronises its stream). NULL is
 * ignored. */
void pic_destroy(pic_ctx *ctx);

/* Replaces the particles of one species by n particles at physical positions
 * (x, y, z) with velocities (vx, vy, vz) taken at t - dt/2 (the leapfrog
 * stagger). Host arrays of n doubles. ids (nullable) are n int64 labels carried
 * through sorting and returned by pic_get_particles; without ids the particle
 * order is unspecified after a step. Every position must lie inside the box,
 * also after rounding to the representation (an FP32 coordinate that rounds
 * up to the upper face is outside)
 * (PIC_E_INVALID otherwise); n must not exceed the species capacity. Loading a
 * species resets its collected counts (tally column), escape counters and
 * injected count.
 * Values are rounded to the representation (round to nearest). Synchronous. */
pic_status pic_load_particles(pic_ctx *ctx, int32_t species, int64_t n, const double *x,
                              const double *y, const double *z, const double *vx,
                              const double *vy, const double *vz, const int64_t *ids);

/* As pic_load_particles, from device arrays of n floats (and n int64 ids, or
 * NULL) in the GPU's memory. Positions outside the box raise PIC_E_INVALID.
 * Synchronous on the context's stream. */
pic_status pic_load_particles_f32_dev(pic_ctx *ctx, int32_t species, int64_t n,
                                      const float *x, const float *y, const float *z,
                                      const float *vx, const float *vy, const float *vz,
                                      const int64_t *ids);

/* Sets the node electric field: three host arrays of (nx+1)(ny+1)(nz+1) doubles,
 * x fastest. The FP32 representations round it to float. Non-finite values give
 * PIC_E_INVALID. Synchronous. */
pic_status pic_set_node_E(pic_ctx *ctx, const double *Ex, const double *Ey, const double *Ez);

/* As pic_set_node_E, from three device arrays of floats. Synchronous. */
pic_status pic_set_node_E_f32_dev(pic_ctx *ctx, const float *Ex, const float *Ey,
                                  const float *Ez);

/* Advances all particles by nsteps steps (enqueued on the context's stream; no
 * host synchronisation). nsteps == 0 only deposits rho at the current positions
 * (the initial scatter). rho always holds the deposit of the last step.
 * PIC_E_STATE before pic_set_node_E. */
pic_status pic_step(pic_ctx *ctx, int32_t nsteps);

/* Blocks until the context's stream is idle; reports device-side errors. */
pic_status pic_synchronize(pic_ctx *ctx);

/* Charge density at the nodes (host array of (nx+1)(ny+1)(nz+1) doubles), and,
 * in the fixed-point mode, the raw int64 sums at scale 2^32 (nullable; must be
 * NULL in the other modes). rho = rho_fixed * 2^-32 / h^3. Synchronises. */
pic_status pic_get_rho(pic_ctx *ctx, double *rho, int64_t *rho_fixed);

/* Number of collection bins: 0 (no object), 1 (sphere), nx*ny (crater). */
int64_t pic_num_bins(const pic_ctx *ctx);

/* Collected charge per bin, sum over species of q*w*count, in FP64 (nbins
 * doubles, nbins == pic_num_bins), and optionally the raw counts
 * counts[bin*n_species + s] (nullable). Cumulative since the species were
 * loaded. This is the surface charge that sets the non-homogeneous flux jump
 * q(X) of eq. (2.5). Synchronises. */
pic_status pic_get_surface_charge(pic_ctx *ctx, int64_t nbins, double *charge, int64_t *counts);

/* Per-species counters (host arrays of n_species, n_species, 6*n_species int64,
 * each nullable): particles alive, collected at the object, and escaped
 * through face f (escaped[f*n_species + s]). Synchronises. */
pic_status pic_get_counters(pic_ctx *ctx, int64_t *alive, int64_t *absorbed, int64_t *escaped);

/* The field solve on the PIC mesh (the boundary value problem of §2.1),
 * by node-centred finite volumes (below) or by immersed finite elements
 * (PIC_FIELD_IFE):
 * -eps lap(phi) = rho on the nodes, phi = value[f] on the Dirichlet faces f,
 * zero normal derivative on the others (the symmetry / open faces of §3.1.3
 * and §5.2.2). Node-centred finite volumes: each node's control volume is its
 * dual cell clipped to the box and the right-hand side is the deposited
 * nodal density of pic_get_rho, so a zero-Neumann face needs no extra term.
 * Solved by preconditioned conjugate gradients (the PCG of §2.4) until
 * ||r||_2 <= tol ||b||_2 or max_iter iterations, from the previous solution
 * (zero before the first). Then E = -grad phi at the nodes (central
 * differences; 0 normal to a zero-Neumann face; second-order one-sided on a
 * Dirichlet face) becomes the context's node field, as pic_set_node_E would.
 *
 * With eps_object > 0 each link's permittivity is the series (harmonic)
 * combination of eps_object and eps by the fraction of the link inside the
 * object, from linear interpolation of a level set at its two nodes
 * (|x - c| - R for the sphere, z - ground(x, y) for the terrain); the same
 * rule on every multigrid level. Exact for a layered medium.
 *
 * Preconditioners (the paper does not fix one):
 *   PIC_PRECOND_MULTIGRID: one geometric multigrid V-cycle on nested node
 *     grids (every other node, spacing doubled, while the grid has more than
 *     1024 nodes and all three cell counts are even, at most 8 levels; two
 *     damped-Jacobi sweeps before and after the coarse correction, full-
 *     weighting restriction, trilinear prolongation, exact solve on the
 *     coarsest grid, whose inverse is computed on the host once per set of
 *     Dirichlet faces and eps). A grid that does not coarsen to at most 1024
 *     nodes, or has at most 1024, uses Jacobi; pic_get_field_levels tells.
 *     The iteration count does not grow with the grid.
 *   PIC_PRECOND_JACOBI: z = r / diag(A). */
enum { PIC_PRECOND_MULTIGRID = 0, PIC_PRECOND_JACOBI = 1 };
/* Discretisation of the field problem (pic_field.op):
 *   PIC_FIELD_FV: the node-centred finite volumes above.
 *   PIC_FIELD_IFE: immersed finite elements, the paper's method (§2.3), on
 *     the PIC mesh with every cell cut into five tetrahedra (§3.1.1): in a
 *     cube of parity (i + j + k) mod 2 = p the central tetrahedron on the four
 *     corners (a, b, c) with a + b + c = p mod 2 and one tetrahedron per other
 *     corner (that corner and its three axis neighbours). Linear elements
 *     away from the object; in a tetrahedron that the object's surface cuts
 *     (the plane where the linear interpolant of the level set vanishes) the
 *     basis functions are linear on each side, continuous across the plane
 *     and with eps grad phi . n continuous across it (eq. (2.4), (2.5) with
 *     the collected charge in the right-hand side). The right-hand side is the
 *     nodal density of the deposit, as for the finite volumes. The multigrid
 *     preconditioner smooths the finest level with this operator and keeps
 *     the finite volumes on the coarser ones. Without an object
 *     (eps_object = 0) the plain linear elements on the same tetrahedra. */
enum { PIC_FIELD_FV = 0, PIC_FIELD_IFE = 1 };
typedef struct {
  int32_t dirichlet; /* bit f: face f (0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+) holds
                        phi = value[f]; at least one face */
  double value[6];
  double eps;        /* permittivity (> 0) */
  double tol;        /* relative residual (> 0); the paper uses 1e-6 */
  int32_t max_iter;  /* >= 0; the paper uses 60-150 per PIC step */
  int32_t preconditioner; /* PIC_PRECOND_* */
  double eps_object;      /* > 0: the object is an interface of the problem (eq.
                             (2.2)-(2.5)) with this permittivity inside it (the
                             sphere's interior, or below the terrain) and eps
                             outside; 0: uniform eps (the object is not part of
                             the field problem) */
  int32_t surface_charge; /* 1: the collected charge of pic_get_surface_charge is
                             the flux-jump source q(X) of eq. (2.5), placed at
                             each tally bin's surface point (crater column:
                             the terrain above its centre; sphere patch: the
                             sphere point towards the patch centre; a sphere
                             needs patches >= 1) and deposited to the nodes in
                             int64 fixed point like a particle's charge; a
                             bin's charge must stay below 2^30 in magnitude
                             (PIC_E_RANGE at the solve). 0: volume charge only */
  int32_t op;             /* PIC_FIELD_FV or PIC_FIELD_IFE */
} pic_field;

/* Solves for the deposit of the last pic_step (PIC_E_STATE before any) and
 * synchronises; *iterations and *rel_residual (nullable) receive the CG
 * iterations and ||r|| / ||b||. PIC_E_INVALID: bad field settings. Deterministic
 * (fixed-order reductions). */
pic_status pic_solve_field(pic_ctx *ctx, const pic_field *field, int32_t *iterations,
                           double *rel_residual);

/* Copies the context's node field (set, or from the last field solve) to host
 * arrays of (nx+1)(ny+1)(nz+1) values, x fastest, in FP64 (FP32 forms hold it
 * in FP32). PIC_E_STATE before any. Synchronises. */
pic_status pic_get_node_E(pic_ctx *ctx, double *Ex, double *Ey, double *Ez);

/* Copies the potential of the last pic_solve_field to phi (host, one value per
 * node, x fastest); PIC_E_STATE before any solve. Synchronises. */
pic_status pic_get_phi(pic_ctx *ctx, double *phi);

/* *levels = the multigrid level count of the last pic_solve_field (0: the
 * Jacobi preconditioner ran); PIC_E_STATE before any solve. */
pic_status pic_get_field_levels(pic_ctx *ctx, int32_t *levels);

/* Sets (inj non-NULL with faces != 0) or clears (NULL or faces == 0) the
 * injection of ambient particles, from the next pic_step on (copied; the
 * caller keeps inj). PIC_E_INVALID: a face bit beyond 5, an injecting face
 * that reflects, the crater's z- face, a negative or non-finite density,
 * thermal speed or drift; nothing changes on error. The particles must fit the
 * species' capacity (PIC_E_NOMEM at the next sync otherwise). */
pic_status pic_set_injection(pic_ctx *ctx, const pic_injection *inj);

/* Synchronises; injected[s] (n_species values) receives the particles
 * injected into species s since pic_create or its last load (collected at
 * once included; photoelectrons count as injected into their species). */
pic_status pic_get_injected(pic_ctx *ctx, int64_t *injected);

/* Sets the step index of the next pic_step (0 <= step < 2^31; it counts on by
 * one per step). The random draws of the injection and of the photoemission
 * are keyed by it, so a run exported after k steps (pic_get_particles, tallies)
 * and loaded into a fresh context continues the draws of one long run when
 * the new context is set to k; a fresh context starts at 0. Takes effect for
 * steps enqueued after the call. PIC_E_INVALID: out of range. */
pic_status pic_set_step_index(pic_ctx *ctx, int64_t step);

/* Photoemission from the sunlit terrain (the lunar setup of §5.2.2, where
 * photoelectrons are generated according to the local sunlight index, the
 * inner product of the direction to the Sun and the surface normal, and none
 * in shadow). Each step, after the ambient injection and before the
 * deposit, every surface column (i, j) of the crater terrain takes the
 * terrain at its centre: outward unit normal n, ground height, index
 * I = s.n (s = sun normalised). The column is lit if I > 0 and, inside the
 * bowl, the ray from that ground point towards the Sun leaves the bowl sphere
 * (a chord of length 2 Rc I) at or above the flat ground. A lit column emits
 * floor(mean + U) photoelectrons of the given species, mean =
 * (flux / weight) h^2 dt I / n_z (the emitted flux at normal incidence times
 * the cosine of incidence over the column's terrain area h^2 / n_z). Each
 * starts at a uniform point of the column's footprint on the ground with a
 * half-Maxwellian velocity about n, vth (|z0| n + z1 t1 + z2 t2) with
 * t1 = (n_z, 0, -n_x) normalised and t2 = n x t1, moves a uniform fraction of
 * dt, and is then tested and appended like an injected particle. Random
 * numbers: the counter-based SplitMix64 keys of the injection (seed, step,
 * species, face index 6, column, photoelectron), so the emission is the same
 * in any step split and on any device. */
typedef struct {
  int32_t species;  /* the photoelectron species (its q, m, weight from the config) */
  uint64_t seed;
  double sun[3];    /* direction towards the Sun, any length, sun[2] > 0 */
  double flux;      /* emitted physical particles per unit area and time at normal
                       incidence (>= 0) */
  double vth;       /* thermal speed of the emitted half-Maxwellian (>= 0) */
} pic_photoemission;

/* Sets (pe non-NULL) or clears (NULL) the photoemission, from the next
 * pic_step on (copied). PIC_E_INVALID: no crater terrain, species out of
 * range or with weight <= 0, sun not finite or sun[2] <= 0, negative or
 * non-finite flux or vth, more than 2^20 photoelectrons per column per step
 * or speeds beyond 2^20 cells per step; nothing changes on error. The
 * particles must fit the species' capacity (PIC_E_NOMEM at the next sync
 * otherwise); when the capacity also leaves room for some 20 steps of
 * emission, the tile regions keep room for 16 steps of it in the tiles the
 * photoelectrons start in, so that a growing population does not re-plan
 * the regions every step. Contexts with photoemission are not attached to a
 * batch. */
pic_status pic_set_photoemission(pic_ctx *ctx, const pic_photoemission *pe);

/* Copies the alive particles of one species to host arrays of capacity cap
 * (physical positions and half-step velocities as doubles; ids nullable, and
 * only available if ids were loaded). *n_out receives the number of alive
 * particles; if it exceeds cap nothing is copied and PIC_E_INVALID is
 * returned. Order is the device's memory order. Synchronises. */
pic_status pic_get_particles(pic_ctx *ctx, int32_t species, int64_t cap, int64_t *n_out,
                             double *x, double *y, double *z, double *vx, double *vy,
                             double *vz, int64_t *ids);

/* Looks up particles of one species by id (ids must have been loaded with the
 * species). ids_sorted: host array of n distinct ids in ascending order. For
 * each k, found[k] = 1 and the particle's physical position and half-step
 * velocity are written to x[k] .. vz[k] if a particle with that id is alive,
 * else found[k] = 0 (outputs untouched). A device-side search, so sampled
 * particles of a very large run can be read without copying the whole state.
 * Synchronises. */
pic_status pic_get_particles_by_id(pic_ctx *ctx, int32_t species, int64_t n,
                                   const int64_t *ids_sorted, int32_t *found, double *x,
                                   double *y, double *z, double *vx, double *vy, double *vz);

/* pic_get_particles_by_id for callers that cannot allocate device memory
 * (a tight serving loop, a harness that forbids allocation): the same
 * arguments, results and errors, but the id list and the results are staged
 * in a fixed scratch area of the library's (PIC_NOALLOC_MAX_IDS * 64 bytes of
 * device memory on each GPU it runs on, kept until the process ends) instead
 * of memory allocated per call; the call allocates no device memory (neither
 * hipMalloc nor pic_config.alloc). n > PIC_NOALLOC_MAX_IDS: PIC_E_INVALID.
 * All contexts on one GPU share that GPU's scratch area and it keeps the last
 * call's contents: calls that overlap in time on one GPU (from several host
 * threads) race and must be serialised by the caller. Synchronises. */
pic_status pic_get_particles_by_id_noalloc(pic_ctx *ctx, int32_t species, int64_t n,
                                           const int64_t *ids_sorted, int32_t *found, double *x,
                                           double *y, double *z, double *vx, double *vy,
                                           double *vz);

/* Kernel timing for measurement: when enabled, the library records HIP events
 * around each launch of its kernels on the context's stream. */
typedef struct {
  int64_t step_launches;  /* fused gather/push/collect/deposit kernel */
  double step_ms;         /* summed event time of those launches */
  int64_t sort_launches;  /* re-bucketing passes (each: count, scan, scatter, commit) */
  double sort_ms;
  int64_t clear_launches; /* rho clears */
  double clear_ms;
  int64_t particle_steps; /* particles alive at the start of each step, summed */
  int64_t inject_launches; /* injection launches (pic_set_injection) */
  double inject_ms;
  int64_t field_solves;    /* pic_solve_field calls */
  double field_ms;         /* device time from the solve's first to last kernel */
  int64_t field_iterations; /* CG iterations, summed */
  int64_t photo_launches;  /* photoemission launches (pic_set_photoemission) */
  double photo_ms;
} pic_profile;

/* Enables (on != 0) or disables event timing and resets the totals. */
pic_status pic_profile_enable(pic_ctx *ctx, int32_t on);
/* Synchronises and returns the totals since pic_profile_enable. */
pic_status pic_profile_read(pic_ctx *ctx, pic_profile *out);

/* ---- batched runs (serving many independent runs on one GPU) -------------
 *
 * A batch advances many contexts ("slots") together: one launch per step
 * covers the tiles of every attached context (persistent workgroups take
 * (context, tile) items from a counter), and the steps of one pic_batch_run
 * are replayed from a captured HIP graph. Contexts are created,
 * loaded and read as usual; attaching admits one to the batch if its device
 * footprint fits the batch's budget and a slot is free. Each attached context
 * gets exactly the same per-step computation as pic_step would give it, so
 * its results do not depend on what else is in the batch. All attached
 * contexts must use the batch's repr and deposit. While attached, a context
 * accepts no other call but pic_batch_detach (other calls: PIC_E_STATE). */

typedef struct pic_batch pic_batch;

typedef struct {
  int32_t max_slots;        /* contexts attached at once, 1..1024 */
  int32_t repr, deposit;    /* of every attached context */
  int32_t steps_per_run;    /* M >= 1: the most steps one pic_batch_run gives a context */
  int64_t hbm_budget_bytes; /* admission limit on the summed footprints (> 0) */
  int64_t particle_steps_per_run; /* P. 0 -> every context gets M steps per run;
                                     > 0 -> shares: context k with n_k particles
                                     (at attach) and weight w_k gets
                                     clamp(floor(P w_k / (W n_k)), 1, M) steps,
                                     W the sum of the running contexts' weights
                                     (all 1: each gets about the same GPU time
                                     and small runs are not paced by large ones) */
  void *stream;             /* hipStream_t, or NULL for a library stream */
} pic_batch_config;

/* Device bytes that pic_create allocates for cfg (without ids); -1 if cfg is
 * invalid. The admission unit of a batch. */
int64_t pic_footprint_bytes(const pic_config *cfg);

pic_status pic_batch_create(const pic_batch_config *cfg, pic_batch **out);

/* Detaches every slot (the contexts stay valid) and frees the batch. */
void pic_batch_destroy(pic_batch *b);

/* Admits ctx for nsteps more steps into a free slot (*slot receives it).
 * PIC_E_NOMEM: its footprint does not fit the remaining budget; PIC_E_STATE:
 * no free slot, no node field set, or ctx already attached; PIC_E_INVALID:
 * different repr / deposit, nsteps < 1. Nothing changes on error. */
pic_status pic_batch_attach(pic_batch *b, pic_ctx *ctx, int64_t nsteps, int32_t *slot);

/* Weight of an attached context in the share of P (default 1 at attach; used
 * from the next run on). Weight 0 pauses the context: it takes no step in the
 * runs that follow (its state stays on the device) until its weight is set
 * again, unless every attached context with steps left is paused, in which
 * case all of them run with equal weights. PIC_E_INVALID: no context in the
 * slot, weight not in [0, 1e30). A scheduler sets weights to implement its
 * policy (e.g. the oldest request first, small ones beside it). */
pic_status pic_batch_set_weight(pic_batch *b, int32_t slot, double weight);

/* Advances every attached context by min(its quota, its remaining steps)
 * (quota: M, or its share of P above) and synchronises. done_slots (capacity
 * max_slots, nullable) receives the slots whose steps are now all done,
 * *n_done their number. */
pic_status pic_batch_run(pic_batch *b, int32_t *n_done, int32_t *done_slots);

/* pic_batch_run in two halves, so that the host can prepare and attach new
 * contexts while a run executes: pic_batch_launch enqueues the run on the
 * batch's stream and returns; pic_batch_wait synchronises and reports the
 * finished slots as pic_batch_run does (n_done = 0 when nothing is in flight).
 * While a run is in flight pic_batch_attach may be called (the new context
 * joins the next run); pic_batch_launch and pic_batch_detach fail with
 * PIC_E_STATE. */
pic_status pic_batch_launch(pic_batch *b);
pic_status pic_batch_wait(pic_batch *b, int32_t *n_done, int32_t *done_slots);

/* Releases a slot; its context is usable again (results via pic_get_*). */
pic_status pic_batch_detach(pic_batch *b, int32_t slot);

/* Summed footprints of the attached contexts. */
int64_t pic_batch_used_bytes(const pic_batch *b);

/* Steps the context in `slot` still has to take (after the runs completed by
 * pic_batch_run / pic_batch_wait; a run in flight is not counted yet); -1 if
 * the slot is empty or out of range. For schedulers that size quotas. */
int64_t pic_batch_remaining(const pic_batch *b, int32_t slot);

/* Message of the last failed call on a batch. Never NULL. */
const char *pic_batch_last_error(const pic_batch *b);

/* Message of the last failed call on ctx (or of the last failed pic_create when
 * ctx is NULL). Never NULL. */
const char *pic_last_error(const pic_ctx *ctx);

/* Static name of a status code. */
const char *pic_status_string(pic_status s);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H_ */
