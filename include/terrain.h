/*
 * terrain.h -- C-ABI of libterrain.so: one time step of the agitated-soil
 * particle system of Servin, Berglund & Nystedt, "A multiscale model of terrain
 * dynamics for real-time earthmoving simulation" (arXiv 2011.00459), on one
 * AMD Instinct MI355X (gfx950).
 *
 * The soil in an active zone is a set of frictional-cohesive spheres (section
 * "Microscopic model": pseudo-particles with parameters [rho, mu_t, mu_r, c_p,
 * E]).  Their equation of motion is Eq. eqmotb (section "Mesoscale model"):
 * gravity plus contact impulses from the other spheres, from the moving
 * equipment B and from the resting terrain C, both treated as geometric
 * boundaries.  One step (Algorithm 1: collision detection, the mesoscale
 * contact constraints, the PGS solve and the position update, plus the
 * aggregation of each active zone into a body with Eqs. aggregate_mass ..
 * aggregate_rot_vel) runs entirely on the GPU.
 *
 * Conventions
 *  - Every function returns TR_OK (0) or a negative TR_E_* code; the message
 *    is available from get_last_error() until the next call on that scene.
 *  - Host arrays passed in are borrowed for the duration of the call and
 *    copied; the library never keeps a host pointer.
 *  - A scene owns its device buffers (allocated through desc.alloc_fn when
 *    given, else hipMalloc) and runs all work on desc.stream (the null stream
 *    when NULL).  Handles are not thread-safe; one scene uses one stream.
 *  - Positions are stored in FP32 in the frame they are given in; callers
 *    should place each environment near the origin (FP32 resolution).
 *  - Particle ids are consecutive per environment: env e owns the id range
 *    [e * cap_particles, (e + 1) * cap_particles).
 *  - A failed step leaves the particle state unchanged.
 */
#ifndef TERRAIN_H
#define TERRAIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TR_OK 0
#define TR_E_INVAL (-1)     /* invalid argument (NULL, out of range, unsupported option) */
#define TR_E_NOMEM (-2)     /* device or host allocation failed */
#define TR_E_DEVICE (-3)    /* HIP runtime error; message carries the HIP error string */
#define TR_E_STATE (-4)     /* call not valid in the scene's current state */
#define TR_E_CAPACITY (-5)  /* a capacity (particles, contacts, colours, cells) was exceeded */
#define TR_E_NONFINITE (-6) /* NaN or Inf in an input */

enum tr_warm_start {
    TR_WARM_COLD = 0,    /* lambda^0 = 0 */
    TR_WARM_PREV = 1,    /* previous step's impulses, matched by contact key */
    TR_WARM_LEARNED = 2  /* MLP prediction, falling back to PREV/COLD */
};

enum tr_shape_type { TR_PLANE = 0, TR_BOX = 1, TR_HEIGHTFIELD = 2 };

/* Particle and contact-law parameters, p_p = [rho, mu_t, mu_r, c_p, E]
 * (section "Microscopic model") and the contact law of Eqs. signCoul1-2 with
 * the Hertz mapping and SPOOK parameters (section "Contacting rigid
 * multibodies").  Defaults from section "Soil library": E = 1e9 Pa,
 * nu = 0.15, restitution 0. */
typedef struct tr_material {
    double rho;         /* particle density [kg/m^3], used when add_particles gets no density */
    double mu_t;        /* Coulomb friction coefficient */
    double mu_r;        /* rolling resistance (Eq. signCoul3), >= 0; 0 = no rolling rows */
    double c_p;         /* particle cohesion [Pa]; 0 disables cohesion and its range */
    double E;           /* Young's modulus [Pa] */
    double nu;          /* Poisson's ratio */
    double restitution; /* Newton restitution e in [0, 1] of the impact stage (unused when v_imp <= 0) */
    double tau_n;       /* normal damping time [s]; <= 0 means 2 dt */
    double gamma_t;     /* tangential regularisation [s]; 0 = ideal Coulomb */
    double kappa_c;     /* cohesive range: delta > -kappa_c (r1 + r2) keeps a contact */
    double kappa_min;   /* compliance uses max(delta, kappa_min (r1 + r2)) */
    double v_imp;       /* impact threshold [m/s] (the impact stage before the main
                           solve): a contact whose start-of-step normal velocity
                           approaches faster than v_imp gets G_n v+ = -e G_n v-, the
                           env's other contacts G v+ = 0 (unilateral normal, Coulomb
                           and rolling bounds), solved by the same coloured sweeps
                           without compliance or cohesion; the main solve then starts
                           from v+.  <= 0 disables the stage. */
} tr_material;

/* Device memory callbacks: alloc returns device memory usable on `stream`
 * (e.g. from a framework's caching allocator); free releases it. */
typedef void* (*tr_alloc_fn)(void* ctx, size_t bytes, void* stream);
typedef void (*tr_free_fn)(void* ctx, void* ptr, void* stream);

typedef struct tr_scene_desc {
    int32_t n_envs;          /* independent environments stepped together (>= 1) */
    double dt;               /* time step [s] */
    double gravity[3];       /* [m/s^2] */
    int32_t max_sweeps;      /* PGS sweeps per step (cap when tol > 0) */
    double tol;              /* stop when the sweep residual R_k <= tol; 0 = fixed sweeps */
    int32_t warm_start;      /* enum tr_warm_start */
    tr_material material;
    int64_t cap_particles;   /* particle capacity per environment */
    int64_t cap_contacts;    /* contact capacity per environment */
    const double* env_bounds;/* n_envs x 6: lo xyz, hi xyz of each env's cell grid
                                (particles outside are clamped to the border cells) */
    double r_ref;            /* nominal radius (learned-start feature scale); <= 0 means 1 m */
    void* stream;            /* hipStream_t, or NULL */
    tr_alloc_fn alloc_fn;    /* NULL: hipMalloc (alloc_fn and free_fn are given together or not at all) */
    tr_free_fn free_fn;      /* NULL: hipFree; called once for every block alloc_fn returned, at latest by destroy_scene */
    void* alloc_ctx;
} tr_scene_desc;

/* Boundary shape of a kinematic body (equipment B or resting terrain C).
 *   TR_PLANE       : surface normal . y = offset in the body frame; particles
 *                    live on the +normal side.
 *   TR_BOX         : oriented box with half extents `half`, centred at
 *                    `center` in the body frame, axes of the body frame.
 *   TR_HEIGHTFIELD : the terrain surface of Eq. surface, heights[j*nx+i] at
 *                    (origin[0] + i l0, origin[1] + j l0), linear between grid
 *                    points, in the world frame; its body must be static. */
typedef struct tr_shape_desc {
    int32_t type;
    double normal[3];
    double offset;
    double half[3];
    double center[3];
    int32_t nx, ny;
    double origin[2];
    double l0;
    const float* heights;    /* nx*ny values, copied */
} tr_shape_desc;

/* A kinematic body: its pose advances every step with its constant linear and
 * angular velocity (x += dt v; q <- normalize(q + dt/2 (0, w) q)).  An optional
 * active zone is given by up to 8 half-spaces in the body frame, a particle
 * being inside when planes[k][0..2] . y <= planes[k][3] for every k (the wedge
 * of Eq. failure_plane; see zones.py for a builder). */
typedef struct tr_body_desc {
    int32_t id;
    double pos[3];
    double quat[4];          /* (w, x, y, z) */
    double linvel[3];
    double angvel[3];
    int32_t n_shapes;
    const tr_shape_desc* shapes;
    int32_t n_halfspaces;    /* 0 = no active zone */
    double planes[8][4];
} tr_body_desc;

/* Digging tool or soil deformer of a kinematic body: its active zone is
 * predicted every step (after the pose update) from the env's terrain
 * heightfield (its first TR_HEIGHTFIELD shape), replacing the body's
 * half-space zone.  For each of n_wedges lateral slices of the cutting edge
 * the zone is the wedge between the separation plate through the edge and
 * the failure plane rising at theta(phi, beta) = pi/2 - (phi + beta)/2
 * against the terrain surface (Eq. failure_plane; beta from the surface
 * tangent to the plate, in the plane normal to the edge), up to where that
 * plane meets the surface plus `heap`, between the slice's lateral planes.
 * The plate normal is normalize((1 - fill) n_c + fill n_tc) (the secondary
 * separation plate of a partly filled bucket).  Geometry in the body frame. */
/* Voxel grid of the mesoscale fields: voxel (i, j, k) spans origin +
 * l0 [i, i+1) x [j, j+1) x [k, k+1); arrays are indexed (k ny + j) nx + i. */
typedef struct tr_voxel_grid {
    double origin[3];
    double l0;               /* voxel edge [m], > 0 */
    int32_t nx, ny, nz;      /* > 0 */
    int32_t pad;
} tr_voxel_grid;

enum { TR_CG_HEAVISIDE = 0, TR_CG_GAUSS = 1 };

#define TR_MAX_WEDGES 16
typedef struct tr_tool_desc {
    int32_t n_wedges;        /* 1 .. TR_MAX_WEDGES */
    int32_t pad;
    double edge0[3];         /* cutting edge end points */
    double edge1[3];
    double n_c[3];           /* normal of the primary separation plate, towards the zone */
    double n_tc[3];          /* normal of the face from cutting edge to top edge (= n_c: a blade) */
    double fill;             /* fill ratio of the inner shape, [0, 1] */
    double phi;              /* soil internal friction angle [rad], (0, pi/2) */
    double heap;             /* zone height above where the failure plane meets the surface [m], >= 0 */
    double v_min;            /* a deformer: a zone only while the edge speed exceeds v_min; <= 0: always */
} tr_tool_desc;

typedef struct tr_step_stats {
    int64_t contacts;        /* all contacts of the env (pairs + boundary) */
    int64_t pair_contacts;
    int32_t colours;         /* colours used by this env's contacts */
    int32_t sweeps;          /* PGS sweeps done */
    double residual;         /* R_k after the last sweep */
    double residual_first;   /* R_1 */
    int32_t fallback_used;   /* learned start rejected, PREV/COLD used */
    int32_t overflow;        /* nonzero when a capacity was exceeded (step aborted) */
    int32_t impacts;         /* contacts treated as impacts (0: no impact stage in this env) */
    int32_t impact_sweeps;   /* sweeps of the env's impact stage */
} tr_step_stats;

/* Aggregate body of one active zone (Eqs. aggregate_mass .. aggregate_rot_vel,
 * particle sums only), FP64, after the step's position update. */
typedef struct tr_aggregate {
    int32_t zone;            /* id of the body that owns the zone */
    int32_t pad;
    int64_t n_particles;
    double M;
    double x[3];             /* centre of mass */
    double v[3];
    double I[6];             /* inertia about x: xx, yy, zz, xy, xz, yz */
    double w[3];             /* I^-1 L */
} tr_aggregate;

typedef struct tr_scene tr_scene;

/* Creates a scene from *d (copied, env_bounds included).  Allocates all
 * device buffers at their capacities.  TR_E_INVAL for bad sizes or options
 * (mu_r negative, restitution outside [0, 1], v_imp not finite), TR_E_NOMEM, TR_E_DEVICE.
 * TR_E_CAPACITY when n_envs x cap_particles exceeds 2^26 (the solver addresses
 * the particles' 32 B velocity records with 31-bit byte offsets) or
 * n_envs x cap_contacts reaches 2^31. */
int create_scene(const tr_scene_desc* d, tr_scene** out);

/* Releases every buffer of the scene.  NULL is accepted. */
int destroy_scene(tr_scene* s);

/* Appends n spheres to env (Eq. eqmotb bodies with m = rho 4/3 pi r^3,
 * I = 2/5 m r^2).  pos: 3n, vel: 3n or NULL (zero), radius: n, density: n or
 * NULL (material.rho).  Ids are consecutive; the first is written to
 * *first_id.  TR_E_CAPACITY when the env would exceed cap_particles,
 * TR_E_NONFINITE for NaN/Inf, TR_E_INVAL for radius <= 0. Clears the
 * warm-start cache. */
int add_particles(tr_scene* s, int32_t env, int64_t n, const double* pos, const double* vel,
                  const double* radius, const double* density, int64_t* first_id);

/* Replaces the env's kinematic bodies (equipment B and resting terrain C,
 * Eq. eqmotb's boundary terms) with b[0..n-1].  Shapes and heights are
 * copied. */
int set_kinematic_bodies(tr_scene* s, int32_t env, int32_t n, const tr_body_desc* b);

/* Attaches the active-zone predictor tool *t to the body with id body_id of
 * env (replacing a previous tool of that body; NULL removes it).  The tool
 * stays with the body id across set_kinematic_bodies.  TR_E_INVAL for an
 * unknown env or body, n_wedges outside 1..TR_MAX_WEDGES, fill outside
 * [0, 1], phi outside (0, pi/2), a negative heap, zero-length edge or zero
 * normals; TR_E_CAPACITY when the env would have more than 4 zones. */
int set_tool(tr_scene* s, int32_t env, int32_t body_id, const tr_tool_desc* t);

/* The wedges the last step predicted for the tool of body body_id of env:
 * counts[w] half-spaces (0: an empty wedge, e.g. the edge above the surface
 * or a slow deformer) in planes[w*20 .. w*20 + 4 counts[w]) as (n, d), world
 * frame, inside iff n . x <= d.  *n_wedges receives the tool's wedge count;
 * cap is the room in counts (and planes / 20).  TR_E_STATE before the
 * first step after a change; TR_E_INVAL when the body has no tool. */
int get_zone_wedges(tr_scene* s, int32_t env, int32_t body_id, int32_t cap, double* planes, int32_t* counts,
                    int32_t* n_wedges);

/* Coarse-grained fields of env's particles (their state after the last
 * step) on grid g, Eq. cg_velocity: rho = sum_a m_a zeta(x - x_a), mom =
 * sum_a m_a v_a zeta(x - x_a), u = mom / rho (0 where rho = 0).
 * TR_CG_HEAVISIDE: zeta = 1/l0^3 in the particle's own voxel (mass preserved
 * exactly; particles outside the grid are skipped); TR_CG_GAUSS: zeta(y) =
 * (sqrt(2 pi) R)^-3 exp(-|y|^2 / 2R^2) at the voxel centres, cut at |y| > 3R.
 * rho (1 per voxel), mom and u (3 per voxel; u may be NULL) are device
 * arrays of the caller, written on the scene's stream (sums in FP64 with
 * atomics: the order of the additions is not fixed).  TR_E_INVAL for a bad
 * env, grid, kernel or R. */
int coarse_grain(tr_scene* s, int32_t env, const tr_voxel_grid* g, int32_t kernel, double R, double* rho,
                 double* mom, double* u);

/* Conversion between resting solid and fluidized mass on a voxel grid
 * (the passage on converting overlapping soil).  Per voxel, device arrays of
 * the caller: phi (solid occupancy in [0, 1]), wc (compaction: solid mass
 * wc phi rho_b l0^3), mf (fluidized mass, kg); every column is full below its
 * surface voxel.  Wedges: n_wedges wedges of counts[w] half-spaces each
 * (host arrays; planes holds 5 x 4 doubles per wedge, inside iff
 * n . x <= d), or, with planes NULL, the wedges the last step predicted for
 * every tool of env (caller wedges are copied to the device, which
 * synchronises the stream).  A total pointer, when not NULL, receives the
 * converted mass (the call then synchronises the stream); with predicted
 * wedges and NULL totals the call only enqueues kernels on the scene's
 * stream (no memset: it may be captured in a graph once the scene's one
 * double of scratch exists, after a first call).  TR_E_INVAL for a bad env, grid,
 * density or wedge count (at most 128 caller wedges, 8 tools), TR_E_STATE for
 * predicted wedges before a step. */

/* Eq. surface per column: h = z' + (phi' - 1/2) l0 of the top-most voxel with
 * solid (the grid's bottom for an empty column) into h (nx ny device doubles,
 * index j nx + i; may be NULL).  With body_id >= 0 the heights also become
 * the FP32 heights of that body's first heightfield in env, whose grid points
 * must be the column centres (nx, ny, l0 equal; origin + l0/2); the contacts
 * and the zone predictor of later steps use them.  TR_E_INVAL otherwise. */
int terrain_from_voxels(tr_scene* s, int32_t env, int32_t body_id, const tr_voxel_grid* g, const double* phi,
                        double* h);

/* Cut: for the vertical line through each column's centre, every wedge it
 * crosses bounds z from below; the column's surface drops to the lowest such
 * bound and the solid above it becomes fluidized mass in the voxel that held
 * it. */
int convert_cut(tr_scene* s, int32_t env, const tr_voxel_grid* g, double rho_b, int32_t n_wedges,
                const int32_t* counts, const double* planes, double* phi, const double* wc, double* mf,
                double* liberated);

/* Deposit: fluidized mass in a voxel with no particles (rho_p == 0, e.g. the
 * coarse-grained density) whose centre is outside every wedge falls to its
 * column's surface and becomes solid of compaction w_dep > 0, raising it; a
 * voxel being filled takes the mass-weighted compaction; mass that finds the
 * column full stays fluid where it was. */
int convert_deposit(tr_scene* s, int32_t env, const tr_voxel_grid* g, double rho_b, double w_dep, int32_t n_wedges,
                    const int32_t* counts, const double* planes, const double* rho_p, double* phi, double* wc,
                    double* mf, double* deposited);

/* Growth of env's particles from the fluidized mass mf of the voxel holding
 * each centre (Eq. eqmotmb): over dt a particle of mass m and diameter d
 * gains at most 3 m d'_max dt / d, not past the diameter d_max; where a
 * voxel's fluid is less than the sum of its particles' bounds, each gains its
 * bound times their ratio.  Radii, masses and inertias change in place
 * (radii in FP32); mf is charged exactly the mass the new radii hold.  d_max
 * may not exceed the env's largest diameter at its last table build (the
 * cell size of detection).  work: 2 nx ny nz device doubles of scratch.
 * *grown, when not NULL, receives the mass grown (the call then
 * synchronises the stream).  TR_E_INVAL for a bad env, grid or parameter,
 * TR_E_STATE before the first step since the bodies or particles changed. */
int grow_particles(tr_scene* s, int32_t env, const tr_voxel_grid* g, double dt, double dprime_max, double d_max,
                   double* mf, double* work, double* grown);

/* Forming new particles in env from the fluidized mass inside the zones: a
 * voxel whose centre is inside a wedge, whose fluid mf is at least the mass
 * of a particle of diameter d_min (the material density), and whose particle
 * volume fraction rho_p / rho (rho_p: the coarse-grained particle mass
 * density) stays at or below phi_max with one more particle, forms one
 * particle at its centre with the voxel velocity u (3 per voxel); its
 * diameter holds all the voxel's fluid, capped at d_max; the fluid is charged
 * exactly the mass the FP32 radius holds.  The particles are appended in
 * increasing voxel order as add_particles does (the next step rebuilds the
 * tables); *n_formed receives their count.  Wedges as for convert_cut.  No
 * change and TR_E_CAPACITY when more than max_new particles, or more than the
 * env can hold, would form; TR_E_INVAL for bad arguments. */
int form_particles(tr_scene* s, int32_t env, const tr_voxel_grid* g, double d_min, double d_max, double phi_max,
                   int32_t n_wedges, const int32_t* counts, const double* planes, const double* rho_p,
                   const double* u, double* mf, int64_t max_new, int64_t* n_formed);

/* Removes the listed particles (ids of env, each once) from the scene; the
 * env's remaining particles keep their order and are renumbered from the
 * env's first id without gaps.  Clears the warm-start cache; the next step
 * rebuilds the tables.  TR_E_INVAL for an id outside env or repeated. */
int remove_particles(tr_scene* s, int32_t env, int64_t n, const int64_t* ids);

/* Particles of env at rest outside the zones turn back into soil: a particle
 * whose speed is below v_rest and whose centre is inside the grid and
 * outside every wedge adds its mass to the fluidized mass mf (device, one per
 * voxel) of its voxel and is removed as by remove_particles (a later
 * convert_deposit, given particle densities without it, makes the fluid
 * solid).  Wedges as for convert_cut.  *n_settled and *mass (both may be
 * NULL) receive the number of particles and their mass.  TR_E_STATE before
 * the first step since the particles or bodies changed. */
int settle_particles(tr_scene* s, int32_t env, const tr_voxel_grid* g, double v_rest, int32_t n_wedges,
                     const int32_t* counts, const double* planes, double* mf, int64_t* n_settled, double* mass);

/* One step of conserved advection of the fluidized mass per voxel (kg),
 * Eq. advection without sources: each interior face carries
 * phi = dt u_f mf_donor / l0 from the upwind voxel, u_f the mean of the two
 * voxels' normal velocities; the grid's outer faces are closed, so the total
 * is conserved to rounding.  u (3 per voxel), mf_in, mf_out: device arrays
 * (mf_out must not alias mf_in).  *cfl, when cfl is not NULL, receives the
 * largest |u_f| dt / l0 (positivity needs <= 1; the call then synchronises
 * the stream to read it; with NULL it only enqueues the step).  The scene
 * keeps a small array of per-block maxima, allocated on the first call and
 * when a larger grid needs more blocks.  TR_E_INVAL for a bad grid or
 * pointers, TR_E_NOMEM. */
int advect_fluid(tr_scene* s, const tr_voxel_grid* g, double dt, const double* u, const double* mf_in,
                 double* mf_out, double* cfl);

/* Advances every env by n_steps steps.  Enqueues the steps on the scene's
 * stream, then waits for them and reads back the failure flags of every step
 * of the call (a few bytes); with stats not NULL it also writes one
 * tr_step_stats per env (of the last step).  TR_E_CAPACITY when contacts,
 * colours or cells overflowed (or a multi-block solve timed out) in any step
 * of the call: that step is abandoned before any particle state changes, the
 * steps after it still run, and the warm-start cache is cleared.  n_steps = 0
 * with stats NULL does nothing. */
int step(tr_scene* s, int32_t n_steps, tr_step_stats* stats);

/* Mean contact force and torque (about the body's position at the start of
 * the step) exerted by the particles on body body_id of env during the last
 * step: impulse / dt, summed in FP64 (the force from which the digging
 * resistance follows, section "Microscopic model").  Synchronises. */
int get_contact_forces(tr_scene* s, int32_t env, int32_t body_id, double force[3], double torque[3]);

/* Aggregate bodies of env's active zones after the last step, one per body
 * with a zone, in body order.  Writes min(cap, count) records and the count
 * to *n_out.  Synchronises. */
int get_aggregates(tr_scene* s, int32_t env, int32_t cap, tr_aggregate* out, int32_t* n_out);

/* Bulk properties of the aggregate body of the macroscale model (section
 * "Macroscale model", Eqs. aggregateNormal and aggregateTangent). */
typedef struct tr_macro_params {
    double E_b;      /* bulk modulus [Pa], > 0 */
    double c_b;      /* bulk cohesion [Pa], >= 0 */
    double mu_ab;    /* friction at the equipment interface AB, >= 0 */
    double mu_ac;    /* friction in the failure surface AC (tan phi_b), >= 0 */
    double cas_ab;   /* aggregate stiffness multiplier c_as at AB, > 0 */
    double cas_ac;   /* aggregate stiffness multiplier c_as at AC, > 0 */
} tr_macro_params;

/* An equipment body that moves under the macroscale step (Eq. mdb:eqEq)
 * instead of being kinematic: its mass and body-frame inertia, and the drive
 * that holds and actuates it, one row per world axis (linear, then angular)
 * pulling its velocity toward the target with compliance gamma_drive and an
 * impulse limit of f_max dt (t_max dt).  Gravity acts on it; the penetration
 * resistance and its contacts with the terrain are not included. */
typedef struct tr_macro_equipment {
    int32_t body_id;         /* id of the body (tr_body_desc.id) */
    int32_t pad;
    double mass;             /* > 0 */
    double inertia[6];       /* body frame: xx, yy, zz, xy, xz, yz (positive definite) */
    double v_target[3];      /* drive target, world frame [m/s] */
    double w_target[3];      /* [rad/s] */
    double f_max;            /* drive force limit per axis [N], >= 0 */
    double t_max;            /* drive torque limit per axis [N m], >= 0 */
    double gamma_drive;      /* drive compliance (velocity per impulse), > 0 */
} tr_macro_equipment;

/* One zone's macroscale step.  Points and impulses of interface AB sit in
 * entries 0..3, those of AC in 4..7; n_points[q] of each are used. */
typedef struct tr_macro_result {
    int32_t zone;            /* id of the body that owns the zone */
    int32_t n_points[2];     /* reduced points of AB, AC (at most 4 each) */
    int32_t sweeps;          /* iterations of the solve: Newton steps plus Gauss-Seidel sweeps */
    int64_t n_cand[2];       /* candidate contacts of AB, AC */
    double area[2];          /* A_AB, A_AC: sum of the candidates' pi r^2 */
    double gamma[2];         /* regularisation of AB, AC (velocity per impulse) */
    double p[8][3];          /* points */
    double n[8][3];          /* normals, from B (or the terrain C) into A */
    int64_t src[8];          /* env-local index (id - env's first id) of each point's particle */
    double lam[8][4];        /* impulses on A: normal, tangential xyz */
    double M, x[3], v0[3], w0[3];  /* the aggregate before the step */
    double v[3], w[3];       /* its velocity after the step */
    double force[3];         /* mean force of A on B (impulse / dt) */
    double torque[3];        /* its torque about B's position */
    double v_b[3], w_b[3];   /* B's velocity after the step (its own when kinematic) */
    double lam_drive[6];     /* drive impulses on B: linear xyz, angular xyz (0 when kinematic) */
} tr_macro_result;

/* The macroscale step (section "Macroscale model") of every zone of env whose
 * body has at least two half-spaces (half-space 0 the separation plate,
 * half-space 1 the failure plane) and holds particles, for the current
 * particle state and body poses: the zone's aggregate body (Eqs.
 * aggregate_mass .. aggregate_rot_vel) advanced one step under Eq. mdb:eqAgg
 * with the constraints of Eqs. aggregateNormal and aggregateTangent at its
 * interface to the equipment (particles touching the body's shapes) and to
 * the failure surface (particles within their radius of the failure plane),
 * each interface reduced to the four candidates extreme along its in-plane
 * axes.  The impulses are the fixed point of the interface rows' projected
 * Gauss-Seidel (normal row, then the tangential disk, per point), found by a
 * damped Newton iteration on the aggregate's six velocities with each point's
 * impulse in closed form and finished by Gauss-Seidel sweeps until no impulse
 * changes by more than 1e-15 of the largest.  The bodies named in eq[0 ..
 * n_eq - 1] (eq may be NULL when n_eq = 0) move with the aggregate under Eq.
 * mdb:eqEq (their AB rows act on both bodies, their drive rows follow the
 * points); the other bodies are kinematic.  A particle belongs to the first body, in body order, whose
 * half-spaces all contain it.  The particle state is not changed.  Writes
 * min(cap, count) results in body order and the count to *n_out.  The scene
 * allocates a small device table on the first call.  Synchronises.
 * TR_E_INVAL for bad arguments or parameters (an equipment entry naming no
 * body of env, twice the same body, a mass, inertia or compliance that is not
 * positive, negative limits), TR_E_CAPACITY for more than 8 bodies with
 * half-spaces in env, TR_E_NOMEM. */
int macro_step(tr_scene* s, int32_t env, const tr_macro_params* mp, int32_t n_eq, const tr_macro_equipment* eq,
               int32_t cap, tr_macro_result* out, int32_t* n_out);

/* Message of the last error on this scene ("" when none); valid until the
 * next call on the scene. */
const char* get_last_error(tr_scene* s);

/* Canonical contact list of env from the last step, sorted by key (a pair of
 * ids a < b has key a<<32 | b; a boundary contact of particle a with the
 * env's shape s has key a<<32 | 0x80000000 | s), with the impulses
 * (lambda_n, lambda_t xyz) of the step.  Writes min(cap, count) entries and
 * the count to *n.  impulse4 may be NULL.  Synchronises. */
int get_contacts(tr_scene* s, int32_t env, int64_t cap, uint64_t* keys, float* impulse4, int64_t* n);

/* Colour of each contact of env's last step, in the order of get_contacts:
 * the deterministic graph colouring whose colour classes the PGS sweeps visit
 * in increasing order (no two contacts of a colour share a sphere; Jones-
 * Plassmann with the priority splitmix64(key), ties by key, each contact
 * taking the smallest colour its already coloured neighbours leave free).
 * Writes min(cap, count) entries and the count to *n.  Synchronises. */
int get_colours(tr_scene* s, int32_t env, int64_t cap, int32_t* colours, int64_t* n);

/* Rolling-resistance impulses of the last step (Eq. signCoul3), in the order
 * of get_contacts: 3 floats per contact, the torque impulse on body 2 (the
 * higher id; -impulse on body 1), zero when mu_r == 0.  Writes min(cap,
 * count) entries and the count to *n.  Synchronises. */
int get_rolling_impulses(tr_scene* s, int32_t env, int64_t cap, float* impulse3, int64_t* n);

/* Particle state of env in id order (any output may be NULL): pos, vel,
 * angvel 3n each, radius n.  *n receives the env's particle count.
 * Synchronises. */
int get_particles(tr_scene* s, int32_t env, double* pos, double* vel, double* angvel, double* radius,
                  int64_t* n);

/* Overwrites the state of env's particles in id order (NULL leaves a field
 * unchanged) and clears the warm-start cache. */
int set_particles(tr_scene* s, int32_t env, const double* pos, const double* vel, const double* angvel);

/* Loads the learned warm-start network (12 -> 64 -> 64 -> 3, SiLU): n = 5199
 * floats laid out W1[64][12], b1[64], W2[64][64], b2[64], W3[3][64], b3[3],
 * in_scale[12] (inputs are multiplied by in_scale).  With warm_start
 * TR_WARM_LEARNED, each step predicts lambda^0 in residual form (the three
 * outputs are added to the previous-step impulse in the contact frame, inputs
 * 3-5, before scaling by m_eff g dt), projects it onto the bounds,
 * and keeps it only when it is finite and its first-sweep residual does not
 * exceed the previous-step start's (else PREV, or COLD without a cache;
 * step_stats.fallback_used).  Without weights LEARNED behaves as PREV.
 * TR_E_INVAL when n differs from 5199. */
int set_mlp_weights(tr_scene* s, const float* weights, int64_t n);

/* Precision of the learned start's network inside step: nonzero (default)
 * runs it in BF16 on the matrix cores (FP32 accumulate), zero in FP32. */
int set_learned_precision(tr_scene* s, int32_t use_bf16);

/* Training samples of env's last step in canonical contact order: the 12
 * learned-start inputs (feat, 12 per contact: overlap / mean radius, normal
 * and tangential relative speed / (g dt), previous-step impulses in the
 * contact frame / (m_eff g dt), the two depths below the column top / mean
 * radius, the two radii / r_ref, is_boundary, is_persistent) and the step's
 * final impulses in the same frame / (m_eff g dt) (label, 3 per contact).
 * Writes min(cap, count) entries and the count to *n.  Synchronises.
 * TR_E_STATE when the last step wrote no features: a step writes them when
 * it runs the learned start (LEARNED with weights) or capture is on. */
int get_learn_samples(tr_scene* s, int32_t env, int64_t cap, float* feat, float* label, int64_t* n);

/* Nonzero: every following step writes the learned start's inputs of its
 * contacts for get_learn_samples (80 B per contact; off by default, when a
 * step writes them only for the learned start it runs). */
int set_learn_capture(tr_scene* s, int32_t on);

/* ---- learned-start network on device buffers (training support) ----
 * weights: the set_mlp_weights layout (W1, b1, W2, b2, W3, b3, in_scale), in
 * device memory; feat: B x 12, label and out: B x 3, all FP32 device memory,
 * enqueued on `stream` (hipStream_t or NULL).  Asynchronous. */

/* out = network(feat): use_bf16 selects the MFMA BF16 kernel, else FP32. */
int mlp_forward(const float* weights, const float* feat, int64_t B, float* out, int32_t use_bf16, void* stream);

/* Floats of device scratch mlp_loss_grad needs for a batch of B. */
int64_t mlp_grad_scratch_floats(int64_t B);

/* loss = 0.5 mean_b ||network(feat_b) - label_b||^2 (written to *loss, device)
 * and its gradient w.r.t. W1, b1, W2, b2, W3, b3 (grad: 5187 floats, device),
 * in FP32.  TR_E_CAPACITY when scratch_floats < mlp_grad_scratch_floats(B). */
int mlp_loss_grad(const float* weights, const float* feat, const float* label, int64_t B, float* grad, float* loss,
                  float* scratch, int64_t scratch_floats, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * loss and gradient as mlp_loss_grad, with the per-block gradient partials in
 * a fixed device array the library holds on each GPU it runs on (until the
 * process ends) instead of a caller workspace.  Calls no allocating routine.
 * B is limited to TR_MLP_NOALLOC_MAX_BATCH: TR_E_CAPACITY
 * above it, TR_E_INVAL for NULL pointers or B <= 0, TR_E_DEVICE when the
 * array cannot be located on the current device.  Every call on one GPU uses
 * that GPU's one array: calls that overlap on one GPU (different streams or
 * threads without ordering between them) race and give wrong gradients.
 * Asynchronous on `stream`. */
#define TR_MLP_NOALLOC_MAX_BATCH 8192
int mlp_loss_grad_noalloc(const float* weights, const float* feat, const float* label, int64_t B, float* grad,
                          float* loss, void* stream);

/* One Adam step (bias-corrected, step count t >= 1) on the 5187 trainable
 * weights in place; m and v are the moment buffers (device, 5187 each). */
int mlp_adam_step(float* weights, const float* grad, float* m, float* v, float lr, float beta1, float beta2, float eps,
                  int32_t t, void* stream);

/* Schedule of the PGS solve (Sec. numerical solver: the sweeps of the
 * projected Gauss-Seidel method over the graph-coloured contacts).  It changes
 * how the work is spread over the GPU, not the arithmetic: with tol == 0 every
 * schedule gives the same impulses.  With tol > 0 the stopping test of
 * TR_PGS_GROUPED is taken per group of envs (one group per env when the scene
 * has at most 8 envs), that of TR_PGS_PER_ENV per env.
 *   TR_PGS_GROUPED: envs in 8 groups, one per XCD; each group is solved by
 *     blocks_per_xcd blocks that meet at a barrier after every colour.
 *   TR_PGS_PER_ENV: each env is solved by one block or by a cluster of
 *     blocks of one XCD.  A block solves a set of envs at once with their
 *     bodies in its LDS (lds_particles slots; an env that does not fit keeps
 *     its first slots there and the rest in global memory); blocks run their
 *     tasks one after another.  cluster_particles 0: the plan of a cost model
 *     measured on MI355X (envs that fit LDS packed into sets, somewhat larger
 *     ones solved alone by one block, the largest by clusters sized to finish
 *     together; the size limit and the cluster sizes searched for the
 *     smallest predicted time).  cluster_particles T > 0: envs of more than T
 *     particles get clusters of ceil(n / T) blocks, the others sets of at
 *     most T particles.  TR_CLUSTER_NONE: no env takes more than one block
 *     (sets of at most lds_particles particles, larger envs alone).
 *   TR_PGS_SPREAD: one env (n_envs must be 1) spread over all 8 XCDs: its
 *     sorted spheres in eighths (compact regions of the Morton order), each
 *     contact solved by the XCD group of its second sphere with
 *     blocks_per_xcd blocks, all groups meeting after every colour; every
 *     body store is written through to be seen across XCDs. */
#define TR_PGS_GROUPED 0
#define TR_PGS_PER_ENV 1
#define TR_PGS_SPREAD 2
#define TR_CLUSTER_NONE (-1)
typedef struct tr_solver_config {
    int32_t mode;              /* TR_PGS_GROUPED, TR_PGS_PER_ENV or TR_PGS_SPREAD */
    int32_t blocks_per_xcd;    /* grouped: >= 1, clamped to the resident limit */
    int32_t lds_particles;     /* per-env: >= 0, clamped to what LDS holds */
    int32_t cluster_particles; /* per-env: T, 0 for the automatic choice, or TR_CLUSTER_NONE */
    int32_t dataflow;          /* 1: inside a multi-block solve the colour order of each sphere's
                                  updates is kept by per-sphere update counters instead of a
                                  barrier after every colour (same results); 0: barriers */
} tr_solver_config;

/* Set / read the schedule.  Takes effect at the next step; TR_E_INVAL on a bad
 * field.  The default is TR_PGS_GROUPED with 32 blocks per XCD for up to 8
 * envs, else TR_PGS_PER_ENV with the LDS limit and automatic clusters. */
int set_solver_config(tr_scene* s, const tr_solver_config* cfg);
int get_solver_config(tr_scene* s, tr_solver_config* cfg);

/* Step graphs (on by default): from the second step after the scene or its
 * tables last changed, each step replays a captured HIP graph of its launches
 * instead of launching them one by one.  Results are identical either way;
 * enable = 0 launches every step eagerly.  A replayed step is timed only as a
 * whole (get_phase_times). */
int set_step_graphs(tr_scene* s, int32_t enable);

/* Autotuner of the PGS schedule.  Times candidate schedules (grouped with 64,
 * 32, 16 or 8 blocks per XCD; spread with 32 for a single env; per-env with
 * automatic, 8192- and 16384-sphere clusters; per-env without LDS; grouped is
 * left out when a residual
 * tolerance is set with more than 8 envs, where it would let envs share their
 * stopping test) over `steps` eager steps each, every
 * candidate from the scene's current state (saved and restored, so the scene
 * is left as it was), and keeps the fastest.  With cache_path, a matching
 * entry (device architecture, log2 of envs, log2 of spheres) is applied
 * without timing, and a new result is appended as one JSON object per line.
 * chosen and best_ms (ms per step; -1 from the cache) may be NULL. */
int autotune(tr_scene* s, int32_t steps, const char* cache_path, tr_solver_config* chosen, float* best_ms);

/* Warm start of the following steps (TR_WARM_COLD / PREV / LEARNED). */
int set_warm_start(tr_scene* s, int32_t mode);

/* Snapshot of the scene's state: particle state and order, the previous-step
 * contact cache, body poses and flags.  save_state with buf == NULL (or cap
 * too small: TR_E_CAPACITY) writes only *size.  load_state restores a
 * snapshot into a scene built with the same envs, particle counts, bodies and
 * capacities (else TR_E_STATE); the scene then steps exactly as the saved one
 * would.  Both synchronise. */
int save_state(tr_scene* s, void* buf, int64_t cap, int64_t* size);
int load_state(tr_scene* s, const void* buf, int64_t size);

/* Device time (ms, from HIP events on the scene's stream) of the last step's
 * phases: [0] detection+ordering, [1] rows+colouring+warm start, [2] PGS,
 * [3] integration+forces+aggregates, [4] whole step.  When the last step was
 * a step-graph replay, [0]-[3] are NaN (the replay is one launch, timed as a
 * whole).  Writes min(cap, 5) values.  Synchronises. */
int get_phase_times(tr_scene* s, float* ms, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif
