/*
 * oracle.h -- plain FP64 CPU reference of one time step of the agitated-soil
 * (coarse-particle) system of Servin, Berglund & Nystedt, "A multiscale model
 * of terrain dynamics for real-time earthmoving simulation" (arXiv 2011.00459).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no header, helper or constant with the
 * GPU library: every formula here is written out independently from the paper.
 *
 * What it computes (section "Mesoscale model", Eq. eqmotb; Algorithm 1, the
 * collision-detection, aggregate and mesoscale-PGS lines):
 *   1. contact detection between spheres and against kinematic boundaries,
 *   2. canonical contact order and warm-start matching,
 *   3. Hertz-mapped SPOOK rows of the frictional-cohesive contact law
 *      (Eqs. signCoul1-2, the Hertz mapping and the SPOOK MCP of section
 *      "Contacting rigid multibodies"),
 *   4. a greedy colouring in hashed-key priority order,
 *   5. projected Gauss-Seidel sweeps in colour order,
 *   6. symplectic position update x += dt v,
 *   7. contact force/torque on each kinematic body,
 *   8. aggregate-body mass/inertia/momentum of each active zone
 *      (Eqs. aggregate_mass .. aggregate_rot_vel), in FP64.
 */
#ifndef TERRAIN_ORACLE_H
#define TERRAIN_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PLANE = 0, ORC_BOX = 1, ORC_HFIELD = 2 };
enum { ORC_COLD = 0, ORC_PREV = 1, ORC_LEARNED = 2 };
enum { ORC_BRUTE = 0, ORC_CELLS = 1 };

typedef struct orc_material {
    double rho;         /* particle density [kg/m^3] (used when rho array is NULL) */
    double mu_t;        /* Coulomb friction coefficient */
    double mu_r;        /* rolling resistance coefficient (Eq. signCoul3), >= 0 */
    double c_p;         /* particle cohesion [Pa] */
    double E;           /* Young's modulus [Pa] */
    double nu;          /* Poisson's ratio */
    double restitution; /* Newton restitution e in [0, 1] of the impact stage */
    double tau_n;       /* normal damping time [s]; <= 0 means 2 dt */
    double gamma_t;     /* tangential regularisation (0 = ideal Coulomb) */
    double kappa_c;     /* cohesive range as a fraction of the summed radii */
    double kappa_min;   /* floor of the overlap used in the compliance */
    double v_imp;       /* impact threshold [m/s]: a contact approaching faster is an
                           impact; <= 0 disables the impact stage */
} orc_material;

typedef struct orc_params {
    double dt;
    double g[3];
    double grid_lo[3];   /* grid bounds of the env: origin and far corner of the column grid */
    double grid_hi[3];   /* used by the learned-start depth feature */
    double r_ref;        /* nominal particle radius (learned-start features) */
    int32_t max_sweeps;
    double tol;          /* 0: fixed number of sweeps */
    int32_t warm;        /* ORC_COLD / ORC_PREV / ORC_LEARNED */
    int32_t detect;      /* ORC_BRUTE or ORC_CELLS */
    orc_material m;
    int32_t ntools;      /* tools whose predicted wedges replace their bodies' zones */
    const struct orc_tool* tools;
} orc_params;

/* Kinematic body: pose, velocities and an optional active zone given as up to
 * eight half-spaces in the body frame (inside iff n.y <= d for all planes). */
typedef struct orc_body {
    double pos[3];
    double quat[4];      /* (w, x, y, z), unit */
    double linvel[3];
    double angvel[3];
    int32_t nplanes;
    double planes[8][4];
} orc_body;

/* Boundary shape attached to a body.
 *   PLANE : surface n.y = d in the body frame, particles on the n side.
 *   BOX   : oriented box, half extents half[], centre off[] in the body frame.
 *   HFIELD: heights h[j*nx+i] at (ox + i l0, oy + j l0), world frame, static.
 */
typedef struct orc_shape {
    int32_t type;
    int32_t body;
    double n[3];
    double d;
    double half[3];
    double off[3];
    int32_t nx, ny;
    double ox, oy, l0;
    const float* h;
} orc_shape;

/* Digging tool or soil deformer of a body, for the active-zone predictor
 * (Eq. failure_plane with the lateral wedges, the fill-dependent secondary
 * separation plate and the deformers' speed gate).  Geometry in the body
 * frame.  The terrain surface is the env's first heightfield shape. */
typedef struct orc_tool {
    int32_t body;          /* index of the tool's body */
    int32_t n_wedges;      /* lateral wedges along the cutting edge, 1..16 */
    double edge0[3];       /* cutting edge end points */
    double edge1[3];
    double n_c[3];         /* normal of the primary separation plate, towards the zone */
    double n_tc[3];        /* normal of the face from cutting edge to top edge (= n_c for a blade) */
    double fill;           /* fill ratio of the inner shape, [0, 1] */
    double phi;            /* soil internal friction angle [rad] */
    double heap;           /* zone height above the point where the failure plane meets the surface [m] */
    double v_min;          /* deformer: a zone only while the edge speed exceeds v_min (<= 0: always) */
} orc_tool;

#define ORC_MAX_WEDGES 16

/* One wedge of a predicted zone: n half-spaces (world frame, inside iff
 * planes[k][0..2] . x <= planes[k][3]); n = 0 for an empty wedge. */
typedef struct orc_wedge {
    int32_t n;
    int32_t pad;
    double planes[5][4];
} orc_wedge;

/* Wedges of one tool at the body's current pose, on the heightfield
 * `terrain` (NULL: every wedge empty).  Writes t->n_wedges wedges; returns
 * their count, or -1 for a bad tool. */
int32_t orc_predict_wedges(const orc_tool* t, const orc_body* bodies, const orc_shape* terrain, orc_wedge* out);

/* Voxel grid of the mesoscale fields: voxel (i, j, k) spans
 * origin + l0 [i, i+1) x [j, j+1) x [k, k+1), index (k ny + j) nx + i. */
typedef struct orc_voxel_grid {
    double origin[3];
    double l0;
    int32_t nx, ny, nz;
    int32_t pad;
} orc_voxel_grid;

enum { ORC_CG_HEAVISIDE = 0, ORC_CG_GAUSS = 1 };

/* Coarse-grained mass and momentum densities of particles (x, v: 3n, m: n)
 * on the voxel grid (Eq. cg_velocity: rho = sum m zeta(x - x_a), p = sum m v
 * zeta(x - x_a)).  HEAVISIDE: zeta = 1/l0^3 inside a particle's voxel (mass
 * preserved exactly); GAUSS: zeta(y) = (sqrt(2 pi) R)^-3 exp(-|y|^2 / 2R^2)
 * at the voxel centres, cut at |y| > 3R.  rho: one per voxel, mom: 3 per
 * voxel, u = p / rho (0 where rho = 0): 3 per voxel (u may be NULL).
 * Particles outside the grid are skipped (HEAVISIDE).  Returns 0, or -1 for a
 * bad grid or kernel. */
int32_t orc_coarse_grain(int64_t n, const double* x, const double* v, const double* m, const orc_voxel_grid* g,
                         int32_t kernel, double R, double* rho, double* mom, double* u);

/* One step of conserved advection of the fluidized mass per voxel mf (kg)
 * with the voxel velocities u (3 per voxel), Eq. advection without sources:
 * donor-cell fluxes through every interior face, phi = dt u_f mf_donor / l0
 * with u_f the mean of the two voxels' normal velocities and the donor the
 * upwind voxel; the grid's outer faces are closed.  mf is updated in place;
 * the largest |u_f| dt / l0 (positivity needs <= 1) is returned. */
double orc_advect(const orc_voxel_grid* g, double dt, const double* u, double* mf);

/* Conversion between resting solid and fluidized mass on the voxel grid.
 * Per voxel: phi (solid occupancy in [0, 1]), wc (compaction: the solid mass
 * is wc phi rho_b l0^3), mf (fluidized mass, kg).  Every column is full
 * below its surface voxel, empty above it. */

/* Eq. surface: h = z' + (phi' - 1/2) l0 for the top-most voxel with solid
 * (z' its centre), origin[2] for an empty column; h: nx ny values, index
 * j nx + i.  Returns 0, or -1 for a bad grid. */
int32_t orc_surface_heights(const orc_voxel_grid* g, const double* phi, double* h);

/* Solid of the columns under active-zone wedges is liberated down to the
 * zone's bottom: for the vertical line through a column's centre, each wedge
 * it crosses bounds z from below (the failure plane, a plate leaning over the
 * column); the column's new surface is the lowest such bound where it is
 * below the surface.  The liberated solid becomes fluidized mass in the
 * voxel that held it.  Returns the liberated mass, or -1 for a bad grid. */
double orc_convert_cut(const orc_voxel_grid* g, double rho_b, int32_t n_wedges, const orc_wedge* wedges,
                       double* phi, const double* wc, double* mf);

/* Fluidized mass in a voxel that holds no particles (rho_p == 0) and whose
 * centre lies outside every wedge falls to its column's surface and becomes
 * solid of compaction w_dep (the loose state of soil that has flowed), raising
 * the surface; a voxel being filled gets the mass-weighted compaction; mass
 * that finds the column full stays fluid where it was.  Returns the deposited
 * mass, or -1 for a bad grid or w_dep. */
double orc_convert_deposit(const orc_voxel_grid* g, double rho_b, double w_dep, int32_t n_wedges,
                           const orc_wedge* wedges, const double* rho_p, double* phi, double* wc, double* mf);

/* Growth of particles from the fluidized mass of their voxel (Eq. eqmotmb
 * with the solid's share already turned into fluid): over dt a particle of
 * mass m and diameter d may gain at most 3 m d'_max dt / d, and no more than
 * takes it to the diameter d_max; where the voxel's fluid A falls short of
 * the sum C of these bounds, each gains its bound times A / C.  The fluid
 * pays for exactly what the particles gain.  x: 3n, r: n (updated), the
 * particles' density rho; particles outside the grid do not grow.  Returns
 * the mass grown, or -1 for a bad grid or parameter. */
double orc_grow_particles(int64_t n, const double* x, double* r, double rho, const orc_voxel_grid* g, double dt,
                          double dprime_max, double d_max, double* mf);

/* Forming new particles from fluidized mass inside the zones: a voxel whose
 * centre is inside a wedge, whose fluid mf is at least the mass of a
 * particle of diameter d_min (density rho), and whose particle volume
 * fraction rho_p / rho (rho_p the coarse-grained particle mass density)
 * leaves room for one more particle below phi_max, forms one particle of
 * diameter min(d_max, the diameter holding all its fluid) at its centre with
 * the voxel velocity u; the voxel's fluid pays its mass.  Writes up to cap
 * particles in increasing voxel order (voxel index, centre 3, velocity 3,
 * radius), returns their count (-1 for a bad grid or parameter). */
int64_t orc_form_particles(const orc_voxel_grid* g, double rho, double d_min, double d_max, double phi_max,
                           int32_t n_wedges, const orc_wedge* wedges, const double* rho_p, const double* u,
                           double* mf, int64_t cap, int64_t* voxel, double* x, double* v, double* r);

/* Particles at rest outside the zones turn back into resting soil: a particle
 * (x, v: 3n, mass m: n) with speed below v_rest whose centre is inside the
 * grid and outside every wedge gives its mass to the fluid of its voxel (the
 * deposit then makes it solid) and leaves the particle set: gone[a] = 1.
 * Returns the mass converted, or -1 for a bad grid or v_rest. */
double orc_settle_particles(int64_t n, const double* x, const double* v, const double* m, const orc_voxel_grid* g,
                            double v_rest, int32_t n_wedges, const orc_wedge* wedges, double* mf, int32_t* gone);

/* MLP 12 -> 64 -> 64 -> 3 with SiLU, weights row-major W[out][in]. */
typedef struct orc_mlp {
    const double* W1; const double* b1;  /* 64x12, 64 */
    const double* W2; const double* b2;  /* 64x64, 64 */
    const double* W3; const double* b3;  /* 3x64,  3  */
    double in_scale[12];                  /* feature normalisation (multiplied) */
    int32_t bf16;                         /* 1: BF16 inference (inputs, weight matrices and hidden
                                             layers rounded to bfloat16, biases and sums wide) */
} orc_mlp;

typedef struct orc_stats {
    int64_t contacts;
    int64_t pair_contacts;
    int32_t colours;
    int32_t sweeps;
    double residual;
    int32_t fallback_used;
    int32_t learned_used;
    double r1_first;     /* residual after the first sweep */
    double r1_trial[2];  /* learned start: first-sweep residual of the learned / previous-step start */
    int32_t impacts;       /* contacts treated as impacts (0: no impact stage this step) */
    int32_t impact_sweeps; /* sweeps of the impact stage */
} orc_stats;

typedef struct orc_aggregate {
    int32_t zone;        /* index of the body owning the zone */
    int64_t n_particles;
    double M;
    double x[3];
    double v[3];
    double I[6];         /* xx, yy, zz, xy, xz, yz about x */
    double w[3];
    double L[3];
} orc_aggregate;

/* ---- Macroscale model: aggregate constraints and the aggregate's solve ----
 * Section "Macroscale model": each active zone is aggregated into a rigid body
 * A (Eqs. aggregate_mass .. aggregate_rot_vel) whose motion obeys Eq.
 * mdb:eqAgg under the frictional-cohesive velocity constraints of Eqs.
 * aggregateNormal and aggregateTangent at its interfaces to the equipment B
 * (AB) and to the terrain's failure surface C (AC), each interface reduced to
 * four contact points.  Readings where the paper is silent: the zone's
 * half-spaces follow the wedge convention (plane 0 the separation plate,
 * plane 1 the failure plane); AB candidates are the zone's particles touching
 * the zone body's shapes, AC candidates the zone's particles within their
 * radius of the failure plane (projected onto it); each interface keeps its
 * candidates extreme along +-e1 and +-e2 of its plane; A is the sum of the
 * candidates' cross sections; gamma = L / (c_as E_b A dt^2), the compliance
 * of the bulk as a spring c_as E_b A / L regularising a velocity row over one
 * step, with L the cube root of the aggregate's solid volume (the printed
 * gamma_n = dt / (c_as E_b) lacks the geometric factor that makes it a
 * velocity per impulse); the equipment is kinematic and the
 * terrain static; the small MCP is solved to machine precision. */
typedef struct orc_macro_params {
    double E_b;       /* bulk modulus [Pa] */
    double c_b;       /* bulk cohesion [Pa] */
    double mu_ab;     /* friction at the equipment interface */
    double mu_ac;     /* friction in the failure surface (tan phi_b) */
    double cas_ab;    /* aggregate stiffness multiplier at the equipment */
    double cas_ac;    /* aggregate stiffness multiplier at the terrain */
} orc_macro_params;

/* A dynamic equipment body in the macroscale step (Eq. mdb:eqEq): its mass,
 * its inertia in the body frame, and the drive that holds and actuates it,
 * a velocity target per world axis reached through rows of compliance
 * gamma_drive with force (torque) limits f_max (t_max).  Bodies not named
 * here are kinematic. */
typedef struct orc_macro_equipment {
    int32_t body;             /* body index */
    double mass;
    double inertia[6];        /* body frame: xx, yy, zz, xy, xz, yz */
    double v_target[3], w_target[3];
    double f_max, t_max;      /* [N], [N m] per world axis */
    double gamma_drive;       /* velocity per impulse, > 0 */
} orc_macro_equipment;

typedef struct orc_macro_out {
    int32_t zone;             /* body index */
    int32_t n_points[2];      /* reduced points of AB, AC */
    int64_t n_cand[2];        /* candidates of AB, AC */
    double area[2];           /* A_AB, A_AC */
    double gamma[2];          /* regularisation of AB, AC (velocity per impulse) */
    double p[8][3];           /* points: AB in 0..3, AC in 4..7 */
    double n[8][3];           /* normals, from B or C into A */
    int64_t src[8];           /* particle index each point comes from */
    double lam[8][4];         /* impulses on A: normal, tangential xyz */
    double M, x[3], v0[3], w0[3];  /* the aggregate before the step */
    double v[3], w[3];        /* its velocity after the step */
    double force_b[3];        /* mean force of A on B (impulse / dt) */
    double torque_b[3];       /* its torque about B's position */
    int32_t sweeps;
    double v_b[3], w_b[3];    /* the equipment's velocity after the step (its own when kinematic) */
    double lam_drive[6];      /* drive impulses on B: linear xyz, angular xyz (0 when kinematic) */
} orc_macro_out;

/* Reduction of an interface's candidate points (n of them, 3 doubles each)
 * with plane normal nrm to at most four: the candidates extreme along +e1,
 * -e1, +e2, -e2 (e1 the normalised projection of the world axis least aligned
 * with nrm, e2 = nrm x e1), ties to the smaller index, a candidate chosen
 * twice kept once.  Writes the indices; returns their count. */
int32_t orc_reduce4(int64_t n, const double* pts, const double nrm[3], int64_t idx[4]);

/* One macroscale step of every zone (bodies with at least two half-spaces)
 * for the state (x, v, w) and the bodies' poses and velocities; the bodies
 * named in eq (neq of them, may be NULL when neq = 0) are dynamic, the others
 * kinematic.  Writes one orc_macro_out per zone; returns their count. */
int32_t orc_macro_step(const orc_params* P, int64_t n, const double* r, const double* rho,
                       const double* x, const double* v, const double* w,
                       int32_t nb, const orc_body* bodies, int32_t ns, const orc_shape* shapes,
                       const orc_macro_params* mp, int32_t neq, const orc_macro_equipment* eq,
                       int32_t cap, orc_macro_out* out);

/* Contact detection only.  Writes the canonical (sorted) keys and the overlap
 * of each contact.  Key of a pair (lower id a, higher id b) is a<<32 | b; key of
 * a boundary contact with shape s is id<<32 | 0x80000000 | s.
 * Returns the contact count, or -5 when it exceeds cap. */
int64_t orc_detect(const orc_params* P, int64_t n, const int64_t* id,
                   const double* x, const double* r,
                   int32_t nb, const orc_body* bodies,
                   int32_t ns, const orc_shape* shapes,
                   int64_t cap, uint64_t* keys, double* delta);

/* One full step.  x, v, w (3n each) and the body poses are updated in place.
 * prev_keys/prev_lam (4 per contact: lambda_n, lambda_t xyz) is the previous
 * step's cache (may be empty), prev_lr (3 per cached contact, may be NULL) its
 * rolling impulses.  Outputs: keys_out, lam_out (4 per contact), lr_out (3 per
 * contact: the rolling torque impulse on body 2, may be NULL), colour_out
 * (per contact), body_ft (6 per body: force, torque about the body origin, as
 * impulse/dt), agg (one per body that owns a zone, in body order, count
 * returned in *n_agg), resid (one per sweep done).
 * Returns the contact count or a negative error. */
int64_t orc_step(const orc_params* P,
                 int64_t n, const int64_t* id, const double* r, const double* rho,
                 double* x, double* v, double* w,
                 int32_t nb, orc_body* bodies,
                 int32_t ns, const orc_shape* shapes,
                 int64_t nprev, const uint64_t* prev_keys, const double* prev_lam, const double* prev_lr,
                 const orc_mlp* mlp,
                 int64_t cap, uint64_t* keys_out, double* lam_out, double* lr_out, int32_t* colour_out,
                 orc_stats* st, double* body_ft,
                 orc_aggregate* agg, int32_t* n_agg, double* resid);

/* Aggregate bodies (Eqs. aggregate_mass .. aggregate_rot_vel) of the zones
 * of the bodies that have one, for the state (x, v, w); inv_m is 1/m per
 * particle.  Returns the number written to agg (one per body with a zone). */
int32_t orc_aggregates(int64_t n, const double* r, const double* inv_m, const double* x, const double* v,
                       const double* w, int32_t nb, const orc_body* bodies, orc_aggregate* agg);

/* As orc_aggregates, with the bodies of the tools (terrain: the first
 * heightfield shape or NULL) taking the union of their predicted wedges as
 * their zone. */
int32_t orc_aggregates_tools(int64_t n, const double* r, const double* inv_m, const double* x, const double* v,
                             const double* w, int32_t nb, const orc_body* bodies, int32_t ntools,
                             const struct orc_tool* tools, const orc_shape* terrain, orc_aggregate* agg);

/* Learned-start features (12 per canonical contact), the contact frame
 * (t1, t2: 6 per contact) and the impulse scale m_eff g dt (1 per contact)
 * for the state (x, v, w) and the previous-step cache.  Returns the contact
 * count (the list is the one orc_detect gives). */
int64_t orc_features(const orc_params* P, int64_t n, const int64_t* id, const double* r, const double* rho,
                     const double* x, const double* v, const double* w,
                     int32_t nb, const orc_body* bodies, int32_t ns, const orc_shape* shapes,
                     int64_t nprev, const uint64_t* prev_keys, const double* prev_lam,
                     int64_t cap, double* feat, double* frame, double* scale);

/* Natural-map complementarity residual of the MCP built for the state
 * (x, v, w) with impulses lam (4 per canonical contact), evaluated at the
 * velocities those impulses give.  Used only by tests. */
double orc_natural_residual(const orc_params* P,
                            int64_t n, const int64_t* id, const double* r, const double* rho,
                            const double* x, const double* v, const double* w,
                            int32_t nb, const orc_body* bodies,
                            int32_t ns, const orc_shape* shapes,
                            int64_t nc, const double* lam);

/* MLP in FP64: forward for a batch (feat: B x 12, out: B x 3), and the
 * gradient of 0.5 * mean_b ||y_b - label_b||^2 w.r.t. every parameter
 * (grads laid out W1,b1,W2,b2,W3,b3 contiguously).  Returns the loss. */
void orc_mlp_forward(const orc_mlp* net, int64_t B, const double* feat, double* out);
double orc_mlp_loss_grad(const orc_mlp* net, int64_t B, const double* feat,
                         const double* label, double* grads);

/* Failure-plane angle of the active zone, Eq. failure_plane. */
double orc_failure_angle(double phi, double beta);

#ifdef __cplusplus
}
#endif
#endif
