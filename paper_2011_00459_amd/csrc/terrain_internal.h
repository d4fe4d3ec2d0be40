// terrain_internal.h -- device data layout and kernel launchers of libterrain.
//
// Layout in HBM (all arrays allocated once at their capacities):
//   particles, sorted every step by (environment, Morton cell, id):
//     xr[P]  float4 (x, y, z, r)         vw[2P] float4 pairs (v, 1/m), (omega, 1/I)
//     pid[P] int32 global id             rho[P] float
//   cells: per environment a dense grid, keys = cell_base + Morton code
//   contacts (capacity C):
//     raw detection output  rkey[C] u64, rpair[C] int2
//     canonical (key order) ckey[C] u64, cpair[C] int2, lamc[C] float4
//     colour order rows     r0 (n, l1), r1 (l2, 1/Dn, 1/Dt, Sigma),
//                           r2 (q, lo, body1, body2), rk (kinematic velocity, update-sequence
//                           bits), lam (impulses)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "terrain.h"

namespace trk {

constexpr int kSlotImpact = 3;     // PGS statistics slot of the impact stage
constexpr int kMaxColours = 64;     // colours of the contact schedule (64-bit masks)
constexpr int kGroups = 8;          // PGS groups: one per XCD of the MI355X (block b runs on XCD b % 8)
constexpr int kBuckets = kMaxColours * kGroups;  // (colour, group) buckets of the PGS order
constexpr int kMaxHits = 32;        // contacts one particle may emit per step
constexpr int kMaxZonesPerEnv = 4;  // bodies with an active zone per environment
constexpr int kZoneMoments = 20;    // M, mx(3), mv(3), mxx(6), m x*v(3), sum Is(1), sum Is w(3)
constexpr int kForceChunks = 32;    // deterministic chunks of the body-force reduction
constexpr int kZoneChunk = 2048;    // particles per chunk of the zone reduction
constexpr int kMlpParams = 64 * 12 + 64 + 64 * 64 + 64 + 3 * 64 + 3 + 12;

// PGS solve modes
enum : int {
    kModeGrouped = 0,  // envs in kGroups XCD groups, grid-wide colour barriers per group
    kModePerEnv = 1,   // each env solved by its own block (or cluster of blocks)
    kModeSpread = 2,   // one env spread over the kGroups XCD groups by space, all groups meeting per colour
};
constexpr int kEnvBlk = 1024;  // threads of a per-env PGS block

// Overflow / failure bits of Counters::overflow
enum : uint32_t {
    kOvfContacts = 1u,
    kOvfHits = 2u,
    kOvfColours = 4u,
    kFailColouring = 8u,
    kFailBarrier = 16u,
    kOvfZones = 32u,
};

struct EnvDev {
    float lo[3];
    float inv_h;
    int dims[3];
    int bits[3];
    uint32_t cell_base;
    int shape_begin, shape_end;   // env's shapes in the shape table
    int body_begin, body_end;     // env's bodies
    int id_base;                  // first particle id of the env
    int n;                        // particles of the env
    int slot_begin;               // first slot of the env in sorted order
    int col_base;                 // first depth column of the env (dims[0] x dims[1] columns)
    int group;                    // PGS group (XCD) that solves this env in grouped mode
    int unit;                     // solve unit: the group (grouped mode) or the env (per-env mode)
    int zone_count;
    int zone_body[kMaxZonesPerEnv];  // global body index of each zone
    int zone_slot[kMaxZonesPerEnv];  // global zone index of each zone
};

struct BodyDev {
    double pos[3];
    double quat[4];
    double linvel[3];
    double angvel[3];
    double R[9];          // rotation of quat, row-major (start of step)
    double planes[8][4];  // zone half-spaces, body frame
    double wplanes[8][4]; // zone half-spaces, world frame (end of step)
    int env;
    int nplanes;
    int user_id;
    int tool;             // index of its zone predictor tool, or -1
};

// zone predictor tool (the tr_tool_desc of a body), global body and terrain indices
struct ToolDev {
    int body;
    int env;
    int n_wedges;
    int terrain;          // global shape index of the env's first heightfield, or -1
    double edge0[3], edge1[3], n_c[3], n_tc[3];
    double fill, phi, heap, v_min;
};

// one predicted wedge: n half-spaces, world frame (0: empty)
struct WedgeDev {
    int n;
    int pad;
    double planes[5][4];
};

struct ShapeDev {
    int type;
    int body;        // global body index
    int env;
    int hf_off;      // offset of the heights in the heightfield pool
    double n[3];     // plane normal (body frame)
    double d;        // plane offset
    double half[3];  // box half extents
    double off[3];   // box centre (body frame)
    int nx, ny;
    double ox, oy, l0, inv_l0;
    // world-frame values of the current step
    double wn[3];
    double wd;
    double wc[3];
    double R[9];
};

struct StepParams {
    float dt;
    float g[3];
    float mu;
    float gamma_dt;     // gamma_t / dt
    double kappa_c;     // cohesive range fraction (0 when c_p == 0)
    double kappa_min;
    double Estar;
    double a_coef;      // (4/dt) Upsilon
    double b_coef;      // Upsilon
    double sig_coef;    // (4/dt^2) Upsilon
    double lo_coef;     // c_p pi dt
    uint32_t id_cap;    // ids per environment
    int n_envs;
    int max_sweeps;
    float tol;
    int warm;
    int n_particles;    // all envs
    int n_bodies;
    int n_shapes;
    int n_zones;
    double dt_d;        // dt in FP64 (learned-start features)
    double gdt;         // |g| dt
    double r_ref;       // nominal radius of the features
    float mu_r;         // rolling resistance (0: no rolling rows)
    float v_imp;        // impact threshold (<= 0: no impact stage)
    int n_units;        // PGS solve units (entries of ustats)
    float restitution;  // Newton restitution of the impact stage
    int n_tools;        // zone predictor tools (all envs)
    int spread;         // 1: spread mode (the PGS groups split the env by space)
};

// per PGS solve unit: an XCD group of envs (grouped mode) or one env
// (per-env mode); envs of one unit share the stopping decision (64 B)
struct UnitStats {
    uint32_t sweeps;
    uint32_t use_learned;  // 1 when the learned start won the first-sweep trial
    uint32_t fallback;
    uint32_t learn_bad;    // non-finite network output in this unit
    double resid;
    double resid_first;
    double r1_trial[2];    // first-sweep residual from the learned / previous start
    uint32_t imp_any;      // some contact of the unit is an impact this step
    uint32_t imp_sweeps;   // sweeps of the unit's impact stage
    uint32_t pad2[2];
};

struct Counters {
    uint32_t n_raw;        // contacts found by detection (may exceed capacity)
    uint32_t n_pairs;
    uint32_t overflow;     // kOvf* / kFail* bits, sticky within a step
    uint32_t n_colours;
    uint32_t failed;       // OR of the overflow bits of every step since the host last read it
    uint32_t pad[11];
    uint32_t bar[kGroups][16];  // per-group barrier counters, one cache line each
    uint32_t gbar[16];          // spread mode: arrivals of the groups at the colour barrier
};

struct EnvStats {
    int64_t contacts;
    int64_t pairs;
    unsigned long long impacts;  // contacts of the env treated as impacts this step
};

// A particle's velocity (v, 1/m) and angular velocity (omega, 1/I) are the
// two halves of its 32 B record in vw: the solver gathers both for every
// contact, and one record is one memory line where two arrays were two.
__host__ __device__ inline float4& vel_at(float4* vw, int64_t s) { return vw[2 * s]; }
__host__ __device__ inline float4& angv_at(float4* vw, int64_t s) { return vw[2 * s + 1]; }

// Everything the kernels touch, as raw device pointers.
struct DevBuffers {
    // particles (capacity P, double buffered for the sort)
    float4 *xr, *vw, *xr2, *vw2;  // vw: two float4 per slot, see vel_at
    int *pid, *pid2;
    float *rho, *rho2;
    uint32_t *pkey, *perm;
    int* id2slot;         // [NID]
    // cells
    uint32_t *cell_count, *cell_start, *cell_fill;  // [NC], [NC+1], [NC]
    // contacts
    unsigned long long *rkey, *ckey, *pkeyc;        // raw, canonical, previous canonical
    int2 *rpair, *cpair;
    float4 *lamc, *plam;                            // canonical impulses (current, previous)
    uint32_t *id_count, *id_start, *id_fill, *pid_start;  // [NID], [NID+1], [NID], [NID+1]
    uint32_t *inc_count, *inc_start, *inc_fill, *inc;     // [P], [P+1], [P], [2C]
    int* colour;                                    // [C]
    uint32_t* col_wait;                             // [C] colouring: the neighbour that blocked a contact
    uint32_t *col_hist, *col_start;                 // [kBuckets*NB], [kBuckets*NB+1]
    uint32_t* cpos;                                 // canonical -> colour position
    float4 *r0, *r1, *r2, *rk, *lam, *lam0;         // colour order
    // [3C] canonical order: each contact's start impulse as the velocity
    // changes of its spheres, (J, slot of sphere 2), (dw of sphere 2, dw.x of
    // sphere 1), (dw.yz of sphere 1, 0, 0), per unit inverse mass / inertia
    float4* wrec;
    // rolling rows (allocated when mu_r > 0): r3 = (1/W_r, r mu_r, kinematic body, 0),
    // lamr = (lambda_r, 0) and its start value, canonical current / previous caches
    float4 *r3, *lamr, *lamr0, *lamrc, *plamr;
    // impact stage (allocated when v_imp > 0): its rows ri1 = (l2, 1/W_n, 1/W_t, 0)
    // and ri2 = (target, 0, body 1, body 2), its impulses, and the overlap part
    // of the main rows' q (q = qg + Upsilon G_n v)
    float4 *ri1, *ri2, *lami, *lamri;
    float* qg;
    // reductions
    double* resid_acc;    // [max_sweeps * 2] per-sweep numerator / denominator... (block partials)
    double* block_part;   // [2 parities][grid][2]
    double* force_part;   // [bodies * kForceChunks * 6]
    double* body_ft;      // [bodies * 6]
    double* zone_part;    // [chunks * kMaxZonesPerEnv * kZoneMoments]
    double* zone_mom;     // [zones * kZoneMoments]
    tr_aggregate* aggs;   // [zones]
    int4* zone_chunks;    // (env, begin, end, first zone) per chunk
    // scene tables
    EnvDev* envs;
    BodyDev* bodies;
    ShapeDev* shapes;
    float* hf_pool;
    ToolDev* tools;       // [n_tools]
    WedgeDev* wedges;     // [n_tools][TR_MAX_WEDGES]
    Counters* cnt;
    EnvStats* env_stats;
    UnitStats* ustats;    // [n_units]
    uint32_t* env_col;    // [n_envs][kMaxColours + 1] colour starts of each env (per-env mode)
    uint32_t* env_ncol;   // [n_envs] colours used by each env
    int4* plan;           // per-env PGS tasks: (env, rank in its cluster, cluster size, first block)
    uint32_t* plan_idx;   // [blocks + 1]: tasks of block b are plan[plan_idx[b] .. plan_idx[b + 1])
    uint32_t* env_bar;    // [n_envs][16] cluster barrier counters (per-env mode)
    uint32_t* ver;        // [P] updates applied to each sphere in the current PGS launch
    uint32_t* scan_tmp;   // scratch of the device-wide scan
    float* mlp;           // learned-start weights (kMlpParams)
    // learned start (colour order) and the depth feature
    float* feat;          // [C * 12]
    float4 *frm1, *frm2;  // (t1, m_eff g dt), (t2, 0)
    float4* lamL;         // learned lambda^0
    float* mlp_out;       // [C * 3]
    float* pdepth;        // [P] depth below the column top
    uint32_t* colmax;     // [columns] ordered-int max of z + r
};

// Sizes that fix the launch shapes.
struct Sizes {
    int64_t P;      // particle capacity (all envs)
    int64_t C;      // contact capacity (all envs)
    int64_t NID;    // id space = n_envs * cap_particles
    int64_t NC;     // cells (all envs)
    int64_t NB;     // blocks of 256 over C (colour bucketing)
    int64_t roll_C; // entries of the rolling-row arrays (C when mu_r > 0, else 1)
    int64_t imp_C;  // entries of the impact-stage arrays (C when v_imp > 0, else 1)
    int n_envs;
    int n_zone_chunks;
    int pgs_grid;   // blocks of the persistent PGS kernel (kGroups x blocks per group)
    int pgs_block;  // threads per PGS block
    int pgs_mode;   // kModeGrouped, kModePerEnv or kModeSpread
    int plan_blocks;  // blocks of the per-env PGS kernel
    int lds_cap;    // particles whose bodies a per-env block keeps in LDS (0: none)
    int n_units;    // entries of ustats
    int flow;       // colour order kept by per-sphere update counters instead of barriers
    int part_sweeps;  // sweeps of block partials held (flow: one slot per sweep)
    int col_grid;   // resident blocks of the colouring kernel
    int64_t NCOL;   // depth columns (all envs)
};

// ---- launchers (terrain_kernels.hip) ----
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
void launch_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t s);
int64_t scan_tmp_words(int64_t n);
void launch_step_begin(const DevBuffers& b, const StepParams& p, hipStream_t s);
// writes the sorted particle arrays into the *2 buffers: swap them after
void launch_sort_particles(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s);
void launch_narrow(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s);
void launch_canonical(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s);
void launch_colour(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s);
void launch_rows(const DevBuffers& b, const StepParams& p, const Sizes& z, bool have_prev, bool features,
                 hipStream_t s);
// wedges of a conversion call: ranges of a wedge table
constexpr int kMaxConvRanges = 8;
struct WedgeSet {
    const WedgeDev* base;
    int n_ranges;
    int off[kMaxConvRanges];
    int cnt[kMaxConvRanges];
};
// conversion between resting solid and fluidized mass (device arrays of the
// caller); total: one device double accumulating the converted mass
void launch_surface(const tr_voxel_grid& g, const double* phi, double* h, float* hf, hipStream_t s);
void launch_convert_cut(const tr_voxel_grid& g, double rho_b, const WedgeSet& ws, double* phi, const double* wc,
                        double* mf, double* total, hipStream_t s);
void launch_convert_deposit(const tr_voxel_grid& g, double rho_b, double w_dep, const WedgeSet& ws,
                            const double* rho_p, double* phi, double* wc, double* mf, double* total, hipStream_t s);
// forming particles from fluid inside the zones: candidates into list (8
// doubles each: voxel, centre 3, velocity 3, radius), *count their number
// (all of them are counted, at most cap written); then the fluid pays
struct FormEntry {
    double voxel;  // index, exact in a double below 2^53
    double x[3], v[3];
    double r;
};
void launch_form_candidates(const tr_voxel_grid& g, double rho, double d_min, double d_max, double phi_max,
                            const WedgeSet& ws, const double* rho_p, const double* u, const double* mf,
                            FormEntry* list, unsigned long long* count, int64_t cap, hipStream_t s);
void launch_form_pay(const FormEntry* list, int64_t n, double rho, double* mf, hipStream_t s);
// particles of env at rest outside the zones: their mass into mf, their ids
// into list (*count of them)
void launch_settle(const DevBuffers& b, const EnvDev& E, const tr_voxel_grid& g, double v_rest, const WedgeSet& ws,
                   double* mf, int* list, unsigned long long* count, double* total, hipStream_t s);
// particle growth from the voxels' fluidized mass; work: 2 nx ny nz doubles
void launch_grow(const DevBuffers& b, const EnvDev& E, const tr_voxel_grid& g, double dt, double dprime_max,
                 double d_max, double* mf, double* work, double* total, hipStream_t s);
// mesoscale voxel fields (device arrays of the caller); cfl_bits: one
// device uint64 receiving the largest Courant number's bits (NULL: not reduced)
void launch_coarse_grain(const DevBuffers& b, const EnvDev& E, const tr_voxel_grid& g, int kernel, double R,
                         double* rho, double* mom, double* u, hipStream_t s);
constexpr int kAdvectTargetBlocks = 2048;  // about 8 blocks per CU
int64_t advect_blocks(const tr_voxel_grid& g);  // size of the per-block maxima launch_advect needs
void launch_advect(const tr_voxel_grid& g, double dt, const double* u, const double* mf_in, double* mf_out,
                   double* bmax, unsigned long long* cfl_bits, hipStream_t s);
// impact stage: rows of envs without impacts neutralised, the stage's sweeps
// (stats slot kSlotImpact), the main rows' q from the post-impact velocities
void launch_impact_stage(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s);
void launch_warm_apply(const DevBuffers& b, const StepParams& p, const Sizes& z, bool rebuild, hipStream_t s);
// sweeps_cap < 0: the scene's max_sweeps; slot 0 writes the step stats,
// slot 1/2 the first-sweep residual of the learned / previous-step trial
void launch_pgs(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s, int sweeps_cap = -1,
                int slot = 0);
void launch_depth(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s);
void launch_vel_copy(const DevBuffers& b, const StepParams& p, bool backup, hipStream_t s);
void launch_select_start(const DevBuffers& b, const StepParams& p, const Sizes& z, int mode, hipStream_t s);
void launch_choose_start(const DevBuffers& b, const StepParams& p, hipStream_t s);
void launch_learn_samples(const DevBuffers& b, int64_t beg, int64_t n, float* feat, float* label, hipStream_t s);
// terrain_mlp.hip
void launch_mlp_infer(const float* W, const float* feat, float* out, const uint32_t* d_n, int64_t cap, bool bf16,
                      hipStream_t s);
void launch_learned_lam(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s);
void launch_mlp_grad(const float* W, const float* feat, const float* label, int64_t B, float* grad, float* loss,
                     float* scratch, hipStream_t s);
void launch_adam(float* W, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps, int t,
                 hipStream_t s);
int64_t mlp_grad_scratch(int64_t B);
int mlp_trainable();
void launch_finish(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s);
// macroscale step (one env): its zones in body order, candidate reductions
constexpr int kMacroMaxZones = 8;
struct MacroZone {
    double mom[kZoneMoments];            // moments as in the zone sums of a step
    double vol;                          // solid volume of the zone's particles
    double area[2];                      // AB, AC: sum of the candidates' pi r^2
    unsigned long long cnt[2];           // candidates of AB, AC
    unsigned long long vmax[2][4];       // order-preserving image of the largest projection along +-e1, +-e2
    unsigned long long kmin[2][4];       // smallest candidate key reaching it
    double wpl[8][4];                    // the body's half-spaces in the world frame at its current pose
    int nplanes;
};
struct MacroArgs {
    int n;                               // particles of the env (ids id_base .. id_base + n - 1)
    int id_base;
    int slot_begin;                      // the env's spheres hold slots slot_begin .. + n - 1 (-1: unknown, go by id)
    int shape_begin, shape_end;          // the env's shapes
    int n_zones;                         // bodies with half-spaces, in body order
    int body[kMacroMaxZones];            // global body index of each
    int eligible[kMacroMaxZones];        // 1: at least two half-spaces (separation plate, failure plane)
    tr_macro_params mp;
    int has_eq[kMacroMaxZones];          // 1: the zone's body is a dynamic equipment (eq below)
    tr_macro_equipment eq[kMacroMaxZones];
    double g[3];                         // gravity (FP64, as the scene was given it)
};
void launch_macro(const DevBuffers& b, const StepParams& p, const MacroArgs& a, MacroZone* mz, tr_macro_result* out,
                  hipStream_t s);

void launch_gather_by_id(const DevBuffers& b, int id_base, int n, float4* xo, float4* vo, float4* wo,
                         hipStream_t s);
void launch_scatter_by_id(const DevBuffers& b, int id_base, int n, const float4* xi, const float4* vi,
                          const float4* wi, int mask, hipStream_t s);
int pgs_resident_blocks(int block);
int pgs_env_resident_blocks(int lds_bytes);
int pgs_env_max_lds();
int colour_resident_blocks();

}  // namespace trk
