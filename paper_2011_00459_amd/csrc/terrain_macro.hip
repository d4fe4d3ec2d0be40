// terrain_macro.hip -- the macroscale step of each active zone (section
// "Macroscale model"): the zone's aggregate body (Eqs. aggregate_mass ..
// aggregate_rot_vel) under Eq. mdb:eqAgg with the frictional-cohesive velocity
// constraints of Eqs. aggregateNormal and aggregateTangent at its interfaces
// to the equipment B (AB) and to the terrain's failure surface C (AC), each
// interface reduced to four contact points.
//
//   k_macro_pass1  per particle of the env: zone membership (planes posed from
//                  the bodies' current poses), the aggregate's moments, and for
//                  the AB / AC candidates their count, cross-section area and
//                  the largest projection along +-e1, +-e2 of the interface
//                  (order-preserving 64-bit atomic maxima of the FP64 values)
//   k_macro_pass2  the smallest candidate key reaching each maximum (ties to
//                  the smaller particle id, then shape index)
//   k_macro_solve  one thread per zone: the aggregate, the (at most) four
//                  points of each interface, and the small complementarity
//                  problem solved to machine precision in FP64: a damped
//                  semismooth Newton iteration on the aggregate's six
//                  velocities reaches the fixed point of the rows' projected
//                  Gauss-Seidel, whose sweeps then confirm it (the regularised
//                  rows of a rigid body with redundant points contract by only
//                  about 1 - gamma / W per sweep, so Gauss-Seidel alone needs
//                  ~1e5 sweeps for a stiff bulk); where Newton stalls at a
//                  kink of the projections, eight sweeps and a restart
//
// Readings: the zone's half-spaces follow the wedge convention (plane 0 the
// separation plate, plane 1 the failure plane); AB candidates are the zone's
// particles touching the zone body's shapes, AC candidates the zone's particles
// within their radius of the failure plane, projected onto it; the interface
// area is the sum of the candidates' cross sections; gamma = L / (c_as E_b A
// dt^2), the compliance of the bulk as a spring c_as E_b A / L regularising a
// velocity row over one step (velocity per impulse), L the cube root of the
// aggregate's solid volume; the equipment is kinematic, the terrain static.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "terrain_geom.h"
#include "terrain_internal.h"

// every FP64 expression below is evaluated as written (no fused multiply-add),
// like the reference arithmetic it is compared with
#pragma clang fp contract(off)

namespace trk {

namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ inline double dot3d(const double* a, const double* b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }
__device__ inline void cross3d(const double* a, const double* b, double* c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// order-preserving image of a double in the unsigned integers (-0 and +0
// map to the same image, as they compare equal)
__device__ inline unsigned long long ord64(double v)
{
    unsigned long long u = (unsigned long long)__double_as_longlong(v + 0.0);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}

// world-frame half-space p of a body at its current pose: normal nw, offset dw
__device__ inline void plane_world(const BodyDev& B, int p, double nw[3], double& dw)
{
#pragma clang fp contract(off)
    double R[9];
    quat_to_R(B.quat, R);
    const double* pl = B.planes[p];
    for (int k = 0; k < 3; ++k) nw[k] = (R[k * 3 + 0] * pl[0] + R[k * 3 + 1] * pl[1]) + R[k * 3 + 2] * pl[2];
    dw = pl[3] + dot3d(nw, B.pos);
}

// in-plane axes: e1 the normalised projection of the world axis least aligned
// with n (the lower axis on ties), e2 = n x e1
__device__ inline void plane_axes(const double* n, double* e1, double* e2)
{
#pragma clang fp contract(off)
    int k0 = 0;
    for (int k = 1; k < 3; ++k)
        if (fabs(n[k]) < fabs(n[k0])) k0 = k;
    double a[3] = {0.0, 0.0, 0.0};
    a[k0] = 1.0;
    double an = dot3d(a, n);
    for (int k = 0; k < 3; ++k) e1[k] = a[k] - an * n[k];
    double m = sqrt(dot3d(e1, e1));
    for (int k = 0; k < 3; ++k) e1[k] /= m;
    cross3d(n, e1, e2);
}

// a shape posed at its body's current pose (the step's kernels pose shapes at
// the start of a step)
__device__ inline ShapeDev posed_shape(const DevBuffers& b, int g)
{
#pragma clang fp contract(off)
    ShapeDev S = b.shapes[g];
    const BodyDev& B = b.bodies[S.body];
    double R[9];
    quat_to_R(B.quat, R);
    for (int k = 0; k < 9; ++k) S.R[k] = R[k];
    for (int k = 0; k < 3; ++k) S.wn[k] = (R[k * 3 + 0] * S.n[0] + R[k * 3 + 1] * S.n[1]) + R[k * 3 + 2] * S.n[2];
    S.wd = S.d + ((S.wn[0] * B.pos[0] + S.wn[1] * B.pos[1]) + S.wn[2] * B.pos[2]);
    for (int k = 0; k < 3; ++k) S.wc[k] = B.pos[k] + ((R[k * 3 + 0] * S.off[0] + R[k * 3 + 1] * S.off[1]) + R[k * 3 + 2] * S.off[2]);
    return S;
}

// the env's zone (index into MacroArgs) containing x: the first body (in the
// env's zone order) whose half-spaces all contain it; -1 when none
__device__ inline int zone_at(const MacroArgs& a, const MacroZone* mz, const double* x)
{
    for (int z = 0; z < a.n_zones; ++z) {
        const MacroZone& Z = mz[z];
        bool in = Z.nplanes > 0;
        for (int p = 0; p < Z.nplanes && in; ++p)
            if (dot3d(Z.wpl[p], x) - Z.wpl[p][3] > 0.0) in = false;
        if (in) return z;
    }
    return -1;
}

// interface q (0: AB, 1: AC) normal of zone z, from B or C into A
__device__ inline void iface_normal(const DevBuffers& b, const MacroArgs& a, int z, int q, double* n, double& dfail)
{
    double nw[3], dw;
    plane_world(b.bodies[a.body[z]], q, nw, dw);
    for (int k = 0; k < 3; ++k) n[k] = -nw[k];
    dfail = dw;
}

// AB candidate of a sphere against shape g: the contact point at the middle
// of the overlap
__device__ inline bool ab_point(const DevBuffers& b, const StepParams& p, int g, const double* x, double r,
                                double* pt)
{
    ShapeDev S = posed_shape(b, g);
    ShapeHit hit;
    if (!shape_touch(S, b.hf_pool, x[0], x[1], x[2], r, p.kappa_c, &hit)) return false;
    const double l2 = r - 0.5 * hit.delta;
    for (int k = 0; k < 3; ++k) pt[k] = x[k] - l2 * hit.n[k];
    return true;
}

// AC candidate of a sphere of zone z: within its radius of the failure plane,
// projected onto it
__device__ inline bool ac_point(const DevBuffers& b, const MacroArgs& a, int z, const double* x, double r, double* pt)
{
    double nw[3], dw;
    plane_world(b.bodies[a.body[z]], 1, nw, dw);
    const double d = dot3d(nw, x) - dw;
    if (!(d >= -r)) return false;
    for (int k = 0; k < 3; ++k) pt[k] = x[k] - d * nw[k];
    return true;
}

// Candidates of sphere id (env-local) in zone z, interface q: calls f(key,
// point) for each (AB: one per touching shape of the zone's body, key = id
// << 16 | shape index in the env; AC: key = id << 16).
template <class F>
__device__ inline void candidates(const DevBuffers& b, const StepParams& p, const MacroArgs& a, int z, int q, int id,
                                  const double* x, double r, F f)
{
    double pt[3];
    if (q == 0) {
        for (int g = a.shape_begin; g < a.shape_end; ++g)
            if (b.shapes[g].body == a.body[z] && ab_point(b, p, g, x, r, pt))
                f(((unsigned long long)id << 16) | (unsigned long long)(g - a.shape_begin), pt);
    } else if (ac_point(b, a, z, x, r, pt)) {
        f((unsigned long long)id << 16, pt);
    }
}

// wave (64 lanes) sum and maximum; every lane of the wave takes part
__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline unsigned long long wave_max(unsigned long long v)
{
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    return v;
}

// this lane's candidate (if `has`) of interface q added to its zone's count,
// area and extreme projections: one atomic per zone and wave
__device__ inline void wave_add_candidate(MacroZone* mz, int n_zones, int z, bool has, int q, double r,
                                          const double* pt, const double* e1, const double* e2)
{
    const int lane = threadIdx.x & 63;
    unsigned long long o4[4] = {0ull, 0ull, 0ull, 0ull};
    if (has) {
        const double s1 = dot3d(pt, e1), s2 = dot3d(pt, e2);
        o4[0] = ord64(s1); o4[1] = ord64(-s1); o4[2] = ord64(s2); o4[3] = ord64(-s2);
    }
    for (int zz = 0; zz < n_zones; ++zz) {
        const bool mine = has && z == zz;
        const unsigned long long m = __ballot(mine);
        if (m == 0) continue;
        const double area = wave_sum(mine ? kPi * r * r : 0.0);
        unsigned long long mx[4];
        for (int d = 0; d < 4; ++d) mx[d] = wave_max(mine ? o4[d] : 0ull);
        if (lane == __ffsll((unsigned long long)m) - 1) {
            atomicAdd(&mz[zz].cnt[q], (unsigned long long)__popcll(m));
            atomicAdd(&mz[zz].area[q], area);
            for (int d = 0; d < 4; ++d) atomicMax(&mz[zz].vmax[q][d], mx[d]);
        }
    }
}

// Pass 1: zone membership, the zones' moments and the candidates' count, area
// and extreme projections, each reduced over the wave before its atomic (all
// the spheres of a zone add to the same few addresses)
__global__ void __launch_bounds__(256) k_macro_pass1(DevBuffers b, StepParams p, MacroArgs a, MacroZone* mz)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    int z = -1;
    double x[3] = {0.0, 0.0, 0.0}, r = 0.0, vol = 0.0;
    double mom[kZoneMoments];
    for (int k = 0; k < kZoneMoments; ++k) mom[k] = 0.0;
    if (t < a.n) {
        const int s = a.slot_begin >= 0 ? a.slot_begin + t : b.id2slot[a.id_base + t];
        const float4 xf = b.xr[s], vf = vel_at(b.vw, s), wf = angv_at(b.vw, s);
        x[0] = xf.x; x[1] = xf.y; x[2] = xf.z;
        r = xf.w;
        z = zone_at(a, mz, x);
        if (z >= 0) {
            const double m = (double)b.rho[s] * (4.0 / 3.0) * kPi * r * r * r;
            const double v[3] = {vf.x, vf.y, vf.z};
            const double Is = 0.4 * m * r * r;
            mom[0] = m;
            for (int k = 0; k < 3; ++k) { mom[1 + k] = m * x[k]; mom[4 + k] = m * v[k]; }
            mom[7] = m * x[0] * x[0]; mom[8] = m * x[1] * x[1]; mom[9] = m * x[2] * x[2];
            mom[10] = m * x[0] * x[1]; mom[11] = m * x[0] * x[2]; mom[12] = m * x[1] * x[2];
            mom[13] = m * (x[1] * v[2] - x[2] * v[1]);
            mom[14] = m * (x[2] * v[0] - x[0] * v[2]);
            mom[15] = m * (x[0] * v[1] - x[1] * v[0]);
            mom[16] = Is;
            mom[17] = Is * wf.x; mom[18] = Is * wf.y; mom[19] = Is * wf.z;
            vol = (4.0 / 3.0) * kPi * r * r * r;
        }
    }
    const int lane = threadIdx.x & 63;
    for (int zz = 0; zz < a.n_zones; ++zz) {
        const unsigned long long m = __ballot(z == zz);
        if (m == 0) continue;
        const int leader = __ffsll((unsigned long long)m) - 1;
        for (int k = 0; k <= kZoneMoments; ++k) {
            const double v = wave_sum(z == zz ? (k < kZoneMoments ? mom[k] : vol) : 0.0);
            if (lane == leader) atomicAdd(k < kZoneMoments ? &mz[zz].mom[k] : &mz[zz].vol, v);
        }
    }
    const bool elig = z >= 0 && a.eligible[z];
    double e1[2][3], e2[2][3];
    for (int q = 0; q < 2; ++q) {
        double n[3], dfail;
        if (elig) {
            iface_normal(b, a, z, q, n, dfail);
            plane_axes(n, e1[q], e2[q]);
        }
    }
    // AB: the env's shapes in turn, the same loop on every lane
    for (int g = a.shape_begin; g < a.shape_end; ++g) {
        double pt[3];
        const bool has = elig && b.shapes[g].body == a.body[z] && ab_point(b, p, g, x, r, pt);
        wave_add_candidate(mz, a.n_zones, z, has, 0, r, pt, e1[0], e2[0]);
    }
    double pt[3];
    const bool has = elig && ac_point(b, a, z, x, r, pt);
    wave_add_candidate(mz, a.n_zones, z, has, 1, r, pt, e1[1], e2[1]);
}

__global__ void __launch_bounds__(256) k_macro_pass2(DevBuffers b, StepParams p, MacroArgs a, MacroZone* mz)
{
#pragma clang fp contract(off)
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n) return;
    const int s = a.slot_begin >= 0 ? a.slot_begin + t : b.id2slot[a.id_base + t];
    float4 xf = b.xr[s];
    double x[3] = {xf.x, xf.y, xf.z};
    const int z = zone_at(a, mz, x);
    if (z < 0 || !a.eligible[z]) return;
    const int id = a.slot_begin >= 0 ? b.pid[s] - a.id_base : t;
    MacroZone& Z = mz[z];
    for (int q = 0; q < 2; ++q) {
        double n[3], e1[3], e2[3], dfail;
        iface_normal(b, a, z, q, n, dfail);
        plane_axes(n, e1, e2);
        candidates(b, p, a, z, q, id, x, (double)xf.w, [&](unsigned long long key, const double* pt) {
            const double s1 = dot3d(pt, e1), s2 = dot3d(pt, e2);
            const double val[4] = {s1, -s1, s2, -s2};
            for (int d = 0; d < 4; ++d)
                if (ord64(val[d]) == Z.vmax[q][d]) atomicMin(&Z.kmin[q][d], key);
        });
    }
}

// the point of a chosen candidate key (recomputed from its particle)
__device__ inline void key_point(const DevBuffers& b, const StepParams& p, const MacroArgs& a, int z, int q,
                                 unsigned long long key, double* pt)
{
    const int id = (int)(key >> 16);
    const int s = b.id2slot[a.id_base + id];
    float4 xf = b.xr[s];
    double x[3] = {xf.x, xf.y, xf.z};
    candidates(b, p, a, z, q, id, x, (double)xf.w, [&](unsigned long long k2, const double* c) {
        if (k2 == key)
            for (int k = 0; k < 3; ++k) pt[k] = c[k];
    });
}

// inverse of a symmetric positive definite 3 x 3 matrix by cofactors
__device__ inline void inv3(const double (*A)[3], double (*B)[3])
{
    const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
    const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
    const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
    const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
    B[0][0] = c00 / det;
    B[1][0] = c01 / det;
    B[2][0] = c02 / det;
    B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
    B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
    B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
    B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
    B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
    B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
}

__device__ inline double point_w(double invM, const double (*Iinv)[3], const double* rr, const double* u,
                                 const double* w)
{
    double ra[3], rb[3], t[3];
    cross3d(rr, u, ra);
    cross3d(rr, w, rb);
    for (int k = 0; k < 3; ++k) t[k] = (Iinv[k][0] * rb[0] + Iinv[k][1] * rb[1]) + Iinv[k][2] * rb[2];
    return invM * dot3d(u, w) + dot3d(ra, t);
}

// Impulse of one interface point at the fixed point of its rows, as a function
// of the point's relative velocity u: lambda_n = max(lo, -u_n / gamma) (the
// normal row's complementarity) and lambda_t the projection of -u_t / gamma
// onto the disk of radius mu |lambda_n| (the tangential rows' variational
// inequality).  lam4 = (lambda_n, lambda_t xyz); K = d(lambda_n n + lambda_t)
// / du (a generalized derivative) when K is not NULL.
__device__ inline void point_impulse(const double* u, const double* n, double gam, double lo, double mu,
                                     double* lam4, double (*K)[3])
{
#pragma clang fp contract(off)
    const double un = dot3d(n, u);
    const double zn = -un / gam;
    const bool nact = zn > lo;
    const double ln = nact ? zn : lo;
    double z[3];
    for (int k = 0; k < 3; ++k) z[k] = -(u[k] - un * n[k]) / gam;
    const double zz = sqrt(dot3d(z, z));
    const double rho = mu * fabs(ln);
    const bool stick = zz <= rho;
    const double sc = stick ? 1.0 : (zz > 0.0 ? rho / zz : 0.0);
    lam4[0] = ln;
    for (int k = 0; k < 3; ++k) lam4[1 + k] = sc * z[k];
    if (!K) return;
    double dln[3];
    for (int k = 0; k < 3; ++k) dln[k] = nact ? -n[k] / gam : 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) K[i][j] = n[i] * dln[j];
    if (stick) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) K[i][j] -= ((i == j ? 1.0 : 0.0) - n[i] * n[j]) / gam;
    } else if (zz > 0.0) {
        const double sg = ln > 0.0 ? 1.0 : (ln < 0.0 ? -1.0 : 0.0);
        double zh[3] = {z[0] / zz, z[1] / zz, z[2] / zz};
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                K[i][j] += zh[i] * (mu * sg) * dln[j] -
                           (rho / zz) * (((i == j ? 1.0 : 0.0) - n[i] * n[j]) - zh[i] * zh[j]) / gam;
    }
}

// The aggregate's small system: its interface points and, with a dynamic
// equipment, the equipment body and its drive.  Unknowns w: the aggregate's
// (v, omega), then the equipment's (v, omega) when ndof = 12.
struct MacroSys {
    int np, ndof;
    double rr[8][3], rb[8][3], uo[8][3], n[8][3], gam[8], lo[8], mu[8];
    int onB[8];                    // AB point of a dynamic equipment: its rows act on both bodies
    double invM, Iinv[3][3];       // aggregate
    double invMB, IBinv[3][3];     // dynamic equipment (world frame)
    double target[6], lim[6], gd;  // drive: velocity targets, impulse limits, compliance
};

__device__ inline void mat3v(const double (*M)[3], const double* x, double* y)
{
    for (int k = 0; k < 3; ++k) y[k] = (M[k][0] * x[0] + M[k][1] * x[1]) + M[k][2] * x[2];
}

// velocity of point c relative to the other side (u = D_c w - uo_c)
__device__ inline void point_vel(const MacroSys& S, int c, const double* w, double* u)
{
    double t[3];
    cross3d(w + 3, S.rr[c], t);
    for (int k = 0; k < 3; ++k) u[k] = w[k] + t[k] - S.uo[c][k];
    if (S.onB[c]) {
        cross3d(w + 9, S.rb[c], t);
        for (int k = 0; k < 3; ++k) u[k] -= w[6 + k] + t[k];
    }
}

// D_c (3 x 12): [I, -[r_A]x, -I, [r_B]x] (the last two blocks only on a dynamic equipment)
__device__ inline void point_D(const MacroSys& S, int c, double (*D)[12])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 12; ++j) D[i][j] = 0.0;
    const double* r = S.rr[c];
    const double X[3][3] = {{0.0, -r[2], r[1]}, {r[2], 0.0, -r[0]}, {-r[1], r[0], 0.0}};
    for (int i = 0; i < 3; ++i) {
        D[i][i] = 1.0;
        for (int j = 0; j < 3; ++j) D[i][3 + j] = -X[i][j];
    }
    if (!S.onB[c]) return;
    const double* q = S.rb[c];
    const double Y[3][3] = {{0.0, -q[2], q[1]}, {q[2], 0.0, -q[0]}, {-q[1], q[0], 0.0}};
    for (int i = 0; i < 3; ++i) {
        D[i][6 + i] = -1.0;
        for (int j = 0; j < 3; ++j) D[i][9 + j] = Y[i][j];
    }
}

// size of G in velocity units: linear parts and the angular parts times Lc
__device__ inline double gnorm(const double* G, int nd, double Lc)
{
    double s = 0.0;
    for (int k = 0; k < nd; ++k) {
        const double g = (k % 6) < 3 ? G[k] : Lc * G[k];
        s += g * g;
    }
    return sqrt(s);
}

// One zone's solve in LDS; one wave (64 lanes) per zone.
struct SolveShared {
    MacroSys S;
    tr_macro_result o;
    double w0[12], w[12], wt[12], G[12], Gt[12], d[12], F[12];
    double Fp[8][12];              // generalized impulse of each point's rows
    double Sp[8][144];             // D_c^T K_c D_c of each point (nd x nd, row-major)
    double lamp[8][4];             // each point's impulses at the evaluated w
    double Fd[6], Kd[6];           // drive impulses and their derivatives
    double A[144];                 // Jacobian, then its LU factors
    double Wn[8], Wt[8], lam[8][4];
    double V[12], ld[6];           // velocities and drive impulses of the Gauss-Seidel sweeps
    double g, scale, Lc;
    int piv, ok, run, again, map[8];
};

// G(w) = w - w0 - M^-1 F(w), F the generalized impulse of every row at its
// closed-form fixed point given w, and with jac dG/dw into sh.A.  Lanes
// 0 .. np-1 evaluate one point each, lanes 8 .. 13 the drive rows, then the
// sums and the block inverse mass are spread over the lanes.  Every lane of
// the wave calls it.
__device__ void eval_G(SolveShared& sh, const double* w, double* G, bool jac)
{
    const int lane = threadIdx.x;
    const MacroSys& S = sh.S;
    const int nd = S.ndof, np = S.np;
    if (lane < np) {
        const int c = lane;
        double u[3], lam4[4], K[3][3], D[3][12], J[3];
        point_vel(S, c, w, u);
        point_impulse(u, S.n[c], S.gam[c], S.lo[c], S.mu[c], lam4, jac ? K : nullptr);
        for (int k = 0; k < 4; ++k) sh.lamp[c][k] = lam4[k];
        for (int k = 0; k < 3; ++k) J[k] = lam4[0] * S.n[c][k] + lam4[1 + k];
        point_D(S, c, D);
        for (int j = 0; j < 12; ++j) sh.Fp[c][j] = (D[0][j] * J[0] + D[1][j] * J[1]) + D[2][j] * J[2];
        if (jac) {
            double KD[3][12];
            for (int r = 0; r < 3; ++r)
                for (int j = 0; j < 12; ++j) KD[r][j] = (K[r][0] * D[0][j] + K[r][1] * D[1][j]) + K[r][2] * D[2][j];
            for (int i = 0; i < 12; ++i)
                for (int j = 0; j < 12; ++j)
                    if (i < nd && j < nd)
                        sh.Sp[c][i * nd + j] = (D[0][i] * KD[0][j] + D[1][i] * KD[1][j]) + D[2][i] * KD[2][j];
        }
    } else if (nd == 12 && lane >= 8 && lane < 14) {
        const int k = lane - 8;
        const double zz = -(w[6 + k] - S.target[k]) / S.gd;
        sh.Fd[k] = zz > S.lim[k] ? S.lim[k] : (zz < -S.lim[k] ? -S.lim[k] : zz);
        sh.Kd[k] = (zz < S.lim[k] && zz > -S.lim[k]) ? -1.0 / S.gd : 0.0;
    }
    __syncthreads();
    if (lane < nd) {
        double f = (nd == 12 && lane >= 6) ? sh.Fd[lane - 6] : 0.0;
        for (int c = 0; c < np; ++c) f += sh.Fp[c][lane];
        sh.F[lane] = f;
    }
    if (jac)
        for (int t = 0; t < 3; ++t) {
            const int e = lane + 64 * t;
            if (e >= nd * nd) continue;
            double v = 0.0;
            for (int c = 0; c < np; ++c) v += sh.Sp[c][e];
            const int i = e / nd, j = e % nd;
            if (nd == 12 && i == j && i >= 6) v += sh.Kd[i - 6];
            sh.A[e] = v;
        }
    __syncthreads();
    if (lane < nd) {
        const int blk = lane / 3, k = lane % 3;
        double mf;
        if (blk == 0) mf = S.invM * sh.F[lane];
        else if (blk == 1) mf = (S.Iinv[k][0] * sh.F[3] + S.Iinv[k][1] * sh.F[4]) + S.Iinv[k][2] * sh.F[5];
        else if (blk == 2) mf = S.invMB * sh.F[lane];
        else mf = (S.IBinv[k][0] * sh.F[9] + S.IBinv[k][1] * sh.F[10]) + S.IBinv[k][2] * sh.F[11];
        G[lane] = w[lane] - sh.w0[lane] - mf;
    }
    if (jac) {
        double jv[3];
        for (int t = 0; t < 3; ++t) {
            const int e = lane + 64 * t;
            jv[t] = 0.0;
            if (e >= nd * nd) continue;
            const int i = e / nd, j = e % nd, blk = i / 3, k = i % 3;
            double ms;
            if (blk == 0) ms = S.invM * sh.A[e];
            else if (blk == 1)
                ms = (S.Iinv[k][0] * sh.A[3 * nd + j] + S.Iinv[k][1] * sh.A[4 * nd + j]) + S.Iinv[k][2] * sh.A[5 * nd + j];
            else if (blk == 2) ms = S.invMB * sh.A[e];
            else
                ms = (S.IBinv[k][0] * sh.A[9 * nd + j] + S.IBinv[k][1] * sh.A[10 * nd + j]) +
                     S.IBinv[k][2] * sh.A[11 * nd + j];
            jv[t] = (i == j ? 1.0 : 0.0) - ms;
        }
        __syncthreads();  // every lane has read the summed S before it becomes the Jacobian
        for (int t = 0; t < 3; ++t) {
            const int e = lane + 64 * t;
            if (e < nd * nd) sh.A[e] = jv[t];
        }
    }
    __syncthreads();
}

// solves sh.A x = sh.d (nd x nd) in place by Gaussian elimination with partial
// pivoting, a row per lane; false (on every lane) when singular
__device__ bool lu_solve(SolveShared& sh, int nd)
{
    const int lane = threadIdx.x;
    for (int k = 0; k < nd; ++k) {
        if (lane == 0) {
            int piv = k;
            double best = fabs(sh.A[k * nd + k]);
            for (int i = k + 1; i < nd; ++i) {
                const double v = fabs(sh.A[i * nd + k]);
                if (v > best) { best = v; piv = i; }
            }
            sh.piv = best > 0.0 ? piv : -1;
        }
        __syncthreads();
        const int piv = sh.piv;
        if (piv < 0) return false;
        if (piv != k) {
            if (lane < nd) {
                const double t = sh.A[k * nd + lane];
                sh.A[k * nd + lane] = sh.A[piv * nd + lane];
                sh.A[piv * nd + lane] = t;
            }
            if (lane == 0) {
                const double t = sh.d[k];
                sh.d[k] = sh.d[piv];
                sh.d[piv] = t;
            }
        }
        __syncthreads();
        if (lane > k && lane < nd) {
            const double f = sh.A[lane * nd + k] / sh.A[k * nd + k];
            for (int j = k; j < nd; ++j) sh.A[lane * nd + j] -= f * sh.A[k * nd + j];
            sh.d[lane] -= f * sh.d[k];
        }
        __syncthreads();
    }
    if (lane == 0)
        for (int i = nd - 1; i >= 0; --i) {
            double s = sh.d[i];
            for (int j = i + 1; j < nd; ++j) s -= sh.A[i * nd + j] * sh.d[j];
            sh.d[i] = s / sh.A[i * nd + i];
        }
    __syncthreads();
    return true;
}

// Up to nsw sweeps of the rows' projected Gauss-Seidel (one lane): the
// impulses sh.lam and drive impulses sh.ld, with the velocities sh.V (v, w of
// the aggregate, then of a dynamic equipment) that they give.  Returns the
// sweeps done, negated when the stopping rule (no impulse changed by more
// than 1e-15 of the largest) was not met within nsw.
__device__ int pgs_sweeps(SolveShared& sh, bool E, int nsw)
{
    const MacroSys& Q = sh.S;
    const int np = Q.np;
    double* vv = sh.V;
    double* ww = sh.V + 3;
    double* vB = sh.V + 6;
    double* wB = sh.V + 9;
    double* ld = sh.ld;
    for (int sweep = 0; sweep < nsw; ++sweep) {
        double dmax = 0.0, lmax = 0.0, t[3];
        for (int c = 0; c < np; ++c) {
            const double* nn = Q.n[c];
            for (int row = 0; row < 2; ++row) {
                double u[3], J[3];
                cross3d(ww, Q.rr[c], t);
                for (int k = 0; k < 3; ++k) u[k] = vv[k] + t[k] - Q.uo[c][k];
                if (Q.onB[c]) {
                    cross3d(wB, Q.rb[c], t);
                    for (int k = 0; k < 3; ++k) u[k] -= vB[k] + t[k];
                }
                const double un = dot3d(nn, u);
                if (row == 0) {
                    double ln = sh.lam[c][0] - (un + Q.gam[c] * sh.lam[c][0]) / (sh.Wn[c] + Q.gam[c]);
                    if (ln < Q.lo[c]) ln = Q.lo[c];
                    const double d = ln - sh.lam[c][0];
                    sh.lam[c][0] = ln;
                    for (int k = 0; k < 3; ++k) J[k] = d * nn[k];
                    if (fabs(d) > dmax) dmax = fabs(d);
                } else {
                    double lt[3];
                    for (int k = 0; k < 3; ++k) {
                        const double ut = u[k] - un * nn[k];
                        lt[k] = sh.lam[c][1 + k] - (ut + Q.gam[c] * sh.lam[c][1 + k]) / (sh.Wt[c] + Q.gam[c]);
                    }
                    const double ltn = dot3d(lt, nn);
                    for (int k = 0; k < 3; ++k) lt[k] -= ltn * nn[k];
                    const double lim = Q.mu[c] * fabs(sh.lam[c][0]);
                    const double m2 = sqrt(dot3d(lt, lt));
                    if (m2 > lim) {
                        const double sc = m2 > 0.0 ? lim / m2 : 0.0;
                        for (int k = 0; k < 3; ++k) lt[k] *= sc;
                    }
                    for (int k = 0; k < 3; ++k) {
                        J[k] = lt[k] - sh.lam[c][1 + k];
                        if (fabs(J[k]) > dmax) dmax = fabs(J[k]);
                        sh.lam[c][1 + k] = lt[k];
                    }
                }
                double tj[3], dw[3];
                cross3d(Q.rr[c], J, tj);
                mat3v(Q.Iinv, tj, dw);
                for (int k = 0; k < 3; ++k) { vv[k] += Q.invM * J[k]; ww[k] += dw[k]; }
                if (Q.onB[c]) {
                    cross3d(Q.rb[c], J, tj);
                    mat3v(Q.IBinv, tj, dw);
                    for (int k = 0; k < 3; ++k) { vB[k] -= Q.invMB * J[k]; wB[k] -= dw[k]; }
                }
            }
            for (int k = 0; k < 4; ++k)
                if (fabs(sh.lam[c][k]) > lmax) lmax = fabs(sh.lam[c][k]);
        }
        if (E) {
            for (int k = 0; k < 6; ++k) {
                const int ax = k % 3;
                const double u = k < 3 ? vB[ax] - Q.target[k] : wB[ax] - Q.target[k];
                const double W = k < 3 ? Q.invMB : Q.IBinv[ax][ax];
                double l = ld[k] - (u + Q.gd * ld[k]) / (W + Q.gd);
                if (l > Q.lim[k]) l = Q.lim[k];
                if (l < -Q.lim[k]) l = -Q.lim[k];
                const double d = l - ld[k];
                ld[k] = l;
                if (k < 3) vB[ax] += Q.invMB * d;
                else
                    for (int j = 0; j < 3; ++j) wB[j] += Q.IBinv[j][ax] * d;
                if (fabs(d) > dmax) dmax = fabs(d);
                if (fabs(l) > lmax) lmax = fabs(l);
            }
        }
        if (dmax <= 1e-15 * lmax || lmax == 0.0) return sweep + 1;
    }
    return -nsw;
}

// one wave per zone (grid = zones, 64 threads)
__global__ void __launch_bounds__(64) k_macro_solve(DevBuffers b, StepParams p, MacroArgs a, MacroZone* mz,
                                                    tr_macro_result* out)
{
    __shared__ SolveShared sh;
    const int z = blockIdx.x, lane = threadIdx.x;
    const MacroZone& Z = mz[z];
    const BodyDev& B = b.bodies[a.body[z]];
    const double dt = p.dt_d;
    const tr_macro_equipment* E = a.has_eq[z] ? &a.eq[z] : nullptr;
    {
        unsigned long long* ow = reinterpret_cast<unsigned long long*>(&sh.o);
        for (int k = lane; k < (int)(sizeof(tr_macro_result) / 8); k += 64) ow[k] = 0ull;
    }
    __syncthreads();
    if (lane == 0) {
        tr_macro_result& o = sh.o;
        o.zone = B.user_id;
        const double* S = Z.mom;
        const double M = S[0];
        o.M = M;
        sh.run = (M > 0.0) && a.eligible[z];
        if (sh.run) {
            // the aggregate (Eqs. aggregate_mass .. aggregate_rot_vel, read R14)
            double xA[3] = {S[1] / M, S[2] / M, S[3] / M}, vA[3] = {S[4] / M, S[5] / M, S[6] / M};
            double Cxx = S[7] - M * xA[0] * xA[0], Cyy = S[8] - M * xA[1] * xA[1], Czz = S[9] - M * xA[2] * xA[2];
            double Cxy = S[10] - M * xA[0] * xA[1], Cxz = S[11] - M * xA[0] * xA[2], Cyz = S[12] - M * xA[1] * xA[2];
            double tr = Cxx + Cyy + Czz;
            double I[3][3] = {{S[16] + tr - Cxx, -Cxy, -Cxz}, {-Cxy, S[16] + tr - Cyy, -Cyz},
                              {-Cxz, -Cyz, S[16] + tr - Czz}};
            double L[3] = {S[13] - (xA[1] * S[6] - xA[2] * S[5]) + S[17], S[14] - (xA[2] * S[4] - xA[0] * S[6]) + S[18],
                           S[15] - (xA[0] * S[5] - xA[1] * S[4]) + S[19]};
            MacroSys& Q = sh.S;
            inv3(I, Q.Iinv);
            double wA[3];
            mat3v(Q.Iinv, L, wA);
            for (int k = 0; k < 3; ++k) { o.x[k] = xA[k]; o.v0[k] = vA[k]; o.w0[k] = wA[k]; }
            Q.invM = 1.0 / M;
            sh.Lc = cbrt(Z.vol);
            // the reduced points of each interface: +e1, -e1, +e2, -e2, each kept once
            int np = 0;
            for (int q = 0; q < 2; ++q) {
                o.n_cand[q] = (int64_t)Z.cnt[q];
                o.area[q] = Z.area[q];
                o.gamma[q] = Z.area[q] > 0.0 ? sh.Lc / ((q == 0 ? a.mp.cas_ab : a.mp.cas_ac) * a.mp.E_b * Z.area[q] *
                                                       dt * dt)
                                             : 0.0;
                if (Z.cnt[q] == 0) continue;
                double n[3], dfail;
                iface_normal(b, a, z, q, n, dfail);
                int m = 0;
                unsigned long long chosen[4];
                for (int d = 0; d < 4; ++d) {
                    bool dup = false;
                    for (int j = 0; j < m; ++j) dup |= chosen[j] == Z.kmin[q][d];
                    if (dup) continue;
                    chosen[m] = Z.kmin[q][d];
                    key_point(b, p, a, z, q, chosen[m], o.p[4 * q + m]);
                    for (int k = 0; k < 3; ++k) o.n[4 * q + m][k] = n[k];
                    o.src[4 * q + m] = (int64_t)(chosen[m] >> 16);
                    sh.map[np++] = 4 * q + m;
                    ++m;
                }
                o.n_points[q] = m;
            }
            // Eq. mdb:eqAgg in impulse form with the rows of Eqs. aggregateNormal
            // and aggregateTangent; with a dynamic equipment (Eq. mdb:eqEq) its
            // body and drive rows join the system
            Q.np = np;
            Q.ndof = E ? 12 : 6;
            Q.invMB = 0.0;
            Q.gd = 1.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) Q.IBinv[i][j] = 0.0;
            for (int k = 0; k < 6; ++k) { Q.target[k] = 0.0; Q.lim[k] = 0.0; }
            for (int k = 0; k < 3; ++k) {
                sh.w0[k] = vA[k] + dt * a.g[k];
                sh.w0[3 + k] = wA[k];
                sh.w0[6 + k] = B.linvel[k];
                sh.w0[9 + k] = B.angvel[k];
            }
            if (E) {
                Q.invMB = 1.0 / E->mass;
                double R[9], Iw[3][3];
                quat_to_R(B.quat, R);
                const double* J6 = E->inertia;
                const double Ib[3][3] = {{J6[0], J6[3], J6[4]}, {J6[3], J6[1], J6[5]}, {J6[4], J6[5], J6[2]}};
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        double acc = 0.0;
                        for (int k = 0; k < 3; ++k)
                            for (int l = 0; l < 3; ++l) acc += R[i * 3 + k] * Ib[k][l] * R[j * 3 + l];
                        Iw[i][j] = acc;
                    }
                inv3(Iw, Q.IBinv);
                for (int k = 0; k < 3; ++k) {
                    sh.w0[6 + k] = B.linvel[k] + dt * a.g[k];
                    Q.target[k] = E->v_target[k];
                    Q.target[3 + k] = E->w_target[k];
                    Q.lim[k] = E->f_max * dt;
                    Q.lim[3 + k] = E->t_max * dt;
                }
                Q.gd = E->gamma_drive;
            }
            for (int c = 0; c < np; ++c) {
                const int k8 = sh.map[c], q = k8 / 4;
                Q.onB[c] = q == 0 && E != nullptr;
                for (int k = 0; k < 3; ++k) {
                    Q.rr[c][k] = o.p[k8][k] - xA[k];
                    Q.rb[c][k] = o.p[k8][k] - B.pos[k];
                    Q.n[c][k] = o.n[k8][k];
                    Q.uo[c][k] = 0.0;
                }
                if (q == 0 && !E) {
                    double t[3];
                    cross3d(B.angvel, Q.rb[c], t);
                    for (int k = 0; k < 3; ++k) Q.uo[c][k] = B.linvel[k] + t[k];
                }
                double t1[3], t2[3];
                plane_axes(o.n[k8], t1, t2);
                sh.Wn[c] = point_w(Q.invM, Q.Iinv, Q.rr[c], o.n[k8], o.n[k8]);
                sh.Wt[c] = 0.5 * (point_w(Q.invM, Q.Iinv, Q.rr[c], t1, t1) + point_w(Q.invM, Q.Iinv, Q.rr[c], t2, t2));
                if (Q.onB[c]) {
                    sh.Wn[c] += point_w(Q.invMB, Q.IBinv, Q.rb[c], o.n[k8], o.n[k8]);
                    sh.Wt[c] += 0.5 * (point_w(Q.invMB, Q.IBinv, Q.rb[c], t1, t1) +
                                       point_w(Q.invMB, Q.IBinv, Q.rb[c], t2, t2));
                }
                Q.lo[c] = -a.mp.c_b * o.area[q] * dt / (double)o.n_points[q];
                Q.mu[c] = q == 0 ? a.mp.mu_ab : a.mp.mu_ac;
                Q.gam[c] = o.gamma[q];
            }
            double scale = dt * sqrt(dot3d(a.g, a.g)) + 1e-300;
            for (int k = 0; k < Q.ndof; ++k) scale += (k % 6) < 3 ? fabs(sh.w0[k]) : sh.Lc * fabs(sh.w0[k]);
            sh.scale = scale;
        }
    }
    __syncthreads();
    if (sh.run) {
        // the fixed point of the rows directly: damped semismooth Newton on the
        // bodies' velocities (six, or twelve with a dynamic equipment) with each
        // row's impulse in closed form, then the rows' projected Gauss-Seidel
        // from there until no impulse changes (one or two sweeps when Newton
        // converged).  Where Newton stalls (at a kink of the projections the
        // residual's norm is a poor merit: no step of eight halvings lowers
        // it), a few Gauss-Seidel sweeps from its point move the active set
        // and Newton restarts from where they end.
        constexpr int kRounds = 8, kRoundSweeps = 8, kHalvings = 8;
        const int nd = sh.S.ndof, np = sh.S.np;
        if (lane < nd) sh.w[lane] = sh.w0[lane];
        int its = 0, sweeps = 0;
        for (int round = 0; round < kRounds; ++round) {
            __syncthreads();
            eval_G(sh, sh.w, sh.G, true);
            if (lane == 0) sh.g = gnorm(sh.G, nd, sh.Lc);
            __syncthreads();
            for (int it = 0; it < 100; ++it) {
                if (!(sh.g > 1e-15 * sh.scale)) break;
                if (lane < nd) sh.d[lane] = -sh.G[lane];
                __syncthreads();
                if (!lu_solve(sh, nd)) break;
                double step = 1.0;
                bool took = false;
                for (int ls = 0; ls < kHalvings; ++ls, step *= 0.5) {
                    if (lane < nd) sh.wt[lane] = sh.w[lane] + step * sh.d[lane];
                    __syncthreads();
                    eval_G(sh, sh.wt, sh.Gt, false);
                    if (lane == 0) {
                        const double gt = gnorm(sh.Gt, nd, sh.Lc);
                        sh.ok = gt < (1.0 - 1e-4 * step) * sh.g;
                        if (sh.ok) sh.g = gt;
                    }
                    __syncthreads();
                    if (sh.ok) {
                        took = true;
                        break;
                    }
                }
                if (!took) break;
                ++its;
                if (lane < nd) sh.w[lane] = sh.wt[lane];
                __syncthreads();
                eval_G(sh, sh.w, sh.G, true);
                if (lane == 0) sh.g = gnorm(sh.G, nd, sh.Lc);
                __syncthreads();
            }
            // the impulses and velocities at the Newton point (the last
            // evaluation may have been a rejected trial)
            eval_G(sh, sh.w, sh.G, false);
            if (lane == 0) {
                const MacroSys& Q = sh.S;
                for (int c = 0; c < np; ++c)
                    for (int k = 0; k < 4; ++k) sh.lam[c][k] = sh.lamp[c][k];
                double t[3];
                for (int k = 0; k < 6; ++k) sh.ld[k] = E ? sh.Fd[k] : 0.0;
                mat3v(Q.Iinv, sh.F + 3, t);
                for (int k = 0; k < 3; ++k) { sh.V[k] = sh.w0[k] + Q.invM * sh.F[k]; sh.V[3 + k] = sh.w0[3 + k] + t[k]; }
                if (E) {
                    mat3v(Q.IBinv, sh.F + 9, t);
                    for (int k = 0; k < 3; ++k) {
                        sh.V[6 + k] = sh.w0[6 + k] + Q.invMB * sh.F[6 + k];
                        sh.V[9 + k] = sh.w0[9 + k] + t[k];
                    }
                } else {
                    for (int k = 0; k < 3; ++k) { sh.V[6 + k] = B.linvel[k]; sh.V[9 + k] = B.angvel[k]; }
                }
                sh.again = 0;
                if (sh.g > 1e-15 * sh.scale && round + 1 < kRounds) {
                    const int r = pgs_sweeps(sh, E != nullptr, kRoundSweeps);
                    sweeps += r > 0 ? r : -r;
                    if (r < 0) sh.again = 1;
                    else sh.again = 2;  // the sweeps met the stopping rule
                    if (r < 0)
                        for (int k = 0; k < nd; ++k) sh.w[k] = sh.V[k];
                }
            }
            __syncthreads();
            if (sh.again != 1) break;
        }
        if (lane == 0) {
            const MacroSys& Q = sh.S;
            tr_macro_result& o = sh.o;
            if (sh.again != 2) {
                const int r = pgs_sweeps(sh, E != nullptr, 200000);
                sweeps += r > 0 ? r : -r;
            }
            const double* vv = sh.V;
            const double* ww = sh.V + 3;
            const double* vB = sh.V + 6;
            const double* wB = sh.V + 9;
            const double* ld = sh.ld;
            double t[3];
            o.sweeps = its + sweeps;
            for (int k = 0; k < 3; ++k) {
                o.v[k] = vv[k]; o.w[k] = ww[k]; o.force[k] = 0.0; o.torque[k] = 0.0;
                o.v_b[k] = vB[k]; o.w_b[k] = wB[k];
            }
            for (int k = 0; k < 6; ++k) o.lam_drive[k] = ld[k];
            for (int c = 0; c < np; ++c) {
                const int k8 = sh.map[c];
                for (int k = 0; k < 4; ++k) o.lam[k8][k] = sh.lam[c][k];
                if (k8 >= 4) continue;
                double J[3];
                for (int k = 0; k < 3; ++k) J[k] = sh.lam[c][0] * Q.n[c][k] + sh.lam[c][1 + k];
                for (int k = 0; k < 3; ++k) o.force[k] -= J[k] / dt;
                cross3d(Q.rb[c], J, t);
                for (int k = 0; k < 3; ++k) o.torque[k] -= t[k] / dt;
            }
        }
        __syncthreads();
    }
    const unsigned long long* ow = reinterpret_cast<const unsigned long long*>(&sh.o);
    unsigned long long* gw = reinterpret_cast<unsigned long long*>(&out[z]);
    for (int k = lane; k < (int)(sizeof(tr_macro_result) / 8); k += 64) gw[k] = ow[k];
}

// clears the zone sums and poses each zone's half-spaces once
__global__ void k_macro_clear(DevBuffers b, MacroArgs a, MacroZone* mz)
{
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= a.n_zones) return;
    MacroZone& Z = mz[z];
    const BodyDev& B = b.bodies[a.body[z]];
    Z.nplanes = B.nplanes;
    for (int q = 0; q < B.nplanes; ++q) plane_world(B, q, Z.wpl[q], Z.wpl[q][3]);
    for (int k = 0; k < kZoneMoments; ++k) Z.mom[k] = 0.0;
    Z.vol = 0.0;
    for (int q = 0; q < 2; ++q) {
        Z.cnt[q] = 0;
        Z.area[q] = 0.0;
        for (int d = 0; d < 4; ++d) {
            Z.vmax[q][d] = 0ull;
            Z.kmin[q][d] = ~0ull;
        }
    }
}

}  // namespace

void launch_macro(const DevBuffers& b, const StepParams& p, const MacroArgs& a, MacroZone* mz, tr_macro_result* out,
                  hipStream_t s)
{
    if (a.n_zones <= 0) return;
    hipLaunchKernelGGL(k_macro_clear, dim3(1), dim3(64), 0, s, b, a, mz);
    if (a.n > 0) {
        const unsigned g = (unsigned)((a.n + 255) / 256);
        hipLaunchKernelGGL(k_macro_pass1, dim3(g), dim3(256), 0, s, b, p, a, mz);
        hipLaunchKernelGGL(k_macro_pass2, dim3(g), dim3(256), 0, s, b, p, a, mz);
    }
    hipLaunchKernelGGL(k_macro_solve, dim3((unsigned)a.n_zones), dim3(64), 0, s, b, p, a, mz, out);
}

}  // namespace trk
