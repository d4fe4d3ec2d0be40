// terrain_voxels.hip -- gfx950 kernels of the mesoscale voxel workload.
//
// Fields on a voxel grid beside the particle step:
//   coarse-grain      particle mass and momentum into voxel densities (FP64
//                     atomics), velocity u = p / rho (Eq. cg_velocity)
//   advect            conserved donor-cell advection of fluidized mass
//                     (Eq. advection), 16 x 16-column tiles marching through
//                     runs of planes
//   convert cut       solid above the predicted zone's bottom becomes fluid
//   convert deposit   particle-free fluid outside the zones becomes solid at
//                     the column's surface (tiles of 16 columns on LDS)
//   surface           Eq. surface per column, into the terrain heightfield
//   grow              particles grow from their voxel's fluid (Eq. eqmotmb)
//   form              new particles from the fluid inside the zones
//   settle            particles at rest outside the zones back to fluid
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "terrain_internal.h"

namespace trk {

constexpr int kBlk = 256;

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Mesoscale voxel fields: coarse-graining (Eq. cg_velocity) and the conserved
// advection of fluidized mass (Eq. advection)
// ---------------------------------------------------------------------------
__global__ void k_fill_f64(double* a, int64_t n, double v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// one thread per particle of the env: its mass and momentum into the voxels
__global__ void k_coarse_grain(DevBuffers b, EnvDev E, tr_voxel_grid g, int kernel, double R, double* rho,
                               double* mom)
{
#pragma clang fp contract(off)
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= E.n) return;
    const int sl = E.slot_begin + a;
    const float4 xf = b.xr[sl], vf = vel_at(b.vw, sl);
    const double x[3] = {xf.x, xf.y, xf.z}, v[3] = {vf.x, vf.y, vf.z};
    const double r = xf.w;
    const double m = (double)b.rho[sl] * (4.0 / 3.0) * 3.14159265358979323846 * r * r * r;
    const int dims[3] = {g.nx, g.ny, g.nz};
    if (kernel == TR_CG_HEAVISIDE) {
        const double V0 = g.l0 * g.l0 * g.l0;
        int c[3];
        for (int k = 0; k < 3; ++k) {
            const double f = floor((x[k] - g.origin[k]) / g.l0);
            if (!(f >= 0.0 && f < (double)dims[k])) return;
            c[k] = (int)f;
        }
        const int64_t id = ((int64_t)c[2] * g.ny + c[1]) * g.nx + c[0];
        atomicAdd(&rho[id], m / V0);
        for (int k = 0; k < 3; ++k) atomicAdd(&mom[3 * id + k], m * v[k] / V0);
        return;
    }
    const double sq = sqrt(2.0 * 3.14159265358979323846) * R;
    const double norm = 1.0 / (sq * sq * sq);
    int lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        const double fl = ceil((x[k] - 3.0 * R - g.origin[k]) / g.l0 - 0.5);
        const double fh = floor((x[k] + 3.0 * R - g.origin[k]) / g.l0 - 0.5);
        lo[k] = fl < 0.0 ? 0 : (int)fl;
        hi[k] = fh > (double)(dims[k] - 1) ? dims[k] - 1 : (int)fh;
    }
    for (int kz = lo[2]; kz <= hi[2]; ++kz)
        for (int jy = lo[1]; jy <= hi[1]; ++jy)
            for (int ix = lo[0]; ix <= hi[0]; ++ix) {
                const double y[3] = {g.origin[0] + (ix + 0.5) * g.l0 - x[0], g.origin[1] + (jy + 0.5) * g.l0 - x[1],
                                     g.origin[2] + (kz + 0.5) * g.l0 - x[2]};
                const double r2 = (y[0] * y[0] + y[1] * y[1]) + y[2] * y[2];
                if (r2 > 9.0 * R * R) continue;
                const double z = norm * exp(-r2 / (2.0 * R * R));
                const int64_t id = ((int64_t)kz * g.ny + jy) * g.nx + ix;
                atomicAdd(&rho[id], m * z);
                for (int k = 0; k < 3; ++k) atomicAdd(&mom[3 * id + k], m * v[k] * z);
            }
}

__global__ void k_cg_velocity(int64_t nv, const double* rho, const double* mom, double* u)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    for (int k = 0; k < 3; ++k) u[3 * i + k] = rho[i] > 0.0 ? mom[3 * i + k] / rho[i] : 0.0;
}

void launch_coarse_grain(const DevBuffers& b, const EnvDev& E, const tr_voxel_grid& g, int kernel, double R,
                         double* rho, double* mom, double* u, hipStream_t s)
{
    const int64_t nv = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)cdiv(nv, kBlk)), dim3(kBlk), 0, s, rho, nv, 0.0);
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)cdiv(3 * nv, kBlk)), dim3(kBlk), 0, s, mom, 3 * nv, 0.0);
    if (E.n > 0)
        hipLaunchKernelGGL(k_coarse_grain, dim3((unsigned)cdiv(E.n, kBlk)), dim3(kBlk), 0, s, b, E, g, kernel, R, rho,
                           mom);
    if (u) hipLaunchKernelGGL(k_cg_velocity, dim3((unsigned)cdiv(nv, kBlk)), dim3(kBlk), 0, s, nv, rho, mom, u);
}

// A block takes a 16 x 16 tile of columns through a run of kc planes: each
// plane of the tile (with a one-voxel halo in x and y) goes through LDS, and
// the planes above and below stay in registers, so every voxel's mass and
// velocity are read once (the halo aside).  The loads of plane k + 1 are in
// flight while plane k is computed (two LDS buffers, one barrier per plane).
// Each block leaves the largest Courant number it met in bmax[b]; one block
// reduces them (device-scope atomics to one address cost about 10 ns each).
constexpr int kAT = 16;  // tile edge (kAT * kAT == kBlk)

struct PlaneRegs {
    double mf, ux, uy, uz;  // the thread's own voxel
    double hx_mf, hx_u;     // across the tile's x edge (tx == 0: i - 1, tx == kAT - 1: i + 1)
    double hy_mf, hy_u;     // across the tile's y edge
};

__device__ inline void load_plane(const tr_voxel_grid& g, const double* u, const double* mf, int i, int j, int k,
                                  int tx, int ty, PlaneRegs& r)
{
    r = PlaneRegs{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (k < 0 || k >= g.nz || i >= g.nx || j >= g.ny) return;
    const int64_t plane = (int64_t)k * g.nx * g.ny;
    const int64_t id = plane + (int64_t)j * g.nx + i;
    r.mf = mf[id];
    r.ux = u[3 * id];
    r.uy = u[3 * id + 1];
    r.uz = u[3 * id + 2];
    const int hi_ = tx == 0 ? i - 1 : (tx == kAT - 1 ? i + 1 : -1);
    if (hi_ >= 0 && hi_ < g.nx) {
        const int64_t h = plane + (int64_t)j * g.nx + hi_;
        r.hx_mf = mf[h];
        r.hx_u = u[3 * h];
    }
    const int hj = ty == 0 ? j - 1 : (ty == kAT - 1 ? j + 1 : -1);
    if (hj >= 0 && hj < g.ny) {
        const int64_t h = plane + (int64_t)hj * g.nx + i;
        r.hy_mf = mf[h];
        r.hy_u = u[3 * h + 1];
    }
}

__global__ void __launch_bounds__(kBlk) k_advect(tr_voxel_grid g, double dt, const double* u, const double* mf,
                                                 double* out, double* bmax, int tiles_x, int tiles_y, int kc,
                                                 int nblocks, int per)
{
#pragma clang fp contract(off)
    __shared__ double smf[2][kAT + 2][kAT + 2], sux[2][kAT + 2][kAT + 2], suy[2][kAT + 2][kAT + 2];
    const int tx = threadIdx.x % kAT, ty = threadIdx.x / kAT;
    // blocks go to the XCDs in turn; XCD x takes the contiguous run
    // [x per, (x + 1) per) of (tile x, tile y, chunk) order, so neighbouring
    // tiles, which read each other's edges as halo, share an L2
    const int lb = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
    const int bx = lb % tiles_x, by = (lb / tiles_x) % tiles_y, bz = lb / (tiles_x * tiles_y);
    const int i = bx * kAT + tx, j = by * kAT + ty;
    // (a block past the last tile has an empty run of planes)
    const int k0 = bz * kc, k1 = lb < nblocks ? min(k0 + kc, g.nz) : k0;
    const bool live = i < g.nx && j < g.ny;
    PlaneRegs prv, cur, nxt;
    load_plane(g, u, mf, i, j, k0 < k1 ? k0 - 1 : -1, tx, ty, prv);
    load_plane(g, u, mf, i, j, k0 < k1 ? k0 : -1, tx, ty, cur);
    double cmax = 0.0;
    for (int k = k0; k < k1; ++k) {
        const int bf = k & 1;
        smf[bf][ty + 1][tx + 1] = cur.mf;
        sux[bf][ty + 1][tx + 1] = cur.ux;
        suy[bf][ty + 1][tx + 1] = cur.uy;
        if (tx == 0) { smf[bf][ty + 1][0] = cur.hx_mf; sux[bf][ty + 1][0] = cur.hx_u; }
        if (tx == kAT - 1) { smf[bf][ty + 1][kAT + 1] = cur.hx_mf; sux[bf][ty + 1][kAT + 1] = cur.hx_u; }
        if (ty == 0) { smf[bf][0][tx + 1] = cur.hy_mf; suy[bf][0][tx + 1] = cur.hy_u; }
        if (ty == kAT - 1) { smf[bf][kAT + 1][tx + 1] = cur.hy_mf; suy[bf][kAT + 1][tx + 1] = cur.hy_u; }
        load_plane(g, u, mf, i, j, k + 1, tx, ty, nxt);
        __syncthreads();
        if (live) {
            // the same faces, operations and order as a voxel-by-voxel sweep:
            // inflow through the lower faces (z, y, x), then outflow through the
            // upper ones (x, y, z); per face (lower voxel a, upper b):
            // u_f = (u_a + u_b) / 2, flux dt u_f m_donor / l0
            const double mi = cur.mf;
            const double ui[3] = {cur.ux, cur.uy, cur.uz};
            const bool lo[3] = {i > 0, j > 0, k > 0};
            const bool hi[3] = {i + 1 < g.nx, j + 1 < g.ny, k + 1 < g.nz};
            const double um[3] = {sux[bf][ty + 1][tx], suy[bf][ty][tx + 1], prv.uz};
            const double mm[3] = {smf[bf][ty + 1][tx], smf[bf][ty][tx + 1], prv.mf};
            const double up[3] = {sux[bf][ty + 1][tx + 2], suy[bf][ty + 2][tx + 1], nxt.uz};
            const double mp[3] = {smf[bf][ty + 1][tx + 2], smf[bf][ty + 2][tx + 1], nxt.mf};
            double m = mi;
#pragma unroll
            for (int d = 2; d >= 0; --d)
                if (lo[d]) {
                    const double uf = 0.5 * (um[d] + ui[d]);
                    m += dt * uf * (uf > 0.0 ? mm[d] : mi) / g.l0;
                }
#pragma unroll
            for (int d = 0; d < 3; ++d)
                if (hi[d]) {
                    const double uf = 0.5 * (ui[d] + up[d]);
                    m -= dt * uf * (uf > 0.0 ? mi : mp[d]) / g.l0;
                    cmax = fmax(cmax, fabs(uf) * dt / g.l0);
                }
            out[(int64_t)k * g.nx * g.ny + (int64_t)j * g.nx + i] = m;
        }
        prv = cur;
        cur = nxt;
    }
    __shared__ double wmax[kBlk / 64];
    for (int o = 32; o > 0; o >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, o));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = cmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) cmax = fmax(cmax, wmax[w]);
        bmax[blockIdx.x] = cmax;
    }
}

// one block: the largest of n per-block maxima, as its bit pattern
__global__ void k_max_reduce(const double* bmax, int n, unsigned long long* bits)
{
    double v = 0.0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) v = fmax(v, bmax[k]);
    __shared__ double wmax[kBlk / 64];
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) v = fmax(v, wmax[w]);
        *bits = (unsigned long long)__double_as_longlong(v);
    }
}

// tiles of kAT x kAT columns, each through chunks of kc planes: at most
// kAdvectTargetBlocks blocks unless the tiles alone are more
static void advect_shape(const tr_voxel_grid& g, int& tiles_x, int& tiles_y, int& kc, int& chunks)
{
    tiles_x = (int)cdiv(g.nx, kAT);
    tiles_y = (int)cdiv(g.ny, kAT);
    const int64_t tiles = (int64_t)tiles_x * tiles_y;
    int64_t want = std::max<int64_t>(1, kAdvectTargetBlocks / tiles);
    want = std::min<int64_t>(want, cdiv(g.nz, 16));  // at least 16 planes a chunk
    want = std::max<int64_t>(want, 1);
    kc = (int)cdiv(g.nz, want);
    chunks = (int)cdiv(g.nz, kc);
}

int64_t advect_blocks(const tr_voxel_grid& g)
{
    int tx, ty, kc, ch;
    advect_shape(g, tx, ty, kc, ch);
    return 8 * cdiv((int64_t)tx * ty * ch, 8);
}

void launch_advect(const tr_voxel_grid& g, double dt, const double* u, const double* mf_in, double* mf_out,
                   double* bmax, unsigned long long* cfl_bits, hipStream_t s)
{
    int tiles_x, tiles_y, kc, chunks;
    advect_shape(g, tiles_x, tiles_y, kc, chunks);
    const int64_t nb = (int64_t)tiles_x * tiles_y * chunks;
    const int per = (int)cdiv(nb, 8);
    hipLaunchKernelGGL(k_advect, dim3((unsigned)(8 * per)), dim3(kBlk), 0, s, g, dt, u, mf_in, mf_out, bmax, tiles_x,
                       tiles_y, kc, (int)nb, per);
    if (cfl_bits) hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(kBlk), 0, s, bmax, 8 * per, cfl_bits);
}

// ---------------------------------------------------------------------------
// Conversion between resting solid and fluidized mass: one thread per column,
// its voxels in increasing height (the columns are independent)
// ---------------------------------------------------------------------------
__global__ void k_surface(tr_voxel_grid g, const double* phi, double* h, float* hf)
{
#pragma clang fp contract(off)
    const int64_t nxy = (int64_t)g.nx * g.ny;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nxy) return;
    double z = g.origin[2];
    // Eq. surface at the top-most voxel with solid, searched downwards kChunk
    // voxels at a time with every load in flight
    constexpr int kChunk = 8;
    bool found = false;
    for (int k1 = g.nz - 1; k1 >= 0 && !found; k1 -= kChunk) {
        double fc[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) fc[q] = k1 - q >= 0 ? phi[(int64_t)(k1 - q) * nxy + c] : 0.0;
        for (int q = 0; q < kChunk && !found; ++q)
            if (fc[q] > 0.0) {
                const int k = k1 - q;
                const double zc = g.origin[2] + (k + 0.5) * g.l0;
                z = zc + (fc[q] - 0.5) * g.l0;
                found = true;
            }
    }
    if (h) h[c] = z;
    if (hf) hf[c] = (float)z;
}

// the z range of the vertical line through (x, y) inside a wedge: its lower bound
__device__ inline bool wedge_bottom(const WedgeDev& w, double x, double y, double& zlo)
{
#pragma clang fp contract(off)
    double lo = -INFINITY, hi = INFINITY;
    if (w.n == 0) return false;
    for (int p = 0; p < w.n; ++p) {
        const double a = w.planes[p][2], b = w.planes[p][3] - w.planes[p][0] * x - w.planes[p][1] * y;
        if (a > 0.0) hi = fmin(hi, b / a);
        else if (a < 0.0) lo = fmax(lo, b / a);
        else if (b < 0.0) return false;
    }
    if (!(lo <= hi) || lo == -INFINITY) return false;
    zlo = lo;
    return true;
}

__device__ inline bool in_wedge_set(const WedgeSet& ws, double x, double y, double z)
{
#pragma clang fp contract(off)
    for (int r = 0; r < ws.n_ranges; ++r)
        for (int k = 0; k < ws.cnt[r]; ++k) {
            const WedgeDev& w = ws.base[ws.off[r] + k];
            if (w.n == 0) continue;
            bool in = true;
            for (int p = 0; p < w.n && in; ++p)
                if (w.planes[p][0] * x + w.planes[p][1] * y + w.planes[p][2] * z - w.planes[p][3] > 0.0) in = false;
            if (in) return true;
        }
    return false;
}

__global__ void k_convert_cut(tr_voxel_grid g, double rho_b, WedgeSet ws, double* phi, const double* wc, double* mf,
                              double* total)
{
#pragma clang fp contract(off)
    const int64_t nxy = (int64_t)g.nx * g.ny;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nxy) return;
    const int i = (int)(c % g.nx), j = (int)(c / g.nx);
    const double x = g.origin[0] + (i + 0.5) * g.l0, y = g.origin[1] + (j + 0.5) * g.l0;
    double zcut = INFINITY, lo;
    for (int r = 0; r < ws.n_ranges; ++r)
        for (int k = 0; k < ws.cnt[r]; ++k)
            if (wedge_bottom(ws.base[ws.off[r] + k], x, y, lo)) zcut = fmin(zcut, lo);
    if (zcut == INFINITY) return;
    const double V0 = g.l0 * g.l0 * g.l0;
    double sum = 0.0;
    // voxels a whole voxel or more below the cut keep their solid (occupancy
    // is at most 1): start one voxel below the cut's, then read kChunk voxels
    // at a time with every load in flight
    const double kc = floor((zcut - g.origin[2]) / g.l0) - 1.0;
    const int k_start = kc <= 0.0 ? 0 : (kc >= (double)g.nz ? g.nz : (int)kc);
    constexpr int kChunk = 8;
    for (int k0 = k_start; k0 < g.nz; k0 += kChunk) {
        double fc[kChunk], wcc[kChunk], mc[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) {
            const bool in = k0 + q < g.nz;
            const int64_t id = (int64_t)(k0 + q) * nxy + c;
            fc[q] = in ? phi[id] : 0.0;
            wcc[q] = in ? wc[id] : 0.0;
            mc[q] = in ? mf[id] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kChunk; ++q) {
            const int k = k0 + q;
            if (k >= g.nz) break;
            double t = (zcut - (g.origin[2] + k * g.l0)) / g.l0;  // occupancy below the cut
            t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
            if (fc[q] > t) {
                const int64_t id = (int64_t)k * nxy + c;
                const double dm = wcc[q] * rho_b * V0 * (fc[q] - t);
                mf[id] = mc[q] + dm;
                sum += dm;
                phi[id] = t;
            }
        }
    }
    if (total && sum > 0.0) atomicAdd(total, sum);
}

__global__ void k_convert_deposit(tr_voxel_grid g, double rho_b, double w_dep, WedgeSet ws, const double* rho_p,
                                  double* phi, double* wc, double* mf, double* total)
{
#pragma clang fp contract(off)
    const int64_t nxy = (int64_t)g.nx * g.ny;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nxy) return;
    const int i = (int)(c % g.nx), j = (int)(c / g.nx);
    const double x = g.origin[0] + (i + 0.5) * g.l0, y = g.origin[1] + (j + 0.5) * g.l0;
    const double V0 = g.l0 * g.l0 * g.l0;
    double sum = 0.0;
    // the first voxel of the column that is not full: fills only raise the
    // occupancy, so it never moves down and each search resumes from the last
    int kfree = 0;
    int kc = -1;               // the last voxel filled, its occupancy and compaction as written
    double fc = 0.0, wcc = 0.0;
    // the column is read kChunk voxels at a time (independent loads in
    // flight); a voxel's own deposit changes only phi and wc, and mf of that
    // voxel alone, so the values read ahead stay current
    constexpr int kChunk = 8;
    for (int k0 = 0; k0 < g.nz; k0 += kChunk) {
        double mc[kChunk], rc[kChunk];
#pragma unroll
        for (int t = 0; t < kChunk; ++t) {
            const bool in = k0 + t < g.nz;
            mc[t] = in ? mf[(int64_t)(k0 + t) * nxy + c] : 0.0;
            rc[t] = in ? rho_p[(int64_t)(k0 + t) * nxy + c] : 0.0;
        }
        for (int t = 0; t < kChunk; ++t) {
            const int k = k0 + t;
            if (!(mc[t] > 0.0) || rc[t] != 0.0 || in_wedge_set(ws, x, y, g.origin[2] + (k + 0.5) * g.l0)) continue;
            double m = mc[t];
            int kk = kfree;
            // the last voxel filled is held as written: when it is the first
            // non-full voxel no search is needed
            for (bool found = kk == kc && fc < 1.0; !found && kk < g.nz;) {  // kChunk at a time
                double pc[kChunk];
#pragma unroll
                for (int q = 0; q < kChunk; ++q) pc[q] = kk + q < g.nz ? phi[(int64_t)(kk + q) * nxy + c] : 0.0;
                int q = 0;
                while (q < kChunk && pc[q] >= 1.0) ++q;
                found = q < kChunk;
                kk += q;
            }
            kk = kk < g.nz ? kk : g.nz;
            kfree = kk;
            while (m > 0.0 && kk < g.nz) {
                const int64_t id = (int64_t)kk * nxy + c;
                const bool held = kk == kc;
                const double f0 = held ? fc : phi[id];
                const double w0 = held ? wcc : wc[id];
                const double cap = (1.0 - f0) * w_dep * rho_b * V0;
                const double take = m < cap ? m : cap;
                const double f = take == cap ? 1.0 : f0 + take / (w_dep * rho_b * V0);
                const double before = w0 * rho_b * V0 * f0;
                const double wn = f0 > 0.0 ? (before + take) / (rho_b * V0 * f) : w_dep;
                wc[id] = wn;
                phi[id] = f;
                kc = kk;
                fc = f;
                wcc = wn;
                sum += take;
                m -= take;
                ++kk;
            }
            // every voxel below the last one filled is full
            if (kc >= kfree) kfree = fc < 1.0 ? kc : kc + 1;
            mf[(int64_t)k * nxy + c] = 0.0 + m;  // what finds the column full stays fluid
        }
    }
    if (total && sum > 0.0) atomicAdd(total, sum);
}

// The deposit on tiles of kTileCols neighbouring columns of at most kTileNz
// voxels.  Columns are strided by nx ny in memory, so a column read by one
// wave touches a cache line per voxel; the tile is read instead as whole
// lines (each wave instruction: 16 columns at 4 heights), with all of a
// thread's loads in flight at once.  The voxels whose fluid falls are marked
// in parallel (bit masks per column), as is each column's first non-full
// voxel; one thread per column then replays the fills over its marked voxels
// in increasing height, as the per-thread kernel does.  Fills start at the
// first non-full voxel and rarely climb far: occupancy and compaction of the
// kWin voxels from there are held in LDS (a fill beyond them reads and writes
// memory directly), which keeps the block's LDS small enough for six blocks
// per CU.  The block writes back what changed.
constexpr int kTileCols = 16;
constexpr int kTileNz = 128;
constexpr int kTileRows = kBlk / kTileCols;  // heights per pass
constexpr int kTileWords = kTileNz / 64;
constexpr int kWin = 32;

__global__ void __launch_bounds__(kBlk) k_convert_deposit_tile(tr_voxel_grid g, double rho_b, double w_dep,
                                                               WedgeSet ws, const double* rho_p, double* phi,
                                                               double* wc, double* mf, double* total)
{
#pragma clang fp contract(off)
    // (+1: a column's entries start two banks after the previous column's)
    __shared__ double M[kTileCols][kTileNz + 1], P[kTileCols][kWin + 1], W[kTileCols][kWin + 1];
    __shared__ unsigned long long mask[kTileCols][kTileWords];
    __shared__ int first_free[kTileCols], range[kTileCols][2];
    __shared__ double ssum[kTileCols];
    const int64_t nxy = (int64_t)g.nx * g.ny;
    const int col = threadIdx.x % kTileCols, row = threadIdx.x / kTileCols;
    const int64_t c = (int64_t)blockIdx.x * kTileCols + col;
    const bool live = c < nxy;
    const int nz = g.nz;
    const double x = g.origin[0] + ((int)(c % g.nx) + 0.5) * g.l0, y = g.origin[1] + ((int)(c / g.nx) + 0.5) * g.l0;
    if (threadIdx.x < kTileCols) {
        for (int w = 0; w < kTileWords; ++w) mask[threadIdx.x][w] = 0ull;
        first_free[threadIdx.x] = nz;
    }
    __syncthreads();
    // a thread's heights row, row + kTileRows, ...: all its loads in flight at once
    constexpr int kPer = kTileNz / kTileRows;
    double mv[kPer], rv[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int k = row + t * kTileRows;
        mv[t] = live && k < nz ? mf[(int64_t)k * nxy + c] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int k = row + t * kTileRows;
        rv[t] = mv[t] > 0.0 ? rho_p[(int64_t)k * nxy + c] : 1.0;
    }
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int k = row + t * kTileRows;
        if (k >= nz) continue;
        M[col][k] = mv[t];
        if (mv[t] > 0.0 && rv[t] == 0.0 && !in_wedge_set(ws, x, y, g.origin[2] + (k + 0.5) * g.l0))
            atomicOr(&mask[col][k >> 6], 1ull << (k & 63));
    }
    __syncthreads();
    bool work = false;
    for (int w = 0; w < kTileWords; ++w) work |= mask[col][w] != 0ull;
    work &= live;
    double pv[kPer], wv[kPer];
    if (work) {
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int k = row + t * kTileRows;
            pv[t] = k < nz ? phi[(int64_t)k * nxy + c] : 1.0;
            wv[t] = k < nz ? wc[(int64_t)k * nxy + c] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int k = row + t * kTileRows;
            if (k < nz && !(pv[t] >= 1.0)) atomicMin(&first_free[col], k);
        }
    }
    __syncthreads();
    const int ff = first_free[col];
    if (work) {
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int k = row + t * kTileRows;
            if (k < nz && k >= ff && k < ff + kWin) {
                P[col][k - ff] = pv[t];
                W[col][k - ff] = wv[t];
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < kTileCols) {
        double sum = 0.0;
        int klo = nz, khi = -1;
        if (work) {
            const double V0 = g.l0 * g.l0 * g.l0;
            // occupancy and compaction of voxel kk: LDS inside the window, memory above it
            auto pget = [&](int kk) { return kk < ff + kWin ? P[col][kk - ff] : phi[(int64_t)kk * nxy + c]; };
            int kfree = ff;  // the first voxel that is not full
            for (int w = 0; w < kTileWords; ++w) {
                unsigned long long mk = mask[col][w];
                while (mk) {
                    const int k = w * 64 + (__ffsll((long long)mk) - 1);
                    mk &= mk - 1;
                    double m = M[col][k];
                    int kk = kfree;
                    while (kk < nz && pget(kk) >= 1.0) ++kk;
                    kfree = kk;
                    klo = kk < klo ? kk : klo;
                    while (m > 0.0 && kk < nz) {
                        const bool in_win = kk < ff + kWin;
                        const int64_t id = (int64_t)kk * nxy + c;
                        const double f0 = in_win ? P[col][kk - ff] : phi[id];
                        const double w0 = in_win ? W[col][kk - ff] : wc[id];
                        const double cap = (1.0 - f0) * w_dep * rho_b * V0;
                        const double take = m < cap ? m : cap;
                        const double f = take == cap ? 1.0 : f0 + take / (w_dep * rho_b * V0);
                        const double before = w0 * rho_b * V0 * f0;
                        const double wn = f0 > 0.0 ? (before + take) / (rho_b * V0 * f) : w_dep;
                        if (in_win) {
                            W[col][kk - ff] = wn;
                            P[col][kk - ff] = f;
                        } else {
                            wc[id] = wn;
                            phi[id] = f;
                        }
                        khi = kk > khi ? kk : khi;
                        sum += take;
                        m -= take;
                        ++kk;
                    }
                    M[col][k] = 0.0 + m;  // what finds the column full stays fluid
                }
            }
        }
        range[col][0] = klo;
        range[col][1] = khi;
        ssum[col] = sum;
    }
    __syncthreads();
    if (work) {
        const int klo = range[col][0], khi = range[col][1];
        for (int k = row; k < nz; k += kTileRows) {
            const int64_t id = (int64_t)k * nxy + c;
            if ((mask[col][k >> 6] >> (k & 63)) & 1ull) mf[id] = M[col][k];
            if (k >= klo && k <= khi && k < ff + kWin) {  // (above the window: written by the fills)
                phi[id] = P[col][k - ff];
                wc[id] = W[col][k - ff];
            }
        }
    }
    if (total && threadIdx.x == 0) {  // one atomic per tile
        double s = 0.0;
        for (int q = 0; q < kTileCols; ++q) s += ssum[q];
        if (s > 0.0) atomicAdd(total, s);
    }
}

void launch_surface(const tr_voxel_grid& g, const double* phi, double* h, float* hf, hipStream_t s)
{
    const int64_t nxy = (int64_t)g.nx * g.ny;
    hipLaunchKernelGGL(k_surface, dim3((unsigned)cdiv(nxy, kBlk)), dim3(kBlk), 0, s, g, phi, h, hf);
}

void launch_convert_cut(const tr_voxel_grid& g, double rho_b, const WedgeSet& ws, double* phi, const double* wc,
                        double* mf, double* total, hipStream_t s)
{
    const int64_t nxy = (int64_t)g.nx * g.ny;
    if (total) hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, total, (int64_t)1, 0.0);
    hipLaunchKernelGGL(k_convert_cut, dim3((unsigned)cdiv(nxy, kBlk)), dim3(kBlk), 0, s, g, rho_b, ws, phi, wc, mf,
                       total);
}

void launch_convert_deposit(const tr_voxel_grid& g, double rho_b, double w_dep, const WedgeSet& ws,
                            const double* rho_p, double* phi, double* wc, double* mf, double* total, hipStream_t s)
{
    const int64_t nxy = (int64_t)g.nx * g.ny;
    if (total) hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, total, (int64_t)1, 0.0);
    if (g.nz <= kTileNz)
        hipLaunchKernelGGL(k_convert_deposit_tile, dim3((unsigned)cdiv(nxy, kTileCols)), dim3(kBlk), 0, s, g, rho_b,
                           w_dep, ws, rho_p, phi, wc, mf, total);
    else
        hipLaunchKernelGGL(k_convert_deposit, dim3((unsigned)cdiv(nxy, kBlk)), dim3(kBlk), 0, s, g, rho_b, w_dep, ws,
                           rho_p, phi, wc, mf, total);
}

// ---------------------------------------------------------------------------
// Particle growth from the fluidized mass of the particle's voxel (Eq. eqmotmb):
// bounds summed per voxel, shares applied, the fluid charged per voxel
// ---------------------------------------------------------------------------
__device__ inline int64_t voxel_index(const tr_voxel_grid& g, const float4& xr)
{
#pragma clang fp contract(off)
    const double x[3] = {xr.x, xr.y, xr.z};
    const int dims[3] = {g.nx, g.ny, g.nz};
    int c[3];
    for (int k = 0; k < 3; ++k) {
        const double f = floor((x[k] - g.origin[k]) / g.l0);
        if (!(f >= 0.0 && f < (double)dims[k])) return -1;
        c[k] = (int)f;
    }
    return ((int64_t)c[2] * g.ny + c[1]) * g.nx + c[0];
}

// the most a particle may gain over dt: 3 m d' dt / d, not past d_max
__device__ inline double growth_bound(double km, double r, double dt, double dpm, double d_max)
{
#pragma clang fp contract(off)
    const double m = km * r * r * r;
    const double m_max = km * (0.5 * d_max) * (0.5 * d_max) * (0.5 * d_max);
    double c = 3.0 * m * dpm * dt / (2.0 * r);
    if (m + c > m_max) c = m_max > m ? m_max - m : 0.0;
    return c;
}

__global__ void k_grow_caps(DevBuffers b, EnvDev E, tr_voxel_grid g, double dt, double dpm, double d_max,
                            double* cap_sum)
{
#pragma clang fp contract(off)
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= E.n) return;
    const int sl = E.slot_begin + a;
    const float4 xr = b.xr[sl];
    const int64_t v = voxel_index(g, xr);
    if (v < 0) return;
    const double km = (double)b.rho[sl] * (4.0 / 3.0) * 3.14159265358979323846;
    const double c = growth_bound(km, (double)xr.w, dt, dpm, d_max);
    if (c > 0.0) atomicAdd(&cap_sum[v], c);
}

__global__ void k_grow_apply(DevBuffers b, EnvDev E, tr_voxel_grid g, double dt, double dpm, double d_max,
                             const double* cap_sum, const double* mf, double* used)
{
#pragma clang fp contract(off)
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= E.n) return;
    const int sl = E.slot_begin + a;
    float4 xr = b.xr[sl];
    const int64_t v = voxel_index(g, xr);
    if (v < 0) return;
    const double km = (double)b.rho[sl] * (4.0 / 3.0) * 3.14159265358979323846;
    const double r = xr.w;
    const double c = growth_bound(km, r, dt, dpm, d_max);
    if (!(c > 0.0)) return;
    const double A = mf[v] > 0.0 ? mf[v] : 0.0;
    const double share = cap_sum[v] <= A ? c : c * (A / cap_sum[v]);
    if (!(share > 0.0)) return;
    const double m = km * r * r * r;
    const float r_new = fminf((float)cbrt((m + share) / km), (float)(0.5 * d_max));
    if (!(r_new > xr.w)) return;
    // the fluid pays for what the FP32 radius holds
    const double rn = r_new;
    const double m_new = km * rn * rn * rn;
    atomicAdd(&used[v], m_new - m);
    xr.w = r_new;
    b.xr[sl] = xr;
    vel_at(b.vw, sl).w = (float)(1.0 / m_new);
    angv_at(b.vw, sl).w = (float)(1.0 / (0.4 * m_new * rn * rn));
}

__global__ void k_grow_fluid(int64_t nv, double* mf, const double* used, double* total)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nv) return;
    const double u = used[i];
    if (u > 0.0) {
        mf[i] -= u;
        if (total) atomicAdd(total, u);
    }
}

void launch_grow(const DevBuffers& b, const EnvDev& E, const tr_voxel_grid& g, double dt, double dprime_max,
                 double d_max, double* mf, double* work, double* total, hipStream_t s)
{
    const int64_t nv = (int64_t)g.nx * g.ny * g.nz;
    double* cap_sum = work;
    double* used = work + nv;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)cdiv(2 * nv, kBlk)), dim3(kBlk), 0, s, work, 2 * nv, 0.0);
    if (total) hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, total, (int64_t)1, 0.0);
    if (E.n > 0) {
        const unsigned nb = (unsigned)cdiv(E.n, kBlk);
        hipLaunchKernelGGL(k_grow_caps, dim3(nb), dim3(kBlk), 0, s, b, E, g, dt, dprime_max, d_max, cap_sum);
        hipLaunchKernelGGL(k_grow_apply, dim3(nb), dim3(kBlk), 0, s, b, E, g, dt, dprime_max, d_max, cap_sum, mf,
                           used);
    }
    hipLaunchKernelGGL(k_grow_fluid, dim3((unsigned)cdiv(nv, kBlk)), dim3(kBlk), 0, s, nv, mf, used, total);
}

// ---------------------------------------------------------------------------
// Forming new particles from the fluid inside the zones: one thread per
// voxel marks a candidate (the list's order is fixed by the host afterwards),
// then the fluid of each listed voxel pays the mass its FP32 radius holds
// ---------------------------------------------------------------------------
__global__ void k_form_candidates(tr_voxel_grid g, double rho, double d_min, double d_max, double phi_max, WedgeSet ws,
                                  const double* rho_p, const double* u, const double* mf, FormEntry* list,
                                  unsigned long long* count, int64_t cap)
{
#pragma clang fp contract(off)
    const int64_t nxy = (int64_t)g.nx * g.ny, nv = nxy * g.nz;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nv) return;
    const double km = rho * 3.14159265358979323846 / 6.0;  // m = km d^3
    const double m_min = km * d_min * d_min * d_min;
    const double f = mf[id];
    if (!(f >= m_min)) return;
    const int k = (int)(id / nxy), j = (int)((id % nxy) / g.nx), i = (int)(id % g.nx);
    const double c[3] = {g.origin[0] + (i + 0.5) * g.l0, g.origin[1] + (j + 0.5) * g.l0, g.origin[2] + (k + 0.5) * g.l0};
    if (!in_wedge_set(ws, c[0], c[1], c[2])) return;
    double d = cbrt(f / km);
    d = d > d_max ? d_max : d;
    const double m = km * d * d * d;
    const double V0 = g.l0 * g.l0 * g.l0;
    if (rho_p[id] / rho + m / (rho * V0) > phi_max) return;  // no room for one more particle
    const unsigned long long slot = atomicAdd(count, 1ull);
    if ((int64_t)slot >= cap) return;
    FormEntry e;
    e.voxel = (double)id;
    for (int q = 0; q < 3; ++q) { e.x[q] = c[q]; e.v[q] = u[3 * id + q]; }
    e.r = 0.5 * d;
    list[slot] = e;
}

// the library's particle mass: FP32 density and radius, FP64 arithmetic
__global__ void k_form_pay(const FormEntry* list, int64_t n, double rho, double* mf)
{
#pragma clang fp contract(off)
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const double r = (double)(float)list[a].r;
    const double m = (double)(float)rho * (4.0 / 3.0) * 3.14159265358979323846 * r * r * r;
    mf[(int64_t)list[a].voxel] -= m;  // one entry per voxel
}

void launch_form_candidates(const tr_voxel_grid& g, double rho, double d_min, double d_max, double phi_max,
                            const WedgeSet& ws, const double* rho_p, const double* u, const double* mf,
                            FormEntry* list, unsigned long long* count, int64_t cap, hipStream_t s)
{
    const int64_t nv = (int64_t)g.nx * g.ny * g.nz;
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, (double*)count, (int64_t)1, 0.0);  // bits of 0
    hipLaunchKernelGGL(k_form_candidates, dim3((unsigned)cdiv(nv, kBlk)), dim3(kBlk), 0, s, g, rho, d_min, d_max,
                       phi_max, ws, rho_p, u, mf, list, count, cap);
}

void launch_form_pay(const FormEntry* list, int64_t n, double rho, double* mf, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_form_pay, dim3((unsigned)cdiv(n, kBlk)), dim3(kBlk), 0, s, list, n, rho, mf);
}

// ---------------------------------------------------------------------------
// Particles at rest outside the zones: their mass joins their voxel's fluid
// (FP64 atomics) and their ids are listed for removal
// ---------------------------------------------------------------------------
__global__ void k_settle(DevBuffers b, EnvDev E, tr_voxel_grid g, double v_rest, WedgeSet ws, double* mf, int* list,
                         unsigned long long* count, double* total)
{
#pragma clang fp contract(off)
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= E.n) return;
    const int sl = E.slot_begin + a;
    const float4 xr = b.xr[sl], vm = vel_at(b.vw, sl);
    const double v[3] = {vm.x, vm.y, vm.z};
    if (!(sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]) < v_rest)) return;
    const int64_t vox = voxel_index(g, xr);
    if (vox < 0 || in_wedge_set(ws, xr.x, xr.y, xr.z)) return;
    const double r = xr.w;
    const double m = (double)b.rho[sl] * (4.0 / 3.0) * 3.14159265358979323846 * r * r * r;
    atomicAdd(&mf[vox], m);
    if (total) atomicAdd(total, m);
    list[atomicAdd(count, 1ull)] = b.pid[sl];
}

void launch_settle(const DevBuffers& b, const EnvDev& E, const tr_voxel_grid& g, double v_rest, const WedgeSet& ws,
                   double* mf, int* list, unsigned long long* count, double* total, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, (double*)count, (int64_t)1, 0.0);  // bits of 0
    if (total) hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, s, total, (int64_t)1, 0.0);
    if (E.n > 0)
        hipLaunchKernelGGL(k_settle, dim3((unsigned)cdiv(E.n, kBlk)), dim3(kBlk), 0, s, b, E, g, v_rest, ws, mf, list,
                           count, total);
}

}  // namespace trk

