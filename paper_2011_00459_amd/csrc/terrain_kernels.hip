// terrain_kernels.hip -- gfx950 kernels of one agitated-soil particle step.
//
// The step (Algorithm 1 of Servin, Berglund & Nystedt: collision detection,
// the mesoscale contact constraints, the aggregate bodies, the PGS solve and
// the position update) is split into these kernel families:
//   bin/scan/scatter/gather   particles sorted by (env, Morton cell, id)
//   narrow                    sphere-sphere and sphere-boundary contacts with
//                             a pinned FP64 predicate, wave-compacted
//   id count/scatter/sort     canonical contact order (key order)
//   incidence + colour        per-particle incidence lists and a greedy
//                             colouring in splitmix64 priority order
//   rows                      Hertz-mapped SPOOK rows (Eqs. signCoul1-2)
//   warm apply                v* = v + dt g + M^-1 G^T lambda^0
//   pgs                       persistent colour-synchronous projected
//                             Gauss-Seidel sweeps with the residual fused in
//   finish                    body forces (FP64), x += dt v, kinematic poses,
//                             zone aggregates (FP64, Eqs. aggregate_mass ..
//                             aggregate_rot_vel)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>

#include "terrain_internal.h"
#include "terrain_geom.h"

namespace trk {

constexpr int kBlk = 256;
#ifndef TRK_BARRIER_SPINS
#define TRK_BARRIER_SPINS (1l << 22)
#endif
constexpr long kBarrierSpins = TRK_BARRIER_SPINS;  // bounded wait of a grid barrier

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// generic fill and device-wide exclusive scan (out[n] = total)
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = v;
}

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    int grid = (int)std::min<int64_t>(cdiv(n, kBlk), 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(kBlk), 0, s, p, v, n);
}

constexpr int kScanItems = 4;
constexpr int kScanTile = kBlk * kScanItems;

__device__ inline uint32_t wave_incl_scan(uint32_t v)
{
    int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// exclusive block scan of one value per thread; returns the block total via *tot
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* tot)
{
    __shared__ uint32_t wsum[kBlk / 64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, all = 0;
    for (int k = 0; k < kBlk / 64; ++k) {
        if (k < w) off += wsum[k];
        all += wsum[k];
    }
    __syncthreads();
    *tot = all;
    return off + inc - v;
}

__global__ void k_scan_reduce(const uint32_t* in, int64_t n, uint32_t* tmp)
{
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        if (i < n) s += in[i];
    }
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) tmp[blockIdx.x] = tot;
}

__global__ void k_scan_top(uint32_t* tmp, int64_t nb)
{
    // single block: exclusive scan of the block totals, total at tmp[nb]
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += kBlk) {
        int64_t i = base + threadIdx.x;
        uint32_t v = i < nb ? tmp[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, &tot);
        if (i < nb) tmp[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) tmp[nb] = carry;
}

__global__ void k_scan_down(const uint32_t* in, uint32_t* out, int64_t n, const uint32_t* tmp, int64_t nb)
{
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t v[kScanItems];
    uint32_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        v[k] = i < n ? in[i] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan(s, &tot) + tmp[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
        if (i < n) out[i] = ex;
        ex += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tmp[nb];
}

int64_t scan_tmp_words(int64_t n) { return cdiv(std::max<int64_t>(n, 1), kScanTile) + 1; }

void launch_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t s)
{
    int64_t nb = cdiv(std::max<int64_t>(n, 1), kScanTile);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kBlk), 0, s, in, n, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlk), 0, s, tmp, nb);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kBlk), 0, s, in, out, n, tmp, nb);
}

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------
__device__ inline uint32_t env_of(int id, uint32_t id_cap) { return (uint32_t)id / id_cap; }

__device__ inline uint32_t morton(int cx, int cy, int cz, const int bits[3])
{
    // non-uniform interleave: one bit of each axis that still has bits, x first
    uint32_t key = 0;
    int pos = 0;
    int mb = max(bits[0], max(bits[1], bits[2]));
    for (int b = 0; b < mb; ++b) {
        if (b < bits[0]) key |= (uint32_t)((cx >> b) & 1) << pos++;
        if (b < bits[1]) key |= (uint32_t)((cy >> b) & 1) << pos++;
        if (b < bits[2]) key |= (uint32_t)((cz >> b) & 1) << pos++;
    }
    return key;
}

__device__ inline void cell_of(const EnvDev& E, float x, float y, float z, int c[3])
{
    float f[3] = {(x - E.lo[0]) * E.inv_h, (y - E.lo[1]) * E.inv_h, (z - E.lo[2]) * E.inv_h};
    for (int k = 0; k < 3; ++k) {
        float g = fminf(fmaxf(floorf(f[k]), 0.0f), (float)(E.dims[k] - 1));
        c[k] = (int)g;
    }
}

__device__ inline unsigned long long splitmix64(unsigned long long x)
{
    unsigned long long z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Pinned sphere-sphere predicate (FP64, fixed order, no contraction).
__device__ inline bool pair_touch(double xi, double yi, double zi, double ri, double xj, double yj, double zj,
                                  double rj, double kappa_c)
{
#pragma clang fp contract(off)
    double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    double d2 = (dx * dx + dy * dy) + dz * dz;
    double rs = ri + rj;
    double R = rs + (kappa_c > 0.0 ? kappa_c * rs : 0.0);
    return d2 < R * R;
}

// ---------------------------------------------------------------------------
// step begin: world data of shapes, clears
// ---------------------------------------------------------------------------
__global__ void k_step_begin(DevBuffers b, StepParams p)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    {
        // every counter starts the step at zero except the failure word, into
        // which one thread folds the previous step's flags before clearing them
        uint32_t* w = reinterpret_cast<uint32_t*>(b.cnt);
        constexpr int kOvfWord = (int)(offsetof(Counters, overflow) / 4);
        constexpr int kFailedWord = (int)(offsetof(Counters, failed) / 4);
        for (int k = t; k < (int)(sizeof(Counters) / 4); k += gridDim.x * blockDim.x)
            if (k != kOvfWord && k != kFailedWord) w[k] = 0u;
        if (t == 0) {
            w[kFailedWord] |= w[kOvfWord];
            w[kOvfWord] = 0u;
        }
    }
    if (t < p.n_envs) {
        b.env_stats[t].contacts = 0;
        b.env_stats[t].pairs = 0;
        b.env_stats[t].impacts = 0;
        b.env_ncol[t] = 0;
    }
    if (t < p.n_units) {
        uint32_t* w = reinterpret_cast<uint32_t*>(&b.ustats[t]);
        for (int k = 0; k < (int)(sizeof(UnitStats) / 4); ++k) w[k] = 0u;
    }
    if (t < p.n_shapes) {
#pragma clang fp contract(off)
        ShapeDev& S = b.shapes[t];
        const BodyDev& B = b.bodies[S.body];
        double R[9];
        quat_to_R(B.quat, R);
        for (int k = 0; k < 9; ++k) S.R[k] = R[k];
        for (int k = 0; k < 3; ++k) S.wn[k] = (R[k * 3 + 0] * S.n[0] + R[k * 3 + 1] * S.n[1]) + R[k * 3 + 2] * S.n[2];
        S.wd = S.d + ((S.wn[0] * B.pos[0] + S.wn[1] * B.pos[1]) + S.wn[2] * B.pos[2]);
        for (int k = 0; k < 3; ++k)
            S.wc[k] = B.pos[k] + ((R[k * 3 + 0] * S.off[0] + R[k * 3 + 1] * S.off[1]) + R[k * 3 + 2] * S.off[2]);
    }
}

void launch_step_begin(const DevBuffers& b, const StepParams& p, hipStream_t s)
{
    int n = std::max((int)(sizeof(Counters) / 4), std::max(p.n_shapes, std::max(p.n_envs, p.n_units)));
    hipLaunchKernelGGL(k_step_begin, dim3((unsigned)cdiv(n, kBlk)), dim3(kBlk), 0, s, b, p);
}

// ---------------------------------------------------------------------------
// A1-A2: binning, counting sort by cell key, per-cell id order, gather
// ---------------------------------------------------------------------------
__global__ void k_bin(DevBuffers b, StepParams p)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n_particles) return;
    float4 x = b.xr[i];
    const EnvDev& E = b.envs[env_of(b.pid[i], p.id_cap)];
    int c[3];
    cell_of(E, x.x, x.y, x.z, c);
    uint32_t key = E.cell_base + morton(c[0], c[1], c[2], E.bits);
    b.pkey[i] = key;
    atomicAdd(&b.cell_count[key], 1u);
}

__global__ void k_scatter_cells(DevBuffers b, StepParams p)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n_particles) return;
    uint32_t key = b.pkey[i];
    uint32_t slot = b.cell_start[key] + atomicAdd(&b.cell_fill[key], 1u);
    b.perm[slot] = (uint32_t)i;
}

// the first slot of every cell orders the cell's particles by id
__global__ void k_cell_order(DevBuffers b, StepParams p)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n_particles) return;
    uint32_t key = b.pkey[b.perm[s]];
    uint32_t beg = b.cell_start[key], end = b.cell_start[key + 1];
    if ((uint32_t)s != beg) return;
    for (uint32_t a = beg + 1; a < end; ++a) {
        uint32_t v = b.perm[a];
        int idv = b.pid[v];
        uint32_t t = a;
        while (t > beg && b.pid[b.perm[t - 1]] > idv) {
            b.perm[t] = b.perm[t - 1];
            --t;
        }
        b.perm[t] = v;
    }
}

__global__ void k_gather(DevBuffers b, StepParams p)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n_particles) return;
    uint32_t i = b.perm[s];
    b.xr2[s] = b.xr[i];
    vel_at(b.vw2, s) = vel_at(b.vw, i);
    angv_at(b.vw2, s) = angv_at(b.vw, i);
    b.rho2[s] = b.rho[i];
    int id = b.pid[i];
    b.pid2[s] = id;
    b.id2slot[id] = s;
}

void launch_sort_particles(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s)
{
    int n = p.n_particles;
    launch_fill_u32(b.cell_count, 0u, z.NC, s);
    launch_fill_u32(b.cell_fill, 0u, z.NC, s);
    if (n <= 0) return;
    unsigned g = (unsigned)cdiv(n, kBlk);
    hipLaunchKernelGGL(k_bin, dim3(g), dim3(kBlk), 0, s, b, p);
    launch_scan_u32(b.cell_count, b.cell_start, z.NC, b.scan_tmp, s);
    hipLaunchKernelGGL(k_scatter_cells, dim3(g), dim3(kBlk), 0, s, b, p);
    hipLaunchKernelGGL(k_cell_order, dim3(g), dim3(kBlk), 0, s, b, p);
    hipLaunchKernelGGL(k_gather, dim3(g), dim3(kBlk), 0, s, b, p);
}

// ---------------------------------------------------------------------------
// A3-A4: narrow phase (pairs through the 27 neighbour cells, then the env's
// boundary shapes), compacted per wave
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlk) void k_narrow(DevBuffers b, StepParams p, int64_t cap)
{
    __shared__ int hits[kBlk][kMaxHits + 1];
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int nh = 0;
    int idi = 0;
    bool ovf = false;
    uint32_t env = 0;
    if (i < p.n_particles) {
        float4 xi = b.xr[i];
        idi = b.pid[i];
        env = env_of(idi, p.id_cap);
        const EnvDev& E = b.envs[env];
        int c[3];
        cell_of(E, xi.x, xi.y, xi.z, c);
        double X = xi.x, Y = xi.y, Z = xi.z, Ri = xi.w;
        // half shell: the own cell's later slots and the 13 cells after it
        // in (z, y, x) order, so that each pair is met once, from the sphere
        // whose cell comes first (the predicate is exactly symmetric)
        for (int dz = 0; dz <= 1; ++dz) {
            int cz = c[2] + dz;
            if (cz >= E.dims[2]) continue;
            for (int dy = dz ? -1 : 0; dy <= 1; ++dy) {
                int cy = c[1] + dy;
                if (cy < 0 || cy >= E.dims[1]) continue;
                for (int dx = (dz || dy) ? -1 : 0; dx <= 1; ++dx) {
                    int cx = c[0] + dx;
                    if (cx < 0 || cx >= E.dims[0]) continue;
                    uint32_t key = E.cell_base + morton(cx, cy, cz, E.bits);
                    uint32_t beg = b.cell_start[key], end = b.cell_start[key + 1];
                    if ((dx | dy | dz) == 0) beg = max(beg, (uint32_t)i + 1);
                    for (uint32_t j = beg; j < end; ++j) {
                        float4 xj = b.xr[j];
                        if (pair_touch(X, Y, Z, Ri, (double)xj.x, (double)xj.y, (double)xj.z, (double)xj.w, p.kappa_c)) {
                            if (nh < kMaxHits) hits[threadIdx.x][nh++] = (int)j;
                            else ovf = true;
                        }
                    }
                }
            }
        }
        for (int sg = E.shape_begin; sg < E.shape_end; ++sg) {
            if (shape_touch(b.shapes[sg], b.hf_pool, X, Y, Z, Ri, p.kappa_c, nullptr)) {
                if (nh < kMaxHits) hits[threadIdx.x][nh++] = -1 - sg;
                else ovf = true;
            }
        }
    }
    // wave-level compaction: one atomic per wave
    int lane = threadIdx.x & 63;
    uint32_t inc = wave_incl_scan((uint32_t)nh);
    uint32_t total = __shfl(inc, 63, 64);
    uint32_t base = 0;
    if (lane == 63 && total > 0) base = atomicAdd(&b.cnt->n_raw, total);
    base = __shfl(base, 63, 64);
    uint32_t off = base + inc - (uint32_t)nh;
    int npairs = 0;
    for (int k = 0; k < nh; ++k) {
        int h = hits[threadIdx.x][k];
        uint64_t idx = (uint64_t)off + (uint64_t)k;
        if (idx >= (uint64_t)cap) { ovf = true; continue; }
        if (h >= 0) {
            // key and pair in id order: (lower id, higher id)
            int idj = b.pid[h];
            const bool first = idi < idj;
            const uint32_t lo = (uint32_t)(first ? idi : idj), hi = (uint32_t)(first ? idj : idi);
            b.rkey[idx] = ((unsigned long long)lo << 32) | hi;
            b.rpair[idx] = first ? make_int2(i, h) : make_int2(h, i);
            ++npairs;
        } else {
            int sg = -1 - h;
            int local = sg - b.envs[env].shape_begin;
            b.rkey[idx] = ((unsigned long long)(uint32_t)idi << 32) | 0x80000000ull | (uint32_t)local;
            b.rpair[idx] = make_int2(h, i);
        }
    }
    // the pair count of the env: one atomic per wave when the wave's particles
    // share an env (same-address atomics from every lane serialise: this one,
    // per lane, took most of the kernel's time on a 50k-sphere bed)
    {
        const uint32_t env0 = __shfl(env, 0, 64);
        if (__ballot(env != env0) == 0ull) {
            unsigned long long t = (unsigned long long)npairs;
            for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
            if (lane == 0 && t) atomicAdd((unsigned long long*)&b.env_stats[env0].pairs, t);
        } else if (npairs) {
            atomicAdd((unsigned long long*)&b.env_stats[env].pairs, (unsigned long long)npairs);
        }
    }
    if (ovf) atomicOr(&b.cnt->overflow, kOvfContacts);
}

void launch_narrow(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s)
{
    if (p.n_particles <= 0) return;
    hipLaunchKernelGGL(k_narrow, dim3((unsigned)cdiv(p.n_particles, kBlk)), dim3(kBlk), 0, s, b, p, z.C);
}

// ---------------------------------------------------------------------------
// A5: canonical order (counting sort by the lower id, then by key inside
// each id), per-particle incidence lists
// ---------------------------------------------------------------------------
__device__ inline uint32_t n_contacts(const DevBuffers& b, int64_t cap)
{
    uint32_t n = b.cnt->n_raw;
    return n < (uint64_t)cap ? n : (uint32_t)cap;
}

// atomicAdd(&counter[a], 1) for every active lane, as one atomic per run of
// equal a in consecutive lanes (same-address atomics from many lanes
// serialise); returns the lane's old value, as its own atomic would have
// (lanes of a run take consecutive values).  Every lane of the wave calls it.
__device__ inline uint32_t wave_run_inc(uint32_t* counter, uint32_t a, bool active)
{
    const int lane = threadIdx.x & 63;
    const uint32_t prev = __shfl_up(a, 1, 64);
    const bool prev_active = __shfl_up((int)active, 1, 64) != 0;
    const bool head = active && (lane == 0 || !prev_active || prev != a);
    const unsigned long long bound = __ballot(head || !active);
    const unsigned long long later = lane == 63 ? 0ull : bound >> (lane + 1);
    const int len = later ? __builtin_ctzll(later) + 1 : 64 - lane;
    uint32_t old = 0;
    if (head) old = atomicAdd(&counter[a], (uint32_t)len);
    const unsigned long long upto = bound & (~0ull >> (63 - lane));
    const int h = 63 - __builtin_clzll(upto | 1ull);
    return __shfl(old, h, 64) + (uint32_t)(lane - h);
}

__global__ void k_id_count(DevBuffers b, int64_t cap)
{
    uint32_t nc = n_contacts(b, cap);
    for (uint32_t c0 = blockIdx.x * blockDim.x; c0 < nc; c0 += gridDim.x * blockDim.x) {
        const uint32_t c = c0 + threadIdx.x;
        const bool on = c < nc;
        (void)wave_run_inc(b.id_count, on ? (uint32_t)(b.rkey[c] >> 32) : 0u, on);
    }
}

__global__ void k_id_scatter(DevBuffers b, int64_t cap)
{
    uint32_t nc = n_contacts(b, cap);
    for (uint32_t c0 = blockIdx.x * blockDim.x; c0 < nc; c0 += gridDim.x * blockDim.x) {
        const uint32_t c = c0 + threadIdx.x;
        const bool on = c < nc;
        const unsigned long long k = on ? b.rkey[c] : 0ull;
        const uint32_t a = (uint32_t)(k >> 32);
        const uint32_t r = wave_run_inc(b.id_fill, a, on);
        if (on) {
            const uint32_t pos = b.id_start[a] + r;
            b.ckey[pos] = k;
            b.cpair[pos] = b.rpair[c];
        }
    }
}

__global__ void k_id_sort(DevBuffers b, int64_t nid)
{
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nid) return;
    uint32_t beg = b.id_start[a], end = b.id_start[a + 1];
    for (uint32_t u = beg + 1; u < end; ++u) {
        unsigned long long k = b.ckey[u];
        int2 pr = b.cpair[u];
        uint32_t t = u;
        while (t > beg && b.ckey[t - 1] > k) {
            b.ckey[t] = b.ckey[t - 1];
            b.cpair[t] = b.cpair[t - 1];
            --t;
        }
        b.ckey[t] = k;
        b.cpair[t] = pr;
    }
}

__global__ void k_inc_count(DevBuffers b, int64_t cap)
{
    uint32_t nc = n_contacts(b, cap);
    for (uint32_t c0 = blockIdx.x * blockDim.x; c0 < nc; c0 += gridDim.x * blockDim.x) {
        const uint32_t c = c0 + threadIdx.x;
        const bool on = c < nc;
        const int2 pr = on ? b.cpair[c] : make_int2(-1, 0);
        // the particle whose id leads the key comes in runs: pr.x for a
        // pair, pr.y for a boundary contact (pr.x < 0)
        const int own = pr.x >= 0 ? pr.x : pr.y, other = pr.x >= 0 ? pr.y : -1;
        (void)wave_run_inc(b.inc_count, (uint32_t)own, on);
        if (other >= 0) atomicAdd(&b.inc_count[other], 1u);
    }
}

__global__ void k_inc_fill(DevBuffers b, int64_t cap)
{
    uint32_t nc = n_contacts(b, cap);
    for (uint32_t c0 = blockIdx.x * blockDim.x; c0 < nc; c0 += gridDim.x * blockDim.x) {
        const uint32_t c = c0 + threadIdx.x;
        const bool on = c < nc;
        const int2 pr = on ? b.cpair[c] : make_int2(-1, 0);
        const int own = pr.x >= 0 ? pr.x : pr.y, other = pr.x >= 0 ? pr.y : -1;
        const uint32_t r = wave_run_inc(b.inc_fill, (uint32_t)own, on);
        if (on) b.inc[b.inc_start[own] + r] = c;
        if (other >= 0) b.inc[b.inc_start[other] + atomicAdd(&b.inc_fill[other], 1u)] = c;
    }
}

__global__ void k_inc_sort(DevBuffers b, int n)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t beg = b.inc_start[s], end = b.inc_start[s + 1];
    for (uint32_t u = beg + 1; u < end; ++u) {
        uint32_t v = b.inc[u];
        uint32_t t = u;
        while (t > beg && b.inc[t - 1] > v) {
            b.inc[t] = b.inc[t - 1];
            --t;
        }
        b.inc[t] = v;
    }
}

void launch_canonical(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s)
{
    unsigned gc = (unsigned)std::min<int64_t>(cdiv(z.C, kBlk), 2048);
    launch_fill_u32(b.id_count, 0u, z.NID, s);
    launch_fill_u32(b.id_fill, 0u, z.NID, s);
    hipLaunchKernelGGL(k_id_count, dim3(gc), dim3(kBlk), 0, s, b, z.C);
    launch_scan_u32(b.id_count, b.id_start, z.NID, b.scan_tmp, s);
    hipLaunchKernelGGL(k_id_scatter, dim3(gc), dim3(kBlk), 0, s, b, z.C);
    hipLaunchKernelGGL(k_id_sort, dim3((unsigned)cdiv(z.NID, kBlk)), dim3(kBlk), 0, s, b, z.NID);
    int n = std::max(p.n_particles, 1);
    launch_fill_u32(b.inc_count, 0u, n, s);
    launch_fill_u32(b.inc_fill, 0u, n, s);
    hipLaunchKernelGGL(k_inc_count, dim3(gc), dim3(kBlk), 0, s, b, z.C);
    launch_scan_u32(b.inc_count, b.inc_start, n, b.scan_tmp, s);
    hipLaunchKernelGGL(k_inc_fill, dim3(gc), dim3(kBlk), 0, s, b, z.C);
    hipLaunchKernelGGL(k_inc_sort, dim3((unsigned)cdiv(n, kBlk)), dim3(kBlk), 0, s, b, n);
}

// ---------------------------------------------------------------------------
// A7: colouring.  Each contact takes the least colour unused by its
// conflicting contacts of higher (splitmix64(key), key) priority, once all of
// those are coloured: the unique Jones-Plassmann result.  Resident grid, each
// thread re-visits its uncoloured contacts until none is left (bounded).
// ---------------------------------------------------------------------------
__device__ inline int ld_colour(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kColChunk = 8;

// Scans the conflicts of contact c.  Ready: returns true with the least
// colour its coloured conflicts leave free (kMaxColours when none is).  Blocked by an uncoloured
// conflict of higher priority: returns false with that conflict in wait.
__device__ inline bool colour_try(const DevBuffers& b, uint32_t c, uint32_t& wait, int& col)
{
    unsigned long long key = b.ckey[c];
    unsigned long long h = splitmix64(key);
    int2 pr = b.cpair[c];
    unsigned long long used = 0;
    int parts[2] = {pr.y, pr.x};
    for (int q = 0; q < 2; ++q) {
        int s = parts[q];
        if (s < 0) continue;
        uint32_t beg = b.inc_start[s], end = b.inc_start[s + 1];
        // eight incident contacts at a time, each round of loads in flight together
        for (uint32_t t0 = beg; t0 < end; t0 += kColChunk) {
            uint32_t e[kColChunk];
            int ce[kColChunk];
            unsigned long long ke[kColChunk];
#pragma unroll
            for (int j = 0; j < kColChunk; ++j) e[j] = t0 + j < end ? b.inc[t0 + j] : c;
#pragma unroll
            for (int j = 0; j < kColChunk; ++j) ce[j] = e[j] != c ? ld_colour(&b.colour[e[j]]) : kMaxColours;
#pragma unroll
            for (int j = 0; j < kColChunk; ++j) ke[j] = ce[j] < 0 ? b.ckey[e[j]] : 0ull;
#pragma unroll
            for (int j = 0; j < kColChunk; ++j) {
                if (e[j] == c) continue;
                if (ce[j] < 0) {
                    unsigned long long he = splitmix64(ke[j]);
                    if (he > h || (he == h && ke[j] > key)) { wait = e[j]; return false; }
                } else {
                    used |= 1ull << ce[j];
                }
            }
        }
    }
    col = used == ~0ull ? kMaxColours : __builtin_ctzll(~used);
    return true;
}

__global__ __launch_bounds__(kBlk) void k_colour(DevBuffers b, int64_t cap, int max_pass)
{
    uint32_t nc = n_contacts(b, cap);
    // consecutive blocks run on the 8 XCDs in turn: the contact list in eight
    // contiguous parts, part x coloured by the blocks of XCD x, so that the
    // colours an env's contacts read and write stay in one XCD's L2 (except
    // where a part boundary cuts an env); measured, about 5 % less colouring
    // time than a grid-stride over the whole list.  Placement only changes
    // the speed: colours are written once, so a late read only delays a contact.
    uint32_t lo = 0, hi = nc, stride = gridDim.x * blockDim.x, first = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nx = gridDim.x / kGroups;
    if (nx > 0) {
        const uint32_t x = blockIdx.x % kGroups, jb = blockIdx.x / kGroups;
        lo = (uint32_t)((uint64_t)nc * x / kGroups);
        hi = (uint32_t)((uint64_t)nc * (x + 1) / kGroups);
        stride = nx * blockDim.x;
        first = jb < nx ? lo + jb * blockDim.x + threadIdx.x : hi;
    }
    int local_max = 0;
    bool ovf = false, left = true;
    for (int pass = 0; pass < max_pass; ++pass) {
        left = false;
        for (uint32_t c = first; c < hi; c += stride) {
            if (ld_colour(&b.colour[c]) >= 0) continue;
            // the conflict that blocked this contact last pass: while it is
            // uncoloured the contact stays blocked (a full scan decides readiness)
            if (pass > 0) {
                const uint32_t wb = b.col_wait[c];
                if (wb != ~0u && ld_colour(&b.colour[wb]) < 0) { left = true; continue; }
            }
            uint32_t w;
            int col;
            if (!colour_try(b, c, w, col)) { b.col_wait[c] = w; left = true; continue; }
            ovf |= col == kMaxColours;
            col = min(col, kMaxColours - 1);
            __hip_atomic_store(&b.colour[c], col, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            local_max = max(local_max, col + 1);
        }
        if (!__syncthreads_or(left)) break;
        __builtin_amdgcn_s_sleep(2);
    }
    // one atomic per wave (same-address atomics from every lane serialise)
    for (int o = 32; o > 0; o >>= 1) local_max = max(local_max, __shfl_xor(local_max, o, 64));
    if ((threadIdx.x & 63) == 0 && local_max) atomicMax(&b.cnt->n_colours, (uint32_t)local_max);
    if (ovf) atomicOr(&b.cnt->overflow, kOvfColours);
    if (left) atomicOr(&b.cnt->overflow, kFailColouring);
}

// stable bucketing of the canonical list by (colour, PGS group)
__device__ inline int contact_group(const DevBuffers& b, unsigned long long key, uint32_t id_cap)
{
    return b.envs[env_of((int)(key >> 32), id_cap)].group;
}

// Spread mode: the XCD group of a sphere slot (its env's slots in eighths:
// the sort keeps them in Morton order, so each eighth is a compact region) and
// of a contact (that of its second sphere, a particle for every contact).
__device__ inline int slot_part(const DevBuffers& b, int sl, uint32_t id_cap)
{
    const EnvDev& E = b.envs[env_of(b.pid[sl], id_cap)];
    return (int)(((int64_t)(sl - E.slot_begin) * kGroups) / max(E.n, 1));
}
__device__ inline int contact_group_of(const DevBuffers& b, uint32_t c, uint32_t id_cap, int spread)
{
    return spread ? slot_part(b, b.cpair[c].y, id_cap) : contact_group(b, b.ckey[c], id_cap);
}

__global__ void k_col_hist(DevBuffers b, int64_t cap, int64_t NB, uint32_t id_cap, int spread)
{
    __shared__ uint32_t h[kBuckets];
    uint32_t nc = n_contacts(b, cap);
    for (int k = threadIdx.x; k < kBuckets; k += blockDim.x) h[k] = 0;
    __syncthreads();
    uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nc) {
        int col = b.colour[c];
        if (col >= 0 && col < kMaxColours) atomicAdd(&h[col * kGroups + contact_group_of(b, c, id_cap, spread)], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kBuckets; k += blockDim.x) b.col_hist[(int64_t)k * NB + blockIdx.x] = h[k];
}

__global__ void k_col_scatter(DevBuffers b, int64_t cap, int64_t NB, uint32_t id_cap, int spread)
{
    __shared__ int bk[kBlk];
    uint32_t nc = n_contacts(b, cap);
    uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    int my = -1;
    if (c < nc) {
        int col = b.colour[c];
        if (col >= 0 && col < kMaxColours) my = col * kGroups + contact_group_of(b, c, id_cap, spread);
    }
    bk[threadIdx.x] = my;
    __syncthreads();
    if (c >= nc) return;
    if (my < 0) {  // failed colouring: the step is abandoned
        b.cpos[c] = c;
        return;
    }
    uint32_t rank = 0;
    for (int t = 0; t < (int)threadIdx.x; ++t) rank += bk[t] == my;
    b.cpos[c] = b.col_start[(int64_t)my * NB + blockIdx.x] + rank;
}

// env e's contacts in canonical order: [id_start[e id_cap], id_start[(e+1) id_cap])
__device__ inline void env_contacts(const DevBuffers& b, int e, uint32_t id_cap, uint32_t& beg, uint32_t& end)
{
    beg = b.id_start[(size_t)e * id_cap];
    end = b.id_start[(size_t)(e + 1) * id_cap];
}

// colours used by each env (zeroed at the step's start): max colour + 1 over
// the canonical list; a block whose contacts all belong to one env (the
// list is in env order) reduces first and updates once
__global__ void k_env_ncol(DevBuffers b, int64_t cap, uint32_t id_cap)
{
    __shared__ int sm[kBlk / 64];
    uint32_t nc = n_contacts(b, cap);
    uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t c0 = blockIdx.x * blockDim.x;
    if (c0 >= nc) return;
    uint32_t c1 = min(nc, c0 + blockDim.x) - 1;
    int e0 = (int)env_of((int)(b.ckey[c0] >> 32), id_cap), e1 = (int)env_of((int)(b.ckey[c1] >> 32), id_cap);
    int m = c < nc ? b.colour[c] + 1 : 0;
    if (e0 != e1) {
        if (c < nc && m > 0) atomicMax(&b.env_ncol[env_of((int)(b.ckey[c] >> 32), id_cap)], (uint32_t)min(m, kMaxColours));
        return;
    }
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_down(m, o, 64));
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = max(m, sm[w]);
        if (m > 0) atomicMax(&b.env_ncol[e0], (uint32_t)min(m, kMaxColours));
    }
}

// Per-env stable counting sort of the canonical list by colour (one block per
// env): env_col[e][k] = first colour-order position of colour k in env e, and
// cpos[c] the position of canonical contact c.  The rank among equal colours
// keeps canonical order: inside a wave from the lanes with the same colour
// (a 7-bit ballot match), across waves and chunks from running counts.
// 1024 threads, so that the largest env takes few chunks.
constexpr int kSortBlk = 1024;
constexpr int kSortWaves = kSortBlk / 64;

__global__ __launch_bounds__(kSortBlk) void k_env_colsort(DevBuffers b, uint32_t id_cap)
{
    __shared__ uint32_t base[kMaxColours + 1];
    __shared__ uint32_t wcount[kSortWaves][kMaxColours + 1];
    __shared__ int failed;
    const int e = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t beg, end;
    env_contacts(b, e, id_cap, beg, end);
    for (int k = threadIdx.x; k <= kMaxColours; k += blockDim.x) base[k] = 0;
    if (threadIdx.x == 0) failed = 0;
    __syncthreads();
    // the lanes of a wave holding the same colour as this lane
    auto same_colour = [&](int col) {
        unsigned long long same = ~0ull;
        for (int bit = 0; bit < 7; ++bit) {
            unsigned long long m = __ballot((col >> bit) & 1);
            same &= ((col >> bit) & 1) ? m : ~m;
        }
        return same;
    };
    const unsigned long long lower = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // histogram (colour kMaxColours collects failed colourings), one LDS
    // atomic per colour and wave
    for (uint32_t c0 = beg; c0 < end; c0 += blockDim.x) {
        const uint32_t c = c0 + threadIdx.x;
        int col = kMaxColours + 1;  // past the end: counted nowhere
        if (c < end) {
            col = b.colour[c];
            if (col < 0 || col >= kMaxColours) { col = kMaxColours; failed = 1; }
        }
        const unsigned long long same = same_colour(col);
        if ((same & lower) == 0 && col <= kMaxColours) atomicAdd(&base[col], (uint32_t)__popcll(same));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = beg, ncol = 0;
        for (int k = 0; k <= kMaxColours; ++k) {
            uint32_t n = base[k];
            base[k] = run;
            if (k < kMaxColours) b.env_col[(size_t)e * (kMaxColours + 1) + k] = run;
            if (n && k < kMaxColours) ncol = k + 1;
            run += n;
        }
        b.env_col[(size_t)e * (kMaxColours + 1) + kMaxColours] = base[kMaxColours];
        b.env_ncol[e] = ncol;
    }
    __syncthreads();
    for (uint32_t c0 = beg; c0 < end; c0 += blockDim.x) {
        uint32_t c = c0 + threadIdx.x;
        int col = kMaxColours + 1;  // past the end: matches no real colour
        if (c < end) {
            col = b.colour[c];
            if (col < 0 || col >= kMaxColours) col = kMaxColours;
        }
        const unsigned long long same = same_colour(col);
        uint32_t rank = (uint32_t)__popcll(same & lower);
        bool leader = (same & lower) == 0;
        for (int k = lane; k <= kMaxColours; k += 64) wcount[wave][k] = 0;
        __syncthreads();
        if (leader && col <= kMaxColours) wcount[wave][col] = (uint32_t)__popcll(same);
        __syncthreads();
        if (c < end) {
            uint32_t off = base[col] + rank;
            for (int w = 0; w < wave; ++w) off += wcount[w][col];
            b.cpos[c] = failed ? c : off;
        }
        __syncthreads();
        for (int k = threadIdx.x; k <= kMaxColours; k += blockDim.x) {
            uint32_t t = 0;
            for (int w = 0; w < kSortWaves; ++w) t += wcount[w][k];
            base[k] += t;
        }
        __syncthreads();
    }
}

void launch_colour(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s)
{
    launch_fill_u32((uint32_t*)b.colour, 0xFFFFFFFFu, z.C, s);
    hipLaunchKernelGGL(k_colour, dim3(z.col_grid), dim3(kBlk), 0, s, b, z.C, 100000);
    if (z.pgs_mode == kModePerEnv) {
        hipLaunchKernelGGL(k_env_colsort, dim3((unsigned)z.n_envs), dim3(kSortBlk), 0, s, b, p.id_cap);
        return;
    }
    const int spread = z.pgs_mode == kModeSpread ? 1 : 0;
    hipLaunchKernelGGL(k_col_hist, dim3((unsigned)z.NB), dim3(kBlk), 0, s, b, z.C, z.NB, p.id_cap, spread);
    launch_scan_u32(b.col_hist, b.col_start, (int64_t)kBuckets * z.NB, b.scan_tmp, s);
    hipLaunchKernelGGL(k_col_scatter, dim3((unsigned)z.NB), dim3(kBlk), 0, s, b, z.C, z.NB, p.id_cap, spread);
    hipLaunchKernelGGL(k_env_ncol, dim3((unsigned)z.NB), dim3(kBlk), 0, s, b, z.C, p.id_cap);

}

// ---------------------------------------------------------------------------
// A6 + A8: contact rows in colour order, with lambda^0 (cold or previous-step
// impulses matched by key, re-projected onto the tangent plane and onto the
// feasible set).  Geometry in FP64, stored in FP32.
// ---------------------------------------------------------------------------
// lambda_r onto the disk |lambda_r| <= lim
__device__ inline float4 project_roll(float4 Lr, float lim)
{
    float m2 = Lr.x * Lr.x + Lr.y * Lr.y + Lr.z * Lr.z;
    if (m2 > lim * lim) {
        float sc = m2 > 0.f ? lim * rsqrtf(m2) : 0.f;
        Lr.x *= sc; Lr.y *= sc; Lr.z *= sc;
    }
    return Lr;
}

// what k_rows writes beside the rows: the previous-step match, the learned
// start's features and frame, the counter-ordered PGS's update sequence
constexpr int kRowsPrev = 1, kRowsFeatures = 2, kRowsSeq = 4;

// A contact's start impulse as the velocity changes of its two spheres
// (layout of wrec): J = lambda_n n + lambda_t acts on sphere 2 with +J and
// on sphere 1 with -J; the angular change of a sphere is its lever times
// (n x J), -l2 for sphere 2 and l1 for sphere 1, plus the rolling impulse.
__device__ inline void warm_record(float4 L, float4 a, float l2, int ib, float4 Lr, bool roll, float4* rec)
{
    float J0 = L.x * a.x + L.y, J1 = L.x * a.y + L.z, J2 = L.x * a.z + L.w;
    float lb = -l2, la = a.w;
    float b0 = lb * (a.y * J2 - a.z * J1), b1 = lb * (a.z * J0 - a.x * J2), b2 = lb * (a.x * J1 - a.y * J0);
    float a0 = la * (a.y * J2 - a.z * J1), a1 = la * (a.z * J0 - a.x * J2), a2 = la * (a.x * J1 - a.y * J0);
    if (roll) {
        b0 += Lr.x; b1 += Lr.y; b2 += Lr.z;
        a0 += Lr.x; a1 += Lr.y; a2 += Lr.z;
    }
    rec[0] = make_float4(J0, J1, J2, __int_as_float(ib));
    rec[1] = make_float4(b0, b1, b2, a0);
    rec[2] = make_float4(a1, a2, 0.f, 0.f);
}

__global__ void k_rows(DevBuffers b, StepParams p, int64_t cap, int flags)
{
    uint32_t nc = n_contacts(b, cap);
    uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    if (b.cnt->overflow) return;
    unsigned long long key = b.ckey[c];
    int2 pr = b.cpair[c];
    int ia = pr.x, ib = pr.y;
    float4 x2 = b.xr[ib];
    float4 v2 = vel_at(b.vw, ib);
    double X2[3] = {x2.x, x2.y, x2.z};
    double r2 = x2.w;
    double n[3], delta, l1, l2, dstar, dref, rmin, im1 = 0.0, iI1 = 0.0, un;
    double vk[3] = {0.0, 0.0, 0.0};
    double u1[3] = {0.0, 0.0, 0.0};  // velocity of body 1 at the contact point
    if (ia >= 0) {
        float4 x1 = b.xr[ia];
        float4 v1 = vel_at(b.vw, ia);
        float4 w1 = angv_at(b.vw, ia);
        double r1 = x1.w;
        double e[3] = {X2[0] - x1.x, X2[1] - x1.y, X2[2] - x1.z};
        double d = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        if (d > 0.0) { n[0] = e[0] / d; n[1] = e[1] / d; n[2] = e[2] / d; }
        else { n[0] = 0.0; n[1] = 0.0; n[2] = 1.0; }
        delta = (r1 + r2) - d;
        l1 = r1 - 0.5 * delta;
        l2 = r2 - 0.5 * delta;
        dstar = 1.0 / (1.0 / (2.0 * r1) + 1.0 / (2.0 * r2));
        dref = r1 + r2;
        rmin = fmin(r1, r2);
        im1 = v1.w;
        iI1 = w1.w;
        un = n[0] * ((double)v2.x - v1.x) + n[1] * ((double)v2.y - v1.y) + n[2] * ((double)v2.z - v1.z);
        // v1 + w1 x (l1 n)
        u1[0] = (double)v1.x + l1 * ((double)w1.y * n[2] - (double)w1.z * n[1]);
        u1[1] = (double)v1.y + l1 * ((double)w1.z * n[0] - (double)w1.x * n[2]);
        u1[2] = (double)v1.z + l1 * ((double)w1.x * n[1] - (double)w1.y * n[0]);
    } else {
        int sg = -1 - ia;
        const ShapeDev& S = b.shapes[sg];
        ShapeHit hit;
        shape_touch(S, b.hf_pool, X2[0], X2[1], X2[2], r2, p.kappa_c, &hit);
        delta = hit.delta;
        n[0] = hit.n[0]; n[1] = hit.n[1]; n[2] = hit.n[2];
        l1 = 0.0;
        l2 = r2 - 0.5 * delta;
        dstar = 2.0 * r2;
        dref = 2.0 * r2;
        rmin = r2;
        const BodyDev& B = b.bodies[S.body];
        double pc[3] = {X2[0] - l2 * n[0], X2[1] - l2 * n[1], X2[2] - l2 * n[2]};
        double arm[3] = {pc[0] - B.pos[0], pc[1] - B.pos[1], pc[2] - B.pos[2]};
        vk[0] = B.linvel[0] + (B.angvel[1] * arm[2] - B.angvel[2] * arm[1]);
        vk[1] = B.linvel[1] + (B.angvel[2] * arm[0] - B.angvel[0] * arm[2]);
        vk[2] = B.linvel[2] + (B.angvel[0] * arm[1] - B.angvel[1] * arm[0]);
        un = n[0] * ((double)v2.x - vk[0]) + n[1] * ((double)v2.y - vk[1]) + n[2] * ((double)v2.z - vk[2]);
        u1[0] = vk[0]; u1[1] = vk[1]; u1[2] = vk[2];
    }
    // Hertz stiffness and the row scaled to unit Jacobian
    double kn = p.Estar * sqrt(dstar) / 3.0;
    double de = fmax(delta, p.kappa_min * dref);
    double eps = 4.0 / (5.0 * kn * sqrt(de));
    double Sig = p.sig_coef * eps;
    double q = p.a_coef * (0.8 * delta) + p.b_coef * un;
    double im2 = v2.w, iI2 = angv_at(b.vw, ib).w;
    double Wn = im1 + im2;
    double Wt = im1 + im2 + l1 * l1 * iI1 + l2 * l2 * iI2;
    double Dn = Wn + Sig;
    double Dt = Wt + (double)p.gamma_dt;
    double lo = -p.lo_coef * rmin * rmin;

    // warm start: previous-step impulses of the same key
    float4 L = make_float4(0.f, 0.f, 0.f, 0.f);
    float4 Lr = make_float4(0.f, 0.f, 0.f, 0.f);
    bool persistent = false;
    if (flags & kRowsPrev) {
        uint32_t a = (uint32_t)(key >> 32);
        uint32_t beg = b.pid_start[a], end = b.pid_start[a + 1];
        for (uint32_t t = beg; t < end; ++t)
            if (b.pkeyc[t] == key) {
                L = b.plam[t];
                if (p.mu_r > 0.f) Lr = b.plamr[t];
                persistent = true;
                break;
            }
    }
    uint32_t pos = b.cpos[c];
    // learned-start features (12), contact frame and impulse scale, in FP64
    if (flags & kRowsFeatures) {
        float4 w2 = angv_at(b.vw, ib);
        double u[3];
        u[0] = ((double)v2.x - l2 * ((double)w2.y * n[2] - (double)w2.z * n[1])) - u1[0];
        u[1] = ((double)v2.y - l2 * ((double)w2.z * n[0] - (double)w2.x * n[2])) - u1[1];
        u[2] = ((double)v2.z - l2 * ((double)w2.x * n[1] - (double)w2.y * n[0])) - u1[2];
        double unf = (n[0] * u[0] + n[1] * u[1]) + n[2] * u[2];
        double ut[3] = {u[0] - unf * n[0], u[1] - unf * n[1], u[2] - unf * n[2]};
        double utm = sqrt((ut[0] * ut[0] + ut[1] * ut[1]) + ut[2] * ut[2]);
        double lp[3] = {L.y, L.z, L.w};
        double lpn = (n[0] * lp[0] + n[1] * lp[1]) + n[2] * lp[2];
        for (int k = 0; k < 3; ++k) lp[k] -= lpn * n[k];
        double t1[3];
        if (utm > 1e-12) {
            for (int k = 0; k < 3; ++k) t1[k] = ut[k] / utm;
        } else {
            double lm = sqrt((lp[0] * lp[0] + lp[1] * lp[1]) + lp[2] * lp[2]);
            if (lm > 0.0) {
                for (int k = 0; k < 3; ++k) t1[k] = lp[k] / lm;
            } else {
                int k0 = 0;
                for (int k = 1; k < 3; ++k) if (fabs(n[k]) < fabs(n[k0])) k0 = k;
                double ax[3] = {0.0, 0.0, 0.0};
                ax[k0] = 1.0;
                double dn = (ax[0] * n[0] + ax[1] * n[1]) + ax[2] * n[2];
                for (int k = 0; k < 3; ++k) t1[k] = ax[k] - dn * n[k];
                double sm = sqrt((t1[0] * t1[0] + t1[1] * t1[1]) + t1[2] * t1[2]);
                for (int k = 0; k < 3; ++k) t1[k] /= sm;
            }
        }
        double t2[3] = {n[1] * t1[2] - n[2] * t1[1], n[2] * t1[0] - n[0] * t1[2], n[0] * t1[1] - n[1] * t1[0]};
        double ls = (1.0 / Wn) * p.gdt;
        double rbar = ia >= 0 ? 0.5 * ((double)b.xr[ia].w + r2) : r2;
        float* f = b.feat + (size_t)pos * 12;
        f[0] = (float)(delta / rbar);
        f[1] = (float)(unf / p.gdt);
        f[2] = (float)(utm / p.gdt);
        f[3] = (float)((double)L.x / ls);
        f[4] = (float)(((lp[0] * t1[0] + lp[1] * t1[1]) + lp[2] * t1[2]) / ls);
        f[5] = (float)(((lp[0] * t2[0] + lp[1] * t2[1]) + lp[2] * t2[2]) / ls);
        f[6] = ia >= 0 ? (float)((double)b.pdepth[ia] / rbar) : 0.0f;
        f[7] = (float)((double)b.pdepth[ib] / rbar);
        f[8] = ia >= 0 ? (float)((double)b.xr[ia].w / p.r_ref) : 0.0f;
        f[9] = (float)(r2 / p.r_ref);
        f[10] = ia >= 0 ? 0.0f : 1.0f;
        f[11] = persistent ? 1.0f : 0.0f;
        b.frm1[pos] = make_float4((float)t1[0], (float)t1[1], (float)t1[2], (float)ls);
        b.frm2[pos] = make_float4((float)t2[0], (float)t2[1], (float)t2[2], 0.0f);
    }
    float nf[3] = {(float)n[0], (float)n[1], (float)n[2]};
    if (p.warm == TR_WARM_COLD) L = make_float4(0.f, 0.f, 0.f, 0.f);
    {
        float ln = fmaxf(L.x, (float)lo);
        float tn = nf[0] * L.y + nf[1] * L.z + nf[2] * L.w;
        float t0 = L.y - tn * nf[0], t1 = L.z - tn * nf[1], t2 = L.w - tn * nf[2];
        float lim = p.mu * fabsf(ln);
        float m2 = t0 * t0 + t1 * t1 + t2 * t2;
        if (m2 > lim * lim) {
            float sc = m2 > 0.f ? lim * rsqrtf(m2) : 0.f;
            t0 *= sc; t1 *= sc; t2 *= sc;
        }
        L = make_float4(ln, t0, t1, t2);
    }
    b.r0[pos] = make_float4(nf[0], nf[1], nf[2], (float)l1);
    b.r1[pos] = make_float4((float)l2, (float)(1.0 / Dn), (float)(1.0 / Dt), (float)Sig);
    b.r2[pos] = make_float4((float)q, (float)lo, __int_as_float(ia), __int_as_float(ib));
    // the contact's place in the colour-ordered update sequence of each of its
    // spheres (position among the sphere's contacts, and their count), for
    // the counter-ordered PGS
    uint32_t seq = 0;
    if (flags & kRowsSeq) {
        const int col = b.colour[c];
        uint32_t pa = 0, da = 0, pb = 0, db = 0;
        auto place = [&](int sl, uint32_t& pr, uint32_t& dg) {
            uint32_t beg = b.inc_start[sl], end = b.inc_start[sl + 1];
            dg = end - beg;
            for (uint32_t t = beg; t < end; ++t) pr += b.colour[b.inc[t]] < col ? 1u : 0u;
        };
        if (ia >= 0) place(ia, pa, da);
        place(ib, pb, db);
        if (da > 255 || db > 255) atomicOr(&b.cnt->overflow, kOvfHits);
        seq = pa | (pb << 8) | (da << 16) | (db << 24);
    }
    b.rk[pos] = make_float4((float)vk[0], (float)vk[1], (float)vk[2], __uint_as_float(seq));
    b.lam[pos] = L;
    b.lam0[pos] = L;
    if (p.v_imp > 0.f) {
        // impact stage (before the main solve): a contact whose start-of-step
        // normal velocity approaches faster than v_imp gets the Newton law
        // G_n v+ = -e G_n v-, every other contact G_n v+ >= 0; no compliance,
        // regularisation or cohesion
        const bool impact = un < -(double)p.v_imp;
        b.ri1[pos] = make_float4((float)l2, (float)(1.0 / Wn), (float)(1.0 / Wt), 0.f);
        b.ri2[pos] = make_float4(impact ? (float)(-(double)p.restitution * un) : 0.f, 0.f, __int_as_float(ia),
                                 __int_as_float(ib));
        b.qg[pos] = (float)(p.a_coef * (0.8 * delta));
        if (impact) {
            const int e = (int)((uint32_t)(key >> 32) / p.id_cap);
            atomicAdd(&b.env_stats[e].impacts, 1ull);
            atomicOr(&b.ustats[b.envs[e].unit].imp_any, 1u);
        }
    }
    if (p.mu_r > 0.f) {
        // rolling row (Eq. signCoul3): 1/(1/I_1 + 1/I_2), r mu_r with r the
        // smaller radius, the kinematic body of a boundary contact; the start
        // impulse projected onto |lambda_r| <= r mu_r |lambda_n|
        float rlim = (float)((double)p.mu_r * rmin);
        int kb = ia >= 0 ? -1 : b.shapes[-1 - ia].body;
        b.r3[pos] = make_float4((float)(1.0 / (iI1 + iI2)), rlim, __int_as_float(kb), 0.f);
        if (p.warm == TR_WARM_COLD) Lr = make_float4(0.f, 0.f, 0.f, 0.f);
        Lr.w = 0.f;
        b.lamr0[pos] = Lr;  // unprojected: the start's lambda_n decides the bound
        Lr = project_roll(Lr, rlim * fabsf(L.x));
        b.lamr[pos] = Lr;
    }
    warm_record(L, make_float4(nf[0], nf[1], nf[2], (float)l1), (float)l2, ib, Lr, p.mu_r > 0.f, b.wrec + 3 * (size_t)c);
}

void launch_rows(const DevBuffers& b, const StepParams& p, const Sizes& z, bool have_prev, bool features,
                 hipStream_t s)
{
    const int flags = (have_prev ? kRowsPrev : 0) | (features ? kRowsFeatures : 0) | (z.flow ? kRowsSeq : 0);
    hipLaunchKernelGGL(k_rows, dim3((unsigned)cdiv(z.C, kBlk)), dim3(kBlk), 0, s, b, p, z.C, flags);
}

// Impact stage set-up: the stage's impulses start at zero, and the rows of an
// env without impacts do nothing (zero inverse masses: the stage leaves that
// env as it is, as if solved alone).
__global__ void k_impact_prep(DevBuffers b, StepParams p, int64_t cap)
{
    uint32_t nc = n_contacts(b, cap);
    uint32_t pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= nc) return;
    if (b.cnt->overflow) return;
    b.lami[pos] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (p.mu_r > 0.f) b.lamri[pos] = make_float4(0.f, 0.f, 0.f, 0.f);
    const int ib = __float_as_int(b.ri2[pos].w);
    const int e = (int)((uint32_t)b.pid[ib] / p.id_cap);
    if (b.env_stats[e].impacts == 0) {
        float4 r = b.ri1[pos];
        b.ri1[pos] = make_float4(r.x, 0.f, 0.f, 0.f);
    }
}

// After the impact stage: the main rows' velocity term from the post-impact
// velocities, q = qg + Upsilon G_n v+ (envs with impacts; the others keep q).
__global__ void k_impact_q(DevBuffers b, StepParams p, int64_t cap)
{
    uint32_t nc = n_contacts(b, cap);
    uint32_t pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= nc) return;
    if (b.cnt->overflow) return;
    float4 q = b.r2[pos];
    const int ia = __float_as_int(q.z), ib = __float_as_int(q.w);
    const int e = (int)((uint32_t)b.pid[ib] / p.id_cap);
    if (b.env_stats[e].impacts == 0) return;
    const float4 a = b.r0[pos], v2 = vel_at(b.vw, ib);
    double v1[3];
    if (ia >= 0) {
        const float4 t = vel_at(b.vw, ia);
        v1[0] = t.x; v1[1] = t.y; v1[2] = t.z;
    } else {
        const float4 k = b.rk[pos];
        v1[0] = k.x; v1[1] = k.y; v1[2] = k.z;
    }
    double un = ((double)a.x * ((double)v2.x - v1[0]) + (double)a.y * ((double)v2.y - v1[1])) +
                (double)a.z * ((double)v2.z - v1[2]);
    q.x = (float)((double)b.qg[pos] + p.b_coef * un);
    b.r2[pos] = q;
}

void launch_impact_stage(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s)
{
    if (!(p.v_imp > 0.f)) return;
    const dim3 g((unsigned)cdiv(z.C, kBlk));
    hipLaunchKernelGGL(k_impact_prep, g, dim3(kBlk), 0, s, b, p, z.C);
    DevBuffers bi = b;
    bi.r1 = b.ri1;
    bi.r2 = b.ri2;
    bi.lam = b.lami;
    bi.lamr = b.lamri;
    StepParams pi = p;
    pi.gamma_dt = 0.f;
    launch_pgs(bi, pi, z, s, -1, kSlotImpact);
    hipLaunchKernelGGL(k_impact_q, g, dim3(kBlk), 0, s, b, p, z.C);
}

// ---------------------------------------------------------------------------
// v* = v + dt g + M^-1 G^T lambda^0, gathered per particle over its sorted
// incidence list (fixed order) from the contacts' records in canonical order
// (one 32 or 48 B record per incident contact)
// ---------------------------------------------------------------------------
__global__ void k_warm_apply(DevBuffers b, StepParams p)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n_particles) return;
    if (b.cnt->overflow) return;
    const bool roll = p.mu_r > 0.f;
    float4 v = vel_at(b.vw, s), w = angv_at(b.vw, s);
    v.x += p.dt * p.g[0];
    v.y += p.dt * p.g[1];
    v.z += p.dt * p.g[2];
    uint32_t beg = b.inc_start[s], end = b.inc_start[s + 1];
    for (uint32_t t = beg; t < end; ++t) {
        const float4* r = b.wrec + 3 * (size_t)b.inc[t];
        float4 R0 = r[0], R1 = r[1];
        if (!roll && R0.x == 0.f && R0.y == 0.f && R0.z == 0.f) continue;
        float sgn, W0, W1, W2;
        if (__float_as_int(R0.w) == s) { sgn = 1.f; W0 = R1.x; W1 = R1.y; W2 = R1.z; }
        else {
            float4 R2 = r[2];
            sgn = -1.f; W0 = R1.w; W1 = R2.x; W2 = R2.y;
        }
        v.x += sgn * v.w * R0.x; v.y += sgn * v.w * R0.y; v.z += sgn * v.w * R0.z;
        w.x += sgn * w.w * W0; w.y += sgn * w.w * W1; w.z += sgn * w.w * W2;
    }
    vel_at(b.vw, s) = v;
    angv_at(b.vw, s) = w;
}

// the records again from the colour-ordered impulses and rows, after a
// kernel other than k_rows has set the start impulses
__global__ void k_warm_rec(DevBuffers b, StepParams p, int64_t cap)
{
    uint32_t nc = n_contacts(b, cap);
    uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    if (b.cnt->overflow) return;
    const uint32_t pos = b.cpos[c];
    const bool roll = p.mu_r > 0.f;
    warm_record(b.lam[pos], b.r0[pos], b.r1[pos].x, __float_as_int(b.r2[pos].w),
                roll ? b.lamr[pos] : make_float4(0.f, 0.f, 0.f, 0.f), roll, b.wrec + 3 * (size_t)c);
}

void launch_warm_apply(const DevBuffers& b, const StepParams& p, const Sizes& z, bool rebuild, hipStream_t s)
{
    if (rebuild) hipLaunchKernelGGL(k_warm_rec, dim3((unsigned)cdiv(z.C, kBlk)), dim3(kBlk), 0, s, b, p, z.C);
    if (p.n_particles <= 0) return;
    hipLaunchKernelGGL(k_warm_apply, dim3((unsigned)cdiv(p.n_particles, kBlk)), dim3(kBlk), 0, s, b, p);
}

// ---------------------------------------------------------------------------
// A9: persistent projected Gauss-Seidel.  Sweeps x colours; inside a colour
// no two contacts share a dynamic particle, so every contact updates its two
// bodies without atomics, and any schedule of a colour's contacts gives the
// same result.
//
// A solve is run by a cluster of blocks that meet at a counter barrier after
// every colour.  Grouped mode: envs are split into kGroups groups, group g
// runs on the blocks b with b % 8 == g.  Per-env mode: every env has its own
// cluster (one block for most envs, whose bodies then sit in LDS and whose
// barrier is a workgroup barrier).  On MI355X consecutive blocks of a launch
// go to the 8 XCDs in turn, so a cluster whose blocks are congruent mod 8
// shares one XCD and its L2: bodies
// are then written with ordinary stores (write-through to that L2) and read
// with device-scope (sc1) loads, which miss the per-CU L1; measured, L1-hit
// loads return data another CU of the XCD has already replaced, and sc1
// stores cost twice the solve time.  Each cluster checks its placement once
// per launch and falls back to agent-scope fences around its barriers when a
// block is not on the expected XCD.
//
// Contact c of a colour is always handled by the same thread, so its rows
// (read-only) and impulses (thread-owned) use the ordinary caches, and the
// rows of the next contact are in flight while the current one is updated.
// The residual R_k = ||d lambda||_D / ||lambda||_D of each sweep is reduced
// per block in a fixed order and combined identically by every block of the
// cluster, which then all take the same stopping decision.
// ---------------------------------------------------------------------------
constexpr int kPgsBlk = 512;
constexpr int kCoherent = 16;  // cache-policy bits of a device-scope (sc1) access

__device__ inline __amdgpu_buffer_rsrc_t raw_rsrc(const void* p)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, 0x7fffffff, 0x00020000);
}
template <int AUX>
__device__ inline float4 ld_body(__amdgpu_buffer_rsrc_t r, int idx)
{
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, idx * 16, 0, AUX));
}
template <int AUX>
__device__ inline void st_body(__amdgpu_buffer_rsrc_t r, int idx, float4 v)
{
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, idx * 16, 0, AUX);
}

// XCD (accelerator complex die) this wave runs on
__device__ inline unsigned xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 0xf; }

// Bounded wait for a barrier counter to reach target; false on timeout or
// when another block has reported a failed barrier.
__device__ inline bool wait_counter(Counters* cnt, uint32_t* counter, unsigned target)
{
    long spins = 0;
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 1023) == 0 &&
            (__hip_atomic_load(&cnt->overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFailBarrier))
            return false;
        if (spins > kBarrierSpins) {
            atomicOr(&cnt->overflow, kFailBarrier);
            return false;
        }
    }
    return true;
}

// Cluster barrier on counter[0] (zeroed before the launch).  Arrive drains
// this block's stores; wait returns false when the barrier failed.
template <bool FENCED>
__device__ inline void cluster_arrive(uint32_t* counter)
{
    if (FENCED) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool FENCED>
__device__ inline bool cluster_wait(Counters* cnt, uint32_t* counter, unsigned target, int& flag)
{
    if (threadIdx.x == 0) flag = wait_counter(cnt, counter, target) ? 1 : 0;
    __syncthreads();
    if (FENCED) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return flag != 0;
}

// Spread mode: after each colour the eight groups meet.  The blocks of a group
// arrive at its counter (cluster_arrive); the group's rank-0 block waits for
// them, arrives at the global counter and waits for all groups, then releases
// its group through the group's release word (counter[2]).  nbar counts the
// group's barriers including the first (placement) one, which the global
// counter does not see.  Returns false when a wait failed.
template <bool FENCED>
__device__ inline bool spread_wait(Counters* cnt, uint32_t* counter, unsigned nbar, unsigned K, unsigned rank,
                                   int& flag)
{
    if (threadIdx.x == 0) {
        bool ok;
        if (rank == 0) {
            ok = wait_counter(cnt, counter, nbar * K);
            if (ok) {
                __hip_atomic_fetch_add(&cnt->gbar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = wait_counter(cnt, &cnt->gbar[0], (nbar - 1) * (unsigned)kGroups);
            }
            if (ok) __hip_atomic_store(&counter[2], nbar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            ok = wait_counter(cnt, &counter[2], nbar);
        }
        flag = ok ? 1 : 0;
    }
    __syncthreads();
    if (FENCED) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return flag != 0;
}

// First barrier of a launch: every block of the cluster sets the bit of its
// XCD in counter[1] (zeroed before the launch).  The round-robin dispatch
// puts blocks congruent mod 8 on one XCD, but which XCD depends on the
// launches before, so only "one XCD for the whole cluster" is checked.
// Returns 1 for XCD-local accesses, 2 for the fenced fallback, 0 when the
// barrier failed; uniform over the cluster.
__device__ inline int cluster_placement(Counters* cnt, uint32_t* counter, unsigned size, int& flag)
{
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_or(&counter[1], 1u << xcc_id(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_s_waitcnt(0);
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        flag = 0;
        if (wait_counter(cnt, counter, size)) {
            uint32_t xcds = __hip_atomic_load(&counter[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            flag = __popc(xcds) == 1 ? 1 : 2;
        }
    }
    __syncthreads();
    return flag;
}

// A contact's rows as the update reads them.  rk (the kinematic velocity of
// a boundary contact, the update sequence of the counter-ordered schedule)
// is fetched with them only by the grouped solve (kin), whose colour phases
// are latency-bound on one XCD; elsewhere the update of a boundary contact
// loads it itself, so a pair's row stream is 48 B of rows and the impulses
// (measured: 256-bed batch PGS 11.1-11.2 -> 9.9-10.0 ms, 500k excavation
// 29.4 -> 26.9 ms; 50k bed 7.1 -> 7.4 ms, hence kin there; same states).
struct RowRegs {
    float4 a, r1, q, L;
    float4 k;       // rk, when fetched with the rows
    float4 r3, Lr;  // rolling rows (loaded when mu_r > 0)
};

__device__ inline RowRegs load_rows(const DevBuffers& b, uint32_t c, bool roll, bool kin = false)
{
    RowRegs R;
    R.a = b.r0[c];
    R.r1 = b.r1[c];
    R.q = b.r2[c];
    R.L = b.lam[c];
    if (kin) R.k = b.rk[c];
    if (roll) {
        R.r3 = b.r3[c];
        R.Lr = b.lamr[c];
    }
    return R;
}

// Body state accessors of the contact update.  Xcd: sc1 loads and ordinary
// stores, for clusters whose blocks share one XCD.  Plain: ordinary accesses,
// for a solve confined to one block (its waves share one CU and its L1) or
// ordered by agent-scope fences.  Lds: the env's bodies staged in LDS.
struct XcdBodies {
    __amdgpu_buffer_rsrc_t r;  // vw: record i is float4 2i (v) and 2i + 1 (omega)
    __device__ float4 v(int i) const { return ld_body<kCoherent>(r, 2 * i); }
    __device__ float4 w(int i) const { return ld_body<kCoherent>(r, 2 * i + 1); }
    __device__ void set(int i, float4 v, float4 w) const { st_body<0>(r, 2 * i, v); st_body<0>(r, 2 * i + 1, w); }
    __device__ float4 half(int i, int h) const { return ld_body<kCoherent>(r, 2 * i + h); }
    __device__ void set_half(int i, int h, float4 v) const { st_body<0>(r, 2 * i + h, v); }
    // half h of record i into LDS at wave_lds + 16 B x lane (a load straight to LDS)
    __device__ void stage_half(float4* wave_lds, int i, int h) const
    {
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)wave_lds, 16,
                                                 (2 * i + h) * 16, 0, 0, kCoherent);
    }
};
// Spread mode: one env's contacts on all XCDs, so every body store is written
// through (sc1) and every load is device-scope: measured on MI355X, such a
// store is seen by another XCD's device-scope load once it has completed.
struct SpreadBodies {
    __amdgpu_buffer_rsrc_t r;
    __device__ float4 v(int i) const { return ld_body<kCoherent>(r, 2 * i); }
    __device__ float4 w(int i) const { return ld_body<kCoherent>(r, 2 * i + 1); }
    __device__ void set(int i, float4 v, float4 w) const
    {
        st_body<kCoherent>(r, 2 * i, v);
        st_body<kCoherent>(r, 2 * i + 1, w);
    }
    __device__ float4 half(int i, int h) const { return ld_body<kCoherent>(r, 2 * i + h); }
    __device__ void set_half(int i, int h, float4 v) const { st_body<kCoherent>(r, 2 * i + h, v); }
    __device__ void stage_half(float4* wave_lds, int i, int h) const
    {
        __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)wave_lds, 16,
                                                 (2 * i + h) * 16, 0, 0, kCoherent);
    }
};
struct PlainBodies {
    float4* vw;
    __device__ float4 v(int i) const { return vel_at(vw, i); }
    __device__ float4 w(int i) const { return angv_at(vw, i); }
    __device__ void set(int i, float4 v, float4 w) const { vel_at(vw, i) = v; angv_at(vw, i) = w; }
    __device__ float4 half(int i, int h) const { return vw[2 * i + h]; }
    __device__ void set_half(int i, int h, float4 v) const { vw[2 * i + h] = v; }
    __device__ void stage_half(float4* wave_lds, int i, int h) const
    {
        __builtin_amdgcn_global_load_lds((const void*)&vw[2 * i + h], (__attribute__((address_space(3))) void*)wave_lds,
                                         16, 0, 0);
    }
};
struct LdsBodies {
    float4 *sv, *sw;  // env slots [base, base + n)
    int base;
    __device__ float4 v(int i) const { return sv[i - base]; }
    __device__ float4 w(int i) const { return sw[i - base]; }
    __device__ void set(int i, float4 v, float4 w) const { sv[i - base] = v; sw[i - base] = w; }
};

// An env solved by one block whose spheres do not all fit its LDS: the
// first cap slots in LDS, the others in global memory (one block, one CU:
// plain accesses are ordered by its workgroup barriers)
struct MixedBodies {
    float4 *sv, *sw;
    int base, cap;
    float4* vw;
    __device__ bool lds(int i) const { return (unsigned)(i - base) < (unsigned)cap; }
    __device__ float4 v(int i) const { return lds(i) ? sv[i - base] : vel_at(vw, i); }
    __device__ float4 w(int i) const { return lds(i) ? sw[i - base] : angv_at(vw, i); }
    __device__ void set(int i, float4 v, float4 w) const
    {
        if (lds(i)) {
            sv[i - base] = v;
            sw[i - base] = w;
        } else {
            vel_at(vw, i) = v;
            angv_at(vw, i) = w;
        }
    }
};

// the two bodies of a contact, loaded ahead of the update (the update
// replaces body 1 of a boundary contact by the boundary's velocity)
struct BodyRegs {
    float4 va, wa, vb, wb;
};

// unconditional loads (a boundary contact reads its sphere twice): no
// divergent branch between the loads and their use
template <class BA>
__device__ inline BodyRegs load_bodies(const BA& ba, const RowRegs& R)
{
    BodyRegs B;
    const int ia = __float_as_int(R.q.z), ib = __float_as_int(R.q.w);
    const int ja = ia >= 0 ? ia : ib;
    B.vb = ba.v(ib);
    B.wb = ba.w(ib);
    B.va = ba.v(ja);
    B.wa = ba.w(ja);
    return B;
}

// Lane pairs.  A wave's body loads and stores scatter: each lane's 16 B
// lands in its own memory line, and the vector memory unit's throughput in
// lines, not bytes, bounds the colour phase.  Lanes 2k and 2k+1 therefore
// access the two 32 B records of their two contacts' sphere together: the
// even lane the velocity half and the odd lane the angular half of the even
// lane's record, then the same for the odd lane's record, and exchange what
// the other needs.  Two lanes share each line an instruction touches; the
// values are those of the lane's own loads and stores.  Both lanes of a pair
// must be active (the swap reads the partner); a lane without a contact
// loads its partner's records and stores nothing.
__device__ inline int pair_swap(int x) { return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false); }
__device__ inline float pair_swap(float x) { return __int_as_float(pair_swap(__float_as_int(x))); }
__device__ inline float4 pair_swap(float4 x)
{
    return make_float4(pair_swap(x.x), pair_swap(x.y), pair_swap(x.z), pair_swap(x.w));
}

// the record of sphere self (own: the lane has a contact) as (v, w)
template <class BA>
__device__ inline void pair_load(const BA& ba, int self, bool own, int odd, float4& v, float4& w)
{
    int part = pair_swap(own ? self : -1);
    if (!own) self = part;      // no contact: the partner's record, never stored
    if (part < 0) part = self;  // the partner has no contact: this lane's record twice
    const int r1 = odd ? part : self, r2 = odd ? self : part;  // the even lane's sphere, the odd lane's
    const float4 x1 = ba.half(r1, odd), x2 = ba.half(r2, odd);
    const float4 recv = pair_swap(odd ? x1 : x2);
    v = odd ? recv : x1;
    w = odd ? x2 : recv;
}

// stores (v, w) as the record of sphere self when want
template <class BA>
__device__ inline void pair_store(const BA& ba, int self, bool want, int odd, float4 v, float4 w)
{
    const int part = pair_swap(self);
    const bool pwant = pair_swap(want ? 1 : 0) != 0;
    const float4 recv = pair_swap(odd ? v : w);
    const int r1 = odd ? part : self, r2 = odd ? self : part;
    if (odd ? pwant : want) ba.set_half(r1, odd, odd ? recv : v);
    if (odd ? want : pwant) ba.set_half(r2, odd, odd ? w : recv);
}

template <class BA>
__device__ inline BodyRegs pair_bodies(const BA& ba, const RowRegs& R, bool own, int odd)
{
    BodyRegs B;
    const int ia = __float_as_int(R.q.z), ib = __float_as_int(R.q.w);
    pair_load(ba, ib, own, odd, B.vb, B.wb);
    pair_load(ba, ia >= 0 ? ia : ib, own, odd, B.va, B.wa);
    return B;
}

template <class BA>
__device__ inline void pair_store_bodies(const BA& ba, const RowRegs& R, const BodyRegs& B, bool own, int odd)
{
    const int ia = __float_as_int(R.q.z), ib = __float_as_int(R.q.w);
    pair_store(ba, ib, own, odd, B.vb, B.wb);
    pair_store(ba, ia, own && ia >= 0, odd, B.va, B.wa);
}

// a contact's bodies with lane pairs (LANES) or by each lane alone (then own
// is true wherever these are called)
template <bool LANES, class BA>
__device__ inline BodyRegs get_bodies(const BA& ba, const RowRegs& R, bool own, int odd)
{
    if (LANES) return pair_bodies(ba, R, own, odd);
    return load_bodies(ba, R);
}
template <bool LANES, class BA>
__device__ inline void put_bodies(const BA& ba, const RowRegs& R, const BodyRegs& B, bool own, int odd)
{
    if (LANES) {
        pair_store_bodies(ba, R, B, own, odd);
        return;
    }
    const int ia = __float_as_int(R.q.z), ib = __float_as_int(R.q.w);
    ba.set(ib, B.vb, B.wb);
    if (ia >= 0) ba.set(ia, B.va, B.wa);
}

// Staging of a thread's second contact of a colour in LDS (1024-thread
// blocks, which have no registers for two contacts in flight).  The layout,
// in float4 per block thread t: rows a, r1, q, L at [j nthr + t], j < 4;
// then the lane pairs' body halves x1, x2 of sphere b and of sphere a at
// [(4 + j) nthr + t], j < 4, as pair_load leaves them in registers.  Loads go
// straight to LDS (16 B per lane, lane order), so the second contact's rows
// are fetched during the barrier and its bodies during the first contact's
// update, without registers.
constexpr int kStageFloat4 = 8;  // float4 per block thread

__device__ inline void stage_rows(const DevBuffers& b, float4* st, uint32_t nthr, uint32_t c)
{
    const uint32_t w = threadIdx.x & ~63u;
    const float4* src[4] = {b.r0, b.r1, b.r2, b.lam};
#pragma unroll
    for (int j = 0; j < 4; ++j)
        __builtin_amdgcn_global_load_lds((const void*)&src[j][c],
                                         (__attribute__((address_space(3))) void*)(st + j * nthr + w), 16, 0, 0);
}

// the body halves of the contact whose indices are in q (own: the lane has
// it), into the staging area, as pair_load splits them
template <class BA>
__device__ inline void stage_bodies(const BA& ba, float4* st, uint32_t nthr, float4 q, bool own, int odd)
{
    const uint32_t w = threadIdx.x & ~63u;
    const int ia = __float_as_int(q.z), ib = __float_as_int(q.w);
    int sb = own ? ib : -1, sa = own ? (ia >= 0 ? ia : ib) : -1;
    int pb = pair_swap(sb), pa = pair_swap(sa);
    if (!own) { sb = pb; sa = pa; }
    if (pb < 0) { pb = sb; pa = sa; }
    ba.stage_half(st + 4 * nthr + w, odd ? pb : sb, odd);
    ba.stage_half(st + 5 * nthr + w, odd ? sb : pb, odd);
    ba.stage_half(st + 6 * nthr + w, odd ? pa : sa, odd);
    ba.stage_half(st + 7 * nthr + w, odd ? sa : pa, odd);
}

__device__ inline RowRegs staged_rows(const float4* st, uint32_t nthr)
{
    const uint32_t t = threadIdx.x;
    RowRegs R;
    R.a = st[t];
    R.r1 = st[nthr + t];
    R.q = st[2 * nthr + t];
    R.L = st[3 * nthr + t];
    return R;
}

__device__ inline BodyRegs staged_bodies(const float4* st, uint32_t nthr, int odd)
{
    const uint32_t t = threadIdx.x, p = t ^ 1u;
    BodyRegs B;
    B.vb = odd ? st[5 * nthr + p] : st[4 * nthr + t];
    B.wb = odd ? st[5 * nthr + t] : st[4 * nthr + p];
    B.va = odd ? st[7 * nthr + p] : st[6 * nthr + t];
    B.wa = odd ? st[7 * nthr + t] : st[6 * nthr + p];
    return B;
}

// One contact's update on the loaded bodies B (left in B), its impulses
// written; the caller stores the bodies.
__device__ inline void pgs_update(const DevBuffers& b, uint32_t c, const RowRegs& R, BodyRegs& B, float mu, float gdt,
                                  float& num, float& den, bool roll, bool kin = false)
{
    float4 a = R.a, r1 = R.r1, q = R.q, L = R.L;
    bool pair = __float_as_int(q.z) >= 0;
    float4 vb = B.vb, wb = B.wb, va = B.va, wa = B.wa;
    if (!pair) {
        const float4 kv = kin ? R.k : b.rk[c];  // the boundary's velocity at the contact point
        va = make_float4(kv.x, kv.y, kv.z, 0.f);
        wa = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float nx = a.x, ny = a.y, nz = a.z, l1 = a.w;
    float l2 = r1.x, iDn = r1.y, iDt = r1.z, Sig = r1.w;
    // normal row
    float un = nx * (vb.x - va.x) + ny * (vb.y - va.y) + nz * (vb.z - va.z);
    float ln = fmaxf(q.y, L.x - (un + Sig * L.x - q.x) * iDn);
    float dn = ln - L.x;
    vb.x += dn * nx * vb.w; vb.y += dn * ny * vb.w; vb.z += dn * nz * vb.w;
    va.x -= dn * nx * va.w; va.y -= dn * ny * va.w; va.z -= dn * nz * va.w;
    // tangential disk row: u = (vb - va) - (l2 wb + l1 wa) x n
    float sx = l2 * wb.x + l1 * wa.x, sy = l2 * wb.y + l1 * wa.y, sz = l2 * wb.z + l1 * wa.z;
    float ux = (vb.x - va.x) - (sy * nz - sz * ny);
    float uy = (vb.y - va.y) - (sz * nx - sx * nz);
    float uz = (vb.z - va.z) - (sx * ny - sy * nx);
    float udn = ux * nx + uy * ny + uz * nz;
    ux -= udn * nx; uy -= udn * ny; uz -= udn * nz;
    float tx = L.y - (ux + gdt * L.y) * iDt;
    float ty = L.z - (uy + gdt * L.z) * iDt;
    float tz = L.w - (uz + gdt * L.w) * iDt;
    float lim = mu * fabsf(ln);
    float m2 = tx * tx + ty * ty + tz * tz;
    if (m2 > lim * lim) {
        float sc = m2 > 0.f ? lim * rsqrtf(m2) : 0.f;
        tx *= sc; ty *= sc; tz *= sc;
    }
    float dx = tx - L.y, dy = ty - L.z, dz = tz - L.w;
    // impulse d at the contact point: +d on body 2 (arm -l2 n), -d on body 1 (arm +l1 n)
    float cx = ny * dz - nz * dy, cy = nz * dx - nx * dz, cz = nx * dy - ny * dx;  // n x d
    vb.x += dx * vb.w; vb.y += dy * vb.w; vb.z += dz * vb.w;
    wb.x -= l2 * wb.w * cx; wb.y -= l2 * wb.w * cy; wb.z -= l2 * wb.w * cz;
    if (pair) {
        va.x -= dx * va.w; va.y -= dy * va.w; va.z -= dz * va.w;
        wa.x -= l1 * wa.w * cx; wa.y -= l1 * wa.w * cy; wa.z -= l1 * wa.w * cz;
    }
    // residual weights (the stopping test only): hardware reciprocals; a row
    // with zero inverse mass (a neutralised impact-stage row) weighs nothing
    float Dn = iDn > 0.f ? __builtin_amdgcn_rcpf(iDn) : 0.f, Dt = iDt > 0.f ? __builtin_amdgcn_rcpf(iDt) : 0.f;
    num += Dn * dn * dn + Dt * (dx * dx + dy * dy + dz * dz);
    den += Dn * ln * ln + Dt * (tx * tx + ty * ty + tz * tz);
    if (roll) {
        // rolling row (Eq. signCoul3): zero relative angular velocity, the
        // torque impulse on the disk |lambda_r| <= r mu_r |lambda_n|
        float4 Lr = R.Lr;
        float ox = 0.f, oy = 0.f, oz = 0.f;
        if (pair) { ox = wa.x; oy = wa.y; oz = wa.z; }
        else {
            const BodyDev& K = b.bodies[__float_as_int(R.r3.z)];
            ox = (float)K.angvel[0]; oy = (float)K.angvel[1]; oz = (float)K.angvel[2];
        }
        float iWr = R.r3.x;
        float rx = Lr.x - (wb.x - ox) * iWr, ry = Lr.y - (wb.y - oy) * iWr, rz = Lr.z - (wb.z - oz) * iWr;
        float rlim = R.r3.y * fabsf(ln);
        float r2 = rx * rx + ry * ry + rz * rz;
        if (r2 > rlim * rlim) {
            float sc = r2 > 0.f ? rlim * rsqrtf(r2) : 0.f;
            rx *= sc; ry *= sc; rz *= sc;
        }
        float ex = rx - Lr.x, ey = ry - Lr.y, ez = rz - Lr.z;
        wb.x += wb.w * ex; wb.y += wb.w * ey; wb.z += wb.w * ez;
        if (pair) { wa.x -= wa.w * ex; wa.y -= wa.w * ey; wa.z -= wa.w * ez; }
        b.lamr[c] = make_float4(rx, ry, rz, 0.f);
        float Wr = __builtin_amdgcn_rcpf(iWr);
        num += Wr * (ex * ex + ey * ey + ez * ez);
        den += Wr * (rx * rx + ry * ry + rz * rz);
    }
    b.lam[c] = make_float4(ln, tx, ty, tz);
    B.vb = vb; B.wb = wb; B.va = va; B.wa = wa;
}

template <class BA>
__device__ inline void pgs_contact(const DevBuffers& b, const BA& ba, uint32_t c, const RowRegs& R, BodyRegs B,
                                   float mu, float gdt, float& num, float& den, bool roll)
{
    pgs_update(b, c, R, B, mu, gdt, num, den, roll);
    const int ia = __float_as_int(R.q.z), ib = __float_as_int(R.q.w);
    ba.set(ib, B.vb, B.wb);
    if (ia >= 0) ba.set(ia, B.va, B.wa);
}

// block sums of the sweep's (num, den) in a fixed order, returned to every thread
template <int NW>
__device__ inline void block_sum2(float num, float den, double (*red)[NW], double& sn, double& sd)
{
    double dnum = num, dden = den;
    for (int o = 32; o > 0; o >>= 1) {
        dnum += __shfl_down(dnum, o, 64);
        dden += __shfl_down(dden, o, 64);
    }
    if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = dnum; red[1][threadIdx.x >> 6] = dden; }
    __syncthreads();
    sn = 0.0; sd = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { sn += red[0][w]; sd += red[1][w]; }
    __syncthreads();  // red is reused
}

// Counter-ordered updates: contact c is update number s deg_j + pos_j of
// sphere j in sweep s (pos_j: its rank among j's contacts by colour), so it
// may run once j's counter shows that many updates; afterwards it drains its
// stores and advances the counters.  This keeps the colour order of every
// sphere's updates without barriers between colours.  The waits are bounded
// and give up when another wait has failed.
__device__ inline bool flow_wait(Counters* cnt, const uint32_t* ver, int j, uint32_t want)
{
    long spins = 0;
    while (__hip_atomic_load(&ver[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != want) {
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 255) == 0) {
            if (__hip_atomic_load(&cnt->overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFailBarrier)
                return false;
            if (spins > kBarrierSpins) {
                atomicOr(&cnt->overflow, kFailBarrier);
                return false;
            }
        }
    }
    return true;
}

// The PGS sweeps of one cluster.  Its contacts of colour col are
// [cstart.beg(col), cstart.end(col)); the block of rank r of K takes the r-th of K
// equal slices.  Blocks of the cluster are first + 8 t, t < K.  FLOW: colours
// are ordered by the per-sphere counters (clusters only); a barrier remains at
// the end of a sweep when a residual tolerance is set, and once at the end.
template <class BA, bool CLUSTER, bool FENCED, bool FLOW, bool ROLL, int NW, class Starts, bool SPREAD = false>
__device__ void pgs_solve(const DevBuffers& b, const StepParams& p, const BA& ba, Starts cstart, uint32_t ncol,
                          uint32_t* counter, unsigned nbar, unsigned rank, unsigned K, unsigned first, int sweeps_cap,
                          int slot, int unit, double (*red)[NW], uint32_t (*cb)[kMaxColours], int& flag,
                          float4* stage = nullptr)
{
    int sweeps = 0;
    double Rk = 0.0, R1 = 0.0;
    const unsigned nblk = gridDim.x;
    constexpr uint32_t kThreads = NW * 64;  // the launch's block size (a constant stride)
    bool alive = true;
    // Trailing colours of at most one block's threads each are solved by the
    // rank-0 block alone, with workgroup barriers between them and a single
    // cluster barrier after the last (same colour order, same results).
    // colour bounds staged in LDS (cb: the kernel's) once: no global load
    // between a barrier and the next colour's row prefetch
    uint32_t* cbeg = cb[0];
    uint32_t* clen = cb[1];
    for (uint32_t q = threadIdx.x; q < ncol; q += blockDim.x) {
        cbeg[q] = cstart.beg(q);
        clen[q] = cstart.end(q) - cbeg[q];
    }
    __syncthreads();
    uint32_t tail = ncol;
    if (CLUSTER && !FLOW && !SPREAD)
        while (tail > 0 && clen[tail - 1] <= kThreads) --tail;
    auto range = [&](uint32_t col, uint32_t& lo, uint32_t& hi) {
        uint32_t beg = cbeg[col], len = clen[col];
        if (col >= tail) {
            lo = beg;
            hi = rank == 0 ? beg + len : beg;
            return;
        }
        lo = beg + (uint32_t)(((uint64_t)len * rank) / K);
        hi = beg + (uint32_t)(((uint64_t)len * (rank + 1)) / K);
    };
    // The cluster's (num, den) of sweep sw, the same value in every thread of
    // every block: wave 0 loads the K block partials in parallel and sums them
    // in a fixed tree order, the result is broadcast through LDS.
    auto combine = [&](int sw, double& sn, double& sd) {
        const double* part = b.block_part + (size_t)(FLOW ? sw : (sw & 1)) * nblk * 2;
        if (threadIdx.x < 64) {
            double a = 0.0, d = 0.0;
            // spread mode: the partials of every block of every group
            const unsigned nb = SPREAD ? nblk : K;
            for (unsigned t = threadIdx.x; t < nb; t += 64) {
                const unsigned blk = SPREAD ? t : first + 8 * t;
                a += __hip_atomic_load(&part[2 * blk], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                d += __hip_atomic_load(&part[2 * blk + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            for (int o = 32; o > 0; o >>= 1) {
                a += __shfl_down(a, o, 64);
                d += __shfl_down(d, o, 64);
            }
            if (threadIdx.x == 0) { red[0][0] = a; red[1][0] = d; }
        }
        __syncthreads();
        sn = red[0][0];
        sd = red[1][0];
        __syncthreads();  // red is reused
    };
    auto resid = [](double sn, double sd) { return sd > 0.0 ? sqrt(sn) / sqrt(sd) : (sn > 0.0 ? 1.0 : 0.0); };
    uint32_t lo = 0, hi = 0, c = 0;
    // 512-thread instances: a thread's first contact of a colour and, when the
    // colour needs a second pass, its second, both fetched ahead (while the
    // block waits at a barrier), and the following two fetched during their
    // updates.  The 1024-thread instances take one contact at a time (two
    // would spill registers: measured slower).  Lane pairs (pair_load) in
    // every instance but the rolling 1024-thread one, which has no registers
    // for them.
    constexpr bool kPair = !FLOW && NW <= 8;
    constexpr bool kLanes = !FLOW && (NW <= 8 || !ROLL);
    // the 1024-thread plain instance: a thread's second contact of a colour
    // staged in LDS (stage_rows) when the block has the room
    constexpr bool kStage = kLanes && !kPair && !ROLL;
    constexpr bool kKin = NW <= 8 && !SPREAD && !FLOW;  // the grouped solve fetches rk with the rows
    const bool staged = kStage && stage != nullptr;
    RowRegs cur, cur2;
    auto fetch = [&]() {
        if (c < hi) cur = load_rows(b, c, ROLL, kKin);
        if (kPair && c + kThreads < hi) cur2 = load_rows(b, c + kThreads, ROLL, kKin);
        if (staged && c + kThreads < hi) stage_rows(b, stage, kThreads, c + kThreads);
    };
    if (ncol > 0) {
        range(0, lo, hi);
        c = lo + threadIdx.x;
        fetch();
    }
    for (int sw = 0; sw < sweeps_cap && ncol > 0; ++sw) {
        float num = 0.f, den = 0.f;
        double* part = b.block_part + (size_t)(FLOW ? sw : (sw & 1)) * nblk * 2;
        for (uint32_t col = 0; col < ncol; ++col) {
            // the rows prefetched for this colour: settled here, outside the
            // loop, so that the loop waits only for its own loads
            if (!FLOW) __builtin_amdgcn_s_waitcnt(0);
            if (FLOW) {
                while (c < hi) {
                    const uint32_t cn = c + kThreads;
                    RowRegs nxt;
                    if (cn < hi) nxt = load_rows(b, cn, ROLL, kKin);
                    const uint32_t seq = __float_as_uint(b.rk[c].w);
                    const int ia = __float_as_int(cur.q.z), ib = __float_as_int(cur.q.w);
                    const uint32_t wa = (uint32_t)sw * ((seq >> 16) & 255u) + (seq & 255u);
                    const uint32_t wb = (uint32_t)sw * (seq >> 24) + ((seq >> 8) & 255u);
                    if (alive) alive = flow_wait(b.cnt, b.ver, ib, wb) && (ia < 0 || flow_wait(b.cnt, b.ver, ia, wa));
                    if (alive) {
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // body loads after the counters
                        pgs_contact(b, ba, c, cur, load_bodies(ba, cur), p.mu, p.gamma_dt, num, den, ROLL);
                        __builtin_amdgcn_s_waitcnt(0);  // the sphere state has reached the XCD's L2
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                        __hip_atomic_store(&b.ver[ib], wb + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (ia >= 0) __hip_atomic_store(&b.ver[ia], wa + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    cur = nxt;
                    c = cn;
                }
            } else {
                // lane pairs (pair_load): a pair runs while its even lane has a
                // contact (kThreads is even, so the even lane's contacts are
                // c - odd + k kThreads); the odd lane may have one fewer
                const int odd = kLanes ? (int)(threadIdx.x & 1u) : 0;
                bool first = true;  // the second contact of the colour is the staged one
                while (c - odd < hi) {
                    const uint32_t cn = c + kThreads;
                    const bool own = c < hi;
                    if (staged && first && cn - odd < hi) {
                        // the second contact's rows arrived in LDS with the first's
                        // registers; its bodies go there while the first updates
                        const bool own2 = cn < hi;
                        BodyRegs B = get_bodies<kLanes>(ba, cur, own, odd);
                        stage_bodies(ba, stage, kThreads, stage[2 * kThreads + threadIdx.x], own2, odd);
                        pgs_update(b, c, cur, B, p.mu, p.gamma_dt, num, den, ROLL, kKin);
                        put_bodies<kLanes>(ba, cur, B, own, odd);
                        __builtin_amdgcn_s_waitcnt(0);
                        const RowRegs R2 = staged_rows(stage, kThreads);
                        BodyRegs B2 = staged_bodies(stage, kThreads, odd);
                        if (own2) pgs_update(b, cn, R2, B2, p.mu, p.gamma_dt, num, den, ROLL, kKin);
                        put_bodies<kLanes>(ba, R2, B2, own2, odd);
                        first = false;
                        c = cn + kThreads;
                        if (c < hi) cur = load_rows(b, c, ROLL, kKin);  // a third (rare): one chain
                        continue;
                    }
                    first = false;
                    if (kPair && cn - odd < hi) {
                        // two contacts of one colour share no sphere: both gathers
                        // in flight before either update (same order of updates
                        // and of the residual sums as one contact at a time)
                        const bool own2 = cn < hi;
                        BodyRegs B1 = get_bodies<kLanes>(ba, cur, true, odd);
                        BodyRegs B2 = get_bodies<kLanes>(ba, cur2, own2, odd);
                        const uint32_t c3 = cn + kThreads;
                        RowRegs n1, n2;
                        if (c3 < hi) n1 = load_rows(b, c3, ROLL, kKin);
                        if (c3 + kThreads < hi) n2 = load_rows(b, c3 + kThreads, ROLL, kKin);
                        pgs_update(b, c, cur, B1, p.mu, p.gamma_dt, num, den, ROLL, kKin);
                        if (own2) pgs_update(b, cn, cur2, B2, p.mu, p.gamma_dt, num, den, ROLL, kKin);
                        put_bodies<kLanes>(ba, cur, B1, true, odd);
                        put_bodies<kLanes>(ba, cur2, B2, own2, odd);
                        cur = n1;
                        cur2 = n2;
                        c = c3;
                        continue;
                    }
                    BodyRegs B = get_bodies<kLanes>(ba, cur, own, odd);
                    RowRegs nxt;
                    if (cn < hi) nxt = load_rows(b, cn, ROLL, kKin);
                    if (own) pgs_update(b, c, cur, B, p.mu, p.gamma_dt, num, den, ROLL, kKin);
                    put_bodies<kLanes>(ba, cur, B, own, odd);
                    cur = nxt;
                    c = cn;
                }
            }
            if (CLUSTER && !FLOW && col >= tail && col + 1 < ncol) {
                // inside the tail: the block's stores drained, then a workgroup
                // barrier orders the rank-0 block's colours
                __builtin_amdgcn_s_waitcnt(0);
                range(col + 1, lo, hi);
                c = lo + threadIdx.x;
                fetch();
                __syncthreads();
            } else if (CLUSTER && !FLOW) {
                if (col + 1 == ncol && (p.tol > 0.f || sw == 0 || sw + 1 == sweeps_cap)) {
                    // block partials of this sweep, published before the last barrier
                    double sn, sd;
                    block_sum2<NW>(num, den, red, sn, sd);
                    if (threadIdx.x == 0) {
                        __hip_atomic_store(&part[2 * blockIdx.x], sn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(&part[2 * blockIdx.x + 1], sd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                cluster_arrive<FENCED>(counter);
                ++nbar;
                // the next phase's first rows are fetched while the block waits
                range(col + 1 < ncol ? col + 1 : 0, lo, hi);
                c = lo + threadIdx.x;
                fetch();
                if (SPREAD) {
                    if (!spread_wait<FENCED>(b.cnt, counter, nbar, K, rank, flag)) return;  // every block leaves
                } else if (!cluster_wait<FENCED>(b.cnt, counter, nbar * K, flag)) {
                    __builtin_amdgcn_s_waitcnt(0);  // no load into LDS outlives the solve
                    return;                         // every block leaves
                }
            } else {
                range(col + 1 < ncol ? col + 1 : 0, lo, hi);
                c = lo + threadIdx.x;
                fetch();
                if (!CLUSTER) __syncthreads();
            }
        }
        double sn = 0.0, sd = 0.0;
        if (FLOW) {
            block_sum2<NW>(num, den, red, sn, sd);
            if (threadIdx.x == 0) {
                __hip_atomic_store(&part[2 * blockIdx.x], sn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&part[2 * blockIdx.x + 1], sd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            sweeps = sw + 1;
            if (p.tol > 0.f) {
                // the stopping test needs every block's partial of this sweep
                cluster_arrive<false>(counter);
                ++nbar;
                if (!cluster_wait<false>(b.cnt, counter, nbar * K, flag)) return;
                combine(sw, sn, sd);
                Rk = resid(sn, sd);
                if (sw == 0) R1 = Rk;
                if (Rk <= (double)p.tol) break;  // uniform: every block holds the same Rk
            }
            continue;
        }
        if (CLUSTER) {
            // without a tolerance only the first and last residuals are reported
            sweeps = sw + 1;
            if (!(p.tol > 0.f) && sw != 0 && sw + 1 != sweeps_cap) continue;
            combine(sw, sn, sd);
        } else {
            block_sum2<NW>(num, den, red, sn, sd);
        }
        Rk = resid(sn, sd);
        if (sw == 0) R1 = Rk;
        sweeps = sw + 1;
        if (p.tol > 0.f && Rk <= (double)p.tol) break;  // uniform: every thread holds the same Rk
    }
    if (FLOW && ncol > 0 && !(p.tol > 0.f)) {
        // fixed sweep count: the first and last residuals once every block is done
        cluster_arrive<false>(counter);
        ++nbar;
        if (!cluster_wait<false>(b.cnt, counter, nbar * K, flag)) return;
        double sn, sd;
        combine(0, sn, sd);
        R1 = resid(sn, sd);
        combine(sweeps - 1, sn, sd);
        Rk = resid(sn, sd);
    }
    if (staged) __builtin_amdgcn_s_waitcnt(0);  // the last prefetch into LDS has landed
    if (rank == 0 && threadIdx.x == 0 && (!SPREAD || first == 0)) {
        UnitStats& G = b.ustats[unit];
        if (slot == 0) {
            G.sweeps = (uint32_t)sweeps;
            G.resid = Rk;
            G.resid_first = R1;
        } else if (slot == kSlotImpact) {
            G.imp_sweeps = (uint32_t)sweeps;
        } else {
            G.r1_trial[slot - 1] = R1;
        }
    }
}

__global__ void k_pgs_reset(DevBuffers b, int n_envs)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < kGroups) { b.cnt->bar[t][0] = 0; b.cnt->bar[t][1] = 0; b.cnt->bar[t][2] = 0; }
    if (t == 0) b.cnt->gbar[0] = 0;
    if (t < n_envs) { b.env_bar[(size_t)t * 16] = 0; b.env_bar[(size_t)t * 16 + 1] = 0; }
}

// grouped mode: colour col of group g is bucket (col, g) of the bucketing
struct GroupStarts {
    const uint32_t* col_start;
    int64_t NB;
    int g;
    __device__ uint32_t beg(uint32_t col) const { return col_start[((int64_t)col * kGroups + g) * NB]; }
    __device__ uint32_t end(uint32_t col) const { return col_start[((int64_t)col * kGroups + g + 1) * NB]; }
};
// per-env mode: colours of one env are consecutive
struct EnvStarts {
    const uint32_t* ec;
    __device__ uint32_t beg(uint32_t col) const { return ec[col]; }
    __device__ uint32_t end(uint32_t col) const { return ec[col + 1]; }
};

template <bool ROLL>
__global__ __launch_bounds__(kPgsBlk) void k_pgs(DevBuffers b, StepParams p, int64_t NB, int sweeps_cap, int slot,
                                                   int flow)
{
    __shared__ double red[2][kPgsBlk / 64];
    __shared__ uint32_t cb[2][kMaxColours];
    __shared__ int flag;
    if (b.cnt->overflow) return;  // uniform: written by earlier kernels only
    const int g = blockIdx.x % kGroups;
    const unsigned rank = blockIdx.x / kGroups, gx = gridDim.x / kGroups;
    GroupStarts cs{b.col_start, NB, g};
    uint32_t ncol = b.cnt->n_colours;
    uint32_t* counter = &b.cnt->bar[g][0];
    if (p.spread) {
        // spread mode: the groups share one env (unit 0) and meet after every
        // colour, so all of them run every colour, with or without contacts
        if (slot == kSlotImpact && !b.ustats[0].imp_any) ncol = 0;  // no impact in the env
        int mode = cluster_placement(b.cnt, counter, gx, flag);
        if (mode == 1)
            pgs_solve<SpreadBodies, true, false, false, ROLL, kPgsBlk / 64, GroupStarts, true>(
                b, p, SpreadBodies{raw_rsrc(b.vw)}, cs, ncol, counter, 1, rank, gx, (unsigned)g,
                sweeps_cap, slot, 0, red, cb, flag);
        else if (mode == 2)
            pgs_solve<PlainBodies, true, true, false, ROLL, kPgsBlk / 64, GroupStarts, true>(
                b, p, PlainBodies{b.vw}, cs, ncol, counter, 1, rank, gx, (unsigned)g, sweeps_cap, slot, 0, red,
                cb, flag);
        return;
    }
    // a group without contacts only records its (trivial) statistics
    uint32_t total = 0;
    for (uint32_t col = 0; col < ncol; ++col) total += cs.end(col) - cs.beg(col);
    if (total == 0) ncol = 0;
    if (slot == kSlotImpact && !b.ustats[g].imp_any) ncol = 0;  // no impact in the group
    int mode = cluster_placement(b.cnt, counter, gx, flag);
    if (mode == 1) {
        XcdBodies ba{raw_rsrc(b.vw)};
        if (flow)
            pgs_solve<XcdBodies, true, false, true, ROLL>(b, p, ba, cs, ncol, counter, 1, rank, gx, (unsigned)g, sweeps_cap,
                                                    slot, g, red, cb, flag);
        else
            pgs_solve<XcdBodies, true, false, false, ROLL>(b, p, ba, cs, ncol, counter, 1, rank, gx, (unsigned)g,
                                                     sweeps_cap, slot, g, red, cb, flag);
    }
    else if (mode == 2)
        pgs_solve<PlainBodies, true, true, false, ROLL>(b, p, PlainBodies{b.vw}, cs, ncol, counter, 1, rank, gx,
                                                  (unsigned)g, sweeps_cap, slot, g, red, cb, flag);
}

// Per-env mode, a set of small envs solved at once by one block: env j of the
// set runs on waves [wb, we) with its bodies in LDS at offset off (global
// memory when off < 0).  The envs share the workgroup barrier after every
// colour (up to the largest colour count of the set) but reduce their own
// residual, stop on their own and record their own statistics.
template <bool ROLL>
__device__ void pgs_local_set(const DevBuffers& b, const StepParams& p, const int4* tasks, int ntask, int sweeps_cap,
                              int slot, float4* dyn, int lds_cap, double (*red)[kEnvBlk / 64])
{
    const int wave = threadIdx.x >> 6;
    int j = -1;
    uint32_t maxcol = 0;
    for (int t = 0; t < ntask; ++t) {
        const int4 q = tasks[t];
        const int wb = q.y & 255, we = (q.y >> 8) & 255;
        if (wave >= wb && wave < we) j = t;
        maxcol = max(maxcol, b.env_ncol[q.x]);
    }
    int e = -1, wb = 0, we = 1, off = -1;
    if (j >= 0) {
        const int4 q = tasks[j];
        e = q.x; wb = q.y & 255; we = (q.y >> 8) & 255; off = q.w;
    }
    const uint32_t nthr = 64u * (uint32_t)(we - wb), lt = threadIdx.x - 64u * (uint32_t)wb;
    const int sb = e >= 0 ? b.envs[e].slot_begin : 0, n = e >= 0 ? b.envs[e].n : 0;
    LdsBodies lb{dyn + (off >= 0 ? off : 0), dyn + lds_cap + (off >= 0 ? off : 0), sb};
    PlainBodies gb{b.vw};
    // the env's first lcap slots in LDS: all of them when they fit (how 0),
    // none without an LDS offset (how 1), else the rest in global memory (how 2)
    const int lcap = off >= 0 ? min(n, lds_cap - off) : 0;
    const int how = off < 0 ? 1 : (lcap < n ? 2 : 0);
    MixedBodies mb{lb.sv, lb.sw, sb, lcap, b.vw};
    for (int i = (int)lt; i < lcap; i += (int)nthr) {
        lb.sv[i] = vel_at(b.vw, sb + i);
        lb.sw[i] = angv_at(b.vw, sb + i);
    }
    __syncthreads();
    const uint32_t* ec = b.env_col + (size_t)(e >= 0 ? e : 0) * (kMaxColours + 1);
    const uint32_t ncol = e >= 0 && !(slot == kSlotImpact && !b.ustats[e].imp_any) ? b.env_ncol[e] : 0;
    bool active = ncol > 0;  // uniform over the env's waves
    int sweeps = 0;
    double Rk = 0.0, R1 = 0.0;
    uint32_t c = 1, hi = 0;
    RowRegs cur;
    auto start_col = [&](uint32_t col) {
        c = ec[col] + lt;
        hi = ec[col + 1];
        if (c < hi) cur = load_rows(b, c, ROLL);
    };
    if (active) start_col(0);
    for (int sw = 0; sw < sweeps_cap; ++sw) {
        if (!__syncthreads_or(active)) break;
        float num = 0.f, den = 0.f;
        for (uint32_t col = 0; col < maxcol; ++col) {
            if (active && col < ncol) {
                while (c < hi) {
                    uint32_t cn = c + nthr;
                    BodyRegs B = how == 0 ? load_bodies(lb, cur) : how == 1 ? load_bodies(gb, cur) : load_bodies(mb, cur);
                    RowRegs nxt;
                    if (cn < hi) nxt = load_rows(b, cn, ROLL);
                    if (how == 0) pgs_contact(b, lb, c, cur, B, p.mu, p.gamma_dt, num, den, ROLL);
                    else if (how == 1) pgs_contact(b, gb, c, cur, B, p.mu, p.gamma_dt, num, den, ROLL);
                    else pgs_contact(b, mb, c, cur, B, p.mu, p.gamma_dt, num, den, ROLL);
                    cur = nxt;
                    c = cn;
                }
                start_col(col + 1 < ncol ? col + 1 : 0);  // the next phase's first rows
            }
            __syncthreads();
        }
        // the env's residual from its waves' partials, in wave order
        double dnum = num, dden = den;
        for (int o = 32; o > 0; o >>= 1) {
            dnum += __shfl_down(dnum, o, 64);
            dden += __shfl_down(dden, o, 64);
        }
        if ((threadIdx.x & 63) == 0) { red[0][wave] = dnum; red[1][wave] = dden; }
        __syncthreads();
        if (active) {
            double sn = 0.0, sd = 0.0;
            for (int w = wb; w < we; ++w) { sn += red[0][w]; sd += red[1][w]; }
            Rk = sd > 0.0 ? sqrt(sn) / sqrt(sd) : (sn > 0.0 ? 1.0 : 0.0);
            if (sw == 0) R1 = Rk;
            sweeps = sw + 1;
            if (p.tol > 0.f && Rk <= (double)p.tol) active = false;
        }
        __syncthreads();  // red is reused
    }
    for (int i = (int)lt; i < lcap; i += (int)nthr) {
        vel_at(b.vw, sb + i) = lb.sv[i];
        angv_at(b.vw, sb + i) = lb.sw[i];
    }
    if (e >= 0 && lt == 0) {
        UnitStats& G = b.ustats[e];
        if (slot == 0) {
            G.sweeps = (uint32_t)sweeps;
            G.resid = Rk;
            G.resid_first = R1;
        } else if (slot == kSlotImpact) {
            G.imp_sweeps = (uint32_t)sweeps;
        } else {
            G.r1_trial[slot - 1] = R1;
        }
    }
}

// Per-env mode: block b runs plan[plan_idx[b] .. plan_idx[b + 1]) in order: at
// most one share (env, rank, cluster size K >= 2, first block) of a
// multi-block cluster, first, then sets of small envs solved at once (entries
// (env, waves wb | we << 8, 1, LDS offset); a set starts at wb == 0).
template <bool ROLL>
__global__ __launch_bounds__(kEnvBlk) void k_pgs_env(DevBuffers b, StepParams p, int sweeps_cap, int slot, int lds_cap,
                                                      int flow)
{
    HIP_DYNAMIC_SHARED(float4, dyn_bodies)
    __shared__ double red[2][kEnvBlk / 64];
    __shared__ uint32_t cb[2][kMaxColours];
    __shared__ int flag;
    if (b.cnt->overflow) return;  // uniform: written by earlier kernels only
    const uint32_t t0 = b.plan_idx[blockIdx.x], t1 = b.plan_idx[blockIdx.x + 1];
    uint32_t t = t0;
    while (t < t1) {
        const int4 pl = b.plan[t];
        if (pl.z < 2) {
            uint32_t u = t + 1;
            while (u < t1 && b.plan[u].z < 2 && (b.plan[u].y & 255) != 0) ++u;
            pgs_local_set<ROLL>(b, p, b.plan + t, (int)(u - t), sweeps_cap, slot, dyn_bodies, lds_cap, red);
            __syncthreads();  // LDS and the reduction scratch are reused
            t = u;
            continue;
        }
        const int e = pl.x;
        const unsigned rank = pl.y, K = pl.z, first = pl.w;
        EnvStarts cs{b.env_col + (size_t)e * (kMaxColours + 1)};
        const uint32_t ncol = slot == kSlotImpact && !b.ustats[e].imp_any ? 0u : b.env_ncol[e];
        uint32_t* counter = b.env_bar + (size_t)e * 16;
        int mode = cluster_placement(b.cnt, counter, K, flag);
        XcdBodies xb{raw_rsrc(b.vw)};
        // the dynamic LDS (idle during a cluster share) stages second contacts
        float4* stage = 2 * lds_cap >= kStageFloat4 * kEnvBlk ? dyn_bodies : nullptr;
        if (mode == 1 && flow)
            pgs_solve<XcdBodies, true, false, true, ROLL>(b, p, xb, cs, ncol, counter, 1, rank, K, first, sweeps_cap, slot,
                                                    e, red, cb, flag);
        else if (mode == 1)
            pgs_solve<XcdBodies, true, false, false, ROLL>(b, p, xb, cs, ncol, counter, 1, rank, K, first, sweeps_cap, slot,
                                                     e, red, cb, flag, stage);
        else if (mode == 2)
            pgs_solve<PlainBodies, true, true, false, ROLL>(b, p, PlainBodies{b.vw}, cs, ncol, counter, 1, rank, K,
                                                      first, sweeps_cap, slot, e, red, cb, flag, stage);
        if (!flag) return;  // failed barrier: the step is abandoned
        __syncthreads();
        ++t;
    }
}

// dynamic LDS one per-env block may take: the device's limit per block less
// the larger static footprint of the two kernel instances
int pgs_env_max_lds()
{
    int dev = 0, lds = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    hipFuncAttributes a0{}, a1{};
    size_t st = 2048;  // if the attributes cannot be read
    if (hipFuncGetAttributes(&a0, (const void*)k_pgs_env<false>) == hipSuccess &&
        hipFuncGetAttributes(&a1, (const void*)k_pgs_env<true>) == hipSuccess)
        st = std::max(a0.sharedSizeBytes, a1.sharedSizeBytes);
    return std::max(0, lds - (int)((st + 255) / 256 * 256));
}

// blocks of either PGS instance (plain or with rolling rows) resident at once:
// the persistent solves rely on every block of a cluster being resident
int pgs_env_resident_blocks(int lds_bytes)
{
    int dev = 0, c0 = 0, c1 = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t pr;
    (void)hipGetDeviceProperties(&pr, dev);
    if (lds_bytes > 0) {
        (void)hipFuncSetAttribute((const void*)k_pgs_env<false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        (void)hipFuncSetAttribute((const void*)k_pgs_env<true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    }
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&c0, k_pgs_env<false>, kEnvBlk, lds_bytes);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&c1, k_pgs_env<true>, kEnvBlk, lds_bytes);
    return std::max(1, std::min(c0, c1)) * pr.multiProcessorCount;
}

int pgs_resident_blocks(int block)
{
    int dev = 0, c0 = 0, c1 = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t pr;
    (void)hipGetDeviceProperties(&pr, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&c0, k_pgs<false>, block, 0);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&c1, k_pgs<true>, block, 0);
    return std::max(1, std::min(c0, c1)) * pr.multiProcessorCount;
}

// The colouring's blocks wait for each other's contacts, so all of them must
// run at once.  The occupancy query reports 7 blocks of k_colour per CU on
// MI355X, but a grid of exactly that many was measured not to be resident at
// once (some blocks start only after others finish: a 578k-contact step
// then gave up with contacts uncoloured), while one block per CU fewer
// always is: keep that slack.
int colour_resident_blocks()
{
    int dev = 0, per_cu = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t pr;
    (void)hipGetDeviceProperties(&pr, dev);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_colour, kBlk, 0);
    return std::max(1, per_cu - 1) * pr.multiProcessorCount;
}

void launch_pgs(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s, int sweeps_cap, int slot)
{
    int sw = sweeps_cap < 0 ? p.max_sweeps : sweeps_cap;
    int nr = std::max(kGroups, z.pgs_mode == kModePerEnv ? z.n_envs : 0);
    hipLaunchKernelGGL(k_pgs_reset, dim3((unsigned)cdiv(nr, 64)), dim3(64), 0, s, b, z.pgs_mode == kModePerEnv ? z.n_envs : 0);
    // counter-ordered solves keep one partial slot per sweep
    int flow = z.flow && sw <= z.part_sweeps ? 1 : 0;
    if (flow && p.n_particles > 0) launch_fill_u32(b.ver, 0u, p.n_particles, s);
    if (z.pgs_mode == kModePerEnv) {
        const dim3 grid((unsigned)z.plan_blocks), blk(kEnvBlk);
        const size_t lds = (size_t)z.lds_cap * 32;
        if (z.plan_blocks > 0 && p.mu_r > 0.f)
            hipLaunchKernelGGL(k_pgs_env<true>, grid, blk, lds, s, b, p, sw, slot, z.lds_cap, flow);
        else if (z.plan_blocks > 0)
            hipLaunchKernelGGL(k_pgs_env<false>, grid, blk, lds, s, b, p, sw, slot, z.lds_cap, flow);
        return;
    }
    if (p.mu_r > 0.f)
        hipLaunchKernelGGL(k_pgs<true>, dim3(z.pgs_grid), dim3(kPgsBlk), 0, s, b, p, z.NB, sw, slot, flow);
    else
        hipLaunchKernelGGL(k_pgs<false>, dim3(z.pgs_grid), dim3(kPgsBlk), 0, s, b, p, z.NB, sw, slot, flow);
}

// ---------------------------------------------------------------------------
// depth below the free surface: per env grid column the max of z + r
// (ordered-integer atomic max, order free), then depth = top - z
// ---------------------------------------------------------------------------
__device__ inline uint32_t f2ord(float f)
{
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float ord2f(uint32_t u) { return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u); }

__device__ inline uint32_t column_of(const EnvDev& E, float4 x)
{
    int c[3];
    cell_of(E, x.x, x.y, x.z, c);
    return (uint32_t)E.col_base + (uint32_t)(c[1] * E.dims[0] + c[0]);
}

__global__ void k_colmax(DevBuffers b, StepParams p)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n_particles) return;
    float4 x = b.xr[s];
    const EnvDev& E = b.envs[env_of(b.pid[s], p.id_cap)];
    atomicMax(&b.colmax[column_of(E, x)], f2ord(x.z + x.w));
}

__global__ void k_depth(DevBuffers b, StepParams p)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n_particles) return;
    float4 x = b.xr[s];
    const EnvDev& E = b.envs[env_of(b.pid[s], p.id_cap)];
    b.pdepth[s] = ord2f(b.colmax[column_of(E, x)]) - x.z;
}

void launch_depth(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s)
{
    launch_fill_u32(b.colmax, 0u, z.NCOL, s);
    if (p.n_particles <= 0) return;
    unsigned g = (unsigned)cdiv(p.n_particles, kBlk);
    hipLaunchKernelGGL(k_colmax, dim3(g), dim3(kBlk), 0, s, b, p);
    hipLaunchKernelGGL(k_depth, dim3(g), dim3(kBlk), 0, s, b, p);
}

// ---------------------------------------------------------------------------
// learned-start trial plumbing: velocity backup/restore, start selection,
// the first-sweep comparison
// ---------------------------------------------------------------------------
__global__ void k_vel_copy(DevBuffers b, int n, int backup)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    if (backup) { vel_at(b.vw2, s) = vel_at(b.vw, s); angv_at(b.vw2, s) = angv_at(b.vw, s); }
    else { vel_at(b.vw, s) = vel_at(b.vw2, s); angv_at(b.vw, s) = angv_at(b.vw2, s); }
}

void launch_vel_copy(const DevBuffers& b, const StepParams& p, bool backup, hipStream_t s)
{
    if (p.n_particles <= 0) return;
    hipLaunchKernelGGL(k_vel_copy, dim3((unsigned)cdiv(p.n_particles, kBlk)), dim3(kBlk), 0, s, b, p.n_particles,
                       backup ? 1 : 0);
}

__global__ void k_select_start(DevBuffers b, int64_t cap, int mode, uint32_t id_cap, float mu_r)
{
    uint32_t nc = n_contacts(b, cap);
    uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    bool learned = mode == 1;
    if (mode == 2) {
        int u = b.envs[env_of(b.pid[__float_as_int(b.r2[c].w)], id_cap)].unit;
        learned = b.ustats[u].use_learned != 0;
    }
    float4 L = learned ? b.lamL[c] : b.lam0[c];
    b.lam[c] = L;
    if (mu_r > 0.f) b.lamr[c] = project_roll(b.lamr0[c], b.r3[c].y * fabsf(L.x));
}

void launch_select_start(const DevBuffers& b, const StepParams& p, const Sizes& z, int mode, hipStream_t s)
{
    hipLaunchKernelGGL(k_select_start, dim3((unsigned)cdiv(z.C, kBlk)), dim3(kBlk), 0, s, b, z.C, mode, p.id_cap, p.mu_r);
}

__global__ void k_choose_start(DevBuffers b, int n_units)
{
    int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_units) return;
    UnitStats& G = b.ustats[u];
    bool finite = G.learn_bad == 0 && isfinite(G.r1_trial[0]);
    bool use = finite && !(G.r1_trial[0] > G.r1_trial[1]);
    G.use_learned = use ? 1u : 0u;
    G.fallback = use ? 0u : 1u;
}

void launch_choose_start(const DevBuffers& b, const StepParams& p, hipStream_t s)
{
    hipLaunchKernelGGL(k_choose_start, dim3((unsigned)cdiv(p.n_units, 64)), dim3(64), 0, s, b, p.n_units);
}

// training samples of the last step in canonical order: the 12 features and
// the final impulses in the contact frame divided by m_eff g dt
__global__ void k_learn_samples(DevBuffers b, int64_t beg, int64_t n, float* feat, float* label)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t pos = b.cpos[beg + k];
    for (int q = 0; q < 12; ++q) feat[k * 12 + q] = b.feat[(size_t)pos * 12 + q];
    float4 L = b.lam[pos], f1 = b.frm1[pos], f2 = b.frm2[pos];
    float ls = f1.w;
    label[k * 3 + 0] = L.x / ls;
    label[k * 3 + 1] = (L.y * f1.x + L.z * f1.y + L.w * f1.z) / ls;
    label[k * 3 + 2] = (L.y * f2.x + L.z * f2.y + L.w * f2.z) / ls;
}

void launch_learn_samples(const DevBuffers& b, int64_t beg, int64_t n, float* feat, float* label, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_learn_samples, dim3((unsigned)cdiv(n, kBlk)), dim3(kBlk), 0, s, b, beg, n, feat, label);
}

// ---------------------------------------------------------------------------
// finish: canonical impulses, body forces (A11), integration (A10), poses,
// zone aggregates (A12), env stats
// ---------------------------------------------------------------------------
__global__ void k_lam_back(DevBuffers b, int64_t cap, float mu_r)
{
    uint32_t nc = n_contacts(b, cap);
    uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    b.lamc[c] = b.cnt->overflow ? make_float4(0.f, 0.f, 0.f, 0.f) : b.lam[b.cpos[c]];
    if (mu_r > 0.f) b.lamrc[c] = b.cnt->overflow ? make_float4(0.f, 0.f, 0.f, 0.f) : b.lamr[b.cpos[c]];
}

__device__ inline double block_sum_d(double v, double* sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += sh[w];
    return s;
}

constexpr int kRedBlk = 128;

// partial force/torque of (body, chunk) over the env's canonical contacts
__global__ __launch_bounds__(kRedBlk) void k_force_part(DevBuffers b, StepParams p, int64_t cap)
{
    __shared__ double sh[kRedBlk / 64];
    int body = blockIdx.x / kForceChunks, ch = blockIdx.x % kForceChunks;
    const BodyDev& B = b.bodies[body];
    const EnvDev& E = b.envs[B.env];
    uint32_t nc = n_contacts(b, cap);
    uint32_t beg = b.id_start[E.id_base], end = b.id_start[E.id_base + p.id_cap];
    if (end > nc) end = nc;
    if (beg > end) beg = end;
    uint32_t len = end - beg;
    uint32_t lo = beg + (uint32_t)(((uint64_t)len * ch) / kForceChunks);
    uint32_t hi = beg + (uint32_t)(((uint64_t)len * (ch + 1)) / kForceChunks);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    if (b.cnt->overflow) hi = lo;
    for (uint32_t c = lo + threadIdx.x; c < hi; c += blockDim.x) {
        int2 pr = b.cpair[c];
        if (pr.x >= 0) continue;
        int sg = -1 - pr.x;
        if (b.shapes[sg].body != body) continue;
        uint32_t pos = b.cpos[c];
        float4 L = b.lam[pos];
        float4 a = b.r0[pos];
        double l2 = b.r1[pos].x;
        float4 x2 = b.xr[pr.y];
        double J[4] = {L.x, L.y, L.z, L.w};
        if (p.v_imp > 0.f) {  // the step's impulses include the impact stage's
            const float4 Li = b.lami[pos];
            J[0] += Li.x; J[1] += Li.y; J[2] += Li.z; J[3] += Li.w;
        }
        double f[3] = {-(J[0] * a.x + J[1]) / p.dt, -(J[0] * a.y + J[2]) / p.dt, -(J[0] * a.z + J[3]) / p.dt};
        double arm[3] = {(double)x2.x - l2 * a.x - B.pos[0], (double)x2.y - l2 * a.y - B.pos[1],
                         (double)x2.z - l2 * a.z - B.pos[2]};
        acc[0] += f[0]; acc[1] += f[1]; acc[2] += f[2];
        acc[3] += arm[1] * f[2] - arm[2] * f[1];
        acc[4] += arm[2] * f[0] - arm[0] * f[2];
        acc[5] += arm[0] * f[1] - arm[1] * f[0];
        if (p.mu_r > 0.f) {  // the rolling couple
            float4 Lr = b.lamr[pos];
            double R[3] = {Lr.x, Lr.y, Lr.z};
            if (p.v_imp > 0.f) {
                const float4 Li = b.lamri[pos];
                R[0] += Li.x; R[1] += Li.y; R[2] += Li.z;
            }
            acc[3] -= R[0] / p.dt;
            acc[4] -= R[1] / p.dt;
            acc[5] -= R[2] / p.dt;
        }
    }
    for (int k = 0; k < 6; ++k) {
        double s = block_sum_d(acc[k], sh);
        if (threadIdx.x == 0) b.force_part[((size_t)body * kForceChunks + ch) * 6 + k] = s;
    }
}

__global__ void k_force_final(DevBuffers b, StepParams p)
{
    int body = blockIdx.x * blockDim.x + threadIdx.x;
    if (body >= p.n_bodies) return;
    for (int k = 0; k < 6; ++k) {
        double s = 0.0;
        for (int ch = 0; ch < kForceChunks; ++ch) s += b.force_part[((size_t)body * kForceChunks + ch) * 6 + k];
        b.body_ft[body * 6 + k] = s;
    }
}

__global__ void k_integrate(DevBuffers b, StepParams p)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n_particles) return;
    if (b.cnt->overflow) return;
    float4 x = b.xr[s];
    float4 v = vel_at(b.vw, s);
    x.x += p.dt * v.x;
    x.y += p.dt * v.y;
    x.z += p.dt * v.z;
    b.xr[s] = x;
}

// poses advance with their constant velocities; world zone planes of the new pose
__global__ void k_bodies_end(DevBuffers b, StepParams p)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p.n_bodies) return;
    if (b.cnt->overflow) return;
    BodyDev& B = b.bodies[t];
    double dt = p.dt;
    for (int k = 0; k < 3; ++k) B.pos[k] += dt * B.linvel[k];
    double q0 = B.quat[0], q1 = B.quat[1], q2 = B.quat[2], q3 = B.quat[3];
    double wx = B.angvel[0], wy = B.angvel[1], wz = B.angvel[2];
    double h = 0.5 * dt;
    double n0 = q0 + h * (-wx * q1 - wy * q2 - wz * q3);
    double n1 = q1 + h * (wx * q0 + wy * q3 - wz * q2);
    double n2 = q2 + h * (-wx * q3 + wy * q0 + wz * q1);
    double n3 = q3 + h * (wx * q2 - wy * q1 + wz * q0);
    double nn = sqrt(n0 * n0 + n1 * n1 + n2 * n2 + n3 * n3);
    B.quat[0] = n0 / nn; B.quat[1] = n1 / nn; B.quat[2] = n2 / nn; B.quat[3] = n3 / nn;
    double R[9];
    quat_to_R(B.quat, R);
    for (int k = 0; k < B.nplanes; ++k) {
        double nw[3];
        for (int r = 0; r < 3; ++r)
            nw[r] = (R[r * 3 + 0] * B.planes[k][0] + R[r * 3 + 1] * B.planes[k][1]) + R[r * 3 + 2] * B.planes[k][2];
        for (int r = 0; r < 3; ++r) B.wplanes[k][r] = nw[r];
        B.wplanes[k][3] = B.planes[k][3] + (nw[0] * B.pos[0] + nw[1] * B.pos[1] + nw[2] * B.pos[2]);
    }
}

// zone moments of one chunk of an env's particles (sorted slots), per zone
// Zone membership of a world point: the union of the body's predicted
// wedges when it has a tool, else its half-spaces (end-of-step pose).
__device__ inline bool in_body_zone(const DevBuffers& b, const BodyDev& B, const double* x)
{
    if (B.tool >= 0) {
        const ToolDev& T = b.tools[B.tool];
        for (int w = 0; w < T.n_wedges; ++w) {
            const WedgeDev& W = b.wedges[(size_t)B.tool * TR_MAX_WEDGES + w];
            bool in = W.n > 0;
            for (int k = 0; k < W.n && in; ++k)
                if (W.planes[k][0] * x[0] + W.planes[k][1] * x[1] + W.planes[k][2] * x[2] - W.planes[k][3] > 0.0)
                    in = false;
            if (in) return true;
        }
        return false;
    }
    bool in = B.nplanes > 0;
    for (int k = 0; k < B.nplanes && in; ++k)
        if (B.wplanes[k][0] * x[0] + B.wplanes[k][1] * x[1] + B.wplanes[k][2] * x[2] - B.wplanes[k][3] > 0.0)
            in = false;
    return in;
}

// height and gradient of a heightfield shape (Eq. surface: bilinear between
// the grid heights, clamped to the border cells)
__device__ inline double hf_height(const ShapeDev& S, const float* hf, double x, double y, double& hx, double& hy)
{
#pragma clang fp contract(off)
    double fx = (x - S.ox) * S.inv_l0;
    double fy = (y - S.oy) * S.inv_l0;
    double fi = floor(fx), fj = floor(fy);
    if (fi < 0.0) fi = 0.0;
    if (fi > (double)(S.nx - 2)) fi = (double)(S.nx - 2);
    if (fj < 0.0) fj = 0.0;
    if (fj > (double)(S.ny - 2)) fj = (double)(S.ny - 2);
    int i = (int)fi, j = (int)fj;
    double t = fx - fi, u = fy - fj;
    const float* h = hf + S.hf_off;
    double h00 = h[j * S.nx + i], h10 = h[j * S.nx + i + 1];
    double h01 = h[(j + 1) * S.nx + i], h11 = h[(j + 1) * S.nx + i + 1];
    hx = ((h10 - h00) * (1.0 - u) + (h11 - h01) * u) * S.inv_l0;
    hy = ((h01 - h00) * (1.0 - t) + (h11 - h10) * t) * S.inv_l0;
    return (h00 * (1.0 - t) + h10 * t) * (1.0 - u) + (h01 * (1.0 - t) + h11 * t) * u;
}

__device__ inline double dot3d(const double* a, const double* c) { return (a[0] * c[0] + a[1] * c[1]) + a[2] * c[2]; }
__device__ inline void cross3d(const double* a, const double* c, double* o)
{
#pragma clang fp contract(off)
    o[0] = a[1] * c[2] - a[2] * c[1];
    o[1] = a[2] * c[0] - a[0] * c[2];
    o[2] = a[0] * c[1] - a[1] * c[0];
}
__device__ inline void unit3d(double* a)
{
    double m = sqrt(dot3d(a, a));
    a[0] /= m; a[1] /= m; a[2] /= m;
}

// Active-zone predictor (Eq. failure_plane): one thread per (tool, lateral
// wedge), at the end-of-step pose.  The wedge lies in front of the separation
// plate through the edge, above the failure plane rising at
// theta = pi/2 - (phi + beta)/2 against the terrain surface, below where that
// plane meets the surface (+ heap), between the slice's lateral planes.
__global__ void k_predict_wedges(DevBuffers b, StepParams p)
{
#pragma clang fp contract(off)
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= p.n_tools * TR_MAX_WEDGES) return;
    const int ti = t / TR_MAX_WEDGES, w = t % TR_MAX_WEDGES;
    const ToolDev& T = b.tools[ti];
    if (w >= T.n_wedges) return;
    WedgeDev& W = b.wedges[t];
    W.n = 0;
    if (T.terrain < 0) return;
    const BodyDev& B = b.bodies[T.body];
    const ShapeDev& S = b.shapes[T.terrain];
    double R[9];
    quat_to_R(B.quat, R);
    double E0[3], E1[3], nc[3], ntc[3];
    for (int k = 0; k < 3; ++k) {
        E0[k] = B.pos[k] + ((R[k * 3 + 0] * T.edge0[0] + R[k * 3 + 1] * T.edge0[1]) + R[k * 3 + 2] * T.edge0[2]);
        E1[k] = B.pos[k] + ((R[k * 3 + 0] * T.edge1[0] + R[k * 3 + 1] * T.edge1[1]) + R[k * 3 + 2] * T.edge1[2]);
        nc[k] = (R[k * 3 + 0] * T.n_c[0] + R[k * 3 + 1] * T.n_c[1]) + R[k * 3 + 2] * T.n_c[2];
        ntc[k] = (R[k * 3 + 0] * T.n_tc[0] + R[k * 3 + 1] * T.n_tc[1]) + R[k * 3 + 2] * T.n_tc[2];
    }
    if (T.v_min > 0.0) {
        double mid[3], arm[3], ve[3];
        for (int k = 0; k < 3; ++k) { mid[k] = 0.5 * (E0[k] + E1[k]); arm[k] = mid[k] - B.pos[k]; }
        cross3d(B.angvel, arm, ve);
        for (int k = 0; k < 3; ++k) ve[k] += B.linvel[k];
        if (!(sqrt(dot3d(ve, ve)) > T.v_min)) return;
    }
    double nf[3], L[3], l[3];
    for (int k = 0; k < 3; ++k) {
        nf[k] = (1.0 - T.fill) * nc[k] + T.fill * ntc[k];
        L[k] = E1[k] - E0[k];
        l[k] = L[k];
    }
    unit3d(nf);
    unit3d(l);
    const double zh[3] = {0.0, 0.0, 1.0};
    double u[3], pl[3];
    cross3d(zh, l, u);
    unit3d(u);
    if (dot3d(u, nf) < 0.0) for (int k = 0; k < 3; ++k) u[k] = -u[k];
    cross3d(l, nf, pl);
    unit3d(pl);
    if (pl[2] < 0.0) for (int k = 0; k < 3; ++k) pl[k] = -pl[k];
    double a[3], c2[3], m[3];
    const double fa = (double)w / T.n_wedges, fb = (double)(w + 1) / T.n_wedges, fm = (w + 0.5) / T.n_wedges;
    for (int k = 0; k < 3; ++k) { a[k] = E0[k] + L[k] * fa; c2[k] = E0[k] + L[k] * fb; m[k] = E0[k] + L[k] * fm; }
    double hx, hy;
    const double h0 = hf_height(S, b.hf_pool, m[0], m[1], hx, hy);
    if (!(m[2] < h0)) return;
    double sv[3] = {u[0], u[1], u[2] + (hx * u[0] + hy * u[1])};
    const double sl = dot3d(sv, l);
    for (int k = 0; k < 3; ++k) sv[k] -= sl * l[k];
    unit3d(sv);
    double ns[3];
    cross3d(l, sv, ns);
    if (ns[2] < 0.0) for (int k = 0; k < 3; ++k) ns[k] = -ns[k];
    const double beta = atan2(dot3d(pl, ns), dot3d(pl, sv));
    const double theta = 0.5 * 3.14159265358979323846 - 0.5 * (T.phi + beta);
    if (!(theta > 0.0 && theta < 0.5 * 3.14159265358979323846)) return;
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = cos(theta) * sv[k] + sin(theta) * ns[k];
    double lo = 0.0, hi = S.l0;
    bool found = false;
    for (int it = 0; it < 40; ++it) {
        const double q[3] = {m[0] + hi * d[0], m[1] + hi * d[1], m[2] + hi * d[2]};
        if (q[2] - hf_height(S, b.hf_pool, q[0], q[1], hx, hy) >= 0.0) { found = true; break; }
        lo = hi;
        hi *= 2.0;
    }
    if (!found) return;
    for (int it = 0; it < 60; ++it) {
        const double md = 0.5 * (lo + hi);
        const double q[3] = {m[0] + md * d[0], m[1] + md * d[1], m[2] + md * d[2]};
        if (q[2] - hf_height(S, b.hf_pool, q[0], q[1], hx, hy) >= 0.0) hi = md;
        else lo = md;
    }
    const double ztop = (m[2] + hi * d[2]) + T.heap;
    double cf[3];
    cross3d(l, d, cf);
    unit3d(cf);
    if (dot3d(cf, pl) > 0.0) for (int k = 0; k < 3; ++k) cf[k] = -cf[k];
    for (int k = 0; k < 3; ++k) {
        W.planes[0][k] = -nf[k];
        W.planes[1][k] = cf[k];
        W.planes[2][k] = zh[k];
        W.planes[3][k] = -l[k];
        W.planes[4][k] = l[k];
    }
    W.planes[0][3] = -dot3d(nf, m);
    W.planes[1][3] = dot3d(cf, m);
    W.planes[2][3] = ztop;
    W.planes[3][3] = -dot3d(l, a);
    W.planes[4][3] = dot3d(l, c2);
    W.n = 5;
}

__global__ __launch_bounds__(kRedBlk) void k_zone_part(DevBuffers b, StepParams p)
{
    __shared__ double sh[kRedBlk / 64];
    int4 ck = b.zone_chunks[blockIdx.x];   // env, begin, end, partial base
    const EnvDev& E = b.envs[ck.x];
    for (int z = 0; z < E.zone_count; ++z) {
        const BodyDev& B = b.bodies[E.zone_body[z]];
        double acc[kZoneMoments];
        for (int k = 0; k < kZoneMoments; ++k) acc[k] = 0.0;
        for (int s = ck.y + threadIdx.x; s < ck.z; s += blockDim.x) {
            float4 xf = b.xr[s];
            double x[3] = {xf.x, xf.y, xf.z};
            // first zone (body order) containing x wins
            int zone = -1;
            for (int zz = 0; zz < E.zone_count && zone < 0; ++zz)
                if (in_body_zone(b, b.bodies[E.zone_body[zz]], x)) zone = zz;
            if (zone != z) continue;
            double r = xf.w;
            double m = (double)b.rho[s] * (4.0 / 3.0) * 3.14159265358979323846 * r * r * r;
            float4 vf = vel_at(b.vw, s), wf = angv_at(b.vw, s);
            double v[3] = {vf.x, vf.y, vf.z};
            double Is = 0.4 * m * r * r;
            acc[0] += m;
            for (int k = 0; k < 3; ++k) { acc[1 + k] += m * x[k]; acc[4 + k] += m * v[k]; }
            acc[7] += m * x[0] * x[0]; acc[8] += m * x[1] * x[1]; acc[9] += m * x[2] * x[2];
            acc[10] += m * x[0] * x[1]; acc[11] += m * x[0] * x[2]; acc[12] += m * x[1] * x[2];
            acc[13] += m * (x[1] * v[2] - x[2] * v[1]);
            acc[14] += m * (x[2] * v[0] - x[0] * v[2]);
            acc[15] += m * (x[0] * v[1] - x[1] * v[0]);
            acc[16] += Is;
            acc[17] += Is * wf.x; acc[18] += Is * wf.y; acc[19] += Is * wf.z;
        }
        (void)B;
        for (int k = 0; k < kZoneMoments; ++k) {
            double s = block_sum_d(acc[k], sh);
            if (threadIdx.x == 0) b.zone_part[((size_t)ck.w + z) * kZoneMoments + k] = s;
        }
    }
}

// per zone: sum the chunk partials in order, then the aggregate body
__global__ void k_zone_final(DevBuffers b, StepParams p, int n_chunks)
{
    int zs = blockIdx.x * blockDim.x + threadIdx.x;
    if (zs >= p.n_zones) return;
    // locate env and zone index of this global zone
    int env = -1, zi = -1;
    for (int e = 0; e < p.n_envs && env < 0; ++e)
        for (int z = 0; z < b.envs[e].zone_count; ++z)
            if (b.envs[e].zone_slot[z] == zs) { env = e; zi = z; }
    if (env < 0) return;
    double S[kZoneMoments];
    for (int k = 0; k < kZoneMoments; ++k) S[k] = 0.0;
    for (int c = 0; c < n_chunks; ++c) {
        int4 ck = b.zone_chunks[c];
        if (ck.x != env) continue;
        for (int k = 0; k < kZoneMoments; ++k) S[k] += b.zone_part[((size_t)ck.w + zi) * kZoneMoments + k];
    }
    for (int k = 0; k < kZoneMoments; ++k) b.zone_mom[(size_t)zs * kZoneMoments + k] = S[k];
    tr_aggregate A;
    A.zone = b.bodies[b.envs[env].zone_body[zi]].user_id;
    A.pad = 0;
    double M = S[0];
    A.M = M;
    A.n_particles = 0;
    for (int k = 0; k < 3; ++k) { A.x[k] = 0.0; A.v[k] = 0.0; A.w[k] = 0.0; }
    for (int k = 0; k < 6; ++k) A.I[k] = 0.0;
    if (M > 0.0) {
        double x[3] = {S[1] / M, S[2] / M, S[3] / M};
        double v[3] = {S[4] / M, S[5] / M, S[6] / M};
        // second moments about x_A
        double Cxx = S[7] - M * x[0] * x[0], Cyy = S[8] - M * x[1] * x[1], Czz = S[9] - M * x[2] * x[2];
        double Cxy = S[10] - M * x[0] * x[1], Cxz = S[11] - M * x[0] * x[2], Cyz = S[12] - M * x[1] * x[2];
        double tr = Cxx + Cyy + Czz;
        double I[3][3] = {{S[16] + tr - Cxx, -Cxy, -Cxz}, {-Cxy, S[16] + tr - Cyy, -Cyz}, {-Cxz, -Cyz, S[16] + tr - Czz}};
        // angular momentum about x_A: sum m x*v - x_A * sum m v + spins
        double L[3] = {S[13] - (x[1] * S[6] - x[2] * S[5]) + S[17], S[14] - (x[2] * S[4] - x[0] * S[6]) + S[18],
                       S[15] - (x[0] * S[5] - x[1] * S[4]) + S[19]};
        double det = I[0][0] * (I[1][1] * I[2][2] - I[1][2] * I[2][1]) - I[0][1] * (I[1][0] * I[2][2] - I[1][2] * I[2][0]) +
                     I[0][2] * (I[1][0] * I[2][1] - I[1][1] * I[2][0]);
        // inverse by cofactors (I symmetric)
        double inv[3][3];
        inv[0][0] = (I[1][1] * I[2][2] - I[1][2] * I[2][1]);
        inv[0][1] = -(I[0][1] * I[2][2] - I[0][2] * I[2][1]);
        inv[0][2] = (I[0][1] * I[1][2] - I[0][2] * I[1][1]);
        inv[1][0] = -(I[1][0] * I[2][2] - I[1][2] * I[2][0]);
        inv[1][1] = (I[0][0] * I[2][2] - I[0][2] * I[2][0]);
        inv[1][2] = -(I[0][0] * I[1][2] - I[0][2] * I[1][0]);
        inv[2][0] = (I[1][0] * I[2][1] - I[1][1] * I[2][0]);
        inv[2][1] = -(I[0][0] * I[2][1] - I[0][1] * I[2][0]);
        inv[2][2] = (I[0][0] * I[1][1] - I[0][1] * I[1][0]);
        for (int r = 0; r < 3; ++r) {
            A.x[r] = x[r];
            A.v[r] = v[r];
            A.w[r] = det != 0.0 ? (inv[r][0] * L[0] + inv[r][1] * L[1] + inv[r][2] * L[2]) / det : 0.0;
        }
        A.I[0] = I[0][0]; A.I[1] = I[1][1]; A.I[2] = I[2][2];
        A.I[3] = I[0][1]; A.I[4] = I[0][2]; A.I[5] = I[1][2];
    }
    b.aggs[zs] = A;
}

// zone particle counts (integers, order free)
__global__ void k_zone_count(DevBuffers b, StepParams p)
{
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= p.n_particles) return;
    const EnvDev& E = b.envs[env_of(b.pid[s], p.id_cap)];
    float4 xf = b.xr[s];
    double x[3] = {xf.x, xf.y, xf.z};
    for (int zz = 0; zz < E.zone_count; ++zz) {
        if (in_body_zone(b, b.bodies[E.zone_body[zz]], x)) {
            atomicAdd((unsigned long long*)&b.aggs[E.zone_slot[zz]].n_particles, 1ull);
            break;
        }
    }
}

__global__ void k_env_stats(DevBuffers b, StepParams p)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= p.n_envs) return;
    int64_t base = (int64_t)e * p.id_cap;
    b.env_stats[e].contacts = (int64_t)b.id_start[base + p.id_cap] - (int64_t)b.id_start[base];
}

void launch_finish(const DevBuffers& b, const StepParams& p, const Sizes& z, hipStream_t s)
{
    hipLaunchKernelGGL(k_lam_back, dim3((unsigned)cdiv(z.C, kBlk)), dim3(kBlk), 0, s, b, z.C, p.mu_r);
    if (p.n_bodies > 0) {
        hipLaunchKernelGGL(k_force_part, dim3(p.n_bodies * kForceChunks), dim3(kRedBlk), 0, s, b, p, z.C);
        hipLaunchKernelGGL(k_force_final, dim3((unsigned)cdiv(p.n_bodies, kBlk)), dim3(kBlk), 0, s, b, p);
    }
    if (p.n_particles > 0)
        hipLaunchKernelGGL(k_integrate, dim3((unsigned)cdiv(p.n_particles, kBlk)), dim3(kBlk), 0, s, b, p);
    if (p.n_bodies > 0)
        hipLaunchKernelGGL(k_bodies_end, dim3((unsigned)cdiv(p.n_bodies, kBlk)), dim3(kBlk), 0, s, b, p);
    if (p.n_tools > 0)  // the tools' zones at the end-of-step poses
        hipLaunchKernelGGL(k_predict_wedges, dim3((unsigned)cdiv(p.n_tools * TR_MAX_WEDGES, 64)), dim3(64), 0, s, b, p);
    if (p.n_zones > 0 && z.n_zone_chunks > 0) {
        hipLaunchKernelGGL(k_zone_part, dim3(z.n_zone_chunks), dim3(kRedBlk), 0, s, b, p);
        hipLaunchKernelGGL(k_zone_final, dim3((unsigned)cdiv(p.n_zones, 64)), dim3(64), 0, s, b, p, z.n_zone_chunks);
        hipLaunchKernelGGL(k_zone_count, dim3((unsigned)cdiv(std::max(p.n_particles, 1), kBlk)), dim3(kBlk), 0, s,
                           b, p);
    }
    hipLaunchKernelGGL(k_env_stats, dim3((unsigned)cdiv(std::max(p.n_envs, 1), 64)), dim3(64), 0, s, b, p);
}

// ---------------------------------------------------------------------------
// host <-> device particle exchange in id order
// ---------------------------------------------------------------------------
__global__ void k_gather_by_id(DevBuffers b, int id_base, int n, float4* xo, float4* vo, float4* wo)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int s = b.id2slot[id_base + k];
    xo[k] = b.xr[s];
    vo[k] = vel_at(b.vw, s);
    wo[k] = angv_at(b.vw, s);
}

void launch_gather_by_id(const DevBuffers& b, int id_base, int n, float4* xo, float4* vo, float4* wo, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_by_id, dim3((unsigned)cdiv(n, kBlk)), dim3(kBlk), 0, s, b, id_base, n, xo, vo, wo);
}

__global__ void k_scatter_by_id(DevBuffers b, int id_base, int n, const float4* xi, const float4* vi,
                                const float4* wi, int mask)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int s = b.id2slot[id_base + k];
    if (mask & 1) { float4 o = b.xr[s]; float4 v = xi[k]; b.xr[s] = make_float4(v.x, v.y, v.z, o.w); }
    if (mask & 2) { float4 o = vel_at(b.vw, s); float4 v = vi[k]; vel_at(b.vw, s) = make_float4(v.x, v.y, v.z, o.w); }
    if (mask & 4) { float4 o = angv_at(b.vw, s); float4 v = wi[k]; angv_at(b.vw, s) = make_float4(v.x, v.y, v.z, o.w); }
}

void launch_scatter_by_id(const DevBuffers& b, int id_base, int n, const float4* xi, const float4* vi,
                          const float4* wi, int mask, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scatter_by_id, dim3((unsigned)cdiv(n, kBlk)), dim3(kBlk), 0, s, b, id_base, n, xi, vi, wi,
                       mask);
}

}  // namespace trk
