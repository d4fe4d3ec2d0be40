// terrain_capi.hip -- the C-ABI of libterrain.so (see include/terrain.h).
//
// Host side of the step: validates and copies inputs, keeps the per-env
// tables (cell grids, bodies, shapes, zones), owns every device buffer and
// enqueues the kernel families of terrain_kernels.hip on the scene's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "terrain.h"
#include "terrain_internal.h"

using namespace trk;

namespace {

struct EnvHost {
    int64_t n = 0;
    double rmax = 0.0;
    std::vector<tr_body_desc> bodies;             // shapes pointer unused (see shapes)
    std::vector<std::vector<tr_shape_desc>> shapes;
    std::vector<std::vector<std::vector<float>>> heights;
    std::vector<std::pair<int32_t, tr_tool_desc>> tools;  // zone predictor tools by body id
};

}  // namespace

struct tr_scene {
    tr_scene_desc desc{};
    std::vector<double> bounds;
    hipStream_t stream = nullptr;
    std::string err;
    std::vector<EnvHost> envs;
    DevBuffers b{};
    Sizes z{};
    StepParams p{};
    int64_t n_total = 0;
    bool tables_dirty = true;
    bool have_prev = false;
    bool stepped = false;
    bool slots_env_major = true;     // every env's spheres hold the slots [slot_begin, slot_begin + n)
    bool last_replay = false;         // the last step was a graph replay: only its total is timed
    std::vector<std::pair<void*, size_t>> allocs;
    int64_t cells_alloc = 0;
    int64_t zone_chunk_alloc = 0;
    int64_t hf_alloc = 0;
    int bodies_alloc = 0, shapes_alloc = 0, zones_alloc = 0, tools_alloc = 0;
    std::vector<ToolDev> tool_host;  // last uploaded tool table
    std::vector<BodyDev> body_host;   // last uploaded body table (poses refreshed on download)
    std::vector<ShapeDev> shape_host; // last uploaded shape table
    WedgeDev* conv_wedges = nullptr;  // caller wedges of the conversion entry points (device)
    MacroZone* macro_zone = nullptr;       // macroscale step: per-zone reductions (device)
    tr_macro_result* macro_out = nullptr;  // and its results (device)
    double* conv_total = nullptr;     // one device double: the converted mass
    double* adv_bmax = nullptr;       // per-block Courant maxima of the advection
    int64_t adv_cap = 0;
    int* settle_list = nullptr;       // ids of settle_particles (cap_particles)
    FormEntry* form_list = nullptr;   // candidates of form_particles
    int64_t form_cap = 0;
    std::vector<EnvDev> env_host;
    std::vector<std::vector<int>> zone_slots;  // per env: global zone index of each zone body
    hipEvent_t ev[5] = {};
    bool events = false;
    float* staging = nullptr;         // 12 floats per particle (device), id-order exchange
    int64_t cols_alloc = 0;
    bool mlp_loaded = false;
    bool mlp_bf16 = true;
    bool capture = false;             // set_learn_capture: every step writes the learned-start features
    bool features_last = false;       // the last step wrote them
    tr_solver_config cfg{};           // PGS schedule
    int64_t plan_alloc = 0;           // plan tasks allocated
    int64_t plan_idx_alloc = 0;       // plan block offsets allocated
    int64_t part_alloc = 0;           // block partials allocated (doubles)
    int max_lds_particles = 0;        // bodies one per-env block can stage in LDS
    // step graphs: a step swaps the sorted-particle and contact-cache buffers,
    // so the launch sequence repeats every two steps; gexec[q] replays the
    // step taken when (steps since capture) % 2 == q
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipStream_t cap_stream = nullptr;
    bool graphs = false;
    bool use_graphs = true;
    int parity = 0;
};

namespace {

int fail(tr_scene* s, int code, const std::string& msg)
{
    if (s) s->err = msg;
    return code;
}

int hip_fail(tr_scene* s, hipError_t e, const char* what)
{
    return fail(s, TR_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_CHECK(s, call)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return hip_fail((s), e_, #call); \
    } while (0)

void* dalloc(tr_scene* s, size_t bytes)
{
    bytes = std::max<size_t>(bytes, 256);
    void* p = nullptr;
    if (s->desc.alloc_fn) {
        p = s->desc.alloc_fn(s->desc.alloc_ctx, bytes, s->desc.stream);
    } else {
        if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
    }
    if (p) s->allocs.push_back({p, bytes});
    return p;
}

void dfree(tr_scene* s, void* p)
{
    if (!p) return;
    for (size_t i = 0; i < s->allocs.size(); ++i) {
        if (s->allocs[i].first == p) {
            if (s->desc.free_fn) s->desc.free_fn(s->desc.alloc_ctx, p, s->desc.stream);
            else (void)hipFree(p);
            s->allocs.erase(s->allocs.begin() + (long)i);
            return;
        }
    }
}

template <class T>
bool alloc_n(tr_scene* s, T*& p, int64_t n)
{
    p = (T*)dalloc(s, sizeof(T) * (size_t)std::max<int64_t>(n, 1));
    return p != nullptr;
}

bool finite3(const double* a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

int ceil_log2(int v)
{
    int b = 0;
    while ((1 << b) < v) ++b;
    return b;
}

void invalidate_graphs(tr_scene* s)
{
    for (int q = 0; q < 2; ++q)
        if (s->gexec[q]) {
            (void)hipGraphExecDestroy(s->gexec[q]);
            s->gexec[q] = nullptr;
        }
    s->graphs = false;
}

// The automatic per-env plan, from a cost model measured on MI355X (the
// 256-bed batch, 100 sweeps, with a timing build that clocks every block's
// tasks; units of microseconds): a block's share of a multi-block cluster
// costs about 1800 (the colour phases' barriers) plus 1.77 per sphere of the
// share, a set of envs solved from LDS by one block 1300 plus 0.6 per sphere,
// and a sphere that a single block keeps in global memory about 2.0 (2.5
// here: those solves vary most).  Envs that fit LDS are packed into sets
// (first fit, largest first); envs up to Ns spheres are solved alone by one
// block with their first slots in LDS; larger ones by clusters of
// ceil(1.77 n / (M - 1800)) blocks of one XCD lane.  Ns and the target M are
// searched for the smallest predicted makespan (jobs placed largest first on
// the least loaded block).  tasks gets each block's cluster share
// (env, rank, K, first block) and then its sets as (env, set number, 1, 0);
// false when no candidate fits the blocks.
bool plan_auto(const tr_scene* s, const std::vector<int>& order, int B, int lds_cap,
               std::vector<std::vector<int4>>& best_tasks)
{
    constexpr double kAc = 1800.0, kWc = 1.77, kWs = 0.6, kWset = 1300.0, kWg = 2.5;
    const int G = kGroups, PL = B / G, waves = kEnvBlk / 64;
    std::vector<std::vector<int>> sets;
    std::vector<double> fill;
    double work0 = 0.0;
    for (int e : order) {
        const double n = (double)s->envs[e].n;
        if (n > lds_cap) {
            work0 += kWc * n;
            continue;
        }
        work0 += kWs * n;
        size_t k = 0;
        while (k < sets.size() && (fill[k] + n > lds_cap || (int)sets[k].size() >= waves)) ++k;
        if (k == sets.size()) {
            sets.emplace_back();
            fill.push_back(0.0);
        }
        sets[k].push_back(e);
        fill[k] += n;
    }
    work0 += kWset * (double)sets.size();
    double best = 1e300;
    for (double fs : {1.0, 1.1, 1.2, 1.3, 1.4, 1.5, 1.6}) {
        const double Ns = fs * lds_cap;
        for (int m = 0; m <= 36; ++m) {
            const double M = work0 / B * (0.7 + 0.025 * m);
            std::vector<double> load(B, 0.0);
            std::vector<int> lane_next(G, 0);
            std::vector<std::vector<int4>> tasks(B);
            std::vector<std::pair<double, int>> jobs;  // (cost, env) or (cost, -1 - set)
            bool ok = true;
            for (int e : order) {
                const double n = (double)s->envs[e].n;
                if (n <= lds_cap) continue;
                if (n <= Ns) {
                    jobs.push_back({kWs * lds_cap + kWg * (n - lds_cap) + kWset, e});
                    continue;
                }
                if (M <= kAc) {
                    ok = false;
                    break;
                }
                const int K = std::max(2, (int)std::ceil(kWc * n / (M - kAc)));
                int lane = 0;
                for (int x = 1; x < G; ++x)
                    if (lane_next[x] < lane_next[lane]) lane = x;
                if (K > PL - lane_next[lane]) {
                    ok = false;
                    break;
                }
                const int first = lane + G * lane_next[lane];
                for (int r = 0; r < K; ++r) {
                    tasks[first + G * r].push_back(make_int4(e, r, K, first));
                    load[first + G * r] += kAc + kWc * n / K;
                }
                lane_next[lane] += K;
            }
            if (!ok) continue;
            for (size_t k = 0; k < sets.size(); ++k) jobs.push_back({kWs * fill[k] + kWset, -1 - (int)k});
            std::stable_sort(jobs.begin(), jobs.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& c) {
                return a.first > c.first;
            });
            int setno = 0;
            for (const auto& j : jobs) {
                int blk = 0;
                for (int i = 1; i < B; ++i)
                    if (load[i] < load[blk]) blk = i;
                load[blk] += j.first;
                if (j.second >= 0) tasks[blk].push_back(make_int4(j.second, setno, 1, 0));
                else
                    for (int e : sets[-1 - j.second]) tasks[blk].push_back(make_int4(e, setno, 1, 0));
                ++setno;
            }
            const double mk = *std::max_element(load.begin(), load.end());
            if (mk < best) {
                best = mk;
                best_tasks = tasks;
            }
        }
    }
    return best < 1e300;
}

// PGS schedule: the solve unit of every env and, in per-env mode, the plan of
// the resident blocks.  Automatic (cluster_particles 0): plan_auto.  With a
// given T: envs larger than T spheres per block get a cluster of ceil(n / T)
// blocks in one XCD lane (indices congruent mod 8, so they share an XCD); the
// others are packed into sets that one block solves at once, each env on its
// own waves.
int rebuild_plan(tr_scene* s)
{
    invalidate_graphs(s);
    const int E = s->desc.n_envs;
    hipStream_t st = s->stream;
    std::vector<int4> plan;
    std::vector<uint32_t> plan_idx;
    int lds_cap = 0;
    int blocks = 0;
    if (s->cfg.mode == TR_PGS_PER_ENV) {
        lds_cap = std::max(0, std::min(s->cfg.lds_particles, s->max_lds_particles));
        // every block is resident (clusters wait for each other); a whole number per XCD
        int B = std::max(kGroups, pgs_env_resident_blocks(lds_cap * 32));
        B -= B % kGroups;
        const int per_lane = B / kGroups;
        const int waves = kEnvBlk / 64;
        double total = 0.0;
        for (int e = 0; e < E; ++e) total += (double)s->envs[e].n;
        std::vector<int> order;
        for (int e = 0; e < E; ++e)
            if (s->envs[e].n > 0) order.push_back(e);
        std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return s->envs[a].n > s->envs[c].n; });
        std::vector<std::vector<int4>> tasks(B);
        // a set of envs solved at once by block blk: waves in proportion to
        // the envs' spheres (at least one each), LDS slots in order while they
        // last (an env that does not fit keeps its first slots there)
        auto place_set = [&](int blk, const std::vector<int>& st) {
            std::vector<int> w(st.size(), 1);
            int left = waves - (int)st.size();
            while (left > 0) {
                size_t best = 0;
                double bv = -1.0;
                for (size_t i = 0; i < st.size(); ++i) {
                    double v = (double)s->envs[st[i]].n / w[i];
                    if (v > bv) { bv = v; best = i; }
                }
                ++w[best];
                --left;
            }
            int wb = 0, off = 0;
            for (size_t i = 0; i < st.size(); ++i) {
                const int n = (int)s->envs[st[i]].n;
                const int lo = off < lds_cap ? off : -1;
                if (lo >= 0) off += std::min(n, lds_cap - off);
                tasks[blk].push_back(make_int4(st[i], wb | ((wb + w[i]) << 8), 1, lo));
                wb += w[i];
            }
        };
        if (s->cfg.cluster_particles == 0 && lds_cap > 0 && plan_auto(s, order, B, lds_cap, tasks)) {
            for (int blk = 0; blk < B; ++blk) {
                // plan_auto lists each block's sets as (env, set number) pairs after its cluster share
                std::vector<int4> mine;
                std::vector<std::vector<int>> sets_b;
                int cur_set = -1;
                for (const int4& t : tasks[blk]) {
                    if (t.z >= 2) { mine.push_back(t); continue; }
                    if (t.y != cur_set) { sets_b.emplace_back(); cur_set = t.y; }
                    sets_b.back().push_back(t.x);
                }
                tasks[blk] = mine;
                for (const auto& st : sets_b) place_set(blk, st);
            }
        } else {
            // T: spheres per block (given, or the mean load).  Envs above T get
            // ceil(n / T) blocks of one XCD lane; the rest are packed (first fit,
            // largest first) into sets of at most T spheres and 16 envs, each solved
            // by one block at once, placed largest first on the least loaded block (a
            // cluster share counts twice its spheres).
            const double T = s->cfg.cluster_particles > 0 ? (double)s->cfg.cluster_particles
                                                           : std::max(total / B, 4096.0);
            // single-block solves only: an env too large for LDS takes a block of
            // its own (measured on MI355X, a multi-block share pays about 12 us of
            // cross-block barrier per colour, where one block of 1,024 threads
            // solving the env alone meets at workgroup barriers)
            const bool solo = s->cfg.cluster_particles == TR_CLUSTER_NONE;
            const double set_cap = solo ? (double)std::max(lds_cap, 1) : T;
            std::vector<double> load(B, 0.0);
            std::vector<int> lane_next(kGroups, 0);
            std::vector<std::vector<int>> sets;
            std::vector<double> fill;
            for (int e : order) {
                const double n = (double)s->envs[e].n;
                int K = solo ? 1 : (int)std::min<double>(std::ceil(n / T), (double)per_lane);
                int lane = 0;
                for (int x = 1; x < kGroups; ++x)
                    if (lane_next[x] < lane_next[lane]) lane = x;
                K = std::min(K, per_lane - lane_next[lane]);
                if (K >= 2) {
                    const int first = lane + kGroups * lane_next[lane];
                    for (int r = 0; r < K; ++r) {
                        tasks[first + kGroups * r].push_back(make_int4(e, r, K, first));
                        load[first + kGroups * r] += 2.0 * n / K;
                    }
                    lane_next[lane] += K;
                    continue;
                }
                size_t k = 0;
                while (k < sets.size() && (fill[k] + n > set_cap || (int)sets[k].size() >= waves)) ++k;
                if (k == sets.size()) {
                    sets.emplace_back();
                    fill.push_back(0.0);
                }
                sets[k].push_back(e);
                fill[k] += n;
            }
            std::vector<size_t> sorder(sets.size());
            for (size_t k = 0; k < sets.size(); ++k) sorder[k] = k;
            std::stable_sort(sorder.begin(), sorder.end(), [&](size_t a, size_t c) { return fill[a] > fill[c]; });
            for (size_t k : sorder) {
                int blk = 0;
                for (int i = 1; i < B; ++i)
                    if (load[i] < load[blk]) blk = i;
                load[blk] += fill[k];
                place_set(blk, sets[k]);
            }
        }
        plan_idx.assign(B + 1, 0);
        for (int blk = 0; blk < B; ++blk) {
            plan_idx[blk] = (uint32_t)plan.size();
            plan.insert(plan.end(), tasks[blk].begin(), tasks[blk].end());
        }
        plan_idx[B] = (uint32_t)plan.size();
        blocks = B;
        for (int e = 0; e < E; ++e) s->env_host[e].unit = e;
    } else {
        for (int e = 0; e < E; ++e) s->env_host[e].unit = s->env_host[e].group;
    }
    if ((int64_t)plan.size() > s->plan_alloc) {
        dfree(s, s->b.plan);
        if (!alloc_n(s, s->b.plan, (int64_t)plan.size())) return fail(s, TR_E_NOMEM, "PGS plan");
        s->plan_alloc = (int64_t)plan.size();
    }
    if ((int64_t)plan_idx.size() > s->plan_idx_alloc) {
        dfree(s, s->b.plan_idx);
        if (!alloc_n(s, s->b.plan_idx, (int64_t)plan_idx.size())) return fail(s, TR_E_NOMEM, "PGS plan");
        s->plan_idx_alloc = (int64_t)plan_idx.size();
    }
    // block partials: two sweeps (barrier order) or one slot per sweep (counter order)
    s->z.part_sweeps = std::min(std::max(s->desc.max_sweeps, 2), 8192);
    s->z.flow = s->cfg.dataflow ? 1 : 0;
    int64_t parts = 2 * std::max<int64_t>(s->z.pgs_grid, blocks) * s->z.part_sweeps;
    if (parts > s->part_alloc) {
        dfree(s, s->b.block_part);
        if (!alloc_n(s, s->b.block_part, parts)) return fail(s, TR_E_NOMEM, "PGS partials");
        s->part_alloc = parts;
    }
    if (!plan.empty()) HIP_CHECK(s, hipMemcpyAsync(s->b.plan, plan.data(), sizeof(int4) * plan.size(), hipMemcpyHostToDevice, st));
    if (!plan_idx.empty())
        HIP_CHECK(s, hipMemcpyAsync(s->b.plan_idx, plan_idx.data(), sizeof(uint32_t) * plan_idx.size(), hipMemcpyHostToDevice, st));
    s->z.pgs_mode = s->cfg.mode;
    s->p.spread = s->cfg.mode == TR_PGS_SPREAD ? 1 : 0;
    s->z.plan_blocks = blocks;
    s->z.lds_cap = lds_cap;
    HIP_CHECK(s, hipMemcpyAsync(s->b.envs, s->env_host.data(), sizeof(EnvDev) * E, hipMemcpyHostToDevice, st));
    HIP_CHECK(s, hipStreamSynchronize(st));  // the host plan dies here
    return TR_OK;
}

// Rebuild the per-env tables (grids, bodies, shapes, zones, chunk list) and
// upload them; device poses are kept by downloading them first.
int rebuild_tables(tr_scene* s)
{
    const int E = s->desc.n_envs;
    const bool cohesive = s->desc.material.c_p > 0.0;
    std::vector<EnvDev> ed(E);
    std::vector<BodyDev> bd;
    std::vector<ShapeDev> sd;
    std::vector<float> pool;
    std::vector<int4> chunks;
    std::vector<ToolDev> td;
    int64_t NC = 0;
    int64_t NCOL = 0;
    int n_zones = 0;
    int64_t slot = 0;
    s->zone_slots.assign(E, {});
    // PGS groups: one env per group when there are at most kGroups envs,
    // else largest-first onto the least loaded group
    std::vector<int> grp(E, 0);
    if (E <= kGroups) {
        for (int e = 0; e < E; ++e) grp[e] = e;
    } else {
        std::vector<int> order(E);
        for (int e = 0; e < E; ++e) order[e] = e;
        std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return s->envs[a].n > s->envs[c].n; });
        int64_t load[kGroups] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int e : order) {
            int best = 0;
            for (int g = 1; g < kGroups; ++g)
                if (load[g] < load[best]) best = g;
            grp[e] = best;
            load[best] += std::max<int64_t>(s->envs[e].n, 1);
        }
    }
    for (int e = 0; e < E; ++e) {
        EnvHost& H = s->envs[e];
        EnvDev& D = ed[e];
        const double* bo = &s->bounds[6 * e];
        double rmax = H.rmax > 0.0 ? H.rmax : 0.05;
        double h = 2.0 * rmax * (1.0 + (cohesive ? s->desc.material.kappa_c : 0.0)) * 1.001;
        for (int k = 0; k < 3; ++k) {
            double ext = bo[3 + k] - bo[k];
            int dims = std::max(1, (int)std::ceil(ext / h));
            if (dims > 1024) return fail(s, TR_E_CAPACITY, "env grid exceeds 1024 cells along an axis");
            D.lo[k] = (float)bo[k];
            D.dims[k] = dims;
            D.bits[k] = ceil_log2(dims);
        }
        D.inv_h = (float)(1.0 / h);
        D.cell_base = (uint32_t)NC;
        D.col_base = (int)NCOL;
        D.group = grp[e];
        NCOL += (int64_t)D.dims[0] * D.dims[1];
        NC += (int64_t)1 << (D.bits[0] + D.bits[1] + D.bits[2]);
        if (NC >= ((int64_t)1 << 31)) return fail(s, TR_E_CAPACITY, "too many cells");
        D.id_base = (int)(e * s->desc.cap_particles);
        D.n = (int)H.n;
        D.slot_begin = (int)slot;
        D.body_begin = (int)bd.size();
        D.shape_begin = (int)sd.size();
        D.zone_count = 0;
        for (size_t bi = 0; bi < H.bodies.size(); ++bi) {
            const tr_body_desc& B = H.bodies[bi];
            BodyDev X;
            memset(&X, 0, sizeof(X));
            int gi = (int)bd.size();
            for (int k = 0; k < 3; ++k) { X.pos[k] = B.pos[k]; X.linvel[k] = B.linvel[k]; X.angvel[k] = B.angvel[k]; }
            for (int k = 0; k < 4; ++k) X.quat[k] = B.quat[k];
            X.env = e;
            X.user_id = B.id;
            X.nplanes = B.n_halfspaces;
            for (int k = 0; k < B.n_halfspaces; ++k)
                for (int j = 0; j < 4; ++j) X.planes[k][j] = B.planes[k][j];
            X.tool = -1;
            for (const auto& tl : H.tools)
                if (tl.first == B.id) {
                    const tr_tool_desc& T = tl.second;
                    ToolDev Y;
                    memset(&Y, 0, sizeof(Y));
                    Y.body = gi;
                    Y.env = e;
                    Y.n_wedges = T.n_wedges;
                    Y.terrain = -1;  // set once the env's shapes are known
                    for (int k = 0; k < 3; ++k) {
                        Y.edge0[k] = T.edge0[k]; Y.edge1[k] = T.edge1[k];
                        Y.n_c[k] = T.n_c[k]; Y.n_tc[k] = T.n_tc[k];
                    }
                    Y.fill = T.fill; Y.phi = T.phi; Y.heap = T.heap; Y.v_min = T.v_min;
                    X.tool = (int)td.size();
                    td.push_back(Y);
                }
            if (B.n_halfspaces > 0 || X.tool >= 0) {
                if (D.zone_count >= kMaxZonesPerEnv) return fail(s, TR_E_CAPACITY, "more than 4 zones in an env");
                D.zone_body[D.zone_count] = gi;
                D.zone_slot[D.zone_count] = n_zones;
                s->zone_slots[e].push_back(n_zones);
                ++D.zone_count;
                ++n_zones;
            }
            bd.push_back(X);
            for (size_t si = 0; si < H.shapes[bi].size(); ++si) {
                const tr_shape_desc& S = H.shapes[bi][si];
                ShapeDev Y;
                memset(&Y, 0, sizeof(Y));
                Y.type = S.type;
                Y.body = gi;
                Y.env = e;
                for (int k = 0; k < 3; ++k) { Y.n[k] = S.normal[k]; Y.half[k] = S.half[k]; Y.off[k] = S.center[k]; }
                Y.d = S.offset;
                if (S.type == TR_HEIGHTFIELD) {
                    Y.nx = S.nx; Y.ny = S.ny;
                    Y.ox = S.origin[0]; Y.oy = S.origin[1];
                    Y.l0 = S.l0;
                    Y.inv_l0 = 1.0 / S.l0;
                    Y.hf_off = (int)pool.size();
                    const std::vector<float>& hh = H.heights[bi][si];
                    pool.insert(pool.end(), hh.begin(), hh.end());
                }
                sd.push_back(Y);
            }
        }
        D.body_end = (int)bd.size();
        D.shape_end = (int)sd.size();
        // the terrain of the env's tools: its first heightfield
        int terrain = -1;
        for (int k = D.shape_begin; k < D.shape_end && terrain < 0; ++k)
            if (sd[k].type == TR_HEIGHTFIELD) terrain = k;
        for (ToolDev& Y : td)
            if (Y.env == e) Y.terrain = terrain;
        for (int64_t b0 = slot; b0 < slot + H.n; b0 += kZoneChunk) {
            int64_t b1 = std::min<int64_t>(b0 + kZoneChunk, slot + H.n);
            chunks.push_back(make_int4(e, (int)b0, (int)b1, (int)(chunks.size() * kMaxZonesPerEnv)));
        }
        slot += H.n;
    }
    hipStream_t st = s->stream;
    // (re)allocate tables whose size depends on the scene content
    if (NC + 1 > s->cells_alloc) {
        dfree(s, s->b.cell_count); dfree(s, s->b.cell_start); dfree(s, s->b.cell_fill);
        dfree(s, s->b.scan_tmp);
        if (!alloc_n(s, s->b.cell_count, NC) || !alloc_n(s, s->b.cell_start, NC + 1) || !alloc_n(s, s->b.cell_fill, NC))
            return fail(s, TR_E_NOMEM, "cell arrays");
        int64_t words = std::max({scan_tmp_words(NC), scan_tmp_words(s->z.NID), scan_tmp_words(s->z.P),
                                  scan_tmp_words((int64_t)kBuckets * s->z.NB)});
        if (!alloc_n(s, s->b.scan_tmp, words)) return fail(s, TR_E_NOMEM, "scan scratch");
        s->cells_alloc = NC + 1;
    }
    if ((int)bd.size() > s->bodies_alloc || (int)sd.size() > s->shapes_alloc || n_zones > s->zones_alloc) {
        dfree(s, s->b.bodies); dfree(s, s->b.shapes); dfree(s, s->b.force_part); dfree(s, s->b.body_ft);
        dfree(s, s->b.zone_mom); dfree(s, s->b.aggs);
        int nb = std::max<int>((int)bd.size(), 1), ns = std::max<int>((int)sd.size(), 1), nz = std::max(n_zones, 1);
        if (!alloc_n(s, s->b.bodies, nb) || !alloc_n(s, s->b.shapes, ns) ||
            !alloc_n(s, s->b.force_part, (int64_t)nb * kForceChunks * 6) || !alloc_n(s, s->b.body_ft, (int64_t)nb * 6) ||
            !alloc_n(s, s->b.zone_mom, (int64_t)nz * kZoneMoments) || !alloc_n(s, s->b.aggs, nz))
            return fail(s, TR_E_NOMEM, "body tables");
        s->bodies_alloc = nb; s->shapes_alloc = ns; s->zones_alloc = nz;
        HIP_CHECK(s, hipMemsetAsync(s->b.body_ft, 0, sizeof(double) * nb * 6, st));
        HIP_CHECK(s, hipMemsetAsync(s->b.aggs, 0, sizeof(tr_aggregate) * nz, st));
    }
    if (NCOL > s->cols_alloc) {
        dfree(s, s->b.colmax);
        if (!alloc_n(s, s->b.colmax, NCOL)) return fail(s, TR_E_NOMEM, "depth columns");
        s->cols_alloc = NCOL;
    }
    if ((int64_t)chunks.size() > s->zone_chunk_alloc) {
        dfree(s, s->b.zone_chunks); dfree(s, s->b.zone_part);
        int64_t nch = std::max<int64_t>((int64_t)chunks.size(), 1);
        if (!alloc_n(s, s->b.zone_chunks, nch) || !alloc_n(s, s->b.zone_part, nch * kMaxZonesPerEnv * kZoneMoments))
            return fail(s, TR_E_NOMEM, "zone chunks");
        s->zone_chunk_alloc = nch;
    }
    if ((int)td.size() > s->tools_alloc) {
        dfree(s, s->b.tools); dfree(s, s->b.wedges);
        int nt = std::max<int>((int)td.size(), 1);
        if (!alloc_n(s, s->b.tools, nt) || !alloc_n(s, s->b.wedges, (int64_t)nt * TR_MAX_WEDGES))
            return fail(s, TR_E_NOMEM, "tool tables");
        s->tools_alloc = nt;
    }
    if ((int64_t)pool.size() > s->hf_alloc) {
        dfree(s, s->b.hf_pool);
        if (!alloc_n(s, s->b.hf_pool, (int64_t)pool.size())) return fail(s, TR_E_NOMEM, "heightfields");
        s->hf_alloc = (int64_t)pool.size();
    }
    HIP_CHECK(s, hipMemcpyAsync(s->b.envs, ed.data(), sizeof(EnvDev) * E, hipMemcpyHostToDevice, st));
    if (!bd.empty()) HIP_CHECK(s, hipMemcpyAsync(s->b.bodies, bd.data(), sizeof(BodyDev) * bd.size(), hipMemcpyHostToDevice, st));
    if (!sd.empty()) HIP_CHECK(s, hipMemcpyAsync(s->b.shapes, sd.data(), sizeof(ShapeDev) * sd.size(), hipMemcpyHostToDevice, st));
    if (!pool.empty()) HIP_CHECK(s, hipMemcpyAsync(s->b.hf_pool, pool.data(), sizeof(float) * pool.size(), hipMemcpyHostToDevice, st));
    if (!td.empty()) HIP_CHECK(s, hipMemcpyAsync(s->b.tools, td.data(), sizeof(ToolDev) * td.size(), hipMemcpyHostToDevice, st));
    if (!chunks.empty()) HIP_CHECK(s, hipMemcpyAsync(s->b.zone_chunks, chunks.data(), sizeof(int4) * chunks.size(), hipMemcpyHostToDevice, st));
    HIP_CHECK(s, hipStreamSynchronize(st));  // host vectors die here
    s->body_host = bd;
    s->env_host = ed;
    s->tool_host = td;
    s->shape_host = sd;
    s->p.n_tools = (int)td.size();
    s->z.NC = NC;
    s->z.NCOL = NCOL;
    s->z.n_zone_chunks = (int)chunks.size();
    s->p.n_bodies = (int)bd.size();
    s->p.n_shapes = (int)sd.size();
    s->p.n_zones = n_zones;
    s->tables_dirty = false;
    return rebuild_plan(s);
}

// Download the device poses into the host body descriptions (they advance on
// the device), so that rebuilding the tables keeps them.
int sync_poses(tr_scene* s)
{
    if (s->body_host.empty()) return TR_OK;
    std::vector<BodyDev> bd(s->body_host.size());
    HIP_CHECK(s, hipMemcpyAsync(bd.data(), s->b.bodies, sizeof(BodyDev) * bd.size(), hipMemcpyDeviceToHost, s->stream));
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    for (const BodyDev& X : bd) {
        EnvHost& H = s->envs[X.env];
        for (tr_body_desc& B : H.bodies)
            if (B.id == X.user_id) {
                for (int k = 0; k < 3; ++k) B.pos[k] = X.pos[k];
                for (int k = 0; k < 4; ++k) B.quat[k] = X.quat[k];
            }
    }
    s->body_host = bd;
    return TR_OK;
}

void fill_params(tr_scene* s)
{
    const tr_scene_desc& d = s->desc;
    const tr_material& m = d.material;
    StepParams& p = s->p;
    double dt = d.dt;
    double tau = m.tau_n > 0.0 ? m.tau_n : 2.0 * dt;
    double ups = 1.0 / (1.0 + 4.0 * tau / dt);
    p.dt = (float)dt;
    for (int k = 0; k < 3; ++k) p.g[k] = (float)d.gravity[k];
    p.mu = (float)m.mu_t;
    p.mu_r = (float)m.mu_r;
    p.v_imp = m.v_imp > 0.0 ? (float)m.v_imp : 0.f;
    p.restitution = (float)m.restitution;
    p.gamma_dt = (float)(m.gamma_t / dt);
    p.kappa_c = m.c_p > 0.0 ? m.kappa_c : 0.0;
    p.kappa_min = m.kappa_min;
    p.Estar = m.E / (2.0 * (1.0 - m.nu * m.nu));
    p.a_coef = (4.0 / dt) * ups;
    p.b_coef = ups;
    p.sig_coef = (4.0 / (dt * dt)) * ups;
    p.lo_coef = m.c_p * 3.14159265358979323846 * dt;
    p.id_cap = (uint32_t)d.cap_particles;
    p.n_envs = d.n_envs;
    p.max_sweeps = d.max_sweeps;
    p.tol = (float)d.tol;
    p.warm = d.warm_start;
    p.dt_d = dt;
    p.gdt = std::sqrt(d.gravity[0] * d.gravity[0] + d.gravity[1] * d.gravity[1] + d.gravity[2] * d.gravity[2]) * dt;
    if (!(p.gdt > 0.0)) p.gdt = 1.0;
    p.r_ref = d.r_ref > 0.0 ? d.r_ref : 1.0;
}

}  // namespace

extern "C" {

int create_scene(const tr_scene_desc* d, tr_scene** out)
{
    if (!d || !out) return TR_E_INVAL;
    *out = nullptr;
    if (d->n_envs < 1 || d->dt <= 0.0 || d->max_sweeps < 0 || d->cap_particles < 1 || d->cap_contacts < 1 ||
        !d->env_bounds)
        return TR_E_INVAL;
    if (!(d->material.mu_r >= 0.0) || !(d->material.restitution >= 0.0 && d->material.restitution <= 1.0) ||
        !std::isfinite(d->material.v_imp))
        return TR_E_INVAL;
    if (d->warm_start < TR_WARM_COLD || d->warm_start > TR_WARM_LEARNED) return TR_E_INVAL;
    if ((d->alloc_fn == nullptr) != (d->free_fn == nullptr)) return TR_E_INVAL;  // both or neither
    // the solver's body loads take 31-bit byte offsets into the 32 B velocity records
    if ((int64_t)d->n_envs * d->cap_particles > ((int64_t)1 << 26) ||
        (int64_t)d->n_envs * d->cap_contacts >= ((int64_t)1 << 31))
        return TR_E_CAPACITY;
    if (!finite3(d->env_bounds, 6 * (int64_t)d->n_envs)) return TR_E_NONFINITE;
    tr_scene* s = new tr_scene();
    s->desc = *d;
    s->bounds.assign(d->env_bounds, d->env_bounds + 6 * d->n_envs);
    s->desc.env_bounds = s->bounds.data();
    s->stream = (hipStream_t)d->stream;
    s->envs.resize(d->n_envs);
    fill_params(s);
    Sizes& z = s->z;
    z.P = (int64_t)d->n_envs * d->cap_particles;
    z.C = (int64_t)d->n_envs * d->cap_contacts;
    z.NID = z.P;
    z.NB = (z.C + 255) / 256;
    z.roll_C = d->material.mu_r > 0.0 ? z.C : 1;  // rolling rows only when mu_r > 0
    z.imp_C = d->material.v_imp > 0.0 ? z.C : 1;  // impact-stage rows only when v_imp > 0
    z.n_envs = d->n_envs;
    z.pgs_block = 512;
    s->p.n_units = std::max(kGroups, d->n_envs);
    // default schedule: grouped for a few envs (XCD groups of 32 blocks, one
    // per CU), per-env blocks with LDS-resident bodies for many envs
    s->max_lds_particles = std::max(0, pgs_env_max_lds() / 32);
    s->cfg.mode = d->n_envs > kGroups ? TR_PGS_PER_ENV : TR_PGS_GROUPED;
    s->cfg.blocks_per_xcd = 32;
    s->cfg.lds_particles = s->max_lds_particles;
    s->cfg.cluster_particles = 0;
    s->cfg.dataflow = 0;
    z.pgs_grid = kGroups * std::max(1, std::min(s->cfg.blocks_per_xcd, pgs_resident_blocks(512) / kGroups));
    z.col_grid = std::min(colour_resident_blocks(), 2048);
    DevBuffers& b = s->b;
    bool ok = alloc_n(s, b.xr, z.P) && alloc_n(s, b.vw, 2 * z.P) && alloc_n(s, b.xr2, z.P) &&
              alloc_n(s, b.vw2, 2 * z.P) && alloc_n(s, b.pid, z.P) && alloc_n(s, b.pid2, z.P) &&
              alloc_n(s, b.rho, z.P) && alloc_n(s, b.rho2, z.P) && alloc_n(s, b.pkey, z.P) &&
              alloc_n(s, b.perm, z.P) && alloc_n(s, b.id2slot, z.NID) && alloc_n(s, b.rkey, z.C) &&
              alloc_n(s, b.ckey, z.C) && alloc_n(s, b.pkeyc, z.C) && alloc_n(s, b.rpair, z.C) &&
              alloc_n(s, b.cpair, z.C) && alloc_n(s, b.lamc, z.C) && alloc_n(s, b.plam, z.C) &&
              alloc_n(s, b.id_count, z.NID) && alloc_n(s, b.id_start, z.NID + 1) && alloc_n(s, b.id_fill, z.NID) &&
              alloc_n(s, b.pid_start, z.NID + 1) && alloc_n(s, b.inc_count, z.P) &&
              alloc_n(s, b.inc_start, z.P + 1) && alloc_n(s, b.inc_fill, z.P) && alloc_n(s, b.inc, 2 * z.C) &&
              alloc_n(s, b.colour, z.C) && alloc_n(s, b.col_wait, z.C) && alloc_n(s, b.col_hist, (int64_t)kBuckets * z.NB) &&
              alloc_n(s, b.col_start, (int64_t)kBuckets * z.NB + 1) && alloc_n(s, b.cpos, z.C) &&
              alloc_n(s, b.r0, z.C) && alloc_n(s, b.r1, z.C) && alloc_n(s, b.r2, z.C) && alloc_n(s, b.rk, z.C) &&
              alloc_n(s, b.r3, z.roll_C) && alloc_n(s, b.lamr, z.roll_C) && alloc_n(s, b.lamr0, z.roll_C) &&
              alloc_n(s, b.lamrc, z.roll_C) && alloc_n(s, b.plamr, z.roll_C) &&
              alloc_n(s, b.ri1, z.imp_C) && alloc_n(s, b.ri2, z.imp_C) && alloc_n(s, b.lami, z.imp_C) &&
              alloc_n(s, b.lamri, std::min(z.imp_C, z.roll_C)) && alloc_n(s, b.qg, z.imp_C) &&
              alloc_n(s, b.lam, z.C) && alloc_n(s, b.lam0, z.C) && alloc_n(s, b.wrec, 3 * z.C) &&
              alloc_n(s, b.envs, d->n_envs) && alloc_n(s, b.ustats, s->p.n_units) &&
              alloc_n(s, b.env_col, (int64_t)d->n_envs * (kMaxColours + 1)) && alloc_n(s, b.env_ncol, d->n_envs) &&
              alloc_n(s, b.env_bar, (int64_t)d->n_envs * 16) && alloc_n(s, b.ver, z.P) &&
              alloc_n(s, b.cnt, 1) && alloc_n(s, b.env_stats, d->n_envs) && alloc_n(s, b.mlp, kMlpParams) &&
              alloc_n(s, s->staging, 12 * z.P) && alloc_n(s, b.feat, 12 * z.C) && alloc_n(s, b.frm1, z.C) &&
              alloc_n(s, b.frm2, z.C) && alloc_n(s, b.lamL, z.C) && alloc_n(s, b.mlp_out, 3 * z.C) &&
              alloc_n(s, b.pdepth, z.P);
    if (!ok) {
        destroy_scene(s);
        return TR_E_NOMEM;
    }
    hipError_t e = hipMemsetAsync(b.cnt, 0, sizeof(Counters), s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b.env_stats, 0, sizeof(EnvStats) * d->n_envs, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b.ustats, 0, sizeof(UnitStats) * s->p.n_units, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b.env_ncol, 0, sizeof(uint32_t) * d->n_envs, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b.id_start, 0, sizeof(uint32_t) * (z.NID + 1), s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b.pid_start, 0, sizeof(uint32_t) * (z.NID + 1), s->stream);
    for (int k = 0; k < 5 && e == hipSuccess; ++k) e = hipEventCreate(&s->ev[k]);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        destroy_scene(s);
        return TR_E_DEVICE;
    }
    s->events = true;
    *out = s;
    return TR_OK;
}

int destroy_scene(tr_scene* s)
{
    if (!s) return TR_OK;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    else (void)hipDeviceSynchronize();
    invalidate_graphs(s);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    while (!s->allocs.empty()) dfree(s, s->allocs.back().first);
    if (s->events)
        for (int k = 0; k < 5; ++k) (void)hipEventDestroy(s->ev[k]);
    delete s;
    return TR_OK;
}

int add_particles(tr_scene* s, int32_t env, int64_t n, const double* pos, const double* vel, const double* radius,
                  const double* density, int64_t* first_id)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs || n < 0 || (n > 0 && (!pos || !radius)))
        return fail(s, TR_E_INVAL, "add_particles: bad arguments");
    EnvHost& H = s->envs[env];
    if (H.n + n > s->desc.cap_particles) return fail(s, TR_E_CAPACITY, "add_particles: env particle capacity");
    if (!finite3(pos, 3 * n) || (vel && !finite3(vel, 3 * n)) || !finite3(radius, n) || (density && !finite3(density, n)))
        return fail(s, TR_E_NONFINITE, "add_particles: non-finite input");
    for (int64_t i = 0; i < n; ++i) {
        if (radius[i] <= 0.0) return fail(s, TR_E_INVAL, "add_particles: radius <= 0");
        if (density && density[i] <= 0.0) return fail(s, TR_E_INVAL, "add_particles: density <= 0");
    }
    int64_t id0 = (int64_t)env * s->desc.cap_particles + H.n;
    if (first_id) *first_id = id0;
    if (n == 0) return TR_OK;
    for (int e2 = env + 1; e2 < s->desc.n_envs; ++e2)
        if (s->envs[e2].n > 0) s->slots_env_major = false;  // appended behind a later env's spheres
    std::vector<float4> xr(n), vw(2 * n);
    std::vector<int> pid(n), id2s(n);
    std::vector<float> rho(n);
    const double pi = 3.14159265358979323846;
    for (int64_t i = 0; i < n; ++i) {
        float r = (float)radius[i];
        double dens = density ? density[i] : s->desc.material.rho;
        float rhof = (float)dens;
        double rr = r;
        double m = (double)rhof * (4.0 / 3.0) * pi * rr * rr * rr;
        xr[i] = make_float4((float)pos[3 * i], (float)pos[3 * i + 1], (float)pos[3 * i + 2], r);
        vel_at(vw.data(), i) = make_float4(vel ? (float)vel[3 * i] : 0.f, vel ? (float)vel[3 * i + 1] : 0.f,
                                           vel ? (float)vel[3 * i + 2] : 0.f, (float)(1.0 / m));
        angv_at(vw.data(), i) = make_float4(0.f, 0.f, 0.f, (float)(1.0 / (0.4 * m * rr * rr)));
        pid[i] = (int)(id0 + i);
        id2s[i] = (int)(s->n_total + i);
        rho[i] = rhof;
        H.rmax = std::max(H.rmax, rr);
    }
    hipStream_t st = s->stream;
    int64_t at = s->n_total;
    HIP_CHECK(s, hipMemcpyAsync(s->b.xr + at, xr.data(), sizeof(float4) * n, hipMemcpyHostToDevice, st));
    HIP_CHECK(s, hipMemcpyAsync(s->b.vw + 2 * at, vw.data(), sizeof(float4) * 2 * n, hipMemcpyHostToDevice, st));
    HIP_CHECK(s, hipMemcpyAsync(s->b.pid + at, pid.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
    HIP_CHECK(s, hipMemcpyAsync(s->b.rho + at, rho.data(), sizeof(float) * n, hipMemcpyHostToDevice, st));
    HIP_CHECK(s, hipMemcpyAsync(s->b.id2slot + id0, id2s.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
    HIP_CHECK(s, hipStreamSynchronize(st));
    H.n += n;
    s->n_total += n;
    s->p.n_particles = (int)s->n_total;
    s->have_prev = false;
    // particles of later envs must follow this env in slot order: the next
    // step's sort restores (env, cell, id) order
    int rc = sync_poses(s);
    if (rc) return rc;
    s->tables_dirty = true;
    return TR_OK;
}

int set_kinematic_bodies(tr_scene* s, int32_t env, int32_t n, const tr_body_desc* b)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs || n < 0 || (n > 0 && !b)) return fail(s, TR_E_INVAL, "set_kinematic_bodies: bad arguments");
    int rc = sync_poses(s);
    if (rc) return rc;
    EnvHost& H = s->envs[env];
    std::vector<tr_body_desc> bodies;
    std::vector<std::vector<tr_shape_desc>> shapes;
    std::vector<std::vector<std::vector<float>>> heights;
    int zones = 0;
    for (int i = 0; i < n; ++i) {
        const tr_body_desc& B = b[i];
        if (B.n_shapes < 0 || (B.n_shapes > 0 && !B.shapes) || B.n_halfspaces < 0 || B.n_halfspaces > 8)
            return fail(s, TR_E_INVAL, "body: bad shapes or half-spaces");
        if (!finite3(B.pos, 3) || !finite3(B.quat, 4) || !finite3(B.linvel, 3) || !finite3(B.angvel, 3) ||
            !finite3(&B.planes[0][0], 4 * B.n_halfspaces))
            return fail(s, TR_E_NONFINITE, "body: non-finite pose");
        double qn = std::sqrt(B.quat[0] * B.quat[0] + B.quat[1] * B.quat[1] + B.quat[2] * B.quat[2] + B.quat[3] * B.quat[3]);
        if (std::fabs(qn - 1.0) > 1e-6) return fail(s, TR_E_INVAL, "body: quaternion not unit");
        if (B.n_halfspaces > 0) ++zones;
        for (int j = 0; j < i; ++j)
            if (b[j].id == B.id) return fail(s, TR_E_INVAL, "body: duplicate id");
        bodies.push_back(B);
        bodies.back().shapes = nullptr;
        shapes.emplace_back();
        heights.emplace_back();
        for (int k = 0; k < B.n_shapes; ++k) {
            tr_shape_desc S = B.shapes[k];
            std::vector<float> hh;
            if (S.type == TR_HEIGHTFIELD) {
                if (S.nx < 2 || S.ny < 2 || S.l0 <= 0.0 || !S.heights) return fail(s, TR_E_INVAL, "heightfield: bad grid");
                hh.assign(S.heights, S.heights + (int64_t)S.nx * S.ny);
                for (float v : hh)
                    if (!std::isfinite(v)) return fail(s, TR_E_NONFINITE, "heightfield: non-finite height");
                S.heights = nullptr;
            } else if (S.type == TR_BOX) {
                if (S.half[0] <= 0 || S.half[1] <= 0 || S.half[2] <= 0) return fail(s, TR_E_INVAL, "box: half extents");
            } else if (S.type == TR_PLANE) {
                double nn = S.normal[0] * S.normal[0] + S.normal[1] * S.normal[1] + S.normal[2] * S.normal[2];
                if (std::fabs(nn - 1.0) > 1e-9) return fail(s, TR_E_INVAL, "plane: normal not unit");
            } else {
                return fail(s, TR_E_INVAL, "shape: unknown type");
            }
            shapes.back().push_back(S);
            heights.back().push_back(std::move(hh));
        }
    }
    if (zones > kMaxZonesPerEnv) return fail(s, TR_E_CAPACITY, "more than 4 zones in an env");
    H.bodies = std::move(bodies);
    H.shapes = std::move(shapes);
    H.heights = std::move(heights);
    s->tables_dirty = true;
    s->have_prev = false;
    return TR_OK;
}

}  // extern "C"

namespace {
// host side of a step's buffer rotation: the sorted particle arrays (written
// into the *2 buffers) and the previous-step contact cache
void swap_particle_buffers(tr_scene* s)
{
    std::swap(s->b.xr, s->b.xr2);
    std::swap(s->b.vw, s->b.vw2);
    std::swap(s->b.pid, s->b.pid2);
    std::swap(s->b.rho, s->b.rho2);
}

void swap_step_buffers(tr_scene* s)
{
    std::swap(s->b.ckey, s->b.pkeyc);
    std::swap(s->b.lamc, s->b.plam);
    std::swap(s->b.lamrc, s->b.plamr);
    std::swap(s->b.id_start, s->b.pid_start);
}

// the learned start's features are written when the step runs the network or
// the caller captures training samples
bool rows_features(const tr_scene* s) { return s->capture || (s->p.warm == TR_WARM_LEARNED && s->mlp_loaded); }

// Every launch of one step, in stream order (A1-A12).  The sorted particle
// arrays are written into the *2 buffers and swapped in; the canonical keys,
// impulses and id ranges become the next step's previous-step cache.
void enqueue_step(tr_scene* s, hipStream_t st, bool events)
{
    if (events) (void)hipEventRecord(s->ev[0], st);
    launch_step_begin(s->b, s->p, st);
    launch_sort_particles(s->b, s->p, s->z, st);
    swap_particle_buffers(s);
    launch_narrow(s->b, s->p, s->z, st);
    launch_canonical(s->b, s->p, s->z, st);
    if (events) (void)hipEventRecord(s->ev[1], st);
    launch_depth(s->b, s->p, s->z, st);
    launch_colour(s->b, s->p, s->z, st);
    launch_rows(s->b, s->p, s->z, s->have_prev, rows_features(s), st);
    launch_impact_stage(s->b, s->p, s->z, st);
    if (s->p.warm == TR_WARM_LEARNED && s->mlp_loaded) {
        // learned start, then the first-sweep trial against the previous-step start
        launch_mlp_infer(s->b.mlp, s->b.feat, s->b.mlp_out, &s->b.cnt->n_raw, s->z.C, s->mlp_bf16, st);
        launch_learned_lam(s->b, s->p, s->z, st);
        launch_vel_copy(s->b, s->p, true, st);
        launch_select_start(s->b, s->p, s->z, 1, st);
        launch_warm_apply(s->b, s->p, s->z, true, st);
        launch_pgs(s->b, s->p, s->z, st, 1, 1);
        launch_vel_copy(s->b, s->p, false, st);
        launch_select_start(s->b, s->p, s->z, 0, st);
        launch_warm_apply(s->b, s->p, s->z, true, st);
        launch_pgs(s->b, s->p, s->z, st, 1, 2);
        launch_choose_start(s->b, s->p, st);
        launch_vel_copy(s->b, s->p, false, st);
        launch_select_start(s->b, s->p, s->z, 2, st);
    }
    // the learned path has replaced the start impulses that k_rows recorded
    launch_warm_apply(s->b, s->p, s->z, s->p.warm == TR_WARM_LEARNED && s->mlp_loaded, st);
    if (events) (void)hipEventRecord(s->ev[2], st);
    launch_pgs(s->b, s->p, s->z, st);
    if (events) (void)hipEventRecord(s->ev[3], st);
    launch_finish(s->b, s->p, s->z, st);
    if (events) (void)hipEventRecord(s->ev[4], st);
    swap_step_buffers(s);
}

// Capture the two steps of the buffer rotation as graphs, on a private
// stream (a scene on the null stream can replay them too).  Capturing
// records launches without running them; the two captured rotations bring
// the host buffer state back to where it was.
int capture_graphs(tr_scene* s)
{
    invalidate_graphs(s);
    if (!s->cap_stream) HIP_CHECK(s, hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    // no phase events inside the graphs: measured on ROCm, a replayed event
    // node keeps the timestamps of its first recording, so a replay is timed
    // as a whole by events recorded around its launch
    hipError_t e = hipSuccess;
    for (int q = 0; q < 2 && e == hipSuccess; ++q) {
        hipGraph_t g = nullptr;
        HIP_CHECK(s, hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
        enqueue_step(s, s->cap_stream, false);
        e = hipStreamEndCapture(s->cap_stream, &g);
        if (e == hipSuccess) e = hipGraphInstantiate(&s->gexec[q], g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
    }
    if (e != hipSuccess) {
        invalidate_graphs(s);
        (void)hipGetLastError();
        return hip_fail(s, e, "step graph capture");
    }
    s->graphs = true;
    s->parity = 0;
    return TR_OK;
}
}  // namespace

extern "C" {

int set_step_graphs(tr_scene* s, int32_t enable)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    s->use_graphs = enable != 0;
    if (!s->use_graphs) invalidate_graphs(s);
    return TR_OK;
}

// Library-internal callers use step_scene: the exported name `step` is also a
// (legacy regex) function of the C library, which a call through the PLT
// could bind to.
static int step_scene(tr_scene* s, int32_t n_steps, tr_step_stats* stats);

int step(tr_scene* s, int32_t n_steps, tr_step_stats* stats) { return step_scene(s, n_steps, stats); }

static int step_scene(tr_scene* s, int32_t n_steps, tr_step_stats* stats)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (n_steps < 0) return fail(s, TR_E_INVAL, "step: n_steps < 0");
    if (s->tables_dirty) {
        int rc = rebuild_tables(s);
        if (rc) return rc;
    }
    hipStream_t st = s->stream;
    for (int k = 0; k < n_steps; ++k) {
        if (s->use_graphs && s->have_prev && !s->graphs) {
            int rc = capture_graphs(s);
            if (rc) return rc;
        }
        if (s->graphs && s->have_prev) {
            (void)hipEventRecord(s->ev[0], st);
            HIP_CHECK(s, hipGraphLaunch(s->gexec[s->parity], st));
            (void)hipEventRecord(s->ev[4], st);
            s->last_replay = true;
            swap_particle_buffers(s);
            swap_step_buffers(s);
        } else {
            enqueue_step(s, st, true);
            s->last_replay = false;
        }
        s->parity ^= 1;
        s->have_prev = true;
        s->stepped = true;
        s->features_last = rows_features(s);
        s->slots_env_major = true;  // the step's sort orders the slots by (env, cell, id)
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(s, e, "step launch");
    if (n_steps == 0 && !stats) return TR_OK;
    // every call waits for its steps and reads the failure flags of all of
    // them: the current step's word and the word earlier steps folded theirs into
    HIP_CHECK(s, hipStreamSynchronize(st));
    Counters c;
    HIP_CHECK(s, hipMemcpy(&c, s->b.cnt, sizeof(c), hipMemcpyDeviceToHost));
    const uint32_t bad = c.failed | c.overflow;
    if (stats) {
        std::vector<EnvStats> es(s->desc.n_envs);
        HIP_CHECK(s, hipMemcpy(es.data(), s->b.env_stats, sizeof(EnvStats) * es.size(), hipMemcpyDeviceToHost));
        std::vector<UnitStats> us(s->p.n_units);
        std::vector<uint32_t> nc(s->desc.n_envs);
        HIP_CHECK(s, hipMemcpy(us.data(), s->b.ustats, sizeof(UnitStats) * us.size(), hipMemcpyDeviceToHost));
        HIP_CHECK(s, hipMemcpy(nc.data(), s->b.env_ncol, sizeof(uint32_t) * nc.size(), hipMemcpyDeviceToHost));
        for (int e2 = 0; e2 < s->desc.n_envs; ++e2) {
            tr_step_stats& o = stats[e2];
            o.contacts = es[e2].contacts;
            o.pair_contacts = es[e2].pairs;
            const UnitStats& G = us[s->env_host[e2].unit];
            o.colours = (int32_t)nc[e2];
            o.sweeps = (int32_t)G.sweeps;
            o.residual = G.resid;
            o.residual_first = G.resid_first;
            o.fallback_used = s->p.warm == TR_WARM_LEARNED && s->mlp_loaded ? (int32_t)G.fallback : 0;
            o.overflow = (int32_t)bad;
            o.impacts = (int32_t)es[e2].impacts;
            o.impact_sweeps = es[e2].impacts > 0 ? (int32_t)G.imp_sweeps : 0;
        }
    }
    if (bad) {
        // the flags are reported once: clear both words for the next call
        const uint32_t zero = 0u;
        HIP_CHECK(s, hipMemcpy(&s->b.cnt->failed, &zero, sizeof(zero), hipMemcpyHostToDevice));
        HIP_CHECK(s, hipMemcpy(&s->b.cnt->overflow, &zero, sizeof(zero), hipMemcpyHostToDevice));
        s->have_prev = false;
        char msg[160];
        snprintf(msg, sizeof msg,
                 "step: capacity or schedule failure in %s (flags 0x%x, %u contacts found in the last step)",
                 c.overflow ? "the last step" : "an earlier step of this call", bad, c.n_raw);
        return fail(s, TR_E_CAPACITY, msg);
    }
    return TR_OK;
}

int get_contact_forces(tr_scene* s, int32_t env, int32_t body_id, double force[3], double torque[3])
{
    if (!s || !force || !torque) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "get_contact_forces: env");
    if (s->tables_dirty) return fail(s, TR_E_STATE, "get_contact_forces: no step since the bodies changed");
    int gi = -1;
    for (size_t i = 0; i < s->body_host.size(); ++i)
        if (s->body_host[i].env == env && s->body_host[i].user_id == body_id) gi = (int)i;
    if (gi < 0) return fail(s, TR_E_INVAL, "get_contact_forces: unknown body");
    double ft[6];
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    HIP_CHECK(s, hipMemcpy(ft, s->b.body_ft + 6 * gi, sizeof(ft), hipMemcpyDeviceToHost));
    for (int k = 0; k < 3; ++k) { force[k] = ft[k]; torque[k] = ft[3 + k]; }
    return TR_OK;
}

int set_tool(tr_scene* s, int32_t env, int32_t body_id, const tr_tool_desc* t)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "set_tool: env");
    EnvHost& H = s->envs[env];
    bool known = false;
    for (const tr_body_desc& B : H.bodies) known |= B.id == body_id;
    if (!known) return fail(s, TR_E_INVAL, "set_tool: unknown body");
    auto it = std::find_if(H.tools.begin(), H.tools.end(), [&](const std::pair<int32_t, tr_tool_desc>& q) {
        return q.first == body_id;
    });
    if (!t) {
        if (it != H.tools.end()) H.tools.erase(it);
        s->tables_dirty = true;
        return TR_OK;
    }
    auto norm = [](const double* a) { return std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); };
    double de[3] = {t->edge1[0] - t->edge0[0], t->edge1[1] - t->edge0[1], t->edge1[2] - t->edge0[2]};
    double fin[18] = {t->edge0[0], t->edge0[1], t->edge0[2], t->edge1[0], t->edge1[1], t->edge1[2],
                      t->n_c[0], t->n_c[1], t->n_c[2], t->n_tc[0], t->n_tc[1], t->n_tc[2],
                      t->fill, t->phi, t->heap, t->v_min, 0.0, 0.0};
    if (!finite3(fin, 16)) return fail(s, TR_E_NONFINITE, "set_tool: non-finite value");
    if (t->n_wedges < 1 || t->n_wedges > TR_MAX_WEDGES || !(t->fill >= 0.0 && t->fill <= 1.0) ||
        !(t->phi > 0.0 && t->phi < 0.5 * M_PI) || !(t->heap >= 0.0) || !(norm(de) > 0.0) || !(norm(t->n_c) > 0.0) ||
        !(norm(t->n_tc) > 0.0))
        return fail(s, TR_E_INVAL, "set_tool: bad tool");
    int zones = 0;
    for (const tr_body_desc& B : H.bodies) {
        bool has_tool = B.id == body_id;
        for (const auto& q : H.tools) has_tool |= q.first == B.id;
        zones += B.n_halfspaces > 0 || has_tool;
    }
    if (zones > kMaxZonesPerEnv) return fail(s, TR_E_CAPACITY, "set_tool: more than 4 zones in the env");
    if (it != H.tools.end()) it->second = *t;
    else H.tools.emplace_back(body_id, *t);
    s->tables_dirty = true;
    return TR_OK;
}

int get_zone_wedges(tr_scene* s, int32_t env, int32_t body_id, int32_t cap, double* planes, int32_t* counts,
                    int32_t* n_wedges)
{
    if (!s || !n_wedges || cap < 0 || (cap > 0 && (!planes || !counts))) return TR_E_INVAL;
    s->err.clear();
    *n_wedges = 0;
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "get_zone_wedges: env");
    if (s->tables_dirty || !s->stepped) return fail(s, TR_E_STATE, "get_zone_wedges: no step since the tools changed");
    int ti = -1;
    for (size_t i = 0; i < s->tool_host.size(); ++i) {
        const BodyDev& B = s->body_host[s->tool_host[i].body];
        if (B.env == env && B.user_id == body_id) ti = (int)i;
    }
    if (ti < 0) return fail(s, TR_E_INVAL, "get_zone_wedges: the body has no tool");
    const int nw = s->tool_host[ti].n_wedges;
    *n_wedges = nw;
    std::vector<WedgeDev> w(nw);
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    HIP_CHECK(s, hipMemcpy(w.data(), s->b.wedges + (size_t)ti * TR_MAX_WEDGES, sizeof(WedgeDev) * nw,
                           hipMemcpyDeviceToHost));
    for (int k = 0; k < nw && k < cap; ++k) {
        counts[k] = w[k].n;
        for (int p = 0; p < 5; ++p)
            for (int q = 0; q < 4; ++q) planes[k * 20 + p * 4 + q] = p < w[k].n ? w[k].planes[p][q] : 0.0;
    }
    return TR_OK;
}

static bool voxel_grid_ok(const tr_voxel_grid* g)
{
    if (!g || !(g->l0 > 0.0) || !std::isfinite(g->l0) || g->nx <= 0 || g->ny <= 0 || g->nz <= 0) return false;
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(g->origin[k])) return false;
    return (int64_t)g->nx * g->ny * g->nz <= ((int64_t)1 << 31);
}

int coarse_grain(tr_scene* s, int32_t env, const tr_voxel_grid* g, int32_t kernel, double R, double* rho,
                 double* mom, double* u)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "coarse_grain: env");
    if (!voxel_grid_ok(g)) return fail(s, TR_E_INVAL, "coarse_grain: grid");
    if (kernel != TR_CG_HEAVISIDE && kernel != TR_CG_GAUSS) return fail(s, TR_E_INVAL, "coarse_grain: kernel");
    if (kernel == TR_CG_GAUSS && !(R > 0.0 && std::isfinite(R))) return fail(s, TR_E_INVAL, "coarse_grain: R");
    if (!rho || !mom) return fail(s, TR_E_INVAL, "coarse_grain: null output");
    if (s->tables_dirty) return fail(s, TR_E_STATE, "coarse_grain: no step since the bodies changed");
    launch_coarse_grain(s->b, s->env_host[env], *g, kernel, R, rho, mom, u, s->stream);
    HIP_CHECK(s, hipGetLastError());
    return TR_OK;
}

int advect_fluid(tr_scene* s, const tr_voxel_grid* g, double dt, const double* u, const double* mf_in,
                 double* mf_out, double* cfl)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (!voxel_grid_ok(g)) return fail(s, TR_E_INVAL, "advect_fluid: grid");
    if (!(dt >= 0.0 && std::isfinite(dt))) return fail(s, TR_E_INVAL, "advect_fluid: dt");
    if (!u || !mf_in || !mf_out) return fail(s, TR_E_INVAL, "advect_fluid: null pointer");
    if (mf_in == mf_out) return fail(s, TR_E_INVAL, "advect_fluid: mf_out aliases mf_in");
    unsigned long long* bits = (unsigned long long*)s->staging;  // at least 12 floats: one uint64 fits
    const int64_t nb = advect_blocks(*g);
    if (nb > s->adv_cap) {
        dfree(s, s->adv_bmax);
        s->adv_bmax = nullptr;
        s->adv_cap = 0;
        if (!alloc_n(s, s->adv_bmax, nb)) return fail(s, TR_E_NOMEM, "advect_fluid");
        s->adv_cap = nb;
    }
    launch_advect(*g, dt, u, mf_in, mf_out, s->adv_bmax, cfl ? bits : nullptr, s->stream);  // no reduction unasked
    HIP_CHECK(s, hipGetLastError());
    if (!cfl) return TR_OK;
    unsigned long long h = 0;
    HIP_CHECK(s, hipMemcpyAsync(&h, bits, sizeof(h), hipMemcpyDeviceToHost, s->stream));
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    memcpy(cfl, &h, sizeof(double));
    return TR_OK;
}

static constexpr int kMaxCallerWedges = 128;

// the wedges of a conversion call: the caller's (copied to the device) or the
// last step's predictions for env's tools
static int conversion_wedges(tr_scene* s, int32_t env, int32_t n_wedges, const int32_t* counts,
                             const double* planes, WedgeSet& ws, const char* what)
{
    memset(&ws, 0, sizeof(ws));
    if (planes) {
        if (n_wedges < 0 || n_wedges > kMaxCallerWedges || (n_wedges > 0 && !counts))
            return fail(s, TR_E_INVAL, std::string(what) + ": wedge count");
        if (n_wedges == 0) return TR_OK;
        std::vector<WedgeDev> w(n_wedges);
        for (int k = 0; k < n_wedges; ++k) {
            if (counts[k] < 0 || counts[k] > 5) return fail(s, TR_E_INVAL, std::string(what) + ": wedge planes");
            memset(&w[k], 0, sizeof(WedgeDev));
            w[k].n = counts[k];
            for (int p = 0; p < counts[k]; ++p)
                for (int q = 0; q < 4; ++q) {
                    w[k].planes[p][q] = planes[k * 20 + p * 4 + q];
                    if (!std::isfinite(w[k].planes[p][q])) return fail(s, TR_E_NONFINITE, std::string(what) + ": plane");
                }
        }
        if (!s->conv_wedges && !alloc_n(s, s->conv_wedges, kMaxCallerWedges))
            return fail(s, TR_E_NOMEM, std::string(what) + ": wedges");
        HIP_CHECK(s, hipMemcpyAsync(s->conv_wedges, w.data(), sizeof(WedgeDev) * n_wedges, hipMemcpyHostToDevice,
                                    s->stream));
        HIP_CHECK(s, hipStreamSynchronize(s->stream));  // the host vector dies here
        ws.base = s->conv_wedges;
        ws.n_ranges = 1;
        ws.cnt[0] = n_wedges;
        return TR_OK;
    }
    if (s->tables_dirty || !s->stepped) return fail(s, TR_E_STATE, std::string(what) + ": no predicted wedges yet");
    ws.base = s->b.wedges;
    for (size_t t = 0; t < s->tool_host.size(); ++t) {
        if (s->body_host[s->tool_host[t].body].env != env) continue;
        if (ws.n_ranges == kMaxConvRanges) return fail(s, TR_E_INVAL, std::string(what) + ": more than 8 tools");
        ws.off[ws.n_ranges] = (int)t * TR_MAX_WEDGES;
        ws.cnt[ws.n_ranges] = s->tool_host[t].n_wedges;
        ++ws.n_ranges;
    }
    return TR_OK;
}

static int read_total(tr_scene* s, double* out)
{
    if (!out) return TR_OK;
    HIP_CHECK(s, hipMemcpyAsync(out, s->conv_total, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    return TR_OK;
}

int terrain_from_voxels(tr_scene* s, int32_t env, int32_t body_id, const tr_voxel_grid* g, const double* phi,
                        double* h)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "terrain_from_voxels: env");
    if (!voxel_grid_ok(g) || !phi) return fail(s, TR_E_INVAL, "terrain_from_voxels: grid");
    float* hf = nullptr;
    int bi = -1, si = -1;
    if (body_id >= 0) {
        if (s->tables_dirty) return fail(s, TR_E_STATE, "terrain_from_voxels: no step since the bodies changed");
        const EnvHost& H = s->envs[env];
        for (size_t k = 0; k < H.bodies.size(); ++k)
            if (H.bodies[k].id == body_id) bi = (int)k;
        if (bi < 0) return fail(s, TR_E_INVAL, "terrain_from_voxels: no such body");
        for (size_t k = 0; k < H.shapes[bi].size() && si < 0; ++k)
            if (H.shapes[bi][k].type == TR_HEIGHTFIELD) si = (int)k;
        if (si < 0) return fail(s, TR_E_INVAL, "terrain_from_voxels: the body has no heightfield");
        const tr_shape_desc& S = H.shapes[bi][si];
        const double tol = 1e-9 * g->l0;
        if (S.nx != g->nx || S.ny != g->ny || std::fabs(S.l0 - g->l0) > tol ||
            std::fabs(S.origin[0] - (g->origin[0] + 0.5 * g->l0)) > tol ||
            std::fabs(S.origin[1] - (g->origin[1] + 0.5 * g->l0)) > tol)
            return fail(s, TR_E_INVAL, "terrain_from_voxels: the heightfield's points are not the column centres");
        const int gi = s->env_host[env].body_begin + bi;
        int k = 0;
        for (const ShapeDev& Y : s->shape_host) {
            if (Y.body != gi || Y.type != TR_HEIGHTFIELD) continue;
            if (k++ == 0) hf = s->b.hf_pool + Y.hf_off;
        }
        if (!hf) return fail(s, TR_E_STATE, "terrain_from_voxels: heightfield table");
    }
    launch_surface(*g, phi, h, hf, s->stream);
    HIP_CHECK(s, hipGetLastError());
    if (hf) {  // the host copy rebuilds the tables
        std::vector<float>& hh = s->envs[env].heights[bi][si];
        HIP_CHECK(s, hipMemcpyAsync(hh.data(), hf, sizeof(float) * hh.size(), hipMemcpyDeviceToHost, s->stream));
        HIP_CHECK(s, hipStreamSynchronize(s->stream));
    }
    return TR_OK;
}

int convert_cut(tr_scene* s, int32_t env, const tr_voxel_grid* g, double rho_b, int32_t n_wedges,
                const int32_t* counts, const double* planes, double* phi, const double* wc, double* mf,
                double* liberated)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "convert_cut: env");
    if (!voxel_grid_ok(g) || !phi || !wc || !mf) return fail(s, TR_E_INVAL, "convert_cut: grid or arrays");
    if (!(rho_b > 0.0 && std::isfinite(rho_b))) return fail(s, TR_E_INVAL, "convert_cut: rho_b");
    WedgeSet ws;
    int rc = conversion_wedges(s, env, n_wedges, counts, planes, ws, "convert_cut");
    if (rc != TR_OK) return rc;
    if (!s->conv_total && !alloc_n(s, s->conv_total, 2)) return fail(s, TR_E_NOMEM, "convert_cut");
    launch_convert_cut(*g, rho_b, ws, phi, wc, mf, liberated ? s->conv_total : nullptr, s->stream);
    HIP_CHECK(s, hipGetLastError());
    return read_total(s, liberated);
}

int convert_deposit(tr_scene* s, int32_t env, const tr_voxel_grid* g, double rho_b, double w_dep, int32_t n_wedges,
                    const int32_t* counts, const double* planes, const double* rho_p, double* phi, double* wc,
                    double* mf, double* deposited)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "convert_deposit: env");
    if (!voxel_grid_ok(g) || !phi || !wc || !mf || !rho_p) return fail(s, TR_E_INVAL, "convert_deposit: grid or arrays");
    if (!(rho_b > 0.0 && std::isfinite(rho_b)) || !(w_dep > 0.0 && std::isfinite(w_dep)))
        return fail(s, TR_E_INVAL, "convert_deposit: rho_b or w_dep");
    WedgeSet ws;
    int rc = conversion_wedges(s, env, n_wedges, counts, planes, ws, "convert_deposit");
    if (rc != TR_OK) return rc;
    if (!s->conv_total && !alloc_n(s, s->conv_total, 2)) return fail(s, TR_E_NOMEM, "convert_deposit");
    launch_convert_deposit(*g, rho_b, w_dep, ws, rho_p, phi, wc, mf, deposited ? s->conv_total : nullptr, s->stream);
    HIP_CHECK(s, hipGetLastError());
    return read_total(s, deposited);
}

int form_particles(tr_scene* s, int32_t env, const tr_voxel_grid* g, double d_min, double d_max, double phi_max,
                   int32_t n_wedges, const int32_t* counts, const double* planes, const double* rho_p,
                   const double* u, double* mf, int64_t max_new, int64_t* n_formed)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (n_formed) *n_formed = 0;
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "form_particles: env");
    if (!voxel_grid_ok(g) || !rho_p || !u || !mf) return fail(s, TR_E_INVAL, "form_particles: grid or arrays");
    if (!(d_min > 0.0) || !(d_max >= d_min) || !std::isfinite(d_max) || !(phi_max > 0.0) || max_new < 0)
        return fail(s, TR_E_INVAL, "form_particles: d_min, d_max, phi_max or max_new");
    WedgeSet ws;
    int rc = conversion_wedges(s, env, n_wedges, counts, planes, ws, "form_particles");
    if (rc != TR_OK) return rc;
    const int64_t room = std::min<int64_t>(max_new, s->desc.cap_particles - s->envs[env].n);
    if (room > s->form_cap) {
        dfree(s, s->form_list);
        s->form_list = nullptr;
        s->form_cap = 0;
        if (!alloc_n(s, s->form_list, room)) return fail(s, TR_E_NOMEM, "form_particles: list");
        s->form_cap = room;
    }
    if (!s->conv_total && !alloc_n(s, s->conv_total, 2)) return fail(s, TR_E_NOMEM, "form_particles");
    unsigned long long* cnt = (unsigned long long*)s->conv_total;
    const double rho = s->desc.material.rho;
    launch_form_candidates(*g, rho, d_min, d_max, phi_max, ws, rho_p, u, mf, s->form_list, cnt, room, s->stream);
    HIP_CHECK(s, hipGetLastError());
    unsigned long long n = 0;
    HIP_CHECK(s, hipMemcpyAsync(&n, cnt, sizeof(n), hipMemcpyDeviceToHost, s->stream));
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    if ((int64_t)n > room) return fail(s, TR_E_CAPACITY, "form_particles: more particles would form than allowed");
    if (n == 0) return TR_OK;
    std::vector<FormEntry> e(n);
    HIP_CHECK(s, hipMemcpy(e.data(), s->form_list, sizeof(FormEntry) * n, hipMemcpyDeviceToHost));
    std::sort(e.begin(), e.end(), [](const FormEntry& a, const FormEntry& b) { return a.voxel < b.voxel; });
    std::vector<double> pos(3 * n), vel(3 * n), rad(n);
    for (size_t a = 0; a < n; ++a) {
        for (int q = 0; q < 3; ++q) { pos[3 * a + q] = e[a].x[q]; vel[3 * a + q] = e[a].v[q]; }
        rad[a] = (double)(float)e[a].r;
    }
    int64_t first = 0;
    rc = add_particles(s, env, (int64_t)n, pos.data(), vel.data(), rad.data(), nullptr, &first);
    if (rc != TR_OK) return rc;
    launch_form_pay(s->form_list, (int64_t)n, rho, mf, s->stream);
    HIP_CHECK(s, hipGetLastError());
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    if (n_formed) *n_formed = (int64_t)n;
    return TR_OK;
}

int remove_particles(tr_scene* s, int32_t env, int64_t n, const int64_t* ids)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs || n < 0 || (n > 0 && !ids)) return fail(s, TR_E_INVAL, "remove_particles: arguments");
    if (n == 0) return TR_OK;
    EnvHost& H = s->envs[env];
    const int64_t id0 = (int64_t)env * s->desc.cap_particles;
    std::vector<char> gone(H.n, 0);
    for (int64_t k = 0; k < n; ++k) {
        const int64_t q = ids[k] - id0;
        if (q < 0 || q >= H.n || gone[q]) return fail(s, TR_E_INVAL, "remove_particles: id not in env or repeated");
        gone[q] = 1;
    }
    int rc = sync_poses(s);
    if (rc) return rc;
    // the env's remaining ids in order: 0, 1, ...
    std::vector<int> renum(H.n, -1);
    int64_t kept = 0;
    for (int64_t q = 0; q < H.n; ++q)
        if (!gone[q]) renum[q] = (int)(id0 + kept++);
    const int64_t N = s->n_total;
    std::vector<float4> xr(N), vw(2 * N);
    std::vector<int> pid(N);
    std::vector<float> rho(N);
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    HIP_CHECK(s, hipMemcpy(xr.data(), s->b.xr, sizeof(float4) * N, hipMemcpyDeviceToHost));
    HIP_CHECK(s, hipMemcpy(vw.data(), s->b.vw, sizeof(float4) * 2 * N, hipMemcpyDeviceToHost));
    HIP_CHECK(s, hipMemcpy(pid.data(), s->b.pid, sizeof(int) * N, hipMemcpyDeviceToHost));
    HIP_CHECK(s, hipMemcpy(rho.data(), s->b.rho, sizeof(float) * N, hipMemcpyDeviceToHost));
    // compact the slots in their order, renumbering env's ids
    int64_t w = 0;
    for (int64_t sl = 0; sl < N; ++sl) {
        const int64_t q = (int64_t)pid[sl] - id0;
        if (q >= 0 && q < H.n) {
            if (gone[q]) continue;
            pid[sl] = renum[q];
        }
        xr[w] = xr[sl]; vw[2 * w] = vw[2 * sl]; vw[2 * w + 1] = vw[2 * sl + 1]; pid[w] = pid[sl]; rho[w] = rho[sl];
        ++w;
    }
    std::vector<int> id2s(s->z.NID, 0);
    for (int64_t sl = 0; sl < w; ++sl) id2s[pid[sl]] = (int)sl;
    HIP_CHECK(s, hipMemcpy(s->b.xr, xr.data(), sizeof(float4) * w, hipMemcpyHostToDevice));
    HIP_CHECK(s, hipMemcpy(s->b.vw, vw.data(), sizeof(float4) * 2 * w, hipMemcpyHostToDevice));
    HIP_CHECK(s, hipMemcpy(s->b.pid, pid.data(), sizeof(int) * w, hipMemcpyHostToDevice));
    HIP_CHECK(s, hipMemcpy(s->b.rho, rho.data(), sizeof(float) * w, hipMemcpyHostToDevice));
    HIP_CHECK(s, hipMemcpy(s->b.id2slot, id2s.data(), sizeof(int) * s->z.NID, hipMemcpyHostToDevice));
    H.n = kept;
    s->n_total = w;
    s->p.n_particles = (int)w;
    s->have_prev = false;
    s->tables_dirty = true;
    return TR_OK;
}

int settle_particles(tr_scene* s, int32_t env, const tr_voxel_grid* g, double v_rest, int32_t n_wedges,
                     const int32_t* counts, const double* planes, double* mf, int64_t* n_settled, double* mass)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (n_settled) *n_settled = 0;
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "settle_particles: env");
    if (!voxel_grid_ok(g) || !mf) return fail(s, TR_E_INVAL, "settle_particles: grid or arrays");
    if (!(v_rest >= 0.0) || !std::isfinite(v_rest)) return fail(s, TR_E_INVAL, "settle_particles: v_rest");
    if (s->tables_dirty) return fail(s, TR_E_STATE, "settle_particles: no step since the particles or bodies changed");
    WedgeSet ws;
    int rc = conversion_wedges(s, env, n_wedges, counts, planes, ws, "settle_particles");
    if (rc != TR_OK) return rc;
    if (!s->conv_total && !alloc_n(s, s->conv_total, 2)) return fail(s, TR_E_NOMEM, "settle_particles");
    if (!s->settle_list && !alloc_n(s, s->settle_list, s->desc.cap_particles))
        return fail(s, TR_E_NOMEM, "settle_particles: list");
    unsigned long long* cnt = (unsigned long long*)s->conv_total;
    launch_settle(s->b, s->env_host[env], *g, v_rest, ws, mf, s->settle_list, cnt, mass ? s->conv_total + 1 : nullptr,
                  s->stream);
    HIP_CHECK(s, hipGetLastError());
    unsigned long long n = 0;
    HIP_CHECK(s, hipMemcpyAsync(&n, cnt, sizeof(n), hipMemcpyDeviceToHost, s->stream));
    if (mass) HIP_CHECK(s, hipMemcpyAsync(mass, s->conv_total + 1, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    if (n == 0) return TR_OK;
    std::vector<int> ids32(n);
    HIP_CHECK(s, hipMemcpy(ids32.data(), s->settle_list, sizeof(int) * n, hipMemcpyDeviceToHost));
    std::vector<int64_t> ids(ids32.begin(), ids32.end());
    std::sort(ids.begin(), ids.end());
    rc = remove_particles(s, env, (int64_t)n, ids.data());
    if (rc != TR_OK) return rc;
    if (n_settled) *n_settled = (int64_t)n;
    return TR_OK;
}

int grow_particles(tr_scene* s, int32_t env, const tr_voxel_grid* g, double dt, double dprime_max, double d_max,
                   double* mf, double* work, double* grown)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "grow_particles: env");
    if (!voxel_grid_ok(g) || !mf || !work) return fail(s, TR_E_INVAL, "grow_particles: grid or arrays");
    if (!(dt >= 0.0 && std::isfinite(dt)) || !(dprime_max >= 0.0 && std::isfinite(dprime_max)) || !(d_max > 0.0))
        return fail(s, TR_E_INVAL, "grow_particles: dt, d'_max or d_max");
    if (s->tables_dirty) return fail(s, TR_E_STATE, "grow_particles: no step since the bodies changed");
    if (0.5 * d_max > s->envs[env].rmax)
        return fail(s, TR_E_INVAL, "grow_particles: d_max exceeds the env's largest diameter");
    if (!s->conv_total && !alloc_n(s, s->conv_total, 2)) return fail(s, TR_E_NOMEM, "grow_particles");
    launch_grow(s->b, s->env_host[env], *g, dt, dprime_max, d_max, mf, work, grown ? s->conv_total : nullptr,
                s->stream);
    HIP_CHECK(s, hipGetLastError());
    return read_total(s, grown);
}

int get_aggregates(tr_scene* s, int32_t env, int32_t cap, tr_aggregate* out, int32_t* n_out)
{
    if (!s || !n_out || cap < 0 || (cap > 0 && !out)) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "get_aggregates: env");
    if (s->tables_dirty) {
        *n_out = 0;
        return fail(s, TR_E_STATE, "get_aggregates: no step since the bodies changed");
    }
    const std::vector<int>& zs = s->zone_slots[env];
    *n_out = (int32_t)zs.size();
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    for (int k = 0; k < (int)zs.size() && k < cap; ++k)
        HIP_CHECK(s, hipMemcpy(&out[k], s->b.aggs + zs[k], sizeof(tr_aggregate), hipMemcpyDeviceToHost));
    return TR_OK;
}

int macro_step(tr_scene* s, int32_t env, const tr_macro_params* mp, int32_t n_eq, const tr_macro_equipment* eq,
               int32_t cap, tr_macro_result* out, int32_t* n_out)
{
    if (!s || !mp || !n_out || cap < 0 || (cap > 0 && !out) || n_eq < 0 || (n_eq > 0 && !eq)) return TR_E_INVAL;
    s->err.clear();
    *n_out = 0;
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "macro_step: env");
    const double pv[6] = {mp->E_b, mp->c_b, mp->mu_ab, mp->mu_ac, mp->cas_ab, mp->cas_ac};
    if (!finite3(pv, 6) || !(mp->E_b > 0.0) || !(mp->cas_ab > 0.0) || !(mp->cas_ac > 0.0) || mp->c_b < 0.0 ||
        mp->mu_ab < 0.0 || mp->mu_ac < 0.0)
        return fail(s, TR_E_INVAL, "macro_step: parameters");
    if (s->tables_dirty) {
        int rc = rebuild_tables(s);
        if (rc) return rc;
    }
    const EnvDev& E = s->env_host[env];
    for (int32_t k = 0; k < n_eq; ++k) {
        const tr_macro_equipment& q = eq[k];
        bool found = false;
        for (int g = E.body_begin; g < E.body_end; ++g) found |= s->body_host[g].user_id == q.body_id;
        for (int32_t j = 0; j < k; ++j)
            if (eq[j].body_id == q.body_id) return fail(s, TR_E_INVAL, "macro_step: equipment named twice");
        const double* I = q.inertia;
        const double vals[13] = {q.mass, I[0], I[1], I[2], I[3], I[4], I[5], q.f_max, q.t_max, q.gamma_drive,
                                 q.v_target[0] + q.v_target[1] + q.v_target[2],
                                 q.w_target[0] + q.w_target[1] + q.w_target[2], 0.0};
        // positive definite inertia: leading principal minors > 0
        const double m2 = I[0] * I[1] - I[3] * I[3];
        const double m3 = I[0] * (I[1] * I[2] - I[5] * I[5]) - I[3] * (I[3] * I[2] - I[5] * I[4]) +
                          I[4] * (I[3] * I[5] - I[1] * I[4]);
        if (!found || !finite3(vals, 13) || !(q.mass > 0.0) || !(I[0] > 0.0) || !(m2 > 0.0) || !(m3 > 0.0) ||
            !(q.gamma_drive > 0.0) || q.f_max < 0.0 || q.t_max < 0.0)
            return fail(s, TR_E_INVAL, "macro_step: equipment entry");
    }
    MacroArgs a;
    memset(&a, 0, sizeof(a));
    a.n = (int)s->envs[env].n;
    a.id_base = E.id_base;
    a.slot_begin = s->slots_env_major ? E.slot_begin : -1;
    a.shape_begin = E.shape_begin;
    a.shape_end = E.shape_end;
    a.mp = *mp;
    for (int k = 0; k < 3; ++k) a.g[k] = s->desc.gravity[k];
    for (int g = E.body_begin; g < E.body_end; ++g) {
        const BodyDev& B = s->body_host[g];
        if (B.nplanes <= 0) continue;
        if (a.n_zones >= kMacroMaxZones) return fail(s, TR_E_CAPACITY, "macro_step: more than 8 bodies with half-spaces");
        a.body[a.n_zones] = g;
        a.eligible[a.n_zones] = B.nplanes >= 2;
        for (int32_t k = 0; k < n_eq; ++k)
            if (eq[k].body_id == B.user_id) {
                a.has_eq[a.n_zones] = 1;
                a.eq[a.n_zones] = eq[k];
            }
        ++a.n_zones;
    }
    if (a.n_zones == 0) return TR_OK;
    if (!s->macro_zone) {
        if (!alloc_n(s, s->macro_zone, kMacroMaxZones) || !alloc_n(s, s->macro_out, kMacroMaxZones))
            return fail(s, TR_E_NOMEM, "macro_step: device table");
    }
    launch_macro(s->b, s->p, a, s->macro_zone, s->macro_out, s->stream);
    HIP_CHECK(s, hipGetLastError());
    std::vector<tr_macro_result> h(a.n_zones);
    HIP_CHECK(s, hipMemcpyAsync(h.data(), s->macro_out, sizeof(tr_macro_result) * a.n_zones, hipMemcpyDeviceToHost,
                                s->stream));
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    int32_t m = 0;
    for (int z = 0; z < a.n_zones; ++z) {
        if (!a.eligible[z] || !(h[z].M > 0.0)) continue;
        if (m < cap) out[m] = h[z];
        ++m;
    }
    *n_out = m;
    return TR_OK;
}

int set_solver_config(tr_scene* s, const tr_solver_config* cfg)
{
    if (!s || !cfg) return TR_E_INVAL;
    s->err.clear();
    if ((cfg->mode != TR_PGS_GROUPED && cfg->mode != TR_PGS_PER_ENV && cfg->mode != TR_PGS_SPREAD) ||
        cfg->blocks_per_xcd < 1 || cfg->lds_particles < 0 || cfg->cluster_particles < TR_CLUSTER_NONE ||
        (cfg->dataflow != 0 && cfg->dataflow != 1))
        return fail(s, TR_E_INVAL, "set_solver_config: bad field");
    if (cfg->mode == TR_PGS_SPREAD && (s->desc.n_envs != 1 || cfg->dataflow))
        return fail(s, TR_E_INVAL, "set_solver_config: the spread schedule takes one env and barriers");
    s->cfg = *cfg;
    s->cfg.blocks_per_xcd = std::min(cfg->blocks_per_xcd, std::max(1, pgs_resident_blocks(512) / kGroups));
    s->cfg.lds_particles = std::min(cfg->lds_particles, s->max_lds_particles);
    s->z.pgs_grid = kGroups * s->cfg.blocks_per_xcd;
    return s->tables_dirty ? TR_OK : rebuild_plan(s);
}

int get_solver_config(tr_scene* s, tr_solver_config* cfg)
{
    if (!s || !cfg) return TR_E_INVAL;
    *cfg = s->cfg;
    return TR_OK;
}

const char* get_last_error(tr_scene* s) { return s ? s->err.c_str() : "null scene"; }

int get_contacts(tr_scene* s, int32_t env, int64_t cap, uint64_t* keys, float* impulse4, int64_t* n)
{
    if (!s || !n || cap < 0 || (cap > 0 && !keys)) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "get_contacts: env");
    *n = 0;
    if (!s->stepped) return TR_OK;
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    // after a step the canonical lists of that step live in the "previous" buffers
    int64_t base = (int64_t)env * s->desc.cap_particles;
    uint32_t r[2];
    HIP_CHECK(s, hipMemcpy(&r[0], s->b.pid_start + base, sizeof(uint32_t), hipMemcpyDeviceToHost));
    HIP_CHECK(s, hipMemcpy(&r[1], s->b.pid_start + base + s->desc.cap_particles, sizeof(uint32_t), hipMemcpyDeviceToHost));
    int64_t cnt = (int64_t)r[1] - (int64_t)r[0];
    *n = cnt;
    int64_t m = std::min(cnt, cap);
    if (m > 0) {
        HIP_CHECK(s, hipMemcpy(keys, s->b.pkeyc + r[0], sizeof(uint64_t) * m, hipMemcpyDeviceToHost));
        if (impulse4) HIP_CHECK(s, hipMemcpy(impulse4, s->b.plam + r[0], sizeof(float4) * m, hipMemcpyDeviceToHost));
    }
    // keys of boundary contacts carry the env-local shape index already
    return TR_OK;
}

int get_colours(tr_scene* s, int32_t env, int64_t cap, int32_t* colours, int64_t* n)
{
    if (!s || !n || cap < 0 || (cap > 0 && !colours)) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "get_colours: env");
    *n = 0;
    if (!s->stepped) return TR_OK;
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    // the colours are indexed by the canonical position of the last step,
    // whose id ranges now live in the "previous" buffers
    int64_t base = (int64_t)env * s->desc.cap_particles;
    uint32_t r[2];
    HIP_CHECK(s, hipMemcpy(&r[0], s->b.pid_start + base, sizeof(uint32_t), hipMemcpyDeviceToHost));
    HIP_CHECK(s, hipMemcpy(&r[1], s->b.pid_start + base + s->desc.cap_particles, sizeof(uint32_t), hipMemcpyDeviceToHost));
    int64_t cnt = (int64_t)r[1] - (int64_t)r[0];
    *n = cnt;
    int64_t m = std::min(cnt, cap);
    if (m > 0) HIP_CHECK(s, hipMemcpy(colours, s->b.colour + r[0], sizeof(int32_t) * m, hipMemcpyDeviceToHost));
    return TR_OK;
}

int get_rolling_impulses(tr_scene* s, int32_t env, int64_t cap, float* impulse3, int64_t* n)
{
    if (!s || !n || cap < 0 || (cap > 0 && !impulse3)) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "get_rolling_impulses: env");
    *n = 0;
    if (!s->stepped) return TR_OK;
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    int64_t base = (int64_t)env * s->desc.cap_particles;
    uint32_t r[2];
    HIP_CHECK(s, hipMemcpy(&r[0], s->b.pid_start + base, sizeof(uint32_t), hipMemcpyDeviceToHost));
    HIP_CHECK(s, hipMemcpy(&r[1], s->b.pid_start + base + s->desc.cap_particles, sizeof(uint32_t), hipMemcpyDeviceToHost));
    int64_t cnt = (int64_t)r[1] - (int64_t)r[0];
    *n = cnt;
    int64_t m = std::min(cnt, cap);
    if (m <= 0) return TR_OK;
    if (!(s->desc.material.mu_r > 0.0)) {
        for (int64_t i = 0; i < 3 * m; ++i) impulse3[i] = 0.f;
        return TR_OK;
    }
    std::vector<float4> h((size_t)m);
    HIP_CHECK(s, hipMemcpy(h.data(), s->b.plamr + r[0], sizeof(float4) * m, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < m; ++i) {
        impulse3[3 * i] = h[i].x;
        impulse3[3 * i + 1] = h[i].y;
        impulse3[3 * i + 2] = h[i].z;
    }
    return TR_OK;
}

int get_particles(tr_scene* s, int32_t env, double* pos, double* vel, double* angvel, double* radius, int64_t* n)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "get_particles: env");
    int64_t ne = s->envs[env].n;
    if (n) *n = ne;
    if (ne == 0) return TR_OK;
    float4* st4 = (float4*)s->staging;
    launch_gather_by_id(s->b, (int)(env * s->desc.cap_particles), (int)ne, st4, st4 + ne, st4 + 2 * ne, s->stream);
    std::vector<float4> h(3 * ne);
    HIP_CHECK(s, hipMemcpyAsync(h.data(), st4, sizeof(float4) * 3 * ne, hipMemcpyDeviceToHost, s->stream));
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    for (int64_t i = 0; i < ne; ++i) {
        const float4 &x = h[i], &v = h[ne + i], &w = h[2 * ne + i];
        if (pos) { pos[3 * i] = x.x; pos[3 * i + 1] = x.y; pos[3 * i + 2] = x.z; }
        if (radius) radius[i] = x.w;
        if (vel) { vel[3 * i] = v.x; vel[3 * i + 1] = v.y; vel[3 * i + 2] = v.z; }
        if (angvel) { angvel[3 * i] = w.x; angvel[3 * i + 1] = w.y; angvel[3 * i + 2] = w.z; }
    }
    return TR_OK;
}

int set_particles(tr_scene* s, int32_t env, const double* pos, const double* vel, const double* angvel)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "set_particles: env");
    int64_t ne = s->envs[env].n;
    if (ne == 0) return TR_OK;
    if ((pos && !finite3(pos, 3 * ne)) || (vel && !finite3(vel, 3 * ne)) || (angvel && !finite3(angvel, 3 * ne)))
        return fail(s, TR_E_NONFINITE, "set_particles: non-finite input");
    std::vector<float4> h(3 * ne, make_float4(0.f, 0.f, 0.f, 0.f));
    for (int64_t i = 0; i < ne; ++i) {
        if (pos) h[i] = make_float4((float)pos[3 * i], (float)pos[3 * i + 1], (float)pos[3 * i + 2], 0.f);
        if (vel) h[ne + i] = make_float4((float)vel[3 * i], (float)vel[3 * i + 1], (float)vel[3 * i + 2], 0.f);
        if (angvel) h[2 * ne + i] = make_float4((float)angvel[3 * i], (float)angvel[3 * i + 1], (float)angvel[3 * i + 2], 0.f);
    }
    float4* st4 = (float4*)s->staging;
    HIP_CHECK(s, hipMemcpyAsync(st4, h.data(), sizeof(float4) * 3 * ne, hipMemcpyHostToDevice, s->stream));
    int mask = (pos ? 1 : 0) | (vel ? 2 : 0) | (angvel ? 4 : 0);
    launch_scatter_by_id(s->b, (int)(env * s->desc.cap_particles), (int)ne, st4, st4 + ne, st4 + 2 * ne, mask, s->stream);
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    s->have_prev = false;
    return TR_OK;
}

int set_learn_capture(tr_scene* s, int32_t on)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (s->capture != (on != 0)) invalidate_graphs(s);
    s->capture = on != 0;
    return TR_OK;
}

int set_learned_precision(tr_scene* s, int32_t use_bf16)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (s->mlp_bf16 != (use_bf16 != 0)) invalidate_graphs(s);
    s->mlp_bf16 = use_bf16 != 0;
    return TR_OK;
}

int get_learn_samples(tr_scene* s, int32_t env, int64_t cap, float* feat, float* label, int64_t* n)
{
    if (!s || !n || cap < 0 || (cap > 0 && (!feat || !label))) return TR_E_INVAL;
    s->err.clear();
    if (env < 0 || env >= s->desc.n_envs) return fail(s, TR_E_INVAL, "get_learn_samples: env");
    *n = 0;
    if (!s->stepped) return TR_OK;
    if (!s->features_last)
        return fail(s, TR_E_STATE, "get_learn_samples: the last step wrote no features (set_learn_capture)");
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    int64_t base = (int64_t)env * s->desc.cap_particles;
    uint32_t r[2];
    HIP_CHECK(s, hipMemcpy(&r[0], s->b.pid_start + base, sizeof(uint32_t), hipMemcpyDeviceToHost));
    HIP_CHECK(s, hipMemcpy(&r[1], s->b.pid_start + base + s->desc.cap_particles, sizeof(uint32_t), hipMemcpyDeviceToHost));
    int64_t cnt = (int64_t)r[1] - (int64_t)r[0];
    *n = cnt;
    int64_t m = std::min(cnt, cap);
    int64_t done = 0;
    // through the staging buffer (12 floats per particle) in chunks
    int64_t chunk = std::max<int64_t>(1, (12 * s->z.P) / 15);
    while (done < m) {
        int64_t k = std::min(chunk, m - done);
        float* df = s->staging;
        float* dl = s->staging + 12 * k;
        launch_learn_samples(s->b, (int64_t)r[0] + done, k, df, dl, s->stream);
        HIP_CHECK(s, hipMemcpyAsync(feat + 12 * done, df, sizeof(float) * 12 * k, hipMemcpyDeviceToHost, s->stream));
        HIP_CHECK(s, hipMemcpyAsync(label + 3 * done, dl, sizeof(float) * 3 * k, hipMemcpyDeviceToHost, s->stream));
        HIP_CHECK(s, hipStreamSynchronize(s->stream));
        done += k;
    }
    return TR_OK;
}

int mlp_forward(const float* weights, const float* feat, int64_t B, float* out, int32_t use_bf16, void* stream)
{
    if (!weights || (B > 0 && (!feat || !out)) || B < 0) return TR_E_INVAL;
    launch_mlp_infer(weights, feat, out, nullptr, B, use_bf16 != 0, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? TR_OK : TR_E_DEVICE;
}

int64_t mlp_grad_scratch_floats(int64_t B) { return B > 0 ? mlp_grad_scratch(B) : 0; }

int mlp_loss_grad(const float* weights, const float* feat, const float* label, int64_t B, float* grad, float* loss,
                  float* scratch, int64_t scratch_floats, void* stream)
{
    if (!weights || !feat || !label || !grad || !scratch || B <= 0) return TR_E_INVAL;
    if (scratch_floats < mlp_grad_scratch(B)) return TR_E_CAPACITY;
    launch_mlp_grad(weights, feat, label, B, grad, loss, scratch, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? TR_OK : TR_E_DEVICE;
}

int mlp_adam_step(float* weights, const float* grad, float* m, float* v, float lr, float beta1, float beta2, float eps,
                  int32_t t, void* stream)
{
    if (!weights || !grad || !m || !v || t < 1 || !(lr > 0.0f)) return TR_E_INVAL;
    launch_adam(weights, grad, m, v, mlp_trainable(), lr, beta1, beta2, eps, t, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? TR_OK : TR_E_DEVICE;
}

int set_mlp_weights(tr_scene* s, const float* weights, int64_t n)
{
    if (!s || !weights) return TR_E_INVAL;
    s->err.clear();
    if (n != kMlpParams) return fail(s, TR_E_INVAL, "set_mlp_weights: wrong parameter count");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(weights[i])) return fail(s, TR_E_NONFINITE, "set_mlp_weights: non-finite weight");
    HIP_CHECK(s, hipMemcpyAsync(s->b.mlp, weights, sizeof(float) * n, hipMemcpyHostToDevice, s->stream));
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    if (!s->mlp_loaded) invalidate_graphs(s);
    s->mlp_loaded = true;
    return TR_OK;
}

int set_warm_start(tr_scene* s, int32_t mode)
{
    if (!s) return TR_E_INVAL;
    s->err.clear();
    if (mode < TR_WARM_COLD || mode > TR_WARM_LEARNED) return fail(s, TR_E_INVAL, "set_warm_start: mode");
    if (s->p.warm != mode) invalidate_graphs(s);
    s->p.warm = mode;
    s->desc.warm_start = mode;
    return TR_OK;
}

}  // extern "C"

namespace {
// Snapshot layout: header, then the arrays that persist across steps, each
// as raw bytes in this order.
struct StateHeader {
    char magic[8];         // "TRSTATE2"
    int32_t n_envs;
    int32_t n_bodies;
    int64_t cap_particles;
    int64_t cap_contacts;
    int64_t n_total;
    int64_t n_cache;       // previous-step contacts
    int32_t have_prev;
    int32_t stepped;
};

struct Span {
    void* dev;
    size_t bytes;
};

// the device arrays of the state, in snapshot order (n_cache known)
std::vector<Span> state_spans(tr_scene* s, int64_t n_cache)
{
    const int64_t n = s->n_total;
    return {{s->b.xr, sizeof(float4) * n},
            {s->b.vw, sizeof(float4) * 2 * n},
            {s->b.pid, sizeof(int) * n},
            {s->b.rho, sizeof(float) * n},
            {s->b.id2slot, sizeof(int) * s->z.NID},
            {s->b.pid_start, sizeof(uint32_t) * (s->z.NID + 1)},
            {s->b.pkeyc, sizeof(unsigned long long) * n_cache},
            {s->b.plam, sizeof(float4) * n_cache},
            {s->b.plamr, s->desc.material.mu_r > 0.0 ? sizeof(float4) * n_cache : 0},
            {s->b.bodies, sizeof(BodyDev) * s->body_host.size()}};
}

int64_t state_bytes(tr_scene* s, int64_t n_cache)
{
    int64_t t = sizeof(StateHeader) + sizeof(int64_t) * s->desc.n_envs;
    for (const Span& sp : state_spans(s, n_cache)) t += (int64_t)sp.bytes;
    return t;
}
}  // namespace

extern "C" {

int save_state(tr_scene* s, void* buf, int64_t cap, int64_t* size)
{
    if (!s || !size || cap < 0 || (cap > 0 && !buf)) return TR_E_INVAL;
    s->err.clear();
    if (s->tables_dirty) {
        int rc = rebuild_tables(s);
        if (rc) return rc;
    }
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    uint32_t n_cache = 0;
    if (s->have_prev)
        HIP_CHECK(s, hipMemcpy(&n_cache, s->b.pid_start + s->z.NID, sizeof(uint32_t), hipMemcpyDeviceToHost));
    *size = state_bytes(s, n_cache);
    if (!buf) return TR_OK;
    if (cap < *size) return fail(s, TR_E_CAPACITY, "save_state: buffer too small");
    char* o = (char*)buf;
    StateHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, "TRSTATE2", 8);
    h.n_envs = s->desc.n_envs;
    h.n_bodies = (int32_t)s->body_host.size();
    h.cap_particles = s->desc.cap_particles;
    h.cap_contacts = s->desc.cap_contacts;
    h.n_total = s->n_total;
    h.n_cache = n_cache;
    h.have_prev = s->have_prev ? 1 : 0;
    h.stepped = s->stepped ? 1 : 0;
    memcpy(o, &h, sizeof(h));
    o += sizeof(h);
    for (int e = 0; e < s->desc.n_envs; ++e, o += sizeof(int64_t)) memcpy(o, &s->envs[e].n, sizeof(int64_t));
    for (const Span& sp : state_spans(s, n_cache)) {
        if (sp.bytes) HIP_CHECK(s, hipMemcpy(o, sp.dev, sp.bytes, hipMemcpyDeviceToHost));
        o += sp.bytes;
    }
    return TR_OK;
}

int load_state(tr_scene* s, const void* buf, int64_t size)
{
    if (!s || !buf || size < (int64_t)sizeof(StateHeader)) return TR_E_INVAL;
    s->err.clear();
    StateHeader h;
    memcpy(&h, buf, sizeof(h));
    if (memcmp(h.magic, "TRSTATE2", 8) != 0) return fail(s, TR_E_INVAL, "load_state: not a state snapshot");
    if (s->tables_dirty) {
        int rc = rebuild_tables(s);
        if (rc) return rc;
    }
    const char* o = (const char*)buf + sizeof(h);
    bool same = h.n_envs == s->desc.n_envs && h.n_bodies == (int32_t)s->body_host.size() &&
                h.cap_particles == s->desc.cap_particles && h.cap_contacts == s->desc.cap_contacts &&
                h.n_total == s->n_total && h.n_cache >= 0 && h.n_cache <= s->z.C &&
                size == state_bytes(s, h.n_cache);
    for (int e = 0; same && e < s->desc.n_envs; ++e) {
        int64_t n;
        memcpy(&n, o + sizeof(int64_t) * e, sizeof(n));
        same = n == s->envs[e].n;
    }
    if (!same) return fail(s, TR_E_STATE, "load_state: snapshot of a scene with other envs, bodies or capacities");
    o += sizeof(int64_t) * s->desc.n_envs;
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    for (const Span& sp : state_spans(s, h.n_cache)) {
        if (sp.bytes) HIP_CHECK(s, hipMemcpy(sp.dev, o, sp.bytes, hipMemcpyHostToDevice));
        o += sp.bytes;
    }
    // the host copy of the body table follows the restored poses
    HIP_CHECK(s, hipMemcpy(s->body_host.data(), s->b.bodies, sizeof(BodyDev) * s->body_host.size(), hipMemcpyDeviceToHost));
    s->have_prev = h.have_prev != 0;
    s->stepped = h.stepped != 0;
    s->features_last = false;  // the snapshot holds no features
    s->slots_env_major = false;  // the snapshot's slot order is not recorded; the next step restores it
    return TR_OK;
}

}  // extern "C"

namespace {
// autotuner cache: one JSON object per line, keyed by the device architecture
// and the scene's size bucket (log2 of envs and of spheres)
struct TuneKey {
    std::string arch;
    int envs_log2;
    int particles_log2;
};

TuneKey tune_key(tr_scene* s)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t pr;
    (void)hipGetDeviceProperties(&pr, dev);
    TuneKey k;
    k.arch = pr.gcnArchName;
    for (char& ch : k.arch)
        if (ch == '"' || ch == '\\' || ch == '\n') ch = '_';
    k.envs_log2 = ceil_log2(std::max(1, s->desc.n_envs));
    k.particles_log2 = ceil_log2((int)std::max<int64_t>(1, s->n_total));
    return k;
}

bool tune_lookup(const char* path, const TuneKey& k, tr_solver_config* cfg)
{
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char arch[128];
        int el, pl;
        tr_solver_config c;
        double ms;
        if (sscanf(line,
                   "{\"arch\": \"%127[^\"]\", \"envs_log2\": %d, \"particles_log2\": %d, \"mode\": %d, "
                   "\"blocks_per_xcd\": %d, \"lds_particles\": %d, \"cluster_particles\": %d, \"dataflow\": %d, "
                   "\"step_ms\": %lf}",
                   arch, &el, &pl, &c.mode, &c.blocks_per_xcd, &c.lds_particles, &c.cluster_particles, &c.dataflow,
                   &ms) == 9 &&
            k.arch == arch && el == k.envs_log2 && pl == k.particles_log2) {
            *cfg = c;  // the last entry for the key wins
            found = true;
        }
    }
    fclose(f);
    return found;
}

void tune_store(const char* path, const TuneKey& k, const tr_solver_config& c, double ms)
{
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f,
            "{\"arch\": \"%s\", \"envs_log2\": %d, \"particles_log2\": %d, \"mode\": %d, \"blocks_per_xcd\": %d, "
            "\"lds_particles\": %d, \"cluster_particles\": %d, \"dataflow\": %d, \"step_ms\": %.4f}\n",
            k.arch.c_str(), k.envs_log2, k.particles_log2, c.mode, c.blocks_per_xcd, c.lds_particles,
            c.cluster_particles, c.dataflow, ms);
    fclose(f);
}
}  // namespace

extern "C" {

int autotune(tr_scene* s, int32_t steps, const char* cache_path, tr_solver_config* chosen, float* best_ms)
{
    if (!s || steps < 1) return TR_E_INVAL;
    s->err.clear();
    if (s->tables_dirty) {
        int rc = rebuild_tables(s);
        if (rc) return rc;
    }
    const TuneKey key = tune_key(s);
    tr_solver_config c;
    if (cache_path && tune_lookup(cache_path, key, &c)) {
        int rc = set_solver_config(s, &c);
        if (rc) return rc;
        if (chosen) *chosen = s->cfg;
        if (best_ms) *best_ms = -1.f;
        return TR_OK;
    }
    // every candidate steps from the same state (restored after each)
    int64_t size = 0;
    int rc = save_state(s, nullptr, 0, &size);
    if (rc) return rc;
    std::vector<char> snap((size_t)size);
    rc = save_state(s, snap.data(), size, &size);
    if (rc) return rc;
    const tr_solver_config base = s->cfg;
    const bool graphs = s->use_graphs;
    s->use_graphs = false;
    std::vector<tr_solver_config> cands;
    // grouped mode shares the stopping test of a group's envs: not offered when
    // that would change results (a residual tolerance with more than 8 envs)
    if (!(s->desc.tol > 0.0 && s->desc.n_envs > kGroups))
        for (int bpx : {64, 32, 16, 8}) cands.push_back({TR_PGS_GROUPED, bpx, s->max_lds_particles, 0, 0});
    if (s->desc.n_envs == 1) cands.push_back({TR_PGS_SPREAD, 32, s->max_lds_particles, 0, 0});
    for (int cp : {0, 8192, 16384, (int)TR_CLUSTER_NONE}) cands.push_back({TR_PGS_PER_ENV, 32, s->max_lds_particles, cp, 0});
    cands.push_back({TR_PGS_PER_ENV, 32, 0, 0, 0});
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_CHECK(s, hipEventCreate(&e0));
    HIP_CHECK(s, hipEventCreate(&e1));
    int best = -1;
    float best_t = 0.f;
    for (size_t i = 0; i < cands.size(); ++i) {
        if (set_solver_config(s, &cands[i]) != TR_OK || load_state(s, snap.data(), size) != TR_OK) continue;
        if (step_scene(s, 1, nullptr) != TR_OK) continue;  // warm-up
        (void)hipEventRecord(e0, s->stream);
        if (step_scene(s, steps, nullptr) != TR_OK) continue;
        (void)hipEventRecord(e1, s->stream);
        std::vector<tr_step_stats> st(s->desc.n_envs);
        if (step_scene(s, 1, st.data()) != TR_OK) continue;  // synchronises; fails on a capacity or barrier failure
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) continue;
        ms /= (float)steps;
        if (best < 0 || ms < best_t) { best = (int)i; best_t = ms; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    s->err.clear();
    tr_solver_config pick = best >= 0 ? cands[best] : base;
    rc = set_solver_config(s, &pick);
    if (rc == TR_OK) rc = load_state(s, snap.data(), size);
    s->use_graphs = graphs;
    if (rc) return rc;
    if (best < 0) return fail(s, TR_E_STATE, "autotune: no candidate schedule completed");
    if (cache_path) tune_store(cache_path, key, s->cfg, best_t);
    if (chosen) *chosen = s->cfg;
    if (best_ms) *best_ms = best_t;
    return TR_OK;
}

int get_phase_times(tr_scene* s, float* ms, int32_t cap)
{
    if (!s || !ms || cap < 0) return TR_E_INVAL;
    s->err.clear();
    if (!s->stepped) return fail(s, TR_E_STATE, "get_phase_times: no step yet");
    HIP_CHECK(s, hipStreamSynchronize(s->stream));
    float t[5];
    for (int k = 0; k < 4; ++k) {
        t[k] = std::numeric_limits<float>::quiet_NaN();
        if (!s->last_replay) HIP_CHECK(s, hipEventElapsedTime(&t[k], s->ev[k], s->ev[k + 1]));
    }
    HIP_CHECK(s, hipEventElapsedTime(&t[4], s->ev[0], s->ev[4]));
    for (int k = 0; k < cap && k < 5; ++k) ms[k] = t[k];
    return TR_OK;
}

}  // extern "C"
