// Host runtime behind the C ABI in include/snake.h: descriptor validation,
// workspace layout, parameter upload, tile packing, graph capture and the
// state/index copies.  All device work is in step.hip and index.hip.
#include "snake.h"

#include <cmath>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "carriage.h"
#include "kernels.h"
#include "snake_mlp.h"

using namespace snake;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(SIM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

struct Sizes {
    int64_t n = 0, N = 0, J = 0, Mt = 0, blocks = 0, pieces = 0;
    int max_B = 0, min_B = 1 << 30;
    bool autotune = false;
    bool mlp = false;
    bool newton = false;
    bool gs = false;
    bool wheels = false;
};

// Carves 256-byte aligned sub-arrays out of the workspace (base == nullptr
// only measures).
struct Carver {
    char* base;
    size_t pos = 0;
    template <class T>
    T* take(int64_t count)
    {
        pos = (pos + 255) & ~(size_t)255;
        T* p = base ? reinterpret_cast<T*>(base + pos) : nullptr;
        pos += (size_t)(count > 0 ? count : 1) * sizeof(T);
        return p;
    }
};

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate(const sim_desc_t* d, Sizes* z)
{
    if (!d) return fail(SIM_EINVAL, "descriptor is NULL");
    if (d->n_snakes < 1) return fail(SIM_EINVAL, "n_snakes must be >= 1");
    if (!d->n_modules || !d->segs_per_module || !d->alpha_stretch || !d->alpha_bend ||
        !d->alpha_twist || !d->mu)
        return fail(SIM_EINVAL, "per-snake array is NULL");
    if (!finite_pos(d->seg_mass) || !finite_pos(d->seg_length) || !finite_pos(d->seg_radius))
        return fail(SIM_EINVAL, "segment mass, length and radius must be finite and > 0");
    if (!std::isfinite(d->gravity)) return fail(SIM_EINVAL, "gravity must be finite");
    if (!finite_pos(d->dt)) return fail(SIM_EINVAL, "dt must be finite and > 0");
    if (d->substeps < 1) return fail(SIM_EINVAL, "substeps must be >= 1");
    if (d->iters < 0 || d->iters > 1000000) return fail(SIM_EINVAL, "iters must be in [0, 1e6]");
    if (!std::isfinite(d->tol)) return fail(SIM_EINVAL, "tol must be finite");
    if (!(d->relax > 0.0 && d->relax <= 1.0)) return fail(SIM_EINVAL, "relax must be in (0, 1]");
    if (d->pressure_law != SIM_LAW_LAG && d->pressure_law != SIM_LAW_PAPER)
        return fail(SIM_EINVAL, "unknown pressure law");
    if (d->pressure_law == SIM_LAW_LAG && (!finite_pos(d->tau_inflate) || !finite_pos(d->tau_deflate)))
        return fail(SIM_EINVAL, "tau_inflate and tau_deflate must be > 0");
    if (d->pressure_law == SIM_LAW_PAPER &&
        (!finite_pos(d->p_source) || !finite_pos(d->amplitude_psi) || !(d->k_inflate > 0.0) ||
         !(d->k_deflate > 0.0) || !(d->T_p >= 0.0)))
        return fail(SIM_EINVAL, "paper pressure-law constants out of range");
    if (!std::isfinite(d->kappa_max)) return fail(SIM_EINVAL, "kappa_max must be finite");
    if (d->warm_start != SIM_WARM_ZERO && d->warm_start != SIM_WARM_PREV && d->warm_start != SIM_WARM_MLP)
        return fail(SIM_EINVAL, "unknown warm start");
    if (d->flags & ~(SIM_FLAG_FIXED_ROOT | SIM_FLAG_NO_GROUND | SIM_FLAG_WHEELS))
        return fail(SIM_EINVAL, "unknown flag bits");
    if (d->controller < SIM_CTRL_EXTERNAL || d->controller > SIM_CTRL_SCHEDULE)
        return fail(SIM_EINVAL, "unknown controller");
    const bool ground = !(d->flags & SIM_FLAG_NO_GROUND);
    z->n = d->n_snakes;
    for (int s = 0; s < d->n_snakes; ++s) {
        const int M = d->n_modules[s], S = d->segs_per_module[s];
        if (M < 1 || S < 1) return fail(SIM_EINVAL, "n_modules and segs_per_module must be >= 1");
        const int64_t B = (int64_t)M * S;
        if (B > 1024) return fail(SIM_EINVAL, "snakes longer than 1024 bodies are not supported");
        const double a[4] = {d->alpha_stretch[s], d->alpha_bend[s], d->alpha_twist[s], d->mu[s]};
        for (double v : a)
            if (!std::isfinite(v) || v < 0.0) return fail(SIM_EINVAL, "compliance and mu must be finite and >= 0");
        z->N += B;
        z->J += B - 1;
        z->Mt += M;
        z->blocks += 2 * (B - 1) + (ground ? B : 0);
        if (B > z->max_B) z->max_B = (int)B;
        if (B < z->min_B) z->min_B = (int)B;
    }
    if (z->N > (int64_t)1 << 28) return fail(SIM_EINVAL, "too many bodies (limit 2^28)");
    const int mw = d->map_waves;
    if (mw != 0 && mw != 1 && mw != 2 && mw != 4 && mw != 8 && mw != 16)
        return fail(SIM_EINVAL, "map_waves must be 0, 1, 2, 4, 8 or 16");
    if (d->map_min_seg != 0 && d->map_min_seg != 16 && d->map_min_seg != 32 && d->map_min_seg != 64)
        return fail(SIM_EINVAL, "map_min_seg must be 0, 16, 32 or 64");
    if (d->map_grid < 0) return fail(SIM_EINVAL, "map_grid must be >= 0");
    if (d->map_rows < 0 || d->map_rows > 2) return fail(SIM_EINVAL, "map_rows must be 0, 1 or 2");
    if (d->mlp_fallback_k < 0 || d->mlp_fallback_k > d->iters)
        return fail(SIM_EINVAL, "mlp_fallback_k must be in [0, iters]");
    if (d->solver != SIM_SOLVER_JACOBI && d->solver != SIM_SOLVER_NEWTON && d->solver != SIM_SOLVER_GS)
        return fail(SIM_EINVAL, "unknown solver");
    if (d->solver == SIM_SOLVER_GS && d->warm_start != SIM_WARM_ZERO)
        return fail(SIM_EINVAL, "the Gauss-Seidel solver starts from zero multipliers");
    z->gs = d->solver == SIM_SOLVER_GS;
    if (d->solver == SIM_SOLVER_NEWTON) {
        if (d->warm_start != SIM_WARM_ZERO && d->warm_start != SIM_WARM_PREV)
            return fail(SIM_EINVAL, "the Newton solver starts from zero or the previous multipliers");
        if (d->newton_iters < 0 || d->newton_iters > 10000)
            return fail(SIM_EINVAL, "newton_iters must be in [0, 10000]");
        if (d->pcr_iters < 1 || d->pcr_iters > 100000) return fail(SIM_EINVAL, "pcr_iters must be in [1, 100000]");
        if (d->newton_keep_best != 0 && d->newton_keep_best != 1)
            return fail(SIM_EINVAL, "newton_keep_best must be 0 or 1");
    }
    z->newton = d->solver == SIM_SOLVER_NEWTON;
    z->wheels = (d->flags & SIM_FLAG_WHEELS) != 0;
    if (z->wheels && (d->solver != SIM_SOLVER_JACOBI || d->warm_start != SIM_WARM_ZERO))
        return fail(SIM_EINVAL, "the wheel carriage takes the Jacobi solver from zero multipliers");
    // the carriage kernels index wheel multipliers as int: component c < 9
    // of wheel w < 2N sits at c * 2N + w, so 18 N must stay below 2^31
    if (z->wheels && z->N > ((int64_t)1 << 31) / 18 - 1)
        return fail(SIM_EINVAL, "too many bodies for a wheel carriage (limit 2^31 / 18)");
    if (mw != 0 && !d->autotune) {
        int seg = 16;
        while (seg < z->max_B) seg <<= 1;
        if (seg > 64 * mw) return fail(SIM_EINVAL, "map_waves too small for the longest snake");
    }
    z->autotune = d->autotune != 0;
    z->mlp = d->warm_start == SIM_WARM_MLP;
    if (d->controller == SIM_CTRL_SERPENOID && (!d->ctrl_freq || !d->ctrl_phase0))
        return fail(SIM_EINVAL, "serpenoid controller needs ctrl_freq and ctrl_phase0");
    if (d->controller == SIM_CTRL_SCHEDULE) {
        if (!d->sched_off || !d->sched_steps || !d->sched_val)
            return fail(SIM_EINVAL, "schedule controller needs sched_off, sched_steps, sched_val");
        if (d->sched_off[0] != 0) return fail(SIM_EINVAL, "sched_off[0] must be 0");
        for (int64_t m = 0; m < z->Mt; ++m) {
            if (d->sched_off[m + 1] <= d->sched_off[m]) return fail(SIM_EINVAL, "every module needs >= 1 piece");
            int64_t len = 0;
            for (int k = d->sched_off[m]; k < d->sched_off[m + 1]; ++k) {
                if (d->sched_steps[k] < 1) return fail(SIM_EINVAL, "piece lengths must be >= 1");
                if (!std::isfinite(d->sched_val[k])) return fail(SIM_EINVAL, "piece value not finite");
                len += d->sched_steps[k];
            }
            if (len > INT32_MAX) return fail(SIM_EINVAL, "schedule too long");
        }
        z->pieces = d->sched_off[z->Mt];
    }
    return SIM_OK;
}

struct Views {
    KParams kp;
    IParams ip;
    int4* hdr;
    int2* slots;
    char* state_begin;      // the mutable state is one contiguous range
    size_t state_bytes;
    char* backup;           // copy of the state while autotuning
    NParams np;
    WParams wp;
    int* newton_list;       // [n] snakes by lane class (Newton and Gauss-Seidel solvers)
    double* comp_d;         // [4][n] compliances / h^2 and mu in double
    float* mlp_y;           // [2J][3] network outputs
    float* mlp_params;      // [6467]
    float* mlp_ms;          // [64]
    int* Bn;
    int* Mn;
    int* Sn;
    float* comp;
    float* mu;
    double* freq;
    double* phase0;
    int* sched_off;
    int* sched_start;
    float* sched_val;
};

size_t carve(const Sizes& z, char* base, Views* v)
{
    Carver c{base};
    const int64_t n = z.n, N = z.N, J = z.J, Mt = z.Mt;
    KParams& k = v->kp;
    IParams& ip = v->ip;
    k.x = c.take<float>(3 * N);
    k.q = c.take<float>(4 * N);
    k.v = c.take<float>(3 * N);
    k.w = c.take<float>(3 * N);
    k.p = c.take<float>(2 * Mt);
    k.cmd = c.take<float>(Mt);
    k.lam_j = c.take<float>(6 * J);
    k.lam_c = c.take<float>(3 * N);
    k.residual = c.take<float>(n);
    k.iters_out = c.take<int>(n);
    k.status = c.take<int>(n);
    k.step = c.take<long long>(n);
    k.iters_total = c.take<long long>(n);
    WParams& wp = v->wp;
    wp.x = z.wheels ? c.take<float>(6 * N) : nullptr;
    wp.q = z.wheels ? c.take<float>(8 * N) : nullptr;
    wp.v = z.wheels ? c.take<float>(6 * N) : nullptr;
    wp.w = z.wheels ? c.take<float>(6 * N) : nullptr;
    wp.lam = z.wheels ? c.take<float>(18 * N) : nullptr;
    v->state_begin = reinterpret_cast<char*>(k.x);
    v->state_bytes = c.pos;
    v->Bn = c.take<int>(n);
    v->Mn = c.take<int>(n);
    v->Sn = c.take<int>(n);
    v->comp = c.take<float>(3 * n);
    v->mu = c.take<float>(n);
    v->freq = c.take<double>(n);
    v->phase0 = c.take<double>(n);
    v->sched_off = c.take<int>(Mt + 1);
    v->sched_start = c.take<int>(z.pieces);
    v->sched_val = c.take<float>(z.pieces);
    ip.body_off = c.take<int>(n + 1);
    ip.joint_off = c.take<int>(n + 1);
    ip.module_off = c.take<int>(n + 1);
    ip.block_off = c.take<int>(n + 1);
    ip.blk_type = c.take<int>(z.blocks);
    ip.blk_a = c.take<int>(z.blocks);
    ip.blk_b = c.take<int>(z.blocks);
    ip.blk_color = c.take<int>(z.blocks);
    ip.degree = c.take<int>(N);
    ip.bucket = c.take<int>(n);
    ip.order = c.take<int>(n);
    ip.color_scratch = c.take<int>(N);
    k.q_pred = c.take<float>(4 * N);
    k.probe = z.mlp ? c.take<float>(16 * N) : nullptr;
    v->mlp_y = z.mlp ? c.take<float>(6 * J) : nullptr;
    v->mlp_params = z.mlp ? c.take<float>(8192) : nullptr;
    v->mlp_ms = z.mlp ? c.take<float>(64) : nullptr;
    v->newton_list = (z.newton || z.gs || z.wheels) ? c.take<int>(n) : nullptr;
    v->comp_d = (z.newton || z.wheels) ? c.take<double>(4 * n) : nullptr;
    v->hdr = c.take<int4>(n + 1);
    v->slots = c.take<int2>(n + 1);
    v->backup = z.autotune ? c.take<char>((int64_t)v->state_bytes) : nullptr;
    return c.pos + 256;
}

int pow2_at_least(int b, int lo)
{
    int p = lo;
    while (p < b) p <<= 1;
    return p;
}

struct Mapping {
    int nw = 1, min_seg = 16, grid = 0, rows = 0;
};

// Pack snakes, in work order (longest first), into tiles of 64*nw lanes.
// Aligned layout: each snake gets max(min_seg, 2^ceil(log2 B)) lanes;
// segments arrive in non-increasing size, so placing them one after another
// keeps every segment aligned to its own size.  Rows layout: each snake gets
// B rounded up to 16 lanes (rows = 2: snakes of up to 8 bodies 8 lanes, two
// to a row), placed one after another.
// Tile header: first slot, slot count, some segment crosses a wave
// boundary, rows layout.  Slot: snake, lane offset << 16 | lanes.
void build_tiles(const std::vector<int>& order, const std::vector<int>& Bn, const Mapping& mp,
                 std::vector<int4>& hdr, std::vector<int2>& slots)
{
    hdr.clear();
    slots.clear();
    const int cap = 64 * mp.nw;
    if (!mp.rows) {
        int pos = cap;
        for (int sidx : order) {
            const int seg = pow2_at_least(Bn[sidx], mp.min_seg);
            if (pos + seg > cap) {
                hdr.push_back(make_int4((int)slots.size(), 0, 0, 0));
                pos = 0;
            }
            slots.push_back(make_int2(sidx, (pos << 16) | seg));
            int4& h = hdr.back();
            h.y += 1;
            if (seg > 64) h.z = 1;
            pos += seg;
        }
        return;
    }
    // Rows layout: best fit in decreasing size.  Each segment goes to the
    // open tile with the least free room that still holds it (a new tile
    // if none does); tiles keep the order in which they were opened, so the
    // longest snakes come first.  Open tiles are bucketed by free rows.
    // With half rows (rows = 2) snakes of up to 8 bodies take 8 lanes, two
    // consecutive ones (in work order) sharing a row.
    struct Item {
        int need, s0, n0, s1;   // rows, first snake and its lanes, partner (-1: none)
    };
    std::vector<Item> items;
    for (int sidx : order) {
        if (mp.rows == 2 && Bn[sidx] <= 8) {
            if (!items.empty() && items.back().n0 == 8 && items.back().s1 < 0) {
                items.back().s1 = sidx;
                continue;
            }
            items.push_back(Item{1, sidx, 8, -1});
            continue;
        }
        const int need = (Bn[sidx] + 15) / 16;
        items.push_back(Item{need, sidx, 16 * need, -1});
    }
    const int nrow = cap / 16;
    std::vector<std::vector<int>> item_of_tile;
    std::vector<int> fill;
    std::vector<std::vector<int>> free_rows(nrow + 1);   // tiles by free rows
    std::vector<int> at(items.size());
    for (size_t k = 0; k < items.size(); ++k) {
        const int need = items[k].need;
        int t = -1;
        for (int r = need; r <= nrow && t < 0; ++r)
            if (!free_rows[r].empty()) {
                t = free_rows[r].back();
                free_rows[r].pop_back();
            }
        if (t < 0) {
            t = (int)fill.size();
            fill.push_back(0);
            item_of_tile.emplace_back();
        }
        item_of_tile[t].push_back((int)k);
        at[k] = fill[t];
        fill[t] += need;
        free_rows[nrow - fill[t]].push_back(t);
    }
    for (size_t t = 0; t < fill.size(); ++t) {
        int4 h = make_int4((int)slots.size(), 0, 0, mp.rows);
        for (int k : item_of_tile[t]) {
            const Item& it = items[k];
            const int pos = 16 * at[k];
            slots.push_back(make_int2(it.s0, (pos << 16) | it.n0));
            h.y += 1;
            if ((pos >> 6) != ((pos + it.n0 - 1) >> 6)) h.z = 1;
            if (it.s1 >= 0) {
                slots.push_back(make_int2(it.s1, ((pos + 8) << 16) | 8));
                h.y += 1;
            }
        }
        hdr.push_back(h);
    }
}

std::mutex g_tune_mu;
std::map<std::string, Mapping> g_tune_cache;

}  // namespace

struct sim {
    Sizes z;
    Views v;
    bool mlp_loaded = false;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    Mapping map;
    int n_tiles = 0;
    bool use_graph = false;
    std::map<int, hipGraphExec_t> graphs;
    std::vector<int> order_host;
    std::vector<int> B_host;
    int newton_off[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // lane classes 8 << c
};

namespace {

int upload_tiles(sim* s, const Mapping& mp)
{
    std::vector<int4> hdr;
    std::vector<int2> slots;
    build_tiles(s->order_host, s->B_host, mp, hdr, slots);
    hipError_t e = hipMemcpy(s->v.hdr, hdr.data(), hdr.size() * sizeof(int4), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(s->v.slots, slots.data(), slots.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "upload tiles");
    s->map = mp;
    s->n_tiles = (int)hdr.size();
    return SIM_OK;
}

int tiles(sim* s, hipStream_t st, int n_steps, int phase, int sub)
{
    hipError_t e = launch_tiles(s->map.nw, s->map.rows, s->v.kp, s->v.hdr, s->v.slots, s->n_tiles, s->map.grid,
                                n_steps, phase, sub, st);
    if (e != hipSuccess) return hip_fail(e, "step launch");
    return SIM_OK;
}

// One substep split in two launches around the network: prediction, the
// network's inputs and outputs, then the warm-started solve.  With feat /
// tgt given (recording) the inputs go there and the final multipliers are
// written as targets.
int split_substep(sim* s, hipStream_t st, int sub, float* feat, float* tgt)
{
    const KParams& k = s->v.kp;
    int rc = tiles(s, st, 1, kPhasePre, sub);
    if (rc) return rc;
    if (feat) {
        // recording: the inputs go to the caller's rows, the network reads them there
        hipError_t e = launch_features(k, feat, st);
        if (e != hipSuccess) return hip_fail(e, "features");
        if (s->z.mlp) {
            rc = mlp_forward(s->v.mlp_params, s->v.mlp_ms, feat, s->v.mlp_y, 2 * (int64_t)s->z.J, st);
            if (rc) return fail(rc, std::string("network: ") + mlp_last_error());
        }
    } else if (s->z.mlp) {
        hipError_t e = launch_warm_net(k, s->v.mlp_params, s->v.mlp_ms, s->v.mlp_y, st);
        if (e != hipSuccess) return hip_fail(e, "network");
    }
    rc = tiles(s, st, 1, kPhaseSolve, sub);
    if (rc) return rc;
    if (tgt) {
        hipError_t e = launch_targets(k, tgt, st);
        if (e != hipSuccess) return hip_fail(e, "targets");
    }
    return SIM_OK;
}

int launch_steps(sim* s, hipStream_t st, int n_steps)
{
    if (s->z.wheels) {
        hipError_t e = launch_carriage(s->v.kp, s->v.np, s->v.wp, s->v.newton_list, s->newton_off, n_steps, st);
        if (e != hipSuccess) return hip_fail(e, "carriage step launch");
        return SIM_OK;
    }
    if (s->z.newton) {
        hipError_t e = launch_newton(s->v.kp, s->v.np, s->v.newton_list, s->newton_off, n_steps, st);
        if (e != hipSuccess) return hip_fail(e, "Newton step launch");
        return SIM_OK;
    }
    if (s->z.gs) {
        hipError_t e = launch_gs(s->v.kp, s->v.ip.block_off, s->v.ip.blk_color, s->v.newton_list, s->newton_off,
                                 n_steps, st);
        if (e != hipSuccess) return hip_fail(e, "Gauss-Seidel step launch");
        return SIM_OK;
    }
    if (!s->z.mlp) return tiles(s, st, n_steps, kPhaseFull, 0);
    for (int k = 0; k < n_steps; ++k)
        for (int sub = 0; sub < s->v.kp.substeps; ++sub) {
            int rc = split_substep(s, st, sub, nullptr, nullptr);
            if (rc) return rc;
        }
    return SIM_OK;
}

// Time every candidate mapping for a few steps on the real batch and keep
// the fastest.  The state is saved first and restored after each trial.
int autotune(sim* s)
{
    const int max_seg = pow2_at_least(s->z.max_B, 16);
    const int nw_min = max_seg > 64 ? max_seg / 64 : 1;
    int cus = 256;
    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            cus = prop.multiProcessorCount;
        }
    }
    std::string key = std::to_string(cus) + ":" + std::to_string(s->z.n) + ":" +
                      std::to_string(s->z.N) + ":" + std::to_string(s->z.max_B) + ":" +
                      std::to_string(s->v.kp.iters) + ":" + std::to_string(s->v.kp.tol > 0.f);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) return upload_tiles(s, it->second);
    }
    int min_pow2 = 1 << 30;
    for (int b : s->B_host) min_pow2 = std::min(min_pow2, pow2_at_least(b, 16));
    std::vector<Mapping> cand;
    for (int nw = nw_min; nw <= 16 && nw <= 4 * nw_min; nw <<= 1)
        for (int ms : {16, 32, 64, 0}) {
            if (ms != 16 && ms != 0 && ms <= min_pow2) continue;   // same packing as 16
            Mapping m;
            m.nw = nw;
            m.min_seg = ms ? ms : 16;
            m.rows = ms == 0;   // rows layout
            cand.push_back(m);
            // persistent variant: one resident wave set per SIMD slot
            Mapping p = m;
            p.grid = cus * (16 / nw > 0 ? 16 / nw : 1);
            cand.push_back(p);
            if (ms == 0 && s->z.min_B <= 8) {
                // half rows for the snakes of up to 8 bodies
                Mapping hr = m, hp = p;
                hr.rows = hp.rows = 2;
                cand.push_back(hr);
                cand.push_back(hp);
            }
        }
    hipError_t e = hipMemcpyAsync(s->v.backup, s->v.state_begin, s->v.state_bytes,
                                  hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return hip_fail(e, "autotune backup");
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
        return hip_fail(e, "autotune events");
    Mapping best;
    float best_ms = 1e30f;
    int rc = SIM_OK;
    for (const Mapping& m : cand) {
        rc = upload_tiles(s, m);
        if (rc) break;
        if (m.grid >= s->n_tiles && m.grid != 0) continue;
        rc = launch_steps(s, s->stream, 1);   // warm-up
        if (rc) break;
        (void)hipEventRecord(e0, s->stream);
        rc = launch_steps(s, s->stream, 1);
        if (rc == SIM_OK) rc = launch_steps(s, s->stream, 1);
        (void)hipEventRecord(e1, s->stream);
        if (rc) break;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) {
            rc = hip_fail(e, "autotune timing");
            break;
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) {
            best_ms = ms;
            best = m;
        }
        e = hipMemcpyAsync(s->v.state_begin, s->v.backup, s->v.state_bytes, hipMemcpyDeviceToDevice,
                           s->stream);
        if (e != hipSuccess) {
            rc = hip_fail(e, "autotune restore");
            break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    e = hipMemcpyAsync(s->v.state_begin, s->v.backup, s->v.state_bytes, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "autotune restore");
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
    }
    return upload_tiles(s, best);
}

}  // namespace

extern "C" {

const char* sim_last_error(void) { return g_err.c_str(); }

int sim_workspace_bytes(const sim_desc_t* d, size_t* bytes)
{
    if (!bytes) return fail(SIM_EINVAL, "bytes is NULL");
    Sizes z;
    int rc = validate(d, &z);
    if (rc) return rc;
    Views v;
    *bytes = carve(z, nullptr, &v);
    return SIM_OK;
}

int sim_create(const sim_desc_t* d, void* workspace, size_t bytes, void* hip_stream, sim_t** out)
{
    if (!out) return fail(SIM_EINVAL, "out is NULL");
    *out = nullptr;
    Sizes z;
    int rc = validate(d, &z);
    if (rc) return rc;
    if (!workspace) return fail(SIM_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(SIM_EINVAL, "workspace must be 256-byte aligned");
    Views v;
    const size_t need = carve(z, nullptr, &v);
    if (bytes < need)
        return fail(SIM_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes, got " +
                                    std::to_string(bytes));
    sim* s = new sim();
    s->z = z;
    s->stream = reinterpret_cast<hipStream_t>(hip_stream);
    carve(z, reinterpret_cast<char*>(workspace), &s->v);
    Views& w = s->v;
    const int n = (int)z.n;
    const bool ground = !(d->flags & SIM_FLAG_NO_GROUND);
    const double h = d->dt / d->substeps;

    // host copies of the per-snake parameters
    std::vector<int> Bn(n), Mn(n), Sn(n);
    std::vector<float> comp(3 * (size_t)n), mu(n);
    std::vector<double> freq(n, 0.0), ph(n, 0.0);
    for (int k = 0; k < n; ++k) {
        Mn[k] = d->n_modules[k];
        Sn[k] = d->segs_per_module[k];
        Bn[k] = Mn[k] * Sn[k];
        comp[k] = (float)(d->alpha_stretch[k] * d->seg_length / (h * h));
        comp[n + k] = (float)(d->alpha_bend[k] * d->seg_length / (h * h));
        comp[2 * (size_t)n + k] = (float)(d->alpha_twist[k] * d->seg_length / (h * h));
        mu[k] = (float)d->mu[k];
        if (d->controller == SIM_CTRL_SERPENOID) {
            freq[k] = d->ctrl_freq[k];
            ph[k] = d->ctrl_phase0[k];
        }
    }
    std::vector<int> soff(z.Mt + 1, 0), sstart(z.pieces > 0 ? z.pieces : 1, 0);
    std::vector<float> sval(z.pieces > 0 ? z.pieces : 1, 0.f);
    if (d->controller == SIM_CTRL_SCHEDULE) {
        for (int64_t m = 0; m <= z.Mt; ++m) soff[m] = d->sched_off[m];
        for (int64_t m = 0; m < z.Mt; ++m) {
            int start = 0;
            for (int k = soff[m]; k < soff[m + 1]; ++k) {
                sstart[k] = start;
                sval[k] = (float)d->sched_val[k];
                start += d->sched_steps[k];
            }
        }
    }

    KParams& k = w.kp;
    k.n_snakes = n;
    k.N = (int)z.N;
    k.J = (int)z.J;
    k.Mt = (int)z.Mt;
    k.Bn = w.Bn;
    k.Mn = w.Mn;
    k.Sn = w.Sn;
    k.body_off = w.ip.body_off;
    k.joint_off = w.ip.joint_off;
    k.module_off = w.ip.module_off;
    k.mlp_y = w.mlp_y;
    k.fallback = d->mlp_fallback ? 1 : 0;
    k.fallback_k = d->mlp_fallback_k;
    k.comp = w.comp;
    k.mu = w.mu;
    k.freq = w.freq;
    k.phase0 = w.phase0;
    k.sched_off = w.sched_off;
    k.sched_start = w.sched_start;
    k.sched_val = w.sched_val;
    const double m = d->seg_mass, L = d->seg_length, R = d->seg_radius;
    const double I_ax = 0.5 * m * R * R, I_pe = m * (3.0 * R * R + L * L) / 12.0;
    k.h = (float)h;
    k.inv_h = (float)(1.0 / h);
    k.inv_m = (float)(1.0 / m);
    k.L = (float)L;
    k.half_L = (float)(0.5 * L);
    k.inv_L = (float)(1.0 / L);
    k.R = (float)R;
    k.g = (float)d->gravity;
    k.c1 = (float)(1.0 / I_pe);
    k.c2 = (float)(1.0 / I_ax - 1.0 / I_pe);
    k.I_ax = (float)I_ax;
    k.I_pe = (float)I_pe;
    k.tol = (float)d->tol;
    k.relax = (float)d->relax;
    k.iters = d->iters;
    k.substeps = d->substeps;
    k.lag_in = d->pressure_law == SIM_LAW_LAG ? (float)std::exp(-h / d->tau_inflate) : 0.f;
    k.lag_de = d->pressure_law == SIM_LAW_LAG ? (float)std::exp(-h / d->tau_deflate) : 0.f;
    k.law = d->pressure_law;
    k.k_i = (float)d->k_inflate;
    k.k_d = (float)d->k_deflate;
    k.T_p = (float)d->T_p;
    k.p_s = (float)d->p_source;
    k.amp = (float)(d->pressure_law == SIM_LAW_PAPER ? d->amplitude_psi : 1.0);
    k.kappa_max = (float)d->kappa_max;
    k.controller = d->controller;
    k.dt = d->dt;
    k.ctrl_alpha = d->ctrl_alpha;
    k.ctrl_offset = d->ctrl_offset;
    k.flags = (int)d->flags;
    k.warm = d->warm_start;
    k.lam_ref = (float)(m * 9.81 * h * h);
    NParams& np = w.np;
    np.comp = w.comp_d;
    np.mu = w.comp_d ? w.comp_d + 3 * (size_t)n : nullptr;
    np.h = h;
    np.m = m;
    np.L = L;
    np.R = R;
    np.g = d->gravity;
    np.I_ax = I_ax;
    np.I_pe = I_pe;
    np.tol = d->tol;
    np.lag_in = d->pressure_law == SIM_LAW_LAG ? std::exp(-h / d->tau_inflate) : 0.0;
    np.lag_de = d->pressure_law == SIM_LAW_LAG ? std::exp(-h / d->tau_deflate) : 0.0;
    np.amp = d->pressure_law == SIM_LAW_PAPER ? d->amplitude_psi : 1.0;
    np.p_s = d->p_source;
    np.k_i = d->k_inflate;
    np.k_d = d->k_deflate;
    np.T_p = d->T_p;
    np.kappa_max = d->kappa_max;
    np.newton_iters = d->newton_iters;
    np.keep_best = d->newton_keep_best;
    np.pcr_iters = d->pcr_iters;
    // wheels: thin discs of radius R/2 and mass m/8 centred at (0, +-R, -R/2)
    // in their segment's frame, axle along the segment's y axis
    WParams& wp = w.wp;
    wp.mw = m / 8.0;
    wp.rw = 0.5 * R;
    wp.dw = R;
    wp.hw = 0.5 * R;
    wp.Ip = 0.25 * wp.mw * wp.rw * wp.rw;
    wp.Ia = 0.5 * wp.mw * wp.rw * wp.rw;
    wp.relax = d->relax;

    IParams& ip = w.ip;
    ip.n_snakes = n;
    ip.N = (int)z.N;
    ip.n_blocks = (int)z.blocks;
    ip.ground = ground ? 1 : 0;
    ip.Bn = w.Bn;
    ip.Mn = w.Mn;

    hipError_t e;
    hipStream_t st = s->stream;
#define CK(expr, what)                      \
    do {                                    \
        e = (expr);                         \
        if (e != hipSuccess) {              \
            rc = hip_fail(e, what);         \
            goto error;                     \
        }                                   \
    } while (0)
    CK(hipMemcpyAsync(w.Bn, Bn.data(), n * sizeof(int), hipMemcpyHostToDevice, st), "upload B");
    CK(hipMemcpyAsync(w.Mn, Mn.data(), n * sizeof(int), hipMemcpyHostToDevice, st), "upload M");
    CK(hipMemcpyAsync(w.Sn, Sn.data(), n * sizeof(int), hipMemcpyHostToDevice, st), "upload S");
    CK(hipMemcpyAsync(w.comp, comp.data(), comp.size() * sizeof(float), hipMemcpyHostToDevice, st), "upload compliance");
    CK(hipMemcpyAsync(w.mu, mu.data(), n * sizeof(float), hipMemcpyHostToDevice, st), "upload mu");
    CK(hipMemcpyAsync(w.freq, freq.data(), n * sizeof(double), hipMemcpyHostToDevice, st), "upload freq");
    CK(hipMemcpyAsync(w.phase0, ph.data(), n * sizeof(double), hipMemcpyHostToDevice, st), "upload phase");
    CK(hipMemcpyAsync(w.sched_off, soff.data(), soff.size() * sizeof(int), hipMemcpyHostToDevice, st), "upload schedule");
    CK(hipMemcpyAsync(w.sched_start, sstart.data(), sstart.size() * sizeof(int), hipMemcpyHostToDevice, st), "upload schedule");
    CK(hipMemcpyAsync(w.sched_val, sval.data(), sval.size() * sizeof(float), hipMemcpyHostToDevice, st), "upload schedule");
    if (z.newton || z.gs || z.wheels) {
        // snakes grouped by lane class (power of two >= B, at least 8)
        std::vector<double> cd(4 * (size_t)n);
        std::vector<int> cls(n), list;
        for (int q = 0; q < n; ++q) {
            cd[q] = d->alpha_stretch[q] * d->seg_length / (h * h);
            cd[n + q] = d->alpha_bend[q] * d->seg_length / (h * h);
            cd[2 * (size_t)n + q] = d->alpha_twist[q] * d->seg_length / (h * h);
            cd[3 * (size_t)n + q] = d->mu[q];
            int c = 0;
            while ((8 << c) < Bn[q]) ++c;
            cls[q] = c;
        }
        for (int c = 0; c < 8; ++c) {
            s->newton_off[c] = (int)list.size();
            for (int q = 0; q < n; ++q)
                if (cls[q] == c) list.push_back(q);
        }
        s->newton_off[8] = (int)list.size();
        if (z.newton || z.wheels)
            CK(hipMemcpyAsync(w.comp_d, cd.data(), cd.size() * sizeof(double), hipMemcpyHostToDevice, st),
               "upload compliance");
        CK(hipMemcpyAsync(w.newton_list, list.data(), n * sizeof(int), hipMemcpyHostToDevice, st),
           "upload snake classes");
    }
    if (z.mlp) {
        CK(hipMemsetAsync(w.mlp_params, 0, 8192 * sizeof(float), st), "zero network");
        CK(hipMemsetAsync(w.mlp_ms, 0, 32 * sizeof(float), st), "zero network");
        std::vector<float> ones(32, 1.f);
        CK(hipMemcpyAsync(w.mlp_ms + 32, ones.data(), 32 * sizeof(float), hipMemcpyHostToDevice, st), "zero network");
        CK(hipStreamSynchronize(st), "zero network");
    }
    CK(launch_index(ip, st), "index kernels");
    CK(hipStreamSynchronize(st), "index work");
    {
        // tiles: snakes in work order (longest first), packed into segments
        std::vector<int> order(n);
        CK(hipMemcpy(order.data(), ip.order, n * sizeof(int), hipMemcpyDeviceToHost), "read order");
        s->order_host = order;
        s->B_host = Bn;
    }
    CK(launch_init_state(k, st), "init state");
    if (z.wheels) CK(launch_init_wheels(k, w.wp, st), "init wheels");
    CK(hipStreamSynchronize(st), "init state");
    if (z.autotune && !z.newton && !z.gs && !z.wheels) {
        rc = autotune(s);
        if (rc) goto error;
    } else {
        Mapping mp;
        const int max_seg = pow2_at_least(z.max_B, 16);
        mp.nw = d->map_waves ? d->map_waves : (max_seg > 64 ? max_seg / 64 : 1);
        mp.min_seg = d->map_min_seg ? d->map_min_seg : 16;
        mp.grid = d->map_grid;
        mp.rows = d->map_rows;
        rc = upload_tiles(s, mp);
        if (rc) goto error;
    }
    CK(hipStreamSynchronize(st), "create");
    s->use_graph = d->use_graph != 0;
    if (s->use_graph) CK(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking), "capture stream");
#undef CK
    *out = s;
    return SIM_OK;
error:
    delete s;
    return rc;
}

int sim_step(sim_t* s, int32_t n_steps)
{
    if (!s) return fail(SIM_EINVAL, "sim is NULL");
    if (s->z.mlp && !s->mlp_loaded) return fail(SIM_ESTATE, "learned warm start needs sim_set_mlp first");
    if (n_steps < 0) return fail(SIM_EINVAL, "n_steps must be >= 0");
    if (n_steps == 0) return SIM_OK;
    if (!s->use_graph) {
        for (int k = 0; k < n_steps; ++k) {
            int rc = launch_steps(s, s->stream, 1);
            if (rc) return rc;
        }
        return SIM_OK;
    }
    auto it = s->graphs.find(n_steps);
    if (it == s->graphs.end()) {
        // a few step counts are kept; a new one beyond that replaces them
        if (s->graphs.size() >= 8) {
            (void)hipStreamSynchronize(s->stream);
            for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
            s->graphs.clear();
        }
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "begin capture");
        int rc = SIM_OK;
        for (int k = 0; k < n_steps && rc == SIM_OK; ++k) rc = launch_steps(s, s->cap_stream, 1);
        e = hipStreamEndCapture(s->cap_stream, &graph);
        if (rc || e != hipSuccess) {
            if (e == hipSuccess && graph) (void)hipGraphDestroy(graph);
            return rc ? rc : hip_fail(e, "end capture");
        }
        hipGraphExec_t exec;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(e, "instantiate graph");
        it = s->graphs.emplace(n_steps, exec).first;
    }
    hipError_t e = hipGraphLaunch(it->second, s->stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return SIM_OK;
}

int sim_set_pressures(sim_t* s, const float* cmd, int64_t n, int mem)
{
    if (!s || !cmd) return fail(SIM_EINVAL, "sim or cmd is NULL");
    if (n != s->z.Mt) return fail(SIM_EINVAL, "expected one command per module (" + std::to_string(s->z.Mt) + ")");
    hipError_t e;
    if (mem == SIM_MEM_HOST) {
        std::vector<float> c(cmd, cmd + n);
        for (auto& a : c) {
            if (std::isnan(a)) return fail(SIM_EINVAL, "command is NaN");
            a = std::fmin(1.f, std::fmax(-1.f, a));
        }
        e = hipMemcpyAsync(s->v.kp.cmd, c.data(), n * sizeof(float), hipMemcpyHostToDevice, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    } else if (mem == SIM_MEM_DEVICE) {
        e = launch_set_cmd(s->v.kp.cmd, cmd, (int)n, s->stream);
    } else {
        return fail(SIM_EINVAL, "unknown memory kind");
    }
    if (e != hipSuccess) return hip_fail(e, "set pressures");
    return SIM_OK;
}

static void field_table(sim* s, void* ptr[SIM_F_COUNT], size_t bytes[SIM_F_COUNT])
{
    const KParams& k = s->v.kp;
    const size_t N = s->z.N, J = s->z.J, Mt = s->z.Mt, n = s->z.n;
    const WParams& wp = s->v.wp;
    void* p[SIM_F_COUNT] = {k.x, k.q, k.v, k.w, k.p, k.lam_j, k.lam_c, k.cmd, k.residual,
                            k.iters_out, k.status, k.step, k.iters_total, wp.x, wp.q, wp.v, wp.w, wp.lam};
    size_t b[SIM_F_COUNT] = {3 * N * 4, 4 * N * 4, 3 * N * 4, 3 * N * 4, 2 * Mt * 4, 6 * J * 4,
                             3 * N * 4, Mt * 4, n * 4, n * 4, n * 4, n * 8, n * 8,
                             6 * N * 4, 8 * N * 4, 6 * N * 4, 6 * N * 4, 18 * N * 4};
    for (int f = 0; f < SIM_F_COUNT; ++f) {
        ptr[f] = p[f];
        bytes[f] = b[f];
    }
}

static int copy_fields(sim_t* s, uint32_t fields, void* const* user, int mem, bool to_user)
{
    if (!s || !user) return fail(SIM_EINVAL, "sim or pointer array is NULL");
    if (fields & ~((1u << SIM_F_COUNT) - 1)) return fail(SIM_EINVAL, "unknown field bits");
    if (mem != SIM_MEM_HOST && mem != SIM_MEM_DEVICE) return fail(SIM_EINVAL, "unknown memory kind");
    void* ptr[SIM_F_COUNT];
    size_t bytes[SIM_F_COUNT];
    field_table(s, ptr, bytes);
    for (int f = 0; f < SIM_F_COUNT; ++f) {
        if (!(fields & (1u << f))) continue;
        if (!user[f]) return fail(SIM_EINVAL, "pointer for a selected field is NULL");
        if (!ptr[f]) return fail(SIM_EINVAL, "wheel fields need a batch with SIM_FLAG_WHEELS");
        hipMemcpyKind kind = mem == SIM_MEM_HOST ? (to_user ? hipMemcpyDeviceToHost : hipMemcpyHostToDevice)
                                                 : hipMemcpyDeviceToDevice;
        hipError_t e = to_user ? hipMemcpyAsync(user[f], ptr[f], bytes[f], kind, s->stream)
                               : hipMemcpyAsync(ptr[f], user[f], bytes[f], kind, s->stream);
        if (e != hipSuccess) return hip_fail(e, "state copy");
    }
    if (mem == SIM_MEM_HOST) {
        hipError_t e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_fail(e, "state copy");
    }
    return SIM_OK;
}

int sim_read_state(sim_t* s, uint32_t fields, void* const* dst, int mem)
{
    return copy_fields(s, fields, dst, mem, true);
}

int sim_write_state(sim_t* s, uint32_t fields, const void* const* src, int mem)
{
    return copy_fields(s, fields, const_cast<void* const*>(src), mem, false);
}

int sim_set_mlp(sim_t* s, const float* params, const float* mean_std, int mem)
{
    if (!s || !params || !mean_std) return fail(SIM_EINVAL, "sim, params or mean_std is NULL");
    if (!s->z.mlp) return fail(SIM_ESTATE, "the descriptor's warm start is not SIM_WARM_MLP");
    if (mem != SIM_MEM_HOST && mem != SIM_MEM_DEVICE) return fail(SIM_EINVAL, "unknown memory kind");
    const hipMemcpyKind kind = mem == SIM_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    hipError_t e = hipMemcpyAsync(s->v.mlp_params, params, mlp_param_count() * sizeof(float), kind, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s->v.mlp_ms, mean_std, 64 * sizeof(float), kind, s->stream);
    if (e == hipSuccess && mem == SIM_MEM_HOST) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "set network");
    s->mlp_loaded = true;
    return SIM_OK;
}

int sim_step_record(sim_t* s, int32_t n_steps, float* features, float* targets, int64_t capacity_rows,
                    int64_t* written)
{
    if (!s || !features || !targets) return fail(SIM_EINVAL, "sim, features or targets is NULL");
    if (n_steps < 0) return fail(SIM_EINVAL, "n_steps must be >= 0");
    if (s->z.mlp && !s->mlp_loaded) return fail(SIM_ESTATE, "learned warm start needs sim_set_mlp first");
    if (s->z.newton || s->z.gs || s->z.wheels)
        return fail(SIM_EINVAL, "recording needs the Jacobi solver on the plain chain");
    const int64_t per_sub = 2 * s->z.J;
    const int64_t rows = per_sub * s->v.kp.substeps * (int64_t)n_steps;
    if (written) *written = rows;
    if (capacity_rows < rows)
        return fail(SIM_ENOMEM, "record buffers hold " + std::to_string(capacity_rows) + " rows, need " +
                                    std::to_string(rows));
    int64_t row = 0;
    for (int k = 0; k < n_steps; ++k)
        for (int sub = 0; sub < s->v.kp.substeps; ++sub) {
            int rc = split_substep(s, s->stream, sub, features + 32 * row, targets + 3 * row);
            if (rc) return rc;
            row += per_sub;
        }
    return SIM_OK;
}

int sim_read_index(sim_t* s, int32_t which, int32_t* dst, int64_t count)
{
    if (!s || !dst) return fail(SIM_EINVAL, "sim or dst is NULL");
    const IParams& ip = s->v.ip;
    const int64_t n = s->z.n, nb = s->z.blocks, N = s->z.N;
    const int* src[SIM_IDX_COUNT] = {ip.body_off, ip.joint_off, ip.module_off, ip.block_off, ip.blk_type,
                                     ip.blk_a, ip.blk_b, ip.blk_color, ip.degree, ip.bucket, ip.order};
    const int64_t len[SIM_IDX_COUNT] = {n + 1, n + 1, n + 1, n + 1, nb, nb, nb, nb, N, n, n};
    if (which < 0 || which >= SIM_IDX_COUNT) return fail(SIM_EINVAL, "unknown index array");
    if (count != len[which]) return fail(SIM_EINVAL, "count does not match the index array's length");
    hipError_t e = hipMemcpyAsync(dst, src[which], count * sizeof(int32_t), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "read index");
    return SIM_OK;
}

int sim_sizes(const sim_t* s, int64_t* out5)
{
    if (!s || !out5) return fail(SIM_EINVAL, "sim or out is NULL");
    out5[0] = s->z.n;
    out5[1] = s->z.N;
    out5[2] = s->z.J;
    out5[3] = s->z.Mt;
    out5[4] = s->z.blocks;
    return SIM_OK;
}

int sim_plan_tiles(const sim_desc_t* d, int32_t waves, int32_t min_seg, int32_t rows, int32_t* hdr,
                   int32_t* slots, int64_t* n_tiles)
{
    if (!hdr || !slots || !n_tiles) return fail(SIM_EINVAL, "output is NULL");
    Sizes z;
    int rc = validate(d, &z);
    if (rc) return rc;
    if (waves != 1 && waves != 2 && waves != 4 && waves != 8 && waves != 16)
        return fail(SIM_EINVAL, "waves must be 1, 2, 4, 8 or 16");
    if (min_seg != 16 && min_seg != 32 && min_seg != 64) return fail(SIM_EINVAL, "min_seg must be 16, 32 or 64");
    if (rows < 0 || rows > 2) return fail(SIM_EINVAL, "rows must be 0, 1 or 2");
    const int n = (int)z.n;
    std::vector<int> Bn(n), order(n);
    for (int k = 0; k < n; ++k) {
        Bn[k] = d->n_modules[k] * d->segs_per_module[k];
        order[k] = k;
    }
    if (pow2_at_least((int)z.max_B, 16) > 64 * waves) return fail(SIM_EINVAL, "waves too few for the longest snake");
    // work order: longest first, ties by snake index
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return Bn[a] > Bn[b]; });
    Mapping mp;
    mp.nw = waves;
    mp.min_seg = min_seg;
    mp.rows = rows;
    std::vector<int4> h;
    std::vector<int2> sl;
    build_tiles(order, Bn, mp, h, sl);
    for (size_t t = 0; t < h.size(); ++t) {
        hdr[4 * t] = h[t].x;
        hdr[4 * t + 1] = h[t].y;
        hdr[4 * t + 2] = h[t].z;
        hdr[4 * t + 3] = h[t].w;
    }
    for (size_t k = 0; k < sl.size(); ++k) {
        slots[2 * k] = sl[k].x;
        slots[2 * k + 1] = sl[k].y;
    }
    *n_tiles = (int64_t)h.size();
    return SIM_OK;
}

int sim_mapping(const sim_t* s, int32_t* out5)
{
    if (!s || !out5) return fail(SIM_EINVAL, "sim or out is NULL");
    out5[0] = s->map.nw;
    out5[1] = s->map.min_seg;
    out5[2] = s->map.grid;
    out5[3] = s->n_tiles;
    out5[4] = s->map.rows;
    return SIM_OK;
}

void sim_destroy(sim_t* s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    delete s;
}

}  // extern "C"
