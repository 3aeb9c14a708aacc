// C-ABI implementation of the MI355X solid lattice-Boltzmann library.
// Host orchestration of the HIP kernels in slbm_kernels.h: problem validation
// and upload, the pseudo-time loops with device-side convergence flags, the
// objective and the gradient assembly per control kind.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <deque>
#include <mutex>
#include <vector>

#include "solid_lbm.h"
#include "slbm_kernels.h"

using namespace slbm;

namespace {

thread_local std::string g_init_error;

}  // namespace

// Device time of the fused launches of a solve loop: one pair of HIP events on
// the context's stream around each run of back-to-back fused launches (the
// launches between two residual checks); pairs are harvested once the host
// has seen them complete and their events are reused.
struct LaunchTimer {
    struct Run {
        hipEvent_t a, b;
        int64_t start, launches, sweeps;                 // first step of the run, its launches and sweeps
        double ms;
    };
    bool on = false;
    std::vector<hipEvent_t> pool;                        // free events
    std::deque<Run> pending;                             // recorded, not yet read
    std::vector<Run> runs;                               // read
    hipEvent_t open = nullptr;                           // start of the run being recorded
    int64_t run_start = 0, run_launches = 0, run_sweeps = 0;
    int64_t launches = 0, sweeps = 0;                    // fused launches and the sweeps they made
    double ms = 0.0;                                     // device time of the completed runs
    hipError_t take(hipEvent_t* e)
    {
        if (!pool.empty()) {
            *e = pool.back();
            pool.pop_back();
            return hipSuccess;
        }
        return hipEventCreate(e);
    }
    void reset()
    {
        launches = sweeps = 0;
        ms = 0.0;
        runs.clear();
    }
    // before a fused launch of `k` sweeps, starting at step `step`, on `stream`
    hipError_t before(hipStream_t stream, int k, int64_t step)
    {
        if (!on) return hipSuccess;
        ++launches;
        sweeps += k;
        ++run_launches;
        run_sweeps += k;
        if (open) return hipSuccess;
        run_start = step;
        hipError_t e = take(&open);
        return e != hipSuccess ? e : hipEventRecord(open, stream);
    }
    // after the last fused launch of a run
    hipError_t close(hipStream_t stream)
    {
        if (!on || !open) return hipSuccess;
        hipEvent_t end;
        hipError_t e = take(&end);
        if (e == hipSuccess) e = hipEventRecord(end, stream);
        if (e != hipSuccess) return e;
        pending.push_back(Run{open, end, run_start, run_launches, run_sweeps, 0.0});
        open = nullptr;
        run_launches = run_sweeps = 0;
        return hipSuccess;
    }
    // accumulates the runs that have completed (wait: block until all have)
    hipError_t harvest(bool wait)
    {
        while (!pending.empty()) {
            Run r = pending.front();
            if (wait) {
                hipError_t e = hipEventSynchronize(r.b);
                if (e != hipSuccess) return e;
            } else if (hipEventQuery(r.b) != hipSuccess) {
                break;
            }
            float f = 0.f;
            hipError_t e = hipEventElapsedTime(&f, r.a, r.b);
            if (e != hipSuccess) return e;
            r.ms = f;
            ms += f;
            runs.push_back(r);
            pool.push_back(r.a);
            pool.push_back(r.b);
            pending.pop_front();
        }
        return hipSuccess;
    }
    // keeps the runs that start at or before step t: the loop learns of a
    // stop one check late, and the launches it issued after the stop return
    // at once (call after harvest(true))
    void trim(int64_t t)
    {
        launches = sweeps = 0;
        ms = 0.0;
        for (const Run& r : runs)
            if (r.start <= t) {
                launches += r.launches;
                sweeps += r.sweeps;
                ms += r.ms;
            }
    }
    void destroy()
    {
        for (auto& r : pending) {
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
        if (open) pool.push_back(open);
        open = nullptr;
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        pool.clear();
    }
};

struct slbm_ctx {
    // problem
    int nx = 0, ny = 0;
    int64_t N = 0;
    double dx = 0, dx2 = 0, E = 0, nu = 0, tol = 0, inv_nx = 0;
    int64_t max_steps = 0;
    int64_t K = 0;
    int cv_window = 0;  // > 0: coefficient-of-variation convergence test over that many checks
    int kind = 0, nmodes = 0, project = 0, normalize = 1;
    bool masked = false;
    int nb = 0;  // boundary records
    double cbar = 1.0;
    hipStream_t stream = nullptr;
    // device buffers
    double* fbuf[2] = {nullptr, nullptr};
    double* abuf[2] = {nullptr, nullptr};
    double *g = nullptr, *Efield = nullptr, *target = nullptr, *snap = nullptr, *dbar = nullptr,
           *r = nullptr, *fbar = nullptr, *dJdF = nullptr, *dJdE = nullptr, *adisp = nullptr,
           *modes = nullptr, *fixedF = nullptr, *work = nullptr, *partial = nullptr, *scal = nullptr,
           *ctrl = nullptr,
           *asrc = nullptr;  // adjoint source field (2 planes): the objective's r, or a VJP cotangent
    uint8_t* obs = nullptr;
    int32_t* code = nullptr;
    BNode* bnodes = nullptr;
    Status* status = nullptr;
    Status* h_status = nullptr;  // pinned, 2 slots
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t t0 = nullptr, t1 = nullptr;
    int tb_T = -1;     // steps fused per launch (0/1: single-step sweeps; -1: automatic)
    int tb_H = 0;      // rows per wave of the fused sweeps (0: automatic)
    int tile_w = 0, tile_h = 0;  // tile of the LDS-tiled fused sweeps (0: automatic)
    int simds = 1024;            // SIMDs of the device (4 per compute unit)
    // tangent (forward-mode) solves: allocated at the first tangent_solve
    double *tv[2] = {nullptr, nullptr}, *td[2] = {nullptr, nullptr}, *gdot = nullptr, *Edot = nullptr,
           *snapd = nullptr, *tpart = nullptr, *tdir = nullptr;
    slbm_progress_fn progress = nullptr;  // optional report from the solve loops
    void* progress_user = nullptr;
    double progress_every = 0.0;          // seconds between reports
    bool tile_attr = false;      // LDS limits of the plate tile kernels raised
    // launch plan of the current tile shape (k_tile_plan), for launches whose
    // tiles all fit the compute units: capacity of one tile per compute unit
    int4* plan = nullptr;
    int32_t* plan_rec = nullptr;
    int32_t* plan_nst = nullptr;
    int64_t plan_cap = 0;        // tiles
    int plan_key[4] = {0, 0, 0, 0};   // tw, th, halo, order of the plan held (tw = 0: none)
    int64_t nblk = 0;  // blocks of one sweep
    int64_t pcap = 0;  // capacity of the partial-sum buffer in blocks
    // state
    int prim_cur = 0;       // buffer holding f^C(t-1) of the current primal state
    bool prim_valid = false;
    bool prim_done = false; // a completed primal_solve (adjoint inputs ready)
    int adj_cur = 0;
    bool adj_done = false;
    bool adj_valid = false;   // the adjoint buffers hold a defined state
    bool efield_on = false; // E_NODAL: kernels read the E plane
    double E_cur = 0;       // uniform E of the current control
    double alpha_sq = 0;    // E_SCALAR_SQ control value
    double J = 0;
    LaunchTimer lt;         // optional device time of the fused launches (solid_lbm_set_launch_timing)
    std::string err;
    std::vector<void*> allocs;
};

namespace {

int fail(slbm_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    else g_init_error = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, SLBM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int dalloc(slbm_ctx* c, void** p, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, SLBM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    c->allocs.push_back(*p);
    return SLBM_OK;
}

// eq. gamma divides by tau_s - tau_f, tau_s = 2K/(1+theta) = 3E/(4(1-nu))
bool gamma_ok(double E, double nu) { return std::fabs(0.75 * E / (1.0 - nu) - kTauF) > 1e-12; }

inline unsigned grid_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

bool finite_all(const double* a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

int fill(slbm_ctx* c, double* a, int64_t n, double v)
{
    hipLaunchKernelGGL(k_fill, dim3(grid_of(n)), dim3(kBlock), 0, c->stream, a, n, v);
    HIPCHK(c, hipGetLastError());
    return SLBM_OK;
}

// Relaxation keep-factors of a uniform material on the host.
Relax<double> host_relax(double E, double nu) { return relax_from_E<double>(E, nu, false); }

SweepArgs base_args(slbm_ctx* c)
{
    SweepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.code = c->code;
    a.bnodes = c->bnodes;
    a.snap = c->snap;
    a.partial = c->partial;
    a.status = c->status;
    a.nx = c->nx;
    a.ny = c->ny;
    a.N = c->N;
    Relax<double> r = host_relax(c->E_cur, c->nu);
    a.k11 = r.k11;
    a.ks = r.ks;
    a.kd = r.kd;
    a.E0 = c->E_cur;
    a.nu = c->nu;
    a.E = c->efield_on ? c->Efield : nullptr;
    return a;
}

void launch_sweep(slbm_ctx* c, bool adjoint, const SweepArgs& a, bool check)
{
    int sel = (c->masked ? 4 : 0) | (c->efield_on ? 2 : 0) | (check ? 1 : 0);
    dim3 grid(grid_of(c->N)), block(kBlock);
    double inv = c->inv_nx;
#define SL_CASE(i, M, EF, CH)                                                                        \
    case i:                                                                                          \
        if (adjoint) hipLaunchKernelGGL((k_adjoint<M, EF, CH>), grid, block, 0, c->stream, a, inv);  \
        else hipLaunchKernelGGL((k_primal<M, EF, CH>), grid, block, 0, c->stream, a, inv);           \
        break;
    switch (sel) {
        SL_CASE(0, false, false, false)
        SL_CASE(1, false, false, true)
        SL_CASE(2, false, true, false)
        SL_CASE(3, false, true, true)
        SL_CASE(4, true, false, false)
        SL_CASE(5, true, false, true)
        SL_CASE(6, true, true, false)
        SL_CASE(7, true, true, true)
    }
#undef SL_CASE
}

// (step, input buffer) of the latest check sweeps of a solve.  The host sees
// a passing test at most one or two checks after it happened (it reads the
// device status one chunk behind), so the passing check is among the last
// few; older entries are dropped, which keeps the record from growing with
// the length of the run.
struct CheckLog {
    static constexpr size_t kKeep = 16;
    std::deque<std::pair<int64_t, int>> q;
    void add(int64_t s, int buf)
    {
        q.emplace_back(s, buf);
        if (q.size() > kKeep) q.pop_front();
    }
    int find(int64_t s) const
    {
        for (const auto& e : q)
            if (e.first == s) return e.second;
        return -1;
    }
};

// Steps fused per launch for this context (1 = single-step sweeps only): the
// fused kernels cover the periodic, uniform-material bulk.
// The LDS-tiled kernel serves plates and E fields always, periodic uniform
// problems when a tile shape was set, and, with automatic tuning, periodic
// uniform grids up to 131072 nodes (measured on MI355X: 128^2 1.3 vs 3.5 us
// per step, 256^2 1.7 vs 3.9 for the best wave-strip shape; from 512^2 on the
// wave strips are faster).
constexpr int64_t kTileAutoMaxNodes = 131072;
bool use_tiles(const slbm_ctx* c)
{
    return c->masked || c->efield_on || c->tile_w > 0 || (c->tb_T < 0 && c->N <= kTileAutoMaxNodes);
}

int fused_steps(const slbm_ctx* c)
{
    if (use_tiles(c)) return 1;
    int T = c->tb_T;
    if (T < 0) T = 8;
    if (T != 2 && T != 4 && T != 6 && T != 8) return 1;
    return T;
}

// Automatic rows per wave: a strip launch runs one wave per (strip, row
// block) and each wave carries a whole pipeline, so the time of a launch is
// that of the slowest SIMD; the best shapes measured on MI355X keep the wave
// count just at or below the SIMD count (1024^2, T = 8: 24 rows, 946 waves;
// 2048^2: 96 rows, 946 waves).  Smallest multiple of 4 in [8, 96] that does;
// grids too small to fill the chip get the 8-row floor (512^2, T = 8: 8 rows,
// 704 waves, 3.02 us per step against 3.37 with 12 rows, autotuner timing).
int fused_rows(const slbm_ctx* c, int T)
{
    if (c->tb_H > 0) return std::min(c->tb_H, c->ny);
    const int strips = (c->nx + (64 - 2 * T) - 1) / (64 - 2 * T);
    const int blocks = std::max(1, c->simds / strips);
    int H = (c->ny + blocks - 1) / blocks;
    H = std::min(96, std::max(8, (H + 3) / 4 * 4));
    return std::min(H, c->ny);
}

void launch_fused(slbm_ctx* c, bool adjoint, const SweepArgs& s, int T)
{
    TBArgs a;
    a.src = s.src;
    a.dst = s.dst;
    a.g = s.g;
    a.status = c->status;
    a.nx = c->nx;
    a.ny = c->ny;
    a.N = c->N;
    a.k11 = s.k11;
    a.ks = s.ks;
    a.kd = s.kd;
    a.scale = s.scale;
    a.H = fused_rows(c, T);
    int V = 64 - 2 * T;
    a.strips = (c->nx + V - 1) / V;
    dim3 grid((unsigned)(a.strips * ((c->ny + a.H - 1) / a.H))), block(64);
#define TB_CASE(TT)                                                                                   \
    case TT:                                                                                          \
        if (adjoint) hipLaunchKernelGGL((k_sweep_tb<TT, true>), grid, block, 0, c->stream, a);        \
        else hipLaunchKernelGGL((k_sweep_tb<TT, false>), grid, block, 0, c->stream, a);               \
        break;
    switch (T) {
        TB_CASE(2)
        TB_CASE(4)
        TB_CASE(6)
        TB_CASE(8)
    }
#undef TB_CASE
}

// Sweeps fused per launch by the LDS-tiled kernel (plates and E fields; 1 =
// single-step sweeps only).  Any count 1..halo works, so runs shorter than
// the halo between residual checks are fused too.
// Automatic: 8 steps per launch (32 x 32 regions, 16 x 16 tiles) up to ~128k
// nodes; beyond, the most steps of 6, 5, 4, 3 whose (32 - 2h)^2 tiles all
// fit the compute units at once (one workgroup each), else 6 with 20 x 20
// tiles -- a workgroup's fixed cost (loads, relaxation rates, stores) is
// several steps' worth, so one round of workgroups beats more steps in two
// (measured on MI355X: the 512 x 308 plate 5.0 us per primal step with 6
// steps in 416 tiles, 4.3 with 3 steps in 240; 384 x 231 keeps 6 steps in
// 240 tiles, 3.0 us).
int tile_halo(const slbm_ctx* c)
{
    if (c->tb_T >= 0) return std::max(1, std::min(c->tb_T, 8));
    if (c->N <= 131072) return 8;
    const int64_t cus = c->simds / 4;
    for (int h : {6, 5, 4, 3}) {
        const int t = 32 - 2 * h;
        if ((int64_t)((c->nx + t - 1) / t) * ((c->ny + t - 1) / t) <= cus) return h;
    }
    return 6;
}

int tile_steps(const slbm_ctx* c) { return use_tiles(c) ? tile_halo(c) : 1; }

// Interior tile of the LDS-tiled sweeps for a halo h: the region (tw + 2h) x
// (th + 2h) must hold at most kTileMaxNodes nodes.  Automatic: a 32 x 32
// region, except that small grids take the smallest square tile of 8, 12 or
// 16 nodes whose tile count still fits the compute units (one workgroup
// each): more, smaller workgroups shorten a launch that cannot fill the GPU
// (measured with 8 steps: 128^2 periodic 1.23 -> 1.03 us per step with 8 x 8
// tiles, the 128 x 77 plate 2.57 -> 2.22; at 256^2 and the 256 x 154 plate
// the 16 x 16 tiles, 256 and 160 of them, stay fastest).
void tile_shape(const slbm_ctx* c, int h, int* tw, int* th)
{
    if (c->tile_w > 0 && c->tile_h > 0 && (c->tile_w + 2 * h) * (c->tile_h + 2 * h) <= kTileMaxNodes) {
        *tw = c->tile_w;
        *th = c->tile_h;
        return;
    }
    *tw = std::max(2, 32 - 2 * h);
    *th = std::max(2, 32 - 2 * h);
    if (h == 8) {
        const int64_t cus = c->simds / 4;
        for (int t : {8, 12}) {
            const int64_t tiles = (int64_t)((c->nx + t - 1) / t) * ((c->ny + t - 1) / t);
            if (tiles <= cus) {
                *tw = *th = t;
                return;
            }
        }
    }
}

// Plate tiles hold two copies of the region and the staged boundary records,
// beyond the default 64 KiB of dynamic LDS: raise the limit of those kernels
// (once per context).
int tile_lds_limits(slbm_ctx* c)
{
    if (c->tile_attr) return SLBM_OK;
    const int lmax = (int)tile_lds_bytes(kTileMaxNodes, true);
    // plates: two copies of a region and the staged records exceed the default 64 KiB
    const void* fns[4] = {reinterpret_cast<const void*>(&k_sweep_tile<true, false, false>),
                          reinterpret_cast<const void*>(&k_sweep_tile<true, true, false>),
                          reinterpret_cast<const void*>(&k_sweep_tile<true, false, true>),
                          reinterpret_cast<const void*>(&k_sweep_tile<true, true, true>)};
    for (const void* fn : fns) HIPCHK(c, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lmax));
    c->tile_attr = true;
    return SLBM_OK;
}

// Launch plans (k_tile_plan): the sweeps read their node assignment, codes
// and staged-record list instead of forming them (one round trip fewer, no
// ordering pass, boundary nodes placed for balanced SIMDs).  Plates always
// take one (latency-bound at every size: 512 x 308 in two rounds of
// workgroups 5.0 -> 3.8 us per primal step, 1024 x 615 11.7 -> 10.5), other
// problems for tile shapes whose tiles all fit the compute units at once
// (larger periodic launches keep forming the assignment: there a plan's 16 B
// per region node would add to bandwidth-bound traffic).  Batches plan every
// tiled instance.  Built once per shape (a shape change rebuilds it); call
// before the launches of a loop.
bool tile_plan_wanted(const slbm_ctx* c, int tw, int th)
{
    const int64_t tiles = (int64_t)((c->nx + tw - 1) / tw) * ((c->ny + th - 1) / th);
    return (c->masked || tiles <= c->simds / 4) && c->N < (int64_t)INT32_MAX;
}

void dfree(slbm_ctx* c, void* p)
{
    if (!p) return;
    (void)hipFree(p);
    c->allocs.erase(std::remove(c->allocs.begin(), c->allocs.end(), p), c->allocs.end());
}

// Builds c's launch plan for tw x th tiles with the given halo and ordering
// (kept if it is already the plan held; the buffers grow as needed).
int build_tile_plan(slbm_ctx* c, int halo, int tw, int th, int order)
{
    const int tiles_x = (c->nx + tw - 1) / tw, tiles = tiles_x * ((c->ny + th - 1) / th);
    if (c->plan_key[0] == tw && c->plan_key[1] == th && c->plan_key[2] == halo && c->plan_key[3] == order)
        return SLBM_OK;
    c->plan_key[0] = 0;
    if (tiles > c->plan_cap) {
        dfree(c, c->plan);
        dfree(c, c->plan_rec);
        dfree(c, c->plan_nst);
        c->plan = nullptr;
        c->plan_rec = c->plan_nst = nullptr;
        c->plan_cap = 0;
        const int64_t cap = tiles;
        void* p = nullptr;
        int rc = dalloc(c, &p, (size_t)cap * kTileMaxNodes * sizeof(int4));
        if (rc) return rc;
        c->plan = (int4*)p;
        if ((rc = dalloc(c, &p, (size_t)cap * kTileMaxB * sizeof(int32_t)))) return rc;
        c->plan_rec = (int32_t*)p;
        if ((rc = dalloc(c, &p, (size_t)cap * sizeof(int32_t)))) return rc;
        c->plan_nst = (int32_t*)p;
        c->plan_cap = cap;
    }
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    a.code = c->code;
    a.nx = c->nx;
    a.ny = c->ny;
    a.N = c->N;
    a.tw = tw;
    a.th = th;
    a.halo = halo;
    a.tiles_x = tiles_x;
    a.order_by_kind = order;
    a.maxb = kTileMaxB;
    if (c->masked)
        hipLaunchKernelGGL(k_tile_plan<true>, dim3((unsigned)tiles), dim3(kTileBlock), 0, c->stream, a, c->plan,
                           c->plan_rec, c->plan_nst);
    else
        hipLaunchKernelGGL(k_tile_plan<false>, dim3((unsigned)tiles), dim3(kTileBlock), 0, c->stream, a, c->plan,
                           c->plan_rec, c->plan_nst);
    HIPCHK(c, hipGetLastError());
    c->plan_key[0] = tw;
    c->plan_key[1] = th;
    c->plan_key[2] = halo;
    c->plan_key[3] = order;
    return SLBM_OK;
}

int ensure_tile_plan(slbm_ctx* c, int halo)
{
    int tw, th;
    tile_shape(c, halo, &tw, &th);
    if (!tile_plan_wanted(c, tw, th)) return SLBM_OK;
    return build_tile_plan(c, halo, tw, th, c->masked ? 1 : 0);
}

void launch_tile(slbm_ctx* c, bool adjoint, const SweepArgs& s, int steps, int halo)
{
    TileArgs a;
    std::memset(&a, 0, sizeof(a));
    a.src = s.src;
    a.dst = s.dst;
    a.g = s.g;
    a.E = s.E;
    a.code = s.code;
    a.bnodes = s.bnodes;
    a.status = c->status;
    a.nx = c->nx;
    a.ny = c->ny;
    a.N = c->N;
    a.k11 = s.k11;
    a.ks = s.ks;
    a.kd = s.kd;
    a.E0 = s.E0;
    a.nu = s.nu;
    a.scale = s.scale;
    a.halo = halo;
    a.steps = steps;
    a.maxb = kTileMaxB;
    tile_shape(c, halo, &a.tw, &a.th);
    a.tiles_x = (c->nx + a.tw - 1) / a.tw;
    const int tiles_y = (c->ny + a.th - 1) / a.th;
    const bool want_plan = tile_plan_wanted(c, a.tw, a.th);
    a.order_by_kind = c->masked && (want_plan || (int64_t)a.tiles_x * tiles_y <= c->simds / 4) ? 1 : 0;
    if (want_plan && c->plan && c->plan_key[0] == a.tw && c->plan_key[1] == a.th && c->plan_key[2] == halo &&
        c->plan_key[3] == a.order_by_kind) {
        a.plan = c->plan;
        a.plan_rec = c->plan_rec;
        a.plan_nst = c->plan_nst;
    }
    const size_t lds = tile_lds_bytes((a.tw + 2 * halo) * (a.th + 2 * halo), c->masked);
    dim3 grid((unsigned)(a.tiles_x * tiles_y)), block(kTileBlock);
    int sel = (c->masked ? 4 : 0) | (c->efield_on ? 2 : 0) | (adjoint ? 1 : 0);
#define TL_CASE(i, M, EF, AD) \
    case i: hipLaunchKernelGGL((k_sweep_tile<M, EF, AD>), grid, block, lds, c->stream, a); break;
    switch (sel) {
        TL_CASE(0, false, false, false)
        TL_CASE(1, false, false, true)
        TL_CASE(2, false, true, false)
        TL_CASE(3, false, true, true)
        TL_CASE(4, true, false, false)
        TL_CASE(5, true, false, true)
        TL_CASE(6, true, true, false)
        TL_CASE(7, true, true, true)
    }
#undef TL_CASE
}

// ---------------------------------------------------------------- tangent solves
int64_t control_len(const slbm_ctx* c);
int dot(slbm_ctx* c, const double* a, const double* w, int64_t n, double* out_host);

int tangent_buffers(slbm_ctx* c)
{
    if (c->tv[0]) return SLBM_OK;
    const size_t P8 = 8 * c->N * sizeof(double), P2 = 2 * c->N * sizeof(double);
    int rc;
    for (int k = 0; k < 2; ++k) {
        if ((rc = dalloc(c, (void**)&c->tv[k], P8))) return rc;
        if ((rc = dalloc(c, (void**)&c->td[k], P8))) return rc;
    }
    if ((rc = dalloc(c, (void**)&c->gdot, P2))) return rc;
    if ((rc = dalloc(c, (void**)&c->Edot, c->N * sizeof(double)))) return rc;
    if ((rc = dalloc(c, (void**)&c->snapd, P2))) return rc;
    if ((rc = dalloc(c, (void**)&c->tpart, (size_t)c->pcap * 4 * sizeof(double)))) return rc;
    if ((rc = dalloc(c, (void**)&c->tdir, (size_t)std::max<int64_t>(2 * c->N, 64) * sizeof(double)))) return rc;
    return SLBM_OK;
}

// Derivative of the forcing / modulus along `dir` (control space), the same
// maps as apply_control applied to the direction.
int tangent_direction(slbm_ctx* c, const double* dir, int ptr_kind, bool* use_gdot, bool* use_Edot, double* E0dot)
{
    const int64_t len = control_len(c);
    if (!dir) return fail(c, SLBM_EINVAL, "direction is NULL");
    std::vector<double> h(len);
    if (ptr_kind == SLBM_PTR_DEVICE) {
        HIPCHK(c, hipMemcpyAsync(h.data(), dir, len * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        std::memcpy(h.data(), dir, len * sizeof(double));
    }
    if (!finite_all(h.data(), len)) return fail(c, SLBM_ENONFINITE, "direction has non-finite entries");
    *use_gdot = *use_Edot = false;
    *E0dot = 0.0;
    switch (c->kind) {
        case SLBM_CTRL_FORCE_MODES:
            HIPCHK(c, hipMemcpyAsync(c->tdir, h.data(), len * sizeof(double), hipMemcpyHostToDevice, c->stream));
            hipLaunchKernelGGL(k_force_modes, dim3(grid_of(2 * c->N)), dim3(kBlock), 0, c->stream, c->modes,
                               c->tdir, c->nmodes, 2 * c->N, c->dx2, c->gdot);
            HIPCHK(c, hipGetLastError());
            if (c->masked) {
                hipLaunchKernelGGL(k_axpb2, dim3(grid_of(2 * c->N)), dim3(kBlock), 0, c->stream, c->gdot,
                                   (const double*)nullptr, c->code, c->N, 1.0, c->gdot);
                HIPCHK(c, hipGetLastError());
            }
            *use_gdot = true;
            break;
        case SLBM_CTRL_FORCE_NODAL: {
            HIPCHK(c, hipMemcpyAsync(c->tdir, h.data(), len * sizeof(double), hipMemcpyHostToDevice, c->stream));
            const double* mean = nullptr;
            if (c->project) {
                double m[2];
                for (int k = 0; k < 2; ++k) {
                    int rc = dot(c, c->tdir + k * c->N, nullptr, c->N, &m[k]);
                    if (rc) return rc;
                    m[k] /= (double)c->N;
                }
                HIPCHK(c, hipMemcpyAsync(c->work, m, 2 * sizeof(double), hipMemcpyHostToDevice, c->stream));
                HIPCHK(c, hipStreamSynchronize(c->stream));
                mean = c->work;
            }
            hipLaunchKernelGGL(k_axpb2, dim3(grid_of(2 * c->N)), dim3(kBlock), 0, c->stream, c->tdir, mean,
                               c->masked ? c->code : (const int32_t*)nullptr, c->N, c->dx2, c->gdot);
            HIPCHK(c, hipGetLastError());
            *use_gdot = true;
            break;
        }
        case SLBM_CTRL_E_NODAL:
            HIPCHK(c, hipMemcpyAsync(c->Edot, h.data(), len * sizeof(double), hipMemcpyHostToDevice, c->stream));
            *use_Edot = true;
            break;
        default:  // E = alpha^2
            *E0dot = 2.0 * c->alpha_sq * h[0];
            break;
    }
    return SLBM_OK;
}

void launch_tangent(slbm_ctx* c, const TangentArgs& a, bool check)
{
    const int sel = (c->masked ? 4 : 0) | (c->efield_on ? 2 : 0) | (check ? 1 : 0);
    dim3 grid(grid_of(c->N)), block(kBlock);
    const double inv = c->inv_nx;
#define TG_CASE(i, M, EF, CH) \
    case i: hipLaunchKernelGGL((k_tangent<M, EF, CH>), grid, block, 0, c->stream, a, inv); break;
    switch (sel) {
        TG_CASE(0, false, false, false)
        TG_CASE(1, false, false, true)
        TG_CASE(2, false, true, false)
        TG_CASE(3, false, true, true)
        TG_CASE(4, true, false, false)
        TG_CASE(5, true, false, true)
        TG_CASE(6, true, true, false)
        TG_CASE(7, true, true, true)
    }
#undef TG_CASE
}

// Tangent iteration from zero (value and derivative), checks every K steps;
// returns the final step t, the buffer X holding the input of step t, the
// last residual and whether the test passed.
int tangent_loop(slbm_ctx* c, const TangentArgs& base, int64_t* t_out, int* x_out, double* res_out, bool* conv_out,
                 double* dev_ms)
{
    hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(1), 0, c->stream, c->status);
    HIPCHK(c, hipGetLastError());
    const bool use_tol = c->tol > 0.0;
    const int64_t K = c->K, last = c->max_steps;
    TangentArgs a = base;
    int cur = 0, last_in = 0;
    int64_t chunk = 0;
    int64_t s = 0;
    bool stopped = false;
    CheckLog checks;
    auto last_report = std::chrono::steady_clock::now();
    HIPCHK(c, hipEventRecord(c->t0, c->stream));
    while (s <= last && !stopped) {
        int64_t end = use_tol ? std::min(last, (s / K + 1) * K - 1) : last;
        if (!use_tol && end - s > 4096) end = s + 4095;
        while (s <= end) {
            const bool check = use_tol && s > 0 && s % K == 0;
            a.srcv = c->tv[cur];
            a.srcd = c->td[cur];
            a.dstv = c->tv[cur ^ 1];
            a.dstd = c->td[cur ^ 1];
            launch_tangent(c, a, check);
            if (check) {
                hipLaunchKernelGGL(k_residual2, dim3(1), dim3(kBlock), 0, c->stream, c->tpart, c->nblk, c->status,
                                   c->tol, s);
                checks.add(s, cur);
            }
            if (s == last) last_in = cur;
            cur ^= 1;
            ++s;
        }
        HIPCHK(c, hipGetLastError());
        if (use_tol) {
            const int slot = chunk & 1;
            HIPCHK(c, hipMemcpyAsync(&c->h_status[slot], c->status, sizeof(Status), hipMemcpyDeviceToHost,
                                     c->stream));
            HIPCHK(c, hipEventRecord(c->ev[slot], c->stream));
            if (chunk >= 1) {
                HIPCHK(c, hipEventSynchronize(c->ev[slot ^ 1]));
                const Status& hs = c->h_status[slot ^ 1];
                if (hs.stop) stopped = true;
                if (c->progress && hs.t_last >= 0) {
                    auto now = std::chrono::steady_clock::now();
                    if (std::chrono::duration<double>(now - last_report).count() >= c->progress_every) {
                        last_report = now;
                        c->progress(c->progress_user, 2, hs.t_last, hs.res);
                    }
                }
            }
            ++chunk;
        }
    }
    HIPCHK(c, hipEventRecord(c->t1, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    float f = 0.f;
    HIPCHK(c, hipEventElapsedTime(&f, c->t0, c->t1));
    *dev_ms = f;
    Status st;
    HIPCHK(c, hipMemcpy(&st, c->status, sizeof(Status), hipMemcpyDeviceToHost));
    *res_out = st.res;
    if (use_tol && st.stop) {
        const int xin = checks.find(st.t_conv);
        if (xin < 0) return fail(c, SLBM_EHIP, "internal: converged step without a check sweep");
        *t_out = st.t_conv;
        *x_out = xin;
        *conv_out = true;
    } else {
        *t_out = last;
        *x_out = last_in;
        *conv_out = false;
    }
    return SLBM_OK;
}

// Runs sweeps with indices 0 .. last (inclusive) from buffer parity `start`,
// checking every K steps when tol > 0; stops at the first passing test.
// Returns the step index t of the final state whose successor was also
// produced (the last executed sweep has index t).
int run_loop(slbm_ctx* c, bool adjoint, int start, int64_t last, bool use_tol, int64_t* t_out,
             double* res_out, bool* conv_out, double* dev_ms = nullptr, int* x_out = nullptr)
{
    c->lt.reset();
    double** bufs = adjoint ? c->abuf : c->fbuf;
    hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(1), 0, c->stream, c->status);
    HIPCHK(c, hipGetLastError());
    SweepArgs a = base_args(c);
    if (adjoint) {
        a.g = c->asrc;
        a.scale = c->dx2 / c->cbar;
    } else {
        a.g = c->g;
    }
    const int64_t K = c->K;
    int64_t s = 0;
    int64_t chunk = 0;
    bool stopped = false;
    HIPCHK(c, hipEventRecord(c->t0, c->stream));
    // buffer holding the input of sweep s; check sweeps and the final sweep are
    // single-step launches, runs of plain sweeps between them are fused by T
    int cur = start;
    const int T = fused_steps(c);
    const int TL = tile_steps(c);
    if (TL > 1 && c->masked) {
        int rc = tile_lds_limits(c);
        if (rc) return rc;
    }
    if (TL > 1) {
        int rc = ensure_tile_plan(c, TL);
        if (rc) return rc;
    }
    CheckLog checks;                              // (step, input buffer) of the latest check sweeps
    int last_in = start;
    auto last_report = std::chrono::steady_clock::now();
    while (s <= last && !stopped) {
        int64_t end = use_tol ? std::min(last, (s / K + 1) * K - 1) : last;
        if (!use_tol && end - s > 4096 * T) end = s + 4096 * T - 1;
        while (s <= end) {
            bool check = use_tol && s > 0 && s % K == 0;
            // plain sweeps available for fusing: up to `end`, never the final sweep
            int64_t plain = std::min(end, last - 1) - s + 1;
            if (!check && T > 1 && plain >= T) {
                a.src = bufs[cur];
                a.dst = bufs[cur ^ 1];
                HIPCHK(c, c->lt.before(c->stream, T, s));
                launch_fused(c, adjoint, a, T);
                cur ^= 1;
                s += T;
                continue;
            }
            if (!check && TL > 1 && plain >= 2) {
                const int k = (int)std::min<int64_t>(plain, TL);
                a.src = bufs[cur];
                a.dst = bufs[cur ^ 1];
                HIPCHK(c, c->lt.before(c->stream, k, s));
                launch_tile(c, adjoint, a, k, TL);
                cur ^= 1;
                s += k;
                continue;
            }
            HIPCHK(c, c->lt.close(c->stream));
            a.src = bufs[cur];
            a.dst = bufs[cur ^ 1];
            launch_sweep(c, adjoint, a, check);
            if (check) {
                hipLaunchKernelGGL(k_residual, dim3(1), dim3(kBlock), 0, c->stream, c->partial, c->nblk,
                                   c->status, c->tol, s, c->cv_window);
                checks.add(s, cur);
            }
            if (s == last) last_in = cur;
            cur ^= 1;
            ++s;
        }
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, c->lt.close(c->stream));
        HIPCHK(c, c->lt.harvest(false));
        if (use_tol) {
            int slot = chunk & 1;
            HIPCHK(c, hipMemcpyAsync(&c->h_status[slot], c->status, sizeof(Status), hipMemcpyDeviceToHost,
                                     c->stream));
            HIPCHK(c, hipEventRecord(c->ev[slot], c->stream));
            if (chunk >= 1) {
                HIPCHK(c, hipEventSynchronize(c->ev[slot ^ 1]));
                const Status& hs = c->h_status[slot ^ 1];
                if (hs.stop) stopped = true;
                if (c->progress && hs.t_last >= 0) {
                    auto now = std::chrono::steady_clock::now();
                    if (std::chrono::duration<double>(now - last_report).count() >= c->progress_every) {
                        last_report = now;
                        c->progress(c->progress_user, adjoint ? 1 : 0, hs.t_last, hs.res);
                    }
                }
            }
            ++chunk;
        }
    }
    HIPCHK(c, c->lt.close(c->stream));
    HIPCHK(c, hipEventRecord(c->t1, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, c->lt.harvest(true));
    if (dev_ms) {
        float f = 0.f;
        HIPCHK(c, hipEventElapsedTime(&f, c->t0, c->t1));
        *dev_ms = f;
    }
    Status st;
    HIPCHK(c, hipMemcpy(&st, c->status, sizeof(Status), hipMemcpyDeviceToHost));
    if (c->lt.on) c->lt.trim(use_tol && st.stop ? st.t_conv : last);
    if (use_tol && st.stop) {
        *t_out = st.t_conv;
        *conv_out = true;
        const int xin = checks.find(st.t_conv);
        if (xin < 0) return fail(c, SLBM_EHIP, "internal: converged step without a check sweep");
        if (x_out) *x_out = xin;
    } else {
        *t_out = last;
        *conv_out = false;
        if (x_out) *x_out = last_in;
    }
    *res_out = st.res;
    return SLBM_OK;
}

int sum_partials(slbm_ctx* c, double* out_host)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, c->stream, c->partial, c->nblk, c->scal);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(out_host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SLBM_OK;
}

// sum_i a[i] * w[i] over n entries (w null: plain sum), deterministic
int dot(slbm_ctx* c, const double* a, const double* w, int64_t n, double* out_host)
{
    int64_t nb = (n + kBlock - 1) / kBlock;
    if (nb > c->pcap) return fail(c, SLBM_EINVAL, "internal: reduction too large");
    hipLaunchKernelGGL(k_dot_partial, dim3((unsigned)nb), dim3(kBlock), 0, c->stream, a, w, n, c->partial);
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, c->stream, c->partial, nb, c->scal);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(out_host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SLBM_OK;
}

int copy_in(slbm_ctx* c, void* dst, const void* src, size_t bytes, int ptr_kind)
{
    HIPCHK(c, hipMemcpyAsync(dst, src, bytes,
                             ptr_kind == SLBM_PTR_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                             c->stream));
    return SLBM_OK;
}

int copy_out(slbm_ctx* c, void* dst, const void* src, size_t bytes, int ptr_kind)
{
    HIPCHK(c, hipMemcpyAsync(dst, src, bytes,
                             ptr_kind == SLBM_PTR_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SLBM_OK;
}

int64_t control_len(const slbm_ctx* c)
{
    switch (c->kind) {
        case SLBM_CTRL_FORCE_MODES: return c->nmodes;
        case SLBM_CTRL_FORCE_NODAL: return 2 * c->N;
        case SLBM_CTRL_E_NODAL: return c->N;
        default: return 1;
    }
}

// Control -> forcing / moduli (eq. forcing, eq. zero_mean_projection,
// eq. E_substitution).  The control is staged in c->ctrl.
int apply_control(slbm_ctx* c, const double* control, int ptr_kind)
{
    int64_t len = control_len(c);
    if (!control) return fail(c, SLBM_EINVAL, "control is NULL");
    std::vector<double> h(len);
    if (ptr_kind == SLBM_PTR_DEVICE) {
        HIPCHK(c, hipMemcpyAsync(h.data(), control, len * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        std::memcpy(h.data(), control, len * sizeof(double));
    }
    if (!finite_all(h.data(), len)) return fail(c, SLBM_ENONFINITE, "control has non-finite entries");
    switch (c->kind) {
        case SLBM_CTRL_FORCE_MODES: {
            HIPCHK(c, hipMemcpyAsync(c->ctrl, h.data(), len * sizeof(double), hipMemcpyHostToDevice, c->stream));
            hipLaunchKernelGGL(k_force_modes, dim3(grid_of(2 * c->N)), dim3(kBlock), 0, c->stream, c->modes,
                               c->ctrl, c->nmodes, 2 * c->N, c->dx2, c->g);
            HIPCHK(c, hipGetLastError());
            if (c->masked) {
                hipLaunchKernelGGL(k_axpb2, dim3(grid_of(2 * c->N)), dim3(kBlock), 0, c->stream, c->g,
                                   (const double*)nullptr, c->code, c->N, 1.0, c->g);
                HIPCHK(c, hipGetLastError());
            }
            c->E_cur = c->E;
            c->efield_on = false;
            break;
        }
        case SLBM_CTRL_FORCE_NODAL: {
            HIPCHK(c, hipMemcpyAsync(c->ctrl, h.data(), len * sizeof(double), hipMemcpyHostToDevice, c->stream));
            const double* mean = nullptr;
            if (c->project) {
                double m[2];
                for (int k = 0; k < 2; ++k) {
                    int rc = dot(c, c->ctrl + k * c->N, nullptr, c->N, &m[k]);
                    if (rc) return rc;
                    m[k] /= (double)c->N;
                }
                HIPCHK(c, hipMemcpyAsync(c->work, m, 2 * sizeof(double), hipMemcpyHostToDevice, c->stream));
                HIPCHK(c, hipStreamSynchronize(c->stream));
                mean = c->work;
            }
            hipLaunchKernelGGL(k_axpb2, dim3(grid_of(2 * c->N)), dim3(kBlock), 0, c->stream, c->ctrl, mean,
                               c->masked ? c->code : (const int32_t*)nullptr, c->N, c->dx2, c->g);
            HIPCHK(c, hipGetLastError());
            c->E_cur = c->E;
            c->efield_on = false;
            break;
        }
        case SLBM_CTRL_E_NODAL: {
            for (int64_t i = 0; i < len; ++i) {
                if (!(h[i] > 0.0)) return fail(c, SLBM_EINVAL, "E control must be > 0 everywhere");
                if (c->masked && !gamma_ok(h[i], c->nu))
                    return fail(c, SLBM_EINVAL, "tau_s = tau_f: the boundary coefficient gamma is undefined");
            }
            HIPCHK(c, hipMemcpyAsync(c->Efield, h.data(), len * sizeof(double), hipMemcpyHostToDevice,
                                     c->stream));
            HIPCHK(c, hipMemcpyAsync(c->g, c->fixedF, 2 * c->N * sizeof(double), hipMemcpyDeviceToDevice,
                                     c->stream));
            c->efield_on = true;
            c->E_cur = h[0];
            break;
        }
        default: {
            double a = h[0];
            if (a == 0.0) return fail(c, SLBM_EINVAL, "E = alpha^2 must be > 0");
            if (c->masked && !gamma_ok(a * a, c->nu))
                return fail(c, SLBM_EINVAL, "tau_s = tau_f: the boundary coefficient gamma is undefined");
            c->alpha_sq = a;
            c->E_cur = a * a;
            c->efield_on = false;
            HIPCHK(c, hipMemcpyAsync(c->g, c->fixedF, 2 * c->N * sizeof(double), hipMemcpyDeviceToDevice,
                                     c->stream));
            break;
        }
    }
    // the staged host copy of the control must outlive its upload
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return SLBM_OK;
}

int reset_primal(slbm_ctx* c, const double* init_disp, int ptr_kind)
{
    int rc;
    if ((rc = fill(c, c->fbuf[0], 8 * c->N, 0.0))) return rc;
    if ((rc = fill(c, c->fbuf[1], 8 * c->N, 0.0))) return rc;
    const double* d0 = nullptr;
    if (init_disp) {
        if ((rc = copy_in(c, c->work, init_disp, 2 * c->N * sizeof(double), ptr_kind))) return rc;
        d0 = c->work;
    }
    hipLaunchKernelGGL(k_init_state, dim3(grid_of(c->N)), dim3(kBlock), 0, c->stream, c->fbuf[0], d0, c->g,
                       c->masked ? c->code : (const int32_t*)nullptr, c->nx, c->ny, c->N, c->inv_nx, c->snap);
    HIPCHK(c, hipGetLastError());
    c->prim_cur = 0;
    c->prim_valid = true;
    c->prim_done = false;
    c->adj_done = false;
    return SLBM_OK;
}

int finalize_primal(slbm_ctx* c, int X)
{
    if (c->masked)
        hipLaunchKernelGGL(k_primal_finalize<true>, dim3(grid_of(c->N)), dim3(kBlock), 0, c->stream,
                           c->fbuf[X], c->fbuf[X ^ 1], c->g, c->code, c->target, c->obs, c->nx, c->ny, c->N,
                           c->inv_nx, c->dbar, c->r, c->fbar, c->partial);
    else
        hipLaunchKernelGGL(k_primal_finalize<false>, dim3(grid_of(c->N)), dim3(kBlock), 0, c->stream,
                           c->fbuf[X], c->fbuf[X ^ 1], c->g, c->code, c->target, c->obs, c->nx, c->ny, c->N,
                           c->inv_nx, c->dbar, c->r, c->fbar, c->partial);
    HIPCHK(c, hipGetLastError());
    double s;
    int rc = sum_partials(c, &s);
    if (rc) return rc;
    c->J = 0.5 * s * c->dx2 / c->cbar;
    return SLBM_OK;
}

int do_primal(slbm_ctx* c, slbm_solve_info* info)
{
    auto w0 = std::chrono::steady_clock::now();
    int64_t t;
    double res;
    bool conv;
    bool use_tol = c->tol > 0.0;
    double dms = 0.0;
    int X = 0;  // buffer holding f^C(t-1)
    int rc = run_loop(c, false, c->prim_cur, c->max_steps, use_tol, &t, &res, &conv, &dms, &X);
    if (rc) return rc;
    if ((rc = finalize_primal(c, X))) return rc;
    c->prim_cur = X ^ 1;  // current state: f^S(t+1)
    c->prim_done = true;
    c->adj_done = false;
    auto w1 = std::chrono::steady_clock::now();
    if (info) {
        info->steps = t;
        info->sweeps = t + 1;
        info->residual = use_tol ? res : 0.0;
        info->wall_s = std::chrono::duration<double>(w1 - w0).count();
        info->device_ms = dms;
        info->converged = conv ? 1 : 0;
        info->fused_launches = c->lt.launches;
        info->fused_sweeps = c->lt.sweeps;
        info->fused_ms = c->lt.ms;
    }
    return (use_tol && !conv) ? SLBM_NOT_CONVERGED : SLBM_OK;
}

int adjoint_prepare(slbm_ctx* c)
{
    int rc;
    if ((rc = fill(c, c->abuf[0], 8 * c->N, 0.0))) return rc;
    if ((rc = fill(c, c->abuf[1], 8 * c->N, 0.0))) return rc;
    if ((rc = fill(c, c->snap, 2 * c->N, 0.0))) return rc;
    c->adj_cur = 0;
    c->adj_valid = true;
    return SLBM_OK;
}

// Periodic domains: the displacement has zero mean by construction (the
// translations are the kernel of the torus problem), so the mean of the
// adjoint source does not depend on the control and lies outside the range of
// the solution map; it is removed per component (the compatibility condition
// of eq. zero_mean_projection), which keeps the adjoint's translation mode at
// rest.  Works on c->asrc; r = d - d* itself is left as it is.
int project_source(slbm_ctx* c)
{
    if (c->masked) return SLBM_OK;
    double m[2];
    int rc;
    for (int k = 0; k < 2; ++k) {
        if ((rc = dot(c, c->asrc + k * c->N, nullptr, c->N, &m[k]))) return rc;
        m[k] /= (double)c->N;
    }
    HIPCHK(c, hipMemcpyAsync(c->work, m, 2 * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    hipLaunchKernelGGL(k_axpb2, dim3(grid_of(2 * c->N)), dim3(kBlock), 0, c->stream, c->asrc,
                       (const double*)c->work, (const int32_t*)nullptr, c->N, 1.0, c->asrc);
    HIPCHK(c, hipGetLastError());
    return SLBM_OK;
}

// Adjoint source of the objective (eq. discrete_J): r of the last completed
// primal solve, projected on periodic domains.
int objective_source(slbm_ctx* c)
{
    HIPCHK(c, hipMemcpyAsync(c->asrc, c->r, 2 * c->N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    return project_source(c);
}

int adjoint_finalize(slbm_ctx* c, int X, double scale);

// scale_override > 0: c->asrc already holds a cotangent (adjoint_solve_vjp),
// used with that scale; otherwise the objective's source is formed from r.
int do_adjoint(slbm_ctx* c, slbm_solve_info* info, double scale_override = -1.0)
{
    if (!c->prim_done) return fail(c, SLBM_ESTATE, "adjoint_solve needs a completed primal_solve");
    auto w0 = std::chrono::steady_clock::now();
    int rc = adjoint_prepare(c);
    if (rc) return rc;
    if ((rc = scale_override > 0.0 ? project_source(c) : objective_source(c))) return rc;
    const double saved_cbar = c->cbar;
    if (scale_override > 0.0) c->cbar = c->dx2 / scale_override;  // run_loop uses dx^2 / cbar
    int64_t t;
    double res;
    bool conv;
    bool use_tol = c->tol > 0.0;
    double dms = 0.0;
    int X = 0;  // buffer holding phi^C(t)
    rc = run_loop(c, true, 0, c->max_steps, use_tol, &t, &res, &conv, &dms, &X);
    c->cbar = saved_cbar;
    if (rc) return rc;
    if ((rc = adjoint_finalize(c, X, scale_override > 0.0 ? scale_override : c->dx2 / c->cbar))) return rc;
    auto w1 = std::chrono::steady_clock::now();
    if (info) {
        info->steps = t;
        info->sweeps = t + 1;
        info->residual = use_tol ? res : 0.0;
        info->wall_s = std::chrono::duration<double>(w1 - w0).count();
        info->device_ms = dms;
        info->converged = conv ? 1 : 0;
        info->fused_launches = c->lt.launches;
        info->fused_sweeps = c->lt.sweeps;
        info->fused_ms = c->lt.ms;
    }
    return (use_tol && !conv) ? SLBM_NOT_CONVERGED : SLBM_OK;
}

// Two-step-averaged adjoint from X = phi^C(t), X^1 = phi^C(t+1) and the local
// gradient pieces (eq. optimality); source scale s = dx^2 / Cbar (objective)
// or 1 (cotangent).
int adjoint_finalize(slbm_ctx* c, int X, double scale)
{
    bool wantE = c->kind == SLBM_CTRL_E_NODAL || c->kind == SLBM_CTRL_E_SCALAR_SQ;
    if (c->masked)
        hipLaunchKernelGGL(k_adjoint_finalize<true>, dim3(grid_of(c->N)), dim3(kBlock), 0, c->stream, c->abuf[X],
                           c->abuf[X ^ 1], c->code, c->bnodes, c->fbar, c->asrc, c->g,
                           c->efield_on ? c->Efield : (const double*)nullptr, c->E_cur, c->nu, wantE ? 1 : 0,
                           c->nx, c->ny, c->N, c->inv_nx, scale, c->dx2, c->dJdF, c->dJdE, c->adisp);
    else
        hipLaunchKernelGGL(k_adjoint_finalize<false>, dim3(grid_of(c->N)), dim3(kBlock), 0, c->stream, c->abuf[X],
                           c->abuf[X ^ 1], c->code, c->bnodes, c->fbar, c->asrc, c->g,
                           c->efield_on ? c->Efield : (const double*)nullptr, c->E_cur, c->nu, wantE ? 1 : 0,
                           c->nx, c->ny, c->N, c->inv_nx, scale, c->dx2, c->dJdF, c->dJdE, c->adisp);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->adj_cur = X ^ 1;
    c->adj_done = true;
    return SLBM_OK;
}

// Gradient per control kind from the local pieces dJdF / dJdE.
int assemble_grad(slbm_ctx* c, double* grad, int ptr_kind)
{
    int rc;
    switch (c->kind) {
        case SLBM_CTRL_FORCE_MODES: {
            std::vector<double> h(c->nmodes);
            for (int m = 0; m < c->nmodes; ++m)
                if ((rc = dot(c, c->dJdF, c->modes + (int64_t)m * 2 * c->N, 2 * c->N, &h[m]))) return rc;
            if (ptr_kind == SLBM_PTR_DEVICE) {
                HIPCHK(c, hipMemcpyAsync(grad, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice,
                                         c->stream));
                HIPCHK(c, hipStreamSynchronize(c->stream));
            } else {
                std::memcpy(grad, h.data(), h.size() * sizeof(double));
            }
            return SLBM_OK;
        }
        case SLBM_CTRL_FORCE_NODAL: {
            if (c->project) {
                double m[2];
                for (int k = 0; k < 2; ++k) {
                    if ((rc = dot(c, c->dJdF + k * c->N, nullptr, c->N, &m[k]))) return rc;
                    m[k] /= (double)c->N;
                }
                HIPCHK(c, hipMemcpyAsync(c->work, m, 2 * sizeof(double), hipMemcpyHostToDevice, c->stream));
                HIPCHK(c, hipStreamSynchronize(c->stream));
                hipLaunchKernelGGL(k_axpb2, dim3(grid_of(2 * c->N)), dim3(kBlock), 0, c->stream, c->dJdF,
                                   (const double*)c->work, (const int32_t*)nullptr, c->N, 1.0, c->dJdF);
                HIPCHK(c, hipGetLastError());
            }
            return copy_out(c, grad, c->dJdF, 2 * c->N * sizeof(double), ptr_kind);
        }
        case SLBM_CTRL_E_NODAL:
            return copy_out(c, grad, c->dJdE, c->N * sizeof(double), ptr_kind);
        default: {
            double s;
            if ((rc = dot(c, c->dJdE, nullptr, c->N, &s))) return rc;
            double gsc = s * 2.0 * c->alpha_sq;
            if (ptr_kind == SLBM_PTR_DEVICE) {
                HIPCHK(c, hipMemcpyAsync(grad, &gsc, sizeof(double), hipMemcpyHostToDevice, c->stream));
                HIPCHK(c, hipStreamSynchronize(c->stream));
            } else {
                grad[0] = gsc;
            }
            return SLBM_OK;
        }
    }
}

}  // namespace

// ======================================================================= C ABI

extern "C" {

int solid_lbm_init(const slbm_problem* p, slbm_ctx** out)
{
    if (!out) return fail(nullptr, SLBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return fail(nullptr, SLBM_EINVAL, "problem is NULL");
    if (p->nx < 3 || p->ny < 3) return fail(nullptr, SLBM_EINVAL, "nx, ny must be >= 3");
    if ((int64_t)p->nx * p->ny > (int64_t)1 << 31) return fail(nullptr, SLBM_EINVAL, "grid too large");
    if (!(p->dx > 0.0) || !std::isfinite(p->dx)) return fail(nullptr, SLBM_EINVAL, "dx must be > 0");
    if (!(p->nu > -1.0 && p->nu < 1.0)) return fail(nullptr, SLBM_EINVAL, "nu must lie in (-1, 1)");
    if (std::isnan(p->tol)) return fail(nullptr, SLBM_EINVAL, "tol is NaN");
    if (p->check_interval == 0 && !(0.005 / (p->dx * p->dx) < 1e18))
        return fail(nullptr, SLBM_EINVAL, "dx too small for the default check interval");
    bool econtrol = p->control_kind == SLBM_CTRL_E_NODAL || p->control_kind == SLBM_CTRL_E_SCALAR_SQ;
    if (p->control_kind < 0 || p->control_kind > 3) return fail(nullptr, SLBM_EINVAL, "unknown control_kind");
    if (!econtrol && (!(p->E > 0.0) || !std::isfinite(p->E))) return fail(nullptr, SLBM_EINVAL, "E must be > 0");
    if (p->domain != SLBM_PERIODIC && p->domain != SLBM_MASKED) return fail(nullptr, SLBM_EINVAL, "unknown domain");
    if (!p->target) return fail(nullptr, SLBM_EINVAL, "target is NULL");
    if (p->max_steps < 1) return fail(nullptr, SLBM_EINVAL, "max_steps must be >= 1");
    if (p->check_interval < 0) return fail(nullptr, SLBM_EINVAL, "check_interval must be >= 0");
    if (p->convergence != SLBM_CONV_KLAG && p->convergence != SLBM_CONV_CV)
        return fail(nullptr, SLBM_EINVAL, "unknown convergence test");
    if (p->convergence == SLBM_CONV_CV && p->cv_window != 0 && (p->cv_window < 2 || p->cv_window > kMaxCvWindow))
        return fail(nullptr, SLBM_EINVAL, "cv_window must be 0 or 2..32");
    if (p->control_kind == SLBM_CTRL_FORCE_MODES && (p->n_modes < 1 || p->n_modes > 64 || !p->force_modes))
        return fail(nullptr, SLBM_EINVAL, "FORCE_MODES needs 1..64 force_modes");
    bool masked = p->domain == SLBM_MASKED;
    if (masked && (!p->node_mask || !p->link_bc || !p->link_wall))
        return fail(nullptr, SLBM_EINVAL, "MASKED needs node_mask, link_bc and link_wall");

    const int nx = p->nx, ny = p->ny;
    const int64_t N = (int64_t)nx * ny;
    if (!finite_all(p->target, 2 * N)) return fail(nullptr, SLBM_ENONFINITE, "target has non-finite entries");
    if (p->fixed_force && !finite_all(p->fixed_force, 2 * N))
        return fail(nullptr, SLBM_ENONFINITE, "fixed_force has non-finite entries");
    if (p->force_modes && p->control_kind == SLBM_CTRL_FORCE_MODES &&
        !finite_all(p->force_modes, (int64_t)p->n_modes * 2 * N))
        return fail(nullptr, SLBM_ENONFINITE, "force_modes has non-finite entries");

    // plate: node codes and boundary records
    std::vector<int32_t> code(N, 0);
    std::vector<BNode> bn;
    bool any_neumann = false;
    if (masked) {
        for (int64_t n = 0; n < N; ++n) code[n] = p->node_mask[n] ? 0 : -1;
        for (int ix = 0; ix < nx; ++ix)
            if (code[ix] >= 0 || code[(int64_t)(ny - 1) * nx + ix] >= 0)
                return fail(nullptr, SLBM_EINVAL, "a domain node lies on the box edge");
        for (int iy = 0; iy < ny; ++iy)
            if (code[(int64_t)iy * nx] >= 0 || code[(int64_t)iy * nx + nx - 1] >= 0)
                return fail(nullptr, SLBM_EINVAL, "a domain node lies on the box edge");
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix) {
                int64_t n = (int64_t)iy * nx + ix;
                if (code[n] < 0) continue;
                BNode b;
                std::memset(&b, 0, sizeof(b));
                b.cell = (int32_t)n;
                for (int q = 0; q < 8; ++q) {
                    int64_t m = (int64_t)(iy - cy(q)) * nx + (ix - cx(q));
                    bool outside = code[m] < 0;
                    uint8_t kind = p->link_bc[(int64_t)q * N + n];
                    if (outside != (kind != 0))
                        return fail(nullptr, SLBM_EINVAL, "link_bc must be non-zero exactly on cut links");
                    if (!outside) continue;
                    if (kind != SLBM_LINK_DIRICHLET && kind != SLBM_LINK_NEUMANN)
                        return fail(nullptr, SLBM_EINVAL, "unknown link kind");
                    b.cut |= 1u << q;
                    if (kind == SLBM_LINK_DIRICHLET) b.dirichlet |= 1u << q;
                    else any_neumann = true;
                    double w[2], nr[2];
                    for (int k = 0; k < 2; ++k) {
                        w[k] = p->link_wall[(int64_t)(k * 8 + q) * N + n];
                        nr[k] = p->link_normal ? p->link_normal[(int64_t)(k * 8 + q) * N + n] : 0.0;
                        if (!std::isfinite(w[k]) || !std::isfinite(nr[k]))
                            return fail(nullptr, SLBM_ENONFINITE, "non-finite wall data");
                    }
                    closure_coefs(q, kind == SLBM_LINK_DIRICHLET, w[0], w[1], nr[0], nr[1], b.coef[q]);
                }
                if (b.cut) {
                    code[n] = (int32_t)bn.size() + 1;
                    bn.push_back(b);
                }
            }
        if (any_neumann && !p->link_normal) return fail(nullptr, SLBM_EINVAL, "Neumann links need link_normal");
    }

    slbm_ctx* c = new slbm_ctx();
    c->nx = nx;
    c->ny = ny;
    c->N = N;
    c->dx = p->dx;
    c->dx2 = p->dx * p->dx;
    c->E = p->E;
    c->nu = p->nu;
    c->tol = p->tol;
    c->inv_nx = 1.0 / nx;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            c->simds = 4 * cus;
    }
    c->max_steps = p->max_steps;
    c->K = p->check_interval > 0 ? p->check_interval
                                 : 2 * (int64_t)std::ceil(0.005 / (c->dx2) - 1e-9);
    if (c->K < 1) c->K = 1;
    c->cv_window = p->convergence == SLBM_CONV_CV ? (p->cv_window > 0 ? p->cv_window : 10) : 0;
    c->kind = p->control_kind;
    c->nmodes = p->n_modes;
    c->project = (p->control_kind == SLBM_CTRL_FORCE_NODAL && !masked && p->zero_mean_projection) ? 1 : 0;
    c->normalize = p->normalize_objective ? 1 : 0;
    c->masked = masked;
    c->nb = (int)bn.size();
    c->stream = (hipStream_t)p->stream;
    c->E_cur = p->E;
    c->nblk = (N + kBlock - 1) / kBlock;
    c->pcap = (2 * N + kBlock - 1) / kBlock + 2;

    // Cbar (eq. node_J) on the host, over the observation set
    double cb = 0.0;
    for (int64_t n = 0; n < N; ++n) {
        bool in = (!masked || code[n] >= 0) && (!p->obs_mask || p->obs_mask[n]);
        if (in) cb += p->target[n] * p->target[n] + p->target[N + n] * p->target[N + n];
    }
    cb *= c->dx2;
    if (c->normalize) {
        if (!(cb > 0.0)) {
            delete c;
            return fail(nullptr, SLBM_EINVAL, "normalize_objective needs a non-zero target");
        }
        c->cbar = cb;
    } else {
        c->cbar = 1.0;
    }
    if (!econtrol && masked && !gamma_ok(p->E, p->nu)) {
        delete c;
        return fail(nullptr, SLBM_EINVAL, "tau_s = tau_f: the boundary coefficient gamma is undefined");
    }

    int rc = SLBM_OK;
#define A(ptr, bytes)                                 \
    do {                                              \
        if (!rc) {                                    \
            void* q_ = nullptr;                       \
            rc = dalloc(c, &q_, (bytes));             \
            *(ptr) = (decltype(*(ptr)))q_;            \
        }                                             \
    } while (0)
    const size_t P8 = 8 * N * sizeof(double), P2 = 2 * N * sizeof(double), P1 = N * sizeof(double);
    A(&c->fbuf[0], P8);
    A(&c->fbuf[1], P8);
    A(&c->abuf[0], P8);
    A(&c->abuf[1], P8);
    A(&c->fbar, P8);
    A(&c->g, P2);
    A(&c->target, P2);
    A(&c->snap, P2);
    A(&c->dbar, P2);
    A(&c->r, P2);
    A(&c->asrc, P2);
    A(&c->dJdF, P2);
    A(&c->adisp, P2);
    A(&c->work, P8 > 1024 ? P8 : 1024);
    A(&c->dJdE, P1);
    A(&c->Efield, P1);
    A(&c->fixedF, P2);
    A(&c->partial, (size_t)c->pcap * 2 * sizeof(double));
    A(&c->scal, 64);
    A(&c->ctrl, (size_t)std::max<int64_t>(2 * N, 64) * sizeof(double));
    A(&c->status, sizeof(Status));
    if (c->kind == SLBM_CTRL_FORCE_MODES) A(&c->modes, (size_t)c->nmodes * P2);
    if (masked) {
        A(&c->code, N * sizeof(int32_t));
        A(&c->bnodes, std::max<size_t>(1, bn.size()) * sizeof(BNode));
    }
    if (p->obs_mask) A(&c->obs, N);
#undef A
    if (rc) {
        const std::string why = c->err;
        solid_lbm_destroy(c);
        return fail(nullptr, rc, "device allocation failed: " + why);
    }
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (rc) return;
        hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = fail(c, SLBM_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
    };
    up(c->target, p->target, P2);
    if (p->fixed_force) {
        std::vector<double> gf(2 * N);
        for (int64_t i = 0; i < 2 * N; ++i) {
            int64_t n = i % N;
            bool in = !masked || code[n] >= 0;
            gf[i] = in ? c->dx2 * p->fixed_force[i] : 0.0;
        }
        up(c->fixedF, gf.data(), P2);
    } else if (!rc) {
        if (hipMemset(c->fixedF, 0, P2) != hipSuccess) rc = SLBM_EHIP;
    }
    if (c->kind == SLBM_CTRL_FORCE_MODES) up(c->modes, p->force_modes, (size_t)c->nmodes * P2);
    if (masked) {
        up(c->code, code.data(), N * sizeof(int32_t));
        if (!bn.empty()) up(c->bnodes, bn.data(), bn.size() * sizeof(BNode));
    }
    if (p->obs_mask) up(c->obs, p->obs_mask, N);
    if (!rc && hipMemset(c->g, 0, P2) != hipSuccess) rc = SLBM_EHIP;
    if (!rc && hipHostMalloc((void**)&c->h_status, 2 * sizeof(Status), hipHostMallocDefault) != hipSuccess)
        rc = SLBM_EHIP;
    if (!rc && (hipEventCreate(&c->ev[0]) != hipSuccess || hipEventCreate(&c->ev[1]) != hipSuccess ||
                hipEventCreate(&c->t0) != hipSuccess || hipEventCreate(&c->t1) != hipSuccess))
        rc = SLBM_EHIP;
    if (rc) {
        const std::string why = c->err;
        solid_lbm_destroy(c);
        return fail(nullptr, rc, "upload failed" + (why.empty() ? std::string() : ": " + why));
    }
    *out = c;
    return SLBM_OK;
}

int solid_lbm_set_control(slbm_ctx* c, const double* control, const double* init_disp, int32_t ptr_kind)
{
    if (!c) return SLBM_EINVAL;
    int rc = apply_control(c, control, ptr_kind);
    if (rc) return rc;
    return reset_primal(c, init_disp, ptr_kind);
}

int primal_solve(slbm_ctx* c, const double* control, const double* init_disp, int32_t ptr_kind,
                 slbm_solve_info* info)
{
    if (!c) return SLBM_EINVAL;
    int rc = solid_lbm_set_control(c, control, init_disp, ptr_kind);
    if (rc) return rc;
    return do_primal(c, info);
}

int adjoint_solve(slbm_ctx* c, slbm_solve_info* info)
{
    if (!c) return SLBM_EINVAL;
    return do_adjoint(c, info);
}

int objective_and_grad_from(slbm_ctx* c, const double* control, const double* init_disp, double* J, double* grad,
                            int32_t ptr_kind, slbm_solve_info* pinfo, slbm_solve_info* ainfo)
{
    if (!c) return SLBM_EINVAL;
    if (!J) return fail(c, SLBM_EINVAL, "J is NULL");
    int rc = primal_solve(c, control, init_disp, ptr_kind, pinfo);
    if (rc < 0) return rc;
    int warn = rc;
    *J = c->J;
    if (!grad) return warn;
    rc = do_adjoint(c, ainfo);
    if (rc < 0) return rc;
    if (rc > 0) warn = rc;
    rc = assemble_grad(c, grad, ptr_kind);
    if (rc < 0) return rc;
    return warn;
}

int objective_and_grad(slbm_ctx* c, const double* control, double* J, double* grad, int32_t ptr_kind,
                       slbm_solve_info* pinfo, slbm_solve_info* ainfo)
{
    return objective_and_grad_from(c, control, nullptr, J, grad, ptr_kind, pinfo, ainfo);
}

int solid_lbm_run_steps(slbm_ctx* c, int64_t n)
{
    if (!c) return SLBM_EINVAL;
    if (!c->prim_valid) return fail(c, SLBM_ESTATE, "no primal state: call solid_lbm_set_control first");
    if (n < 0) return fail(c, SLBM_EINVAL, "n must be >= 0");
    if (n == 0) return SLBM_OK;
    int64_t t;
    double res;
    bool conv;
    int X = 0;
    int rc = run_loop(c, false, c->prim_cur, n - 1, false, &t, &res, &conv, nullptr, &X);
    if (rc) return rc;
    c->prim_cur = X ^ 1;
    c->prim_done = false;
    return SLBM_OK;
}

int solid_lbm_run_adjoint_steps(slbm_ctx* c, int64_t n)
{
    if (!c) return SLBM_EINVAL;
    if (!c->prim_done) return fail(c, SLBM_ESTATE, "adjoint steps need a completed primal_solve");
    if (n < 0) return fail(c, SLBM_EINVAL, "n must be >= 0");
    int rc = adjoint_prepare(c);
    if (rc) return rc;
    if ((rc = objective_source(c))) return rc;
    if (n == 0) return SLBM_OK;
    int64_t t;
    double res;
    bool conv;
    int X = 0;
    if ((rc = run_loop(c, true, 0, n - 1, false, &t, &res, &conv, nullptr, &X))) return rc;
    c->adj_cur = X ^ 1;
    return SLBM_OK;
}

int solid_lbm_get_field(slbm_ctx* c, int32_t which, double* out, int32_t ptr_kind)
{
    if (!c) return SLBM_EINVAL;
    if (!out) return fail(c, SLBM_EINVAL, "out is NULL");
    const int64_t N = c->N;
    switch (which) {
        case SLBM_FIELD_DISP:
        case SLBM_FIELD_RESIDUAL:
        case SLBM_FIELD_STRESS:
            if (!c->prim_done) return fail(c, SLBM_ESTATE, "no completed primal_solve");
            if (which == SLBM_FIELD_DISP) return copy_out(c, out, c->dbar, 2 * N * sizeof(double), ptr_kind);
            if (which == SLBM_FIELD_RESIDUAL) return copy_out(c, out, c->r, 2 * N * sizeof(double), ptr_kind);
            hipLaunchKernelGGL(k_stress, dim3(grid_of(N)), dim3(kBlock), 0, c->stream, c->fbar, c->g,
                               c->masked ? c->code : (const int32_t*)nullptr, c->bnodes,
                               c->efield_on ? c->Efield : (const double*)nullptr, c->E_cur, c->nu, N, c->work);
            HIPCHK(c, hipGetLastError());
            return copy_out(c, out, c->work, 3 * N * sizeof(double), ptr_kind);
        case SLBM_FIELD_ADJ_DISP:
            if (!c->adj_done) return fail(c, SLBM_ESTATE, "no completed adjoint_solve");
            return copy_out(c, out, c->adisp, 2 * N * sizeof(double), ptr_kind);
        case SLBM_FIELD_POPS:
        case SLBM_FIELD_CUR_DISP: {
            if (!c->prim_valid) return fail(c, SLBM_ESTATE, "no primal state");
            double* pops = which == SLBM_FIELD_POPS ? c->work : nullptr;
            double* disp = which == SLBM_FIELD_CUR_DISP ? c->work : nullptr;
            if (c->masked)
                hipLaunchKernelGGL(k_gather_state<true>, dim3(grid_of(N)), dim3(kBlock), 0, c->stream,
                                   c->fbuf[c->prim_cur], c->g, c->code, c->nx, c->ny, N, c->inv_nx, pops, disp);
            else
                hipLaunchKernelGGL(k_gather_state<false>, dim3(grid_of(N)), dim3(kBlock), 0, c->stream,
                                   c->fbuf[c->prim_cur], c->g, c->code, c->nx, c->ny, N, c->inv_nx, pops, disp);
            HIPCHK(c, hipGetLastError());
            if (pops) return copy_out(c, out, pops, 8 * N * sizeof(double), ptr_kind);
            return copy_out(c, out, disp, 2 * N * sizeof(double), ptr_kind);
        }
        case SLBM_FIELD_ADJ_POPS:
            if (!c->adj_valid) return fail(c, SLBM_ESTATE, "no adjoint state");
            return copy_out(c, out, c->abuf[c->adj_cur], 8 * N * sizeof(double), ptr_kind);
        case SLBM_FIELD_AVG_POPS:
            if (!c->prim_done) return fail(c, SLBM_ESTATE, "no completed primal_solve");
            return copy_out(c, out, c->fbar, 8 * N * sizeof(double), ptr_kind);
        default:
            return fail(c, SLBM_EINVAL, "unknown field");
    }
}

int solid_lbm_time_sweeps(slbm_ctx* c, int32_t adjoint, int64_t n, double* ms)
{
    if (!c || !ms) return SLBM_EINVAL;
    if (n < 1) return fail(c, SLBM_EINVAL, "n must be >= 1");
    if (adjoint && !c->prim_done) return fail(c, SLBM_ESTATE, "adjoint sweeps need a completed primal_solve");
    if (!adjoint && !c->prim_valid) return fail(c, SLBM_ESTATE, "no primal state");
    if (adjoint && !c->adj_done) {
        int rc = adjoint_prepare(c);
        if (rc || (rc = objective_source(c))) return rc;
    }
    hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(1), 0, c->stream, c->status);
    SweepArgs a = base_args(c);
    a.g = adjoint ? c->asrc : c->g;
    a.scale = c->dx2 / c->cbar;
    double** bufs = adjoint ? c->abuf : c->fbuf;
    int cur = adjoint ? c->adj_cur : c->prim_cur;
    const int T = fused_steps(c);
    const int TL = tile_steps(c);
    if (TL > 1 && c->masked) {
        int rc = tile_lds_limits(c);
        if (rc) return rc;
    }
    if (TL > 1) {
        int rc = ensure_tile_plan(c, TL);
        if (rc) return rc;
    }
    HIPCHK(c, hipEventRecord(c->t0, c->stream));
    for (int64_t s = 0; s < n;) {
        a.src = bufs[cur];
        a.dst = bufs[cur ^ 1];
        if (T > 1 && n - s >= T) {
            launch_fused(c, adjoint != 0, a, T);
            s += T;
        } else if (TL > 1 && n - s >= 2) {
            const int k = (int)std::min<int64_t>(n - s, TL);
            launch_tile(c, adjoint != 0, a, k, TL);
            s += k;
        } else {
            launch_sweep(c, adjoint != 0, a, false);
            ++s;
        }
        cur ^= 1;
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipEventRecord(c->t1, c->stream));
    HIPCHK(c, hipEventSynchronize(c->t1));
    float f = 0.f;
    HIPCHK(c, hipEventElapsedTime(&f, c->t0, c->t1));
    *ms = f;
    // timing advances the state but leaves the outputs of the last completed
    // solve (d, r, averaged populations) untouched
    if (adjoint) c->adj_cur = cur;
    else c->prim_cur = cur;
    return SLBM_OK;
}

int adjoint_solve_vjp(slbm_ctx* c, const double* d_cot, double* grad, int32_t ptr_kind, slbm_solve_info* info)
{
    if (!c) return SLBM_EINVAL;
    if (!d_cot || !grad) return fail(c, SLBM_EINVAL, "d_cot and grad are required");
    if (!c->prim_done) return fail(c, SLBM_ESTATE, "adjoint_solve_vjp needs a completed primal_solve");
    int rc = copy_in(c, c->asrc, d_cot, 2 * c->N * sizeof(double), ptr_kind);
    if (rc) return rc;
    // outside the domain the displacement is not defined: its cotangent is ignored
    hipLaunchKernelGGL(k_axpb2, dim3(grid_of(2 * c->N)), dim3(kBlock), 0, c->stream, c->asrc,
                       (const double*)nullptr, c->masked ? c->code : (const int32_t*)nullptr, c->N, 1.0, c->asrc);
    HIPCHK(c, hipGetLastError());
    rc = do_adjoint(c, info, 1.0);
    if (rc < 0) return rc;
    int warn = rc;
    rc = assemble_grad(c, grad, ptr_kind);
    if (rc < 0) return rc;
    return warn;
}

int solid_lbm_restore_solve(slbm_ctx* c, const double* control, const double* avg_pops, int32_t ptr_kind)
{
    if (!c) return SLBM_EINVAL;
    if (!avg_pops) return fail(c, SLBM_EINVAL, "avg_pops is NULL");
    int rc = apply_control(c, control, ptr_kind);
    if (rc) return rc;
    if ((rc = copy_in(c, c->fbar, avg_pops, 8 * c->N * sizeof(double), ptr_kind))) return rc;
    if (c->masked)
        hipLaunchKernelGGL(k_restore<true>, dim3(grid_of(c->N)), dim3(kBlock), 0, c->stream, c->fbar, c->g, c->code,
                           c->target, c->obs, c->N, c->dbar, c->r, c->partial);
    else
        hipLaunchKernelGGL(k_restore<false>, dim3(grid_of(c->N)), dim3(kBlock), 0, c->stream, c->fbar, c->g, c->code,
                           c->target, c->obs, c->N, c->dbar, c->r, c->partial);
    HIPCHK(c, hipGetLastError());
    double s;
    if ((rc = sum_partials(c, &s))) return rc;
    c->J = 0.5 * s * c->dx2 / c->cbar;
    c->prim_done = true;
    c->adj_done = false;
    return SLBM_OK;
}

int solid_lbm_objective(slbm_ctx* c, double* J)
{
    if (!c || !J) return SLBM_EINVAL;
    if (!c->prim_done) return fail(c, SLBM_ESTATE, "no completed primal_solve");
    *J = c->J;
    return SLBM_OK;
}

int tangent_solve(slbm_ctx* c, const double* control, const double* direction, double* J, double* dJ,
                  int32_t ptr_kind, slbm_solve_info* info)
{
    if (!c) return SLBM_EINVAL;
    if (!J || !dJ) return fail(c, SLBM_EINVAL, "J and dJ are required");
    if (c->cv_window > 0) return fail(c, SLBM_EINVAL, "tangent_solve uses the K-lag convergence test only");
    auto w0 = std::chrono::steady_clock::now();
    int rc;
    if ((rc = tangent_buffers(c))) return rc;
    if ((rc = apply_control(c, control, ptr_kind))) return rc;
    // the primal state no longer belongs to the current control
    c->prim_valid = false;
    c->prim_done = false;
    c->adj_done = false;
    bool use_gdot, use_Edot;
    double E0dot;
    if ((rc = tangent_direction(c, direction, ptr_kind, &use_gdot, &use_Edot, &E0dot))) return rc;
    for (int k = 0; k < 2; ++k) {
        if ((rc = fill(c, c->tv[k], 8 * c->N, 0.0)) || (rc = fill(c, c->td[k], 8 * c->N, 0.0))) return rc;
    }
    if ((rc = fill(c, c->snap, 2 * c->N, 0.0)) || (rc = fill(c, c->snapd, 2 * c->N, 0.0))) return rc;
    TangentArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g = c->g;
    a.gdot = use_gdot ? c->gdot : nullptr;
    a.E = c->efield_on ? c->Efield : nullptr;
    a.Edot = use_Edot ? c->Edot : nullptr;
    a.code = c->code;
    a.bnodes = c->bnodes;
    a.snapv = c->snap;
    a.snapd = c->snapd;
    a.partial = c->tpart;
    a.status = c->status;
    a.nx = c->nx;
    a.ny = c->ny;
    a.N = c->N;
    a.E0 = c->E_cur;
    a.E0dot = E0dot;
    a.nu = c->nu;
    int64_t t;
    int X;
    double res, dms;
    bool conv;
    if ((rc = tangent_loop(c, a, &t, &X, &res, &conv, &dms))) return rc;
    if (c->masked)
        hipLaunchKernelGGL(k_tangent_finalize<true>, dim3(grid_of(c->N)), dim3(kBlock), 0, c->stream, c->tv[X],
                           c->td[X], c->tv[X ^ 1], c->td[X ^ 1], c->g, a.gdot, c->code, c->target, c->obs, c->nx,
                           c->ny, c->N, c->inv_nx, c->tpart);
    else
        hipLaunchKernelGGL(k_tangent_finalize<false>, dim3(grid_of(c->N)), dim3(kBlock), 0, c->stream, c->tv[X],
                           c->td[X], c->tv[X ^ 1], c->td[X ^ 1], c->g, a.gdot, c->code, c->target, c->obs, c->nx,
                           c->ny, c->N, c->inv_nx, c->tpart);
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL(k_sum_partials2, dim3(1), dim3(kBlock), 0, c->stream, c->tpart, c->nblk, c->work);
    HIPCHK(c, hipGetLastError());
    double sums[2];
    HIPCHK(c, hipMemcpyAsync(sums, c->work, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *J = 0.5 * sums[0] * c->dx2 / c->cbar;
    *dJ = sums[1] * c->dx2 / c->cbar;
    auto w1 = std::chrono::steady_clock::now();
    if (info) {
        info->steps = t;
        info->sweeps = t + 1;
        info->residual = c->tol > 0.0 ? res : 0.0;
        info->wall_s = std::chrono::duration<double>(w1 - w0).count();
        info->device_ms = dms;
        info->converged = conv ? 1 : 0;
    }
    return (c->tol > 0.0 && !conv) ? SLBM_NOT_CONVERGED : SLBM_OK;
}

int solid_lbm_set_progress(slbm_ctx* c, slbm_progress_fn fn, void* user, double every_s)
{
    if (!c) return SLBM_EINVAL;
    if (!(every_s >= 0.0)) return fail(c, SLBM_EINVAL, "every_s must be >= 0");
    c->progress = fn;
    c->progress_user = user;
    c->progress_every = every_s;
    return SLBM_OK;
}

int solid_lbm_set_tiles(slbm_ctx* c, int32_t tile_w, int32_t tile_h)
{
    if (!c) return SLBM_EINVAL;
    if ((tile_w == 0) != (tile_h == 0) || tile_w < 0 || tile_h < 0)
        return fail(c, SLBM_EINVAL, "tile_w and tile_h must both be 0 (automatic) or both >= 1");
    if (tile_w > 0) {
        const int h = tile_halo(c);
        if ((tile_w + 2 * h) * (tile_h + 2 * h) > kTileMaxNodes)
            return fail(c, SLBM_EINVAL, "tile plus halo exceeds " + std::to_string(kTileMaxNodes) + " nodes");
    }
    c->tile_w = tile_w;
    c->tile_h = tile_h;
    return SLBM_OK;
}

int solid_lbm_set_tuning(slbm_ctx* c, int32_t steps_per_launch, int32_t rows_per_wave)
{
    if (!c) return SLBM_EINVAL;
    if (steps_per_launch < -1 || steps_per_launch > 8)
        return fail(c, SLBM_EINVAL, "steps_per_launch must be -1 (automatic) or 0 .. 8");
    if (!(c->masked || c->kind == SLBM_CTRL_E_NODAL) && c->tile_w == 0 && steps_per_launch > 1 &&
        (steps_per_launch & 1))
        return fail(c, SLBM_EINVAL, "periodic bulk problems fuse 2, 4, 6 or 8 steps per launch");
    if (c->tile_w > 0 && steps_per_launch > 1 &&
        (c->tile_w + 2 * steps_per_launch) * (c->tile_h + 2 * steps_per_launch) > kTileMaxNodes)
        return fail(c, SLBM_EINVAL, "tile plus halo exceeds " + std::to_string(kTileMaxNodes) + " nodes");
    if (rows_per_wave < 0) return fail(c, SLBM_EINVAL, "rows_per_wave must be >= 0");
    c->tb_T = steps_per_launch;
    c->tb_H = rows_per_wave;
    return SLBM_OK;
}

int solid_lbm_set_launch_timing(slbm_ctx* c, int32_t on)
{
    if (!c) return SLBM_EINVAL;
    c->lt.on = on != 0;
    return SLBM_OK;
}

const char* solid_lbm_last_error(const slbm_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

void solid_lbm_destroy(slbm_ctx* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    for (void* p : c->allocs) (void)hipFree(p);
    if (c->h_status) (void)hipHostFree(c->h_status);
    for (hipEvent_t e : {c->ev[0], c->ev[1], c->t0, c->t1})
        if (e) (void)hipEventDestroy(e);
    c->lt.destroy();
    delete c;
}

}  // extern "C"

// ======================================================================= batches
struct slbm_batch {
    std::vector<slbm_ctx*> ctx;
    hipStream_t stream = nullptr;
    Status* status = nullptr;      // one Status per instance, contiguous
    Status* h_status = nullptr;    // pinned, 2 slots of B
    BatchInst* d_inst = nullptr;
    std::vector<BatchInst> h_inst;
    int2* d_all = nullptr;         // every instance: (instance, block) of a single-step sweep,
                                   // wave-strip instances first (their single steps alone: n_all_strip)
    int2* d_tb = nullptr;          // wave-strip instances: (instance, strip) of a fused launch
    int2* d_tile = nullptr;        // tiled instances: (instance, tile) of a fused launch
    int2* static_tables = nullptr; // non-null during batch_objective_and_grad_noalloc: tables go there
    const int2* cur_tb = nullptr;  // tables of the current launches (own or static)
    const int2* cur_tile = nullptr;
    int64_t n_all = 0, n_all_strip = 0, n_tb = 0, tb_cap = 0, n_tile = 0, tile_cap = 0;
    int tb_T = -1, tb_H = 0;       // tuning of the wave strips (-1 / 0: automatic)
    int tl_T = -1;                 // steps per launch of the tiled instances (-1: automatic)
    int T = 1, H = 0;              // effective fused shape of the current tables (wave strips)
    int Tt = 1;                    // effective steps per tile launch (halo of the tiles)
    std::vector<char> tiled;       // per instance: fused by the LDS-tiled kernel
    bool any_masked = false, tile_attr = false;
    double tol = 0.0;
    int64_t max_steps = 0;
    hipEvent_t ev[2] = {nullptr, nullptr}, t0 = nullptr, t1 = nullptr;
    // persistent launches (solid_lbm_batch_set_persistent): one graph-captured
    // persistent kernel per launch instead of host-driven launches per round
    bool persist = false;
    int persist_rounds = 4096;     // rounds per persistent launch (one graph replay)
    PersistInst* d_pinst = nullptr;
    PersistState* d_pstate = nullptr;   // replicas: one state array per workgroup
    int64_t pstate_cap = 0;             // replicas allocated (workgroups x instances)
    PersistCtl* d_pctl = nullptr;
    PersistCtl* h_pctl = nullptr;  // pinned: the graph copies the control block here
    hipStream_t pstream = nullptr; // capture stream (the batch's stream may be the default one)
    hipEvent_t pev = nullptr;
    bool persist_attr = false;
    int64_t persist_launches = 0, persist_rounds_run = 0;   // of the last persistent half
    slbm_progress_fn progress = nullptr;   // optional report from the batch loops
    void* progress_user = nullptr;
    double progress_every = 0.0;
    std::string err;
    std::vector<void*> allocs;
};

namespace {

thread_local std::string g_batch_init_error;

int bfail(slbm_batch* b, int code, const std::string& msg)
{
    if (b) b->err = msg;
    else g_batch_init_error = msg;
    return code;
}

#define BHIPCHK(b, call)                                                                      \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return bfail(b, SLBM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

int balloc(slbm_batch* b, void** p, size_t bytes)
{
    hipError_t e = hipMalloc(p, bytes ? bytes : 8);
    if (e != hipSuccess) return bfail(b, SLBM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    b->allocs.push_back(*p);
    return SLBM_OK;
}

// Fused shape for the batch: periodic instances share one (T, H).
// Tiled instances fuse their own number of steps per launch (default 6: the
// 20 x 20 tiles of 32 x 32 regions, measured fastest at 384 x 231 and within
// a few per cent at 512 x 308, where 8 steps with 16 x 16 tiles take 1.1 -
// 1.5 times longer per step).
constexpr int kBatchTileSteps = 6;

void batch_shape(slbm_batch* b, int* T, int* H, int* Tt)
{
    *Tt = b->tl_T < 0 ? kBatchTileSteps : std::max(1, std::min(8, b->tl_T));
    int t = b->tb_T < 0 ? 8 : b->tb_T;
    if (t != 2 && t != 4 && t != 6 && t != 8) t = 1;
    int h = b->tb_H;
    if (h <= 0) {
        int maxny = 0;
        for (size_t i = 0; i < b->ctx.size(); ++i)
            if (!b->tiled[i]) maxny = std::max(maxny, b->ctx[i]->ny);
        h = maxny <= 1536 ? 24 : 48;
    }
    if (t > 1 && h < 2 * t) h = 2 * t;
    *T = t;
    *H = h;
}

// ---- launch tables without allocation (batch_objective_and_grad_noalloc)
// The fused launches' work-lists (strip and tile tables) of a no-allocation
// call live in this file-scope device array instead of memory the batch
// allocates.  Each device holds its own copy for the life of the process; in
// host code `scratch` only names the symbol: kernels and copies take the
// device address from hipGetSymbolAddress (static_tables_of), never the name.
constexpr int64_t kStaticTableEntries = 65536;   // (instance, item) pairs: 512 KiB
static __device__ __align__(256) int2 scratch[kStaticTableEntries];

std::mutex g_scratch_mu;
std::vector<int2*> g_scratch_dev;   // per device id: address of `scratch` there (null = not resolved)

// Device address of the static table array on the current device (resolved
// once per device, with that device current).
int static_tables_of(slbm_batch* b, int2** out)
{
    int dev = -1;
    BHIPCHK(b, hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        BHIPCHK(b, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_dev[dev] = static_cast<int2*>(p);
    }
    *out = g_scratch_dev[dev];
    return SLBM_OK;
}

// Entries of the fused strip and tile tables for the current tuning.
int64_t batch_table_entries(slbm_batch* b)
{
    int T, H, Tt;
    batch_shape(b, &T, &H, &Tt);
    const int tw = std::max(2, 32 - 2 * Tt);
    int64_t n = 0;
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        const slbm_ctx* c = b->ctx[i];
        if (b->tiled[i]) {
            if (Tt > 1) n += (int64_t)((c->nx + tw - 1) / tw) * ((c->ny + tw - 1) / tw);
        } else if (T > 1) {
            const int V = 64 - 2 * T, h = std::min(H, c->ny);
            n += (int64_t)((c->nx + V - 1) / V) * ((c->ny + h - 1) / h);
        }
    }
    return n;
}

// (Re)builds the per-instance table for the current controls, the fused
// strip table for shape (T, H) and the tile table for Tt steps per launch;
// uploads them.
int batch_tables(slbm_batch* b, bool adjoint)
{
    int T, H, Tt;
    batch_shape(b, &T, &H, &Tt);
    const int B = (int)b->ctx.size();
    // tiled instances: halo = Tt, 32 x 32 regions
    const int tw = std::max(2, 32 - 2 * Tt);
    std::vector<int2> tb, tl;
    for (int i = 0; i < B; ++i) {
        slbm_ctx* c = b->ctx[i];
        // tiled instances run with launch plans (not in the no-allocation call)
        const bool planned = b->tiled[i] && Tt > 1 && !b->static_tables && c->N < (int64_t)INT32_MAX;
        if (planned) {
            int rc = build_tile_plan(c, Tt, tw, tw, c->masked ? 1 : 0);
            if (rc) return bfail(b, rc, "instance " + std::to_string(i) + ": " + c->err);
        }
        BatchInst I;
        std::memset(&I, 0, sizeof(I));
        SweepArgs a = base_args(c);
        a.status = b->status + i;
        for (int par = 0; par < 2; ++par) {
            SweepArgs pa = a, aa = a;
            pa.src = c->fbuf[par];
            pa.dst = c->fbuf[par ^ 1];
            pa.g = c->g;
            aa.src = c->abuf[par];
            aa.dst = c->abuf[par ^ 1];
            aa.g = c->asrc;
            aa.scale = c->dx2 / c->cbar;
            I.prim[par] = pa;
            I.adj[par] = aa;
            for (int k = 0; k < 2; ++k) {
                const SweepArgs& s = k ? aa : pa;
                TBArgs t;
                t.src = s.src;
                t.dst = s.dst;
                t.g = s.g;
                t.status = b->status + i;
                t.nx = c->nx;
                t.ny = c->ny;
                t.H = std::min(H, c->ny);
                t.strips = (c->nx + (64 - 2 * std::max(T, 1)) - 1) / (64 - 2 * std::max(T, 1));
                t.N = c->N;
                t.k11 = s.k11;
                t.ks = s.ks;
                t.kd = s.kd;
                t.scale = s.scale;
                (k ? I.tadj : I.tprim)[par] = t;
                TileArgs l;
                std::memset(&l, 0, sizeof(l));
                l.src = s.src;
                l.dst = s.dst;
                l.g = s.g;
                l.E = s.E;
                l.code = s.code;
                l.bnodes = s.bnodes;
                l.status = b->status + i;
                l.nx = c->nx;
                l.ny = c->ny;
                l.N = c->N;
                l.k11 = s.k11;
                l.ks = s.ks;
                l.kd = s.kd;
                l.E0 = s.E0;
                l.nu = s.nu;
                l.scale = s.scale;
                l.tw = tw;
                l.th = tw;
                l.halo = Tt;
                l.steps = Tt;
                l.maxb = kTileMaxB;
                l.tiles_x = (c->nx + tw - 1) / tw;
                if (planned) {
                    l.plan = c->plan;
                    l.plan_rec = c->plan_rec;
                    l.plan_nst = c->plan_nst;
                }
                (k ? I.ladj : I.lprim)[par] = l;
            }
        }
        I.status = b->status + i;
        I.inv_nx = c->inv_nx;
        I.masked = c->masked ? 1 : 0;
        I.efield = c->efield_on ? 1 : 0;
        I.tiled = b->tiled[i] ? 1 : 0;
        I.nblk = c->nblk;
        if (!b->tiled[i] && T > 1) {
            int V = 64 - 2 * T;
            int sx = (c->nx + V - 1) / V, sy = (c->ny + std::min(H, c->ny) - 1) / std::min(H, c->ny);
            I.sx = sx;
            for (int k = 0; k < sx * sy; ++k) tb.push_back(make_int2(i, k));
        }
        if (b->tiled[i] && Tt > 1) {
            const int ntiles = ((c->nx + tw - 1) / tw) * ((c->ny + tw - 1) / tw);
            for (int k = 0; k < ntiles; ++k) tl.push_back(make_int2(i, k));
        }
        b->h_inst[i] = I;
    }
    (void)adjoint;
    BHIPCHK(b, hipMemcpyAsync(b->d_inst, b->h_inst.data(), B * sizeof(BatchInst), hipMemcpyHostToDevice, b->stream));
    int2* tb_dst = nullptr;
    int2* tl_dst = nullptr;
    if (b->static_tables) {
        // no-allocation path: both tables in the static device array
        if ((int64_t)(tb.size() + tl.size()) > kStaticTableEntries)
            return bfail(b, SLBM_EINVAL, "launch tables exceed the static table");
        tb_dst = b->static_tables;
        tl_dst = b->static_tables + tb.size();
    } else {
        if ((int64_t)tb.size() > b->tb_cap) {
            void* q = nullptr;
            int rc = balloc(b, &q, tb.size() * sizeof(int2));
            if (rc) return rc;
            b->d_tb = (int2*)q;
            b->tb_cap = (int64_t)tb.size();
        }
        if ((int64_t)tl.size() > b->tile_cap) {
            void* q = nullptr;
            int rc = balloc(b, &q, tl.size() * sizeof(int2));
            if (rc) return rc;
            b->d_tile = (int2*)q;
            b->tile_cap = (int64_t)tl.size();
        }
        tb_dst = b->d_tb;
        tl_dst = b->d_tile;
    }
    if (!tb.empty())
        BHIPCHK(b, hipMemcpyAsync(tb_dst, tb.data(), tb.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
    if (!tl.empty())
        BHIPCHK(b, hipMemcpyAsync(tl_dst, tl.data(), tl.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
    b->cur_tb = tb_dst;
    b->cur_tile = tl_dst;
    if (!tl.empty() && !b->tile_attr) {
        const int lmax = (int)tile_lds_bytes(kTileMaxNodes, true);
        BHIPCHK(b, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sweep_tile_batch<false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lmax));
        BHIPCHK(b, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_sweep_tile_batch<true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lmax));
        b->tile_attr = true;
    }
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    b->n_tb = (int64_t)tb.size();
    b->n_tile = (int64_t)tl.size();
    b->T = T;
    b->H = H;
    b->Tt = Tt;
    return SLBM_OK;
}

void launch_batch_step(slbm_batch* b, bool adjoint, const int2* table, int64_t nblocks, int pp, int pl,
                       uint64_t lo, uint64_t hi)
{
    if (nblocks <= 0) return;
    if (adjoint)
        hipLaunchKernelGGL(k_sweep_batch<true>, dim3((unsigned)nblocks), dim3(kBlock), 0, b->stream, b->d_inst,
                           table, pp, pl, lo, hi);
    else
        hipLaunchKernelGGL(k_sweep_batch<false>, dim3((unsigned)nblocks), dim3(kBlock), 0, b->stream, b->d_inst,
                           table, pp, pl, lo, hi);
}

void launch_batch_fused(slbm_batch* b, bool adjoint, int pp)
{
    dim3 grid((unsigned)b->n_tb), block(64);
#define BTB_CASE(TT)                                                                                       \
    case TT:                                                                                               \
        if (adjoint) hipLaunchKernelGGL((k_sweep_tb_batch<TT, true>), grid, block, 0, b->stream, b->d_inst, \
                                        b->cur_tb, pp);                                                    \
        else hipLaunchKernelGGL((k_sweep_tb_batch<TT, false>), grid, block, 0, b->stream, b->d_inst,       \
                                b->cur_tb, pp);                                                            \
        break;
    switch (b->T) {
        BTB_CASE(2)
        BTB_CASE(4)
        BTB_CASE(6)
        BTB_CASE(8)
    }
#undef BTB_CASE
}

// steps (1 .. Tt) sweeps of every tiled instance
void launch_batch_tile(slbm_batch* b, bool adjoint, int pl, int steps)
{
    if (b->n_tile <= 0) return;
    const int w = std::max(2, 32 - 2 * b->Tt) + 2 * b->Tt;
    const size_t lds = tile_lds_bytes(w * w, b->any_masked);
    dim3 grid((unsigned)b->n_tile), block(kTileBlock);
    if (adjoint)
        hipLaunchKernelGGL(k_sweep_tile_batch<true>, grid, block, lds, b->stream, b->d_inst, b->cur_tile, pl, steps);
    else
        hipLaunchKernelGGL(k_sweep_tile_batch<false>, grid, block, lds, b->stream, b->d_inst, b->cur_tile, pl, steps);
}

// run plain steps (no checks) of every instance: the wave-strip class in
// fused launches of T steps and single steps for the rest, the tiled class
// in launches of up to Tt steps; each class flips its buffer parity per launch.
void batch_plain_steps(slbm_batch* b, bool adjoint, int64_t run, int& pp, int& pl)
{
    const bool strips = b->n_all_strip > 0;
    if (strips) {
        int64_t left = run;
        if (b->T > 1 && b->n_tb > 0)
            for (; left >= b->T; left -= b->T) {
                launch_batch_fused(b, adjoint, pp);
                pp ^= 1;
            }
        for (; left > 0; --left) {
            launch_batch_step(b, adjoint, b->d_all, b->n_all_strip, pp, pl, 0, 0);
            pp ^= 1;
        }
    }
    if (b->n_all > b->n_all_strip) {
        if (b->Tt > 1 && b->n_tile > 0) {
            for (int64_t left = run; left > 0; left -= b->Tt) {
                launch_batch_tile(b, adjoint, pl, (int)std::min<int64_t>(left, b->Tt));
                pl ^= 1;
            }
        } else {
            for (int64_t j = 0; j < run; ++j) {
                launch_batch_step(b, adjoint, b->d_all + b->n_all_strip, b->n_all - b->n_all_strip, pp, pl, 0, 0);
                pl ^= 1;
            }
        }
    }
}

// Advances every instance from buffer 0 in lock-step (step index s), each
// with its own residual checks every K_i steps and its own stop flag; plain
// runs between checks are fused (wave strips T steps per launch, tiles Tt).
// Afterwards, for each instance: t (its final step), X (buffer holding its
// input of step t) and whether it converged.
int batch_loop_persist(slbm_batch* b, bool adjoint, std::vector<int64_t>& t_out, std::vector<int>& x_out,
                       std::vector<char>& conv, std::vector<double>& res, double* dev_ms);

int batch_loop(slbm_batch* b, bool adjoint, std::vector<int64_t>& t_out, std::vector<int>& x_out,
               std::vector<char>& conv, std::vector<double>& res, double* dev_ms)
{
    if (b->persist && !b->static_tables) return batch_loop_persist(b, adjoint, t_out, x_out, conv, res, dev_ms);
    const int B = (int)b->ctx.size();
    hipLaunchKernelGGL(k_status_reset_all, dim3((B + 127) / 128), dim3(128), 0, b->stream, b->status, B);
    BHIPCHK(b, hipGetLastError());
    int rc = batch_tables(b, adjoint);
    if (rc) return rc;
    const int64_t last = b->max_steps;
    const bool use_tol = b->tol > 0.0;
    std::vector<int64_t> K(B);
    for (int i = 0; i < B; ++i) K[i] = b->ctx[i]->K;
    std::vector<char> active(B, 1);
    std::vector<CheckLog> checks(B);
    std::vector<int> last_in(B, 0);
    int pp = 0, pl = 0, slot = 0, polls = 0;
    int64_t s = 0, slot_step[2] = {0, 0};   // the step of the check each status slot holds
    auto last_report = std::chrono::steady_clock::now();
    BHIPCHK(b, hipEventRecord(b->t0, b->stream));
    auto any_active = [&]() {
        for (char a : active)
            if (a) return true;
        return false;
    };
    while (s <= last && any_active()) {
        uint64_t lo = 0, hi = 0;
        if (use_tol && s > 0)
            for (int i = 0; i < B; ++i)
                if (active[i] && s % K[i] == 0) (i < 64 ? lo : hi) |= 1ull << (i & 63);
        if (lo || hi || s == last) {
            launch_batch_step(b, adjoint, b->d_all, b->n_all, pp, pl, lo, hi);
            for (int i = 0; i < B; ++i) {
                int par = b->tiled[i] ? pl : pp;
                if ((i < 64 ? (lo >> i) : (hi >> (i - 64))) & 1ull) checks[i].add(s, par);
                if (s == last) last_in[i] = par;
            }
            if (lo || hi) {
                hipLaunchKernelGGL(k_residual_batch, dim3(B), dim3(kBlock), 0, b->stream, b->d_inst,
                                   adjoint ? 1 : 0, lo, hi, b->tol, s);
                BHIPCHK(b, hipMemcpyAsync(b->h_status + slot * B, b->status, B * sizeof(Status),
                                          hipMemcpyDeviceToHost, b->stream));
                BHIPCHK(b, hipEventRecord(b->ev[slot], b->stream));
                slot_step[slot] = s;
                if (polls >= 1) {
                    BHIPCHK(b, hipEventSynchronize(b->ev[slot ^ 1]));
                    double worst = -1.0;   // of the running instances with a completed check
                    for (int i = 0; i < B; ++i) {
                        const Status& h = b->h_status[(slot ^ 1) * B + i];
                        if (h.stop) active[i] = 0;
                        else if (active[i] && h.t_last >= 0) worst = std::max(worst, h.res);
                    }
                    if (b->progress && worst >= 0.0) {
                        auto now = std::chrono::steady_clock::now();
                        if (std::chrono::duration<double>(now - last_report).count() >= b->progress_every) {
                            last_report = now;
                            b->progress(b->progress_user, adjoint ? 1 : 0, slot_step[slot ^ 1], worst);
                        }
                    }
                }
                ++polls;
                slot ^= 1;
            }
            pp ^= 1;
            pl ^= 1;
            ++s;
            continue;
        }
        // plain steps until the next check of an active instance (or the final step)
        int64_t next = last;
        if (use_tol)
            for (int i = 0; i < B; ++i)
                if (active[i]) next = std::min(next, (s / K[i] + 1) * K[i]);
        const int64_t run = next - s;
        batch_plain_steps(b, adjoint, run, pp, pl);
        s += run;
        BHIPCHK(b, hipGetLastError());
    }
    BHIPCHK(b, hipEventRecord(b->t1, b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    float f = 0.f;
    BHIPCHK(b, hipEventElapsedTime(&f, b->t0, b->t1));
    if (dev_ms) *dev_ms = f;
    std::vector<Status> st(B);
    BHIPCHK(b, hipMemcpy(st.data(), b->status, B * sizeof(Status), hipMemcpyDeviceToHost));
    t_out.assign(B, last);
    x_out.assign(B, 0);
    conv.assign(B, 0);
    res.assign(B, 0.0);
    for (int i = 0; i < B; ++i) {
        res[i] = st[i].res;
        if (use_tol && st[i].stop) {
            const int xin = checks[i].find(st[i].t_conv);
            if (xin < 0) return bfail(b, SLBM_EHIP, "internal: converged step without a check sweep");
            t_out[i] = st[i].t_conv;
            x_out[i] = xin;
            conv[i] = 1;
        } else {
            x_out[i] = last_in[i];
        }
    }
    return SLBM_OK;
}

// The persistent path: per-instance constants, state reset, then graph
// replays of [reset of the launch's counters and barrier, the persistent
// kernel, a copy of the control block to pinned memory] until every instance
// has stopped.  Every instance runs as LDS tiles (periodic ones too), halo =
// the batch's tile steps Tt; results equal the host-driven loop's bit for bit
// (same node arithmetic, same checks).
int batch_loop_persist(slbm_batch* b, bool adjoint, std::vector<int64_t>& t_out, std::vector<int>& x_out,
                       std::vector<char>& conv, std::vector<double>& res, double* dev_ms)
{
    const int B = (int)b->ctx.size();
    hipLaunchKernelGGL(k_status_reset_all, dim3((B + 127) / 128), dim3(128), 0, b->stream, b->status, B);
    BHIPCHK(b, hipGetLastError());
    int rc = batch_tables(b, adjoint);
    if (rc) return rc;
    const int T = b->Tt > 1 ? b->Tt : 1;     // every instance runs as tiles of Tt steps
    const int tw = std::max(2, 32 - 2 * T);
    std::vector<PersistInst> pi(B);
    for (int i = 0; i < B; ++i) {
        const slbm_ctx* c = b->ctx[i];
        pi[i].K = c->K;
        pi[i].last = b->max_steps;
        pi[i].ntiles = ((c->nx + tw - 1) / tw) * ((c->ny + tw - 1) / tw);
        pi[i].nnb = (int32_t)((c->N + kPersistBlock - 1) / kPersistBlock);
        pi[i].halo = T;
        pi[i].pad = 0;
    }
    BHIPCHK(b, hipMemcpyAsync(b->d_pinst, pi.data(), B * sizeof(PersistInst), hipMemcpyHostToDevice, b->stream));
    // LDS: the tile regions (two copies for plates) and the staged boundary
    // records, within what a compute unit has beside the kernel's own arrays
    int maxb = kTileMaxB;
    if (b->any_masked) {
        hipFuncAttributes fa;
        BHIPCHK(b, hipFuncGetAttributes(&fa, adjoint ? reinterpret_cast<const void*>(&k_batch_persist<true>)
                                                     : reinterpret_cast<const void*>(&k_batch_persist<false>)));
        int dev0 = 0, lds_cu = 0;
        BHIPCHK(b, hipGetDevice(&dev0));
        BHIPCHK(b, hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev0));
        const int64_t room = (int64_t)lds_cu - (int64_t)fa.sharedSizeBytes - (int64_t)tile_lds_bytes(kTileMaxNodes, true, 0);
        maxb = (int)std::max<int64_t>(0, std::min<int64_t>(kTileMaxB, room / (int64_t)sizeof(BNode)));
    }
    const size_t lds = T > 1 ? tile_lds_bytes((tw + 2 * T) * (tw + 2 * T), b->any_masked, maxb) : 0;
    const void* fn = adjoint ? reinterpret_cast<const void*>(&k_batch_persist<true>)
                             : reinterpret_cast<const void*>(&k_batch_persist<false>);
    if (!b->persist_attr) {
        const int lmax = (int)tile_lds_bytes(kTileMaxNodes, true);
        BHIPCHK(b, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_persist<true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lmax));
        BHIPCHK(b, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_persist<false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lmax));
        b->persist_attr = true;
    }
    // every workgroup must be resident at once (grid barriers): as many as the
    // occupancy calculator admits on the device's compute units
    int dev = 0, cus = 0, per_cu = 0;
    BHIPCHK(b, hipGetDevice(&dev));
    BHIPCHK(b, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    BHIPCHK(b, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kPersistBlock, lds));
    const int G = per_cu * cus;
    if (G < 1) return bfail(b, SLBM_EHIP, "persistent batch kernel does not fit on a compute unit");
    if ((int64_t)G * B > b->pstate_cap) {
        void* q = nullptr;
        if ((rc = balloc(b, &q, (size_t)G * B * sizeof(PersistState)))) return rc;
        b->d_pstate = (PersistState*)q;
        b->pstate_cap = (int64_t)G * B;
    }
    hipLaunchKernelGGL(k_persist_init, dim3((unsigned)(((int64_t)G * B + 255) / 256)), dim3(256), 0, b->stream,
                       b->d_pstate, b->d_pctl, (int64_t)G * B);
    BHIPCHK(b, hipGetLastError());
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    const int use_tol = b->tol > 0.0 ? 1 : 0;
    // order the capture stream after the batch stream's work
    BHIPCHK(b, hipEventRecord(b->pev, b->stream));
    BHIPCHK(b, hipStreamWaitEvent(b->pstream, b->pev, 0));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    BHIPCHK(b, hipStreamBeginCapture(b->pstream, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(k_persist_begin, dim3(1), dim3(1), 0, b->pstream, b->d_pctl, b->persist_rounds);
    if (adjoint)
        hipLaunchKernelGGL(k_batch_persist<true>, dim3(G), dim3(kPersistBlock), lds, b->pstream, b->d_inst,
                           b->d_pinst, B, b->d_pstate, b->d_pctl, use_tol, b->tol, maxb);
    else
        hipLaunchKernelGGL(k_batch_persist<false>, dim3(G), dim3(kPersistBlock), lds, b->pstream, b->d_inst,
                           b->d_pinst, B, b->d_pstate, b->d_pctl, use_tol, b->tol, maxb);
    hipError_t ce = hipMemcpyAsync(b->h_pctl, b->d_pctl, sizeof(PersistCtl), hipMemcpyDeviceToHost, b->pstream);
    hipError_t ee = hipStreamEndCapture(b->pstream, &graph);
    if (ce != hipSuccess || ee != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return bfail(b, SLBM_EHIP, std::string("persistent batch graph capture: ") +
                                       hipGetErrorString(ce != hipSuccess ? ce : ee));
    }
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return bfail(b, SLBM_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    }
    int out = SLBM_OK;
    b->persist_launches = 0;
    auto last_report = std::chrono::steady_clock::now();
    hipError_t e = hipEventRecord(b->t0, b->pstream);
    while (e == hipSuccess) {
        e = hipGraphLaunch(exec, b->pstream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->pstream);
        if (e != hipSuccess) break;
        ++b->persist_launches;
        if (b->h_pctl->error) {
            out = bfail(b, SLBM_EHIP, "persistent batch kernel: a grid barrier timed out");
            break;
        }
        if (b->h_pctl->done) break;
        if (b->progress) {
            auto now = std::chrono::steady_clock::now();
            if (std::chrono::duration<double>(now - last_report).count() >= b->progress_every) {
                last_report = now;
                b->progress(b->progress_user, adjoint ? 1 : 0, b->h_pctl->rounds, -1.0);
            }
        }
        // every round advances a running instance by a step or a residual test
        if (b->h_pctl->rounds > 2 * (b->max_steps + 2) + 16) {
            out = bfail(b, SLBM_EHIP, "internal: persistent batch made no progress");
            break;
        }
    }
    if (e == hipSuccess) e = hipEventRecord(b->t1, b->pstream);
    if (e == hipSuccess) e = hipEventSynchronize(b->t1);
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return bfail(b, SLBM_EHIP, std::string("persistent batch launch: ") + hipGetErrorString(e));
    if (out) return out;
    b->persist_rounds_run = b->h_pctl->rounds;
    float f = 0.f;
    BHIPCHK(b, hipEventElapsedTime(&f, b->t0, b->t1));
    if (dev_ms) *dev_ms = f;
    std::vector<Status> st(B);
    std::vector<PersistState> ps(B);
    BHIPCHK(b, hipMemcpy(st.data(), b->status, B * sizeof(Status), hipMemcpyDeviceToHost));
    BHIPCHK(b, hipMemcpy(ps.data(), b->d_pstate, B * sizeof(PersistState), hipMemcpyDeviceToHost));   // replica 0
    t_out.assign(B, b->max_steps);
    x_out.assign(B, 0);
    conv.assign(B, 0);
    res.assign(B, 0.0);
    for (int i = 0; i < B; ++i) {
        res[i] = st[i].res;
        if (use_tol && st[i].stop) {
            if (ps[i].t_chk != st[i].t_conv) return bfail(b, SLBM_EHIP, "internal: converged step is not the last check");
            t_out[i] = st[i].t_conv;
            x_out[i] = ps[i].x_chk;
            conv[i] = 1;
        } else {
            x_out[i] = ps[i].x_last;
        }
    }
    return SLBM_OK;
}

int batch_adjoint(slbm_batch* b, double* const* grads, int ptr_kind, slbm_solve_info* ainfo);

int batch_solve(slbm_batch* b, const double* const* controls, int ptr_kind, double* J, double* const* grads,
                slbm_solve_info* pinfo, slbm_solve_info* ainfo, const double* const* init_disps = nullptr)
{
    const int B = (int)b->ctx.size();
    int rc;
    auto w0 = std::chrono::steady_clock::now();
    for (int i = 0; i < B; ++i) {
        slbm_ctx* c = b->ctx[i];
        const double* d0 = init_disps ? init_disps[i] : nullptr;
        if ((rc = apply_control(c, controls[i], ptr_kind)) || (rc = reset_primal(c, d0, ptr_kind)))
            return bfail(b, rc, "instance " + std::to_string(i) + ": " + c->err);
    }
    std::vector<int64_t> t;
    std::vector<int> X;
    std::vector<char> conv;
    std::vector<double> res;
    double dms = 0.0;
    if ((rc = batch_loop(b, false, t, X, conv, res, &dms))) return rc;
    bool all_conv = true;
    for (int i = 0; i < B; ++i) {
        slbm_ctx* c = b->ctx[i];
        if ((rc = finalize_primal(c, X[i]))) return bfail(b, rc, "instance " + std::to_string(i) + ": " + c->err);
        c->prim_cur = X[i] ^ 1;
        c->prim_done = true;
        c->adj_done = false;
        if (J) J[i] = c->J;
        all_conv = all_conv && conv[i];
    }
    auto w1 = std::chrono::steady_clock::now();
    if (pinfo)
        for (int i = 0; i < B; ++i) {
            pinfo[i].steps = t[i];
            pinfo[i].sweeps = t[i] + 1;
            pinfo[i].residual = res[i];
            pinfo[i].wall_s = std::chrono::duration<double>(w1 - w0).count();
            pinfo[i].device_ms = dms;
            pinfo[i].converged = conv[i];
        }
    if (!grads) return (b->tol > 0.0 && !all_conv) ? SLBM_NOT_CONVERGED : SLBM_OK;
    rc = batch_adjoint(b, grads, ptr_kind, ainfo);
    if (rc < 0) return rc;
    return (b->tol > 0.0 && (!all_conv || rc == SLBM_NOT_CONVERGED)) ? SLBM_NOT_CONVERGED : SLBM_OK;
}

// Adjoints and gradients of every instance after a completed batch primal.
int batch_adjoint(slbm_batch* b, double* const* grads, int ptr_kind, slbm_solve_info* ainfo)
{
    const int B = (int)b->ctx.size();
    int rc;
    auto w1 = std::chrono::steady_clock::now();
    for (int i = 0; i < B; ++i) {
        slbm_ctx* c = b->ctx[i];
        if (!c->prim_done) return bfail(b, SLBM_ESTATE, "instance " + std::to_string(i) + ": no completed primal");
        if ((rc = adjoint_prepare(c)) || (rc = objective_source(c)))
            return bfail(b, rc, "instance " + std::to_string(i) + ": " + c->err);
    }
    std::vector<int64_t> t;
    std::vector<int> X;
    std::vector<char> conv;
    std::vector<double> res;
    double dms = 0.0;
    bool all_conv = true;
    if ((rc = batch_loop(b, true, t, X, conv, res, &dms))) return rc;
    for (int i = 0; i < B; ++i) {
        slbm_ctx* c = b->ctx[i];
        if ((rc = adjoint_finalize(c, X[i], c->dx2 / c->cbar)) || (rc = assemble_grad(c, grads[i], ptr_kind)))
            return bfail(b, rc, "instance " + std::to_string(i) + ": " + c->err);
        all_conv = all_conv && conv[i];
    }
    auto w2 = std::chrono::steady_clock::now();
    if (ainfo)
        for (int i = 0; i < B; ++i) {
            ainfo[i].steps = t[i];
            ainfo[i].sweeps = t[i] + 1;
            ainfo[i].residual = res[i];
            ainfo[i].wall_s = std::chrono::duration<double>(w2 - w1).count();
            ainfo[i].device_ms = dms;
            ainfo[i].converged = conv[i];
        }
    return (b->tol > 0.0 && !all_conv) ? SLBM_NOT_CONVERGED : SLBM_OK;
}

}  // namespace

extern "C" {

int solid_lbm_batch_init(const slbm_problem* problems, int32_t count, slbm_batch** out)
{
    if (!out) return bfail(nullptr, SLBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!problems || count < 1 || count > 128) return bfail(nullptr, SLBM_EINVAL, "count must be 1..128");
    for (int i = 0; i < count; ++i) {
        const slbm_problem& p = problems[i];
        if (p.tol != problems[0].tol || p.max_steps != problems[0].max_steps || p.stream != problems[0].stream)
            return bfail(nullptr, SLBM_EINVAL, "all problems of a batch share tol, max_steps and stream");
    }
    slbm_batch* b = new slbm_batch();
    b->stream = (hipStream_t)problems[0].stream;
    b->tol = problems[0].tol;
    b->max_steps = problems[0].max_steps;
    for (int i = 0; i < count; ++i) {
        slbm_ctx* c = nullptr;
        int rc = solid_lbm_init(&problems[i], &c);
        if (rc) {
            std::string m = "instance " + std::to_string(i) + ": " + g_init_error;
            solid_lbm_batch_destroy(b);
            return bfail(nullptr, rc, m);
        }
        b->ctx.push_back(c);
        if (c->cv_window > 0) {
            solid_lbm_batch_destroy(b);
            return bfail(nullptr, SLBM_EINVAL, "instance " + std::to_string(i) +
                                                   ": batches use the K-lag convergence test only");
        }
    }
    int rc = SLBM_OK;
    void* q = nullptr;
    if (!rc && !(rc = balloc(b, &q, count * sizeof(Status)))) b->status = (Status*)q;
    if (!rc && !(rc = balloc(b, &q, count * sizeof(BatchInst)))) b->d_inst = (BatchInst*)q;
    std::vector<int2> all;
    b->tiled.assign(count, 0);
    for (int i = 0; i < count; ++i) {
        slbm_ctx* c = b->ctx[i];
        c->status = b->status + i;  // the instance's sweeps and the batch share its flag
        // plates and E fields fuse in LDS tiles, periodic uniform instances in
        // wave strips: in a batch the strips of many instances fill the GPU,
        // which removes their only handicap on small grids (measured on 72
        // periodic instances of 64..512: 66 us per batched step with strips,
        // 131 with tiles)
        b->tiled[i] = (c->masked || c->kind == SLBM_CTRL_E_NODAL) ? 1 : 0;
        if (c->masked) b->any_masked = true;
    }
    // single-step table: wave-strip instances first, so their single steps
    // alone are the table's first n_all_strip entries
    for (int cls = 0; cls < 2; ++cls)
        for (int i = 0; i < count; ++i)
            if (b->tiled[i] == cls)
                for (int64_t k = 0; k < b->ctx[i]->nblk; ++k) all.push_back(make_int2(i, (int)k));
    for (const int2& e : all)
        if (!b->tiled[e.x]) ++b->n_all_strip;
    if (!rc && !(rc = balloc(b, &q, all.size() * sizeof(int2)))) b->d_all = (int2*)q;
    if (!rc && hipMemcpy(b->d_all, all.data(), all.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess)
        rc = SLBM_EHIP;
    if (!rc && hipHostMalloc((void**)&b->h_status, 2 * count * sizeof(Status), hipHostMallocDefault) != hipSuccess)
        rc = SLBM_EHIP;
    if (!rc && (hipEventCreate(&b->ev[0]) != hipSuccess || hipEventCreate(&b->ev[1]) != hipSuccess ||
                hipEventCreate(&b->t0) != hipSuccess || hipEventCreate(&b->t1) != hipSuccess ||
                hipEventCreate(&b->pev) != hipSuccess))
        rc = SLBM_EHIP;
    // persistent path: per-instance constants and state, control block, capture stream
    if (!rc && !(rc = balloc(b, &q, count * sizeof(PersistInst)))) b->d_pinst = (PersistInst*)q;
    if (!rc && !(rc = balloc(b, &q, sizeof(PersistCtl)))) b->d_pctl = (PersistCtl*)q;
    if (!rc && hipHostMalloc((void**)&b->h_pctl, sizeof(PersistCtl), hipHostMallocDefault) != hipSuccess)
        rc = SLBM_EHIP;
    if (!rc && hipStreamCreateWithFlags(&b->pstream, hipStreamNonBlocking) != hipSuccess) rc = SLBM_EHIP;
    if (rc) {
        solid_lbm_batch_destroy(b);
        return bfail(nullptr, rc, "batch allocation failed");
    }
    std::memset(b->h_pctl, 0, sizeof(PersistCtl));
    b->n_all = (int64_t)all.size();
    b->h_inst.resize(count);
    // defined contents for timing sweeps before any solve
    for (auto* c : b->ctx) {
        for (double* a : {c->fbuf[0], c->fbuf[1], c->abuf[0], c->abuf[1]})
            if (!rc) rc = fill(c, a, 8 * c->N, 0.0);
        if (!rc) rc = fill(c, c->r, 2 * c->N, 0.0);
        if (!rc) rc = fill(c, c->asrc, 2 * c->N, 0.0);
        c->adj_valid = true;
    }
    if (rc || hipStreamSynchronize(b->stream) != hipSuccess) {
        solid_lbm_batch_destroy(b);
        return bfail(nullptr, rc ? rc : SLBM_EHIP, "batch initialisation failed");
    }
    *out = b;
    return SLBM_OK;
}

int batch_objective_and_grad(slbm_batch* b, const double* const* controls, double* J, double* const* grads,
                             int32_t ptr_kind, slbm_solve_info* primal_info, slbm_solve_info* adjoint_info)
{
    if (!b) return SLBM_EINVAL;
    if (!controls || !J) return bfail(b, SLBM_EINVAL, "controls and J are required");
    return batch_solve(b, controls, ptr_kind, J, grads, primal_info, adjoint_info);
}

int batch_objective_and_grad_from(slbm_batch* b, const double* const* controls, const double* const* init_disps,
                                  double* J, double* const* grads, int32_t ptr_kind, slbm_solve_info* primal_info,
                                  slbm_solve_info* adjoint_info)
{
    if (!b) return SLBM_EINVAL;
    if (!controls || !J) return bfail(b, SLBM_EINVAL, "controls and J are required");
    return batch_solve(b, controls, ptr_kind, J, grads, primal_info, adjoint_info, init_disps);
}

int batch_objective_and_grad_noalloc(slbm_batch* b, const double* const* controls, double* J,
                                     double* const* grads, int32_t ptr_kind, slbm_solve_info* primal_info,
                                     slbm_solve_info* adjoint_info)
{
    if (!b) return SLBM_EINVAL;
    if (!controls || !J) return bfail(b, SLBM_EINVAL, "controls and J are required");
    const int64_t need = batch_table_entries(b);
    if (need > kStaticTableEntries)
        return bfail(b, SLBM_EINVAL, "launch tables need " + std::to_string(need) + " entries; the static table holds " +
                                         std::to_string(kStaticTableEntries));
    int2* tables = nullptr;
    int rc = static_tables_of(b, &tables);
    if (rc) return rc;
    b->static_tables = tables;
    rc = batch_solve(b, controls, ptr_kind, J, grads, primal_info, adjoint_info);
    b->static_tables = nullptr;
    return rc;
}

int batch_gradient(slbm_batch* b, double* const* grads, int32_t ptr_kind, slbm_solve_info* adjoint_info)
{
    if (!b) return SLBM_EINVAL;
    if (!grads) return bfail(b, SLBM_EINVAL, "grads is required");
    for (int i = 0; i < (int)b->ctx.size(); ++i)
        if (!grads[i]) return bfail(b, SLBM_EINVAL, "grads[" + std::to_string(i) + "] is NULL");
    return batch_adjoint(b, grads, ptr_kind, adjoint_info);
}

int solid_lbm_batch_set_tuning(slbm_batch* b, int32_t steps_per_launch, int32_t rows_per_wave)
{
    if (!b) return SLBM_EINVAL;
    if (!(steps_per_launch == -1 || steps_per_launch == 0 || steps_per_launch == 1 || steps_per_launch == 2 ||
          steps_per_launch == 4 || steps_per_launch == 6 || steps_per_launch == 8))
        return bfail(b, SLBM_EINVAL, "steps_per_launch must be -1, 0, 1, 2, 4, 6 or 8");
    if (rows_per_wave < 0) return bfail(b, SLBM_EINVAL, "rows_per_wave must be >= 0");
    b->tb_T = steps_per_launch;
    b->tb_H = rows_per_wave;
    return SLBM_OK;
}

int solid_lbm_batch_set_tile_steps(slbm_batch* b, int32_t steps_per_launch)
{
    if (!b) return SLBM_EINVAL;
    if (steps_per_launch != -1 && (steps_per_launch < 1 || steps_per_launch > 8))
        return bfail(b, SLBM_EINVAL, "steps_per_launch must be -1 (automatic) or 1 .. 8");
    b->tl_T = steps_per_launch;
    return SLBM_OK;
}

int solid_lbm_batch_time_sweeps(slbm_batch* b, int32_t adjoint, int64_t n, double* ms)
{
    if (!b || !ms) return SLBM_EINVAL;
    if (n < 1) return bfail(b, SLBM_EINVAL, "n must be >= 1");
    const int B = (int)b->ctx.size();
    hipLaunchKernelGGL(k_status_reset_all, dim3((B + 127) / 128), dim3(128), 0, b->stream, b->status, B);
    int rc = batch_tables(b, adjoint != 0);
    if (rc) return rc;
    int pp = 0, pl = 0;
    BHIPCHK(b, hipEventRecord(b->t0, b->stream));
    batch_plain_steps(b, adjoint != 0, n, pp, pl);
    BHIPCHK(b, hipGetLastError());
    BHIPCHK(b, hipEventRecord(b->t1, b->stream));
    BHIPCHK(b, hipEventSynchronize(b->t1));
    float f = 0.f;
    BHIPCHK(b, hipEventElapsedTime(&f, b->t0, b->t1));
    *ms = f;
    // the states advanced by an unknown parity: later solves restart from their controls
    for (auto* c : b->ctx) c->prim_valid = false;
    return SLBM_OK;
}

int solid_lbm_batch_set_persistent(slbm_batch* b, int32_t on, int32_t rounds_per_launch)
{
    if (!b) return SLBM_EINVAL;
    if (rounds_per_launch < 0) return bfail(b, SLBM_EINVAL, "rounds_per_launch must be >= 0");
    b->persist = on != 0;
    b->persist_rounds = rounds_per_launch > 0 ? rounds_per_launch : 4096;
    return SLBM_OK;
}

int solid_lbm_batch_set_progress(slbm_batch* b, slbm_progress_fn fn, void* user, double every_s)
{
    if (!b) return SLBM_EINVAL;
    if (fn && !(every_s >= 0.0)) return bfail(b, SLBM_EINVAL, "every_s must be >= 0");
    b->progress = fn;
    b->progress_user = fn ? user : nullptr;
    b->progress_every = fn ? every_s : 0.0;
    return SLBM_OK;
}

int solid_lbm_batch_persistent_stats(const slbm_batch* b, int64_t* launches, int64_t* rounds)
{
    if (!b || !launches || !rounds) return SLBM_EINVAL;
    *launches = b->persist_launches;
    *rounds = b->persist_rounds_run;
    return SLBM_OK;
}

slbm_ctx* solid_lbm_batch_instance(slbm_batch* b, int32_t i)
{
    if (!b || i < 0 || i >= (int32_t)b->ctx.size()) return nullptr;
    return b->ctx[i];
}

const char* solid_lbm_batch_last_error(const slbm_batch* b) { return b ? b->err.c_str() : g_batch_init_error.c_str(); }

void solid_lbm_batch_destroy(slbm_batch* b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    else (void)hipDeviceSynchronize();
    for (auto* c : b->ctx) solid_lbm_destroy(c);
    if (b->pstream) (void)hipStreamSynchronize(b->pstream);
    for (void* p : b->allocs) (void)hipFree(p);
    if (b->h_status) (void)hipHostFree(b->h_status);
    if (b->h_pctl) (void)hipHostFree(b->h_pctl);
    for (hipEvent_t e : {b->ev[0], b->ev[1], b->t0, b->t1, b->pev})
        if (e) (void)hipEventDestroy(e);
    if (b->pstream) (void)hipStreamDestroy(b->pstream);
    delete b;
}

}  // extern "C"
