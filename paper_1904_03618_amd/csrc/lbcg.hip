// lbcg.hip -- host side of the C ABI declared in include/lbcg.h: parameter
// validation and derivation (FP64 on the host), device memory, tile tables,
// kernel launches.  Every arithmetic step of the method runs in the kernels of
// kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "kernels.hpp"

using namespace lbcg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(LBCG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr float kFp16Scale = 1024.0f;   // 2^10: typical deviations land in FP16's normal range

}  // namespace

struct lbcg_handle {
    hipStream_t stream = nullptr;
    int storage = LBCG_FP32, elem = 4, diag_every = 0, block = 256, persistent = 0;
    int ncases = 0;
    std::vector<DevCase> dc;
    std::vector<std::array<double, 2>> alpha_in;     // FP64 alpha_k per case (equilibrium start)
    std::vector<int> tile_begin, tile_count;
    DevCase *d_cases = nullptr;
    int2 *d_tiles = nullptr, *d_gtiles = nullptr;
    int ntiles = 0, ngtiles = 0;
    void *pop[2] = {nullptr, nullptr};
    int cur = 0;                       // pop[cur] holds the current level
    float4 *aux = nullptr, *ghost = nullptr;
    float *wallq = nullptr;            // per ghost entry: first-layer Qbar density factor (moving walls)
    float2 *rho2[2] = {nullptr, nullptr};
    // compact levels: the writers' recoloring data, double-buffered like rho2
    int level = LV_PAIR;
    float4 *dsc[2] = {nullptr, nullptr};
    float *crs[2] = {nullptr, nullptr};
    std::vector<uint8_t> pairlvl;      // per case: its current level is in pair format
    bool one_rsrc[2] = {false, false}; // per level format: every case's level fits one buffer resource
    double *partial = nullptr, *red = nullptr;
    int64_t steps = 0, total_nodes = 0, total_pop = 0, total_ghost = 0;
    float scale = 1.0f, inv_scale = 1.0f;
    bool has_wall = false;
    bool moving = false;               // some case has a moving wall: step kernels with the wall gain
    int walls = WALLS_NONE;            // which walls the cases have (selects the step-kernel instantiation)
    bool alive = true;
    // kernel timing (lbcg_timing): event pool and pending (kernel, start, end)
    bool timing = false;
    std::vector<hipEvent_t> events;
    size_t ev_used = 0;
    std::vector<int3> pending;
    double ms_acc[4] = {0, 0, 0, 0};
    int64_t launches[4] = {0, 0, 0, 0};
    // fused single-pass step
    bool fused = false;
    int zc = 16;
    int4 *d_ftiles = nullptr;
    int nftiles = 0;
    std::vector<int> ftile_begin, ftile_count;
    // captured step loops
    int graph_steps = 0;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int graph_parity = 0;              // steps & 1 at capture
};

namespace {

int validate(const lbcg_case &c, int idx)
{
    char buf[256];
    auto bad = [&](const char *what) {
        snprintf(buf, sizeof buf, "case %d: %s", idx, what);
        return fail(LBCG_EINVAL, buf);
    };
    if (c.nx < 1 || c.ny < 1 || c.nz < 1) return bad("dimensions must be >= 1");
    // the kernels address a case's arrays through 32-bit byte offsets: a pair of
    // FP32 population arrays (2 x 8 B per node) and the aux array (16 B per
    // node) must stay below 4 GiB
    if ((int64_t)c.nx * c.ny * c.nz > ((int64_t)1 << 28) - 64)
        return bad("more than 2^28 - 64 nodes in one case (32-bit buffer offsets)");
    int walls = 0;
    for (int a = 0; a < 3; ++a) {
        if (c.bc[a] != LBCG_PERIODIC && c.bc[a] != LBCG_WALL) return bad("bc must be PERIODIC or WALL");
        walls += c.bc[a] == LBCG_WALL;
    }
    if (walls > 1) return bad("at most one wall axis is supported");
    for (int k = 0; k < 2; ++k) {
        if (!(c.alpha[k] >= 0.0 && c.alpha[k] < 1.0)) return bad("alpha must lie in [0, 1)");
        if (!(c.rho_in[k] > 0.0)) return bad("rho_in must be > 0");
        if (!(c.tau_v[k] > 0.5)) return bad("tau_v must be > 1/2");
        if (!(c.theta_deg[k] > 0.0 && c.theta_deg[k] < 180.0)) return bad("theta must lie in (0, 180)");
        if (!std::isfinite(c.A[k])) return bad("A must be finite");
    }
    if (!(c.tau_e > 0.5 && c.tau_q > 0.5 && c.tau_pi > 0.5)) return bad("tau_e, tau_q, tau_pi must be > 1/2");
    if (!(c.delta > 0.0 && c.delta <= 1.0)) return bad("delta must lie in (0, 1]");
    const double pR = c.rho_in[0] * (1.0 - c.alpha[0]), pB = c.rho_in[1] * (1.0 - c.alpha[1]);
    if (std::fabs(pR - pB) > 1e-12 * std::max(pR, pB))
        return bad("pressure balance rho_R^in (1 - alpha_R) = rho_B^in (1 - alpha_B) violated");
    if (c.improved != 0 && c.improved != 1) return bad("improved must be 0 or 1");
    if (c.meq4 != 0 && c.meq4 != 1) return bad("meq4 must be 0 or 1");
    int wall_axis = -1;
    for (int a = 0; a < 3; ++a)
        if (c.bc[a] == LBCG_WALL) wall_axis = a;
    for (int sd = 0; sd < 2; ++sd)
        for (int a = 0; a < 3; ++a) {
            const double v = c.wall_u[sd][a];
            if (!std::isfinite(v)) return bad("wall_u must be finite");
            if (v != 0.0 && wall_axis < 0) return bad("wall_u needs a wall axis");
            if (v != 0.0 && a == wall_axis) return bad("wall_u must be tangential to the wall");
        }
    return LBCG_OK;
}

DevCase derive(const lbcg_case &c)
{
    DevCase d;
    std::memset(&d, 0, sizeof d);
    d.nx = c.nx; d.ny = c.ny; d.nz = c.nz;
    d.wall = -1;
    for (int a = 0; a < 3; ++a)
        if (c.bc[a] == LBCG_WALL) d.wall = a;
    d.N = c.nx * c.ny * c.nz;
    d.NS = (d.N + 63) / 64 * 64;      // every array of a case starts on a 128-byte boundary (64 FP16 values)
    d.plane = d.wall < 0 ? 0 : d.N / (d.wall == 0 ? c.nx : (d.wall == 1 ? c.ny : c.nz));
    d.improved = c.improved;
    // rows 16-18 of m^eq: rho (u_a^2 + u_b^2) times 1/2 (M f^eq) or 1/3 (the Appendix as printed)
    d.c16 = c.meq4 ? (float)(1.0 / 3.0) : 0.5f;
    for (int k = 0; k < 2; ++k) {
        const double al = c.alpha[k], cs2 = 0.5 * (1.0 - al);
        d.rin_inv[k] = (float)(1.0 / c.rho_in[k]);
        d.cs2[k] = (float)cs2;
        d.qc[k] = (float)(1.0 - 3.0 * cs2);
        d.phi[k][0] = (float)al;
        d.phi[k][1] = (float)((1.0 - al) / 12.0);
        d.phi[k][2] = (float)((1.0 - al) / 24.0);
        d.neg_tol[k] = (float)(-1e-3 * c.rho_in[k]);
        d.cot[k] = (float)std::tan((90.0 - c.theta_deg[k]) * M_PI / 180.0);
        // twice the odd part of f^{k,eq} per unit rho_k (e_i . U): 2 w_i [3 + 3 (3 c_s^2 - 1)(3|e_i|^2 - 5)]
        // with the third-order term of the improved equilibrium, 2 w_i 3 without it
        const double ex3 = c.improved ? 3.0 * (3.0 * cs2 - 1.0) : 0.0;
        d.wg[k][0] = (float)(2.0 / 18.0 * (3.0 - 2.0 * ex3));
        d.wg[k][1] = (float)(2.0 / 36.0 * (3.0 + ex3));
    }
    const double tR = c.tau_v[0], tB = c.tau_v[1], dl = c.delta;
    const double s1 = 2.0 * tR * tB / (tR + tB), s2 = 2.0 * (tR - s1) / dl, s3 = -s2 / (2.0 * dl);
    const double t2 = 2.0 * (s1 - tB) / dl, t3 = t2 / (2.0 * dl);
    d.tauR = (float)tR; d.tauB = (float)tB;
    d.s1 = (float)s1; d.s2 = (float)s2; d.s3 = (float)s3; d.t2 = (float)t2; d.t3 = (float)t3;
    d.delta = (float)dl;
    d.s_e = (float)(1.0 / c.tau_e); d.s_q = (float)(1.0 / c.tau_q); d.s_pi = (float)(1.0 / c.tau_pi);
    d.Asum = (float)(c.A[0] + c.A[1]);
    d.beta = (float)c.beta;
    for (int a = 0; a < 3; ++a) { d.F[a] = (float)c.force[a]; d.g[a] = (float)c.grav[a]; }
    d.rho_ref = (float)c.rho_ref;
    d.moving = 0;
    for (int sd = 0; sd < 2; ++sd)
        for (int a = 0; a < 3; ++a) {
            d.uw[sd][a] = (float)c.wall_u[sd][a];
            if (c.wall_u[sd][a] != 0.0) d.moving = 1;
        }
    return d;
}

StepArgs args_for(const lbcg_handle *h)
{
    StepArgs a;
    a.fin = h->pop[h->cur];
    a.fout = h->pop[h->cur ^ 1];
    a.aux = h->aux;
    a.ghost = h->ghost;
    a.wallq = h->wallq;
    // level t was written with the densities of level t-1 (rho2[(t+1)&1]);
    // the collision of level t records its own densities in rho2[t&1]
    a.rho_prev = h->rho2[(h->steps + 1) & 1];
    a.rho_cur = h->rho2[h->steps & 1];
    a.dsc_prev = h->dsc[(h->steps + 1) & 1];
    a.dsc_cur = h->dsc[h->steps & 1];
    a.crs_prev = h->crs[(h->steps + 1) & 1];
    a.crs_cur = h->crs[h->steps & 1];
    a.cases = h->d_cases;
    a.tiles = h->d_tiles;
    a.ntiles = h->ntiles;
    a.scale = h->scale;
    a.inv_scale = h->inv_scale;
    return a;
}

int next_event(lbcg_handle *h, hipEvent_t *ev, int *idx)
{
    if (h->ev_used == h->events.size()) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        h->events.push_back(e);
    }
    *idx = (int)h->ev_used++;
    *ev = h->events[*idx];
    return LBCG_OK;
}

// Record an event pair around launch() when timing is on.
template <class F>
int timed(lbcg_handle *h, int kernel, F &&launch)
{
    if (!h->timing) {
        launch();
        return LBCG_OK;
    }
    hipEvent_t e0, e1;
    int i0, i1;
    int rc = next_event(h, &e0, &i0);
    if (!rc) rc = next_event(h, &e1, &i1);
    if (rc) return rc;
    HIPCHK(hipEventRecord(e0, h->stream));
    launch();
    HIPCHK(hipEventRecord(e1, h->stream));
    h->pending.push_back(make_int3(kernel, i0, i1));
    return LBCG_OK;
}

// Level format of case c's current level.
int fmt_of(const lbcg_handle *h, int c)
{
    return h->level == LV_COMPACT && !h->pairlvl[c] ? LV_COMPACT : LV_PAIR;
}

// Call f(fmt, c0, c1) for each maximal run [c0, c1) of cases whose current
// levels share a format (one run unless a compact handle holds a case just
// (re)initialised in pair format).
template <class F>
int for_format_runs(const lbcg_handle *h, F &&f)
{
    for (int c0 = 0; c0 < h->ncases;) {
        const int fmt = fmt_of(h, c0);
        int c1 = c0 + 1;
        while (c1 < h->ncases && fmt_of(h, c1) == fmt) ++c1;
        const int rc = f(fmt, c0, c1);
        if (rc) return rc;
        c0 = c1;
    }
    return LBCG_OK;
}

template <int ST, int IN, int OUT, bool SO>
void launch_fused(lbcg_handle *h, hipStream_t st, const FusedArgs &fa, int grid)
{
    const dim3 g(grid), b(FTX * FTY);
    if (h->moving) hipLaunchKernelGGL((k_fused<ST, true, WALLS_Z, IN, OUT, SO>), g, b, 0, st, fa);
    else if (h->walls == WALLS_Z) hipLaunchKernelGGL((k_fused<ST, false, WALLS_Z, IN, OUT, SO>), g, b, 0, st, fa);
    else hipLaunchKernelGGL((k_fused<ST, false, WALLS_NONE, IN, OUT, SO>), g, b, 0, st, fa);
}

// A step that reads and writes one level format, with every case's level
// within one buffer resource, takes the single-resource instantiation (fewer
// scalar registers live); the one-off pair-to-compact conversion does not.
template <int ST, int IN, int OUT>
void launch_fused(lbcg_handle *h, hipStream_t st, const FusedArgs &fa, int grid)
{
    if constexpr (IN == OUT) {
        if (h->one_rsrc[IN]) {
            launch_fused<ST, IN, OUT, true>(h, st, fa, grid);
            return;
        }
    }
    launch_fused<ST, IN, OUT, false>(h, st, fa, grid);
}

// Workgroups of the handle's steady-state fused kernel that one CU holds at
// once (its registers and LDS), as the runtime computes it; 0 on failure.
template <int ST, int LV, bool SO>
int fused_blocks_per_cu(const lbcg_handle *h)
{
    int nb = 0;
    hipError_t e;
    if (h->moving)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fused<ST, true, WALLS_Z, LV, LV, SO>, FNT, 0);
    else if (h->walls == WALLS_Z)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fused<ST, false, WALLS_Z, LV, LV, SO>, FNT, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_fused<ST, false, WALLS_NONE, LV, LV, SO>, FNT, 0);
    return e == hipSuccess ? nb : 0;
}

template <int ST, int LV>
int fused_blocks_per_cu(const lbcg_handle *h)
{
    return h->one_rsrc[LV] ? fused_blocks_per_cu<ST, LV, true>(h) : fused_blocks_per_cu<ST, LV, false>(h);
}

int fused_blocks_per_cu(const lbcg_handle *h)
{
    const bool c = h->level == LV_COMPACT;
    switch (h->storage) {
    case LBCG_FP32: return c ? fused_blocks_per_cu<LBCG_FP32, LV_COMPACT>(h) : fused_blocks_per_cu<LBCG_FP32, LV_PAIR>(h);
    case LBCG_FP16S:
        return c ? fused_blocks_per_cu<LBCG_FP16S, LV_COMPACT>(h) : fused_blocks_per_cu<LBCG_FP16S, LV_PAIR>(h);
    default: return c ? fused_blocks_per_cu<LBCG_BF16S, LV_COMPACT>(h) : fused_blocks_per_cu<LBCG_BF16S, LV_PAIR>(h);
    }
}

template <int ST>
int launch_step(lbcg_handle *h, hipStream_t st)
{
    StepArgs a = args_for(h);
    if (h->fused) {
        int rc = for_format_runs(h, [&](int fmt, int c0, int c1) {
            const int t0 = h->ftile_begin[c0];
            const int nt = h->ftile_begin[c1 - 1] + h->ftile_count[c1 - 1] - t0;
            if (nt <= 0) return (int)LBCG_OK;
            FusedArgs fa{a, h->d_ftiles + t0, nt, h->zc};
            const int grid = h->persistent > 0 ? h->persistent : nt;
            return timed(h, 3, [&] {
                if (h->level == LV_PAIR) launch_fused<ST, LV_PAIR, LV_PAIR>(h, st, fa, grid);
                else if (fmt == LV_PAIR) launch_fused<ST, LV_PAIR, LV_COMPACT>(h, st, fa, grid);
                else launch_fused<ST, LV_COMPACT, LV_COMPACT>(h, st, fa, grid);
            });
        });
        if (rc) return rc;
        HIPCHK(hipGetLastError());
        std::fill(h->pairlvl.begin(), h->pairlvl.end(), (uint8_t)0);
        h->cur ^= 1;
        h->steps += 1;
        return LBCG_OK;
    }
    const int grid = h->persistent > 0 ? h->persistent : h->ntiles;
    // instantiation by what the handle's cases need: moving walls, walls on
    // any axis, walls only on z, no walls
    int rc = timed(h, 0, [&] {
        if (h->moving) hipLaunchKernelGGL((k_aux<ST, true, WALLS_ANY>), dim3(grid), dim3(h->block), 0, st, a);
        else if (h->walls == WALLS_ANY)
            hipLaunchKernelGGL((k_aux<ST, false, WALLS_ANY>), dim3(grid), dim3(h->block), 0, st, a);
        else if (h->walls == WALLS_Z)
            hipLaunchKernelGGL((k_aux<ST, false, WALLS_Z>), dim3(grid), dim3(h->block), 0, st, a);
        else hipLaunchKernelGGL((k_aux<ST, false, WALLS_NONE>), dim3(grid), dim3(h->block), 0, st, a);
    });
    if (!rc && h->has_wall)
        rc = timed(h, 1, [&] {
            hipLaunchKernelGGL(k_ghost, dim3(std::min(h->ngtiles, 65536)), dim3(256), 0, st, a,
                               (const int2 *)h->d_gtiles, h->ngtiles);
        });
    if (!rc)
        rc = timed(h, 2, [&] {
            if (h->moving)
                hipLaunchKernelGGL((k_collide<ST, true, WALLS_ANY>), dim3(grid), dim3(h->block), 0, st, a);
            else if (h->walls == WALLS_ANY)
                hipLaunchKernelGGL((k_collide<ST, false, WALLS_ANY>), dim3(grid), dim3(h->block), 0, st, a);
            else if (h->walls == WALLS_Z)
                hipLaunchKernelGGL((k_collide<ST, false, WALLS_Z>), dim3(grid), dim3(h->block), 0, st, a);
            else hipLaunchKernelGGL((k_collide<ST, false, WALLS_NONE>), dim3(grid), dim3(h->block), 0, st, a);
        });
    if (rc) return rc;
    HIPCHK(hipGetLastError());
    h->cur ^= 1;
    h->steps += 1;
    return LBCG_OK;
}

int step_once(lbcg_handle *h, hipStream_t st)
{
    switch (h->storage) {
    case LBCG_FP32: return launch_step<LBCG_FP32>(h, st);
    case LBCG_FP16S: return launch_step<LBCG_FP16S>(h, st);
    default: return launch_step<LBCG_BF16S>(h, st);
    }
}

// Capture graph_steps steps (from the current buffer parity) into a graph on
// the private capture stream; the handle's level is left unchanged.
int capture_graph(lbcg_handle *h)
{
    if (!h->capture_stream) HIPCHK(hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking));
    const int cur0 = h->cur;
    const int64_t steps0 = h->steps;
    const bool timing0 = h->timing;
    h->timing = false;
    HIPCHK(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
    int rc = LBCG_OK;
    for (int s = 0; s < h->graph_steps && rc == LBCG_OK; ++s) rc = step_once(h, h->capture_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->capture_stream, &g);
    h->cur = cur0;
    h->steps = steps0;
    h->timing = timing0;
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(LBCG_EDEVICE, std::string("stream capture: ") + hipGetErrorString(e));
    h->graph = g;
    HIPCHK(hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0));
    h->graph_parity = (int)(steps0 & 1);
    return LBCG_OK;
}

// FP64 sums over tiles [t0, t0 + nt) into h->red[0..5]; optional field exports.
// FP64 sums over the whole cases whose tiles are [t0, t0 + nt), one launch per
// run of cases with the same level format.
template <int ST>
int moments_impl(lbcg_handle *h, int t0, int nt, float *rR, float *rB, float *rN, float *ux, float *uy,
                 float *uz)
{
    StepArgs a = args_for(h);
    int rc = for_format_runs(h, [&](int fmt, int c0, int c1) {
        const int r0 = std::max(t0, h->tile_begin[c0]);
        const int r1 = std::min(t0 + nt, h->tile_begin[c1 - 1] + h->tile_count[c1 - 1]);
        if (r1 <= r0) return (int)LBCG_OK;
        double *part = h->partial + (size_t)6 * (r0 - t0);
        if (fmt == LV_COMPACT)
            hipLaunchKernelGGL((k_moments<ST, LV_COMPACT>), dim3(r1 - r0), dim3(h->block), 0, h->stream, a, r0, rR,
                               rB, rN, ux, uy, uz, part);
        else
            hipLaunchKernelGGL((k_moments<ST, LV_PAIR>), dim3(r1 - r0), dim3(h->block), 0, h->stream, a, r0, rR,
                               rB, rN, ux, uy, uz, part);
        return (int)LBCG_OK;
    });
    if (rc) return rc;
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(256), 0, h->stream, (const double *)h->partial, nt, h->red);
    HIPCHK(hipGetLastError());
    return LBCG_OK;
}

int moments_any(lbcg_handle *h, int t0, int nt, float *rR, float *rB, float *rN, float *ux, float *uy,
                float *uz)
{
    switch (h->storage) {
    case LBCG_FP32: return moments_impl<LBCG_FP32>(h, t0, nt, rR, rB, rN, ux, uy, uz);
    case LBCG_FP16S: return moments_impl<LBCG_FP16S>(h, t0, nt, rR, rB, rN, ux, uy, uz);
    default: return moments_impl<LBCG_BF16S>(h, t0, nt, rR, rB, rN, ux, uy, uz);
    }
}

int stability_check(lbcg_handle *h)
{
    int rc = moments_any(h, 0, h->ntiles, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (rc) return rc;
    double out[6];
    HIPCHK(hipMemcpyAsync(out, h->red, sizeof out, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (out[5] != 0.0 || !std::isfinite(out[0]) || !std::isfinite(out[1]))
        return fail(LBCG_EUNSTABLE, "unstable state (NaN/Inf or negative colour density) at step " +
                                        std::to_string(h->steps));
    return LBCG_OK;
}

void release(lbcg_handle *h)
{
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
    h->graph_exec = nullptr;
    h->graph = nullptr;
    h->capture_stream = nullptr;
    for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
    h->events.clear();
    (void)hipFree(h->d_cases);
    (void)hipFree(h->d_tiles);
    (void)hipFree(h->d_ftiles);
    (void)hipFree(h->d_gtiles);
    (void)hipFree(h->pop[0]);
    (void)hipFree(h->pop[1]);
    (void)hipFree(h->aux);
    (void)hipFree(h->ghost);
    (void)hipFree(h->wallq);
    (void)hipFree(h->rho2[0]);
    (void)hipFree(h->rho2[1]);
    for (int b = 0; b < 2; ++b) {
        (void)hipFree(h->dsc[b]);
        (void)hipFree(h->crs[b]);
    }
    (void)hipFree(h->partial);
    (void)hipFree(h->red);
}

template <int ST>
int init_case(lbcg_handle *h, int cid, const lbcg_case &c, const lbcg_fields &f)
{
    const int64_t N = h->dc[cid].N;
    const double *src[5] = {f.rhoR, f.rhoB, f.ux, f.uy, f.uz};
    double *dev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    double *tmp = nullptr;
    if (!f.on_device) {
        if (hipMalloc(&tmp, sizeof(double) * 5 * N) != hipSuccess) return fail(LBCG_ENOMEM, "init staging");
        for (int q = 0; q < 5; ++q) {
            dev[q] = tmp + q * N;
            if (hipMemcpyAsync(dev[q], src[q], sizeof(double) * N, hipMemcpyHostToDevice, h->stream) !=
                hipSuccess) {
                (void)hipFree(tmp);
                return fail(LBCG_EDEVICE, "init field copy");
            }
        }
    } else {
        for (int q = 0; q < 5; ++q) dev[q] = const_cast<double *>(src[q]);
    }
    StepArgs a = args_for(h);
    a.fout = h->pop[h->cur];                 // the level is written into the current buffer
    a.rho_cur = h->rho2[(h->steps + 1) & 1]; // and decoded with rho2[(t + 1) & 1]
    InitCase ic{{c.alpha[0], c.alpha[1]}, c.improved};
    hipLaunchKernelGGL(k_init<ST>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, h->stream, a, cid, ic,
                       (const double *)dev[0], (const double *)dev[1], (const double *)dev[2],
                       (const double *)dev[3], (const double *)dev[4]);
    hipError_t e = hipGetLastError();
    if (tmp) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(tmp);
    }
    if (e != hipSuccess) return fail(LBCG_EDEVICE, std::string("k_init: ") + hipGetErrorString(e));
    h->pairlvl[cid] = 1;                     // the start level is in pair format
    return LBCG_OK;
}

int init_any(lbcg_handle *h, int cid, const lbcg_case &c, const lbcg_fields &f)
{
    switch (h->storage) {
    case LBCG_FP32: return init_case<LBCG_FP32>(h, cid, c, f);
    case LBCG_FP16S: return init_case<LBCG_FP16S>(h, cid, c, f);
    default: return init_case<LBCG_BF16S>(h, cid, c, f);
    }
}

// Handles returned by lbcg_init and not yet freed.  A freed (or never
// issued) pointer is recognised without reading it.
std::mutex g_handles_mu;
std::unordered_set<const lbcg_handle *> g_handles;

bool live(const lbcg_handle *h)
{
    std::lock_guard<std::mutex> lk(g_handles_mu);
    return h && g_handles.count(h) && h->alive;
}

int check_handle(const lbcg_handle *h)
{
    {
        std::lock_guard<std::mutex> lk(g_handles_mu);
        if (!h || !g_handles.count(h)) return fail(LBCG_ESTATE, "invalid or freed handle");
    }
    if (!h->alive) return fail(LBCG_ESTATE, "invalid or freed handle");
    return LBCG_OK;
}

}  // namespace

// Checkpoint image: header, one descriptor per case (extents, array stride
// and offsets, and the format of its current level, in case order), then the
// current level's populations of every case (pop[cur]) and the writers'
// densities of that level (rho2[(t+1)&1]); a compact handle adds the writers'
// recoloring data of that level (dsc, crs).
namespace {
struct CkptHeader {
    char magic[8];
    int64_t version, storage, ncases, total_pop, total_nodes, steps, level;
};
struct CkptCase {
    int64_t nx, ny, nz, NS, pop_off, node_off;
    int64_t pair_level;          // state, not layout: not compared on load
};
constexpr char kMagic[8] = {'L', 'B', 'C', 'G', 'C', 'K', 'P', 'T'};
constexpr int64_t kCkptVersion = 4;

CkptCase ckpt_case(const lbcg_handle *h, int c)
{
    const DevCase &d = h->dc[c];
    return CkptCase{d.nx, d.ny, d.nz, d.NS, d.pop_off, d.node_off, h->pairlvl[c]};
}

int64_t ckpt_bytes(const lbcg_handle *h)
{
    int64_t b = (int64_t)sizeof(CkptHeader) + (int64_t)sizeof(CkptCase) * h->ncases +
                (int64_t)h->elem * h->total_pop + (int64_t)sizeof(float2) * h->total_nodes;
    if (h->level == LV_COMPACT) b += (int64_t)(sizeof(float4) + sizeof(float)) * h->total_nodes;
    return b;
}
}  // namespace

extern "C" {

const char *lbcg_last_error(void) { return g_err.c_str(); }

int lbcg_init(const lbcg_case *cases, int32_t n_cases, const lbcg_fields *init, const lbcg_options *opt,
              void *hip_stream, lbcg_handle **out)
{
    g_err.clear();
    if (!out) return fail(LBCG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!cases || !init || n_cases < 1) return fail(LBCG_EINVAL, "cases/init NULL or n_cases < 1");
    lbcg_options o = {LBCG_FP32, 0, 256, 0, LBCG_KERNEL_AUTO, 0, 0, 0};
    if (opt) o = *opt;
    if (o.graph_steps < 0) return fail(LBCG_EINVAL, "graph_steps must be >= 0");
    if (o.kernel < LBCG_KERNEL_AUTO || o.kernel > LBCG_KERNEL_FUSED) return fail(LBCG_EINVAL, "unknown kernel");
    if (o.zchunk < 0) return fail(LBCG_EINVAL, "zchunk must be >= 0");
    if (o.level < LBCG_LEVEL_AUTO || o.level > LBCG_LEVEL_COMPACT) return fail(LBCG_EINVAL, "unknown level format");
    if (o.storage != LBCG_FP32 && o.storage != LBCG_FP16S && o.storage != LBCG_BF16S)
        return fail(LBCG_EINVAL, "unknown storage format");
    if (o.block_nodes == 0) o.block_nodes = 256;
    if (o.block_nodes < 64 || o.block_nodes > 256 || o.block_nodes % 64)
        return fail(LBCG_EINVAL, "block_nodes must be 64, 128, 192 or 256");
    if (o.diag_every < 0 || o.persistent_blocks < 0) return fail(LBCG_EINVAL, "negative option");
    for (int c = 0; c < n_cases; ++c) {
        int rc = validate(cases[c], c);
        if (rc) return rc;
        const lbcg_fields &f = init[c];
        if (!f.rhoR || !f.rhoB || !f.ux || !f.uy || !f.uz) return fail(LBCG_EINVAL, "NULL init field");
    }

    lbcg_handle *h = new lbcg_handle();
    h->stream = (hipStream_t)hip_stream;
    h->storage = o.storage;
    h->elem = o.storage == LBCG_FP32 ? 4 : 2;
    h->diag_every = o.diag_every;
    h->block = o.block_nodes;
    h->persistent = o.persistent_blocks;
    h->ncases = n_cases;
    h->scale = o.storage == LBCG_FP16S ? kFp16Scale : 1.0f;
    h->inv_scale = 1.0f / h->scale;

    std::vector<int2> tiles, gtiles;
    for (int c = 0; c < n_cases; ++c) {
        DevCase d = derive(cases[c]);
        d.pop_off = h->total_pop;
        d.node_off = h->total_nodes;
        d.ghost_off = h->total_ghost;
        h->total_pop += (int64_t)2 * Q * d.NS;
        h->total_nodes += d.NS;
        h->total_ghost += (int64_t)2 * d.plane;
        if (d.wall >= 0) h->has_wall = true;
        if (d.wall >= 0) h->walls = std::max(h->walls, d.wall == 2 ? WALLS_Z : WALLS_ANY);
        if (d.moving) h->moving = true;
        h->tile_begin.push_back((int)tiles.size());
        for (int n0 = 0; n0 < d.N; n0 += h->block) tiles.push_back(make_int2(c, n0));
        h->tile_count.push_back((int)tiles.size() - h->tile_begin.back());
        for (int e0 = 0; e0 < 2 * d.plane; e0 += 256) gtiles.push_back(make_int2(c, e0));
        h->dc.push_back(d);
        h->alpha_in.push_back({cases[c].alpha[0], cases[c].alpha[1]});
    }
    h->ntiles = (int)tiles.size();
    h->ngtiles = (int)gtiles.size();

    // fused eligibility: walls, if any, only on z
    bool eligible = true;
    for (const DevCase &d : h->dc)
        if (d.wall == 0 || d.wall == 1) eligible = false;
    if (o.kernel == LBCG_KERNEL_FUSED && !eligible) {
        delete h;
        return fail(LBCG_EINVAL, "fused kernel needs walls, if any, on the z axis");
    }
    // AUTO takes the fused step wherever it applies (measured faster than the
    // two-pass step on the benchmark boxes) and the two-pass step otherwise.
    h->fused = eligible && (o.kernel == LBCG_KERNEL_FUSED || o.kernel == LBCG_KERNEL_AUTO);
    if (o.level == LBCG_LEVEL_COMPACT && !h->fused) {
        delete h;
        return fail(LBCG_EINVAL, "the compact level format needs the fused step");
    }
    // AUTO: the compact format for FP32 with the fused step (measured faster
    // than pairs there); the 16-bit forms keep pairs (their compact rings
    // leave 2 instead of 3 waves per SIMD and measured slower)
    h->level = h->fused && (o.level == LBCG_LEVEL_COMPACT || (o.level == LBCG_LEVEL_AUTO && o.storage == LBCG_FP32))
                   ? LV_COMPACT
                   : LV_PAIR;
    h->pairlvl.assign(n_cases, 1);
    // level bytes: pairs 19 NS pairs, compact levels 20 NS values
    h->one_rsrc[LV_PAIR] = h->one_rsrc[LV_COMPACT] = true;
    for (const DevCase &d : h->dc) {
        const int64_t elem = o.storage == LBCG_FP32 ? 4 : 2, lim = (int64_t)1 << 31;
        if ((int64_t)38 * d.NS * elem >= lim) h->one_rsrc[LV_PAIR] = false;
        if ((int64_t)20 * d.NS * elem >= lim) h->one_rsrc[LV_COMPACT] = false;
    }
    h->zc = o.zchunk;
    if (h->zc == 0 && h->fused) {
        // default chunk: a workgroup's tile of zc planes pulls zc + 2 planes,
        // and a launch of T tiles on S workgroup slots (CUs x workgroups of
        // this kernel per CU) takes about ceil(T / S) such tiles in turn, so
        // the chunk (8 .. 128 planes for FP32, 8 .. 64 for the 16-bit forms)
        // minimises ceil(T / S) (zc + 2), the longer chunk on a tie; where the
        // longest chunk already leaves two rounds or more it is taken.
        // Measured: 128 x 128 x 512 FP16S 43 planes (one tile per slot) 0.449
        // ms against 0.465 at 16; the 128^3 droplet FP16S 11 planes 0.1225
        // against 0.134; FP32 there 64 and 16, the 256 x 256 x 1024 box 128
        // and 64, as before.
        int dev = 0, ncu = 0;
        const int nb = fused_blocks_per_cu(h);
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0 ||
            nb <= 0) {
            delete h;
            return fail(LBCG_EDEVICE, "occupancy query of the fused kernel failed");
        }
        const int64_t slots = (int64_t)ncu * nb;
        auto tiles = [&](int zc) {
            int64_t n = 0;
            for (const DevCase &d : h->dc)
                n += (int64_t)((d.nx + FTX - 1) / FTX) * ((d.ny + FTY - 1) / FTY) * ((d.nz + zc - 1) / zc);
            return n;
        };
        const int cap = o.storage == LBCG_FP32 ? 128 : 64;
        h->zc = cap;
        if (tiles(cap) < 2 * slots) {
            int64_t best = -1;
            for (int zc = cap; zc >= 8; --zc) {
                const int64_t cost = (tiles(zc) + slots - 1) / slots * (zc + 2);
                if (best < 0 || cost < best) {
                    best = cost;
                    h->zc = zc;
                }
            }
        }
    } else if (h->zc == 0) {
        h->zc = 16;                                  // not used by the two-pass step
    }
    h->graph_steps = o.graph_steps + (o.graph_steps & 1);
    std::vector<int4> ftiles;
    for (int c = 0; c < n_cases; ++c) {
        h->ftile_begin.push_back((int)ftiles.size());
        const DevCase &d = h->dc[c];
        if (h->fused)
            for (int z0 = 0; z0 < d.nz; z0 += h->zc)
                for (int y0 = 0; y0 < d.ny; y0 += FTY)
                    for (int x0 = 0; x0 < d.nx; x0 += FTX) ftiles.push_back(make_int4(c, x0, y0, z0));
        h->ftile_count.push_back((int)ftiles.size() - h->ftile_begin.back());
    }
    h->nftiles = (int)ftiles.size();

    auto alloc = [&](void **p, size_t bytes) {
        if (bytes == 0) bytes = 256;
        return hipMalloc(p, bytes) == hipSuccess;
    };
    bool ok = alloc((void **)&h->d_cases, sizeof(DevCase) * n_cases) &&
              alloc((void **)&h->d_tiles, sizeof(int2) * tiles.size()) &&
              alloc((void **)&h->d_gtiles, sizeof(int2) * std::max<size_t>(1, gtiles.size())) &&
              alloc(&h->pop[0], (size_t)h->elem * h->total_pop) &&
              alloc(&h->pop[1], (size_t)h->elem * h->total_pop) &&
              alloc((void **)&h->aux, sizeof(float4) * h->total_nodes) &&
              alloc((void **)&h->ghost, sizeof(float4) * std::max<int64_t>(1, h->total_ghost)) &&
              alloc((void **)&h->wallq, sizeof(float) * std::max<int64_t>(1, h->total_ghost)) &&
              alloc((void **)&h->partial, sizeof(double) * 6 * (size_t)h->ntiles) &&
              alloc((void **)&h->red, sizeof(double) * 8) &&
              alloc((void **)&h->d_ftiles, sizeof(int4) * std::max<size_t>(1, ftiles.size()));
    if (ok)
        ok = alloc((void **)&h->rho2[0], sizeof(float2) * h->total_nodes) &&
             alloc((void **)&h->rho2[1], sizeof(float2) * h->total_nodes);
    for (int b = 0; b < 2 && ok && h->level == LV_COMPACT; ++b)
        ok = alloc((void **)&h->dsc[b], sizeof(float4) * h->total_nodes) &&
             alloc((void **)&h->crs[b], sizeof(float) * h->total_nodes);
    if (!ok) {
        release(h);
        delete h;
        return fail(LBCG_ENOMEM, "device allocation failed");
    }
    int rc = LBCG_OK;
    if (hipMemcpyAsync(h->d_cases, h->dc.data(), sizeof(DevCase) * n_cases, hipMemcpyHostToDevice,
                       h->stream) != hipSuccess ||
        hipMemcpyAsync(h->d_tiles, tiles.data(), sizeof(int2) * tiles.size(), hipMemcpyHostToDevice,
                       h->stream) != hipSuccess ||
        (!gtiles.empty() && hipMemcpyAsync(h->d_gtiles, gtiles.data(), sizeof(int2) * gtiles.size(),
                                           hipMemcpyHostToDevice, h->stream) != hipSuccess) ||
        (!ftiles.empty() && hipMemcpyAsync(h->d_ftiles, ftiles.data(), sizeof(int4) * ftiles.size(),
                                           hipMemcpyHostToDevice, h->stream) != hipSuccess))
        rc = fail(LBCG_EDEVICE, "table upload failed");
    // the padding between a case's population arrays is never read; clearing it
    // keeps checkpoint images a function of the state alone
    for (int b = 0; b < 2 && rc == LBCG_OK; ++b)
        if (hipMemsetAsync(h->pop[b], 0, (size_t)h->elem * h->total_pop, h->stream) != hipSuccess ||
            hipMemsetAsync(h->rho2[b], 0, sizeof(float2) * h->total_nodes, h->stream) != hipSuccess ||
            (h->dsc[b] && hipMemsetAsync(h->dsc[b], 0, sizeof(float4) * h->total_nodes, h->stream) != hipSuccess) ||
            (h->crs[b] && hipMemsetAsync(h->crs[b], 0, sizeof(float) * h->total_nodes, h->stream) != hipSuccess))
            rc = fail(LBCG_EDEVICE, "buffer clear failed");
    for (int c = 0; c < n_cases && rc == LBCG_OK; ++c) rc = init_any(h, c, cases[c], init[c]);
    if (rc == LBCG_OK && hipStreamSynchronize(h->stream) != hipSuccess)
        rc = fail(LBCG_EDEVICE, "synchronise after init failed");
    if (rc != LBCG_OK) {
        release(h);
        delete h;
        return rc;
    }
    {
        std::lock_guard<std::mutex> lk(g_handles_mu);
        g_handles.insert(h);
    }
    *out = h;
    return LBCG_OK;
}

int lbcg_step(lbcg_handle *h, int64_t nsteps)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (nsteps < 0) return fail(LBCG_EINVAL, "nsteps < 0");
    int64_t left = nsteps;
    if (h->graph_steps > 0 && !h->timing) {
        while (left > 0) {
            if (h->level == LV_COMPACT &&
                std::find(h->pairlvl.begin(), h->pairlvl.end(), (uint8_t)1) != h->pairlvl.end()) {
                rc = step_once(h, h->stream);           // the converting step is not part of the graph
                if (rc) return rc;
                --left;
                continue;
            }
            if (!h->graph_exec) {
                rc = capture_graph(h);
                if (rc) return rc;
            }
            if (left < h->graph_steps) break;
            if ((int)(h->steps & 1) != h->graph_parity) {   // one eager step restores the captured parity
                rc = step_once(h, h->stream);
                if (rc) return rc;
                --left;
                continue;
            }
            HIPCHK(hipGraphLaunch(h->graph_exec, h->stream));
            const int64_t before = h->steps;
            h->steps += h->graph_steps;                        // even: buffer parity unchanged
            left -= h->graph_steps;
            if (h->diag_every > 0 && h->steps / h->diag_every != before / h->diag_every) {
                rc = stability_check(h);
                if (rc) return rc;
            }
        }
    }
    for (int64_t s = 0; s < left; ++s) {
        rc = step_once(h, h->stream);
        if (rc) return rc;
        if (h->diag_every > 0 && h->steps % h->diag_every == 0) {
            rc = stability_check(h);
            if (rc) return rc;
        }
    }
    return LBCG_OK;
}

int lbcg_moments(lbcg_handle *h, int32_t case_id, float *rhoR, float *rhoB, float *rhoN, float *ux, float *uy,
                 float *uz, double *diag)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (case_id < 0 || case_id >= h->ncases) return fail(LBCG_EINVAL, "case_id out of range");
    rc = moments_any(h, h->tile_begin[case_id], h->tile_count[case_id], rhoR, rhoB, rhoN, ux, uy, uz);
    if (rc) return rc;
    if (diag) {
        double out[6];
        HIPCHK(hipMemcpyAsync(out, h->red, sizeof out, hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (int k = 0; k < 5; ++k) diag[k] = out[k];
    }
    return LBCG_OK;
}

int lbcg_set_fields(lbcg_handle *h, int32_t case_id, const lbcg_fields *fields)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (case_id < 0 || case_id >= h->ncases || !fields) return fail(LBCG_EINVAL, "bad argument");
    const lbcg_fields &f = *fields;
    if (!f.rhoR || !f.rhoB || !f.ux || !f.uy || !f.uz) return fail(LBCG_EINVAL, "NULL field");
    lbcg_case c{};
    // the init kernel only needs alpha and the model flag, recovered from the case constants
    const DevCase &d = h->dc[case_id];
    c.alpha[0] = h->alpha_in[case_id][0];
    c.alpha[1] = h->alpha_in[case_id][1];
    c.improved = d.improved;
    rc = init_any(h, case_id, c, f);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(h->stream));
    return LBCG_OK;
}

int lbcg_free(lbcg_handle *h)
{
    int rc = check_handle(h);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_handles_mu);
        g_handles.erase(h);
    }
    (void)hipStreamSynchronize(h->stream);
    release(h);
    h->alive = false;
    delete h;
    return LBCG_OK;
}

int64_t lbcg_steps_done(const lbcg_handle *h) { return live(h) ? h->steps : -1; }

int64_t lbcg_case_nodes(const lbcg_handle *h, int32_t case_id)
{
    if (!live(h) || case_id < 0 || case_id >= h->ncases) return -1;
    return h->dc[case_id].N;
}

int32_t lbcg_storage_bytes(const lbcg_handle *h) { return live(h) ? h->elem : -1; }

int32_t lbcg_step_kernel(const lbcg_handle *h)
{
    return live(h) ? (h->fused ? LBCG_KERNEL_FUSED : LBCG_KERNEL_TWOPASS) : -1;
}

int32_t lbcg_level_format(const lbcg_handle *h)
{
    return live(h) ? (h->level == LV_COMPACT ? LBCG_LEVEL_COMPACT : LBCG_LEVEL_PAIR) : -1;
}

int32_t lbcg_zchunk(const lbcg_handle *h)
{
    return live(h) ? (h->fused ? h->zc : 0) : -1;
}

int lbcg_timing(lbcg_handle *h, int32_t enable)
{
    int rc = check_handle(h);
    if (rc) return rc;
    h->timing = enable != 0;
    return LBCG_OK;
}

int lbcg_timing_read(lbcg_handle *h, double *ms, int64_t *launches)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (!ms || !launches) return fail(LBCG_EINVAL, "NULL output");
    HIPCHK(hipStreamSynchronize(h->stream));
    for (const int3 &p : h->pending) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, h->events[p.y], h->events[p.z]));
        h->ms_acc[p.x] += t;
        h->launches[p.x] += 1;
    }
    h->pending.clear();
    h->ev_used = 0;
    for (int k = 0; k < 4; ++k) {
        ms[k] = h->ms_acc[k];
        launches[k] = h->launches[k];
        h->ms_acc[k] = 0.0;
        h->launches[k] = 0;
    }
    return LBCG_OK;
}

int lbcg_index_map(lbcg_handle *h, int32_t case_id, int64_t *src_node, int8_t *src_dir)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (case_id < 0 || case_id >= h->ncases || !src_node || !src_dir) return fail(LBCG_EINVAL, "bad argument");
    const int N = h->dc[case_id].N;
    hipLaunchKernelGGL(k_index_map, dim3((N + 255) / 256), dim3(256), 0, h->stream, (const DevCase *)h->d_cases,
                       case_id, src_node, src_dir);
    HIPCHK(hipGetLastError());
    return LBCG_OK;
}

int lbcg_get_populations(lbcg_handle *h, int32_t case_id, float *f)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (case_id < 0 || case_id >= h->ncases || !f) return fail(LBCG_EINVAL, "bad argument");
    const int N = h->dc[case_id].N;
    StepArgs a = args_for(h);
    dim3 g((N + 255) / 256), b(256);
    const bool cp = fmt_of(h, case_id) == LV_COMPACT;
    switch (h->storage) {
    case LBCG_FP32:
        if (cp) hipLaunchKernelGGL((k_get_pop<LBCG_FP32, LV_COMPACT>), g, b, 0, h->stream, a, case_id, f);
        else hipLaunchKernelGGL((k_get_pop<LBCG_FP32, LV_PAIR>), g, b, 0, h->stream, a, case_id, f);
        break;
    case LBCG_FP16S:
        if (cp) hipLaunchKernelGGL((k_get_pop<LBCG_FP16S, LV_COMPACT>), g, b, 0, h->stream, a, case_id, f);
        else hipLaunchKernelGGL((k_get_pop<LBCG_FP16S, LV_PAIR>), g, b, 0, h->stream, a, case_id, f);
        break;
    default:
        if (cp) hipLaunchKernelGGL((k_get_pop<LBCG_BF16S, LV_COMPACT>), g, b, 0, h->stream, a, case_id, f);
        else hipLaunchKernelGGL((k_get_pop<LBCG_BF16S, LV_PAIR>), g, b, 0, h->stream, a, case_id, f);
        break;
    }
    HIPCHK(hipGetLastError());
    return LBCG_OK;
}

int64_t lbcg_checkpoint_bytes(const lbcg_handle *h)
{
    if (!live(h)) return -1;
    return ckpt_bytes(h);
}

int lbcg_checkpoint_save(lbcg_handle *h, void *host, int64_t bytes)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (!host || bytes < ckpt_bytes(h)) return fail(LBCG_EINVAL, "checkpoint buffer NULL or too small");
    CkptHeader hd;
    std::memcpy(hd.magic, kMagic, 8);
    hd.version = kCkptVersion;
    hd.storage = h->storage;
    hd.ncases = h->ncases;
    hd.total_pop = h->total_pop;
    hd.total_nodes = h->total_nodes;
    hd.steps = h->steps;
    hd.level = h->level;
    char *p = static_cast<char *>(host);
    std::memcpy(p, &hd, sizeof hd);
    p += sizeof hd;
    for (int c = 0; c < h->ncases; ++c) {
        const CkptCase cc = ckpt_case(h, c);
        std::memcpy(p, &cc, sizeof cc);
        p += sizeof cc;
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    HIPCHK(hipMemcpy(p, h->pop[h->cur], (size_t)h->elem * h->total_pop, hipMemcpyDeviceToHost));
    p += (size_t)h->elem * h->total_pop;
    HIPCHK(hipMemcpy(p, h->rho2[(h->steps + 1) & 1], sizeof(float2) * h->total_nodes, hipMemcpyDeviceToHost));
    p += sizeof(float2) * h->total_nodes;
    if (h->level == LV_COMPACT) {
        HIPCHK(hipMemcpy(p, h->dsc[(h->steps + 1) & 1], sizeof(float4) * h->total_nodes, hipMemcpyDeviceToHost));
        p += sizeof(float4) * h->total_nodes;
        HIPCHK(hipMemcpy(p, h->crs[(h->steps + 1) & 1], sizeof(float) * h->total_nodes, hipMemcpyDeviceToHost));
    }
    return LBCG_OK;
}

int lbcg_checkpoint_load(lbcg_handle *h, const void *host, int64_t bytes)
{
    int rc = check_handle(h);
    if (rc) return rc;
    if (!host || bytes < (int64_t)sizeof(CkptHeader)) return fail(LBCG_EINVAL, "checkpoint buffer NULL or too small");
    CkptHeader hd;
    std::memcpy(&hd, host, sizeof hd);
    if (std::memcmp(hd.magic, kMagic, 8) != 0 || hd.version != kCkptVersion)
        return fail(LBCG_EINVAL, "not a checkpoint image");
    if (hd.storage != h->storage || hd.ncases != h->ncases || hd.total_pop != h->total_pop ||
        hd.total_nodes != h->total_nodes || hd.steps < 0 || hd.level != h->level)
        return fail(LBCG_EINVAL, "checkpoint of another case shape, storage or level format");
    if (bytes < ckpt_bytes(h)) return fail(LBCG_EINVAL, "checkpoint buffer too small");
    const char *p = static_cast<const char *>(host) + sizeof hd;
    std::vector<uint8_t> plv(h->ncases);
    for (int c = 0; c < h->ncases; ++c) {
        CkptCase cc;
        std::memcpy(&cc, p, sizeof cc);
        p += sizeof cc;
        const CkptCase mine = ckpt_case(h, c);
        if (cc.nx != mine.nx || cc.ny != mine.ny || cc.nz != mine.nz || cc.NS != mine.NS ||
            cc.pop_off != mine.pop_off || cc.node_off != mine.node_off || (cc.pair_level & ~(int64_t)1) != 0)
            return fail(LBCG_EINVAL, "checkpoint case " + std::to_string(c) + " has other extents or layout");
        plv[c] = (uint8_t)cc.pair_level;
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    h->steps = hd.steps;
    h->cur = (int)(hd.steps & 1);       // the handle keeps pop[steps & 1] as the current level
    HIPCHK(hipMemcpy(h->pop[h->cur], p, (size_t)h->elem * h->total_pop, hipMemcpyHostToDevice));
    p += (size_t)h->elem * h->total_pop;
    HIPCHK(hipMemcpy(h->rho2[(h->steps + 1) & 1], p, sizeof(float2) * h->total_nodes, hipMemcpyHostToDevice));
    p += sizeof(float2) * h->total_nodes;
    if (h->level == LV_COMPACT) {
        HIPCHK(hipMemcpy(h->dsc[(h->steps + 1) & 1], p, sizeof(float4) * h->total_nodes, hipMemcpyHostToDevice));
        p += sizeof(float4) * h->total_nodes;
        HIPCHK(hipMemcpy(h->crs[(h->steps + 1) & 1], p, sizeof(float) * h->total_nodes, hipMemcpyHostToDevice));
    }
    h->pairlvl = plv;
    return LBCG_OK;
}

}  // extern "C"
