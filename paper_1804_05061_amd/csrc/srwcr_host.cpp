// srwcr_host.cpp -- C ABI of the SRWCR library: validation, plans, workspace
// layout and launch sequences (see include/srwcr.h for the contract).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "srwcr.h"
#include "srwcr_internal.h"

using namespace srwcr;

static_assert(kMaxBatch == SRWCR_MAX_BATCH, "batch limit of the ABI and the kernels differ");

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(SRWCR_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                          \
    do {                                             \
        hipError_t _e = (expr);                      \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int validate_problem(const srwcr_problem *p)
{
    if (!p) return fail(SRWCR_E_INVALID_ARG, "problem is NULL");
    const bool at_nodes = p->spatial_bins[0] == 0 && p->spatial_bins[1] == 0 && p->spatial_bins[2] == 0;
    for (int e = 0; e < 3; ++e) {
        if (p->fixed_dims[e] < 2 || p->moving_dims[e] < 2)
            return fail(SRWCR_E_INVALID_ARG, "grid axis %d must have at least 2 voxels (fixed %d, moving %d)", e,
                        p->fixed_dims[e], p->moving_dims[e]);
        if (!at_nodes && (p->spatial_bins[e] < 4 || p->spatial_bins[e] > 64))
            return fail(SRWCR_E_INVALID_ARG, "spatial_bins[%d] = %d outside 4..64 (all three 0: regions at the FFD "
                        "nodes)", e, p->spatial_bins[e]);
        if (p->ctrl_spacing[e] < 1)
            return fail(SRWCR_E_INVALID_ARG, "ctrl_spacing[%d] = %d must be >= 1", e, p->ctrl_spacing[e]);
        if ((int64_t)p->fixed_dims[e] > (1 << 20) || (int64_t)p->moving_dims[e] > (1 << 20))
            return fail(SRWCR_E_INVALID_ARG, "grid axis %d too long", e);
    }
    if (p->n_bins < 2 || p->n_bins > kMaxBins)
        return fail(SRWCR_E_INVALID_ARG, "n_bins = %d outside 2..%d", p->n_bins, kMaxBins);
    if (p->role != SRWCR_MOVING_AS_A && p->role != SRWCR_MOVING_AS_B)
        return fail(SRWCR_E_INVALID_ARG, "role = %d is neither MOVING_AS_A nor MOVING_AS_B", p->role);
    for (int d : {p->fixed_dtype, p->moving_dtype})
        if (d < SRWCR_F32 || d > SRWCR_BF16) return fail(SRWCR_E_INVALID_ARG, "dtype %d unknown", d);
    return SRWCR_OK;
}

double bspline_piece(int l, double t)
{
    switch (l) {
    case 0: return (1 - t) * (1 - t) * (1 - t) / 6.0;
    case 1: return (3 * t * t * t - 6 * t * t + 4) / 6.0;
    case 2: return (-3 * t * t * t + 3 * t * t + 3 * t + 1) / 6.0;
    default: return t * t * t / 6.0;
    }
}

// The staged value pass of a set of value blocks (blocks[i].prob = problem) of
// 5 x bw x bw regions: the block visits of the G persistent workgroups, as the
// value pass walks them (workgroup w takes rows [w T / G, (w + 1) T / G) and
// visits every block they touch), and, per region of every problem (problem by
// problem), the visits that hold it as entries visit * 5 bw^2 + local region.
struct StagePlan {
    std::vector<int> vstart;        // [G + 1] first visit id of each workgroup
    std::vector<int> reg_start;     // [regions + 1]
    std::vector<int> ent;
    std::vector<int2> reg_id;       // (problem, region) per merged region
    size_t visits = 0;
    int waves = 1;                  // merge waves per region
};

StagePlan stage_plan(const std::vector<WorkItem> &vb, const std::vector<int> &vr, int G,
                     const std::vector<const Geom *> &geoms, int bw)
{
    const int nreg = kXN * bw * bw, jkn = bw * bw;
    StagePlan sp;
    const long T = vr.back();
    sp.vstart.assign(G + 1, 0);
    std::vector<int> vblock;
    for (int w = 0; w < G; ++w) {
        long r0 = (long)w * T / G;
        const long r1 = (long)(w + 1) * T / G;
        int bi = 0;
        while (bi + 1 < (int)vb.size() && vr[bi + 1] <= r0) ++bi;
        while (r0 < r1) {
            vblock.push_back(bi);
            r0 = std::min(r1, (long)vr[bi + 1]);
            ++bi;
        }
        sp.vstart[w + 1] = (int)vblock.size();
    }
    sp.visits = vblock.size();
    std::vector<int> base(geoms.size() + 1, 0);
    for (size_t p = 0; p < geoms.size(); ++p) base[p + 1] = base[p] + geoms[p]->R;
    std::vector<std::vector<int>> per(base.back());
    for (size_t v = 0; v < sp.visits; ++v) {
        const WorkItem &b = vb[vblock[v]];
        const Geom &g = *geoms[b.prob];
        for (int loc = 0; loc < nreg; ++loc) {
            const int i = loc / jkn, jk = loc - i * jkn, k = jk / bw, j = jk - k * bw;
            if (b.cx + i >= g.K[0] || b.cy + j >= g.K[1] || b.cz + k >= g.K[2]) continue;
            const int R = ((b.cz + k) * g.K[1] + (b.cy + j)) * g.K[0] + (b.cx + i);
            per[base[b.prob] + R].push_back((int)(v * nreg + loc));
        }
    }
    sp.reg_start.assign(base.back() + 1, 0);
    size_t emax = 0;
    for (size_t p = 0; p < geoms.size(); ++p)
        for (int R = 0; R < geoms[p]->R; ++R) {
            const int q = base[p] + R;
            sp.ent.insert(sp.ent.end(), per[q].begin(), per[q].end());
            sp.reg_start[q + 1] = (int)sp.ent.size();
            sp.reg_id.push_back(make_int2((int)p, R));
            emax = std::max(emax, per[q].size());
        }
    sp.waves = (int)std::max<size_t>(1, std::min<size_t>(16, (emax + 7) / 8));
    return sp;
}

constexpr size_t kStageLimit = (size_t)512 << 20;   // staging slots above this: atomic merge
constexpr int kColUnit = 128;                        // columns of a work unit of the column value pass

// Work units of the column value pass over a list of value blocks: runs of up
// to kColUnit columns of one block (x, y), columns numbered x fastest.
std::vector<int4> column_units(const std::vector<WorkItem> &vb)
{
    std::vector<int4> cu;
    for (size_t b = 0; b < vb.size(); ++b) {
        const int ncol = (vb[b].x1 - vb[b].x0) * (vb[b].y1 - vb[b].y0);
        for (int c = 0; c < ncol; c += kColUnit) cu.push_back(make_int4((int)b, c, std::min(ncol, c + kColUnit), 0));
    }
    return cu;
}

}  // namespace

struct srwcr_plan {
    srwcr_problem prob;
    Geom g;
    Geom *geom_dev = nullptr;     // g on the device (kernels read it through a one-problem array)
    std::vector<void *> dev_allocs;
    WorkItem *items = nullptr;           // warp and gradient passes: boxes sized for the LDS node block
    std::vector<WorkItem> items_host;
    int nitems = 0;
    WorkItem *vblocks = nullptr;         // value pass: whole region blocks, rows listed block by block
    int *vrow = nullptr;                 // first row of each block, then the total
    std::vector<WorkItem> vblocks_host;
    std::vector<int> vrow_host;
    int nvblocks = 0;
    int nwg = 0;                         // persistent value-pass workgroups (one per compute unit)
    // warp pass rows: the value blocks, or, when the spatial cells are narrower
    // than a row (regions at the FFD nodes), x-chunks of a full row width over
    // the whole y-z plane (the warp pass does not depend on the regions)
    const WorkItem *wblocks = nullptr;
    const int *wrow = nullptr;
    std::vector<int> wrow_host;
    int nwblocks = 0;
    int value_bw = 4;                    // (y, z) regions per axis of a value block: 4 (one cell) or 5 (two)
    bool cols = false;                   // value pass per block column on the matrix cores (launch_value_cols)
    const int4 *cunits = nullptr;        // its work units (value block, first column, end column)
    int ncunits = 0;
    bool gcols = false;                  // FFD gradient by box columns (launch_grad_cols)
    // staged value pass (when the staging slots fit): per workgroup its first
    // block-visit id; per region the visits that hold it (CSR: reg_start, ent =
    // visit * 80 + local region); waves per region of the merge
    bool staged = false;
    const int *visit_start = nullptr;
    const int *reg_start = nullptr;
    const int *ent = nullptr;
    int merge_waves = 1;
    size_t stage_visits = 0;
    size_t staging_off = 0;
    size_t value_lds = 0, grad_lds = 0, prep_lds = 0;
    WsLayout ws;
    int device = 0;
    // diagnostics: per-phase HIP events recorded by srwcr_grad while profiling is on
    mutable int profiling = 0;           // 0 off, 1 every phase, 2 the value pass (or patch sums) only
    mutable std::vector<hipEvent_t> ev_pool;
    mutable size_t ev_used = 0;
    mutable int32_t prof_calls = 0;
};

namespace {
constexpr int kPhases = 6;            // zero, warp, value, finalise, gradient, gradient output
constexpr size_t kProfCalls = 4096;   // calls recorded per profiling session

// the one phase that modes 2 and 3 time: the value pass, the gradient pass
inline int prof_phase(int mode) { return mode == 2 ? 2 : 4; }

// record event `k` of the current profiled call (no-op when profiling is off;
// in modes 2 and 3 only the two events around that mode's phase)
void prof_mark(const srwcr_plan *P, int k, hipStream_t s)
{
    if (!P->profiling) return;
    if (P->profiling >= 2 && k != prof_phase(P->profiling) && k != prof_phase(P->profiling) + 1) return;
    const size_t base = (size_t)P->prof_calls * (kPhases + 1);
    if (base + kPhases + 1 > P->ev_pool.size()) return;
    (void)hipEventRecord(P->ev_pool[base + k], s);
}
}  // namespace

int srwcr::report_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int srwcr::plan_device(const srwcr_plan *plan) { return plan->device; }

extern "C" {

const char *srwcr_last_error(void) { return g_last_error.c_str(); }

int srwcr_ctrl_dims(const srwcr_problem *prob, int32_t out_nc[3])
{
    if (!prob || !out_nc) return fail(SRWCR_E_INVALID_ARG, "NULL argument");
    for (int e = 0; e < 3; ++e) {
        if (prob->fixed_dims[e] < 2 || prob->ctrl_spacing[e] < 1)
            return fail(SRWCR_E_INVALID_ARG, "invalid fixed_dims / ctrl_spacing on axis %d", e);
        out_nc[e] = (prob->fixed_dims[e] - 1) / prob->ctrl_spacing[e] + 4;
    }
    return SRWCR_OK;
}

void srwcr_plan_destroy(srwcr_plan *plan)
{
    if (!plan) return;
    for (hipEvent_t e : plan->ev_pool) (void)hipEventDestroy(e);
    for (void *p : plan->dev_allocs) (void)hipFree(p);
    delete plan;
}

int srwcr_plan_create(const srwcr_problem *prob, srwcr_plan **out)
{
    return srwcr_plan_create_tuned(prob, nullptr, out);
}

int srwcr_plan_create_tuned(const srwcr_problem *prob, const srwcr_tuning *tuning, srwcr_plan **out)
{
    if (!out) return fail(SRWCR_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int st = validate_problem(prob);
    if (st != SRWCR_OK) return st;
    srwcr_tuning tune{0, 0};
    if (tuning) tune = *tuning;
    if (tune.grad_item_voxels < 0 || tune.value_workgroups < 0)
        return fail(SRWCR_E_INVALID_ARG, "tuning values must be >= 0 (0: default)");
    const bool at_nodes = prob->spatial_bins[0] == 0;   // validated: all three 0, regions at the FFD nodes
    srwcr_plan *P = new srwcr_plan();
    P->prob = *prob;
    Geom &g = P->g;
    std::memset(&g, 0, sizeof g);
    for (int e = 0; e < 3; ++e) {
        g.nf[e] = prob->fixed_dims[e];
        g.nm[e] = prob->moving_dims[e];
        g.delta[e] = prob->ctrl_spacing[e];
        g.nc[e] = (g.nf[e] - 1) / g.delta[e] + 4;
        g.K[e] = at_nodes ? g.nc[e] : prob->spatial_bins[e];
        g.same_grid[e] = g.nm[e] == g.nf[e];
        g.ratio[e] = (float)((double)g.nm[e] / (double)g.nf[e]);
        g.ratio_d[e] = (double)g.nm[e] / (double)g.nf[e];
    }
    g.nb = prob->n_bins;
    g.role = prob->role;
    g.fdt = prob->fixed_dtype;
    g.mdt = prob->moving_dtype;
    g.R = g.K[0] * g.K[1] * g.K[2];
    g.bw = 4;
    const double nvox = (double)g.nf[0] * g.nf[1] * g.nf[2];
    g.inv_Z = 1.0 / nvox;     // sum_r w(r, x) = 1 and sum_a h = 1 make Z the voxel count (eq 3)

    auto upload = [&](const void *host, size_t bytes, void **dev) -> int {
        hipError_t e = hipMalloc(dev, bytes);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(plan tables)");
        P->dev_allocs.push_back(*dev);
        e = hipMemcpy(*dev, host, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(plan tables)");
        return SRWCR_OK;
    };

    // per-axis tables
    std::vector<std::vector<int>> cells(3);
    for (int e = 0; e < 3; ++e) {
        const int N = g.nf[e], K = g.K[e];
        std::vector<int> sp_cell(N), ffd_p(N), mv_base(N);
        std::vector<float4> sp_w(N);
        std::vector<double4> ffd_w(N);
        std::vector<double> mv_frac(N);
        for (int x = 0; x < N; ++x) {
            // spatial bins: node j at (j - 1) (N - 1) / (K - 3), integer cell
            // arithmetic; or, with the regions at the FFD nodes, node j at (j - 1) delta
            int c;
            double t;
            if (at_nodes) {
                c = x / g.delta[e];
                t = (double)(x % g.delta[e]) / g.delta[e];
            } else {
                const long num = (long)x * (K - 3);
                c = (int)(num / (N - 1));
                if (c > K - 4) c = K - 4;
                t = (double)(num - (long)c * (N - 1)) / (double)(N - 1);
            }
            sp_cell[x] = c;
            sp_w[x] = make_float4((float)bspline_piece(0, t), (float)bspline_piece(1, t), (float)bspline_piece(2, t),
                                  (float)bspline_piece(3, t));
            // FFD: p = floor(x / delta), eta = (x mod delta) / delta (eq 17)
            const int d = g.delta[e];
            ffd_p[x] = x / d;
            const double eta = (double)(x % d) / d;
            ffd_w[x] = make_double4(bspline_piece(0, eta), bspline_piece(1, eta), bspline_piece(2, eta),
                                    bspline_piece(3, eta));
            // moving-grid mapping y = (x + 1/2) M / N - 1/2 (+ u M / N)
            const double yv = ((double)x + 0.5) * g.nm[e] / g.nf[e] - 0.5;
            const double fl = std::floor(yv);
            mv_base[x] = (int)fl;
            mv_frac[x] = yv - fl;
        }
        cells[e] = sp_cell;
        void *d;
        if ((st = upload(sp_cell.data(), N * sizeof(int), &d))) goto bad;
        g.sp_cell[e] = (const int *)d;
        if ((st = upload(sp_w.data(), N * sizeof(float4), &d))) goto bad;
        g.sp_w[e] = (const float4 *)d;
        if ((st = upload(ffd_p.data(), N * sizeof(int), &d))) goto bad;
        g.ffd_p[e] = (const int *)d;
        if ((st = upload(ffd_w.data(), N * sizeof(double4), &d))) goto bad;
        g.ffd_w[e] = (const double4 *)d;
        if ((st = upload(mv_base.data(), N * sizeof(int), &d))) goto bad;
        g.mv_base[e] = (const int *)d;
        if ((st = upload(mv_frac.data(), N * sizeof(double), &d))) goto bad;
        g.mv_frac[e] = (const double *)d;
    }

    {
        // work items: boxes inside one spatial cell, sized for ~600 items and the LDS budget
        int dev = 0;
        hipError_t he = hipGetDevice(&dev);
        if (he != hipSuccess) { st = hip_fail(he, "hipGetDevice"); goto bad; }
        P->device = dev;
        int max_lds = 0;
        he = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (he != hipSuccess) { st = hip_fail(he, "hipDeviceGetAttribute(shared memory)"); goto bad; }
        // item rows: 2 x 64 voxels per wave when the FFD x-spacing leaves room in
        // the per-wave scratch, else 64
        g.xw = g.delta[0] >= 3 ? kSlots * kWave : kWave;
        g.c1n = (g.xw - 1) / g.delta[0] + 5;
        g.gscr = grad_scratch_floats((g.xw - 1) / g.delta[0] + 2);
        P->value_lds = value_lds_bytes(g, 4);
        P->prep_lds = prep_lds_bytes(g);
        if (P->value_lds > (size_t)max_lds) {
            st = fail(SRWCR_E_UNSUPPORTED, "value pass needs %zu B of LDS, device allows %d", P->value_lds, max_lds);
            goto bad;
        }
        std::vector<int> lo[3], hi[3];
        for (int e = 0; e < 3; ++e) {
            lo[e].assign(g.K[e] - 3, -1);
            hi[e].assign(g.K[e] - 3, -1);
            for (int x = 0; x < g.nf[e]; ++x) {
                const int c = cells[e][x];
                if (lo[e][c] < 0) lo[e][c] = x;
                hi[e][c] = x + 1;
            }
        }
        // value blocks of two cells along y and z (5 x 5 x 5 regions) when the
        // cells are so small that a one-cell block has fewer rows than 4 per wave
        // and the larger histogram fits
        {
            long max_rows = 0;
            for (int cy = 0; cy < g.K[1] - 3; ++cy)
                for (int cz = 0; cz < g.K[2] - 3; ++cz)
                    if (lo[1][cy] >= 0 && lo[2][cz] >= 0)
                        max_rows = std::max(max_rows, (long)(hi[1][cy] - lo[1][cy]) * (hi[2][cz] - lo[2][cz]));
            const size_t lds5 = value_lds_bytes(g, 5);
            g.bw = 5;                                   // the gradient pass's tables of 125 regions must fit too
            const size_t glds5 = grad_lds_bytes(g, 8, 8, 8);
            g.bw = 4;
            if (max_rows < 4 * (kValueThreads / kWave) && lds5 <= (size_t)max_lds && glds5 <= (size_t)max_lds) {
                P->value_bw = 5;
                P->value_lds = lds5;
                g.bw = 5;
            }
        }
        // cells per block along y and z, and the voxel range of the non-empty
        // cells c .. c + cstep - 1 of axis e
        const int cstep = P->value_bw == 5 ? 2 : 1;
        auto span = [&](int e, int c, int &a, int &b) {
            a = b = -1;
            for (int cc = c; cc < std::min(c + cstep, g.K[e] - 3); ++cc)
                if (lo[e][cc] >= 0) {
                    if (a < 0) a = lo[e][cc];
                    b = hi[e][cc];
                }
            return a >= 0;
        };
        // x chunks: runs of up to xmax voxels that touch at most two spatial
        // cells, so their regions fit the 5 x-node block of a work item
        auto x_chunks = [&](int xmax) {
            std::vector<std::pair<int, int>> ch;
            for (int x = 0; x < g.nf[0];) {
                const int c = cells[0][x];
                int end = std::min(g.nf[0], x + xmax);
                if (c + 2 < g.K[0] - 3 && lo[0][c + 2] >= 0) end = std::min(end, lo[0][c + 2]);
                for (int cc = c + 2; cc < g.K[0] - 3; ++cc)
                    if (lo[0][cc] >= 0) { end = std::min(end, lo[0][cc]); break; }
                ch.push_back({x, end});
                x = end;
            }
            return ch;
        };
        const double target = tune.grad_item_voxels > 0 ? std::max(256.0, (double)tune.grad_item_voxels)
                                                         : std::min(65536.0, std::max(2048.0, nvox / 600.0));
        int xc_max = g.xw, yc_max = 0, zc_max = 0;
        std::vector<WorkItem> items;
        for (int attempt = 0; attempt < 64; ++attempt) {
            items.clear();
            size_t worst_lds = 0;
            const auto xch = x_chunks(xc_max);
            for (int cz = 0; cz < g.K[2] - 3; cz += cstep) {
                int za, zb;
                if (!span(2, cz, za, zb)) continue;
                for (int cy = 0; cy < g.K[1] - 3; cy += cstep) {
                    int ya, yb;
                    if (!span(1, cy, ya, yb)) continue;
                    const int yw = yb - ya, zw = zb - za;
                    for (const auto &xr : xch) {
                        const int xw = xr.second - xr.first;
                        const double side = std::sqrt(target / xw);
                        int yc = std::max(1, std::min(yw, (int)std::lround(side * 1.5)));
                        if (yc_max) yc = std::min(yc, yc_max);
                        int zc = std::max(1, std::min(zw, (int)std::ceil(target / ((double)xw * yc))));
                        if (zc_max) zc = std::min(zc, zc_max);
                        // z-ranges end on FFD cell boundaries (mz whole FFD z-cells, fewer
                        // at the spatial cell's edges), so that a wave's consecutive rows
                        // share an FFD z-cell and the gradient pass scatters them together
                        const int dz = g.delta[2];
                        const int mz = std::max(1, (int)std::lround((double)zc / dz));
                        for (int z0 = za, z1 = 0; z0 < zb; z0 = z1) {
                            z1 = std::min(zb, (z0 / dz + mz) * dz);
                            if (zc_max) z1 = std::min(z1, z0 + zc_max);
                            for (int y0 = ya; y0 < yb; y0 += yc) {
                                WorkItem w{};
                                w.x0 = xr.first; w.x1 = xr.second;
                                w.y0 = y0; w.y1 = std::min(y0 + yc, yb);
                                w.z0 = z0; w.z1 = z1;
                                w.cx = cells[0][w.x0]; w.cy = cy; w.cz = cz;
                                w.gx0 = w.x0 / g.delta[0];
                                w.gy0 = w.y0 / g.delta[1];
                                w.gz0 = w.z0 / g.delta[2];
                                w.gnx = (w.x1 - 1) / g.delta[0] - w.gx0 + 4;
                                w.gny = (w.y1 - 1) / g.delta[1] - w.gy0 + 4;
                                w.gnz = (w.z1 - 1) / g.delta[2] - w.gz0 + 4;
                                worst_lds = std::max(worst_lds, grad_lds_bytes(g, w.gnx, w.gny, w.gnz));
                                items.push_back(w);
                            }
                        }
                    }
                }
            }
            if (worst_lds <= (size_t)max_lds) {
                P->grad_lds = worst_lds;
                break;
            }
            // shrink the boxes until the gradient pass fits in LDS
            if (xc_max > 64) xc_max /= 2;
            else {
                yc_max = yc_max ? std::max(1, yc_max / 2) : 32;
                zc_max = zc_max ? std::max(1, zc_max / 2) : 16;
                if (yc_max == 1 && zc_max == 1 && attempt > 40) {
                    st = fail(SRWCR_E_UNSUPPORTED, "gradient pass does not fit in %d B of LDS", max_lds);
                    goto bad;
                }
            }
        }
        // the largest boxes first: the hardware hands boxes to the compute units
        // in launch order, so the small ones fill the tail
        {
            auto rows = [](const WorkItem &w) { return (long)(w.y1 - w.y0) * (w.z1 - w.z0) * (w.x1 - w.x0); };
            std::stable_sort(items.begin(), items.end(),
                             [&](const WorkItem &a, const WorkItem &c) { return rows(a) > rows(c); });
        }
        P->nitems = (int)items.size();
        P->items_host = items;
        // the column gradient pass: boxes of two small cells per axis, the moving
        // image as A, and boxes small enough for its one-wave layout
        P->gcols = P->value_bw == 5 && g.role == 0;
        for (const WorkItem &w : items)
            P->gcols = P->gcols && (w.x1 - w.x0) * (w.y1 - w.y0) <= 2 * kWave && w.gnx * w.gny <= 32 && w.gnz <= kXN &&
                       w.z1 - w.z0 <= 12;
        // value-pass blocks: an x-chunk by one spatial cell in y and z (or two, see above)
        {
            std::vector<WorkItem> vb;
            std::vector<int> vr(1, 0);
            const auto xch = x_chunks(g.xw);
            for (int cz = 0; cz < g.K[2] - 3; cz += cstep) {
                int za, zb;
                if (!span(2, cz, za, zb)) continue;
                for (int cy = 0; cy < g.K[1] - 3; cy += cstep) {
                    int ya, yb;
                    if (!span(1, cy, ya, yb)) continue;
                    for (const auto &xr : xch) {
                        WorkItem w{};
                        w.x0 = xr.first; w.x1 = xr.second;
                        w.y0 = ya; w.y1 = yb;
                        w.z0 = za; w.z1 = zb;
                        w.cx = cells[0][w.x0]; w.cy = cy; w.cz = cz;
                        vb.push_back(w);
                        vr.push_back(vr.back() + (w.y1 - w.y0) * (w.z1 - w.z0));
                    }
                }
            }
            P->vblocks_host = vb;
            P->vrow_host = vr;
            P->nvblocks = (int)vb.size();
            void *dv;
            if ((st = upload(vb.data(), vb.size() * sizeof(WorkItem), &dv))) goto bad;
            P->vblocks = (WorkItem *)dv;
            if ((st = upload(vr.data(), vr.size() * sizeof(int), &dv))) goto bad;
            P->vrow = (int *)dv;
            int ncu = 0;
            he = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
            if (he != hipSuccess) { st = hip_fail(he, "hipDeviceGetAttribute(compute units)"); goto bad; }
            P->nwg = std::max(1, std::min(tune.value_workgroups > 0 ? tune.value_workgroups : ncu, vr.back()));
            // blocks of two small cells per axis (short rows): the column value
            // pass (FP64 atomics into the moments, no staging); for one-cell
            // blocks, whose rows are long, the row value pass
            P->cols = P->value_bw == 5;
            if (P->cols) {
                const std::vector<int4> cu = column_units(vb);
                if ((st = upload(cu.data(), cu.size() * sizeof(int4), &dv))) goto bad;
                P->cunits = (const int4 *)dv;
                P->ncunits = (int)cu.size();
            } else {
                const StagePlan sp = stage_plan(vb, vr, P->nwg, {&g}, P->value_bw);
                const size_t nreg = (size_t)kXN * P->value_bw * P->value_bw;
                const size_t stage_bytes = sp.visits * nreg * g.nb * 3 * sizeof(double);
                if (stage_bytes <= kStageLimit && sp.visits * nreg < (size_t)INT32_MAX && !sp.ent.empty()) {
                    if ((st = upload(sp.vstart.data(), sp.vstart.size() * sizeof(int), &dv))) goto bad;
                    P->visit_start = (const int *)dv;
                    if ((st = upload(sp.reg_start.data(), sp.reg_start.size() * sizeof(int), &dv))) goto bad;
                    P->reg_start = (const int *)dv;
                    if ((st = upload(sp.ent.data(), sp.ent.size() * sizeof(int), &dv))) goto bad;
                    P->ent = (const int *)dv;
                    P->merge_waves = sp.waves;
                    P->staged = true;
                    P->stage_visits = sp.visits;
                }
            }
            P->wblocks = P->vblocks;
            P->wrow = P->vrow;
            P->wrow_host = vr;
            P->nwblocks = P->nvblocks;
            if (at_nodes) {
                std::vector<WorkItem> wb;
                std::vector<int> wr(1, 0);
                for (int x0 = 0; x0 < g.nf[0]; x0 += g.xw) {
                    WorkItem w{};
                    w.x0 = x0; w.x1 = std::min(g.nf[0], x0 + g.xw);
                    w.y0 = 0; w.y1 = g.nf[1];
                    w.z0 = 0; w.z1 = g.nf[2];
                    wb.push_back(w);
                    wr.push_back(wr.back() + g.nf[1] * g.nf[2]);
                }
                if ((st = upload(wb.data(), wb.size() * sizeof(WorkItem), &dv))) goto bad;
                P->wblocks = (const WorkItem *)dv;
                if ((st = upload(wr.data(), wr.size() * sizeof(int), &dv))) goto bad;
                P->wrow = (const int *)dv;
                P->wrow_host = wr;
                P->nwblocks = (int)wb.size();
            }
        }
        void *d;
        if ((st = upload(items.data(), items.size() * sizeof(WorkItem), &d))) goto bad;
        P->items = (WorkItem *)d;
    }

    {
        // workspace: zeroed block first (moments, gradient accumulators)
        WsLayout &w = P->ws;
        const size_t ncell = (size_t)g.nc[0] * g.nc[1] * g.nc[2];
        size_t off = 0;
        w.moments = off;
        off += (size_t)g.R * g.nb * 3 * sizeof(double);
        w.grad = off;
        off += 3 * ncell * sizeof(double);
        w.counter = off;
        off += sizeof(double);
        off = align_up(off, 256);
        w.region = off;
        off += (size_t)g.R * 4 * sizeof(double);
        off = align_up(off, 256);
        w.tables = off;
        off += (size_t)g.R * g.nb * 4 * sizeof(float);
        off = align_up(off, 256);
        w.alpha = off;
        off += (size_t)g.R * sizeof(float);
        off = align_up(off, 256);
        const size_t nvox = (size_t)g.nf[0] * g.nf[1] * g.nf[2];
        w.kt = off;
        off = align_up(off + nvox * sizeof(PrepKT), 256);
        w.dm = off;
        off += 3 * nvox * sizeof(float);
        off = align_up(off, 256);
        P->staging_off = off;
        if (P->staged) off += P->stage_visits * (size_t)kXN * P->value_bw * P->value_bw * g.nb * 3 * sizeof(double);
        w.total = align_up(off, 256);
        w.rds = w.total;
        g.ws = w;
        void *d;
        if ((st = upload(&g, sizeof(Geom), &d))) goto bad;
        P->geom_dev = (Geom *)d;
    }
    {
        hipError_t he = prepare_kernels();
        if (he != hipSuccess) { st = hip_fail(he, "kernel attributes"); goto bad; }
    }
    *out = P;
    return SRWCR_OK;
bad:
    srwcr_plan_destroy(P);
    return st;
}

size_t srwcr_workspace_bytes(const srwcr_plan *plan) { return plan ? plan->ws.total : 0; }

int srwcr_normalize(const float *in, int64_t n, double lo, double hi, int32_t n_bins, void *out, int32_t out_dtype,
                    void *stream)
{
    if (!in || !out) return fail(SRWCR_E_INVALID_ARG, "NULL volume");
    if (n <= 0) return fail(SRWCR_E_INVALID_ARG, "n = %lld must be positive", (long long)n);
    if (n_bins < 2 || n_bins > kMaxBins) return fail(SRWCR_E_INVALID_ARG, "n_bins = %d outside 2..%d", n_bins, kMaxBins);
    if (out_dtype < SRWCR_F32 || out_dtype > SRWCR_BF16) return fail(SRWCR_E_INVALID_ARG, "dtype %d unknown", out_dtype);
    if (!std::isfinite(lo) || !std::isfinite(hi)) return fail(SRWCR_E_NONFINITE, "normalisation range is not finite");
    if (!(hi > lo)) return fail(SRWCR_E_DEGENERATE, "normalisation range hi (%g) <= lo (%g)", hi, lo);
    const float lo_f = (float)lo;
    const float scale = (float)((double)(n_bins - 1) / (hi - lo));
    HIP_TRY(launch_normalize(in, n, lo_f, scale, (float)(n_bins - 1), out, out_dtype, (hipStream_t)stream),
            "normalize launch");
    return SRWCR_OK;
}

int srwcr_minmax(const float *in, int64_t n, double *lo, double *hi, void *stream)
{
    if (!in || !lo || !hi) return fail(SRWCR_E_INVALID_ARG, "NULL argument");
    if (n <= 0) return fail(SRWCR_E_INVALID_ARG, "n must be positive");
    const int nblocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
    float *partial = nullptr;
    HIP_TRY(hipMalloc(&partial, (size_t)nblocks * 3 * sizeof(float)), "hipMalloc(minmax)");
    hipError_t e = launch_minmax(in, n, partial, nblocks, (hipStream_t)stream);
    std::vector<float> h((size_t)nblocks * 3);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), partial, h.size() * sizeof(float), hipMemcpyDeviceToHost,
                                            (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    (void)hipFree(partial);
    if (e != hipSuccess) return hip_fail(e, "minmax");
    float mn = INFINITY, mx = -INFINITY, bad = 0;
    for (int b = 0; b < nblocks; ++b) {
        mn = std::min(mn, h[3 * b]);
        mx = std::max(mx, h[3 * b + 1]);
        bad += h[3 * b + 2];
    }
    if (bad > 0) return fail(SRWCR_E_NONFINITE, "volume holds %.0f non-finite values", bad);
    *lo = mn;
    *hi = mx;
    return SRWCR_OK;
}

static int check_call(const srwcr_plan *plan, const void *fixed, const void *moving, const float *ffd, void *ws,
                      size_t ws_bytes)
{
    if (!plan) return fail(SRWCR_E_INVALID_ARG, "plan is NULL");
    if (!fixed || !moving || !ffd) return fail(SRWCR_E_INVALID_ARG, "NULL volume or FFD pointer");
    if (!ws) return fail(SRWCR_E_INVALID_ARG, "workspace is NULL");
    if (ws_bytes < plan->ws.total)
        return fail(SRWCR_E_WORKSPACE, "workspace has %zu B, the plan needs %zu B", ws_bytes, plan->ws.total);
    return SRWCR_OK;
}

static BatchArgs one_problem(const void *fixed, const void *moving, const float *ffd, double *d_value,
                             float *d_grad)
{
    BatchArgs a;
    std::memset(&a, 0, sizeof a);
    a.n = 1;
    a.p[0] = ProbPtrs{fixed, moving, ffd, d_value, d_grad};
    return a;
}

// zero -> warp pass -> value pass -> finalise (phases 0..3 of the profile; a
// staged plan has no zero launch, its warp pass clears what needs clearing)
static int run_value(const srwcr_plan *P, const BatchArgs &args, int dense, int with_grad, unsigned char *ws,
                     hipStream_t s)
{
    const Geom &g = P->g;
    double *moments = (double *)(ws + P->ws.moments);
    const size_t nzero = (P->ws.counter + sizeof(double) - P->ws.moments) / sizeof(double);
    // A staged value pass writes every moment slot, so only an FFD gradient's
    // accumulators need clearing, and the warp pass does that on the side;
    // otherwise a fill kernel clears the moments and accumulators first.
    double *side_zero = nullptr;
    long side_n = 0;
    prof_mark(P, 0, s);
    if (!P->staged) {
        HIP_TRY(launch_zero(moments, nzero, s), "zero launch");
    } else if (with_grad && !dense) {
        side_zero = (double *)(ws + P->ws.grad);
        side_n = 3L * g.nc[0] * g.nc[1] * g.nc[2];
    }
    prof_mark(P, 1, s);
    HIP_TRY(launch_prep(P->geom_dev, g.mdt, dense, with_grad, P->wblocks, P->wrow, P->nwblocks, P->wrow_host.back(),
                        args, ws, P->prep_lds, s, side_zero, side_n),
            "warp launch");
    prof_mark(P, 2, s);
    const int nreg = kXN * P->value_bw * P->value_bw;
    const long stride = (long)nreg * g.nb * 3;
    if (P->cols)
        HIP_TRY(launch_value_cols(P->geom_dev, g.fdt, P->vblocks, P->cunits, P->ncunits, args, ws, s, P->value_bw),
                "value launch");
    else
        HIP_TRY(launch_value(P->geom_dev, g.fdt, P->vblocks, P->vrow, P->nvblocks, P->nwg, args, ws, P->value_lds, s,
                             P->staged ? (double *)(ws + P->staging_off) : nullptr, P->visit_start, stride,
                             P->value_bw),
                "value launch");
    prof_mark(P, 3, s);                     // the merge is timed with the finalisation
    if (P->staged)
        HIP_TRY(launch_merge(P->geom_dev, (const double *)(ws + P->staging_off), stride, nreg, P->reg_start, P->ent,
                             nullptr, g.R, g.nb, P->merge_waves, ws, s),
                "merge launch");
    HIP_TRY(launch_finalize(P->geom_dev, 1, g.R, args, ws, s, P->staged), "finalize launch");
    prof_mark(P, 4, s);
    return SRWCR_OK;
}

int srwcr_eval(const srwcr_plan *plan, const void *fixed, const void *moving, const float *ffd, double *d_value,
               void *workspace, size_t workspace_bytes, void *stream)
{
    int st = check_call(plan, fixed, moving, ffd, workspace, workspace_bytes);
    if (st) return st;
    if (!d_value) return fail(SRWCR_E_INVALID_ARG, "d_value is NULL");
    return run_value(plan, one_problem(fixed, moving, ffd, d_value, nullptr), 0, 0, (unsigned char *)workspace,
                     (hipStream_t)stream);
}

int srwcr_eval_dense(const srwcr_plan *plan, const void *fixed, const void *moving, const float *field,
                     double *d_value, void *workspace, size_t workspace_bytes, void *stream)
{
    int st = check_call(plan, fixed, moving, field, workspace, workspace_bytes);
    if (st) return st;
    if (!d_value) return fail(SRWCR_E_INVALID_ARG, "d_value is NULL");
    return run_value(plan, one_problem(fixed, moving, field, d_value, nullptr), 1, 0, (unsigned char *)workspace,
                     (hipStream_t)stream);
}

int srwcr_grad(const srwcr_plan *plan, const void *fixed, const void *moving, const float *ffd, double *d_value,
               float *d_grad, void *workspace, size_t workspace_bytes, void *stream)
{
    int st = check_call(plan, fixed, moving, ffd, workspace, workspace_bytes);
    if (st) return st;
    if (!d_value || !d_grad) return fail(SRWCR_E_INVALID_ARG, "d_value or d_grad is NULL");
    unsigned char *ws = (unsigned char *)workspace;
    hipStream_t s = (hipStream_t)stream;
    const BatchArgs args = one_problem(fixed, moving, ffd, d_value, d_grad);
    st = run_value(plan, args, 0, 1, ws, s);
    if (st) return st;
    const Geom &g = plan->g;
    if (plan->gcols)
        HIP_TRY(launch_grad_cols(plan->geom_dev, g.fdt, plan->items, plan->nitems, args, ws, s), "gradient launch");
    else
        HIP_TRY(launch_grad(plan->geom_dev, g.fdt, g.role, 0, plan->items, plan->nitems, args, ws, plan->grad_lds, s,
                            g.bw),
                "gradient launch");
    prof_mark(plan, 5, s);
    const size_t n = 3 * (size_t)g.nc[0] * g.nc[1] * g.nc[2];
    HIP_TRY(launch_grad_out(plan->geom_dev, 1, n, args, ws, s), "gradient output launch");
    prof_mark(plan, 6, s);
    if (plan->profiling && (size_t)(plan->prof_calls + 1) * (kPhases + 1) <= plan->ev_pool.size()) ++plan->prof_calls;
    return SRWCR_OK;
}

int srwcr_grad_dense(const srwcr_plan *plan, const void *fixed, const void *moving, const float *field,
                     double *d_value, float *d_grad, void *workspace, size_t workspace_bytes, void *stream)
{
    int st = check_call(plan, fixed, moving, field, workspace, workspace_bytes);
    if (st) return st;
    if (!d_value || !d_grad) return fail(SRWCR_E_INVALID_ARG, "d_value or d_grad is NULL");
    unsigned char *ws = (unsigned char *)workspace;
    hipStream_t s = (hipStream_t)stream;
    const BatchArgs args = one_problem(fixed, moving, field, d_value, d_grad);
    st = run_value(plan, args, 1, 1, ws, s);
    if (st) return st;
    const Geom &g = plan->g;
    HIP_TRY(launch_grad(plan->geom_dev, g.fdt, g.role, 1, plan->items, plan->nitems, args, ws, plan->grad_lds, s,
                        g.bw),
            "gradient launch");
    return SRWCR_OK;
}

int srwcr_grad_fixed(const srwcr_plan *plan, const void *fixed, const void *moving, const float *disp, int32_t dense,
                     double *d_value, float *d_grad_fixed, void *workspace, size_t workspace_bytes, void *stream)
{
    int st = check_call(plan, fixed, moving, disp, workspace, workspace_bytes);
    if (st) return st;
    if (dense != 0 && dense != 1) return fail(SRWCR_E_INVALID_ARG, "dense = %d is neither 0 nor 1", dense);
    if (!d_value || !d_grad_fixed) return fail(SRWCR_E_INVALID_ARG, "d_value or d_grad_fixed is NULL");
    unsigned char *ws = (unsigned char *)workspace;
    hipStream_t s = (hipStream_t)stream;
    const BatchArgs args = one_problem(fixed, moving, disp, d_value, d_grad_fixed);
    st = run_value(plan, args, dense, 0, ws, s);
    if (st) return st;
    const Geom &g = plan->g;
    HIP_TRY(launch_grad(plan->geom_dev, g.fdt, g.role, 2, plan->items, plan->nitems, args, ws, plan->grad_lds, s,
                        g.bw),
            "fixed-image adjoint launch");
    return SRWCR_OK;
}

int ffd_warp(const srwcr_plan *plan, const void *moving, const float *ffd, float *out, void *stream)
{
    if (!plan || !moving || !ffd || !out) return fail(SRWCR_E_INVALID_ARG, "NULL argument");
    HIP_TRY(launch_warp(plan->g, moving, ffd, out, (hipStream_t)stream), "warp launch");
    return SRWCR_OK;
}

int srwcr_debug_moments(const srwcr_plan *plan, const void *fixed, const void *moving, const float *ffd,
                        double *d_moments, void *workspace, size_t workspace_bytes, void *stream)
{
    int st = check_call(plan, fixed, moving, ffd, workspace, workspace_bytes);
    if (st) return st;
    if (!d_moments) return fail(SRWCR_E_INVALID_ARG, "d_moments is NULL");
    unsigned char *ws = (unsigned char *)workspace;
    hipStream_t s = (hipStream_t)stream;
    double *moments = (double *)(ws + plan->ws.moments);
    const size_t nzero = (plan->ws.counter + sizeof(double) - plan->ws.moments) / sizeof(double);
    HIP_TRY(launch_zero(moments, nzero, s), "zero launch");
    const Geom &g = plan->g;
    const BatchArgs args = one_problem(fixed, moving, ffd, nullptr, nullptr);
    HIP_TRY(launch_prep(plan->geom_dev, g.mdt, 0, 0, plan->wblocks, plan->wrow, plan->nwblocks,
                        plan->wrow_host.back(), args, ws, plan->prep_lds, s),
            "warp launch");
    const int nreg = kXN * plan->value_bw * plan->value_bw;
    const long stride = (long)nreg * g.nb * 3;
    if (plan->cols)
        HIP_TRY(launch_value_cols(plan->geom_dev, g.fdt, plan->vblocks, plan->cunits, plan->ncunits, args, ws, s,
                                  plan->value_bw),
                "value launch");
    else
        HIP_TRY(launch_value(plan->geom_dev, g.fdt, plan->vblocks, plan->vrow, plan->nvblocks, plan->nwg, args, ws,
                             plan->value_lds, s, plan->staged ? (double *)(ws + plan->staging_off) : nullptr,
                             plan->visit_start, stride, plan->value_bw),
                "value launch");
    if (plan->staged)
        HIP_TRY(launch_merge(plan->geom_dev, (const double *)(ws + plan->staging_off), stride, nreg, plan->reg_start,
                             plan->ent, nullptr, g.R, g.nb, plan->merge_waves, ws, s),
                "merge launch");
    const size_t bytes = (size_t)plan->g.R * plan->g.nb * 3 * sizeof(double);
    HIP_TRY(hipMemcpyAsync(d_moments, moments, bytes, hipMemcpyDeviceToDevice, s), "moments copy");
    return SRWCR_OK;
}

int srwcr_debug_samples(const srwcr_plan *plan, const void *moving, const float *ffd, int32_t *d_bin,
                        float *d_frac, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!plan) return fail(SRWCR_E_INVALID_ARG, "plan is NULL");
    if (!moving || !ffd) return fail(SRWCR_E_INVALID_ARG, "NULL volume or FFD pointer");
    if (!d_bin || !d_frac) return fail(SRWCR_E_INVALID_ARG, "d_bin or d_frac is NULL");
    if (!workspace) return fail(SRWCR_E_INVALID_ARG, "workspace is NULL");
    if (workspace_bytes < plan->ws.total)
        return fail(SRWCR_E_WORKSPACE, "workspace has %zu B, the plan needs %zu B", workspace_bytes, plan->ws.total);
    unsigned char *ws = (unsigned char *)workspace;
    hipStream_t s = (hipStream_t)stream;
    const Geom &g = plan->g;
    const BatchArgs args = one_problem(nullptr, moving, ffd, nullptr, nullptr);
    HIP_TRY(launch_prep(plan->geom_dev, g.mdt, 0, 0, plan->wblocks, plan->wrow, plan->nwblocks,
                        plan->wrow_host.back(), args, ws, plan->prep_lds, s),
            "warp launch");
    const size_t nvox = (size_t)g.nf[0] * g.nf[1] * g.nf[2];
    HIP_TRY(launch_unpack_samples((const PrepKT *)(ws + plan->ws.kt), nvox, d_bin, d_frac, s), "unpack launch");
    return SRWCR_OK;
}

int srwcr_plan_info(const srwcr_plan *plan, int32_t *n_items, int32_t *value_lds, int32_t *grad_lds)
{
    if (!plan) return fail(SRWCR_E_INVALID_ARG, "plan is NULL");
    if (n_items) *n_items = plan->nitems;
    if (value_lds) *value_lds = (int32_t)plan->value_lds;
    if (grad_lds) *grad_lds = (int32_t)plan->grad_lds;
    return SRWCR_OK;
}

int srwcr_profile(const srwcr_plan *plan, int32_t enable)
{
    if (!plan) return fail(SRWCR_E_INVALID_ARG, "plan is NULL");
    if (enable && plan->ev_pool.empty()) {
        plan->ev_pool.resize(kProfCalls * (kPhases + 1));
        for (auto &e : plan->ev_pool) HIP_TRY(hipEventCreate(&e), "hipEventCreate");
    }
    if (enable < 0 || enable > 3) return fail(SRWCR_E_INVALID_ARG, "profile mode %d is not 0, 1, 2 or 3", enable);
    plan->profiling = enable;
    plan->prof_calls = 0;
    return SRWCR_OK;
}

int srwcr_profile_read(const srwcr_plan *plan, double ms[6], int32_t *calls)
{
    if (!plan || !ms) return fail(SRWCR_E_INVALID_ARG, "NULL argument");
    for (int k = 0; k < kPhases; ++k) ms[k] = 0.0;
    for (int32_t c = 0; c < plan->prof_calls; ++c) {
        const size_t base = (size_t)c * (kPhases + 1);
        if (plan->profiling >= 2) {
            const int k = prof_phase(plan->profiling);
            float t = 0.0f;
            HIP_TRY(hipEventSynchronize(plan->ev_pool[base + k + 1]), "hipEventSynchronize");
            HIP_TRY(hipEventElapsedTime(&t, plan->ev_pool[base + k], plan->ev_pool[base + k + 1]),
                    "hipEventElapsedTime");
            ms[k] += t;
            continue;
        }
        HIP_TRY(hipEventSynchronize(plan->ev_pool[base + kPhases]), "hipEventSynchronize");
        for (int k = 0; k < kPhases; ++k) {
            float t = 0.0f;
            HIP_TRY(hipEventElapsedTime(&t, plan->ev_pool[base + k], plan->ev_pool[base + k + 1]),
                    "hipEventElapsedTime");
            ms[k] += t;
        }
    }
    if (calls) *calls = plan->prof_calls;
    return SRWCR_OK;
}

// ------------------------------------------------------------------ batches
struct srwcr_batch {
    std::vector<const srwcr_plan *> plans;   // not owned: their per-axis tables are referenced
    int fdt = 0, mdt = 0, role = 0;
    Geom *geoms_dev = nullptr;
    WorkItem *items_dev = nullptr;
    int nitems = 0;
    WorkItem *vblocks_dev = nullptr;
    int *vrow_dev = nullptr;
    int nvblocks = 0, nwg = 0;
    long nrows = 0;
    size_t value_lds = 0, grad_lds = 0, prep_lds = 0, ws_total = 0, zero_bytes = 0, max_params = 0;
    int max_regions = 0;
    // staged value pass (see stage_plan)
    bool staged = false;
    int *visit_start = nullptr, *reg_start = nullptr, *ent = nullptr;
    int2 *reg_id = nullptr;
    int nregions = 0, max_nb = 0, merge_waves = 1;
    int bw = 4, nreg = kXN * 16;                 // value-block shape (see srwcr_plan::value_bw)
    int4 *cunits_dev = nullptr;                  // column value pass (bw = 5), see srwcr_plan::cols
    int ncunits = 0;
    bool gcols = false;                          // every plan takes the column gradient pass
    long stage_stride = 0;
    size_t staging_off = 0;
};

void srwcr_batch_destroy(srwcr_batch *b)
{
    if (!b) return;
    if (b->geoms_dev) (void)hipFree(b->geoms_dev);
    if (b->items_dev) (void)hipFree(b->items_dev);
    if (b->cunits_dev) (void)hipFree(b->cunits_dev);
    if (b->vblocks_dev) (void)hipFree(b->vblocks_dev);
    if (b->vrow_dev) (void)hipFree(b->vrow_dev);
    for (void *p : {(void *)b->visit_start, (void *)b->reg_start, (void *)b->ent, (void *)b->reg_id})
        if (p) (void)hipFree(p);
    delete b;
}

int srwcr_batch_create(int32_t n, const srwcr_plan *const *plans, srwcr_batch **out)
{
    if (!out) return fail(SRWCR_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!plans) return fail(SRWCR_E_INVALID_ARG, "plans is NULL");
    if (n < 1 || n > kMaxBatch) return fail(SRWCR_E_INVALID_ARG, "batch of %d problems outside 1..%d", n, kMaxBatch);
    for (int p = 0; p < n; ++p) {
        if (!plans[p]) return fail(SRWCR_E_INVALID_ARG, "plans[%d] is NULL", p);
        const Geom &g = plans[p]->g, &g0 = plans[0]->g;
        if (g.fdt != g0.fdt || g.mdt != g0.mdt || g.role != g0.role)
            return fail(SRWCR_E_INVALID_ARG, "plans[%d] differs from plans[0] in role or storage dtypes", p);
        if (plans[p]->device != plans[0]->device)
            return fail(SRWCR_E_INVALID_ARG, "plans[%d] was made on another device", p);
        if (plans[p]->value_bw != plans[0]->value_bw)
            return fail(SRWCR_E_UNSUPPORTED, "plans[%d] uses value blocks of %d (y, z) regions per axis, plans[0] %d",
                        p, plans[p]->value_bw, plans[0]->value_bw);
    }
    srwcr_batch *b = new srwcr_batch();
    b->plans.assign(plans, plans + n);
    b->fdt = plans[0]->g.fdt;
    b->mdt = plans[0]->g.mdt;
    b->role = plans[0]->g.role;
    // workspace: every problem's zeroed block (moments, gradient) first, then the rest
    std::vector<Geom> geoms(n);
    size_t off = 0;
    for (int p = 0; p < n; ++p) {
        const Geom &g = plans[p]->g;
        geoms[p] = g;
        WsLayout &w = geoms[p].ws;
        const size_t ncell = (size_t)g.nc[0] * g.nc[1] * g.nc[2];
        w.moments = off;
        off += (size_t)g.R * g.nb * 3 * sizeof(double);
        w.grad = off;
        off += 3 * ncell * sizeof(double);
        w.counter = off;
        off += sizeof(double);
        off = align_up(off, 256);
        b->max_regions = std::max(b->max_regions, g.R);
        b->max_params = std::max(b->max_params, 3 * ncell);
        b->value_lds = std::max(b->value_lds, plans[p]->value_lds);
        b->prep_lds = std::max(b->prep_lds, plans[p]->prep_lds);
        b->grad_lds = std::max(b->grad_lds, plans[p]->grad_lds);
    }
    b->zero_bytes = off;
    for (int p = 0; p < n; ++p) {
        const Geom &g = plans[p]->g;
        WsLayout &w = geoms[p].ws;
        w.region = off;
        off = align_up(off + (size_t)g.R * 4 * sizeof(double), 256);
        w.tables = off;
        off = align_up(off + (size_t)g.R * g.nb * 4 * sizeof(float), 256);
        w.alpha = off;
        off = align_up(off + (size_t)g.R * sizeof(float), 256);
        const size_t nvox = (size_t)g.nf[0] * g.nf[1] * g.nf[2];
        w.kt = off;
        off = align_up(off + nvox * sizeof(PrepKT), 256);
        w.dm = off;
        off = align_up(off + 3 * nvox * sizeof(float), 256);
        w.total = 0;
    }
    b->ws_total = off;
    // one work list: the largest boxes first, so the small problems fill the tail
    std::vector<WorkItem> items;
    for (int p = 0; p < n; ++p)
        for (WorkItem w : plans[p]->items_host) {
            w.prob = p;
            items.push_back(w);
        }
    auto vox = [](const WorkItem &w) { return (long)(w.x1 - w.x0) * (w.y1 - w.y0) * (w.z1 - w.z0); };
    std::stable_sort(items.begin(), items.end(), [&](const WorkItem &a, const WorkItem &c) { return vox(a) > vox(c); });
    b->nitems = (int)items.size();
    b->gcols = true;
    for (int p = 0; p < n; ++p) b->gcols = b->gcols && plans[p]->gcols;
    // value-pass blocks of every problem, one row list
    std::vector<WorkItem> vb;
    std::vector<int> vr(1, 0);
    for (int p = 0; p < n; ++p)
        for (size_t i = 0; i < plans[p]->vblocks_host.size(); ++i) {
            WorkItem w = plans[p]->vblocks_host[i];
            w.prob = p;
            vb.push_back(w);
            vr.push_back(vr.back() + (plans[p]->vrow_host[i + 1] - plans[p]->vrow_host[i]));
        }
    b->nvblocks = (int)vb.size();
    b->nrows = vr.back();
    int nwg_max = 0;
    for (int p = 0; p < n; ++p) nwg_max = std::max(nwg_max, plans[p]->nwg);
    b->nwg = std::max(1, std::min(nwg_max, vr.back()));
    hipError_t e = hipMalloc(&b->geoms_dev, n * sizeof(Geom));
    if (e == hipSuccess) e = hipMemcpy(b->geoms_dev, geoms.data(), n * sizeof(Geom), hipMemcpyHostToDevice);
    if (e == hipSuccess && !items.empty()) e = hipMalloc(&b->items_dev, items.size() * sizeof(WorkItem));
    if (e == hipSuccess && !items.empty())
        e = hipMemcpy(b->items_dev, items.data(), items.size() * sizeof(WorkItem), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&b->vblocks_dev, vb.size() * sizeof(WorkItem));
    if (e == hipSuccess) e = hipMemcpy(b->vblocks_dev, vb.data(), vb.size() * sizeof(WorkItem), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&b->vrow_dev, vr.size() * sizeof(int));
    if (e == hipSuccess) e = hipMemcpy(b->vrow_dev, vr.data(), vr.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        for (int p = 0; p < n; ++p) b->max_nb = std::max(b->max_nb, plans[p]->g.nb);
        b->bw = plans[0]->value_bw;
        b->nreg = kXN * b->bw * b->bw;
        if (b->bw == 5) {
            // the single plans' column value pass, over all problems' blocks
            const std::vector<int4> cu = column_units(vb);
            b->ncunits = (int)cu.size();
            e = hipMalloc(&b->cunits_dev, cu.size() * sizeof(int4));
            if (e == hipSuccess) e = hipMemcpy(b->cunits_dev, cu.data(), cu.size() * sizeof(int4), hipMemcpyHostToDevice);
        }
    }
    if (e == hipSuccess && b->bw != 5) {
        // staged value pass over all problems' blocks, when its slots fit
        std::vector<const Geom *> gp(n);
        for (int p = 0; p < n; ++p) gp[p] = &plans[p]->g;
        const StagePlan sp = stage_plan(vb, vr, b->nwg, gp, b->bw);
        b->stage_stride = (long)b->nreg * b->max_nb * 3;
        const size_t stage_bytes = sp.visits * (size_t)b->stage_stride * sizeof(double);
        if (stage_bytes <= kStageLimit && sp.visits * b->nreg < (size_t)INT32_MAX && !sp.ent.empty()) {
            auto put = [&](const void *src, size_t bytes, void **dst) {
                if (e == hipSuccess) e = hipMalloc(dst, bytes);
                if (e == hipSuccess) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
            };
            put(sp.vstart.data(), sp.vstart.size() * sizeof(int), (void **)&b->visit_start);
            put(sp.reg_start.data(), sp.reg_start.size() * sizeof(int), (void **)&b->reg_start);
            put(sp.ent.data(), sp.ent.size() * sizeof(int), (void **)&b->ent);
            put(sp.reg_id.data(), sp.reg_id.size() * sizeof(int2), (void **)&b->reg_id);
            b->nregions = (int)sp.reg_id.size();
            b->merge_waves = sp.waves;
            b->staging_off = align_up(b->ws_total, 256);
            b->ws_total = align_up(b->staging_off + stage_bytes, 256);
            b->staged = e == hipSuccess;
        }
    }
    if (e != hipSuccess) {
        srwcr_batch_destroy(b);
        return hip_fail(e, "batch tables");
    }
    *out = b;
    return SRWCR_OK;
}

size_t srwcr_batch_workspace_bytes(const srwcr_batch *b) { return b ? b->ws_total : 0; }

int srwcr_grad_batched(const srwcr_batch *b, const srwcr_batch_item *items, void *workspace, size_t workspace_bytes,
                       void *stream)
{
    if (!b || !items) return fail(SRWCR_E_INVALID_ARG, "NULL batch or items");
    if (!workspace) return fail(SRWCR_E_INVALID_ARG, "workspace is NULL");
    if (workspace_bytes < b->ws_total)
        return fail(SRWCR_E_WORKSPACE, "workspace has %zu B, the batch needs %zu B", workspace_bytes, b->ws_total);
    const int n = (int)b->plans.size();
    BatchArgs args;
    std::memset(&args, 0, sizeof args);
    args.n = n;
    for (int p = 0; p < n; ++p) {
        const srwcr_batch_item &it = items[p];
        if (!it.fixed || !it.moving || !it.ffd || !it.d_value || !it.d_grad)
            return fail(SRWCR_E_INVALID_ARG, "items[%d] has a NULL pointer", p);
        args.p[p] = ProbPtrs{it.fixed, it.moving, it.ffd, it.d_value, it.d_grad};
    }
    unsigned char *ws = (unsigned char *)workspace;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_zero((double *)ws, b->zero_bytes / sizeof(double), s), "zero launch");
    HIP_TRY(launch_prep(b->geoms_dev, b->mdt, 0, 1, b->vblocks_dev, b->vrow_dev, b->nvblocks, b->nrows, args, ws,
                        b->prep_lds, s),
            "warp launch");
    double *staging = b->staged ? (double *)(ws + b->staging_off) : nullptr;
    if (b->bw == 5)
        HIP_TRY(launch_value_cols(b->geoms_dev, b->fdt, b->vblocks_dev, b->cunits_dev, b->ncunits, args, ws, s, b->bw),
                "value launch");
    else
        HIP_TRY(launch_value(b->geoms_dev, b->fdt, b->vblocks_dev, b->vrow_dev, b->nvblocks, b->nwg, args, ws,
                             b->value_lds, s, staging, b->visit_start, b->stage_stride, b->bw),
                "value launch");
    if (b->staged)
        HIP_TRY(launch_merge(b->geoms_dev, staging, b->stage_stride, b->nreg, b->reg_start, b->ent, b->reg_id,
                             b->nregions,
                             b->max_nb, b->merge_waves, ws, s),
                "merge launch");
    HIP_TRY(launch_finalize(b->geoms_dev, n, b->max_regions, args, ws, s, b->staged), "finalize launch");
    if (b->gcols)
        HIP_TRY(launch_grad_cols(b->geoms_dev, b->fdt, b->items_dev, b->nitems, args, ws, s), "gradient launch");
    else
        HIP_TRY(launch_grad(b->geoms_dev, b->fdt, b->role, 0, b->items_dev, b->nitems, args, ws, b->grad_lds, s,
                            b->bw),
                "gradient launch");
    HIP_TRY(launch_grad_out(b->geoms_dev, n, b->max_params, args, ws, s), "gradient output launch");
    return SRWCR_OK;
}

// ------------------------------------------------------------------- RaPTOR
struct raptor_patches {
    const srwcr_plan *plan = nullptr;        // the plan the set was made for (not owned)
    int npatch = 0, npieces = 0;
    RaptorPatch *patches_dev = nullptr;
    RaptorPiece *pieces_dev = nullptr;
    // workspace offsets beyond the plan's SRWCR slots (rds starts at ws.total)
    size_t stats = 0, stats_end = 0, tval = 0, mu = 0, scal = 0, total = 0;
};

namespace {
constexpr int kRaptorPiece = 2048;           // voxels of one workgroup of the RaPTOR passes
constexpr int kRaptorMaxPatches = 1 << 24;
}  // namespace

void raptor_patches_destroy(raptor_patches *pt)
{
    if (!pt) return;
    if (pt->patches_dev) (void)hipFree(pt->patches_dev);
    if (pt->pieces_dev) (void)hipFree(pt->pieces_dev);
    delete pt;
}

int raptor_patches_create(const srwcr_plan *plan, const srwcr_patch *patches, int32_t n, raptor_patches **out)
{
    if (!out) return fail(SRWCR_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!plan || !patches) return fail(SRWCR_E_INVALID_ARG, "NULL plan or patches");
    if (n < 1 || n > kRaptorMaxPatches)
        return fail(SRWCR_E_INVALID_ARG, "%d patches outside 1..%d", n, kRaptorMaxPatches);
    const Geom &g = plan->g;
    if ((double)g.nf[0] * g.nf[1] * g.nf[2] >= 2147483648.0)
        return fail(SRWCR_E_UNSUPPORTED, "RaPTOR needs a fixed grid of fewer than 2^31 voxels");
    std::vector<RaptorPatch> pv(n);
    std::vector<RaptorPiece> pc;
    for (int r = 0; r < n; ++r) {
        const srwcr_patch &q = patches[r];
        const int lo[3] = {q.x0, q.y0, q.z0}, hi[3] = {q.x1, q.y1, q.z1};
        int b0[3], ext[3];
        bool empty = false;
        for (int e = 0; e < 3; ++e) {
            b0[e] = std::max(lo[e], 0);
            const int b1 = std::min(hi[e], g.nf[e]);
            ext[e] = b1 - b0[e];
            if (ext[e] <= 0) empty = true;
        }
        RaptorPatch &P = pv[r];
        P = RaptorPatch{b0[0], b0[1], b0[2], 0, 0, 0, 0, 0};
        if (empty) continue;                // counts in N_p, adds nothing (clipped away)
        P.nx = ext[0];
        P.ny = ext[1];
        P.nz = ext[2];
        P.n = ext[0] * ext[1] * ext[2];     // < 2^31: inside the grid
        for (int st = 0; st < P.n; st += kRaptorPiece) pc.push_back(RaptorPiece{r, st, std::min(kRaptorPiece, P.n - st), 0});
    }
    raptor_patches *pt = new raptor_patches();
    pt->plan = plan;
    pt->npatch = n;
    pt->npieces = (int)pc.size();
    hipError_t e = hipMalloc(&pt->patches_dev, pv.size() * sizeof(RaptorPatch));
    if (e == hipSuccess) e = hipMemcpy(pt->patches_dev, pv.data(), pv.size() * sizeof(RaptorPatch), hipMemcpyHostToDevice);
    if (e == hipSuccess && !pc.empty()) e = hipMalloc(&pt->pieces_dev, pc.size() * sizeof(RaptorPiece));
    if (e == hipSuccess && !pc.empty())
        e = hipMemcpy(pt->pieces_dev, pc.data(), pc.size() * sizeof(RaptorPiece), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        raptor_patches_destroy(pt);
        return hip_fail(e, "RaPTOR patch tables");
    }
    // workspace: the plan's SRWCR slots, then rds [nvox] and the zeroed patch
    // sums, then the finalised tables
    const size_t nvox = (size_t)g.nf[0] * g.nf[1] * g.nf[2];
    size_t off = plan->ws.rds + align_up(nvox * sizeof(float), 256);
    pt->stats = off;
    off += (size_t)n * (2 * g.nb + 3) * sizeof(double);
    pt->stats_end = off;
    off = align_up(off, 256);
    pt->tval = off;
    off = align_up(off + (size_t)n * sizeof(double), 256);
    pt->mu = off;
    off = align_up(off + (size_t)n * g.nb * sizeof(float2), 256);
    pt->scal = off;
    off = align_up(off + (size_t)n * sizeof(float4), 256);
    pt->total = off;
    *out = pt;
    return SRWCR_OK;
}

size_t raptor_workspace_bytes(const srwcr_plan *plan, const raptor_patches *pt)
{
    return plan && pt && pt->plan == plan ? pt->total : 0;
}

static int run_raptor(const srwcr_plan *plan, const raptor_patches *pt, const void *fixed, const void *moving,
                      const float *disp, int32_t dense, double *d_value, float *d_grad, void *workspace,
                      size_t workspace_bytes, void *stream)
{
    if (!plan || !pt) return fail(SRWCR_E_INVALID_ARG, "NULL plan or patch set");
    if (pt->plan != plan) return fail(SRWCR_E_INVALID_ARG, "the patch set was made for another plan");
    if (!fixed || !moving || !disp) return fail(SRWCR_E_INVALID_ARG, "NULL volume or displacement pointer");
    if (dense != 0 && dense != 1) return fail(SRWCR_E_INVALID_ARG, "dense = %d is neither 0 nor 1", dense);
    if (!d_value) return fail(SRWCR_E_INVALID_ARG, "d_value is NULL");
    if (!workspace) return fail(SRWCR_E_INVALID_ARG, "workspace is NULL");
    if (workspace_bytes < pt->total)
        return fail(SRWCR_E_WORKSPACE, "workspace has %zu B, RaPTOR needs %zu B", workspace_bytes, pt->total);
    const Geom &g = plan->g;
    unsigned char *ws = (unsigned char *)workspace;
    hipStream_t s = (hipStream_t)stream;
    const bool with_grad = d_grad != nullptr;
    const BatchArgs args = one_problem(fixed, moving, disp, d_value, d_grad);
    RaptorArgs ra;
    ra.patches = pt->patches_dev;
    ra.pieces = pt->pieces_dev;
    ra.npatch = pt->npatch;
    ra.npieces = pt->npieces;
    ra.stats = (double *)(ws + pt->stats);
    ra.tval = (double *)(ws + pt->tval);
    ra.mu = (float2 *)(ws + pt->mu);
    ra.scal = (float4 *)(ws + pt->scal);
    ra.rds = (float *)(ws + plan->ws.rds);
    ra.value = d_value;
    // profiled gradient calls mark: zero, warp, patch sums, patch finalise,
    // derivative, chain rule (gradient pass and output), end
    auto mark = [&](int k) {
        if (with_grad) prof_mark(plan, k, s);
    };
    // zero: the patch sums, and for a gradient rds and the FFD accumulators
    const size_t zlo = with_grad ? plan->ws.rds : pt->stats;
    mark(0);
    HIP_TRY(launch_zero((double *)(ws + zlo), (pt->stats_end - zlo) / sizeof(double), s), "zero launch");
    if (with_grad && !dense)
        HIP_TRY(launch_zero((double *)(ws + plan->ws.grad), 3 * (size_t)g.nc[0] * g.nc[1] * g.nc[2], s), "zero launch");
    mark(1);
    HIP_TRY(launch_prep(plan->geom_dev, g.mdt, dense, with_grad ? 1 : 0, plan->wblocks, plan->wrow, plan->nwblocks,
                        plan->wrow_host.back(), args, ws, plan->prep_lds, s),
            "warp launch");
    mark(2);
    HIP_TRY(launch_raptor_acc(plan->geom_dev, g.fdt, g.role, ra, args, ws, s), "RaPTOR accumulation launch");
    mark(3);
    HIP_TRY(launch_raptor_finalize(plan->geom_dev, ra, s), "RaPTOR finalize launch");
    if (!with_grad) return SRWCR_OK;
    mark(4);
    HIP_TRY(launch_raptor_ds(plan->geom_dev, g.fdt, g.role, ra, args, ws, s), "RaPTOR derivative launch");
    mark(5);
    HIP_TRY(launch_grad(plan->geom_dev, 0, 2, dense, plan->items, plan->nitems, args, ws, plan->grad_lds, s, g.bw),
            "gradient launch");
    if (!dense) {
        const size_t n = 3 * (size_t)g.nc[0] * g.nc[1] * g.nc[2];
        HIP_TRY(launch_grad_out(plan->geom_dev, 1, n, args, ws, s), "gradient output launch");
    }
    mark(6);
    if (plan->profiling && (size_t)(plan->prof_calls + 1) * (kPhases + 1) <= plan->ev_pool.size()) ++plan->prof_calls;
    return SRWCR_OK;
}

int raptor_eval(const srwcr_plan *plan, const raptor_patches *patches, const void *fixed, const void *moving,
                const float *disp, int32_t dense, double *d_value, void *workspace, size_t workspace_bytes,
                void *stream)
{
    return run_raptor(plan, patches, fixed, moving, disp, dense, d_value, nullptr, workspace, workspace_bytes, stream);
}

int raptor_grad(const srwcr_plan *plan, const raptor_patches *patches, const void *fixed, const void *moving,
                const float *disp, int32_t dense, double *d_value, float *d_grad, void *workspace,
                size_t workspace_bytes, void *stream)
{
    if (!d_grad) return fail(SRWCR_E_INVALID_ARG, "d_grad is NULL");
    return run_raptor(plan, patches, fixed, moving, disp, dense, d_value, d_grad, workspace, workspace_bytes, stream);
}

void srwcr_lbfgs_default_opts(srwcr_lbfgs_opts *o)
{
    if (!o) return;
    o->levels = 3;
    o->max_iter[0] = 200;
    o->max_iter[1] = 200;
    o->max_iter[2] = 120;
    o->history = 5;
    o->stall_window = 20;
    o->stall_tol = 1e-6;
    o->bending_weight = 0.0;
}

}  // extern "C"
