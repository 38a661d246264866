// srwcr_internal.h -- types shared by the host library and the gfx950 kernels.
// Not part of the public ABI (include/srwcr.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct srwcr_plan;

namespace srwcr {

constexpr int kMaxBins = 64;      // L_eps + 1 <= 64: one wave lane per intensity bin
constexpr int kWave = 64;         // CDNA wavefront width
constexpr int kXN = 5;            // x-nodes of a work item (its x-range spans at most two spatial cells)
constexpr int kNReg = kXN * 16;   // regions of a work item: 5 (x) x 4 (y) x 4 (z)
constexpr int kWin = 4;           // bin slots of one value-pass window (A-bins kmin .. kmin + 3)
constexpr int kValueThreads = 768;
constexpr int kGradThreads = 1024;
constexpr int kRowBins = 32;      // gradient pass: bins of one chunk of a row's tables
constexpr int kRowEntry = 20;     // floats per row-table entry: 15 used, padded for 16-byte loads on distinct banks
constexpr int kMaxNodeSeg = 68;   // FFD x-nodes one 64-voxel row segment can touch (delta >= 1)
constexpr int kSlots = 2;         // voxels per lane: an item row holds up to 2 x 64 voxels
constexpr int kMaxBatch = 32;     // problems of one batched launch
constexpr int kXcds = 8;          // accelerator complex dies of an MI355X, each with its own L2

// One unit of work of the value and gradient passes: a box of fixed voxels
// inside one spatial-bin cell along y and z and at most two cells along x, so
// that all its voxels draw their 64 regions (eq 7) from the same 5x4x4 block.
struct WorkItem {
    int x0, x1, y0, y1, z0, z1;   // half-open voxel ranges
    int cx, cy, cz;               // first region of the block: (cx+i, cy+j, cz+k), i < 5, j, k < 4
    int gx0, gy0, gz0;            // first FFD node of the item's control support
    int gnx, gny, gnz;            // extent of that support
    int prob;                     // problem of a batched launch (0 for a single plan)
};

// Workspace layout (device bytes, offsets from the workspace base of a launch).
struct WsLayout {
    size_t moments;    // double [R][nb][3]   (P, S1, S2)
    size_t region;     // double [R][4]       per-region results written by finalise
    size_t tables;     // float  [R][nb][4]   gradient tables (role dependent)
    size_t alpha;      // float  [R]          role B: CR_r / (sigma_r^2 Z)
    size_t grad;       // double [3][nc]      gradient accumulators
    size_t counter;    // 8 B                 end of the zeroed block (unused slot)
    size_t kt;         // PrepKT [nvox]       warped moving bin and in-bin position per fixed voxel
    size_t dm;         // float  [3][nvox]    dM/dy at the warped position (gradient calls)
    size_t total;      // end of the SRWCR slots
    size_t rds;        // float  [nvox]       RaPTOR: dRaPTOR/ds_M per voxel (starts at `total`)
};

// One fixed voxel's warped moving sample s, as the value and gradient passes
// use it: bin k = min(floor(s), L - 1) decided in FP64, t = s - k in FP32.
struct PrepKT {
    float t;
    int k;
};

// Per-call device pointers of one problem, passed by value in the kernel
// arguments (up to kMaxBatch of them per launch).
struct ProbPtrs {
    const void *fixed;
    const void *moving;
    const float *ffd;  // FFD coefficients, or a dense field [3][nz][ny][nx]
    double *value;     // D
    float *grad;       // dD/d(displacement), layout of ffd (unused by value-only calls)
};

struct BatchArgs {
    int n;
    int pad;
    ProbPtrs p[kMaxBatch];
};

// Everything a kernel needs to know about a problem, passed by value.
struct Geom {
    int nf[3];        // fixed grid
    int nm[3];        // moving grid
    int nc[3];        // FFD control grid
    int K[3];         // spatial bins per axis
    int delta[3];     // FFD spacing
    int nb;           // intensity bins (L + 1)
    int role;         // 0: moving is A, 1: moving is B
    int fdt, mdt;     // storage dtypes of the normalised volumes
    int R;            // K[0] K[1] K[2]
    int same_grid[3]; // moving axis length == fixed axis length
    float ratio[3];   // nm / nf per axis
    double inv_Z;     // 1 / number of fixed voxels
    // per-axis tables (device pointers)
    const int *sp_cell[3];     // spatial cell of each fixed coordinate, 0..K-4
    const float4 *sp_w[3];     // its four cubic B-spline weights (eq 8)
    const int *ffd_p[3];       // x / delta
    const double4 *ffd_w[3];   // beta_0..3((x mod delta) / delta), FP64 (the warp runs in FP64)
    const int *mv_base[3];     // floor((x + 1/2) M / N - 1/2) (unequal grids only)
    const double *mv_frac[3];  // (x + 1/2) M / N - 1/2 - base
    double ratio_d[3];         // nm / nf per axis
    int xw;                    // x-width of the work items (64 or 128 voxels)
    int c1n;                   // FFD x-nodes an item row touches at most: (xw - 1) / delta + 5 (warp pass)
    int gscr;                  // floats of per-wave scratch in the gradient pass
    int bw;                    // (y, z) regions per axis of a value block and gradient item: 4 (one
                               // spatial cell) or 5 (two cells, for small cells)
    WsLayout ws;               // this problem's slots in the workspace of a launch
};

// RaPTOR (eqs 6, 13, 14).  A patch clipped to the fixed grid: origin, extent
// and voxel count (0 for a patch that lies outside the grid).
struct RaptorPatch {
    int x0, y0, z0;
    int nx, ny, nz;
    int n;
    int pad;
};

// A run of consecutive voxels of one patch (x fastest, then y, then z),
// the unit of one workgroup of the RaPTOR passes.
struct RaptorPiece {
    int patch;
    int start;
    int count;
    int pad;
};

// Device slots of one RaPTOR call.  B enters the sums shifted by c_r, the
// value of B at the patch's first voxel, which leaves eq 13 unchanged and
// keeps the FP32 products small.
struct RaptorArgs {
    const RaptorPatch *patches;
    const RaptorPiece *pieces;
    int npatch;
    int npieces;
    double *stats;     // [npatch][2 nb + 2]: P_a, S1_a (a < nb), sum B', sum B'^2
    double *tval;      // [npatch] the patch terms T_r
    float2 *mu;        // [npatch][nb] (mu_r(a) - c_r, 1), or (0, 0) for an empty bin
    float4 *scal;      // [npatch] (1 / (N_r sigma_r^2), or 0 for a skipped patch; T_r; E1 - c_r; c_r)
    float *rds;        // [nvox] dRaPTOR/ds_M
    double *value;     // RaPTOR
};

// Launchers (srwcr_kernels.hip).  `geoms` is a device array with one Geom per
// problem; items carry their problem index; `ws` is the launch's workspace base.
hipError_t launch_zero(double *p, size_t n, hipStream_t s);
hipError_t launch_normalize(const float *in, int64_t n, float lo, float scale, float L, void *out, int dt,
                            hipStream_t s);
hipError_t launch_minmax(const float *in, int64_t n, float *partial, int nblocks, hipStream_t s);
// zero / nzero: doubles the warp pass clears on the side (or none).
hipError_t launch_prep(const Geom *geoms, int mdt, int dense, int with_grad, const WorkItem *blocks,
                       const int *row_start, int nblocks, long nrows, const BatchArgs &args, unsigned char *ws,
                       size_t lds_bytes, hipStream_t s, double *zero = nullptr, long nzero = 0);
// Value pass over region blocks: row_start[b] = first row (in a list of all
// blocks' rows) of block b, row_start[nblocks] = total; nwg persistent
// workgroups share the rows evenly.
// bw: the (y, z) regions of a value block per axis, 4 (one spatial cell) or 5
// (two cells).  With `staging` set, each workgroup writes its histogram per block visit
// (visit_start[w] = the first visit id of workgroup w) to the staging slots
// of the visit, [80 local regions][nb][3] from visit * stage_stride, and
// launch_merge forms the moments; otherwise the histograms are merged with
// FP64 atomics.
hipError_t launch_value(const Geom *geoms, int fdt, const WorkItem *blocks, const int *row_start, int nblocks,
                        int nwg, const BatchArgs &args, unsigned char *ws, size_t lds_bytes, hipStream_t s,
                        double *staging = nullptr, const int *visit_start = nullptr, long stage_stride = 0,
                        int bw = 4);
// Value pass by block columns: units[u] = (value block, first column, end
// column) with columns (x, y) of the block numbered x fastest; one wave per
// unit, column sums on the matrix cores, FP64 atomics into the global moments
// (which must start at zero).  bw: the blocks' (y, z) regions per axis.
hipError_t launch_value_cols(const Geom *geoms, int fdt, const WorkItem *blocks, const int4 *units, int nunits,
                             const BatchArgs &args, unsigned char *ws, hipStream_t s, int bw);
size_t value_cols_lds_bytes();
// Gradient pass by box columns (moving image as A, FFD): one wave per box of
// at most 128 columns (x, y), 5 FFD z-nodes and 32 FFD (x, y) nodes, inside
// two spatial cells per axis; FP64 atomics into the gradient accumulators.
hipError_t launch_grad_cols(const Geom *geoms, int fdt, const WorkItem *items, int nitems, const BatchArgs &args,
                            unsigned char *ws, hipStream_t s);
// reg_id: (problem, region) per merged region, or null for regions 0 .. n - 1
// of problem 0.  Also finalises each region (results, gradient tables).
hipError_t launch_merge(const Geom *geoms, const double *staging, long stage_stride, int nreg, const int *reg_start,
                        const int *ent, const int2 *reg_id, int nregions, int max_nb, int waves, unsigned char *ws,
                        hipStream_t s);
// Region results and tables (skipped when `merged`: launch_merge wrote them),
// then the value D of each problem.
hipError_t launch_finalize(const Geom *geoms, int nprob, int max_regions, const BatchArgs &args, unsigned char *ws,
                           hipStream_t s, bool merged = false);
hipError_t launch_grad(const Geom *geoms, int fdt, int role, int dense, const WorkItem *items, int nitems,
                       const BatchArgs &args, unsigned char *ws, size_t lds_bytes, hipStream_t s, int bw = 4);
hipError_t launch_grad_out(const Geom *geoms, int nprob, size_t max_params, const BatchArgs &args, unsigned char *ws,
                           hipStream_t s);
hipError_t launch_raptor_acc(const Geom *geoms, int fdt, int role, const RaptorArgs &ra, const BatchArgs &args,
                             const unsigned char *ws, hipStream_t s);
hipError_t launch_raptor_finalize(const Geom *geoms, const RaptorArgs &ra, hipStream_t s);
hipError_t launch_raptor_ds(const Geom *geoms, int fdt, int role, const RaptorArgs &ra, const BatchArgs &args,
                            const unsigned char *ws, hipStream_t s);
hipError_t launch_warp(const Geom &g, const void *moving, const float *ffd, float *out, hipStream_t s);
// The warp pass's per-voxel moving bin and in-bin position, unpacked into two arrays.
hipError_t launch_unpack_samples(const PrepKT *kt, size_t n, int32_t *bin, float *frac, hipStream_t s);
hipError_t launch_downsample(const float *in, int nx, int ny, int nz, float *out, int ox, int oy, int oz,
                             hipStream_t s);
hipError_t prepare_kernels();   // once per device: LDS limits of the value and gradient kernels

// Host library (srwcr_host.cpp): set the calling thread's srwcr_last_error()
// message (printf format) and return `code`; the device a plan was made on.
int report_error(int code, const char *fmt, ...);
int plan_device(const ::srwcr_plan *plan);
size_t prep_lds_bytes(const Geom &g);
size_t value_lds_bytes(const Geom &g, int bw);
size_t grad_lds_bytes(const Geom &g, int gnx, int gny, int gnz);
// Floats of per-wave LDS scratch of the gradient pass, for rows whose FFD
// x-range covers at most np_max cells: the row's bin list (64), its row
// tables (kRowBins entries) or, later in the row, q per voxel ([128][3]), and
// the cell moments ([np_max + 6][4][3], three zero cells on either side).
inline int grad_scratch_floats(int np_max)
{
    const int tables = kRowBins * kRowEntry, q = 3 * kSlots * kWave;
    return (64 + (tables > q ? tables : q) + 12 * (np_max + 6) + 3) / 4 * 4;
}

}  // namespace srwcr
