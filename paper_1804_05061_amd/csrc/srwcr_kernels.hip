// srwcr_kernels.hip -- gfx950 kernels for the SRWCR value and gradient
// (Gong et al., arXiv 1804.05061) and for RaPTOR, the patch-based metric it
// reduces to (eqs 6, 13, 14).
//
// Work decomposition.  The fixed grid is cut into boxes that each lie in one
// spatial-bin cell along y and z and at most two along x, so every voxel of a
// box draws its 64 regions (eq 7) from one 5x4x4 block.  Waves take rows of up
// to 128 voxels (two per lane); along a row the y and z weights of the regions
// and of the FFD are wave-uniform, which makes both B-spline sums separable.
//
// Warp pass (eqs 8, 17, Sec. II-F).  Per row: FFD displacement from
// contracted coefficients in LDS (or a dense field), FP64 trilinear sample of
// the moving image, its bin k and in-bin position t and, for gradient calls,
// dM/dy, stored per voxel for the passes that follow.
//
// Value pass (eqs 3, 5, 7).  The joint PDF is never formed: summed over b,
// eq (3) only needs per (region, A-bin) the moments P = sum w h(a - A),
// S1 = sum w h(a - A) m1(B), S2 = sum w h(a - A) m2(B).  One persistent
// workgroup per compute unit walks a share of the rows; a wave folds its
// voxels into windows of four A-bins x 5 x-nodes x 3 moments (a row's last
// one or two bins into a half window), sums them across lanes with a
// register transpose (v_permlane32/16_swap and DPP) and spreads each total
// over the 16 (y, z) regions with FP64 LDS atomics.  When the workgroup
// leaves a region block its histogram goes to staging slots of its own,
// which k_merge sums per region in a fixed order (or, when the slots would
// be too large, into the global moments with FP64 atomics).
//
// Finalisation (eqs 4, 9-12, 18-21) runs in FP64, one wave per region (wave 0
// of the region's merge workgroup, or k_finalize after an atomic merge), and
// writes the per-region terms and gradient tables (FP32, scaled by
// 1/(Z sigma_r^2)); k_value_sum then adds the terms into D in a fixed order.
//
// Gradient pass (eqs 16-21).  Stages the block's region tables in LDS with
// the 16 (y, z) regions of one (x-node, bin, coefficient) contiguous,
// interpolates them through the same separable weights (row tables per
// wave), forms q = dD/ds * grad M * dy/dT per voxel and scatters it to the
// FFD nodes.  The scatter is contracted over z first: a wave takes
// consecutive rows of one y (boxes end on FFD z-cell boundaries) and sums
// beta_c(z) q per voxel in registers; once per such group it forms, per
// z-node, the per-cell moments along x and adds them to the four y-nodes
// with FP64 LDS atomics; the box's node block is merged globally once.  A
// dense field's gradient is q itself.
#include "srwcr.h"
#include "srwcr_internal.h"

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

namespace srwcr {

// ------------------------------------------------------------ small helpers
template <int DT>
__device__ __forceinline__ float ld_int(const void *p, size_t i)
{
    if constexpr (DT == 0) {
        return reinterpret_cast<const float *>(p)[i];
    } else if constexpr (DT == 1) {
        return __half2float(reinterpret_cast<const __half *>(p)[i]);
    } else {
        unsigned short b = reinterpret_cast<const unsigned short *>(p)[i];
        return __uint_as_float(((unsigned)b) << 16);
    }
}

// Bounds checks of the debug build (SRWCR_CHECK): a computed index outside
// its array sets bit `bit` of g_check_flags (read by srwcr_debug_check_flags)
// and the access is skipped; in the normal build the checks compile away.
#ifdef SRWCR_CHECK
__device__ unsigned g_check_flags;
__device__ __forceinline__ bool check_ok(bool c, int bit)
{
    if (!c) atomicOr(&g_check_flags, 1u << bit);
    return c;
}
#else
__device__ __forceinline__ constexpr bool check_ok(bool, int) { return true; }
#endif
enum CheckBit {
    kChkPrepVoxel = 0,     // warp pass: voxel index < nvox
    kChkHistJK = 1,        // value pass: (y, z) region offset inside the block
    kChkMoments = 2,       // moment slot < R nb 3
    kChkTabJK = 3,         // gradient pass: table (y, z) slot < JKS
    kChkScratch = 4,       // gradient pass: per-wave scratch of the row range fits
    kChkNodeBlock = 5,     // gradient pass: node block index < nG
    kChkGrad = 6,          // gradient accumulator < 3 n_c
    kChkGradVoxel = 7,     // gradient pass: voxel index < nvox
    kChkColVoxel = 8,      // column value pass: voxel index < nvox
};

// Read of a per-axis table through a global-address-space pointer.  The
// tables are reached through generic pointers held in Geom, which the
// compiler would load with FLAT instructions; waiting for a FLAT load also
// waits for every pending LDS operation of the wave (FLAT may address LDS),
// so each row would stall until the previous row's LDS atomics drained.
template <typename T>
__device__ __forceinline__ T gld(const T *p, size_t i)
{
    return ((const __attribute__((address_space(1))) T *)p)[i];
}
__device__ __forceinline__ float4 gld(const float4 *p, size_t i)
{
    const __attribute__((address_space(1))) float *q = (const __attribute__((address_space(1))) float *)p + 4 * i;
    return make_float4(q[0], q[1], q[2], q[3]);
}
__device__ __forceinline__ double4 gld(const double4 *p, size_t i)
{
    const __attribute__((address_space(1))) double *q = (const __attribute__((address_space(1))) double *)p + 4 * i;
    return make_double4(q[0], q[1], q[2], q[3]);
}

// Per-row values that are the same for the whole wave, fetched with vector
// loads by a few lanes and broadcast with readlane.  As scalar loads they
// would share the LDS wait counter, and waiting for them would also wait for
// the wave's pending LDS atomics.
__device__ __forceinline__ float bcast(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
__device__ __forceinline__ int bcast(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

// The 4 + 4 spatial weights of rows y and z (eq 8).  Table pointers are
// passed in (hoisted out of the row loops, where the compiler would reload
// them from Geom with scalar loads).
__device__ __forceinline__ void row_sp_weights(const float4 *spw_y, const float4 *spw_z, int y, int z, int lane,
                                               float (&wy)[4], float (&wz)[4])
{
    const float *ty = reinterpret_cast<const float *>(spw_y), *tz = reinterpret_cast<const float *>(spw_z);
    float v = 0.0f;
    if (lane < 4) v = gld(ty, 4 * (size_t)y + lane);
    else if (lane < 8) v = gld(tz, 4 * (size_t)z + lane - 4);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        wy[j] = bcast(v, j);
        wz[j] = bcast(v, 4 + j);
    }
}

// FFD cells and weights of rows y and z (eq 17), the weights rounded to FP32.
__device__ __forceinline__ void row_ffd_weights(const double4 *fw_y, const double4 *fw_z, const int *fp_y,
                                                const int *fp_z, int y, int z, int lane, int &py, int &pz,
                                                float (&by)[4], float (&bz)[4])
{
    const double *ty = reinterpret_cast<const double *>(fw_y), *tz = reinterpret_cast<const double *>(fw_z);
    float v = 0.0f;
    int c = 0;
    if (lane < 4) v = (float)gld(ty, 4 * (size_t)y + lane);
    else if (lane < 8) v = (float)gld(tz, 4 * (size_t)z + lane - 4);
    else if (lane == 8) c = gld(fp_y, y);
    else if (lane == 9) c = gld(fp_z, z);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        by[j] = bcast(v, j);
        bz[j] = bcast(v, 4 + j);
    }
    py = bcast(c, 8);
    pz = bcast(c, 9);
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ int wave_min_i(int v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = min(v, __shfl_xor(v, d));
    return v;
}

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// Pairwise exchange-and-add steps of the 64 x 64 register transpose.
__device__ __forceinline__ float xadd_swap32(float a, float b)
{
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float xadd_swap16(float a, float b)
{
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
// lanes whose bit is clear keep `a`, the others `b`; each adds its xor-partner's copy
__device__ __forceinline__ float xadd_x8(float a, float b, bool hi)
{
    float keep = hi ? b : a, send = hi ? a : b;
    return keep + dpp<0x128>(send);                 // row_ror:8 == lane ^ 8
}
__device__ __forceinline__ float xadd_x4(float a, float b, bool hi)
{
    float keep = hi ? b : a, send = hi ? a : b;
    return keep + dpp<0x1B>(dpp<0x141>(send));      // half-mirror (^7) then quad reverse (^3)
}
__device__ __forceinline__ float xadd_x2(float a, float b, bool hi)
{
    float keep = hi ? b : a, send = hi ? a : b;
    return keep + dpp<0x4E>(send);                  // quad_perm [2,3,0,1]
}
__device__ __forceinline__ float xadd_x1(float a, float b, bool hi)
{
    float keep = hi ? b : a, send = hi ? a : b;
    return keep + dpp<0xB1>(send);                  // quad_perm [1,0,3,2]
}

// Lane l returns sum over all 64 lanes of v[l].  Must run with all lanes active.
__device__ __forceinline__ float wave_transpose_sum(const float (&v)[64], int lane)
{
    float w32[32], w16[16], w8[8], w4[4], w2[2];
#pragma unroll
    for (int i = 0; i < 32; ++i) w32[i] = xadd_swap32(v[i], v[i + 32]);
#pragma unroll
    for (int i = 0; i < 16; ++i) w16[i] = xadd_swap16(w32[i], w32[i + 16]);
    const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
#pragma unroll
    for (int i = 0; i < 8; ++i) w8[i] = xadd_x8(w16[i], w16[i + 8], b3);
#pragma unroll
    for (int i = 0; i < 4; ++i) w4[i] = xadd_x4(w8[i], w8[i + 4], b2);
#pragma unroll
    for (int i = 0; i < 2; ++i) w2[i] = xadd_x2(w4[i], w4[i + 2], b1);
    return xadd_x1(w2[0], w2[1], b0);
}

// Second-order Parzen window (eq 5) in two-tap form: s = k + t, t in [0, 1],
// h(t) on bin k and h(1 - t) = 1 - h(t) on bin k + 1.
__device__ __forceinline__ void parzen(float s, int L, int &k, float &t, float &w0, float &w1)
{
    int kk = (int)s;                         // s >= 0
    if (kk > L - 1) kk = L - 1;
    float tt = s - (float)kk;
    float w = (tt < 0.5f) ? 1.0f - tt * (0.1f + 1.8f * tt) : 1.9f - tt * (3.7f - 1.8f * tt);
    w = fminf(fmaxf(w, 0.0f), 1.0f);
    k = kk;
    t = tt;
    w0 = w;
    w1 = 1.0f - w;
}
// d h(t) / ds for the lower tap; the upper tap has the opposite sign
__device__ __forceinline__ float parzen_dw0(float t) { return (t < 0.5f) ? -0.1f - 3.6f * t : -3.7f + 3.6f * t; }

// FFD displacement of the 64 voxels of a row segment (eqs 8, 17), in FP64.
// The wave first contracts the y and z B-spline weights into per-x-node
// coefficients c1[e][n] (one node per lane), then each lane applies its four
// x weights.  The warp runs in FP64 (full rate on CDNA, like non-packed FP32)
// so that the bin of a warped sample is decided as the FP64 definition does.
__device__ __forceinline__ void ffd_row(const Geom &g, const float *__restrict__ ffd, int xs, int xe, int y, int z,
                                        int xc, double *c1, int lane, double u[3])
{
    const int py = gld(g.ffd_p[1], y), pz = gld(g.ffd_p[2], z);
    const double4 by = gld(g.ffd_w[1], y), bz = gld(g.ffd_w[2], z);
    const int px_lo = gld(g.ffd_p[0], xs), px_hi = gld(g.ffd_p[0], xe - 1);
    const int nn = px_hi - px_lo + 4;
    const size_t ncell = (size_t)g.nc[0] * g.nc[1] * g.nc[2];
    const double wy[4] = {by.x, by.y, by.z, by.w}, wz[4] = {bz.x, bz.y, bz.z, bz.w};
    for (int t = lane; t < 3 * nn; t += kWave) {
        const int e = t / nn, n = t - e * nn;
        const float *dp = ffd + e * ncell + ((size_t)pz * g.nc[1] + py) * g.nc[0] + px_lo + n;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double r = 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b) r = fma(wy[b], (double)dp[((size_t)c * g.nc[1] + b) * g.nc[0]], r);
            acc = fma(wz[c], r, acc);
        }
        c1[e * kMaxNodeSeg + n] = acc;
    }
    wave_sync();
    const int px = gld(g.ffd_p[0], xc) - px_lo;
    const double4 bx = gld(g.ffd_w[0], xc);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const double *c = c1 + e * kMaxNodeSeg + px;
        u[e] = fma(bx.x, c[0], fma(bx.y, c[1], fma(bx.z, c[2], bx.w * c[3])));
    }
    wave_sync();
}

// Per-row FFD coefficients c1[e][n] = sum_{m,n'} beta_m(eta_y) beta_n'(eta_z)
// d_e[pz + n'][py + m][px_lo + n] for the x-nodes of an item row [xs, xe)
// (one node-component per lane, FP64, 32-bit element offsets).
__device__ __forceinline__ int ffd_c1(const Geom &g, const float *__restrict__ ffd, int xs, int xe, int y, int z,
                                      double *c1, int lane)
{
    const int py = gld(g.ffd_p[1], y), pz = gld(g.ffd_p[2], z);
    const double4 by = gld(g.ffd_w[1], y), bz = gld(g.ffd_w[2], z);
    const int px_lo = gld(g.ffd_p[0], xs), px_hi = gld(g.ffd_p[0], xe - 1);
    const int nn = px_hi - px_lo + 4;
    const unsigned sy = (unsigned)g.nc[0], sz = (unsigned)g.nc[0] * g.nc[1], ncell = sz * g.nc[2];
    const double wy[4] = {by.x, by.y, by.z, by.w}, wz[4] = {bz.x, bz.y, bz.z, bz.w};
    for (int t = lane; t < 3 * nn; t += kWave) {
        const int e = t / nn, n = t - e * nn;
        const unsigned off = e * ncell + pz * sz + py * sy + (unsigned)(px_lo + n);
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double r = 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b) r = fma(wy[b], (double)ffd[off + c * sz + b * sy], r);
            acc = fma(wz[c], r, acc);
        }
        c1[e * g.c1n + n] = acc;
    }
    return px_lo;
}

// Displacement of voxel xc from the row coefficients (four x weights).
__device__ __forceinline__ void ffd_u(const Geom &g, const double *c1, int px_lo, int xc, double u[3])
{
    const int px = gld(g.ffd_p[0], xc) - px_lo;
    const double4 bx = gld(g.ffd_w[0], xc);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const double *c = c1 + e * g.c1n + px;
        u[e] = fma(bx.x, c[0], fma(bx.y, c[1], fma(bx.z, c[2], bx.w * c[3])));
    }
}

// Displacement of fixed voxel (x, y, z) from a dense field u[3][nz][ny][nx]
// (T(x) = x + u(x)), widened to FP64 like the FFD path.
__device__ __forceinline__ void dense_u(const Geom &g, const float *__restrict__ field, int x, int y, int z, double u[3])
{
    const size_t nv = (size_t)g.nf[0] * g.nf[1] * g.nf[2];
    const size_t vi = ((size_t)z * g.nf[1] + y) * g.nf[0] + x;
#pragma unroll
    for (int e = 0; e < 3; ++e) u[e] = (double)field[e * nv + vi];
}

// Backward warping: trilinear sample of the moving volume at T(x) mapped to
// the moving grid, coordinates clamped to [0, M - 1]; grad (if non-null) gets
// dM/dy, zero along clamped axes.  y = base + frac + u * ratio keeps the
// integer part exact.  FP64 arithmetic on the stored intensities.
template <int MDT>
__device__ __forceinline__ double sample_moving(const Geom &g, const void *__restrict__ mov, int x, int y, int z,
                                                const double u[3], double *grad)
{
    const int coord[3] = {x, y, z};
    int i0[3];
    double f[3];
    bool cl[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int M = g.nm[e];
        int b;
        double t;
        if (g.same_grid[e]) {
            b = coord[e];
            t = u[e];
        } else {
            b = gld(g.mv_base[e], coord[e]);
            t = fma(u[e], g.ratio_d[e], gld(g.mv_frac[e], coord[e]));
        }
        const double ft = floor(t);
        int i = b + (int)ft;
        double fr = t - ft;
        bool c = false;
        if (i < 0) { i = 0; fr = 0.0; c = true; }
        else if (i > M - 1 || (i == M - 1 && fr > 0.0)) { i = M - 1; fr = 0.0; c = true; }
        if (i == M - 1) { i = M - 2; fr = 1.0; }
        i0[e] = i;
        f[e] = fr;
        cl[e] = c;
    }
    const size_t sx = 1, sy = (size_t)g.nm[0], sz = (size_t)g.nm[0] * g.nm[1];
    const size_t base = i0[2] * sz + i0[1] * sy + i0[0];
    const double v000 = ld_int<MDT>(mov, base), v100 = ld_int<MDT>(mov, base + sx);
    const double v010 = ld_int<MDT>(mov, base + sy), v110 = ld_int<MDT>(mov, base + sy + sx);
    const double v001 = ld_int<MDT>(mov, base + sz), v101 = ld_int<MDT>(mov, base + sz + sx);
    const double v011 = ld_int<MDT>(mov, base + sz + sy), v111 = ld_int<MDT>(mov, base + sz + sy + sx);
    // lerp(a, b, f) = a - f a + f b: exact at f = 0 and at f = 1 (the last grid plane)
    auto lerp = [](double a, double b, double t) { return fma(t, b, fma(-t, a, a)); };
    const double a00 = lerp(v000, v100, f[0]), a10 = lerp(v010, v110, f[0]);
    const double a01 = lerp(v001, v101, f[0]), a11 = lerp(v011, v111, f[0]);
    const double b0 = lerp(a00, a10, f[1]), b1 = lerp(a01, a11, f[1]);
    const double val = lerp(b0, b1, f[2]);
    if (grad) {
        const double d00 = v100 - v000, d10 = v110 - v010, d01 = v101 - v001, d11 = v111 - v011;
        const double dy0 = fma(f[1], d10 - d00, d00), dy1 = fma(f[1], d11 - d01, d01);
        grad[0] = cl[0] ? 0.0 : fma(f[2], dy1 - dy0, dy0);
        const double e0 = a10 - a00, e1 = a11 - a01;
        grad[1] = cl[1] ? 0.0 : fma(f[2], e1 - e0, e0);
        grad[2] = cl[2] ? 0.0 : b1 - b0;
    }
    return val;
}

// Tap weights h(t), 1 - h(t) of an in-bin position t (eq 5), in FP32.
__device__ __forceinline__ void parzen_w(float t, float &w0, float &w1)
{
    float w = (t < 0.5f) ? 1.0f - t * (0.1f + 1.8f * t) : 1.9f - t * (3.7f - 1.8f * t);
    w = fminf(fmaxf(w, 0.0f), 1.0f);
    w0 = w;
    w1 = 1.0f - w;
}

// ------------------------------------------------------------------ zero
__global__ void k_zero(double *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

hipError_t launch_zero(double *p, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    int blocks = (int)std::min<size_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

// ---------------------------------------------------- a1: normalisation
template <int DT>
__global__ void k_normalize(const float *__restrict__ in, int64_t n, float lo, float scale, float L, void *out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        // two separately rounded single-precision operations (no contraction)
        float d = __fsub_rn(in[i], lo);
        float s = __fmul_rn(d, scale);
        s = fminf(fmaxf(s, 0.0f), L);
        if constexpr (DT == 0) {
            reinterpret_cast<float *>(out)[i] = s;
        } else if constexpr (DT == 1) {
            reinterpret_cast<__half *>(out)[i] = __float2half_rn(s);
        } else {
            // round to nearest even into bfloat16 (s is finite and non-negative)
            unsigned b = __float_as_uint(s);
            b += 0x7fffu + ((b >> 16) & 1u);
            reinterpret_cast<unsigned short *>(out)[i] = (unsigned short)(b >> 16);
        }
    }
}

hipError_t launch_normalize(const float *in, int64_t n, float lo, float scale, float L, void *out, int dt,
                            hipStream_t s)
{
    int blocks = (int)std::min<int64_t>((n + 255) / 256, 8192);
    if (blocks < 1) blocks = 1;
    if (dt == 0) hipLaunchKernelGGL(k_normalize<0>, dim3(blocks), dim3(256), 0, s, in, n, lo, scale, L, out);
    else if (dt == 1) hipLaunchKernelGGL(k_normalize<1>, dim3(blocks), dim3(256), 0, s, in, n, lo, scale, L, out);
    else hipLaunchKernelGGL(k_normalize<2>, dim3(blocks), dim3(256), 0, s, in, n, lo, scale, L, out);
    return hipGetLastError();
}

// ------------------------------------------------------------- min / max
// partial[3 * b + 0..2] = (min, max, count of non-finite values) of block b
__global__ void k_minmax(const float *__restrict__ in, int64_t n, float *partial)
{
    __shared__ float smin[256], smax[256], sbad[256];
    float mn = INFINITY, mx = -INFINITY, bad = 0.0f;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float v = in[i];
        if (!isfinite(v)) { bad += 1.0f; continue; }
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
    }
    smin[threadIdx.x] = mn;
    smax[threadIdx.x] = mx;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int d = 128; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
            smin[threadIdx.x] = fminf(smin[threadIdx.x], smin[threadIdx.x + d]);
            smax[threadIdx.x] = fmaxf(smax[threadIdx.x], smax[threadIdx.x + d]);
            sbad[threadIdx.x] += sbad[threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x + 0] = smin[0];
        partial[3 * blockIdx.x + 1] = smax[0];
        partial[3 * blockIdx.x + 2] = sbad[0];
    }
}

hipError_t launch_minmax(const float *in, int64_t n, float *partial, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(k_minmax, dim3(nblocks), dim3(256), 0, s, in, n, partial);
    return hipGetLastError();
}

// ------------------------------------------------------------- warp pass
// The warp T (FFD of eq 17, or x + u(x) for a dense field) and the trilinear
// sample of the moving image, once per call, in FP64: per fixed voxel the
// moving bin k = min(floor(s), L - 1) decided in FP64 and the in-bin position
// t = s - k rounded to FP32, plus dM/dy (FP32) when a gradient follows.  The
// value and gradient passes read these (coalesced) instead of repeating the
// dependent FFD loads and gathers.  One wave per item row, as in those passes.
size_t prep_lds_bytes(const Geom &g) { return (size_t)(kValueThreads / kWave) * 3 * g.c1n * sizeof(double); }

// Rows come from the value pass's block-ordered row list: wave w of
// workgroup b takes row 12 b + w, so the grid is balanced to the row.
template <int MDT, int DISP, int GRAD>
__global__ void __launch_bounds__(kValueThreads)
k_prep(const Geom *__restrict__ geoms, const WorkItem *__restrict__ blocks, const int *__restrict__ row_start,
       int nblocks, BatchArgs args, unsigned char *ws, double *__restrict__ zero, long nzero)
{
    extern __shared__ __align__(16) unsigned char smem[];
    // clear `zero` (accumulators of a later pass) on the side, saving a launch
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nzero; i += (long)gridDim.x * blockDim.x)
        zero[i] = 0.0;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // workgroups are dealt to the 8 XCDs in turn; give each XCD a contiguous
    // run of rows, so that the moving-image rows that neighbouring output rows
    // share are fetched into one L2 (the grid is a multiple of kXcds)
    const long per = gridDim.x / kXcds;
    const long wg = (long)(blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
    const long r = wg * (kValueThreads / kWave) + wave;
    if (r >= row_start[nblocks]) return;
    int lo = 0, hi = nblocks - 1;                       // block of row r: row_start[lo] <= r < row_start[lo + 1]
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_start[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    const WorkItem it = blocks[lo];
    const Geom &g = geoms[it.prob];
    const void *__restrict__ moving = args.p[it.prob].moving;
    const float *__restrict__ ffd = args.p[it.prob].ffd;
    PrepKT *__restrict__ kt = reinterpret_cast<PrepKT *>(ws + g.ws.kt);
    float *__restrict__ dmo = reinterpret_cast<float *>(ws + g.ws.dm);
    const int L = g.nb - 1;
    const int lane = threadIdx.x & (kWave - 1);
    double *c1 = reinterpret_cast<double *>(smem) + wave * 3 * g.c1n;
    const size_t nv = (size_t)g.nf[0] * g.nf[1] * g.nf[2];
    const int ny = it.y1 - it.y0;
    const int xs = it.x0, xe = it.x1;
    {
        const int row = (int)(r - row_start[lo]);
        const int y = it.y0 + row % ny, z = it.z0 + row / ny;
        int px_lo = 0;
        if (DISP == 0) px_lo = ffd_c1(g, ffd, xs, xe, y, z, c1, lane);
        wave_sync();
        const size_t rowb = ((size_t)z * g.nf[1] + y) * g.nf[0];
#pragma unroll
        for (int sl = 0; sl < kSlots; ++sl) {
            const int x = xs + sl * kWave + lane;
            if (x < xe && check_ok(rowb + x < nv, kChkPrepVoxel)) {
                double u[3], dm[3];
                if (DISP == 0) ffd_u(g, c1, px_lo, x, u);
                else dense_u(g, ffd, x, y, z, u);
                double sm = sample_moving<MDT>(g, moving, x, y, z, u, GRAD ? dm : nullptr);
                sm = fmin(fmax(sm, 0.0), (double)L);
                int kk = (int)sm;                        // sm >= 0
                if (kk > L - 1) kk = L - 1;
                kt[rowb + x] = PrepKT{(float)(sm - (double)kk), kk};
                if (GRAD) {
#pragma unroll
                    for (int e = 0; e < 3; ++e) dmo[e * nv + rowb + x] = (float)dm[e];
                }
            }
        }
    }
}

#define SRWCR_PREP(M, D, G)                                                                                   \
    hipLaunchKernelGGL((k_prep<M, D, G>), dim3(nwg), dim3(kValueThreads), lds_bytes, s, geoms, blocks, row_start, \
                       nblocks, args, ws, zero, nzero)

hipError_t launch_prep(const Geom *geoms, int mdt, int dense, int with_grad, const WorkItem *blocks,
                       const int *row_start, int nblocks, long nrows, const BatchArgs &args, unsigned char *ws,
                       size_t lds_bytes, hipStream_t s, double *zero, long nzero)
{
    if (nblocks <= 0 || nrows <= 0) return nzero > 0 ? launch_zero(zero, (size_t)nzero, s) : hipSuccess;
    int nwg = (int)((nrows + kValueThreads / kWave - 1) / (kValueThreads / kWave));
    nwg = (nwg + kXcds - 1) / kXcds * kXcds;
#define SRWCR_PREP_M(M)                                                                                      \
    if (mdt == M) {                                                                                          \
        if (dense) { if (with_grad) SRWCR_PREP(M, 1, 1); else SRWCR_PREP(M, 1, 0); }                         \
        else { if (with_grad) SRWCR_PREP(M, 0, 1); else SRWCR_PREP(M, 0, 0); }                               \
    }
    SRWCR_PREP_M(0) SRWCR_PREP_M(1) SRWCR_PREP_M(2)
#undef SRWCR_PREP_M
    return hipGetLastError();
}

// ------------------------------------------------------------ value pass
// Block histogram layout: H[((a * 3 + m) * 5 + i) * HS + jk] holds moment m of
// A-bin a in region (i, j, k) of the block's 5 x BW x BW regions, jk = BW k + j.
// BW = 4: the block lies in one spatial cell along y and z; BW = 5: in two
// (small cells, see the plan).  The (y, z) regions of one (a, m, i) are
// adjacent, so a lane's 16 atomics share one address with immediate offsets;
// the pad of one double (HS = BW^2 + 1) spreads the 60 lanes of a window
// (consecutive (a, m, i)) over the banks, so that with BW = 4 an atomic
// touches each bank at most twice.
template <int BW>
struct Hist {
    static constexpr int kJK = BW * BW;          // (y, z) regions of the block
    static constexpr int kHS = BW * BW + 1;      // doubles per (a, m, i)
    static constexpr int kReg = kXN * BW * BW;   // regions of the block
};

// The histogram, then a row counter (16 B).
size_t value_lds_bytes(const Geom &g, int bw)
{
    return (size_t)g.nb * 3 * kXN * (bw * bw + 1) * sizeof(double) + 16;
}

// Wave-uniform minimum: butterfly inside each 16-lane row (DPP), then the
// four row results through scalar reads.
__device__ __forceinline__ int wave_min_dpp(int v)
{
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xf, 0xf, false));   // quad_perm [1,0,3,2]
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xf, 0xf, false));   // quad_perm [2,3,0,1]
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x124, 0xf, 0xf, false));  // row_ror:4
    v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x128, 0xf, 0xf, false));  // row_ror:8
    const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    return min(min(r0, r1), min(r2, r3));
}

__device__ __forceinline__ unsigned long long wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Wave-uniform bitwise OR, with the same DPP steps as wave_min_dpp.
__device__ __forceinline__ unsigned wave_or_dpp(unsigned v)
{
    v |= (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0xB1, 0xf, 0xf, false);
    v |= (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x4E, 0xf, 0xf, false);
    v |= (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x124, 0xf, 0xf, false);
    v |= (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x128, 0xf, 0xf, false);
    const unsigned r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const unsigned r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    return (r0 | r1) | (r2 | r3);
}

// A voxel's four x weights on its block's five x-nodes: its cell is the
// block's first x-cell (o1 false) or the second (rows span at most two).
__device__ __forceinline__ void x_node_weights(const float4 &w, bool o1, float (&wn)[kXN])
{
    wn[0] = o1 ? 0.0f : w.x;
    wn[1] = o1 ? w.x : w.y;
    wn[2] = o1 ? w.y : w.z;
    wn[3] = o1 ? w.z : w.w;
    wn[4] = o1 ? w.w : 0.0f;
}

// Per-voxel quantities of the value pass.
struct VoxA {
    int k;          // A-bin (lower tap)
    float a0, a1;   // Parzen weights of bins k and k + 1
    float wxv[15];  // x-node weight (5 nodes) times (1, m1(B), m2(B))
};

// One bin window of the value pass: four A-bins b[0..3] (any four of the bins
// the row's taps touch, ascending; unused slots hold a bin above L).  Each of
// the lane's two voxels puts weight a0 on the slot of bin k and a1 on the
// slot of bin k + 1 when those bins are in the window; the wave sums 4 slots
// x 15 (x-node, moment) values across lanes and each lane spreads one total
// over the 16 (y, z) regions of its column with FP64 LDS atomics.  A voxel
// outside the row has k < -1 and matches no slot.
template <int BW>
__device__ __forceinline__ void value_window(double *H, int L, const int (&b)[kWin], const VoxA (&v)[kSlots],
                                             const float (&wyz)[16], int oyz, int lane)
{
    float t[kSlots][kWin];
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl)
#pragma unroll
        for (int w = 0; w < kWin; ++w)
            t[sl][w] = (v[sl].k == b[w]) ? v[sl].a0 : ((v[sl].k + 1 == b[w]) ? v[sl].a1 : 0.0f);
    float V[64];
#pragma unroll
    for (int w = 0; w < kWin; ++w)
#pragma unroll
        for (int q = 0; q < 15; ++q) V[w * 15 + q] = fmaf(t[1][w], v[1].wxv[q], t[0][w] * v[0].wxv[q]);
#pragma unroll
    for (int q = kWin * 15; q < 64; ++q) V[q] = 0.0f;
    const float T = wave_transpose_sum(V, lane);
    if (lane < kWin * 15 && T != 0.0f) {
        const int w = lane / 15, q = lane - 15 * w, i = q / 3, m = q - 3 * i;
        const int a = w == 0 ? b[0] : (w == 1 ? b[1] : (w == 2 ? b[2] : b[3]));
        if (a <= L && check_ok(oyz + 3 * BW + 3 < BW * BW, kChkHistJK)) {
            double *h = H + ((a * 3 + m) * kXN + i) * Hist<BW>::kHS + oyz;
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int j = 0; j < 4; ++j) atomicAdd(h + k * BW + j, (double)(T * wyz[k * 4 + j]));
        }
    }
}

// The last window of a row when it holds at most two bins b0 < b1 (b1 above
// L when unused): 30 sums instead of 60, so the transpose runs one stage
// short -- the total of value i ends in lanes 2i and 2i + 1 -- and the two
// lanes split the 16 (y, z) atomics, z-nodes 0-1 and 2-3.  The odd lane's
// weights are picked by multiplying with 0 or 1 (exact for finite weights):
// a select would become an indexed load and move wyz to scratch memory.
template <int BW>
__device__ __forceinline__ void value_window2(double *H, int L, int b0, int b1, const VoxA (&v)[kSlots],
                                              const float (&wyz)[16], int oyz, int lane)
{
    float t[kSlots][2];
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
        t[sl][0] = (v[sl].k == b0) ? v[sl].a0 : ((v[sl].k + 1 == b0) ? v[sl].a1 : 0.0f);
        t[sl][1] = (v[sl].k == b1) ? v[sl].a0 : ((v[sl].k + 1 == b1) ? v[sl].a1 : 0.0f);
    }
    float V[32];
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
        for (int q = 0; q < 15; ++q) V[w * 15 + q] = fmaf(t[1][w], v[1].wxv[q], t[0][w] * v[0].wxv[q]);
    V[30] = 0.0f;
    V[31] = 0.0f;
    float w16[16], w8[8], w4[4], w2[2];
#pragma unroll
    for (int i = 0; i < 16; ++i) w16[i] = xadd_swap32(V[i], V[i + 16]);
#pragma unroll
    for (int i = 0; i < 8; ++i) w8[i] = xadd_swap16(w16[i], w16[i + 8]);
    const bool b3 = lane & 8, b2 = lane & 4, b1l = lane & 2;
#pragma unroll
    for (int i = 0; i < 4; ++i) w4[i] = xadd_x8(w8[i], w8[i + 4], b3);
#pragma unroll
    for (int i = 0; i < 2; ++i) w2[i] = xadd_x4(w4[i], w4[i + 2], b2);
    float T = xadd_x2(w2[0], w2[1], b1l);
    T += dpp<0xB1>(T);                                   // lanes 2i and 2i + 1 hold the same partial sums
    const int idx = lane >> 1, odd = lane & 1;
    const float fo = (float)odd, fe = 1.0f - fo;
    if (idx < 30 && T != 0.0f) {
        const int w = idx / 15, q = idx - 15 * w, i = q / 3, m = q - 3 * i;
        const int a = w == 0 ? b0 : b1;
        if (a <= L && check_ok(oyz + 3 * BW + 3 < BW * BW, kChkHistJK)) {
            double *h = H + ((a * 3 + m) * kXN + i) * Hist<BW>::kHS + oyz + 2 * BW * odd;
#pragma unroll
            for (int kk = 0; kk < 2; ++kk)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float wv = fmaf(wyz[(kk + 2) * 4 + j], fo, wyz[kk * 4 + j] * fe);
                    atomicAdd(h + kk * BW + j, (double)(T * wv));
                }
        }
    }
}

// Value pass.  Schedule: one persistent workgroup per compute unit (the FP64
// histogram of a 5 x BW x BW region block fills most of its LDS).  The rows
// of all region blocks (an x-chunk of at most two spatial cells by one cell in
// y and z, or two for small cells) form one list ordered by block; workgroup w
// takes rows [w T / G, (w + 1) T / G) of the T rows, accumulates them in LDS
// and empties the histogram only when its range leaves a block: into staging
// slots of its own (merged by k_merge in a fixed order) or, without staging,
// into the global moments with FP64 atomics.  Inside the workgroup the rows of
// a block go to the waves one at a time from an LDS counter (long runs) or
// round-robin (short runs).  Reads the warp pass's per-voxel moving bins
// (k_prep) and the fixed image.
template <int FDT, int BW>
__global__ void __launch_bounds__(kValueThreads)
k_value(const Geom *__restrict__ geoms, const WorkItem *__restrict__ blocks, const int *__restrict__ row_start,
        int nblocks, int lds_doubles, BatchArgs args, unsigned char *ws, double *__restrict__ staging,
        const int *__restrict__ visit_start, long stage_stride)
{
    extern __shared__ __align__(16) unsigned char smem[];
    double *H = reinterpret_cast<double *>(smem);     // [nb][3][5][HS], see Hist
    constexpr int HS = Hist<BW>::kHS, JK = Hist<BW>::kJK, NREG = Hist<BW>::kReg;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwaves = blockDim.x >> 6;
    const long total = row_start[nblocks];
    long r0 = (long)blockIdx.x * total / gridDim.x;
    const long r1 = (long)(blockIdx.x + 1) * total / gridDim.x;
    int bi = 0;
    while (bi + 1 < nblocks && row_start[bi + 1] <= r0) ++bi;

    for (int i = threadIdx.x; i < lds_doubles; i += blockDim.x) H[i] = 0.0;
    __syncthreads();

    int visit = 0;                                       // blocks this workgroup has left so far
    while (r0 < r1) {
        const WorkItem it = blocks[bi];
        const long bstart = row_start[bi];
        const long bend = min(r1, (long)row_start[bi + 1]);
        const Geom &g = geoms[it.prob];
        const void *__restrict__ fixed = args.p[it.prob].fixed;
        const PrepKT *__restrict__ kt = reinterpret_cast<const PrepKT *>(ws + g.ws.kt);
        double *__restrict__ moments = reinterpret_cast<double *>(ws + g.ws.moments);
        const float4 *spw_x = g.sp_w[0], *spw_y = g.sp_w[1], *spw_z = g.sp_w[2];
        const int *spc_x = g.sp_cell[0];
        const int role = g.role, nfx = g.nf[0], nfy = g.nf[1];
        const int nb = g.nb, L = nb - 1;
        const int nH = nb * 3 * kXN * HS;
        const int ny = it.y1 - it.y0;
        const int xs = it.x0, xe = it.x1;                // xe - xs <= 64 kSlots
        // A long run of rows is handed out one row at a time from an LDS
        // counter, so that waves whose rows hold fewer bins take more of them;
        // a short one (small spatial cells) is dealt round-robin, which saves
        // the barrier.
        const bool dyn = bend - r0 >= 4 * nwaves;
        unsigned &next_row = *reinterpret_cast<unsigned *>(H + nH);
        if (dyn) {
            if (threadIdx.x == 0) next_row = 0u;
            __syncthreads();
        }
        long rs = r0 + wave;
        for (;;) {
            long r;
            if (dyn) {
                unsigned rr = 0u;
                if (lane == 0) rr = atomicAdd(&next_row, 1u);
                r = r0 + (long)__builtin_amdgcn_readfirstlane(rr);
            } else {
                r = rs;
                rs += nwaves;
            }
            if (r >= bend) break;
            const int row = (int)(r - bstart);
            const int y = it.y0 + row % ny, z = it.z0 + row / ny;
            const size_t rowb = ((size_t)z * nfy + y) * nfx;
            VoxA v[kSlots];
            bool pend[kSlots];
#pragma unroll
            for (int sl = 0; sl < kSlots; ++sl) {
                const int x = xs + sl * kWave + lane;
                pend[sl] = x < xe;
                const int xc = pend[sl] ? x : xe - 1;
                const PrepKT pk = kt[rowb + xc];
                const float sf = ld_int<FDT>(fixed, rowb + xc);
                int kF;
                float tF, m0w, m1w, f0w, f1w;
                const int kM = pk.k;
                parzen_w(pk.t, m0w, m1w);
                parzen(sf, L, kF, tF, f0w, f1w);
                const int kB = role ? kM : kF;
                const float b1w = role ? m1w : f1w;
                v[sl].k = pend[sl] ? (role ? kF : kM) : -8;
                v[sl].a0 = role ? f0w : m0w;
                v[sl].a1 = role ? f1w : m1w;
                const float m1 = (float)kB + b1w;
                const float m2 = fmaf((float)(2 * kB + 1), b1w, (float)(kB * kB));
                // x weights on the item's 5 x-nodes (the voxel's cell is it.cx or it.cx + 1)
                float wn[kXN];
                x_node_weights(gld(spw_x, xc), gld(spc_x, xc) != it.cx, wn);
#pragma unroll
                for (int n = 0; n < kXN; ++n) {
                    v[sl].wxv[3 * n + 0] = wn[n];
                    v[sl].wxv[3 * n + 1] = wn[n] * m1;
                    v[sl].wxv[3 * n + 2] = wn[n] * m2;
                }
            }
            float wyv[4], wzv[4];
            row_sp_weights(spw_y, spw_z, y, z, lane, wyv, wzv);
            int oyz = 0;                                 // the row's (y, z) cells within a two-cell block
            if constexpr (BW == 5) {
                int c = 0;
                if (lane == 0) c = gld(g.sp_cell[1], y);
                else if (lane == 1) c = gld(g.sp_cell[2], z);
                oyz = (bcast(c, 1) - it.cz) * BW + (bcast(c, 0) - it.cy);
            }
            float wyz[16];
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int j = 0; j < 4; ++j) wyz[k * 4 + j] = wyv[j] * wzv[k];

            // the A-bins the row's taps touch (a wave-uniform 64-bit set), four per window
            unsigned long long mine = 0ull;
#pragma unroll
            for (int sl = 0; sl < kSlots; ++sl)
                if (pend[sl]) mine |= 3ull << v[sl].k;
            unsigned long long bins = (unsigned long long)wave_or_dpp((unsigned)(mine >> 32)) << 32 |
                                      wave_or_dpp((unsigned)mine);
            while (bins != 0ull) {
                if (__builtin_popcountll(bins) <= 2) {      // a last window of one or two bins
                    const int b0 = (int)__builtin_ctzll(bins);
                    bins &= bins - 1;
                    const int b1 = bins ? (int)__builtin_ctzll(bins) : 1 << 20;
                    value_window2<BW>(H, L, b0, b1, v, wyz, oyz, lane);
                    break;
                }
                int b[kWin];
#pragma unroll
                for (int w = 0; w < kWin; ++w) {
                    b[w] = bins ? (int)__builtin_ctzll(bins) : 1 << 20;
                    bins &= bins - 1;
                }
                value_window<BW>(H, L, b, v, wyz, oyz, lane);
            }
        }
        __syncthreads();
        if (staging) {
            // the histogram to this visit's staging slots, region-major ([5 BW^2 local
            // regions][nb][3]), in plain coalesced stores, clearing it for the next
            // block; k_merge adds up the visits of each region in a fixed order
            double *dst = staging + (size_t)(visit_start[blockIdx.x] + visit) * stage_stride;
            const int n = NREG * nb * 3, nb3 = nb * 3;
            for (int o = threadIdx.x; o < n; o += blockDim.x) {
                const int loc = o / nb3, rem = o - loc * nb3, a = rem / 3, m = rem - 3 * a;
                const int i = loc / JK, jk = loc - i * JK;
                const int e = ((a * 3 + m) * kXN + i) * HS + jk;
                dst[o] = H[e];
                H[e] = 0.0;
            }
        } else {
            // merge into the global moments, clearing the histogram for the next block
            for (int e = threadIdx.x; e < nH; e += blockDim.x) {
                const double val = H[e];
                const int idx = e / HS, jk = e - idx * HS;
                if (val != 0.0) {
                    H[e] = 0.0;
                    const int am = idx / kXN, i = idx - am * kXN, a = am / 3, m = am - 3 * a;
                    const int k = jk / BW, j = jk - k * BW;
                    if (jk < JK && it.cx + i < g.K[0] && it.cy + j < g.K[1] && it.cz + k < g.K[2]) {
                        const int R = ((it.cz + k) * g.K[1] + (it.cy + j)) * g.K[0] + (it.cx + i);
                        if (check_ok(R < g.R && a < nb, kChkMoments))
                            unsafeAtomicAdd(&moments[((size_t)R * nb + a) * 3 + m], val);
                    }
                }
            }
        }
        __syncthreads();
        r0 = bend;
        ++bi;
        ++visit;
    }
}

// Value pass by block columns.  A work unit is a range of columns (x, y) of
// one region block (an x-chunk of at most two spatial cells by BW = 4 (one
// cell) or BW = 5 (two cells) regions along y and z); one wave per unit.  A
// lane owns a column and sums over its z voxels, for a window of four A-bins,
// Acc[w][m][k] = sum_z h_w(A) m_m(B) wz_k(z) (eqs 3, 5, 7) in registers -- the
// z weights are wave-uniform.  What is left of the block's sums is a dense
// product over the columns,
//   H[(i, j)][(w, m, k)] += sum_col wx_i(x) wy_j(y) Acc_col[w][m][k],
// which runs on the matrix cores (v_mfma_f32_16x16x4f32, four columns per
// step) from the columns' weights and Acc staged in LDS 16 values at a time
// (the weights become matrix operands in registers); the unit's sums go to
// the global moments with FP64 atomics once per window.
constexpr int kColWaves = 4;                 // waves (units) per workgroup
constexpr int kColRow = 17;                  // LDS floats per column of a staged piece (16 used, odd stride)
constexpr int kColStage = 64 * kColRow;      // per wave: [column][kColRow]

size_t value_cols_lds_bytes() { return (size_t)kColWaves * kColStage * sizeof(float); }

// Rotated LDS slots: the writes (one column per lane) and the MFMA operand
// reads (16 consecutive entries of four columns) both touch 64 distinct banks.
__device__ __forceinline__ int col_acc_slot(int col, int n) { return col * 64 + ((n + 16 * (col & 3) + (col >> 2)) & 63); }
__device__ __forceinline__ int col_wxy_slot(int col, int m) { return col * 32 + ((m + 8 * (col & 3)) & 31); }

// One voxel of the value pass: its A-bin, the two Parzen tap weights and the
// moments m1, m2 of B (as in k_value).
template <int FDT>
__device__ __forceinline__ void value_voxel(const PrepKT *__restrict__ kt, const void *__restrict__ fixed, size_t v,
                                            int L, int role, int &kA, float &a0, float &a1, float &m1, float &m2)
{
    const PrepKT pk = kt[v];
    const float sf = ld_int<FDT>(fixed, v);
    int kF;
    float tF, m0w, m1w, f0w, f1w;
    const int kM = pk.k;
    parzen_w(pk.t, m0w, m1w);
    parzen(sf, L, kF, tF, f0w, f1w);
    const int kB = role ? kM : kF;
    const float b1w = role ? m1w : f1w;
    kA = role ? kF : kM;
    a0 = role ? f0w : m0w;
    a1 = role ? f1w : m1w;
    m1 = (float)kB + b1w;
    m2 = fmaf((float)(2 * kB + 1), b1w, (float)(kB * kB));
}

// A coordinate's spatial weights on the block's BW nodes along y or z: its
// four B-spline weights, shifted by one node when it lies in the block's
// second cell (BW = 5).
template <int BW>
__device__ __forceinline__ void block_node_weights(const float4 &w, bool o1, float (&wn)[BW])
{
    if constexpr (BW == 5) {
        x_node_weights(w, o1, wn);
    } else {
        wn[0] = w.x;
        wn[1] = w.y;
        wn[2] = w.z;
        wn[3] = w.w;
    }
}

template <int FDT, int BW>
__global__ void __launch_bounds__(kColWaves * kWave)
k_value_cols(const Geom *__restrict__ geoms, const WorkItem *__restrict__ blocks, const int4 *__restrict__ units,
             int nunits, BatchArgs args, unsigned char *ws)
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr int NIJ = kXN * BW;            // (x, y) nodes of a block: 20 or 25 (two 16-row tiles)
    constexpr int NN = kWin * 3 * BW;        // (w, m, k) sums of a window: 48 or 60
    constexpr int NT = (NN + 15) / 16;       // 16-column tiles of them
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ui = blockIdx.x * kColWaves + wave;
    if (ui >= nunits) return;
    float *stg = reinterpret_cast<float *>(smem) + wave * kColStage;  // [column][kColRow]
    const int4 un = units[ui];                                   // (block, first column, end column)
    const WorkItem it = blocks[un.x];
    const Geom &g = geoms[it.prob];
    const void *__restrict__ fixed = args.p[it.prob].fixed;
    const PrepKT *__restrict__ kt = reinterpret_cast<const PrepKT *>(ws + g.ws.kt);
    double *__restrict__ moments = reinterpret_cast<double *>(ws + g.ws.moments);
    const float4 *spw_x = g.sp_w[0], *spw_y = g.sp_w[1], *spw_z = g.sp_w[2];
    const int *spc_x = g.sp_cell[0], *spc_y = g.sp_cell[1], *spc_z = g.sp_cell[2];
    const int nb = g.nb, L = nb - 1, role = g.role;
    const int nfx = g.nf[0], nfy = g.nf[1];
    const size_t nvox = (size_t)nfx * nfy * g.nf[2];
    const int nx = it.x1 - it.x0;

    // the A-bins the unit's taps touch
    unsigned long long mine = 0ull;
    for (int c0 = un.y; c0 < un.z; c0 += kWave) {
        const int col = c0 + lane;
        if (col >= un.z) continue;
        const int x = it.x0 + col % nx, y = it.y0 + col / nx;
        for (int z = it.z0; z < it.z1; ++z) {
            const size_t v = ((size_t)z * nfy + y) * nfx + x;
            if (!check_ok(v < nvox, kChkColVoxel)) continue;
            int kA;
            float a0, a1, m1, m2;
            value_voxel<FDT>(kt, fixed, v, L, role, kA, a0, a1, m1, m2);
            mine |= 3ull << kA;
        }
    }
    unsigned long long bins = (unsigned long long)wave_or_dpp((unsigned)(mine >> 32)) << 32 | wave_or_dpp((unsigned)mine);

    const int l16 = lane & 15, kq = lane >> 4;
    while (bins != 0ull) {
        int b[kWin];
#pragma unroll
        for (int w = 0; w < kWin; ++w) {
            b[w] = bins ? (int)__builtin_ctzll(bins) : 1 << 20;
            bins &= bins - 1;
        }
        f4 D[2][NT];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) D[mt][nt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int c0 = un.y; c0 < un.z; c0 += kWave) {
            const int col = c0 + lane;
            float acc[NN];
#pragma unroll
            for (int n = 0; n < NN; ++n) acc[n] = 0.0f;
            float wx5[kXN] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f}, wy[BW];
#pragma unroll
            for (int j = 0; j < BW; ++j) wy[j] = 0.0f;
            if (col < un.z) {
                const int x = it.x0 + col % nx, y = it.y0 + col / nx;
                x_node_weights(gld(spw_x, x), gld(spc_x, x) != it.cx, wx5);
                block_node_weights<BW>(gld(spw_y, y), gld(spc_y, y) != it.cy, wy);
                for (int z = it.z0; z < it.z1; ++z) {
                    const size_t v = ((size_t)z * nfy + y) * nfx + x;
                    if (!check_ok(v < nvox, kChkColVoxel)) continue;
                    int kA;
                    float a0, a1, m1, m2;
                    value_voxel<FDT>(kt, fixed, v, L, role, kA, a0, a1, m1, m2);
                    float wz[BW];
                    block_node_weights<BW>(gld(spw_z, z), gld(spc_z, z) != it.cz, wz);
#pragma unroll
                    for (int w = 0; w < kWin; ++w) {
                        const float t = kA == b[w] ? a0 : (kA + 1 == b[w] ? a1 : 0.0f);
                        const float tm[3] = {t, t * m1, t * m2};
#pragma unroll
                        for (int m = 0; m < 3; ++m)
#pragma unroll
                            for (int k = 0; k < BW; ++k)
                                acc[(w * 3 + m) * BW + k] = fmaf(tm[m], wz[k], acc[(w * 3 + m) * BW + k]);
                    }
                }
            }
            // D[(i, j)][(w, m, k)] += sum over this chunk's columns, four per step:
            // A[r][q] = weight (i, j) = 16 mt + r of column 4 s + q, B[q][c] =
            // sum 16 nt + c of that column (lane r + 16 q / c + 16 q).  Each
            // 16-value piece of a column (weights, then sums) goes to LDS with
            // one column per lane (odd row stride: distinct banks); the
            // weights are read back as the steps' A operands into registers.
            // A lane past the unit's columns writes zeros.
            const int steps = (min(kWave, un.z - c0) + 3) >> 2;
            float aop[2][16];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int m = 16 * mt + e;
                    stg[lane * kColRow + e] = m < NIJ ? wx5[m < NIJ ? m / BW : 0] * wy[m % BW] : 0.0f;
                }
                wave_sync();
#pragma unroll
                for (int st = 0; st < 16; ++st) aop[mt][st] = stg[(4 * st + kq) * kColRow + l16];
                wave_sync();
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
                for (int e = 0; e < 16; ++e) stg[lane * kColRow + e] = 16 * nt + e < NN ? acc[16 * nt + e] : 0.0f;
                wave_sync();
#pragma unroll
                for (int st = 0; st < 16; ++st) {
                    if (st < steps) {
                        const float B = stg[(4 * st + kq) * kColRow + l16];
                        D[0][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[0][st], B, D[0][nt], 0, 0, 0);
                        D[1][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[1][st], B, D[1][nt], 0, 0, 0);
                    }
                }
                wave_sync();
            }
        }
        // the window's sums to the global moments: D[mt][nt][r] holds
        // (i, j) = 16 mt + 4 kq + r, (w, m, k) = 16 nt + l16
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int ij = 16 * mt + 4 * kq + r, n = 16 * nt + l16;
                    const float val = D[mt][nt][r];
                    if (ij >= NIJ || n >= NN || val == 0.0f) continue;
                    const int i = ij / BW, j = ij - BW * i, w = n / (3 * BW), m = (n - 3 * BW * w) / BW, k = n % BW;
                    const int a = w == 0 ? b[0] : (w == 1 ? b[1] : (w == 2 ? b[2] : b[3]));
                    if (a > L || it.cx + i >= g.K[0] || it.cy + j >= g.K[1] || it.cz + k >= g.K[2]) continue;
                    const int R = ((it.cz + k) * g.K[1] + (it.cy + j)) * g.K[0] + (it.cx + i);
                    if (check_ok(R < g.R && a < nb, kChkMoments))
                        unsafeAtomicAdd(&moments[((size_t)R * nb + a) * 3 + m], (double)val);
                }
    }
}

hipError_t launch_value_cols(const Geom *geoms, int fdt, const WorkItem *blocks, const int4 *units, int nunits,
                             const BatchArgs &args, unsigned char *ws, hipStream_t s, int bw)
{
    if (nunits <= 0) return hipSuccess;
    const int nwg = (nunits + kColWaves - 1) / kColWaves;
    const size_t lds = value_cols_lds_bytes();
#define SRWCR_COLS(F, W) \
    if (fdt == F && bw == W) \
        hipLaunchKernelGGL((k_value_cols<F, W>), dim3(nwg), dim3(kColWaves * kWave), lds, s, geoms, blocks, units, \
                           nunits, args, ws);
    SRWCR_COLS(0, 4) SRWCR_COLS(1, 4) SRWCR_COLS(2, 4) SRWCR_COLS(0, 5) SRWCR_COLS(1, 5) SRWCR_COLS(2, 5)
#undef SRWCR_COLS
    return hipGetLastError();
}

// Gradient pass by box columns for boxes of two small cells per axis (the
// regions at the FFD nodes), the moving image as A and an FFD.  One wave per
// box (at most 128 columns (x, y), kGcZ slices, 5 FFD z-nodes and 32 FFD
// (x, y) nodes).  For a window of four A-bins the box's region tables are
// contracted over the 25 (x, y) region weights of every column on the matrix
// cores,
//   Tc[col][(k, w, c)] = sum_(i, j) wx_i(x) wy_j(y) T[(i, j, k)][b_w][c],
// then a lane walks its column's voxels whose bin is in the window: the
// z-contraction gives the interpolated tables C_c (eq 21), dD/ds_M and
// q = dD/ds_M * dM/dy * dy/dT (eq 16), summed over the FFD z-nodes in
// registers, Qz[col][(gz, e)] += beta_gz(z) q_e.  Last, the x and y B-spline
// weights of the FFD (eq 17) are applied on the matrix cores,
//   G[(gx, gy)][(gz, e)] += sum_col bx_gx(x) by_gy(y) Qz[col][(gz, e)],
// and added to the global accumulators with FP64 atomics.
constexpr int kGcWaves = 2;                  // waves (boxes) per workgroup
constexpr int kGcZ = 12;                     // z slices of a box at most
// per wave: operands (tables [32][64] + column weights [32][64], then the
// column sums [64][64] over them) | the chunk's voxels [6][kGcZ][64]
constexpr int kGcFloats = 64 * 64 + 6 * kGcZ * 64;

size_t grad_cols_lds_bytes() { return (size_t)kGcWaves * kGcFloats * sizeof(float); }

// [row][64] with rows rotated by 16 entries: reads of 16 consecutive entries
// of four consecutive rows, and writes of one entry per lane, hit distinct banks
__device__ __forceinline__ int gc_tab_slot(int row, int n) { return row * 64 + ((n + 16 * (row & 3)) & 63); }
// [column][16] rotated for reads of 16 entries of four consecutive columns
__device__ __forceinline__ int gc_q_slot(int col, int n) { return col * 16 + ((n + 4 * (col & 3)) & 15); }

template <int FDT>
__global__ void __launch_bounds__(kGcWaves * kWave)
k_grad_cols(const Geom *__restrict__ geoms, const WorkItem *__restrict__ items, int nitems, BatchArgs args,
            unsigned char *ws)
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int bi = blockIdx.x * kGcWaves + wave;
    if (bi >= nitems) return;
    float *U = reinterpret_cast<float *>(smem) + wave * kGcFloats;
    float *Tw = U, *Wl = U + 32 * 64, *Dc = U;                          // Dc overlays Tw and Wl
    float *Cv = U + 64 * 64;                                            // [6][kGcZ][64]: k, t, F, dM/dy
    const WorkItem it = items[bi];
    const Geom &g = geoms[it.prob];
    const void *__restrict__ fixed = args.p[it.prob].fixed;
    const PrepKT *__restrict__ kt = reinterpret_cast<const PrepKT *>(ws + g.ws.kt);
    const float *__restrict__ dmi = reinterpret_cast<const float *>(ws + g.ws.dm);
    const float *__restrict__ tables = reinterpret_cast<const float *>(ws + g.ws.tables);
    double *__restrict__ grad = reinterpret_cast<double *>(ws + g.ws.grad);
    const int nfx = g.nf[0], nfy = g.nf[1];
    const size_t nvox = (size_t)nfx * nfy * g.nf[2];
    const size_t ncell = (size_t)g.nc[0] * g.nc[1] * g.nc[2];
    const float ratio[3] = {g.ratio[0], g.ratio[1], g.ratio[2]};
    const int nb = g.nb, L = nb - 1;
    const int nx = it.x1 - it.x0, ncol = nx * (it.y1 - it.y0), nz = it.z1 - it.z0;   // nz <= kGcZ
    const int l16 = lane & 15, kq = lane >> 4;

    // the z weights of the box's slices, lane zi holding slice z0 + zi: the
    // regions' (spatial) and the FFD's, each on the box's 5 z-nodes
    float wzl[kXN] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f}, bzl[kXN] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (lane < nz) {
        const int z = it.z0 + lane;
        x_node_weights(gld(g.sp_w[2], z), gld(g.sp_cell[2], z) != it.cz, wzl);
        const double4 bd = gld(g.ffd_w[2], z);
        x_node_weights(make_float4((float)bd.x, (float)bd.y, (float)bd.z, (float)bd.w), gld(g.ffd_p[2], z) != it.gz0,
                       bzl);
    }

    f4 G2[2] = {f4{0.0f, 0.0f, 0.0f, 0.0f}, f4{0.0f, 0.0f, 0.0f, 0.0f}};
    for (int c0 = 0; c0 < ncol; c0 += kWave) {
        const int col = c0 + lane;
        const bool on = col < ncol;
        const int x = it.x0 + (on ? col % nx : 0), y = it.y0 + (on ? col / nx : 0);
        // the column's voxels to LDS, all loads issued together: warped bin and
        // position, fixed value, dM/dy (bin -1 marks a slice past the box)
        unsigned long long mine = 0ull;
#pragma unroll
        for (int zi = 0; zi < kGcZ; ++zi) {
            int k = -1;
            float t = 0.0f, sf = 0.0f, d0 = 0.0f, d1 = 0.0f, d2 = 0.0f;
            const size_t v = ((size_t)(it.z0 + zi) * nfy + y) * nfx + x;
            if (on && zi < nz && check_ok(v < nvox, kChkGradVoxel)) {
                const PrepKT pk = kt[v];
                k = pk.k;
                t = pk.t;
                sf = ld_int<FDT>(fixed, v);
                d0 = dmi[v];
                d1 = dmi[nvox + v];
                d2 = dmi[2 * nvox + v];
                mine |= 1ull << pk.k;
            }
            Cv[(0 * kGcZ + zi) * 64 + lane] = __int_as_float(k);
            Cv[(1 * kGcZ + zi) * 64 + lane] = t;
            Cv[(2 * kGcZ + zi) * 64 + lane] = sf;
            Cv[(3 * kGcZ + zi) * 64 + lane] = d0;
            Cv[(4 * kGcZ + zi) * 64 + lane] = d1;
            Cv[(5 * kGcZ + zi) * 64 + lane] = d2;
        }
        unsigned long long bins = (unsigned long long)wave_or_dpp((unsigned)(mine >> 32)) << 32 |
                                  wave_or_dpp((unsigned)mine);
        float wx5[kXN] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f}, wy5[kXN] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        if (on) {
            x_node_weights(gld(g.sp_w[0], x), gld(g.sp_cell[0], x) != it.cx, wx5);
            x_node_weights(gld(g.sp_w[1], y), gld(g.sp_cell[1], y) != it.cy, wy5);
        }
        float Qz[kXN][3];
#pragma unroll
        for (int k = 0; k < kXN; ++k) Qz[k][0] = Qz[k][1] = Qz[k][2] = 0.0f;
        while (bins != 0ull) {
            int b[kWin];
#pragma unroll
            for (int w = 0; w < kWin; ++w) {
                b[w] = bins ? (int)__builtin_ctzll(bins) : 1 << 20;
                bins &= bins - 1;
            }
            // the window's tables: row (i, j) (25 of 32), entry n = lane = (k, w, c)
            // (60 of 64), every load issued unconditionally (region 0 for an
            // entry outside the lattice, then zeroed); the columns' region
            // weights: row (i, j), entry column
            {
                const int k = lane / 12, w = (lane % 12) / 3, c = lane % 3;
                const int a = w == 0 ? b[0] : (w == 1 ? b[1] : (w == 2 ? b[2] : b[3]));
                const bool okn = lane < 60 && a <= L - 1 && it.cz + k < g.K[2];
                const int Rk = (it.cz + (okn ? k : 0)) * g.K[1];
                const size_t ac = (size_t)(okn ? a : 0) * 4 + c;
#pragma unroll
                for (int i = 0; i < kXN; ++i) {
                    float vj[kXN];
#pragma unroll
                    for (int j = 0; j < kXN; ++j) {
                        const bool ok = okn && it.cx + i < g.K[0] && it.cy + j < g.K[1];
                        const int R = ok ? (Rk + it.cy + j) * g.K[0] + it.cx + i : 0;
                        vj[j] = tables[(size_t)R * nb * 4 + (ok ? ac : 0)];
                        vj[j] = ok ? vj[j] : 0.0f;
                    }
#pragma unroll
                    for (int j = 0; j < kXN; ++j) Tw[gc_tab_slot(i * kXN + j, lane)] = vj[j];
                }
#pragma unroll
                for (int ij = kXN * kXN; ij < 32; ++ij) Tw[gc_tab_slot(ij, lane)] = 0.0f;
            }
#pragma unroll
            for (int m = 0; m < 32; ++m)
                Wl[gc_tab_slot(m, lane)] = m < kXN * kXN ? wx5[m / kXN] * wy5[m % kXN] : 0.0f;
            wave_sync();
            // Tc[col][n] = sum_ij Wl[ij][col] Tw[ij][n]: A[r][q] = weight q of column
            // 16 mt + r, B[q][c] = table entry 16 nt + c of row q (rows 4 s ..)
            f4 D[4][4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) D[mt][nt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int s = 0; s < 7; ++s) {
                float A[4], B[4];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) A[mt] = Wl[gc_tab_slot(4 * s + kq, 16 * mt + l16)];
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) B[nt] = Tw[gc_tab_slot(4 * s + kq, 16 * nt + l16)];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt)
                        D[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[mt], B[nt], D[mt][nt], 0, 0, 0);
            }
            wave_sync();                                             // the column sums overwrite the operands
            // D[mt][nt][r]: column 16 mt + 4 kq + r, entry 16 nt + l16
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                    for (int r = 0; r < 4; ++r) Dc[col_acc_slot(16 * mt + 4 * kq + r, 16 * nt + l16)] = D[mt][nt][r];
            wave_sync();
            // this lane's voxels whose A-bin is in the window
            for (int zi = 0; zi < nz; ++zi) {
                const int kA = __float_as_int(Cv[(0 * kGcZ + zi) * 64 + lane]);
                const int w = kA == b[0] ? 0 : (kA == b[1] ? 1 : (kA == b[2] ? 2 : (kA == b[3] ? 3 : -1)));
                float wz[kXN], bz[kXN];
#pragma unroll
                for (int k = 0; k < kXN; ++k) {
                    wz[k] = bcast(wzl[k], zi);
                    bz[k] = bcast(bzl[k], zi);
                }
                if (w < 0) continue;
                int kF;
                float tF, f0w, f1w;
                parzen(Cv[(2 * kGcZ + zi) * 64 + lane], L, kF, tF, f0w, f1w);
                const float m1 = (float)kF + f1w;
                float C[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float acc = 0.0f;
#pragma unroll
                    for (int k = 0; k < kXN; ++k) acc = fmaf(wz[k], Dc[col_acc_slot(lane, (k * 4 + w) * 3 + c)], acc);
                    C[c] = acc;
                }
                const float gs = parzen_dw0(Cv[(1 * kGcZ + zi) * 64 + lane]) * fmaf(fmaf(C[0], m1, C[1]), m1, C[2]);
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    const float q = gs * Cv[((3 + e) * kGcZ + zi) * 64 + lane] * ratio[e];
#pragma unroll
                    for (int k = 0; k < kXN; ++k) Qz[k][e] = fmaf(bz[k], q, Qz[k][e]);
                }
            }
            wave_sync();                                             // the next window restages the operands
        }
        // G[(gx, gy)][(gz, e)] += sum_col bx_gx(x) by_gy(y) Qz[col][(gz, e)] for this chunk:
        // the FFD weights [column][32] (col_wxy_slot) at U, the sums [column][16] after them
        float *Wg = U, *Qs = U + 64 * 32;
        {
            float bx4[4] = {0.0f, 0.0f, 0.0f, 0.0f}, by4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            int ox = 0, oy = 0;
            if (on) {
                const double4 bxd = gld(g.ffd_w[0], x), byd = gld(g.ffd_w[1], y);
                bx4[0] = (float)bxd.x; bx4[1] = (float)bxd.y; bx4[2] = (float)bxd.z; bx4[3] = (float)bxd.w;
                by4[0] = (float)byd.x; by4[1] = (float)byd.y; by4[2] = (float)byd.z; by4[3] = (float)byd.w;
                ox = gld(g.ffd_p[0], x) - it.gx0;
                oy = gld(g.ffd_p[1], y) - it.gy0;
            }
            const unsigned rgny = (65536u + it.gny - 1) / it.gny;     // m / gny = (m rgny) >> 16 for m < 32
#pragma unroll
            for (int m = 0; m < 32; ++m) {
                const int gx = (int)(((unsigned)m * rgny) >> 16), gy = m - gx * it.gny;
                const int lx = gx - ox, ly = gy - oy;
                float wv = 0.0f;
                if (m < it.gnx * it.gny && lx >= 0 && lx < 4 && ly >= 0 && ly < 4)
                    wv = (lx == 0 ? bx4[0] : (lx == 1 ? bx4[1] : (lx == 2 ? bx4[2] : bx4[3]))) *
                         (ly == 0 ? by4[0] : (ly == 1 ? by4[1] : (ly == 2 ? by4[2] : by4[3])));
                Wg[col_wxy_slot(lane, m)] = wv;
            }
#pragma unroll
            for (int n = 0; n < 16; ++n) {
                const int k = n / 3, e = n - 3 * k;
                Qs[gc_q_slot(lane, n)] = n < 3 * kXN ? Qz[k < kXN ? k : 0][e] : 0.0f;
            }
            wave_sync();
            // A[r][q] = weight of node 16 mt + r for column 4 s + q, B[q][c] = sum c of that column
            const int steps = (min(kWave, ncol - c0) + 3) >> 2;
            for (int s = 0; s < steps; ++s) {
                const int cq = 4 * s + kq;
                const float A0 = Wg[col_wxy_slot(cq, l16)], A1 = Wg[col_wxy_slot(cq, 16 + l16)];
                const float B = Qs[gc_q_slot(cq, l16)];
                G2[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(A0, B, G2[0], 0, 0, 0);
                G2[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(A1, B, G2[1], 0, 0, 0);
            }
            wave_sync();
        }
    }
    // G2[mt][r]: node (gx, gy) = 16 mt + 4 kq + r, entry (gz, e) = l16
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int m = 16 * mt + 4 * kq + r, n = l16;
            const float val = G2[mt][r];
            if (m >= it.gnx * it.gny || n >= 3 * it.gnz || val == 0.0f) continue;
            const int gx = (int)(((unsigned)m * ((65536u + it.gny - 1) / it.gny)) >> 16), gy = m - gx * it.gny;
            const int gz = n / 3, e = n - 3 * gz;
            const size_t node = ((size_t)(it.gz0 + gz) * g.nc[1] + (it.gy0 + gy)) * g.nc[0] + (it.gx0 + gx);
            if (check_ok(node < ncell, kChkGrad)) unsafeAtomicAdd(&grad[e * ncell + node], (double)val);
        }
}

hipError_t launch_grad_cols(const Geom *geoms, int fdt, const WorkItem *items, int nitems, const BatchArgs &args,
                            unsigned char *ws, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    const int nwg = (nitems + kGcWaves - 1) / kGcWaves;
    const size_t lds = grad_cols_lds_bytes();
    if (fdt == 0) hipLaunchKernelGGL(k_grad_cols<0>, dim3(nwg), dim3(kGcWaves * kWave), lds, s, geoms, items, nitems, args, ws);
    else if (fdt == 1) hipLaunchKernelGGL(k_grad_cols<1>, dim3(nwg), dim3(kGcWaves * kWave), lds, s, geoms, items, nitems, args, ws);
    else hipLaunchKernelGGL(k_grad_cols<2>, dim3(nwg), dim3(kGcWaves * kWave), lds, s, geoms, items, nitems, args, ws);
    return hipGetLastError();
}

// ---------------------------------------------------------- finalisation
// Called by one whole wave for region r of g, lane = intensity bin a holding
// the bin's moments (P, S1, S2) (zeros for a >= nb):
// region[4 r + 0..3] = (U_r / sigma_r^2, p_r, sigma_r^2, CR_r), and the
// region's gradient tables and alpha_r.
__device__ void finalize_region(const Geom &g, int r, int a, double P, double S1, double S2, unsigned char *ws)
{
    const int nb = g.nb;
    double *region = reinterpret_cast<double *>(ws + g.ws.region);
    float *tables = reinterpret_cast<float *>(ws + g.ws.tables);
    float *alpha = reinterpret_cast<float *>(ws + g.ws.alpha);
    const double Pr = wave_sum_d(P), S1r = wave_sum_d(S1), S2r = wave_sum_d(S2);
    const bool filled = P > 0.0;
    const double mu_a = filled ? S1 / P : 0.0;
    const double U = wave_sum_d(filled ? S2 - S1 * mu_a : 0.0);
    double var = 0.0;
    bool ok = Pr > 0.0;
    if (ok) {
        // degenerate region (B constant to 0.3 %): sigma_r^2 <= 1e-5 E_r[b^2], a
        // margin of ~50x over the rounding of the FP32 window sums
        const double mu = S1r / Pr, e2 = S2r / Pr;
        var = e2 - mu * mu;
        ok = var > 1e-5 * e2;
    }
    const double mu_r = ok ? S1r / Pr : 0.0;
    const double omc = ok ? U / (Pr * var) : 0.0;       // 1 - CR_r
    const double cr = ok ? 1.0 - omc : 0.0;
    const double s = ok ? g.inv_Z / var : 0.0;
    // Tables of both adjoints, each scaled by 1/(Z sigma_r^2): the image that
    // plays B needs E'_a = 2 mu_r(a) - 2 (1 - CR_r) mu_r and alpha_r = CR_r; the
    // image that plays A needs the coefficients (c2, c1, c0) of m1^2, m1, 1 in
    // (m1 - mu(a))^2 - (m1 - mu(a+1))^2, an empty bin's square taken as 0.
    // Slots per (r, a): moving is A: (c2, c1, c0, E'); moving is B:
    // (E', c2, c1, c0) -- the moving image's adjoint first, the fixed image's
    // after it.
    float *tp = tables + ((size_t)r * nb + a) * 4;
    const double mu_n = __shfl_down(mu_a, 1);
    const int fill_n = __shfl_down(filled ? 1 : 0, 1);
    if (a < nb) {
        const double E = (filled ? 2.0 * mu_a : 0.0) - 2.0 * omc * mu_r;
        double c2 = 0.0, c1 = 0.0, c0 = 0.0;
        const bool f0 = filled, f1 = (a + 1 < nb) && fill_n;
        if (f0 && f1) {
            c1 = 2.0 * (mu_n - mu_a);
            c0 = -(mu_n - mu_a) * (mu_n + mu_a);
        } else if (f0) {
            c2 = 1.0;
            c1 = -2.0 * mu_a;
            c0 = mu_a * mu_a;
        } else if (f1) {
            c2 = -1.0;
            c1 = 2.0 * mu_n;
            c0 = -mu_n * mu_n;
        }
        const float tE = (float)(s * E), t2 = (float)(s * c2), t1 = (float)(s * c1), t0 = (float)(s * c0);
        if (g.role == 1) {
            tp[0] = tE;
            tp[1] = t2;
            tp[2] = t1;
            tp[3] = t0;
        } else {
            tp[0] = t2;
            tp[1] = t1;
            tp[2] = t0;
            tp[3] = tE;
        }
    }
    if (a == 0) alpha[r] = (float)(s * cr);
    if (a == 0) {
        region[4 * r + 0] = ok ? U / var : 0.0;
        region[4 * r + 1] = Pr;
        region[4 * r + 2] = var;
        region[4 * r + 3] = cr;
    }
}

// One wave per region r (lane = intensity bin a) of problem blockIdx.y,
// reading the moments the value pass merged with atomics; k_value_sum then
// writes D = (1/Z) sum_r U_r / sigma_r^2.
__global__ void __launch_bounds__(64)
k_finalize(const Geom *__restrict__ geoms, BatchArgs args, unsigned char *ws)
{
    const Geom &g = geoms[blockIdx.y];
    const int r = blockIdx.x, a = threadIdx.x, nb = g.nb;
    if (r >= g.R) return;
    const double *__restrict__ moments = reinterpret_cast<const double *>(ws + g.ws.moments);
    double P = 0.0, S1 = 0.0, S2 = 0.0;
    if (a < nb) {
        const double *mp = moments + ((size_t)r * nb + a) * 3;
        P = mp[0];
        S1 = mp[1];
        S2 = mp[2];
    }
    finalize_region(g, r, a, P, S1, S2, ws);
}

// Moments of a region from the staged value pass: the sum, in a fixed order,
// of the staging slots of every visit whose block holds it (visits
// ent[reg_start[q] ..], each entry visit * nreg + local region; a visit's slots
// start at visit * stage_stride).  Workgroup q takes region reg_id[q] =
// (problem, region), or (0, q) without reg_id; 64 W threads: wave w takes
// entries w, w + W, ...; lane a < nb the three moments of bin a; the W
// partial sums are added in wave order, and wave 0 then finalises the region.
__global__ void __launch_bounds__(1024)
k_merge(const Geom *__restrict__ geoms, const double *__restrict__ staging, long stage_stride, int nreg,
        const int *__restrict__ reg_start, const int *__restrict__ ent, const int2 *__restrict__ reg_id,
        unsigned char *ws)
{
    extern __shared__ double part[];                     // [W][nb][3]
    const int q = blockIdx.x;
    const int2 id = reg_id ? reg_id[q] : make_int2(0, q);
    const Geom &g = geoms[id.x];
    double *__restrict__ moments = reinterpret_cast<double *>(ws + g.ws.moments);
    const int r = id.y, nb = g.nb, lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
    const int W = blockDim.x >> 6, nb3 = nb * 3;
    const int e0 = reg_start[q], e1 = reg_start[q + 1];
    auto slot = [&](int e) {
        const int v = ent[e];
        return staging + (size_t)(v / nreg) * stage_stride + (size_t)(v % nreg) * nb3 + 3 * lane;
    };
    double s[3] = {0.0, 0.0, 0.0};
    if (lane < nb) {
        int e = e0 + w;
        for (; e + 3 * W < e1; e += 4 * W) {             // four entries in flight
            double v[4][3];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double *p = slot(e + u * W);
#pragma unroll
                for (int m = 0; m < 3; ++m) v[u][m] = p[m];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int m = 0; m < 3; ++m) s[m] += v[u][m];
        }
        for (; e < e1; e += W) {
            const double *p = slot(e);
#pragma unroll
            for (int m = 0; m < 3; ++m) s[m] += p[m];
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) part[(w * nb + lane) * 3 + m] = s[m];
    }
    __syncthreads();
    if (w == 0) {
        double t[3] = {0.0, 0.0, 0.0};
        if (lane < nb) {
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                for (int ww = 0; ww < W; ++ww) t[m] += part[(ww * nb + lane) * 3 + m];
                moments[((size_t)r * nb + lane) * 3 + m] = t[m];
            }
        }
        finalize_region(g, r, lane, t[0], t[1], t[2], ws);
    }
}

hipError_t launch_merge(const Geom *geoms, const double *staging, long stage_stride, int nreg, const int *reg_start,
                        const int *ent, const int2 *reg_id, int nregions, int max_nb, int waves, unsigned char *ws,
                        hipStream_t s)
{
    if (nregions <= 0) return hipSuccess;
    const size_t lds = (size_t)waves * max_nb * 3 * sizeof(double);
    hipLaunchKernelGGL(k_merge, dim3(nregions), dim3(waves * kWave), lds, s, geoms, staging, stage_stride, nreg,
                       reg_start, ent, reg_id, ws);
    return hipGetLastError();
}

template <typename F>
static hipError_t set_lds(F *kernel, size_t bytes)
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

hipError_t launch_value(const Geom *geoms, int fdt, const WorkItem *blocks, const int *row_start, int nblocks,
                        int nwg, const BatchArgs &args, unsigned char *ws, size_t lds_bytes, hipStream_t s,
                        double *staging, const int *visit_start, long stage_stride, int bw)
{
    if (nblocks <= 0 || nwg <= 0) return hipSuccess;
    const int ld = (int)(lds_bytes / sizeof(double));
#define SRWCR_VAL(F)                                                                                               \
    if (bw == 5)                                                                                                   \
        hipLaunchKernelGGL((k_value<F, 5>), dim3(nwg), dim3(kValueThreads), lds_bytes, s, geoms, blocks, row_start, \
                           nblocks, ld, args, ws, staging, visit_start, stage_stride);                             \
    else                                                                                                           \
        hipLaunchKernelGGL((k_value<F, 4>), dim3(nwg), dim3(kValueThreads), lds_bytes, s, geoms, blocks, row_start, \
                           nblocks, ld, args, ws, staging, visit_start, stage_stride)
    if (fdt == 0) SRWCR_VAL(0);
    else if (fdt == 1) SRWCR_VAL(1);
    else SRWCR_VAL(2);
#undef SRWCR_VAL
    return hipGetLastError();
}

// D = (1/Z) sum_r U_r / sigma_r^2 of problem blockIdx.x, summed in a fixed
// order: thread t adds regions t, t + 1024, ... in increasing order (eight
// loads in flight), then a fixed tree over the 1024 partial sums.  A launch of
// its own: it sees every region's term without a device-scope fence in each
// finalising wave.
constexpr int kSumThreads = 1024;

__global__ void __launch_bounds__(kSumThreads)
k_value_sum(const Geom *__restrict__ geoms, BatchArgs args, unsigned char *ws)
{
    __shared__ double part[kSumThreads];
    const Geom &g = geoms[blockIdx.x];
    const double *region = reinterpret_cast<const double *>(ws + g.ws.region);
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int q0 = t; q0 < g.R; q0 += 8 * kSumThreads) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = q0 + u * kSumThreads < g.R ? region[4 * (q0 + u * kSumThreads)] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += x[u];
    }
    part[t] = acc;
    __syncthreads();
    for (int h = kSumThreads / 2; h > 0; h >>= 1) {
        if (t < h) part[t] += part[t + h];
        __syncthreads();
    }
    if (t == 0) *args.p[blockIdx.x].value = part[0] * g.inv_Z;
}

hipError_t launch_finalize(const Geom *geoms, int nprob, int max_regions, const BatchArgs &args, unsigned char *ws,
                           hipStream_t s, bool merged)
{
    if (!merged) {
        hipLaunchKernelGGL(k_finalize, dim3(max_regions, nprob), dim3(64), 0, s, geoms, args, ws);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_value_sum, dim3(nprob), dim3(kSumThreads), 0, s, geoms, args, ws);
    return hipGetLastError();
}

// --------------------------------------------------------- gradient pass

// LDS copy of the gradient tables: tab[x-node i][bin a][coefficient c][jk],
// the BW^2 (y, z) regions jk = BW k + j of one (i, a, c) contiguous, so that a
// row-table entry reads them at fixed offsets (four 16-byte loads when BW =
// 4).  The stride of 20 (BW = 4) or 28 (BW = 5) floats keeps the loads of
// consecutive (a, c) on distinct banks.
__host__ __device__ constexpr int tab_jk_stride(int bw) { return bw == 5 ? 28 : 20; }

// Stride of the x-nodes in the tables, in floats: nb * 3 * JKS, padded.  The
// lanes that build a row table read the 15 (i, c) entries of one bin together,
// and unpadded (a multiple of 64 floats at 64 bins) all five x-nodes of one
// coefficient would sit on the same banks.  Padded to -4 mod 64 floats (BW =
// 4), the 16-byte loads of any 8 consecutive (i, c) take distinct 16-byte
// slots of 128 bytes, and those of all 15 distinct slots of 256 bytes; padded
// to 3 mod 64 (BW = 5, 4-byte loads), the 15 fall on distinct banks of 32 and
// of 64.
__host__ __device__ constexpr int tab_i_stride(int nb, int bw)
{
    const int s = nb * 3 * tab_jk_stride(bw), want = bw == 5 ? 3 : 60;
    return s + ((want - s % 64) % 64 + 64) % 64;
}

// Floats of the tables, rounded up to 16 bytes (the alpha values follow).
__host__ __device__ constexpr int tab_floats(int nb, int bw) { return (kXN * tab_i_stride(nb, bw) + 3) / 4 * 4; }

// Offset of the tables in the gradient pass's LDS: after the item's FFD x
// weights and node block, rounded up to 16 bytes.
__host__ __device__ __forceinline__ size_t grad_tab_offset(int xw, int nG)
{
    return ((size_t)xw * 16 + (size_t)nG * 8 + 15) / 16 * 16;
}

// Regions of an item's block, padded so that the per-wave scratch after their
// alpha values starts on 16 bytes.
__host__ __device__ constexpr int grad_nreg_padded(int bw) { return (kXN * bw * bw + 3) / 4 * 4; }

size_t grad_lds_bytes(const Geom &g, int gnx, int gny, int gnz)
{
    const size_t tab = (size_t)tab_floats(g.nb, g.bw) * sizeof(float) + (size_t)grad_nreg_padded(g.bw) * sizeof(float);
    const size_t scratch = (size_t)(kGradThreads / kWave) * g.gscr * sizeof(float);
    return grad_tab_offset(g.xw, gnx * gny * gnz * 3) + tab + scratch;
}

// Global inputs of one row of the gradient pass, loaded a row ahead.
struct RowG {
    PrepKT pk[kSlots];  // the warped moving sample
    float s[kSlots];    // the fixed image's value, or dD/ds_M of the voxel (ROLE 2)
    float dm[kSlots][3];// dM/dy
    float us;           // lanes 0-3 / 4-7: spatial weights of y / z
    double uf;          // lanes 0-3 / 4-7: FFD weights of y / z
    int c;              // lanes 0 / 1: FFD cells of y / z; 2 / 3: spatial cells of y / z
};

// Row-uniform tables the gradient pass reads per row (hoisted pointers).
struct RowTabs {
    const float *spy, *spz;     // spatial weights [4 per coordinate]
    const double *fwy, *fwz;    // FFD weights [4 per coordinate]
    const int *fpy, *fpz;       // FFD cells
    const int *scy, *scz;       // spatial cells
};

// Every lane issues each load (at a valid address) and keeps the value its
// lane stands for: lane-dependent branches around loads into one register
// would make the compiler wait for all loads in flight, the prefetch included.
template <int FDT, int ROLE, int DISP, int BW>
__device__ __forceinline__ void grad_load_row(RowG &in, const RowTabs &tb, const void *__restrict__ fixed,
                                              const PrepKT *__restrict__ kt, const float *__restrict__ dmi,
                                              const float *__restrict__ rds, size_t nvox, size_t rowb, int y, int z,
                                              const int (&xc)[kSlots], int lane)
{
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
        if (!check_ok(rowb + xc[sl] < nvox, kChkGradVoxel)) continue;
        if constexpr (DISP != 2) {
#pragma unroll
            for (int e = 0; e < 3; ++e) in.dm[sl][e] = dmi[e * nvox + rowb + xc[sl]];
        }
        if constexpr (ROLE == 2) {
            in.s[sl] = gld(rds, rowb + xc[sl]);
        } else {
            in.pk[sl] = kt[rowb + xc[sl]];
            in.s[sl] = ld_int<FDT>(fixed, rowb + xc[sl]);
        }
    }
    const int l3 = lane & 3;
    const bool zl = lane & 4;
    if constexpr (ROLE < 2) in.us = gld(zl ? tb.spz + 4 * z : tb.spy + 4 * y, l3);
    if constexpr (DISP == 0) in.uf = gld(zl ? tb.fwz + 4 * z : tb.fwy + 4 * y, l3);
    if constexpr (DISP == 0 || (ROLE < 2 && BW == 5)) {
        const int *pc = tb.fpy + y;
        if (DISP == 0 && l3 == 1) pc = tb.fpz + z;
        if (ROLE < 2 && BW == 5 && l3 == 2) pc = tb.scy + y;
        if (ROLE < 2 && BW == 5 && l3 == 3) pc = tb.scz + z;
        in.c = gld(pc, 0);
    }
}

// DISP 0: scatter dD/dT to the FFD nodes (eq 17) into the workspace
// accumulators; DISP 1: write dD/du(x) of a dense field to args.p[].grad;
// DISP 2: write dD/ds_F, the fixed image's adjoint, per voxel to
// args.p[].grad (no chain rule).  ROLE 0 / 1: the adjoints from the SRWCR
// region tables, moving image as A / B; ROLE 2: dD/ds_M read per voxel from
// the workspace (RaPTOR), so only the chain rule (eq 16) and the scatter run.
template <int FDT, int ROLE, int DISP, int BW>
__global__ void __launch_bounds__(kGradThreads)
k_grad(const Geom *__restrict__ geoms, const WorkItem *__restrict__ items, BatchArgs args, unsigned char *ws)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const WorkItem it = items[blockIdx.x];
    const Geom &g = geoms[it.prob];
    const void *__restrict__ fixed = args.p[it.prob].fixed;
    const PrepKT *__restrict__ kt = reinterpret_cast<const PrepKT *>(ws + g.ws.kt);
    const float *__restrict__ dmi = reinterpret_cast<const float *>(ws + g.ws.dm);
    const size_t nvox = (size_t)g.nf[0] * g.nf[1] * g.nf[2];
    const float *__restrict__ tables = reinterpret_cast<const float *>(ws + g.ws.tables);
    const float *__restrict__ alpha = reinterpret_cast<const float *>(ws + g.ws.alpha);
    const float *__restrict__ rds = reinterpret_cast<const float *>(ws + g.ws.rds);
    double *__restrict__ grad = reinterpret_cast<double *>(ws + g.ws.grad);
    const int nfx = g.nf[0], nfy = g.nf[1], dx = g.delta[0];
    const float ratio[3] = {g.ratio[0], g.ratio[1], g.ratio[2]};
    const int nb = g.nb, L = nb - 1;
    const int nG = it.gnx * it.gny * it.gnz * 3;
    float4 *bxw = reinterpret_cast<float4 *>(smem);                     // FFD x weights of the item's x range
    double *G = reinterpret_cast<double *>(bxw + g.xw);                 // [gnz][gny][gnx][3]
    float *tab = reinterpret_cast<float *>(smem + grad_tab_offset(g.xw, nG));   // [kXN (stride TS)][nb][3][JKS]
    constexpr int NR = kXN * BW * BW;                                    // regions of the item's block
    constexpr int JKS = tab_jk_stride(BW);
    const int TS = tab_i_stride(nb, BW);
    float *alph = tab + tab_floats(nb, BW);                              // [NR]
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nwaves = blockDim.x >> 6;
    // per-wave scratch: bin list [64] | row tables [kRowBins][NE] or q [128][3] | cell moments
    float *scr = alph + grad_nreg_padded(BW) + wave * g.gscr;
    int *blist = reinterpret_cast<int *>(scr);
    float *rowt = scr + 64;
    float *qb = rowt;
    float *cm = rowt + (kRowBins * kRowEntry > 3 * kSlots * kWave ? kRowBins * kRowEntry : 3 * kSlots * kWave);
    // the adjoint taken: of the image that plays A (eq 21) or B (eq 19), and
    // where its tables sit in the four slots per (region, bin)
    constexpr bool FA = DISP == 2 ? ROLE == 1 : ROLE == 0;
    constexpr int CO = DISP == 2 ? (ROLE == 0 ? 3 : 1) : 0;
    // a row-table entry: the 5 x-nodes x 3 coefficients of a bin of A (15 of
    // kRowEntry floats), or the 5 x-nodes of a bin of B (5 of 8)
    constexpr int NE = FA ? kRowEntry : 8;
    constexpr int NU = FA ? kXN * 3 : kXN;

    const int xs = it.x0, xe = it.x1;
    if (DISP == 0)
        for (int i = threadIdx.x; i < nG; i += blockDim.x) G[i] = 0.0;
    for (int i = threadIdx.x; DISP == 0 && i < xe - xs; i += blockDim.x) {
        const double4 b = gld(g.ffd_w[0], xs + i);
        bxw[i] = make_float4((float)b.x, (float)b.y, (float)b.z, (float)b.w);
    }
    // the block's tables to LDS: lane = bin (nb <= 64) and regions rl = wave,
    // wave + nwaves, ... so that the index arithmetic is wave-uniform; kStage
    // regions per wave at a time, all their loads issued before the first
    // store (a region outside the lattice reads region 0 and stores zeros)
    constexpr int kStage = 8;
    for (int r0 = wave; ROLE < 2 && r0 < NR; r0 += kStage * nwaves) {
        float t0[kStage], t1[kStage], t2[kStage], al[kStage];
        bool ok[kStage];
        const int a = lane < nb ? lane : 0;
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int rl = r0 + u * nwaves;
            const int ii = rl % kXN, jk = rl / kXN, kk = jk / BW, jj = jk - kk * BW;
            ok[u] = rl < NR && it.cx + ii < g.K[0] && it.cy + jj < g.K[1] && it.cz + kk < g.K[2];
            const int R = ok[u] ? ((it.cz + kk) * g.K[1] + (it.cy + jj)) * g.K[0] + (it.cx + ii) : 0;
            const size_t o = ((size_t)R * nb + a) * 4 + CO;
            if constexpr (FA && CO == 0) {
                const float4 q = gld(reinterpret_cast<const float4 *>(tables), o / 4);
                t0[u] = q.x;
                t1[u] = q.y;
                t2[u] = q.z;
            } else {
                t0[u] = gld(tables, o);
                t1[u] = FA ? gld(tables, o + 1) : 0.0f;
                t2[u] = FA ? gld(tables, o + 2) : 0.0f;
            }
            al[u] = gld(alpha, R);
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int rl = r0 + u * nwaves;
            if (rl >= NR) break;
            const int ii = rl % kXN, jk = rl / kXN;
            if (lane < nb && check_ok(jk < JKS, kChkTabJK)) {
                float *tq = tab + ii * TS + lane * 3 * JKS + jk;
                tq[0] = ok[u] ? t0[u] : 0.0f;
                tq[JKS] = ok[u] ? t1[u] : 0.0f;
                tq[2 * JKS] = ok[u] ? t2[u] : 0.0f;
            }
            if (lane == 0) alph[rl] = ok[u] ? al[u] : 0.0f;
        }
    }
    // the item's x range is the same for all its rows: the voxels of each
    // lane, their x-node weights and the FFD cells of the range
    bool pend[kSlots];
    int xcl[kSlots];
    float wx5[kSlots][kXN];
#pragma unroll
    for (int sl = 0; sl < kSlots; ++sl) {
        const int x = xs + sl * kWave + lane;
        pend[sl] = x < xe;
        xcl[sl] = pend[sl] ? x : xe - 1;
        if constexpr (ROLE < 2) x_node_weights(gld(g.sp_w[0], xcl[sl]), gld(g.sp_cell[0], xcl[sl]) != it.cx, wx5[sl]);
    }
    int px_lo = 0, np = 0;
    if constexpr (DISP == 0) {
        int pxc = 0;
        if (lane == 0) pxc = gld(g.ffd_p[0], xs);
        else if (lane == 1) pxc = gld(g.ffd_p[0], xe - 1);
        px_lo = bcast(pxc, 0);
        np = bcast(pxc, 1) - px_lo + 1;
        if (!check_ok(64 + (kRowBins * kRowEntry > 3 * kSlots * kWave ? kRowBins * kRowEntry : 3 * kSlots * kWave) +
                          12 * (np + 6) <= g.gscr, kChkScratch))
            np = 0;
        for (int i = lane; i < 12 * (np + 6); i += kWave) cm[i] = 0.0f;   // pad cells stay zero
    }
    __syncthreads();

    // each wave takes a contiguous run of the item's rows, z fastest, so that
    // consecutive rows of a wave mostly share y and the FFD z-cell (see the
    // scatter below); its global inputs are loaded a row ahead
    const int ny = it.y1 - it.y0, nz = it.z1 - it.z0, nrows = ny * nz;
    const int rb = wave * nrows / nwaves, re = (wave + 1) * nrows / nwaves;
    const RowTabs tb{reinterpret_cast<const float *>(g.sp_w[1]), reinterpret_cast<const float *>(g.sp_w[2]),
                     reinterpret_cast<const double *>(g.ffd_w[1]), reinterpret_cast<const double *>(g.ffd_w[2]),
                     g.ffd_p[1], g.ffd_p[2], g.sp_cell[1], g.sp_cell[2]};
    RowG cur{}, nxt{};
    if (rb < re) {
        const int y = it.y0 + rb / nz, z = it.z0 + rb % nz;
        grad_load_row<FDT, ROLE, DISP, BW>(cur, tb, fixed, kt, dmi, rds, nvox, ((size_t)z * nfy + y) * nfx, y, z, xcl,
                                           lane);
    }
    // the scatter's group: q of the rows with one y and one FFD z-cell,
    // contracted over the z-nodes, Q[sl][c][e] = sum_rows beta_c(z) q_e
    float Q[kSlots][4][3];
    int gyr = 0, gpy = 0, gpz = -1;
    float gby[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    // ... then per z-node c the x-scatter of the group (eq 17): per FFD cell p
    // of the row range the four moments M[p][l][e] = sum_{x in p}
    // beta_l(eta_x) Q_c,e(x), node sums R1[n][e] = sum_l M[n - l][l][e]
    // (cells outside the range read the zero pads), and the four y-nodes
    auto flush = [&]() {
        const int sy = it.gnx * 3;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
            for (int sl = 0; sl < kSlots; ++sl)
#pragma unroll
                for (int e = 0; e < 3; ++e) qb[(sl * kWave + lane) * 3 + e] = Q[sl][c][e];
            wave_sync();
            for (int t = lane; t < np * 3; t += kWave) {
                const int p = t / 3, e = t - 3 * p;
                const int xa = max(xs, (px_lo + p) * dx), xb = min(xe, (px_lo + p + 1) * dx);
                float m0 = 0.0f, m1_ = 0.0f, m2_ = 0.0f, m3 = 0.0f;
                for (int xx = xa; xx < xb; xx += 2) {                // two voxels per step, loads issued together
                    const int x1 = min(xx + 1, xb - 1);
                    const float qa = qb[(xx - xs) * 3 + e], qn = qb[(x1 - xs) * 3 + e];
                    const float4 ba = bxw[xx - xs], bn = bxw[x1 - xs];
                    const float q2 = xx + 1 < xb ? qn : 0.0f;
                    m0 = fmaf(bn.x, q2, fmaf(ba.x, qa, m0));
                    m1_ = fmaf(bn.y, q2, fmaf(ba.y, qa, m1_));
                    m2_ = fmaf(bn.z, q2, fmaf(ba.z, qa, m2_));
                    m3 = fmaf(bn.w, q2, fmaf(ba.w, qa, m3));
                }
                float *cp = cm + (p + 3) * 12 + e;
                cp[0] = m0;
                cp[3] = m1_;
                cp[6] = m2_;
                cp[9] = m3;
            }
            wave_sync();
            for (int t = lane; t < (np + 3) * 3; t += kWave) {
                const int n = t / 3, e = t - 3 * n;
                const float *cp = cm + (n + 3) * 12 + e;
                const float r1 = ((cp[0] + cp[-12 + 3]) + cp[-24 + 6]) + cp[-36 + 9];
                if (r1 != 0.0f) {
                    const int o = ((gpz + c - it.gz0) * it.gny + (gpy - it.gy0)) * sy + (px_lo + n - it.gx0) * 3 + e;
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if (check_ok(o >= 0 && o + b * sy < nG, kChkNodeBlock))
                            atomicAdd(G + o + b * sy, (double)(r1 * gby[b]));
                }
            }
            wave_sync();
        }
    };
    for (int row = rb; row < re; ++row) {
        const int y = it.y0 + row / nz, z = it.z0 + row % nz;
        const size_t rowb = ((size_t)z * nfy + y) * nfx;
        if (row + 1 < re) {
            const int yn = it.y0 + (row + 1) / nz, zn = it.z0 + (row + 1) % nz;
            grad_load_row<FDT, ROLE, DISP, BW>(nxt, tb, fixed, kt, dmi, rds, nvox, ((size_t)zn * nfy + yn) * nfx, yn,
                                               zn, xcl, lane);
        }
        float gs[kSlots] = {0.0f, 0.0f};
        if constexpr (ROLE == 2) {
#pragma unroll
            for (int sl = 0; sl < kSlots; ++sl) gs[sl] = pend[sl] ? cur.s[sl] : 0.0f;   // dD/ds_M of the voxel
        } else {
        int kA[kSlots], kB[kSlots];
        float tA[kSlots], tB[kSlots], a0[kSlots], a1[kSlots], m1[kSlots];
#pragma unroll
        for (int sl = 0; sl < kSlots; ++sl) {
            int kF;
            float tF, m0w, m1w, f0w, f1w;
            const int kM = cur.pk[sl].k;
            const float tM = cur.pk[sl].t;
            parzen_w(tM, m0w, m1w);
            parzen(cur.s[sl], L, kF, tF, f0w, f1w);
            kA[sl] = ROLE ? kF : kM;
            kB[sl] = ROLE ? kM : kF;
            tA[sl] = ROLE ? tF : tM;
            tB[sl] = ROLE ? tM : tF;
            a0[sl] = ROLE ? f0w : m0w;
            a1[sl] = ROLE ? f1w : m1w;
            m1[sl] = (float)kB[sl] + (ROLE ? m1w : f1w);
        }
        float wyv[4], wzv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            wyv[j] = bcast(cur.us, j);
            wzv[j] = bcast(cur.us, 4 + j);
        }
        int oyz = 0;                                                 // the row's (y, z) cells in a two-cell item
        if constexpr (BW == 5) oyz = (bcast(cur.c, 3) - it.cz) * BW + (bcast(cur.c, 2) - it.cy);

        // dD/ds_M: the region tables interpolated by w(r, x) = wx wy wz.  Row
        // tables T_row[s][i][c] = sum_jk wy_j wz_k T[(i, j, k)][bin_s][c] are
        // built for the bins s the row's voxels need (a wave-uniform 64-bit
        // set: k_A, and k_A + 1 when the moving image is B), one entry per
        // lane, kRowBins bins at a time; each voxel then combines its bin's 5
        // x-node entries, found at slot popcount(bins below k_A).
        unsigned long long mine = 0ull;
#pragma unroll
        for (int sl = 0; sl < kSlots; ++sl)
            if (pend[sl]) mine |= (FA ? 1ull : 3ull) << kA[sl];
        const unsigned long long bins = (unsigned long long)wave_or_dpp((unsigned)(mine >> 32)) << 32 |
                                        wave_or_dpp((unsigned)mine);
        const int nd = __builtin_popcountll(bins);
        int sbv[kSlots];
#pragma unroll
        for (int sl = 0; sl < kSlots; ++sl) sbv[sl] = __builtin_popcountll(bins & ((1ull << kA[sl]) - 1ull));
        if ((bins >> lane) & 1ull) blist[__builtin_popcountll(bins & ((1ull << lane) - 1ull))] = lane;
        float arow[kXN];                                             // B's adjoint: CR_r / (sigma_r^2 Z) per x-node
        if (!FA) {
            float al = 0.0f;
            if (lane < kXN) {
#pragma unroll
                for (int kz = 0; kz < 4; ++kz)
#pragma unroll
                    for (int jy = 0; jy < 4; ++jy)
                        al = fmaf(wyv[jy] * wzv[kz], alph[(oyz + kz * BW + jy) * kXN + lane], al);
            }
#pragma unroll
            for (int i = 0; i < kXN; ++i) arow[i] = bcast(al, i);
        }
        wave_sync();
        // chunks of kRowBins bins; with B's adjoint a voxel needs bins k_A and
        // k_A + 1 (adjacent in the set), so chunks overlap by one bin
        constexpr int STEP = FA ? kRowBins : kRowBins - 1;
        for (int c0 = 0; c0 + (FA ? 0 : 1) < nd; c0 += STEP) {
            const int nc = min(kRowBins, nd - c0);
            for (int e = lane; e < nc * NU; e += kWave) {
                const int sb = e / NU, r = e - sb * NU;
                const int a = blist[c0 + sb];
                float acc = 0.0f;
                if (a <= (FA ? L - 1 : L)) {
                    const int i = FA ? r / 3 : r, c = FA ? r - 3 * i : 0;
                    const float *tp = tab + i * TS + (a * 3 + c) * JKS + oyz;
                    if constexpr (BW == 4) {
#pragma unroll
                        for (int kz = 0; kz < 4; ++kz) {
                            const float4 q = reinterpret_cast<const float4 *>(tp)[kz];
                            acc = fmaf(wyv[0] * wzv[kz], q.x, acc);
                            acc = fmaf(wyv[1] * wzv[kz], q.y, acc);
                            acc = fmaf(wyv[2] * wzv[kz], q.z, acc);
                            acc = fmaf(wyv[3] * wzv[kz], q.w, acc);
                        }
                    } else {
#pragma unroll
                        for (int kz = 0; kz < 4; ++kz)
#pragma unroll
                            for (int jy = 0; jy < 4; ++jy) acc = fmaf(wyv[jy] * wzv[kz], tp[kz * BW + jy], acc);
                    }
                }
                rowt[sb * NE + r] = acc;
            }
            wave_sync();
#pragma unroll
            for (int sl = 0; sl < kSlots; ++sl) {
                const int s = sbv[sl] - c0;
                if (!pend[sl] || s < 0 || s > nc - (FA ? 1 : 2)) continue;
                if (FA) {
                    const float4 *rt = reinterpret_cast<const float4 *>(rowt + s * NE);
                    const float4 q0 = rt[0], q1 = rt[1], q2 = rt[2], q3 = rt[3];
                    const float r[16] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w,
                                         q2.x, q2.y, q2.z, q2.w, q3.x, q3.y, q3.z, q3.w};
                    float C[3];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        float acc = 0.0f;
#pragma unroll
                        for (int i = 0; i < kXN; ++i) acc = fmaf(wx5[sl][i], r[i * 3 + c], acc);
                        C[c] = acc;
                    }
                    gs[sl] = parzen_dw0(tA[sl]) * fmaf(fmaf(C[0], m1[sl], C[1]), m1[sl], C[2]);
                } else {
                    const float *r0 = rowt + s * NE, *r1 = r0 + NE;     // bins k_A and k_A + 1
                    const float4 p0 = *reinterpret_cast<const float4 *>(r0);
                    const float4 p1 = *reinterpret_cast<const float4 *>(r1);
                    const float e0[kXN] = {p0.x, p0.y, p0.z, p0.w, r0[4]};
                    const float e1[kXN] = {p1.x, p1.y, p1.z, p1.w, r1[4]};
                    const float k21 = (float)(2 * kB[sl] + 1);
                    float acc = 0.0f;
#pragma unroll
                    for (int i = 0; i < kXN; ++i) {
                        const float t = k21 * arow[i] - a0[sl] * e0[i] - a1[sl] * e1[i];
                        acc = fmaf(wx5[sl][i], t, acc);
                    }
                    gs[sl] = -parzen_dw0(tB[sl]) * acc;                   // d m1 / d s_B = -d w0 / d s
                }
            }
            wave_sync();                                             // the next chunk or q reuses the tables
        }
        }

        if (DISP == 2) {                                             // the fixed image's dD/ds_F
            float *out = args.p[it.prob].grad;
#pragma unroll
            for (int sl = 0; sl < kSlots; ++sl)
                if (pend[sl]) out[rowb + xs + sl * kWave + lane] = gs[sl];
            cur = nxt;
            continue;
        }
        // q = dD/ds * dM/dy * dy/dT  (eq 16): a dense field's gradient is q itself
        if (DISP == 1) {
            float *out = args.p[it.prob].grad;
#pragma unroll
            for (int sl = 0; sl < kSlots; ++sl)
                if (pend[sl]) {
                    const size_t vi = rowb + xs + sl * kWave + lane;
#pragma unroll
                    for (int e = 0; e < 3; ++e) out[e * nvox + vi] = gs[sl] * cur.dm[sl][e] * ratio[e];
                }
            cur = nxt;
            continue;
        }
        // ... then the scatter to the control points (eq 17), first contracted
        // over the z-nodes into the wave's group (flushed when y or the FFD
        // z-cell changes)
        const float fu = (float)cur.uf;
        float byv[4], bzv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            byv[j] = bcast(fu, j);
            bzv[j] = bcast(fu, 4 + j);
        }
        const int py = bcast(cur.c, 0), pz = bcast(cur.c, 1);
        if (gpz >= 0 && (y != gyr || pz != gpz)) {
            flush();
            gpz = -1;
        }
        if (gpz < 0) {
            gyr = y;
            gpy = py;
            gpz = pz;
#pragma unroll
            for (int b = 0; b < 4; ++b) gby[b] = byv[b];
#pragma unroll
            for (int sl = 0; sl < kSlots; ++sl)
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int e = 0; e < 3; ++e) Q[sl][c][e] = 0.0f;
        }
#pragma unroll
        for (int sl = 0; sl < kSlots; ++sl)
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                const float q = gs[sl] * cur.dm[sl][e] * ratio[e];
#pragma unroll
                for (int c = 0; c < 4; ++c) Q[sl][c][e] = fmaf(bzv[c], q, Q[sl][c][e]);
            }
        cur = nxt;
    }
    if (DISP != 0) return;
    if (gpz >= 0) flush();
    __syncthreads();
    // the item's node block to the global accumulators, one (gz, gy) row of
    // nodes per wave at a time
    const size_t ncell = (size_t)g.nc[0] * g.nc[1] * g.nc[2];
    for (int r = wave; r < it.gny * it.gnz; r += nwaves) {
        const int gy = r % it.gny, gz = r / it.gny;
        const size_t node0 = ((size_t)(gz + it.gz0) * g.nc[1] + (gy + it.gy0)) * g.nc[0] + it.gx0;
        const double *src = G + (size_t)r * it.gnx * 3;
        for (int t = lane; t < it.gnx * 3; t += kWave) {
            const double val = src[t];
            if (val != 0.0) {
                const int gx = t / 3, e = t - 3 * gx;
                if (check_ok(node0 + gx < ncell, kChkGrad)) unsafeAtomicAdd(&grad[e * ncell + node0 + gx], val);
            }
        }
    }
}
hipError_t launch_grad(const Geom *geoms, int fdt, int role, int dense, const WorkItem *items, int nitems,
                       const BatchArgs &args, unsigned char *ws, size_t lds_bytes, hipStream_t s, int bw)
{
    if (nitems <= 0) return hipSuccess;
#define SRWCR_GRAD(F, R, D)                                                                                     \
    if (fdt == F && role == R && dense == D) {                                                                  \
        if (bw == 5)                                                                                            \
            hipLaunchKernelGGL((k_grad<F, R, D, 5>), dim3(nitems), dim3(kGradThreads), lds_bytes, s, geoms, items,   \
                               args, ws);                                                                       \
        else                                                                                                    \
            hipLaunchKernelGGL((k_grad<F, R, D, 4>), dim3(nitems), dim3(kGradThreads), lds_bytes, s, geoms, items,   \
                               args, ws);                                                                       \
    }
    SRWCR_GRAD(0, 0, 0) SRWCR_GRAD(0, 0, 1) SRWCR_GRAD(0, 1, 0) SRWCR_GRAD(0, 1, 1)
    SRWCR_GRAD(1, 0, 0) SRWCR_GRAD(1, 0, 1) SRWCR_GRAD(1, 1, 0) SRWCR_GRAD(1, 1, 1)
    SRWCR_GRAD(2, 0, 0) SRWCR_GRAD(2, 0, 1) SRWCR_GRAD(2, 1, 0) SRWCR_GRAD(2, 1, 1)
    SRWCR_GRAD(0, 2, 0) SRWCR_GRAD(0, 2, 1)      // per-voxel dD/ds_M: the fixed image is not read
    SRWCR_GRAD(0, 0, 2) SRWCR_GRAD(0, 1, 2) SRWCR_GRAD(1, 0, 2) SRWCR_GRAD(1, 1, 2)
    SRWCR_GRAD(2, 0, 2) SRWCR_GRAD(2, 1, 2)
#undef SRWCR_GRAD
    return hipGetLastError();
}

// The largest dynamic LDS of the value and gradient kernels is raised to the
// device limit once per device, outside any stream capture.
hipError_t prepare_kernels()
{
    static bool done[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 64 && done[dev]) return hipSuccess;
    int max_lds = 0;
    e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    const size_t b = (size_t)max_lds;
#define SRWCR_SET(W)                                                                \
    if (e == hipSuccess) e = set_lds(k_value<0, W>, b);                             \
    if (e == hipSuccess) e = set_lds(k_value<1, W>, b);                             \
    if (e == hipSuccess) e = set_lds(k_value<2, W>, b);
    SRWCR_SET(4) SRWCR_SET(5)
#undef SRWCR_SET
#define SRWCR_SET(A, B)                                                             \
    if (e == hipSuccess) e = set_lds(k_grad<0, A, B, 4>, b);                        \
    if (e == hipSuccess) e = set_lds(k_grad<1, A, B, 4>, b);                        \
    if (e == hipSuccess) e = set_lds(k_grad<2, A, B, 4>, b);                        \
    if (e == hipSuccess) e = set_lds(k_grad<0, A, B, 5>, b);                        \
    if (e == hipSuccess) e = set_lds(k_grad<1, A, B, 5>, b);                        \
    if (e == hipSuccess) e = set_lds(k_grad<2, A, B, 5>, b);                        \
    if (e == hipSuccess) e = set_lds(k_prep<0, A, B>, b);                           \
    if (e == hipSuccess) e = set_lds(k_prep<1, A, B>, b);                           \
    if (e == hipSuccess) e = set_lds(k_prep<2, A, B>, b);
    SRWCR_SET(0, 0) SRWCR_SET(0, 1) SRWCR_SET(1, 0) SRWCR_SET(1, 1)
#undef SRWCR_SET
    if (e == hipSuccess) e = set_lds(k_grad<0, 2, 0, 4>, b);
    if (e == hipSuccess) e = set_lds(k_grad<0, 2, 1, 4>, b);
    if (e == hipSuccess) e = set_lds(k_grad<0, 2, 0, 5>, b);
    if (e == hipSuccess) e = set_lds(k_grad<0, 2, 1, 5>, b);
#define SRWCR_SET(F)                                                                \
    if (e == hipSuccess) e = set_lds(k_grad<F, 0, 2, 4>, b);                        \
    if (e == hipSuccess) e = set_lds(k_grad<F, 1, 2, 4>, b);                        \
    if (e == hipSuccess) e = set_lds(k_grad<F, 0, 2, 5>, b);                        \
    if (e == hipSuccess) e = set_lds(k_grad<F, 1, 2, 5>, b);
    SRWCR_SET(0) SRWCR_SET(1) SRWCR_SET(2)
#undef SRWCR_SET
    if (e == hipSuccess && dev < 64) done[dev] = true;
    return e;
}

// FP64 accumulators to the caller's FP32 gradient; blockIdx.y = problem.
__global__ void k_grad_out(const Geom *__restrict__ geoms, BatchArgs args, unsigned char *ws)
{
    const Geom &g = geoms[blockIdx.y];
    const double *__restrict__ grad = reinterpret_cast<const double *>(ws + g.ws.grad);
    float *__restrict__ out = args.p[blockIdx.y].grad;
    const size_t n = 3 * (size_t)g.nc[0] * g.nc[1] * g.nc[2];
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = (float)grad[i];
}

hipError_t launch_grad_out(const Geom *geoms, int nprob, size_t max_params, const BatchArgs &args, unsigned char *ws,
                           hipStream_t s)
{
    const int blocks = (int)std::min<size_t>((max_params + 255) / 256, 1024);
    hipLaunchKernelGGL(k_grad_out, dim3(blocks, nprob), dim3(256), 0, s, geoms, args, ws);
    return hipGetLastError();
}

// ----------------------------------------------------------------- RaPTOR
// The patch-based correlation ratio of eqs (6, 13, 14): boxcar patches, a
// linear window h(t) = max(0, 1 - |t|) on the A-bins and plain frequency
// moments of B.  Per patch r the accumulation pass gathers
//   P_a = sum h(a - A),  S1_a = sum h(a - A) B',  sum B',  sum B'^2
// over its voxels, with B' = B - c_r and c_r the value of B at the patch's
// first voxel (eq 13 is unchanged by the shift; it keeps the FP32 products
// and the cancellation in E[B^2] - sum p mu^2 small).  One workgroup takes a
// run of the patch's voxels; its waves take 64 voxels at a time, form the
// wave-uniform set of A-bins they touch (two per voxel) and add, per bin,
// the wave's sums of h and h B' to FP64 LDS slots; the slots are merged into
// the patch's global sums once per workgroup.

constexpr int kRaptorThreads = 256;

// Wave-uniform FP32 sum: butterfly within each 16-lane row (DPP), then the
// four row sums through readlane.  Must run with all lanes active.
__device__ __forceinline__ float wave_sum_f(float v)
{
    v += dpp<0xB1>(v);     // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);     // quad_perm [2,3,0,1]
    v += dpp<0x124>(v);    // row_ror:4
    v += dpp<0x128>(v);    // row_ror:8
    return (bcast(v, 0) + bcast(v, 16)) + (bcast(v, 32) + bcast(v, 48));
}

// B of one voxel as an integer part and a fraction: the moving sample's bin
// and in-bin position (moving is B), or the fixed value (moving is A).
template <int FDT, int ROLE>
__device__ __forceinline__ void raptor_b(const PrepKT *__restrict__ kt, const void *__restrict__ fixed, size_t vi,
                                         int &kb, float &tb)
{
    if constexpr (ROLE == 0) {
        kb = 0;
        tb = ld_int<FDT>(fixed, vi);
    } else {
        const PrepKT pk = kt[vi];
        kb = pk.k;
        tb = pk.t;
    }
}

// A lane's position inside a patch box (x fastest), advanced by a fixed
// stride without divisions: the stride is split once as sx + nx (sy + ny sz)
// with sx < nx and sy < ny, so each step carries at most once per axis.
struct PatchWalk {
    int x, y, z, sx, sy, sz;

    __device__ __forceinline__ void init(const RaptorPatch &pt, int v, int stride)
    {
        x = v % pt.nx;
        const int yz = v / pt.nx;
        y = yz % pt.ny;
        z = yz / pt.ny;
        sx = stride % pt.nx;
        const int r = stride / pt.nx;
        sy = r % pt.ny;
        sz = r / pt.ny;
    }
    __device__ __forceinline__ void step(const RaptorPatch &pt)
    {
        x += sx;
        y += sy;
        z += sz;
        if (x >= pt.nx) {
            x -= pt.nx;
            ++y;
        }
        if (y >= pt.ny) {
            y -= pt.ny;
            ++z;
        }
    }
    __device__ __forceinline__ size_t index(const RaptorPatch &pt, int nfx, int nfy) const
    {
        return ((size_t)(pt.z0 + z) * nfy + (pt.y0 + y)) * nfx + (pt.x0 + x);
    }
};

// One voxel's A-bin k, in-bin position t (k = min(floor(A), L - 1)) and
// shifted B' = (kb - ck) + (tb - ct).
template <int FDT, int ROLE>
__device__ __forceinline__ void raptor_ab(const PrepKT *__restrict__ kt, const void *__restrict__ fixed, size_t vi,
                                          int L, int ck, float ct, int &kA, float &tA, float &Bs)
{
    int kb;
    float tb;
    raptor_b<FDT, ROLE>(kt, fixed, vi, kb, tb);
    if constexpr (ROLE == 0) {
        const PrepKT pk = kt[vi];
        kA = pk.k;
        tA = pk.t;
    } else {
        const float sf = ld_int<FDT>(fixed, vi);
        kA = max(min((int)sf, L - 1), 0);                            // in range for any input
        tA = sf - (float)kA;
    }
    Bs = (float)(kb - ck) + (tb - ct);
}

// The patch sums.  Each lane keeps FP32 sums for a window of kRWin
// consecutive A-bins placed around the bin of the piece's first voxel; a
// voxel whose two taps both fall in the window only updates its registers.
// The others (a patch across a tissue boundary) take the exact per-bin path:
// the wave-uniform set of their bins, one cross-lane sum of h and h B' per
// bin, added to FP64 LDS slots.  The window sums are reduced across the wave
// once per piece.
constexpr int kRWin = 8;

template <int FDT, int ROLE>
__global__ void __launch_bounds__(kRaptorThreads)
k_raptor_acc(const Geom *__restrict__ geoms, RaptorArgs ra, BatchArgs args, const unsigned char *ws)
{
    extern __shared__ double rsh[];                                   // [2 nb + 2]
    const Geom &g = geoms[0];
    const RaptorPiece pc = ra.pieces[blockIdx.x];
    const RaptorPatch pt = ra.patches[pc.patch];
    const int nb = g.nb, L = nb - 1, nst = 2 * nb + 3;
    const PrepKT *__restrict__ kt = reinterpret_cast<const PrepKT *>(ws + g.ws.kt);
    const void *__restrict__ fixed = args.p[0].fixed;
    const int nfx = g.nf[0], nfy = g.nf[1];
    for (int i = threadIdx.x; i < 2 * nb + 2; i += blockDim.x) rsh[i] = 0.0;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    int ck, wb;
    float ct;
    {
        PatchWalk w0;
        w0.init(pt, 0, 1);
        const size_t v0 = w0.index(pt, nfx, nfy);
        raptor_b<FDT, ROLE>(kt, fixed, v0, ck, ct);
        int k0;
        float t0, b0;
        raptor_ab<FDT, ROLE>(kt, fixed, v0, L, ck, ct, k0, t0, b0);
        wb = max(0, min(k0 - kRWin / 2 + 1, nb - kRWin));              // window bins wb .. wb + kRWin - 1
    }
    __syncthreads();
    const int end = pc.start + pc.count;
    float accP[kRWin], accS[kRWin];
#pragma unroll
    for (int j = 0; j < kRWin; ++j) accP[j] = accS[j] = 0.0f;
    double sb = 0.0, sb2 = 0.0;
    PatchWalk pw;
    pw.init(pt, min(pc.start + wave * kWave + lane, pt.n - 1), nwaves * kWave);
    for (int base = pc.start + wave * kWave; base < end; base += nwaves * kWave, pw.step(pt)) {
        const bool act = base + lane < end;
        int kA = 0;
        float tA = 0.0f, Bs = 0.0f;
        if (act) raptor_ab<FDT, ROLE>(kt, fixed, pw.index(pt, nfx, nfy), L, ck, ct, kA, tA, Bs);
        if (act) {
            sb += (double)Bs;
            sb2 += (double)Bs * (double)Bs;
        }
        const int j0 = kA - wb;
        const bool inw = act && j0 >= 0 && j0 <= kRWin - 2;
        const float h0 = 1.0f - tA, h1 = tA;
        const float wh0 = inw ? h0 : 0.0f, wh1 = inw ? h1 : 0.0f;
#pragma unroll
        for (int j = 0; j < kRWin; ++j) {
            const float w = j == j0 ? wh0 : (j == j0 + 1 ? wh1 : 0.0f);
            accP[j] += w;
            accS[j] = fmaf(w, Bs, accS[j]);
        }
        const unsigned long long mine = act && !inw ? 3ull << kA : 0ull;   // k_A <= L - 1 <= 62
        unsigned long long bins = (unsigned long long)wave_or_dpp((unsigned)(mine >> 32)) << 32 |
                                  wave_or_dpp((unsigned)mine);
        while (bins) {
            const int a = __builtin_ctzll(bins);
            bins &= bins - 1ull;
            const float w = inw || !act ? 0.0f : (kA == a ? h0 : (kA + 1 == a ? h1 : 0.0f));
            const float p = wave_sum_f(w), q = wave_sum_f(w * Bs);
            if (lane == 0) {
                atomicAdd(&rsh[a], (double)p);
                atomicAdd(&rsh[nb + a], (double)q);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kRWin; ++j) {
        const float p = wave_sum_f(accP[j]), q = wave_sum_f(accS[j]);
        if (lane == 0 && wb + j <= L && (p != 0.0f || q != 0.0f)) {
            atomicAdd(&rsh[wb + j], (double)p);
            atomicAdd(&rsh[nb + wb + j], (double)q);
        }
    }
    sb = wave_sum_d(sb);
    sb2 = wave_sum_d(sb2);
    if (lane == 0) {
        atomicAdd(&rsh[2 * nb], sb);
        atomicAdd(&rsh[2 * nb + 1], sb2);
    }
    __syncthreads();
    double *st = ra.stats + (size_t)pc.patch * nst;
    for (int i = threadIdx.x; i < 2 * nb + 2; i += blockDim.x)
        if (rsh[i] != 0.0) unsafeAtomicAdd(&st[i], rsh[i]);
    if (threadIdx.x == 0) st[2 * nb + 2] = (double)ck + (double)ct;   // c_r (every piece writes the same value)
}

// One wave per patch (lane = A-bin): the patch term
//   T_r = (E[B'^2] - sum_a p_r(a) mu'_r(a)^2) / sigma_r^2,
// mu'_r(a) = S1_a / P_a, and the tables of the derivative pass.  RaPTOR
// itself is summed by k_raptor_value in the next launch, which sees every
// T_r without a device-scope fence per wave (each such fence writes back the
// compute unit's L2 slice, and 1700 of them cost more than the sums).
__global__ void __launch_bounds__(kRaptorThreads) k_raptor_finalize(const Geom *__restrict__ geoms, RaptorArgs ra)
{
    const Geom &g = geoms[0];
    const int lane = threadIdx.x & (kWave - 1);
    const int p = blockIdx.x * (kRaptorThreads / kWave) + (threadIdx.x >> 6);
    if (p >= ra.npatch) return;
    const int nb = g.nb, nst = 2 * nb + 3;
    const double *st = ra.stats + (size_t)p * nst;
    const double N = (double)ra.patches[p].n;
    double P = 0.0, S = 0.0;
    if (lane < nb) {
        P = st[lane];
        S = st[nb + lane];
    }
    const bool filled = P > 0.0;
    const double mu = filled ? S / P : 0.0;
    double T = 0.0, inv_nvar = 0.0, E1 = 0.0, c = 0.0;
    const double Q = wave_sum_d(filled ? S * mu : 0.0);               // N sum_a p mu'^2
    if (N > 0.0) {
        c = st[2 * nb + 2];
        E1 = st[2 * nb] / N;
        const double E2s = st[2 * nb + 1] / N, var = E2s - E1 * E1;
        const double E2 = E2s + c * (2.0 * E1 + c);                   // E[B^2] of the unshifted B
        // a patch whose B is constant to 0.3 % (sigma^2 <= 1e-5 E[B^2]) is skipped
        if (var > 1e-5 * E2) {
            T = (E2s - Q / N) / var;
            inv_nvar = 1.0 / (N * var);
        }
    }
    if (lane < nb) ra.mu[(size_t)p * nb + lane] = make_float2((float)mu, filled ? 1.0f : 0.0f);
    if (lane == 0) {
        ra.scal[p] = make_float4((float)inv_nvar, (float)T, (float)E1, (float)c);
        ra.tval[p] = T;
    }
}

// RaPTOR = (1 / N_p) sum_r T_r, summed in patch order (lane-strided partial
// sums, then the fixed wave reduction), one wave.
__global__ void __launch_bounds__(kWave) k_raptor_value(RaptorArgs ra)
{
    const int lane = threadIdx.x;
    double part = 0.0;
    for (int q0 = lane; q0 < ra.npatch; q0 += 8 * kWave) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = q0 + u * kWave < ra.npatch ? ra.tval[q0 + u * kWave] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) part += x[u];
    }
    const double R = wave_sum_d(part);
    if (lane == 0) *ra.value = R / (double)ra.npatch;
}

// Derivative pass: per patch voxel, dT_r/ds_M (the exact derivative of eq 13
// with the one-sided window derivative), added over the patches that hold
// the voxel into rds = dRaPTOR/ds_M.
//   moving is A: dT/dA = ((B - mu(k+1))^2 - (B - mu(k))^2) / (N sigma^2),
//   moving is B: dT/dB = 2 (B - sum_a h mu(a) - T (B - E1)) / (N sigma^2),
// an empty bin's mu taken as the voxel's own B.
template <int FDT, int ROLE>
__global__ void __launch_bounds__(kRaptorThreads)
k_raptor_ds(const Geom *__restrict__ geoms, RaptorArgs ra, BatchArgs args, const unsigned char *ws)
{
    extern __shared__ float2 rmu[];                                   // [nb]
    const Geom &g = geoms[0];
    const RaptorPiece pc = ra.pieces[blockIdx.x];
    const float4 sc = ra.scal[pc.patch];
    if (sc.x == 0.0f) return;                                         // skipped patch: no derivative
    const RaptorPatch pt = ra.patches[pc.patch];
    const int nb = g.nb, L = nb - 1;
    const PrepKT *__restrict__ kt = reinterpret_cast<const PrepKT *>(ws + g.ws.kt);
    const void *__restrict__ fixed = args.p[0].fixed;
    const int nfx = g.nf[0], nfy = g.nf[1];
    for (int i = threadIdx.x; i < nb; i += blockDim.x) rmu[i] = ra.mu[(size_t)pc.patch * nb + i];
    int ck;
    float ct;
    raptor_b<FDT, ROLE>(kt, fixed, ((size_t)pt.z0 * nfy + pt.y0) * nfx + pt.x0, ck, ct);
    __syncthreads();
    const float scale = sc.x / (float)ra.npatch;
    const int end = pc.start + pc.count;
    PatchWalk pw;
    pw.init(pt, min(pc.start + (int)threadIdx.x, pt.n - 1), blockDim.x);
    for (int v = pc.start + threadIdx.x; v < end; v += blockDim.x, pw.step(pt)) {
        const size_t vi = pw.index(pt, nfx, nfy);
        int kA;
        float tA, Bs;
        raptor_ab<FDT, ROLE>(kt, fixed, vi, L, ck, ct, kA, tA, Bs);
        const float2 m0 = rmu[kA], m1 = rmu[kA + 1];
        float d;
        if constexpr (ROLE == 0) {
            const float d0 = m0.y != 0.0f ? Bs - m0.x : 0.0f, d1 = m1.y != 0.0f ? Bs - m1.x : 0.0f;
            d = (d1 - d0) * (d1 + d0);
        } else {
            const float hm = (1.0f - tA) * (m0.y != 0.0f ? m0.x : Bs) + tA * (m1.y != 0.0f ? m1.x : Bs);
            d = 2.0f * (Bs - hm - sc.y * (Bs - sc.z));
        }
        unsafeAtomicAdd(&ra.rds[vi], scale * d);
    }
}

hipError_t launch_raptor_acc(const Geom *geoms, int fdt, int role, const RaptorArgs &ra, const BatchArgs &args,
                             const unsigned char *ws, hipStream_t s)
{
    if (ra.npieces <= 0) return hipSuccess;
    const size_t lds = (size_t)(2 * kMaxBins + 2) * sizeof(double);
#define RAPTOR_ACC(F, R)                                                                                       \
    if (fdt == F && role == R)                                                                                 \
        hipLaunchKernelGGL((k_raptor_acc<F, R>), dim3(ra.npieces), dim3(kRaptorThreads), lds, s, geoms, ra, args, ws);
    RAPTOR_ACC(0, 0) RAPTOR_ACC(0, 1) RAPTOR_ACC(1, 0) RAPTOR_ACC(1, 1) RAPTOR_ACC(2, 0) RAPTOR_ACC(2, 1)
#undef RAPTOR_ACC
    return hipGetLastError();
}

hipError_t launch_raptor_finalize(const Geom *geoms, const RaptorArgs &ra, hipStream_t s)
{
    const int per = kRaptorThreads / kWave;
    hipLaunchKernelGGL(k_raptor_finalize, dim3((ra.npatch + per - 1) / per), dim3(kRaptorThreads), 0, s, geoms, ra);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_raptor_value, dim3(1), dim3(kWave), 0, s, ra);
    return hipGetLastError();
}

hipError_t launch_raptor_ds(const Geom *geoms, int fdt, int role, const RaptorArgs &ra, const BatchArgs &args,
                            const unsigned char *ws, hipStream_t s)
{
    if (ra.npieces <= 0) return hipSuccess;
    const size_t lds = (size_t)kMaxBins * sizeof(float2);
#define RAPTOR_DS(F, R)                                                                                        \
    if (fdt == F && role == R)                                                                                 \
        hipLaunchKernelGGL((k_raptor_ds<F, R>), dim3(ra.npieces), dim3(kRaptorThreads), lds, s, geoms, ra, args, ws);
    RAPTOR_DS(0, 0) RAPTOR_DS(0, 1) RAPTOR_DS(1, 0) RAPTOR_DS(1, 1) RAPTOR_DS(2, 0) RAPTOR_DS(2, 1)
#undef RAPTOR_DS
    return hipGetLastError();
}

// ------------------------------------------------------------- ffd_warp
template <int MDT>
__global__ void __launch_bounds__(256) k_warp(Geom g, const void *__restrict__ moving, const float *__restrict__ ffd,
                                              float *__restrict__ out)
{
    __shared__ double c1s[4][3 * kMaxNodeSeg];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nseg = (g.nf[0] + kWave - 1) / kWave;
    const long unit = (long)blockIdx.x * 4 + wave;
    const long nunits = (long)nseg * g.nf[1] * g.nf[2];
    if (unit >= nunits) return;                          // wave-uniform exit
    const int seg = (int)(unit % nseg);
    const long row = unit / nseg;
    const int y = (int)(row % g.nf[1]), z = (int)(row / g.nf[1]);
    const int xs = seg * kWave, xe = min(xs + kWave, g.nf[0]);
    const int x = xs + lane;
    const bool valid = x < xe;
    const int xc = valid ? x : xe - 1;
    double u[3];
    ffd_row(g, ffd, xs, xe, y, z, xc, c1s[wave], lane, u);
    double v = sample_moving<MDT>(g, moving, xc, y, z, u, nullptr);
    v = fmin(fmax(v, 0.0), (double)(g.nb - 1));
    if (valid) out[((size_t)z * g.nf[1] + y) * g.nf[0] + x] = (float)v;
}

hipError_t launch_warp(const Geom &g, const void *moving, const float *ffd, float *out, hipStream_t s)
{
    const long nseg = (g.nf[0] + kWave - 1) / kWave;
    const long nunits = nseg * g.nf[1] * g.nf[2];
    const int blocks = (int)((nunits + 3) / 4);
    if (g.mdt == 0) hipLaunchKernelGGL(k_warp<0>, dim3(blocks), dim3(256), 0, s, g, moving, ffd, out);
    else if (g.mdt == 1) hipLaunchKernelGGL(k_warp<1>, dim3(blocks), dim3(256), 0, s, g, moving, ffd, out);
    else hipLaunchKernelGGL(k_warp<2>, dim3(blocks), dim3(256), 0, s, g, moving, ffd, out);
    return hipGetLastError();
}

// ------------------------------------------------------ sample read-out
__global__ void k_unpack_samples(const PrepKT *__restrict__ kt, size_t n, int32_t *__restrict__ bin,
                                 float *__restrict__ frac)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const PrepKT p = kt[i];
        bin[i] = p.k;
        frac[i] = p.t;
    }
}

hipError_t launch_unpack_samples(const PrepKT *kt, size_t n, int32_t *bin, float *frac, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_unpack_samples, dim3(blocks), dim3(256), 0, s, kt, n, bin, frac);
    return hipGetLastError();
}

// ------------------------------------------------------- pyramid level
// Next-coarser level of the registration pyramid: Gaussian smoothing with
// sigma = 1 voxel (taps -3..3, edges clamped) sampled at every other voxel,
// corner aligned: out(X) = (G * in)(2 X).
__global__ void __launch_bounds__(256) k_downsample(const float *__restrict__ in, int nx, int ny, int nz,
                                                    float *__restrict__ out, int ox, int oy, int oz)
{
    const long n = (long)ox * oy * oz;
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int X = (int)(i % ox), Y = (int)((i / ox) % oy), Z = (int)(i / ((long)ox * oy));
    float w[7];
    float wsum = 0.0f;
#pragma unroll
    for (int d = -3; d <= 3; ++d) {
        w[d + 3] = expf(-0.5f * (float)(d * d));
        wsum += w[d + 3];
    }
    float acc = 0.0f;
    for (int dz = -3; dz <= 3; ++dz) {
        const int z = min(max(2 * Z + dz, 0), nz - 1);
        for (int dy = -3; dy <= 3; ++dy) {
            const int y = min(max(2 * Y + dy, 0), ny - 1);
            const float wzy = w[dz + 3] * w[dy + 3];
            const float *row = in + ((size_t)z * ny + y) * nx;
            float r = 0.0f;
#pragma unroll
            for (int dx = -3; dx <= 3; ++dx) r = fmaf(w[dx + 3], row[min(max(2 * X + dx, 0), nx - 1)], r);
            acc = fmaf(wzy, r, acc);
        }
    }
    out[i] = acc / (wsum * wsum * wsum);
}

hipError_t launch_downsample(const float *in, int nx, int ny, int nz, float *out, int ox, int oy, int oz,
                             hipStream_t s)
{
    const long n = (long)ox * oy * oz;
    hipLaunchKernelGGL(k_downsample, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, nx, ny, nz, out, ox,
                       oy, oz);
    return hipGetLastError();
}

}  // namespace srwcr

extern "C" int srwcr_debug_check_flags(int32_t *flags, int32_t reset)
{
#ifdef SRWCR_CHECK
    if (!flags) return srwcr::report_error(SRWCR_E_INVALID_ARG, "flags is NULL");
    unsigned v = 0;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpyFromSymbol(&v, HIP_SYMBOL(srwcr::g_check_flags), sizeof v);
    if (e == hipSuccess && reset) {
        const unsigned zero = 0;
        e = hipMemcpyToSymbol(HIP_SYMBOL(srwcr::g_check_flags), &zero, sizeof zero);
    }
    if (e != hipSuccess) return srwcr::report_error(SRWCR_E_HIP, "bounds-check flags: %s", hipGetErrorString(e));
    *flags = (int32_t)v;
    return SRWCR_OK;
#else
    (void)flags;
    (void)reset;
    return srwcr::report_error(SRWCR_E_UNSUPPORTED, "this library was built without SRWCR_CHECK");
#endif
}

