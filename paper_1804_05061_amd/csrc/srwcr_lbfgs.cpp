// srwcr_lbfgs.cpp -- multi-resolution L-BFGS registration driver (Sec. II-F).
//
// Cost (eq 1): C = D + w_p C_p, D = SRWCR evaluated with its gradient by
// srwcr_grad on the GPU, C_p the bending energy of the FFD evaluated on the
// control lattice (host, FP64).  The optimiser is a limited-memory BFGS with
// m corrections (two-loop recursion, Nocedal & Wright, Alg. 7.4) and a
// backtracking line search that enforces the Armijo and curvature (weak
// Wolfe) conditions inside a bracket: it halves the step on an Armijo failure
// and grows it by 2.1 on a curvature failure until both ends of the bracket
// are known, then bisects the bracket, so every trial shrinks it.  A level
// stops when C has been stable over `stall_window` iterations, after
// max_iter iterations, or when no step along the quasi-Newton direction nor
// along -g lowers C (convergence at the FP32 resolution of the FFD the cost
// is evaluated on).  Levels are Gaussian pyramids of the normalised
// volumes; the displacement found on a level is carried to the next finer one
// by doubling it and refining the control lattice by cubic B-spline
// subdivision, which represents the coarse field exactly.  A caller's start
// is carried down to the coarsest level by keeping every second control node
// and halving it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <functional>
#include <string>
#include <vector>

#include "srwcr.h"
#include "srwcr_internal.h"

using namespace srwcr;

namespace {

struct Grid3 {
    int n[3];
    size_t count() const { return (size_t)n[0] * n[1] * n[2]; }
};

// ---------------------------------------------------------- bending energy
// C_p = sum over control-node positions inside the image of
// sum_e [u_xx^2 + u_yy^2 + u_zz^2 + 2 (u_xy^2 + u_xz^2 + u_yz^2)], with the
// derivatives of the cubic B-spline at a node: value weights (1, 4, 1) / 6,
// first derivative (-1, 0, 1) / (2 delta), second (1, -2, 1) / delta^2 over
// the nodes i - 1, i, i + 1.
double bending_energy(const std::vector<double> &c, const int nc[3], const int nf[3], const int delta[3],
                      std::vector<double> *grad)
{
    const double V[3] = {1.0 / 6, 4.0 / 6, 1.0 / 6};
    double D1[3][3], D2[3][3];
    for (int e = 0; e < 3; ++e) {
        D1[e][0] = -0.5 / delta[e]; D1[e][1] = 0.0; D1[e][2] = 0.5 / delta[e];
        const double d2 = 1.0 / ((double)delta[e] * delta[e]);
        D2[e][0] = d2; D2[e][1] = -2.0 * d2; D2[e][2] = d2;
    }
    // derivative types: (order along x, y, z) and multiplicity
    const int types[6][3] = {{2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
    const double mult[6] = {1, 1, 1, 2, 2, 2};
    const size_t ncell = (size_t)nc[0] * nc[1] * nc[2];
    int np[3];
    for (int e = 0; e < 3; ++e) np[e] = (nf[e] - 1) / delta[e] + 1;     // paper nodes 0 .. floor((N-1)/delta)
    if (grad) grad->assign(3 * ncell, 0.0);
    double E = 0.0;
    for (int pz = 0; pz < np[2]; ++pz)
        for (int py = 0; py < np[1]; ++py)
            for (int px = 0; px < np[0]; ++px) {
                const int s[3] = {px + 1, py + 1, pz + 1};               // stored index of the node
                for (int t = 0; t < 6; ++t) {
                    const double *w[3];
                    for (int e = 0; e < 3; ++e)
                        w[e] = types[t][e] == 2 ? D2[e] : (types[t][e] == 1 ? D1[e] : V);
                    for (int comp = 0; comp < 3; ++comp) {
                        double val = 0.0;
                        for (int c2 = 0; c2 < 3; ++c2)
                            for (int b = 0; b < 3; ++b)
                                for (int a = 0; a < 3; ++a) {
                                    const size_t idx = ((size_t)(s[2] - 1 + c2) * nc[1] + (s[1] - 1 + b)) * nc[0] +
                                                       (s[0] - 1 + a);
                                    val += w[0][a] * w[1][b] * w[2][c2] * c[comp * ncell + idx];
                                }
                        E += mult[t] * val * val;
                        if (grad) {
                            const double gv = 2.0 * mult[t] * val;
                            for (int c2 = 0; c2 < 3; ++c2)
                                for (int b = 0; b < 3; ++b)
                                    for (int a = 0; a < 3; ++a) {
                                        const size_t idx = ((size_t)(s[2] - 1 + c2) * nc[1] + (s[1] - 1 + b)) * nc[0] +
                                                           (s[0] - 1 + a);
                                        (*grad)[comp * ncell + idx] += gv * w[0][a] * w[1][b] * w[2][c2];
                                    }
                        }
                    }
                }
            }
    return E;
}

// ------------------------------------------------- lattice refinement
// Coarse level (voxel size 2) -> fine level (voxel size 1): u_f(x) = 2 u_c(x / 2).
// With paper node indices (stored = paper + 1) the subdivision of a cubic
// B-spline gives fine node 2i = (c[i-1] + 6 c[i] + c[i+1]) / 8 and fine node
// 2i+1 = (c[i] + c[i+1]) / 2; nodes outside the coarse lattice count as 0.
std::vector<double> refine(const std::vector<double> &cc, const int ncc[3], const int ncf[3])
{
    // separable: refine x, then y, then z (each component independently)
    const size_t cc_cells = (size_t)ncc[0] * ncc[1] * ncc[2];
    auto coarse_at = [](const std::vector<double> &a, int i, int n) { return (i >= 0 && i < n) ? a[i] : 0.0; };
    std::vector<double> out(3 * (size_t)ncf[0] * ncf[1] * ncf[2]);
    for (int comp = 0; comp < 3; ++comp) {
        // stage x: [ncc z][ncc y][ncf x]
        std::vector<double> sx((size_t)ncc[2] * ncc[1] * ncf[0]);
        std::vector<double> line;
        for (int z = 0; z < ncc[2]; ++z)
            for (int y = 0; y < ncc[1]; ++y) {
                line.assign(ncc[0], 0.0);
                for (int x = 0; x < ncc[0]; ++x)
                    line[x] = cc[comp * cc_cells + ((size_t)z * ncc[1] + y) * ncc[0] + x];
                for (int jf = 0; jf < ncf[0]; ++jf) {
                    const int j = jf - 1;                                  // paper index of the fine node
                    double v;
                    if ((j & 1) == 0) {
                        const int i = j / 2;                              // paper coarse index
                        v = (coarse_at(line, i, ncc[0]) + 6.0 * coarse_at(line, i + 1, ncc[0]) +
                             coarse_at(line, i + 2, ncc[0])) / 8.0;
                    } else {
                        const int i = (j - 1) / 2;
                        v = (coarse_at(line, i + 1, ncc[0]) + coarse_at(line, i + 2, ncc[0])) / 2.0;
                    }
                    sx[((size_t)z * ncc[1] + y) * ncf[0] + jf] = v;
                }
            }
        // stage y: [ncc z][ncf y][ncf x]
        std::vector<double> sy((size_t)ncc[2] * ncf[1] * ncf[0]);
        for (int z = 0; z < ncc[2]; ++z)
            for (int x = 0; x < ncf[0]; ++x) {
                line.assign(ncc[1], 0.0);
                for (int y = 0; y < ncc[1]; ++y) line[y] = sx[((size_t)z * ncc[1] + y) * ncf[0] + x];
                for (int jf = 0; jf < ncf[1]; ++jf) {
                    const int j = jf - 1;
                    double v;
                    if ((j & 1) == 0) {
                        const int i = j / 2;
                        v = (coarse_at(line, i, ncc[1]) + 6.0 * coarse_at(line, i + 1, ncc[1]) +
                             coarse_at(line, i + 2, ncc[1])) / 8.0;
                    } else {
                        const int i = (j - 1) / 2;
                        v = (coarse_at(line, i + 1, ncc[1]) + coarse_at(line, i + 2, ncc[1])) / 2.0;
                    }
                    sy[((size_t)z * ncf[1] + jf) * ncf[0] + x] = v;
                }
            }
        // stage z
        for (int y = 0; y < ncf[1]; ++y)
            for (int x = 0; x < ncf[0]; ++x) {
                line.assign(ncc[2], 0.0);
                for (int z = 0; z < ncc[2]; ++z) line[z] = sy[((size_t)z * ncf[1] + y) * ncf[0] + x];
                for (int jf = 0; jf < ncf[2]; ++jf) {
                    const int j = jf - 1;
                    double v;
                    if ((j & 1) == 0) {
                        const int i = j / 2;
                        v = (coarse_at(line, i, ncc[2]) + 6.0 * coarse_at(line, i + 1, ncc[2]) +
                             coarse_at(line, i + 2, ncc[2])) / 8.0;
                    } else {
                        const int i = (j - 1) / 2;
                        v = (coarse_at(line, i + 1, ncc[2]) + coarse_at(line, i + 2, ncc[2])) / 2.0;
                    }
                    out[comp * (size_t)ncf[0] * ncf[1] * ncf[2] + ((size_t)jf * ncf[1] + y) * ncf[0] + x] = 2.0 * v;
                }
            }
    }
    return out;
}

// Fine level -> coarse level, the start of a registration carried down the
// pyramid: coarse paper node j sits on fine paper node 2 j (stored index
// 2 s - 1 for coarse stored index s, clamped to the fine lattice) and a
// displacement of d fine voxels is d / 2 coarse voxels.  Exact for fields
// that are linear along each axis; an approximation otherwise, which the
// coarse level's optimisation then refines.
std::vector<double> decimate(const std::vector<double> &cf, const int ncf[3], const int ncc[3])
{
    const size_t fcells = (size_t)ncf[0] * ncf[1] * ncf[2], ccells = (size_t)ncc[0] * ncc[1] * ncc[2];
    std::vector<double> out(3 * ccells);
    auto fidx = [](int s, int nf) { return std::min(std::max(2 * s - 1, 0), nf - 1); };
    for (int comp = 0; comp < 3; ++comp)
        for (int z = 0; z < ncc[2]; ++z)
            for (int y = 0; y < ncc[1]; ++y)
                for (int x = 0; x < ncc[0]; ++x) {
                    const size_t fi = ((size_t)fidx(z, ncf[2]) * ncf[1] + fidx(y, ncf[1])) * ncf[0] + fidx(x, ncf[0]);
                    out[comp * ccells + ((size_t)z * ncc[1] + y) * ncc[0] + x] = 0.5 * cf[comp * fcells + fi];
                }
    return out;
}

// ------------------------------------------------------------ one level
struct Level {
    srwcr_problem prob;
    const float *fixed = nullptr, *moving = nullptr;   // device, normalised
    int nc[3];
};

class Evaluator {
  public:
    Evaluator(const Level &lv, double wp, hipStream_t s) : lv_(lv), wp_(wp), s_(s) {}
    ~Evaluator()
    {
        if (plan_) srwcr_plan_destroy(plan_);
        if (ws_) (void)hipFree(ws_);
        if (dffd_) (void)hipFree(dffd_);
        if (dgrad_) (void)hipFree(dgrad_);
        if (dval_) (void)hipFree(dval_);
    }
    int init()
    {
        int st = srwcr_plan_create(&lv_.prob, &plan_);
        if (st) return st;
        n_ = 3 * (size_t)lv_.nc[0] * lv_.nc[1] * lv_.nc[2];
        wsb_ = srwcr_workspace_bytes(plan_);
        if (hipMalloc(&ws_, wsb_) != hipSuccess || hipMalloc(&dffd_, n_ * sizeof(float)) != hipSuccess ||
            hipMalloc(&dgrad_, n_ * sizeof(float)) != hipSuccess || hipMalloc(&dval_, sizeof(double)) != hipSuccess)
            return SRWCR_E_HIP;
        if (hipMemsetAsync(ws_, 0, wsb_, s_) != hipSuccess) return SRWCR_E_HIP;
        hf_.resize(n_);
        hg_.resize(n_);
        return SRWCR_OK;
    }
    size_t size() const { return n_; }
    // f(x) and its gradient; returns a status
    int eval(const std::vector<double> &x, double &f, std::vector<double> &g, double *D_out = nullptr)
    {
        for (size_t i = 0; i < n_; ++i) hf_[i] = (float)x[i];
        if (hipMemcpyAsync(dffd_, hf_.data(), n_ * sizeof(float), hipMemcpyHostToDevice, s_) != hipSuccess)
            return SRWCR_E_HIP;
        int st = srwcr_grad(plan_, lv_.fixed, lv_.moving, dffd_, dval_, dgrad_, ws_, wsb_, s_);
        if (st) return st;
        double D = 0.0;
        if (hipMemcpyAsync(hg_.data(), dgrad_, n_ * sizeof(float), hipMemcpyDeviceToHost, s_) != hipSuccess ||
            hipMemcpyAsync(&D, dval_, sizeof(double), hipMemcpyDeviceToHost, s_) != hipSuccess ||
            hipStreamSynchronize(s_) != hipSuccess)
            return SRWCR_E_HIP;
        g.resize(n_);
        for (size_t i = 0; i < n_; ++i) g[i] = hg_[i];
        f = D;
        if (wp_ > 0.0) {
            std::vector<double> gb;
            f += wp_ * bending_energy(x, lv_.nc, lv_.prob.fixed_dims, lv_.prob.ctrl_spacing, &gb);
            for (size_t i = 0; i < n_; ++i) g[i] += wp_ * gb[i];
        }
        if (D_out) *D_out = D;
        ++evals;
        return SRWCR_OK;
    }
    int evals = 0;

  private:
    Level lv_;
    double wp_;
    hipStream_t s_;
    srwcr_plan *plan_ = nullptr;
    void *ws_ = nullptr;
    float *dffd_ = nullptr, *dgrad_ = nullptr;
    double *dval_ = nullptr;
    size_t wsb_ = 0, n_ = 0;
    std::vector<float> hf_, hg_;
};

double dot(const std::vector<double> &a, const std::vector<double> &b)
{
    double s = 0.0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
}

using EvalFn = std::function<int(const std::vector<double> &, double &, std::vector<double> &)>;

// L-BFGS on one level; x is updated in place.  Returns a status.
int lbfgs_level(const EvalFn &eval, std::vector<double> &x, int max_iter, int m, int stall_window, double stall_tol,
                int &iters, double &f0_out, double &f_out)
{
    const size_t n = x.size();
    std::vector<double> g(n), xn(n), gn(n), d(n);
    double f = 0.0;
    int st = eval(x, f, g);
    if (st) return st;
    if (!std::isfinite(f)) return SRWCR_E_NONFINITE;
    f0_out = f;
    std::deque<std::vector<double>> S, Y;
    std::deque<double> RHO;
    std::deque<double> hist;
    int status = SRWCR_OK;
    iters = 0;
    for (int k = 0; k < max_iter; ++k) {
        // two-loop recursion: d = -H g
        std::vector<double> q = g;
        std::vector<double> alpha(S.size());
        for (int i = (int)S.size() - 1; i >= 0; --i) {
            alpha[i] = RHO[i] * dot(S[i], q);
            for (size_t j = 0; j < n; ++j) q[j] -= alpha[i] * Y[i][j];
        }
        double gamma = 1.0;
        if (!S.empty()) gamma = dot(S.back(), Y.back()) / dot(Y.back(), Y.back());
        for (size_t j = 0; j < n; ++j) q[j] *= gamma;
        for (size_t i = 0; i < S.size(); ++i) {
            const double beta = RHO[i] * dot(Y[i], q);
            for (size_t j = 0; j < n; ++j) q[j] += S[i][j] * (alpha[i] - beta);
        }
        for (size_t j = 0; j < n; ++j) d[j] = -q[j];
        double gd = dot(g, d);
        if (!(gd < 0.0)) {                         // not a descent direction: restart from steepest descent
            S.clear(); Y.clear(); RHO.clear();
            for (size_t j = 0; j < n; ++j) d[j] = -g[j];
            gd = dot(g, d);
        }
        const double gnorm = std::sqrt(dot(g, g));
        if (gnorm == 0.0) break;
        // backtracking line search with the (weak) Wolfe conditions, bracketed:
        // lo satisfies Armijo but not the curvature condition, hi fails Armijo.
        // When no trial lowers the cost along a quasi-Newton direction, the
        // search is repeated once along -g with the history cleared.
        const double c1 = 1e-4, c2 = 0.9;
        bool ok = false, decreased = false;
        double fn = 0.0;
        for (int attempt = 0; attempt < 2 && !ok && !decreased; ++attempt) {
            if (attempt == 1) {
                if (S.empty()) break;               // already steepest descent
                S.clear(); Y.clear(); RHO.clear();
                for (size_t j = 0; j < n; ++j) d[j] = -g[j];
                gd = dot(g, d);
            }
            double step = S.empty() ? 1.0 / std::sqrt(dot(d, d)) : 1.0;
            double best_f = f, best_step = 0.0;
            double lo = 0.0, hi = INFINITY;
            for (int trial = 0; trial < 40; ++trial) {
                for (size_t j = 0; j < n; ++j) xn[j] = x[j] + step * d[j];
                st = eval(xn, fn, gn);
                if (st) return st;
                if (std::isfinite(fn) && fn < best_f) { best_f = fn; best_step = step; }
                if (!std::isfinite(fn) || fn > f + c1 * step * gd) {
                    hi = step;
                } else if (dot(gn, d) < c2 * gd) {
                    lo = step;
                } else {
                    ok = true;
                    break;
                }
                step = std::isfinite(hi) ? 0.5 * (lo + hi) : 2.1 * lo;
            }
            if (!ok && best_step > 0.0) {           // keep the best point seen
                for (size_t j = 0; j < n; ++j) xn[j] = x[j] + best_step * d[j];
                st = eval(xn, fn, gn);
                if (st) return st;
                decreased = true;
            }
        }
        if (!ok && !decreased) {
            // no step lowers the cost: D is evaluated on the FFD rounded to FP32,
            // so below that resolution the cost is flat.  After progress this is
            // convergence at working precision; at the first iteration it means
            // the gradient does not describe the cost.
            if (iters == 0) status = SRWCR_E_LINESEARCH;
            break;
        }
        std::vector<double> s(n), yv(n);
        for (size_t j = 0; j < n; ++j) { s[j] = xn[j] - x[j]; yv[j] = gn[j] - g[j]; }
        const double sy = dot(s, yv);
        if (sy > 1e-300) {
            S.push_back(s); Y.push_back(yv); RHO.push_back(1.0 / sy);
            if ((int)S.size() > m) { S.pop_front(); Y.pop_front(); RHO.pop_front(); }
        }
        x.swap(xn);
        g.swap(gn);
        f = fn;
        ++iters;
        hist.push_back(f);
        if ((int)hist.size() > stall_window) hist.pop_front();
        if ((int)hist.size() == stall_window) {
            const auto mm = std::minmax_element(hist.begin(), hist.end());
            if (*mm.second - *mm.first <= stall_tol * std::fabs(f)) break;
        }
    }
    f_out = f;
    return status;
}

}  // namespace

extern "C" int srwcr_lbfgs_minimize(int64_t n, double *x, srwcr_fg_fn fg, void *user, int32_t max_iter,
                                    int32_t history, int32_t stall_window, double stall_tol, int32_t *iterations,
                                    int32_t *evaluations, double *f_final)
{
    if (n < 1 || !x || !fg || max_iter < 0 || history < 1 || stall_window < 2) return SRWCR_E_INVALID_ARG;
    std::vector<double> xv(x, x + n);
    int evals = 0;
    const EvalFn eval = [&](const std::vector<double> &p, double &f, std::vector<double> &g) {
        g.assign((size_t)n, 0.0);
        ++evals;
        return fg(user, p.data(), &f, g.data());
    };
    int iters = 0;
    double f0 = 0.0, f1 = 0.0;
    const int st = lbfgs_level(eval, xv, max_iter, history, stall_window, stall_tol, iters, f0, f1);
    std::copy(xv.begin(), xv.end(), x);
    if (iterations) *iterations = iters;
    if (evaluations) *evaluations = evals;
    if (f_final) *f_final = f1;
    return st;
}

extern "C" int srwcr_refine_ffd(const int32_t coarse_nc[3], const float *coarse, const int32_t fine_nc[3],
                                float *fine)
{
    if (!coarse_nc || !coarse || !fine_nc || !fine) return SRWCR_E_INVALID_ARG;
    int cn[3], fn[3];
    for (int e = 0; e < 3; ++e) {
        cn[e] = coarse_nc[e];
        fn[e] = fine_nc[e];
        if (cn[e] < 4 || fn[e] < 4) return SRWCR_E_INVALID_ARG;
    }
    std::vector<double> c(3 * (size_t)cn[0] * cn[1] * cn[2]);
    for (size_t i = 0; i < c.size(); ++i) c[i] = coarse[i];
    const std::vector<double> f = refine(c, cn, fn);
    for (size_t i = 0; i < f.size(); ++i) fine[i] = (float)f[i];
    return SRWCR_OK;
}

extern "C" double srwcr_bending_energy(const srwcr_problem *prob, const float *ffd, float *grad)
{
    if (!prob || !ffd) return -1.0;
    int nc[3];
    if (srwcr_ctrl_dims(prob, nc) != SRWCR_OK) return -1.0;
    std::vector<double> c(3 * (size_t)nc[0] * nc[1] * nc[2]);
    for (size_t i = 0; i < c.size(); ++i) c[i] = ffd[i];
    std::vector<double> g;
    const double E = bending_energy(c, nc, prob->fixed_dims, prob->ctrl_spacing, grad ? &g : nullptr);
    if (grad)
        for (size_t i = 0; i < g.size(); ++i) grad[i] = (float)g[i];
    return E;
}

extern "C" int register_lbfgs(const srwcr_problem *prob, const float *fixed, const float *moving, float *ffd_inout,
                              const srwcr_lbfgs_opts *opts, srwcr_lbfgs_report *report, void *stream)
{
    if (!prob || !fixed || !moving || !ffd_inout || !opts) return SRWCR_E_INVALID_ARG;
    if (opts->levels < 1 || opts->levels > 3 || opts->history < 1 || opts->stall_window < 2)
        return SRWCR_E_INVALID_ARG;
    if (prob->fixed_dtype != SRWCR_F32 || prob->moving_dtype != SRWCR_F32) return SRWCR_E_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    srwcr_lbfgs_report rep;
    std::memset(&rep, 0, sizeof rep);

    // pyramid: level 0 = finest
    const int nl = opts->levels;
    std::vector<Level> lv(nl);
    std::vector<float *> owned;
    lv[0].prob = *prob;
    lv[0].fixed = fixed;
    lv[0].moving = moving;
    int st = SRWCR_OK;
    for (int l = 1; l < nl; ++l) {
        Level &c = lv[l];
        const Level &f = lv[l - 1];
        c.prob = f.prob;
        for (int e = 0; e < 3; ++e) {
            c.prob.fixed_dims[e] = (f.prob.fixed_dims[e] + 1) / 2;
            c.prob.moving_dims[e] = (f.prob.moving_dims[e] + 1) / 2;
            if (c.prob.fixed_dims[e] < 2 || c.prob.moving_dims[e] < 2) st = SRWCR_E_INVALID_ARG;
        }
        if (st) break;
        float *cf = nullptr, *cm = nullptr;
        const size_t nfc = (size_t)c.prob.fixed_dims[0] * c.prob.fixed_dims[1] * c.prob.fixed_dims[2];
        const size_t nmc = (size_t)c.prob.moving_dims[0] * c.prob.moving_dims[1] * c.prob.moving_dims[2];
        if (hipMalloc(&cf, nfc * sizeof(float)) != hipSuccess || hipMalloc(&cm, nmc * sizeof(float)) != hipSuccess) {
            st = SRWCR_E_HIP;
            if (cf) owned.push_back(cf);
            break;
        }
        owned.push_back(cf);
        owned.push_back(cm);
        if (launch_downsample(f.fixed, f.prob.fixed_dims[0], f.prob.fixed_dims[1], f.prob.fixed_dims[2], cf,
                              c.prob.fixed_dims[0], c.prob.fixed_dims[1], c.prob.fixed_dims[2], s) != hipSuccess ||
            launch_downsample(f.moving, f.prob.moving_dims[0], f.prob.moving_dims[1], f.prob.moving_dims[2], cm,
                              c.prob.moving_dims[0], c.prob.moving_dims[1], c.prob.moving_dims[2], s) != hipSuccess) {
            st = SRWCR_E_HIP;
            break;
        }
        c.fixed = cf;
        c.moving = cm;
    }
    for (int l = 0; l < nl && !st; ++l) st = srwcr_ctrl_dims(&lv[l].prob, lv[l].nc);

    std::vector<double> x;
    for (int l = nl - 1; l >= 0 && !st; --l) {
        const int ri = nl - 1 - l;                               // report index, coarsest first
        const size_t n = 3 * (size_t)lv[l].nc[0] * lv[l].nc[1] * lv[l].nc[2];
        if (l == nl - 1) {
            // the caller's start, carried down to the coarsest level
            const size_t n0 = 3 * (size_t)lv[0].nc[0] * lv[0].nc[1] * lv[0].nc[2];
            x.assign(ffd_inout, ffd_inout + n0);
            for (int k = 1; k < nl; ++k) x = decimate(x, lv[k - 1].nc, lv[k].nc);
        } else {
            x = refine(x, lv[l + 1].nc, lv[l].nc);
        }
        const auto t0 = std::chrono::steady_clock::now();
        Evaluator ev(lv[l], opts->bending_weight, s);
        st = ev.init();
        if (st) break;
        int iters = 0;
        double f0 = 0.0, f1 = 0.0;
        const EvalFn eval = [&ev](const std::vector<double> &p, double &f, std::vector<double> &g) {
            return ev.eval(p, f, g);
        };
        const int lvl_status = lbfgs_level(eval, x, opts->max_iter[ri], opts->history, opts->stall_window,
                                           opts->stall_tol, iters, f0, f1);
        rep.seconds[ri] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        rep.iterations[ri] = iters;
        rep.evaluations[ri] = ev.evals;
        rep.initial_value[ri] = f0;
        rep.final_value[ri] = f1;
        rep.status[ri] = lvl_status;
        if (lvl_status != SRWCR_OK && lvl_status != SRWCR_E_LINESEARCH) st = lvl_status;
    }
    if (!st) {
        const size_t n = 3 * (size_t)lv[0].nc[0] * lv[0].nc[1] * lv[0].nc[2];
        for (size_t i = 0; i < n; ++i) ffd_inout[i] = (float)x[i];
    }
    (void)hipStreamSynchronize(s);
    for (float *p : owned) (void)hipFree(p);
    if (report) *report = rep;
    return st;
}
