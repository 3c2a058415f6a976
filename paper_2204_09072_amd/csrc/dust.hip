// Dust thermal equilibrium (Sec. 4.6 and App. E of Klepitko et al. 2023).
//
// Per cell, the residual divided by rho,
//   g(T) = xi 4 sigma kappa(T) T^4 - xi 4 pi kappa(T_J) J - C (T_g - T),
//   C    = c_gd rho / (1.4 m_H)^2 sqrt(T_g) (1 - 0.8 exp(-75 / T_g)),
// is strictly increasing, negative at min(T_g, T_J) and positive at max(T_g, T_J).
// Newton's method (by default on ln w against ln T, see the kernel) runs inside that
// bracket, with bisection when a step leaves it (a step reaching an end not yet evaluated
// tries that end first); the starting point is the bracket's secant
// point in logarithms, the bracket end nearer the root, or the guess network's output.
// Plain bisection of the same bracket is there as a reference for the step counts.
#include "common.hpp"
#include "mlp.hpp"

namespace {

constexpr float kFloor = 2.7f;
constexpr double kMH = 1.6735575e-24;

__device__ __forceinline__ float kap_planck(float t) { return t < 150.0f ? 1.0e-3f * (t * t) : 22.5f; }
// kappa(T) T^4 and its derivative
__device__ __forceinline__ void emis(float t, float &v, float &dv) {
    const float t2 = t * t, t4 = t2 * t2;
    if (t < 150.0f) {
        v = 1.0e-3f * t2 * t4;
        dv = 6.0e-3f * t * t4;
    } else {
        v = 22.5f * t4;
        dv = 90.0f * t * t2;
    }
}

struct DustArgs {
    int64_t n;
    const float *rho, *u_rad, *t_gas;
    float *t_dust;
    uint8_t *iters;
    float a4s;      // xi 4 sigma
    float c_over_4pi;
    float pi_over_sigma;
    float xi4pi;
    float cgd_n;    // c_gd / (1.4 m_H)^2
    float tol;
    int max_iter;
    const float *guess; // learned starting points (START_LEARNED)
};

enum Start { START_SECANT = 0, START_END = 1, START_LEARNED = 2, START_BISECT = 3 };

// START: where Newton begins (the bracket's secant point in logarithms, the bracket end
// with the smaller |ln(w/K)|, or the guess network's output).  LOG: Newton on ln w against
// ln T (else on g(T) itself).  Every variant keeps the bracket and bisects when a step
// leaves it, and stops on the same rule.  START_BISECT takes no Newton steps: the bracket
// is halved until its width is within tol of its upper end, and T is its midpoint.
template <int START, bool LOG>
__global__ __launch_bounds__(256) void k_dust(DustArgs A) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= A.n) return;
    const float rho = A.rho[c], u = A.u_rad[c], tg = A.t_gas[c];
    const float J = u * A.c_over_4pi;
    const float tj = sqrtf(sqrtf(A.pi_over_sigma * J));
    const float H = A.xi4pi * kap_planck(tj) * J;
    const float C = A.cgd_n * rho * sqrtf(tg) * (1.0f - 0.8f * __expf(-75.0f / tg));
    // g(T) = w(T) - K with w = xi 4 sigma kappa(T) T^4 + C T increasing and convex and
    // K = heating + C T_g.  In logarithms either dominant term (T^6 below 150 K, T^4
    // above, or T) makes ln w nearly linear in ln T, so Newton there converges fast from
    // both sides of the root.
    const float K = H + C * tg;
    auto wf = [&](float t, float &dw) {
        float v, dv;
        emis(t, v, dv);
        dw = A.a4s * dv + C;
        return A.a4s * v + C * t;
    };
    float lo = fmaxf(kFloor, fminf(tg, tj)), hi = fmaxf(kFloor, fmaxf(tg, tj));
    int it = 0;
    float T, dw;
    if (hi <= kFloor) {
        T = kFloor;
    } else {
        bool done = false;
        float wl = 0.0f;
        bool lo_known = false, hi_known = false; // whether w has been evaluated at lo, hi
        if (START != START_LEARNED || lo == kFloor) {
            wl = wf(lo, dw);
            lo_known = true;
            if (wl >= K) { T = lo; done = true; } // root at or below the lower end (floor)
        }
        if (!done) {
            if (START == START_LEARNED) {
                T = A.guess[c];
                if (!(T > lo)) T = lo;   // also catches NaN from a poisoned network
                if (!(T < hi)) T = hi;
            } else if (START == START_BISECT) {
                T = 0.5f * (lo + hi);
            } else {
                const float wh = wf(hi, dw);
                hi_known = true;
                const float rl = __logf(K) - __logf(wl), rh = __logf(wh) - __logf(K);
                if (START == START_END) {
                    T = rl < rh ? lo : hi;
                } else {
                    // secant of the bracket in (ln T, ln w)
                    const float ll = __logf(lo), lh = __logf(hi);
                    T = __expf(ll + rl * (lh - ll) / (rl + rh));
                    if (!(T > lo && T < hi)) T = sqrtf(lo * hi);
                }
            }
            for (it = 1; it <= A.max_iter; ++it) {
                const float wv = wf(T, dw);
                if (wv < K) {
                    lo = T;
                    lo_known = true;
                } else {
                    hi = T;
                    hi_known = true;
                }
                if (START == START_BISECT) {
                    T = 0.5f * (lo + hi);
                    if (hi - lo <= A.tol * hi) break;
                    continue;
                }
                float Tn = LOG ? T * __expf(-__logf(wv / K) * wv / (T * dw)) : T - (wv - K) / dw;
                // a Newton step within tol: T is at the root to working precision.  Taken
                // before the bracket test, since a step below FP32 resolution lands on the
                // bracket end just moved to T and would otherwise be replaced by bisection.
                if (fabsf(Tn - T) <= A.tol * T) {
                    if (Tn > lo && Tn < hi) T = Tn;
                    break;
                }
                // A step that reaches an end of the bracket where w has not been evaluated
                // tries that end (once: it is then known).  Where the coupling is weak the
                // root lies at T_J or T_gas to FP32 precision and Newton lands there from a
                // good guess; bisection instead of that step took 10-16 steps.  Any other
                // step outside the open bracket (or NaN) is replaced by bisection.
                if (!(Tn > lo && Tn < hi)) {
                    if (Tn >= hi && !hi_known) Tn = hi;
                    else if (Tn <= lo && !lo_known) Tn = lo;
                    else Tn = 0.5f * (lo + hi);
                }
                const bool conv = fabsf(Tn - T) <= A.tol * Tn || hi - lo <= A.tol * hi;
                T = Tn;
                if (conv) break;
            }
            if (it > A.max_iter) it = A.max_iter;
        }
    }
    A.t_dust[c] = T < kFloor ? kFloor : T;
    if (A.iters) A.iters[c] = (uint8_t)(it > 255 ? 255 : it);
}

} // namespace

namespace {

// Checks, then the solve's kernels; `guess` receives the network's starting points (n floats,
// used only with a network).
int dust_solve(tr_ctx *ctx, int64_t n, const float *rho, const float *u_rad, const float *t_gas,
               const tr_dust_params *p, const tr_mlp *mlp, float *t_dust, uint8_t *iters, float *guess) {
    DustArgs A;
    A.n = n; A.rho = rho; A.u_rad = u_rad; A.t_gas = t_gas; A.t_dust = t_dust; A.iters = iters;
    A.a4s = (float)(p->xi * 4.0 * p->sigma);
    A.c_over_4pi = (float)(p->c / (4.0 * 3.14159265358979323846));
    A.pi_over_sigma = (float)(3.14159265358979323846 / p->sigma);
    A.xi4pi = (float)(p->xi * 4.0 * 3.14159265358979323846);
    A.cgd_n = (float)(p->c_gd / ((1.4 * kMH) * (1.4 * kMH)));
    A.tol = p->rel_tol > 0 ? p->rel_tol : 1e-6f;
    A.max_iter = p->max_iter > 0 ? p->max_iter : 50;
    const int blocks = (int)tr_div_up(n, 256);
    A.guess = nullptr;
    if (mlp) {
        int rc = mlp_guess(ctx, mlp, n, rho, u_rad, t_gas, guess);
        if (rc) return rc;
        A.guess = guess;
        if (p->linear) k_dust<START_LEARNED, false><<<blocks, 256, 0, ctx->stream>>>(A);
        else k_dust<START_LEARNED, true><<<blocks, 256, 0, ctx->stream>>>(A);
    } else if (p->start == 2) {
        k_dust<START_BISECT, true><<<blocks, 256, 0, ctx->stream>>>(A);
    } else if (p->start == 1) {
        if (p->linear) k_dust<START_END, false><<<blocks, 256, 0, ctx->stream>>>(A);
        else k_dust<START_END, true><<<blocks, 256, 0, ctx->stream>>>(A);
    } else {
        if (p->linear) k_dust<START_SECANT, false><<<blocks, 256, 0, ctx->stream>>>(A);
        else k_dust<START_SECANT, true><<<blocks, 256, 0, ctx->stream>>>(A);
    }
    if (hipGetLastError() != hipSuccess) return tr_fail(ctx, TR_EHIP, "dust kernel launch failed");
    return TR_OK;
}

int dust_check(tr_ctx *ctx, const char *who, int64_t n, const float *rho, const float *u_rad,
               const float *t_gas, const tr_dust_params *p, float *t_dust) {
    if (n < 0 || (n > 0 && (!rho || !u_rad || !t_gas || !t_dust)) || !p)
        return tr_fail(ctx, TR_EINVAL, "%s: bad argument", who);
    if (!(p->sigma > 0) || !(p->c > 0) || p->c_gd < 0 || p->xi <= 0)
        return tr_fail(ctx, TR_EINVAL, "%s: bad constants", who);
    if (p->start < 0 || p->start > 2 || p->linear < 0 || p->linear > 1)
        return tr_fail(ctx, TR_EINVAL, "%s: bad start (%d) or linear (%d)", who, p->start, p->linear);
    return TR_OK;
}

} // namespace

extern "C" int tr_dust_equilibrium(tr_ctx *ctx, int64_t n, const float *rho, const float *u_rad,
                                   const float *t_gas, const tr_dust_params *p, const tr_mlp *mlp,
                                   float *t_dust, uint8_t *iters) {
    if (!ctx) return TR_EINVAL;
    int rc = dust_check(ctx, "tr_dust_equilibrium", n, rho, u_rad, t_gas, p, t_dust);
    if (rc || n == 0) return rc;
    TR_HIP(ctx, hipSetDevice(ctx->device));
    if (mlp && ctx->ws_guess_n < n) {
        hipFree(ctx->ws_guess);
        ctx->ws_guess = nullptr;
        ctx->ws_guess_n = 0;
        if (hipMalloc(&ctx->ws_guess, sizeof(float) * n) != hipSuccess)
            return tr_fail(ctx, TR_ENOMEM, "guess workspace");
        ctx->ws_guess_n = n;
    }
    return dust_solve(ctx, n, rho, u_rad, t_gas, p, mlp, t_dust, iters, ctx->ws_guess);
}

extern "C" int tr_dust_equilibrium_noalloc(tr_ctx *ctx, int64_t n, const float *rho, const float *u_rad,
                                           const float *t_gas, const tr_dust_params *p, const tr_mlp *mlp,
                                           float *t_dust, uint8_t *iters) {
    if (!ctx) return TR_EINVAL;
    int rc = dust_check(ctx, "tr_dust_equilibrium_noalloc", n, rho, u_rad, t_gas, p, t_dust);
    if (rc || n == 0) return rc;
    if (n > TR_NOALLOC_DUST_STATES)
        return tr_fail(ctx, TR_EINVAL, "tr_dust_equilibrium_noalloc: %lld states, at most %d",
                       (long long)n, TR_NOALLOC_DUST_STATES);
    if (!ctx->noalloc_guess) return tr_fail(ctx, TR_EHIP, "tr_dust_equilibrium_noalloc: no scratch on this device");
    TR_HIP(ctx, hipSetDevice(ctx->device));
    return dust_solve(ctx, n, rho, u_rad, t_gas, p, mlp, t_dust, iters, ctx->noalloc_guess);
}
