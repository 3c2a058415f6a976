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
// blocks of 4 waves per compute unit for the one-kernel learned solve (3 waves per SIMD fit
// its registers); each wave then loops over groups of 64 states
constexpr int kLearnedBlocksPerCu = 3;
constexpr double kMH = 1.6735575e-24;

__device__ __forceinline__ float kap_planck(float t) { return t < 150.0f ? 1.0e-3f * (t * t) : 22.5f; }
// hardware reciprocal and square root (about 1 ulp): the solve's quantities need no correctly
// rounded division or root, since the stopping rule (a Newton step within rel_tol = 1e-6 of
// T) and not the last bit of a step fixes the root, and a 1-ulp change of T_J or sqrt(T_g)
// moves the residual's coefficients, hence the root, by about 1e-7 of itself
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
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
__device__ __forceinline__ void dust_cell(const DustArgs &A, float rho, float u, float tg, float guess, float &T_out,
                                          int &it_out) {
    const float J = u * A.c_over_4pi;
    const float tj = fsqrt(fsqrt(A.pi_over_sigma * J));
    const float H = A.xi4pi * kap_planck(tj) * J;
    const float C = A.cgd_n * rho * fsqrt(tg) * (1.0f - 0.8f * __expf(-75.0f * frcp(tg)));
    // g(T) = w(T) - K with w = xi 4 sigma kappa(T) T^4 + C T increasing and convex and
    // K = heating + C T_g.  In logarithms either dominant term (T^6 below 150 K, T^4
    // above, or T) makes ln w nearly linear in ln T, so Newton there converges fast from
    // both sides of the root.
    const float K = H + C * tg;
    const float rK = frcp(K);
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
                T = guess;
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
                    T = __expf(ll + rl * (lh - ll) * frcp(rl + rh));
                    if (!(T > lo && T < hi)) T = fsqrt(lo * hi);
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
                float Tn = LOG ? T * __expf(-__logf(wv * rK) * wv * frcp(T * dw)) : T - (wv - K) * frcp(dw);
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
    T_out = T < kFloor ? kFloor : T;
    it_out = it;
}

template <int START, bool LOG>
__global__ __launch_bounds__(256) void k_dust(DustArgs A) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= A.n) return;
    float T;
    int it;
    dust_cell<START, LOG>(A, A.rho[c], A.u_rad[c], A.t_gas[c], START == START_LEARNED ? A.guess[c] : 0.0f, T, it);
    A.t_dust[c] = T;
    if (A.iters) A.iters[c] = (uint8_t)(it > 255 ? 255 : it);
}

// The learned start in one kernel: each wave takes 64 states at a time, evaluates the guess
// network on them in two 32-column products (its weights held in registers for the whole
// launch) and solves all 64 from the guesses, which never leave the registers.  The matrix
// products of one wave overlap the Newton iterations of others on the same SIMD.  The
// network is the one tr_mlp_forward runs (same operands and operation order), so the
// starting points equal those of the staged form (network into a buffer, then k_dust).
struct NetArgs {
    const float *p;  // FP32 parameters
    float shift[3], scale[3], out_shift, inv_out_scale;
};

template <bool LOG>
__global__ __launch_bounds__(256) void k_dust_learned(DustArgs A, NetArgs N) {
    const int lane = threadIdx.x & 63, col = lane & 31, half = lane >> 5;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwave = ((int64_t)gridDim.x * blockDim.x) >> 6;
    trnet::Net net;
    net.load(N.p, col, half);
    const int64_t ngroup = (A.n + 63) >> 6;
    for (int64_t g = wave; g < ngroup; g += nwave) {
        const int64_t c = (g << 6) + lane;
        const bool own = c < A.n;
        const int64_t cc = own ? c : A.n - 1;
        const float rho = A.rho[cc], u = A.u_rad[cc], tg = A.t_gas[cc];
        // this lane's state as a sample column; half-wave 1's columns move to half-wave 0 for
        // the second product
        const trnet::sh4 bx = trnet::input_operand(trnet::feature(rho, N.shift[0], N.scale[0]),
                                                   trnet::feature(u, N.shift[1], N.scale[1]),
                                                   trnet::feature(tg, N.shift[2], N.scale[2]));
        const uint32_t bx0 = __builtin_bit_cast(trnet::u2v, bx)[0], bx1 = __builtin_bit_cast(trnet::u2v, bx)[1];
        const uint32_t up0 = (uint32_t)__shfl_xor((int)bx0, 32), up1 = (uint32_t)__shfl_xor((int)bx1, 32);
        const trnet::sh4 zero4 = trnet::sh4_of(0u, 0u);
        const float ya = net.eval(half == 0 ? bx : zero4);
        const float yb = net.eval(half == 0 ? trnet::sh4_of(up0, up1) : zero4);
        // lanes 0..31 hold the outputs of both products; lanes 32..63 take the second's.  The
        // exchange runs on every lane before the select: as an arm of ?: it would run on
        // lanes 32..63 alone, and a permute reads nothing from lanes that do not take part.
        const float yb_up = __shfl_xor(yb, 32);
        const float y = half == 0 ? ya : yb_up;
        float T;
        int it;
        dust_cell<START_LEARNED, LOG>(A, rho, u, tg, trnet::temperature(y, N.inv_out_scale, N.out_shift), T, it);
        if (own) {
            A.t_dust[c] = T;
            if (A.iters) A.iters[c] = (uint8_t)(it > 255 ? 255 : it);
        }
    }
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
    if (mlp && !p->staged) {
        // one kernel: the network's guesses stay in registers (no buffer)
        NetArgs N;
        N.p = mlp_params(mlp);
        for (int k = 0; k < 3; ++k) {
            N.shift[k] = mlp->norm[k];
            N.scale[k] = mlp->norm[3 + k];
        }
        N.out_shift = mlp->norm[6];
        N.inv_out_scale = 1.0f / mlp->norm[7];
        const int64_t waves = (n + 63) / 64;
        int64_t grid = (waves + 3) / 4;
        const int64_t cap = (int64_t)ctx->n_cu * kLearnedBlocksPerCu;
        grid = grid < cap ? grid : cap;
        if (p->linear) k_dust_learned<false><<<(int)grid, 256, 0, ctx->stream>>>(A, N);
        else k_dust_learned<true><<<(int)grid, 256, 0, ctx->stream>>>(A, N);
    } else if (mlp) {
        // staged: the network's guesses through `guess`, then the solve
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
    if (p->start < 0 || p->start > 2 || p->linear < 0 || p->linear > 1 || p->staged < 0 || p->staged > 1)
        return tr_fail(ctx, TR_EINVAL, "%s: bad start (%d), linear (%d) or staged (%d)", who, p->start, p->linear,
                       p->staged);
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
    if (mlp && p->staged && ctx->ws_guess_n < n) {
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
    tr_dust_params ps = *p;
    ps.staged = 1; // the network's guesses through this device's scratch
    return dust_solve(ctx, n, rho, u_rad, t_gas, &ps, mlp, t_dust, iters, ctx->noalloc_guess);
}
