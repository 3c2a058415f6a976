// Guess network of the dust-equilibrium solve: 3 -> 64 -> 64 -> 1, ReLU hidden layers.
#pragma once
#include "common.hpp"

#define MLP_H 64
#define MLP_NPARAM (3 * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1)
#define MLP_OFF_B1 (3 * MLP_H)
#define MLP_OFF_W2 (MLP_OFF_B1 + MLP_H)
#define MLP_OFF_B2 (MLP_OFF_W2 + MLP_H * MLP_H)
#define MLP_OFF_W3 (MLP_OFF_B2 + MLP_H)
#define MLP_OFF_B3 (MLP_OFF_W3 + MLP_H)

struct tr_mlp {
    tr_ctx *ctx = nullptr;
    float *p = nullptr;       // FP32 master parameters
    float *wq = nullptr;      // parameters rounded to bfloat16 (held as float)
    float *m = nullptr, *v = nullptr, *grad = nullptr, *loss = nullptr;
    int64_t step = 0;         // Adam steps taken
    float norm[8] = {0, 0, 0, 1, 1, 1, 0, 1};
};

// FP32 parameters of a network (device)
inline const float *mlp_params(const tr_mlp *m) { return m->p; }

// temperature guesses of the network for raw (rho, u_rad, T_gas) fields, on the matrix cores
int mlp_guess(tr_ctx *ctx, const tr_mlp *m, int64_t n, const float *rho, const float *u_rad,
              const float *t_gas, float *guess);

__device__ __forceinline__ float bf16_round(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}

// ---------------------------------------------------------------------------------------
// Inference of the network with every operand in registers, on the matrix cores (shared by
// the inference kernel and the learned-start dust solve).  One call evaluates 32 samples:
// hidden units are rows and samples columns of 32 x 32 tiles (transposed products),
//   a1[n][s] = sum_k [W1 | b1][n][k] [x; 1][k][s]          (v_mfma_f32_32x32x8_bf16, K = 3 + bias)
//   a2[n][s] = sum_k W2[n][k] h1[k][s] + b2[n]             (v_mfma_f32_32x32x16_bf16)
//   y[s]     = sum_k w3[k] h2[k][s] + b3                   (w3 as row 0 of a third product)
// 32x32x8 layout: lane l holds A[l%32][4(l/32)+0..3] and B[4(l/32)+0..3][l%32]; the 16
// accumulators of lane l are C[8(v/4) + 4(l/32) + v%4][l%32], v = 0..15.  32x32x16: lane l
// contributes 8 K-slots, A and B slot for slot; a contraction may visit K in any order, so
// K-block kk takes accumulators v = 8 (kk % 2) + j of first-layer tile kk / 2 as its B slots
// and the matching columns of W2 (and w3) as its A slots, and h1 never leaves the registers.
// The second layer's bias enters as the accumulators' starting value.  Operands are
// bfloat16 (round to nearest even), accumulation FP32.
// ---------------------------------------------------------------------------------------
namespace trnet {

typedef short sh4 __attribute__((ext_vector_type(4)));
typedef short sh2 __attribute__((ext_vector_type(2)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

// two floats to packed bfloat16 (round to nearest even, v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t pk_bf16(float a, float b) {
    const f2v x = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(x, bf2v));
}
__device__ __forceinline__ sh4 sh4_of(uint32_t lo, uint32_t hi) {
    const u2v v = {lo, hi};
    return __builtin_bit_cast(sh4, v);
}
__device__ __forceinline__ bf8v bf8_of(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    const u4v v = {a, b, c, d};
    return __builtin_bit_cast(bf8v, v);
}
// max(x, 0) in one integer max: negative floats have negative bit patterns
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }
// ReLU of two packed bfloat16 values in one packed 16-bit integer max: a negative value
// (its sign bit set) is a negative int16, and rounding to bfloat16 keeps the sign, so
// max(round(x), 0) = round(max(x, 0))
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t v) {
    const sh2 x = __builtin_bit_cast(sh2, v);
    const sh2 z = {0, 0};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(x, z));
}
// eight accumulators v0 .. v0 + 7 of a tile, rounded to bfloat16, ReLU'd, packed as a
// K = 16 operand
__device__ __forceinline__ bf8v relu_pack8(const f16v &a, int v0) {
    return bf8_of(relu_bf16x2(pk_bf16(a[v0], a[v0 + 1])), relu_bf16x2(pk_bf16(a[v0 + 2], a[v0 + 3])),
                  relu_bf16x2(pk_bf16(a[v0 + 4], a[v0 + 5])), relu_bf16x2(pk_bf16(a[v0 + 6], a[v0 + 7])));
}


__device__ __forceinline__ float bf16_of(float x) { return bf16_round(x); }

constexpr float kLog10of2 = 0.30102999566398120f, kLog2of10 = 3.32192809488736235f;

// normalised network input of a raw field value: (log10 max(v, 1e-37) - shift) * scale, the
// logarithm from the hardware's base-2 instruction (about 1 ulp, far finer than the
// operands' bfloat16 rounding; 1e-37 is a normal float, as v_log_f32 requires)
__device__ __forceinline__ float feature(float v, float shift, float scale) {
    return (__builtin_amdgcn_logf(fmaxf(v, 1e-37f)) * kLog10of2 - shift) * scale;
}
// the first product's B operand for one sample column: (x0, x1, x2, 1) in half-wave 0
__device__ __forceinline__ sh4 input_operand(float x0, float x1, float x2) {
    return sh4_of(pk_bf16(x0, x1), pk_bf16(x2, 1.0f));
}
// temperature from the network's output: 10^(y / out_scale + out_shift)
__device__ __forceinline__ float temperature(float y, float inv_out_scale, float out_shift) {
    return __builtin_amdgcn_exp2f((y * inv_out_scale + out_shift) * kLog2of10);
}

struct Net {
    sh4 aw1[2];                       // [W1 | b1] rows 32 t + col (half-wave 1: zero padding)
    bf8v aw2[2][MLP_H / 16];          // W2 rows 32 t + col, K-slot order as the h1 operand
    bf8v aw3[MLP_H / 16];             // w3 in row 0 (lanes 0 and 32), same slot order
    f16v c2[2];                       // b2 as the second product's starting accumulators
    float b3;

    // parameters p (FP32, layout of MLP_OFF_*), rounded to bfloat16
    __device__ __forceinline__ void load(const float *p, int col, int half) {
        const float *W1 = p, *B1 = p + MLP_OFF_B1, *W2 = p + MLP_OFF_W2, *B2 = p + MLP_OFF_B2, *W3 = p + MLP_OFF_W3;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int n = 32 * t + col;
            aw1[t] = half == 0 ? sh4_of(pk_bf16(W1[3 * n], W1[3 * n + 1]), pk_bf16(W1[3 * n + 2], B1[n]))
                               : sh4_of(0u, 0u);
#pragma unroll
            for (int kk = 0; kk < MLP_H / 16; ++kk) {
                // slot j <-> hidden unit 32 (kk / 2) + 16 (kk % 2) + 8 (j / 4) + 4 half + j % 4
                const float *w = W2 + MLP_H * n + 32 * (kk >> 1) + 16 * (kk & 1) + 4 * half;
                aw2[t][kk] = bf8_of(pk_bf16(w[0], w[1]), pk_bf16(w[2], w[3]), pk_bf16(w[8], w[9]), pk_bf16(w[10], w[11]));
            }
#pragma unroll
            for (int v = 0; v < 16; ++v) c2[t][v] = bf16_of(B2[32 * t + 8 * (v >> 2) + 4 * half + (v & 3)]);
        }
#pragma unroll
        for (int kk = 0; kk < MLP_H / 16; ++kk) {
            const float *w = W3 + 32 * (kk >> 1) + 16 * (kk & 1) + 4 * half;
            aw3[kk] = col == 0 ? bf8_of(pk_bf16(w[0], w[1]), pk_bf16(w[2], w[3]), pk_bf16(w[8], w[9]), pk_bf16(w[10], w[11]))
                               : bf8_of(0u, 0u, 0u, 0u);
        }
        b3 = bf16_of(p[MLP_OFF_B3]);
    }

    // the network on 32 sample columns (bx: input_operand in half-wave 0, zero in half-wave
    // 1); the output of sample col is the return value of lanes 0..31
    __device__ __forceinline__ float eval(sh4 bx) const {
        const f16v zero = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        f16v a1[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) a1[t] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(aw1[t], bx, zero, 0, 0, 0);
        // h1 = ReLU(a1) in bfloat16: K-block kk holds accumulators 8 (kk % 2) + 0..7 of tile kk / 2
        bf8v bh[MLP_H / 16];
#pragma unroll
        for (int kk = 0; kk < MLP_H / 16; ++kk) bh[kk] = relu_pack8(a1[kk >> 1], 8 * (kk & 1));
        f16v a2[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            a2[t] = c2[t];
#pragma unroll
            for (int kk = 0; kk < MLP_H / 16; ++kk)
                a2[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aw2[t][kk], bh[kk], a2[t], 0, 0, 0);
        }
        f16v a3 = zero;
#pragma unroll
        for (int kk = 0; kk < MLP_H / 16; ++kk)
            a3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aw3[kk], relu_pack8(a2[kk >> 1], 8 * (kk & 1)), a3, 0, 0, 0);
        return a3[0] + b3;
    }
};

} // namespace trnet
