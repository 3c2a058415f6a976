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
    uint16_t *w16 = nullptr;  // bfloat16 bits of W2 for the matrix cores
    float *m = nullptr, *v = nullptr, *grad = nullptr, *loss = nullptr;
    int step = 0;
    float norm[8] = {0, 0, 0, 1, 1, 1, 0, 1};
};

// temperature guesses of the network for raw (rho, u_rad, T_gas) fields, on the matrix cores
int mlp_guess(tr_ctx *ctx, const tr_mlp *m, int64_t n, const float *rho, const float *u_rad,
              const float *t_gas, float *guess);

__device__ __forceinline__ float bf16_round(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xffff0000u);
}
