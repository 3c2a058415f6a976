// Internal declarations shared by the library's HIP translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "treeray.h"

#define TR_FX 256 /* fixed-point subdivisions of the lattice unit (mapping positions) */
#define TR_MAX_DEPTH 9

struct RayTable {
    int n_side = 0, cube_m = 0;
    int16_t *table = nullptr; // [6][M][M] pixel ids
    float4 *dirs = nullptr;   // [npix] unit vectors
    // tabulated angular kernel: [6][M][M][classes 6 .. alpha_c1 - 1] packed 64-bit entries
    // (4 pixels of 10 bits, 3 counts of 7 bits out of 64, the 4th by difference, and the
    // more-than-4-pixels flag at bit 61); classes from alpha_c1 on hold the direction cell's
    // own pixel only and are read from the pixel table
    unsigned long long *alpha = nullptr;
    int alpha_c1 = 21;
    // per-node angular kernel of a leaf at an integer offset m (in its edges, |m_a| <= 7,
    // [mx + 7][my + 7][mz + 7]) from a target of its own size: the pixel ids of its 2x2x2
    // sub-points in ascending order (10 bits each, x: 0-2, y: 3-5, z: 6-7) and in w the
    // mask of the first of each run of equal ids
    int4 *near = nullptr;
};

struct tr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_cu = 0;
    std::string err;
    int validate = 0; // tr_build_tree checks its cell arrays (tr_ctx_set_validation)
    // device scratch: [0..7] work counters, [16] trace error word, [17] tree error word,
    // [24] largest relative change of a fixed-point sweep
    int *d_ctl = nullptr;
    std::map<std::pair<int, int>, RayTable> tables;
    // pinned host word for reading back the error flag
    int *h_err = nullptr;
    // this device's scratch of the allocation-free dust solve (TR_NOALLOC_DUST_STATES
    // floats, shared by every context on the device; never allocated or freed by a call)
    float *noalloc_guess = nullptr;
    // grow-only workspace for the dust solve's learned starting points
    float *ws_guess = nullptr;
    int64_t ws_guess_n = 0;
    // grow-only per-wave accumulators of the ray tracer's optically thick segment content
    // (kept all-zero between launches: the tracer clears every entry it reads)
    float4 *ws_thick = nullptr;
    int64_t ws_thick_n = 0;
};

struct tr_tree {
    tr_ctx *ctx = nullptr;
    int nb = 0, max_level = 0, n_blk = 0, D = 0;
    int64_t n_fine = 0, root_edge = 0, n_node = 0, n_leaf = 0, n_cells = 0;
    int n_bins = 0;
    double x0[3] = {0, 0, 0}, box_len = 0, u_len = 0, sigma = 0, c_light = 1;
    int64_t depth_off[TR_MAX_DEPTH + 2] = {0};
    // node arrays (SoA, node id order)
    int4 *geo = nullptr;       // centre (u) and first child (-1 for leaves)
    uint32_t *meta = nullptr;  // depth | mask << 4 | leaf << 12 | thick content << 13
    float4 *q = nullptr;       // node content
    float *vthick = nullptr;   // thick volume of h-nodes (u^3)
    int4 *pcol = nullptr;      // mapping position (u / 256); .w = thick volume (float bits)
    int4 *packed = nullptr;    // walk record: centre, depth, flags, child mask, first child
    int32_t *leaf_cell = nullptr;
    // per cell
    int32_t *node_of_cell = nullptr;
    int32_t *targets = nullptr;   // leaf node ids in node order
    int32_t *target_cell = nullptr;
    float *cell_tau = nullptr;    // rho kappa dx
    float *cell_kappa = nullptr;
    float *cell_src = nullptr;    // hosted star luminosity / u_len^2 (0 if none)
    // kept for tr_tree_refill: the FP64 sums of the up-sweep (L_thin, LV_thick, A_thin,
    // A_thick, V_thick, centre-of-luminosity weight; n_node each) and the per-cell star light
    double *s64[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    double *src = nullptr;
};

int tr_fail(tr_ctx *ctx, int code, const char *fmt, ...);

#define TR_HIP(ctx, call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return tr_fail((ctx), TR_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

int tr_get_table(tr_ctx *ctx, int n_side, int cube_m, RayTable **out);
// fills rt.near (allocated here) on the context's stream; the trace's own direction cells
int tr_build_near_table(tr_ctx *ctx, RayTable &rt, int log2m);

static inline int64_t tr_div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }
