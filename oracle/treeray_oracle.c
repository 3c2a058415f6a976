/*
 * TreeRay/RadPressure FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain reference the HIP library is compared against.  It follows
 * Klepitko et al. (MNRAS 2023) step by step, in FP64, with no blocking, fusion or
 * reordering beyond what the paper's definitions state:
 *
 *   tree build ............ Sec. 4.1 (b-nodes), App. A (h-nodes, centre of luminosity)
 *   rays .................. Sec. 4.2 (HEALPix pixels, quadratic evaluation points)
 *   mapping ............... Sec. 4.2, 4.2.1, 4.2.2 (angular and radial kernels)
 *   integration ........... Sec. 4.3 (merging, optical depth, extinction, emission)
 *   finalisation .......... Sec. 4.4
 *   radiation pressure .... Sec. 4.5
 *   dust equilibrium ...... Sec. 4.6, App. E
 *
 * Where the paper is silent or ambiguous the reading taken is stated next to the code
 * that implements it.
 *
 * Parity unpinned: the host-cell source terms J_src (Sec. 4.4) and P_src (Sec. 4.5) follow
 * a reading of definitions the paper leaves open (the source volume and area); nothing
 * outside this code fixes their values, so only their limits are tested.  Likewise the UV
 * radiation-pressure rates of App. C, which are the paper's expressions restated.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg load this code; it shares nothing with the library under paper_2204_09072_amd/.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared  (no fast-math: the fixed
 * operation order below is part of the definition the bit-exact tree test relies on).
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define FX 256 /* fixed-point subdivisions of the lattice unit for mapping positions */

struct or_tree {
    int nb, max_level, n_blk, D;
    int64_t n_fine;    /* finest cells per domain edge */
    int64_t root_edge; /* root edge in lattice units u (u = half the finest cell edge) */
    double x0[3], box_len, u_len, sigma;
    int64_t n_node, n_leaf, n_cells;
    int64_t *depth_off; /* [D+2] */
    uint64_t *key;      /* Morton key at the node's depth */
    int *depth;
    int64_t *g;    /* [n][3] geometric centre (u) */
    int64_t *edge; /* node edge (u) */
    int64_t *first_child;
    uint8_t *mask, *leaf, *thick;
    int64_t *cell, *node_of_cell;
    /* FP64 node content (lattice units: lengths in u, luminosities divided by u_len^2) */
    double *Lt;  /* thin luminosity entering the rays (leaf: L_thin + S, or S if thick) */
    double *LVk; /* thick luminosity per area times volume */
    double *At, *Ak, *Vk, *xi;
    double *Lb;  /* leaf: thin L, or thick luminosity per area (unsigned) */
    double *S, *tau, *Lsrc;
    int64_t *p; /* [n][3] mapping position in 1/FX lattice units */
};

/* ------------------------------------------------------------------------------------
 * Morton keys: bit 3k is x bit k, 3k+1 is y bit k, 3k+2 is z bit k.
 * ---------------------------------------------------------------------------------- */
static uint64_t morton3(uint64_t x, uint64_t y, uint64_t z, int bits) {
    uint64_t k = 0;
    for (int b = 0; b < bits; ++b) {
        k |= ((x >> b) & 1ull) << (3 * b);
        k |= ((y >> b) & 1ull) << (3 * b + 1);
        k |= ((z >> b) & 1ull) << (3 * b + 2);
    }
    return k;
}
static void unmorton3(uint64_t k, int bits, int64_t *x, int64_t *y, int64_t *z) {
    *x = *y = *z = 0;
    for (int b = 0; b < bits; ++b) {
        *x |= (int64_t)((k >> (3 * b)) & 1ull) << b;
        *y |= (int64_t)((k >> (3 * b + 1)) & 1ull) << b;
        *z |= (int64_t)((k >> (3 * b + 2)) & 1ull) << b;
    }
}

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

static int64_t find_key(const uint64_t *keys, int64_t n, uint64_t k) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (keys[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    return (lo < n && keys[lo] == k) ? lo : -1;
}

/* Planck-mean dust opacity (Sec. 2): 0.1 cm^2/g per 100 K^2 times T^2 below 150 K,
 * its 150 K value above. */
static double kappa_planck(double t) { return t < 150.0 ? 1.0e-3 * (t * t) : 22.5; }

/* ------------------------------------------------------------------------------------
 * Tree build
 * ---------------------------------------------------------------------------------- */
void or_tree_free(or_tree *t) {
    if (!t) return;
    free(t->depth_off); free(t->key); free(t->depth); free(t->g); free(t->edge);
    free(t->first_child); free(t->mask); free(t->leaf); free(t->thick); free(t->cell);
    free(t->node_of_cell); free(t->Lt); free(t->LVk); free(t->At); free(t->Ak);
    free(t->Vk); free(t->xi); free(t->Lb); free(t->S); free(t->tau); free(t->Lsrc);
    free(t->p); free(t);
}

or_tree *or_build_tree(int nb, int max_level, int n_blk, const int32_t *blocks,
                       const double *x0, double box_len, const float *rho,
                       const float *kappa, const float *t_dust, int n_star,
                       const double *stars, double sigma) {
    if (nb <= 0 || max_level < 0 || max_level > 8 || n_blk <= 0 || box_len <= 0) return NULL;
    or_tree *t = (or_tree *)calloc(1, sizeof(or_tree));
    t->nb = nb; t->max_level = max_level; t->n_blk = n_blk;
    t->box_len = box_len; t->sigma = sigma;
    for (int a = 0; a < 3; ++a) t->x0[a] = x0[a];
    t->n_fine = (int64_t)nb * 8 << max_level;
    int D = 0;
    while (((int64_t)1 << D) < t->n_fine) ++D;
    t->D = D;
    t->root_edge = (int64_t)2 << D;
    t->u_len = box_len / (2.0 * (double)t->n_fine);
    t->n_cells = (int64_t)n_blk * 512;

    /* every node is an ancestor-or-self of a leaf cell; collect keys per depth */
    int64_t *cnt = (int64_t *)calloc(D + 1, sizeof(int64_t));
    for (int b = 0; b < n_blk; ++b) {
        int lev = blocks[4 * b];
        int64_t nbl = (int64_t)nb << lev;
        if (lev < 0 || lev > max_level) { free(cnt); or_tree_free(t); return NULL; }
        for (int a = 1; a < 4; ++a)
            if (blocks[4 * b + a] < 0 || blocks[4 * b + a] >= nbl) { free(cnt); or_tree_free(t); return NULL; }
        int dc = D - (max_level - lev);
        for (int d = 0; d <= dc; ++d) cnt[d] += 512;
    }
    uint64_t **keys = (uint64_t **)calloc(D + 1, sizeof(uint64_t *));
    int64_t *nk = (int64_t *)calloc(D + 1, sizeof(int64_t));
    for (int d = 0; d <= D; ++d) keys[d] = (uint64_t *)malloc((cnt[d] + 1) * sizeof(uint64_t));
    for (int b = 0; b < n_blk; ++b) {
        int lev = blocks[4 * b];
        int dc = D - (max_level - lev);
        for (int lc = 0; lc < 512; ++lc) {
            int64_t x = (int64_t)blocks[4 * b + 1] * 8 + (lc & 7);
            int64_t y = (int64_t)blocks[4 * b + 2] * 8 + ((lc >> 3) & 7);
            int64_t z = (int64_t)blocks[4 * b + 3] * 8 + (lc >> 6);
            for (int d = 0; d <= dc; ++d)
                keys[d][nk[d]++] = morton3(x >> (dc - d), y >> (dc - d), z >> (dc - d), d);
        }
    }
    t->depth_off = (int64_t *)calloc(D + 2, sizeof(int64_t));
    for (int d = 0; d <= D; ++d) {
        qsort(keys[d], nk[d], sizeof(uint64_t), cmp_u64);
        int64_t u = 0;
        for (int64_t i = 0; i < nk[d]; ++i)
            if (u == 0 || keys[d][i] != keys[d][u - 1]) keys[d][u++] = keys[d][i];
        nk[d] = u;
        t->depth_off[d + 1] = t->depth_off[d] + u;
    }
    int64_t n = t->depth_off[D + 1];
    t->n_node = n;
    t->key = (uint64_t *)malloc(n * sizeof(uint64_t));
    t->depth = (int *)malloc(n * sizeof(int));
    t->g = (int64_t *)malloc(3 * n * sizeof(int64_t));
    t->edge = (int64_t *)malloc(n * sizeof(int64_t));
    t->first_child = (int64_t *)malloc(n * sizeof(int64_t));
    t->mask = (uint8_t *)calloc(n, 1);
    t->leaf = (uint8_t *)calloc(n, 1);
    t->thick = (uint8_t *)calloc(n, 1);
    t->cell = (int64_t *)malloc(n * sizeof(int64_t));
    t->node_of_cell = (int64_t *)malloc(t->n_cells * sizeof(int64_t));
    t->Lt = (double *)calloc(n, sizeof(double));
    t->LVk = (double *)calloc(n, sizeof(double));
    t->At = (double *)calloc(n, sizeof(double));
    t->Ak = (double *)calloc(n, sizeof(double));
    t->Vk = (double *)calloc(n, sizeof(double));
    t->xi = (double *)calloc(n, sizeof(double));
    t->Lb = (double *)calloc(n, sizeof(double));
    t->S = (double *)calloc(n, sizeof(double));
    t->tau = (double *)calloc(n, sizeof(double));
    t->Lsrc = (double *)calloc(n, sizeof(double));
    t->p = (int64_t *)malloc(3 * n * sizeof(int64_t));
    for (int d = 0; d <= D; ++d) {
        int64_t s = t->root_edge >> d;
        for (int64_t i = 0; i < nk[d]; ++i) {
            int64_t id = t->depth_off[d] + i, x, y, z;
            t->key[id] = keys[d][i];
            t->depth[id] = d;
            unmorton3(keys[d][i], d, &x, &y, &z);
            t->g[3 * id] = x * s + s / 2;
            t->g[3 * id + 1] = y * s + s / 2;
            t->g[3 * id + 2] = z * s + s / 2;
            t->edge[id] = s;
            t->first_child[id] = -1;
            t->cell[id] = -1;
        }
    }
    /* leaves: mark cells, detect overlapping blocks */
    int bad = 0;
    for (int b = 0; b < n_blk && !bad; ++b) {
        int lev = blocks[4 * b];
        int dc = D - (max_level - lev);
        for (int lc = 0; lc < 512; ++lc) {
            int64_t x = (int64_t)blocks[4 * b + 1] * 8 + (lc & 7);
            int64_t y = (int64_t)blocks[4 * b + 2] * 8 + ((lc >> 3) & 7);
            int64_t z = (int64_t)blocks[4 * b + 3] * 8 + (lc >> 6);
            int64_t i = find_key(keys[dc], nk[dc], morton3(x, y, z, dc));
            int64_t id = t->depth_off[dc] + i;
            if (t->leaf[id]) { bad = 1; break; }
            t->leaf[id] = 1;
            t->cell[id] = (int64_t)b * 512 + lc;
            t->node_of_cell[(int64_t)b * 512 + lc] = id;
        }
    }
    /* children of h-nodes, in Morton (child index) order */
    for (int d = 0; d < D && !bad; ++d) {
        for (int64_t i = 0; i < nk[d]; ++i) {
            int64_t id = t->depth_off[d] + i;
            for (int k = 0; k < 8; ++k) {
                int64_t c = find_key(keys[d + 1], nk[d + 1], keys[d][i] * 8 + (uint64_t)k);
                if (c < 0) continue;
                if (t->leaf[id]) { bad = 1; break; }
                if (t->first_child[id] < 0) t->first_child[id] = t->depth_off[d + 1] + c;
                t->mask[id] |= (uint8_t)(1u << k);
            }
        }
    }
    t->n_leaf = 0;
    for (int64_t id = 0; id < n; ++id) {
        if (t->leaf[id]) ++t->n_leaf;
        else if (t->first_child[id] < 0) bad = 1; /* cannot happen for well-formed input */
    }
    for (int d = 0; d <= D; ++d) free(keys[d]);
    free(keys); free(nk); free(cnt);
    if (bad || t->n_leaf != t->n_cells) { or_tree_free(t); return NULL; }

    /* point sources: host cell = the leaf containing the star, cells half-open [a, b). */
    const double u2 = t->u_len * t->u_len;
    const double dxmin = box_len / (double)t->n_fine;
    for (int s = 0; s < n_star; ++s) {
        int64_t f[3];
        for (int a = 0; a < 3; ++a) {
            double q = floor((stars[4 * s + a] - x0[a]) / dxmin);
            if (q < 0) q = 0;
            if (q > (double)(t->n_fine - 1)) q = (double)(t->n_fine - 1);
            f[a] = (int64_t)q;
        }
        for (int lev = max_level; lev >= 0; --lev) {
            int sh = max_level - lev, dc = D - sh;
            uint64_t k = morton3(f[0] >> sh, f[1] >> sh, f[2] >> sh, dc);
            int64_t lo = t->depth_off[dc], hi = t->depth_off[dc + 1];
            int64_t i = find_key(t->key + lo, hi - lo, k);
            if (i >= 0 && t->leaf[lo + i]) {
                t->Lsrc[lo + i] = t->Lsrc[lo + i] + stars[4 * s + 3] / u2;
                break;
            }
        }
    }

    /* b-nodes (Sec. 4.1.1): tau = rho kappa dr; thin if tau < 1, thick otherwise.
     * Lattice units: A = rho kappa dV / u_len^2, luminosities / u_len^2. */
    for (int64_t id = 0; id < n; ++id) {
        if (!t->leaf[id]) continue;
        int64_t c = t->cell[id];
        int64_t e = t->edge[id];
        double tt = (double)t_dust[c];
        double kap = kappa ? (double)kappa[c] : kappa_planck(tt);
        double rk = (double)rho[c] * kap;
        double tau = rk * ((double)e * t->u_len);
        double V = (double)e * (double)e * (double)e;
        double A = (rk * t->u_len) * V;
        double sT4 = sigma * ((tt * tt) * (tt * tt));
        double S = t->Lsrc[id] * exp(-0.5 * tau);
        t->tau[id] = tau;
        t->S[id] = S;
        if (tau < 1.0) {
            double L = (4.0 * sT4) * A;  /* 4 sigma rho kappa T^4 dV */
            t->Lb[id] = L;
            t->Lt[id] = L + S;
            t->At[id] = A;
            t->xi[id] = L + S;
        } else {
            double La = sT4 / M_PI;      /* sigma T^4 / pi per unit area */
            t->thick[id] = 1;
            t->Lb[id] = La;
            t->Lt[id] = S;
            t->LVk[id] = La * V;
            t->Ak[id] = A;
            t->Vk[id] = V;
            t->xi[id] = La * ((double)e * (double)e) + S;
        }
        t->p[3 * id] = t->g[3 * id] * FX;
        t->p[3 * id + 1] = t->g[3 * id + 1] * FX;
        t->p[3 * id + 2] = t->g[3 * id + 2] * FX;
    }
    /* h-nodes (App. A): sums over sub-nodes, thin and thick kept apart; the star
     * luminosity S of every b-node enters the thin luminosity.  Centre of luminosity:
     * weights xi = L (thin b-node), L V^(2/3) (thick b-node), L_thin + L_thick V_thick^(2/3)
     * (h-node), positions = the sub-nodes' own mapping positions. */
    for (int d = D - 1; d >= 0; --d) {
        for (int64_t id = t->depth_off[d]; id < t->depth_off[d + 1]; ++id) {
            if (t->leaf[id]) continue;
            double Lt = 0, LVk = 0, At = 0, Ak = 0, Vk = 0, X = 0, num[3] = {0, 0, 0};
            int64_t c = t->first_child[id];
            int64_t g256[3] = {t->g[3 * id] * FX, t->g[3 * id + 1] * FX, t->g[3 * id + 2] * FX};
            for (int k = 0; k < 8; ++k) {
                if (!(t->mask[id] >> k & 1)) continue;
                Lt = Lt + t->Lt[c];
                LVk = LVk + t->LVk[c];
                At = At + t->At[c];
                Ak = Ak + t->Ak[c];
                Vk = Vk + t->Vk[c];
                X = X + t->xi[c];
                for (int a = 0; a < 3; ++a)
                    num[a] = num[a] + t->xi[c] * (double)(t->p[3 * c + a] - g256[a]);
                ++c;
            }
            t->Lt[id] = Lt; t->LVk[id] = LVk; t->At[id] = At; t->Ak[id] = Ak; t->Vk[id] = Vk;
            t->xi[id] = Lt + (Vk > 0.0 ? LVk / cbrt(Vk) : 0.0);
            for (int a = 0; a < 3; ++a)
                t->p[3 * id + a] = g256[a] + (X > 0.0 ? (int64_t)nearbyint(num[a] / X) : 0);
        }
    }
    return t;
}

int64_t or_tree_count(const or_tree *t, int what) {
    switch (what) {
    case 0: return t->n_node;
    case 1: return t->n_leaf;
    case 2: return t->D;
    case 3: return t->root_edge;
    case 4: {
        /* evaluation points R_i = i^2 u (quadratic spacing, Sec. 4.2); the last one is the
         * largest R_i below the domain diagonal sqrt(3) * 2 n_fine u */
        int64_t lim = 3 * (2 * t->n_fine) * (2 * t->n_fine), i = 1;
        while ((i + 1) * (i + 1) * (i + 1) * (i + 1) < lim) ++i;
        return i;
    }
    case 5: return t->n_cells;
    default: return -1;
    }
}
double or_tree_u_len(const or_tree *t) { return t->u_len; }

void or_tree_export(const or_tree *t, int32_t *geo, uint32_t *meta, float *q, float *vthick,
                    int32_t *pcol, int64_t *leaf_cell) {
    for (int64_t id = 0; id < t->n_node; ++id) {
        if (geo) {
            for (int a = 0; a < 3; ++a) geo[4 * id + a] = (int32_t)t->g[3 * id + a];
            geo[4 * id + 3] = (int32_t)t->first_child[id];
        }
        if (meta)
            meta[id] = (uint32_t)t->depth[id] | (uint32_t)t->mask[id] << 4 | (uint32_t)t->leaf[id] << 12 |
                       (uint32_t)(t->Vk[id] > 0.0) << 13;
        if (q) {
            if (t->leaf[id]) {
                float L = (float)t->Lb[id];
                q[4 * id] = t->thick[id] ? copysignf(L, -1.0f) : L;
                q[4 * id + 1] = (float)(t->thick[id] ? t->Ak[id] : t->At[id]);
                q[4 * id + 2] = (float)t->S[id];
                q[4 * id + 3] = 0.0f;
            } else {
                q[4 * id] = (float)t->Lt[id];
                q[4 * id + 1] = (float)t->LVk[id];
                q[4 * id + 2] = (float)t->At[id];
                q[4 * id + 3] = (float)t->Ak[id];
            }
        }
        if (vthick) vthick[id] = t->leaf[id] ? 0.0f : (float)t->Vk[id];
        if (pcol) for (int a = 0; a < 3; ++a) pcol[3 * id + a] = (int32_t)t->p[3 * id + a];
        if (leaf_cell) leaf_cell[id] = t->cell[id];
    }
}

void or_tree_export_f64(const or_tree *t, double *out) {
    for (int64_t id = 0; id < t->n_node; ++id) {
        out[6 * id] = t->Lt[id];
        out[6 * id + 1] = t->LVk[id];
        out[6 * id + 2] = t->At[id];
        out[6 * id + 3] = t->Ak[id];
        out[6 * id + 4] = t->Vk[id];
        out[6 * id + 5] = t->xi[id];
    }
}

/* ------------------------------------------------------------------------------------
 * HEALPix, NESTED numbering (Gorski et al. 2005).  Twelve base faces (0-3 north, 4-7
 * equatorial, 8-11 south), each an n_side x n_side grid; within a face the pixel index
 * interleaves the face coordinates (x in even bits, y in odd bits).
 * ---------------------------------------------------------------------------------- */
static int interleave2(int x, int y) {
    int r = 0;
    for (int b = 0; b < 16; ++b) r |= ((x >> b) & 1) << (2 * b) | ((y >> b) & 1) << (2 * b + 1);
    return r;
}
static void deinterleave2(int v, int *x, int *y) {
    *x = *y = 0;
    for (int b = 0; b < 16; ++b) {
        *x |= ((v >> (2 * b)) & 1) << b;
        *y |= ((v >> (2 * b + 1)) & 1) << b;
    }
}

/* pixel centre: rings of constant z, equally spaced in phi within a ring */
void or_pix2vec(int ns, int pix, double *v) {
    static const int face_row[12] = {2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4};
    static const int face_col[12] = {1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7};
    int face = pix / (ns * ns), x, y;
    deinterleave2(pix % (ns * ns), &x, &y);
    int ring = face_row[face] * ns - x - y - 1; /* 1 .. 4 ns - 1, counted from the north pole */
    int nr, shift;
    double z;
    if (ring < ns) {
        nr = ring; shift = 0;
        z = 1.0 - (double)(nr * nr) / (3.0 * ns * ns);
    } else if (ring > 3 * ns) {
        nr = 4 * ns - ring; shift = 0;
        z = -1.0 + (double)(nr * nr) / (3.0 * ns * ns);
    } else {
        nr = ns; shift = (ring - ns) & 1;
        z = (double)(2 * ns - ring) * 2.0 / (3.0 * ns);
    }
    int jp = (face_col[face] * nr + x - y + 1 + shift) / 2;
    if (jp > 4 * nr) jp -= 4 * nr;
    if (jp < 1) jp += 4 * nr;
    double phi = ((double)jp - 0.5 * (double)(shift + 1)) * (M_PI / 2.0) / (double)nr;
    double st = sqrt((1.0 - z) * (1.0 + z));
    v[0] = st * cos(phi);
    v[1] = st * sin(phi);
    v[2] = z;
}

/* pixel containing a direction */
int or_vec2pix(int ns, double x, double y, double z0) {
    double r = sqrt(x * x + y * y + z0 * z0);
    double z = z0 / r, za = fabs(z);
    double phi = atan2(y, x);
    if (phi < 0) phi += 2.0 * M_PI;
    double tt = phi / (M_PI / 2.0); /* [0, 4) */
    if (tt >= 4.0) tt -= 4.0;
    int face, ix, iy;
    if (za <= 2.0 / 3.0) {
        /* equatorial belt: pixel edges are the lines of constant ns (tt + 1/2 -+ 3z/4) */
        double up = ns * (0.5 + tt - 0.75 * z), dn = ns * (0.5 + tt + 0.75 * z);
        long ju = (long)floor(up), jd = (long)floor(dn);
        long fu = ju / ns, fd = jd / ns;
        if (fu == fd) face = (int)(fu % 4) + 4;
        else if (fu < fd) face = (int)fu;
        else face = (int)fd + 8;
        ix = (int)(jd % ns);
        iy = ns - 1 - (int)(ju % ns);
    } else {
        /* polar caps: distance from the pole scales as sqrt(3 (1 - |z|)) */
        int q = (int)tt;
        if (q > 3) q = 3;
        double tp = tt - q;
        double w = ns * sqrt(3.0 * (1.0 - za));
        long a = (long)floor(tp * w), b = (long)floor((1.0 - tp) * w);
        if (a > ns - 1) a = ns - 1;
        if (b > ns - 1) b = ns - 1;
        if (z > 0) { face = q; ix = ns - 1 - (int)b; iy = ns - 1 - (int)a; }
        else { face = q + 8; ix = (int)a; iy = (int)b; }
    }
    return face * ns * ns + interleave2(ix, iy);
}

/* Angular kernel table (reading of Sec. 4.2: the alpha kernel is tabulated over
 * discrete directions).  Directions are binned on the six faces of a cube, M x M cells
 * per face; each cell holds the pixel of its centre direction.  Face f = 2*axis + (neg),
 * the two other axes in increasing order give the cell coordinates (i, j). */
void or_cube_table(int ns, int M, int32_t *out) {
    for (int f = 0; f < 6; ++f) {
        int ax = f / 2;
        double sgn = (f & 1) ? -1.0 : 1.0;
        int oa = ax == 0 ? 1 : 0, ob = ax == 2 ? 1 : 2;
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                double v[3];
                v[ax] = sgn;
                v[oa] = (2.0 * i + 1.0) / M - 1.0;
                v[ob] = (2.0 * j + 1.0) / M - 1.0;
                out[(f * M + i) * M + j] = or_vec2pix(ns, v[0], v[1], v[2]);
            }
    }
}

/* direction cell of an integer direction vector (exact integer arithmetic) */
static int cube_cell(const int64_t *d, int M) {
    int64_t ax0 = d[0] < 0 ? -d[0] : d[0], ay = d[1] < 0 ? -d[1] : d[1], az = d[2] < 0 ? -d[2] : d[2];
    int ax;
    if (ax0 >= ay && ax0 >= az) ax = 0;
    else if (ay >= az) ax = 1;
    else ax = 2;
    int oa = ax == 0 ? 1 : 0, ob = ax == 2 ? 1 : 2;
    int64_t m = d[ax] < 0 ? -d[ax] : d[ax];
    int f = 2 * ax + (d[ax] < 0 ? 1 : 0);
    int64_t i = ((int64_t)M * (d[oa] + m)) / (2 * m);
    int64_t j = ((int64_t)M * (d[ob] + m)) / (2 * m);
    if (i > M - 1) i = M - 1;
    if (j > M - 1) j = M - 1;
    return (int)((f * M + i) * M + j);
}

/* Tabulated angular kernel (Sec. 4.2: alpha is tabulated over discrete angles and
 * distances).  For a node at least 8 edges away (r / s >= 8) alpha depends on its direction
 * cell and its distance class c = floor(log2(r^2 / s^2)), c = 6 .. 20 (the last class
 * takes everything farther).  The entry of (cell, c) is the share per pixel of the 4^3
 * stratified sub-points of a cube of edge s_c = |d| 2^(-(c + 1/2)/2) centred on the cell's
 * centre direction d, each binned to its direction cell and that cell's pixel.  In exact
 * integers: d = K (2i + 1 - M, 2j + 1 - M, +-M) on the face (K = 2^16), s_c rounded to a
 * multiple of 8 so that the sub-point offsets (2k - 3) s_c / 8 are integers.  Entries
 * hold up to 4 pixels (ascending) with their counts out of 64; a key whose sub-points
 * reach more pixels is marked and its nodes take the per-node kernel. */
#define A_NSUB 4
#define A_CFAR 6
#define A_CMAX 20
#define A_NCLASS (A_CMAX - A_CFAR + 1)
#define A_WIDTH 9 /* pixel 0..3, count 0..3, more-than-4 flag */

static int cube_cell(const int64_t *d, int M);

void or_alpha_table(int M, const int32_t *pixtab, int32_t *out) {
    const int64_t K = (int64_t)1 << 16;
    for (int f = 0; f < 6; ++f) {
        int ax = f / 2;
        int oa = ax == 0 ? 1 : 0, ob = ax == 2 ? 1 : 2;
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                int64_t d[3];
                d[ax] = (f & 1) ? -(int64_t)M * K : (int64_t)M * K;
                d[oa] = K * (2 * i + 1 - M);
                d[ob] = K * (2 * j + 1 - M);
                double len = sqrt((double)d[0] * d[0] + (double)d[1] * d[1] + (double)d[2] * d[2]);
                for (int c = A_CFAR; c <= A_CMAX; ++c) {
                    double x = len * 0.8408964152537145 * ((c & 1) ? 0.7071067811865476 : 1.0) * ldexp(1.0, -(c / 2));
                    int64_t S = 8 * llround(x / 8.0);
                    int pix[64], cnt[64], np = 0;
                    for (int q = 0; q < A_NSUB * A_NSUB * A_NSUB; ++q) {
                        int64_t e[3] = {d[0] + (2 * (q % 4) - 3) * S / 8, d[1] + (2 * ((q / 4) % 4) - 3) * S / 8,
                                        d[2] + (2 * (q / 16) - 3) * S / 8};
                        int px = pixtab[cube_cell(e, M)], k;
                        for (k = 0; k < np; ++k)
                            if (pix[k] == px) break;
                        if (k == np) { pix[np] = px; cnt[np] = 0; ++np; }
                        cnt[k]++;
                    }
                    /* ascending pixel order */
                    for (int a = 1; a < np; ++a)
                        for (int b = a; b > 0 && pix[b - 1] > pix[b]; --b) {
                            int tp = pix[b]; pix[b] = pix[b - 1]; pix[b - 1] = tp;
                            int tc = cnt[b]; cnt[b] = cnt[b - 1]; cnt[b - 1] = tc;
                        }
                    int32_t *o = out + (((int64_t)(f * M + i) * M + j) * A_NCLASS + (c - A_CFAR)) * A_WIDTH;
                    for (int k = 0; k < 4; ++k) {
                        o[k] = k < np && np <= 4 ? pix[k] : 0;
                        o[4 + k] = k < np && np <= 4 ? cnt[k] : 0;
                    }
                    o[8] = np > 4;
                }
            }
    }
}

/* ------------------------------------------------------------------------------------
 * Ray mapping (Sec. 4.2) and integration (Sec. 4.3)
 * ---------------------------------------------------------------------------------- */
enum { B_LT = 0, B_AT, B_LK, B_AK, B_VK, B_Q, NB_FIELDS };

typedef struct {
    const or_tree *t;
    const or_params *p;
    const int32_t *table;
    const int32_t *alpha; /* tabulated kernel, NULL = per-node kernel only */
    int npix, nbins;
    int64_t c[3], c256[3];
    int64_t target;
    int perm[3], sgn[3]; /* orientation of the ray set for this target */
    double *bins;    /* [npix][nbins+1][6] */
    uint8_t *flags;  /* [npix][nbins+1]: merge segment i with i+1 */
    int64_t n_b, n_h, n_open;
} walk_ctx;

/* largest i <= nbins with R_i <= x, where R_i = i^2 (lattice units) and the comparison
 * is exact: R_i + off <= r  <=>  (FX i^2 + off)^2 <= r2 (all in 1/FX units) */
static int bin_below(int64_t r2, int64_t off, int nbins) {
    int i = 0;
    while (i < nbins) {
        int64_t e = (int64_t)FX * (i + 1) * (i + 1) + off;
        if (e > 0 && e * e > r2) break;
        ++i;
    }
    return i;
}

static void map_node(walk_ctx *w, int64_t id) {
    const or_tree *t = w->t;
    int64_t d0[3], dl[3], r2 = 0;
    for (int a = 0; a < 3; ++a) {
        d0[a] = t->p[3 * id + a] - w->c256[a];
        r2 += d0[a] * d0[a];
    }
    /* the node offset in the frame of the (re-oriented) ray set */
    for (int a = 0; a < 3; ++a) dl[a] = w->sgn[a] * d0[w->perm[a]];
    int i = bin_below(r2, 0, w->nbins);
    if (i == 0) return; /* the target's own segment carries nothing (tau_0 = 0) */
    /* radial kernel: beta = R_i^2 / r^2 keeps inverse-square quantities conserved */
    double Ri2fx = (double)((int64_t)FX * i * i) * (double)((int64_t)FX * i * i);
    double beta = Ri2fx / (double)r2;
    /* angular kernel.  Nodes at least 8 edges away: the tabulated kernel of their
     * direction cell and distance class.  Nearer nodes (and table keys reaching more than 4
     * pixels): 2x2x2 stratified sub-points of the node cube around its mapping position,
     * each binned to a direction cell and its pixel; alpha = share per pixel */
    int64_t h = 64 * t->edge[id]; /* a quarter edge in 1/FX units */
    int pix[8], n_pix = 0, cnt[8];
    double denom = 8.0;
    const int64_t s2 = ((int64_t)FX * t->edge[id]) * ((int64_t)FX * t->edge[id]);
    if (w->alpha && r2 >= 64 * s2) {
        int c = A_CFAR;
        while (c < A_CMAX && (s2 << (c + 1)) <= r2) ++c;
        const int32_t *e = w->alpha + ((int64_t)cube_cell(dl, w->p->cube_m) * A_NCLASS + (c - A_CFAR)) * A_WIDTH;
        if (!e[8]) {
            for (int k = 0; k < 4; ++k)
                if (e[4 + k] > 0) { pix[n_pix] = e[k]; cnt[n_pix] = e[4 + k]; ++n_pix; }
            denom = 64.0;
        }
    }
    for (int q = 0; q < 8 && denom == 8.0; ++q) {
        int64_t d[3] = {dl[0] + ((q & 1) ? h : -h), dl[1] + ((q & 2) ? h : -h), dl[2] + ((q & 4) ? h : -h)};
        int px = w->table[cube_cell(d, w->p->cube_m)];
        int k;
        for (k = 0; k < n_pix; ++k)
            if (pix[k] == px) break;
        if (k == n_pix) { pix[n_pix] = px; cnt[n_pix] = 0; ++n_pix; }
        cnt[k]++;
    }
    int has_thick = t->Vk[id] > 0.0;
    int lo = 0, hi = 0;
    if (has_thick && w->p->merge) {
        /* Sec. 4.3: thick material spread over adjacent segments merges them.  Radial
         * extent of the node's material: its mapping distance +- half its edge. */
        int64_t half = (int64_t)FX * t->edge[id] / 2;
        lo = bin_below(r2, half, w->nbins);
        if (lo < 1) lo = 1;
        hi = bin_below(r2, -half, w->nbins);
    }
    int stride = (w->nbins + 1);
    for (int k = 0; k < n_pix; ++k) {
        double al = cnt[k] / denom;
        double *b = w->bins + ((int64_t)pix[k] * stride + i) * NB_FIELDS;
        b[B_LT] += al * beta * t->Lt[id];
        b[B_AT] += al * beta * t->At[id];
        if (has_thick) {
            b[B_LK] += al * t->LVk[id];
            b[B_AK] += al * t->Ak[id];
            b[B_VK] += al * t->Vk[id];
            b[B_Q] += al * beta * t->Vk[id];
            for (int m = lo; m < hi; ++m) w->flags[(int64_t)pix[k] * stride + m] = 1;
        }
    }
}

/* Opening-angle walk (Sec. 4): b-nodes are always accepted; an h-node of edge s whose
 * geometric centre is at distance d is accepted when s / d < theta (exact integers). */
static void walk(walk_ctx *w, int64_t id) {
    const or_tree *t = w->t;
    if (t->leaf[id]) {
        if (id == w->target) return;
        w->n_b++;
        map_node(w, id);
        return;
    }
    int64_t d2 = 0;
    for (int a = 0; a < 3; ++a) {
        int64_t dd = t->g[3 * id + a] - w->c[a];
        d2 += dd * dd;
    }
    int64_t s = t->edge[id], num = w->p->theta_num, den = w->p->theta_den;
    if (s * s * den * den < num * num * d2) {
        w->n_h++;
        map_node(w, id);
        return;
    }
    w->n_open++;
    int64_t c = t->first_child[id];
    for (int k = 0; k < 8; ++k)
        if (t->mask[id] >> k & 1) walk(w, c++);
}

static double phi_ext(double tau) { return tau > 0.0 ? -expm1(-tau) / tau : 1.0; }

/* One ray: merge linked segments (Sec. 4.3), then integrate outwards (Sec. 4.3.1-4.3.2). */
double or_integrate_ray(int ns, int nbins, const double *bins, const uint8_t *flags, double j_bg) {
    const double npix = 12.0 * ns * ns;
    const double om = 4.0 * M_PI / npix;
    double eps_thin_tau = 0.0, eps_thick = 1.0, Fh = 0.0;
    int k = 1;
    while (k <= nbins) {
        int i = k;
        double s[NB_FIELDS];
        for (int f = 0; f < NB_FIELDS; ++f) s[f] = bins[(int64_t)k * NB_FIELDS + f];
        while (flags[k] && k < nbins) {
            ++k;
            /* inverse-square content of segment k moves to R_i: factor R_i^2 / R_k^2 */
            double T = ((double)i * i * i * i) / ((double)k * k * k * k);
            const double *b = bins + (int64_t)k * NB_FIELDS;
            s[B_LT] += T * b[B_LT];
            s[B_AT] += T * b[B_AT];
            s[B_Q] += T * b[B_Q];
            s[B_LK] += b[B_LK];
            s[B_AK] += b[B_AK];
            s[B_VK] += b[B_VK];
        }
        double R2 = (double)i * i * i * i;
        double tau_thin = s[B_AT] / (om * R2);
        double omt = 0.0, tau_thick = 0.0, Fk = 0.0;
        if (s[B_VK] > 0.0) {
            double c = cbrt(s[B_VK]);
            omt = (s[B_Q] / s[B_VK]) * (c * c) / R2;
            if (omt > om) omt = om;
            if (omt > 0.0) tau_thick = s[B_AK] / (omt * R2);
            Fk = omt * s[B_LK] / s[B_VK];
        }
        double f = omt / om;
        double Ft = phi_ext(tau_thin) * s[B_LT] / (4.0 * M_PI * R2);
        double den = s[B_AT] + f * s[B_AK];
        double Fs = den > 0.0 ? (Ft * s[B_AT] + Fk * f * s[B_AK]) / den : Ft;
        double eps = exp(-eps_thin_tau) * eps_thick;
        Fh += eps * Fs;
        eps_thin_tau += tau_thin;
        eps_thick *= (1.0 - f) + f * exp(-tau_thick);
        ++k;
    }
    Fh += exp(-eps_thin_tau) * eps_thick * om * j_bg;
    return Fh;
}

/* Orientation of the ray set (Sec. 7.6 names different HEALPix orientations as the remedy for
 * ray artefacts): one of the 48 signed permutations of the axes, which
 * map the integer lattice onto itself.  Index o: axis permutation o / 8 (in the order
 * 012 021 102 120 201 210), sign flip of axis a when bit a of o % 8 is set; a node offset
 * d becomes (s_0 d[p_0], s_1 d[p_1], s_2 d[p_2]).  A per-target draw uses the SplitMix64
 * generator (Steele, Lea and Flood 2014) of seed * 2^32 + cell. */
static uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

static void orientation(const or_params *p, int64_t cell, int *perm, int *sgn) {
    static const int P[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int o = p->orient;
    if (o < 0) o = (int)(splitmix64(((uint64_t)p->orient_seed << 32) | (uint64_t)(uint32_t)cell) % 48u);
    for (int a = 0; a < 3; ++a) {
        perm[a] = P[o >> 3][a];
        sgn[a] = ((o >> a) & 1) ? -1 : 1;
    }
}

static int trace_target(const or_tree *t, const or_params *p, const int32_t *table,
                        const int32_t *alpha, const double *dirs, int64_t cell, int brute, double *bins,
                        uint8_t *flags, double *Fh_out, double *tau_out, double *J,
                        double *F, int64_t *counters) {
    const int npix = 12 * p->n_side * p->n_side;
    const int nbins = (int)or_tree_count(t, 4);
    const int stride = nbins + 1;
    walk_ctx w;
    memset(&w, 0, sizeof(w));
    w.t = t; w.p = p; w.table = table; w.alpha = alpha; w.npix = npix; w.nbins = nbins;
    w.target = t->node_of_cell[cell];
    orientation(p, cell, w.perm, w.sgn);
    for (int a = 0; a < 3; ++a) {
        w.c[a] = t->g[3 * w.target + a];
        w.c256[a] = w.c[a] * FX;
    }
    w.bins = bins; w.flags = flags;
    memset(bins, 0, sizeof(double) * (size_t)npix * stride * NB_FIELDS);
    memset(flags, 0, (size_t)npix * stride);
    if (brute) {
        for (int64_t id = 0; id < t->n_node; ++id)
            if (t->leaf[id] && id != w.target) { w.n_b++; map_node(&w, id); }
    } else {
        walk(&w, 0);
    }
    double Fv[3] = {0, 0, 0}, Js = 0.0;
    for (int h = 0; h < npix; ++h) {
        const double *b = bins + (int64_t)h * stride * NB_FIELDS;
        double Fh = or_integrate_ray(p->n_side, nbins, b, flags + (int64_t)h * stride, p->j_bg);
        if (Fh_out) Fh_out[h] = Fh;
        if (tau_out) {
            double s = 0.0;
            for (int i = 1; i <= nbins; ++i)
                s += b[(int64_t)i * NB_FIELDS + B_AT] / ((4.0 * M_PI / npix) * ((double)i * i * i * i));
            tau_out[h] = s;
        }
        /* Sec. 4.4: the radiation moves against the ray direction */
        for (int a = 0; a < 3; ++a) Fv[a] -= Fh * dirs[3 * h + a];
        Js += Fh;
    }
    int64_t tn = w.target;
    double Jsrc = 0.0;
    if (t->Lsrc[tn] > 0.0) {
        /* eq. for J_src with V_src = the host b-node and a 1/(4 pi) turning the absorbed
         * flux into a mean intensity */
        double e = (double)t->edge[tn];
        Jsrc = -expm1(-0.5 * t->tau[tn]) * t->Lsrc[tn] / (4.0 * M_PI * (e * e));
    }
    if (J) *J = Js / (4.0 * M_PI) + Jsrc;
    /* Fv is in the ray set's frame: back to the grid's axes */
    if (F) for (int a = 0; a < 3; ++a) F[w.perm[a]] = w.sgn[a] * Fv[a];
    if (counters) { counters[0] = w.n_b; counters[1] = w.n_h; counters[2] = w.n_open; }
    return 0;
}

static int check_params(const or_tree *t, const or_params *p) {
    if (!t || !p) return -1;
    if (p->n_side < 1 || p->n_side > 64 || (p->n_side & (p->n_side - 1))) return -1;
    if (p->theta_num < 0 || p->theta_den <= 0 || p->cube_m < 1) return -1;
    if (p->orient < -1 || p->orient > 47) return -1;
    return 0;
}

static int32_t *alpha_for(const or_params *p, const int32_t *table) {
    if (!p->alpha_table) return NULL;
    const int M = p->cube_m;
    int32_t *a = (int32_t *)malloc(sizeof(int32_t) * (size_t)6 * M * M * A_NCLASS * A_WIDTH);
    or_alpha_table(M, table, a);
    return a;
}

int or_trace(const or_tree *t, const or_params *p, int64_t n, const int64_t *cells,
             double *J, double *F, int64_t *counters, int n_threads) {
    if (check_params(t, p)) return -1;
    const int npix = 12 * p->n_side * p->n_side;
    const int nbins = (int)or_tree_count(t, 4);
    int32_t *table = (int32_t *)malloc(sizeof(int32_t) * 6 * (size_t)p->cube_m * p->cube_m);
    double *dirs = (double *)malloc(sizeof(double) * 3 * npix);
    or_cube_table(p->n_side, p->cube_m, table);
    int32_t *alpha = alpha_for(p, table);
    for (int h = 0; h < npix; ++h) or_pix2vec(p->n_side, h, dirs + 3 * h);
    int err = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#endif
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1)
    {
        double *bins = (double *)malloc(sizeof(double) * (size_t)npix * (nbins + 1) * NB_FIELDS);
        uint8_t *flags = (uint8_t *)malloc((size_t)npix * (nbins + 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < n; ++k) {
            int64_t cell = cells ? cells[k] : k;
            if (cell < 0 || cell >= t->n_cells) { err = -1; continue; }
            trace_target(t, p, table, alpha, dirs, cell, 0, bins, flags, NULL, NULL,
                         J ? J + k : NULL, F ? F + 3 * k : NULL, counters ? counters + 3 * k : NULL);
        }
        free(bins); free(flags);
    }
    free(table); free(alpha); free(dirs);
    return err;
}

int or_trace_one(const or_tree *t, const or_params *p, int64_t cell, int brute, double *bins,
                 uint8_t *flags, double *Fh, double *tau_thin_tot, double *J, double *F) {
    if (check_params(t, p) || cell < 0 || cell >= t->n_cells) return -1;
    const int npix = 12 * p->n_side * p->n_side;
    int32_t *table = (int32_t *)malloc(sizeof(int32_t) * 6 * (size_t)p->cube_m * p->cube_m);
    double *dirs = (double *)malloc(sizeof(double) * 3 * npix);
    or_cube_table(p->n_side, p->cube_m, table);
    int32_t *alpha = alpha_for(p, table);
    for (int h = 0; h < npix; ++h) or_pix2vec(p->n_side, h, dirs + 3 * h);
    trace_target(t, p, table, alpha, dirs, cell, brute, bins, flags, Fh, tau_thin_tot, J, F, NULL);
    free(table); free(alpha); free(dirs);
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Direct ray marching without the tree: a brute-force reference for the method's
 * end-to-end error (the tree walk, the radial and angular kernels and the segment
 * integration of Sec. 4.2-4.3 are all bypassed).  A ray from point p along the unit
 * vector u crosses the cells of a uniform n^3 grid over [0, box)^3 one by one (the
 * cell-stepping traversal of Amanatides & Woo 1987); a crossing of length l through a
 * cell of absorption coefficient k (= rho kappa, per unit length) and source function B
 * adds B (1 - e^{-k l}) e^{-tau} to the intensity (the formal solution of the transfer
 * equation of Sec. 2 for a piecewise constant medium) and k l to the optical depth tau.
 * Dense cell arrays are indexed (i n + j) n + k for the cell (i, j, k) along (x, y, z).
 * skip_own: the start cell neither absorbs nor emits (the reading of the target's own
 * segment, which carries nothing in the tree method).
 * ---------------------------------------------------------------------------------- */
double or_march(int n, double box, const double *kr, const double *B, const double *p,
                const double *u, int skip_own, double *tau_out) {
    const double dx = box / n;
    int64_t c[3];
    int step[3];
    double tmax[3], tdel[3];
    for (int a = 0; a < 3; ++a) {
        c[a] = (int64_t)floor(p[a] / dx);
        if (c[a] < 0) c[a] = 0;
        if (c[a] > n - 1) c[a] = n - 1;
        if (u[a] > 0.0) {
            step[a] = 1;
            tmax[a] = ((double)(c[a] + 1) * dx - p[a]) / u[a];
            tdel[a] = dx / u[a];
        } else if (u[a] < 0.0) {
            step[a] = -1;
            tmax[a] = ((double)c[a] * dx - p[a]) / u[a];
            tdel[a] = -dx / u[a];
        } else {
            step[a] = 0;
            tmax[a] = INFINITY;
            tdel[a] = INFINITY;
        }
    }
    double t = 0.0, tau = 0.0, I = 0.0;
    int first = 1;
    for (;;) {
        int a = 0;
        if (tmax[1] < tmax[a]) a = 1;
        if (tmax[2] < tmax[a]) a = 2;
        const double l = tmax[a] - t;
        if (!(first && skip_own) && l > 0.0) {
            const int64_t id = (c[0] * n + c[1]) * n + c[2];
            const double dt = kr[id] * l;
            I += B[id] * (-expm1(-dt)) * exp(-tau);
            tau += dt;
        }
        first = 0;
        t = tmax[a];
        c[a] += step[a];
        if (c[a] < 0 || c[a] >= n) break;
        tmax[a] += tdel[a];
    }
    if (tau_out) *tau_out = tau;
    return I;
}

/* Mean intensity at each of n_pt points from direct marching: every ray h of the
 * N_side = ns HEALPix set is sampled by its 4^sub NESTED sub-pixels at N_side ns 2^sub
 * (equal-area, so the plain mean over them is the pixel average), J = the mean of the
 * intensities over all of them.  esc_out[n_pt] (may be NULL) receives the mean of
 * 1 - e^{-tau} over the same directions (the absorbed fraction of a point source's
 * light). */
void or_march_mean(int n, double box, const double *kr, const double *B, int64_t n_pt,
                   const double *pts, int ns, int sub, int skip_own, double *J, double *absorbed) {
    const int64_t nsub = (int64_t)1 << (2 * sub), nfine = 12 * (int64_t)ns * ns * nsub;
    const int nsf = ns << sub;
    double *dirs = (double *)malloc(sizeof(double) * 3 * nfine);
    for (int64_t q = 0; q < nfine; ++q) or_pix2vec(nsf, (int)q, dirs + 3 * q);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < n_pt; ++k) {
        double sI = 0.0, sA = 0.0;
        for (int64_t q = 0; q < nfine; ++q) {
            double tau;
            sI += or_march(n, box, kr, B, pts + 3 * k, dirs + 3 * q, skip_own, &tau);
            sA += -expm1(-tau);
        }
        if (J) J[k] = sI / (double)nfine;
        if (absorbed) absorbed[k] = sA / (double)nfine;
    }
    free(dirs);
}

/* pixel of each of n directions [n][3] */
void or_vec2pix_many(int ns, int64_t n, const double *v, int32_t *out) {
    for (int64_t k = 0; k < n; ++k) out[k] = or_vec2pix(ns, v[3 * k], v[3 * k + 1], v[3 * k + 2]);
}

/* ------------------------------------------------------------------------------------
 * Radiation pressure (Sec. 4.5): a = kappa F / c * (1 - e^-tau) / tau with the factor
 * taken as 1 below tau = 1e-4; trapped pressure of a hosted source uses the host
 * cell's face area dV^(2/3).
 * ---------------------------------------------------------------------------------- */
void or_rad_force(const or_tree *t, const float *rho, const float *kappa, const float *t_dust,
                  const double *F, double c, double *a, double *p_src) {
    for (int64_t id = 0; id < t->n_node; ++id) {
        if (!t->leaf[id]) continue;
        int64_t cell = t->cell[id];
        double tt = (double)t_dust[cell];
        double kap = kappa ? (double)kappa[cell] : kappa_planck(tt);
        double tau = t->tau[id];
        (void)rho;
        double fac = tau < 1e-4 ? 1.0 : -expm1(-tau) / tau;
        for (int k = 0; k < 3; ++k) a[3 * cell + k] = kap * F[3 * cell + k] / c * fac;
        double e = (double)t->edge[id];
        p_src[cell] = t->Lsrc[id] > 0.0 ? -expm1(-0.5 * tau) * t->Lsrc[id] / (c * (e * e)) : 0.0;
    }
}

/* ------------------------------------------------------------------------------------
 * Dust thermal equilibrium (Sec. 4.6, App. E).  Cooling 4 sigma rho kappa(T_d) T_d^4
 * (times xi), heating 4 pi rho kappa(T_J) J (times xi), gas-dust coupling
 * C_gd n_H^2 sqrt(T_g) (T_g - T_d) (1 - 0.8 exp(-75/T_g)), n_H = rho / (1.4 m_H).
 * The residual is strictly increasing in T_d, so the root is unique; floor 2.7 K.
 * ---------------------------------------------------------------------------------- */
#define OR_TFLOOR 2.7
#define OR_MH 1.6735575e-24

double or_dust_residual(double T, double rho, double u_rad, double t_gas, double sigma,
                        double c, double c_gd, double xi) {
    double J = u_rad * c / (4.0 * M_PI);
    double TJ = pow(M_PI * J / sigma, 0.25);
    double nH = rho / (1.4 * OR_MH);
    double cool = xi * 4.0 * sigma * rho * kappa_planck(T) * ((T * T) * (T * T));
    double heat = xi * 4.0 * M_PI * rho * kappa_planck(TJ) * J;
    double gd = c_gd * nH * nH * sqrt(t_gas) * (t_gas - T) * (1.0 - 0.8 * exp(-75.0 / t_gas));
    return cool - heat - gd;
}

void or_dust_eq(int64_t n, const double *rho, const double *u_rad, const double *t_gas,
                double sigma, double c, double c_gd, double xi, double *t_dust, int *iters) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double J = u_rad[k] * c / (4.0 * M_PI);
        double TJ = pow(M_PI * J / sigma, 0.25);
        double tg = t_gas[k];
        double lo = fmax(OR_TFLOOR, fmin(tg, TJ));
        double hi = fmax(OR_TFLOOR, fmax(tg, TJ));
        int it = 0;
        double T;
        if (or_dust_residual(lo, rho[k], u_rad[k], tg, sigma, c, c_gd, xi) >= 0.0) {
            T = lo; /* root at or below the floor (or exactly at the lower bracket end) */
        } else {
            while (hi - lo > 1e-13 * hi && it < 200) {
                double mid = 0.5 * (lo + hi);
                if (or_dust_residual(mid, rho[k], u_rad[k], tg, sigma, c, c_gd, xi) < 0.0) lo = mid;
                else hi = mid;
                ++it;
            }
            T = 0.5 * (lo + hi);
        }
        t_dust[k] = T < OR_TFLOOR ? OR_TFLOOR : T;
        if (iters) iters[k] = it;
    }
}

/* ------------------------------------------------------------------------------------
 * MLP 3 -> H -> H -> 1 with ReLU hidden activations, max(a, 0) (guess of the equilibrium
 * solve; the network is not part of the paper, its architecture is this library's choice)
 * ---------------------------------------------------------------------------------- */
static double to_bf16(double v) {
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) != 0x7f800000u) {
        uint32_t lsb = (u >> 16) & 1u;
        u += 0x7fffu + lsb;
    }
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

double or_mlp(int H, const double *prm, int64_t n, const double *x, const double *y,
              int rb, double *out, double *grad) {
    const double *W1 = prm, *b1 = W1 + 3 * H, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H,
                 *b3 = W3 + H;
    const int np = 3 * H + H + H * H + H + H + 1;
    if (H > 1024) return -1.0;
    if (grad) memset(grad, 0, sizeof(double) * np);
    double *g1 = grad, *gb1 = grad ? g1 + 3 * H : NULL, *g2 = grad ? gb1 + H : NULL,
           *gb2 = grad ? g2 + H * H : NULL, *g3 = grad ? gb2 + H : NULL, *gb3 = grad ? g3 + H : NULL;
    double *h1 = (double *)malloc(sizeof(double) * H), *h2 = (double *)malloc(sizeof(double) * H),
           *d2 = (double *)malloc(sizeof(double) * H), *d1 = (double *)malloc(sizeof(double) * H);
    double loss = 0.0;
    for (int64_t s = 0; s < n; ++s) {
        double xi[3];
        for (int k = 0; k < 3; ++k) xi[k] = rb ? to_bf16(x[3 * s + k]) : x[3 * s + k];
        for (int j = 0; j < H; ++j) {
            double a = b1[j];
            for (int k = 0; k < 3; ++k) a += W1[3 * j + k] * xi[k];
            h1[j] = a > 0.0 ? a : 0.0;
        }
        double h1r[1024];
        for (int j = 0; j < H; ++j) h1r[j] = rb ? to_bf16(h1[j]) : h1[j];
        for (int j = 0; j < H; ++j) {
            double a = b2[j];
            for (int k = 0; k < H; ++k) a += W2[H * j + k] * h1r[k];
            h2[j] = a > 0.0 ? a : 0.0;
        }
        double h2r[1024];
        for (int j = 0; j < H; ++j) h2r[j] = rb ? to_bf16(h2[j]) : h2[j];
        double o = b3[0];
        for (int k = 0; k < H; ++k) o += W3[k] * h2r[k];
        if (out) out[s] = o;
        double r = y ? o - y[s] : 0.0;
        loss += r * r;
        if (grad && y) {
            double dy = 2.0 * r / (double)n;
            gb3[0] += dy;
            for (int k = 0; k < H; ++k) {
                g3[k] += dy * h2r[k];
                d2[k] = h2[k] > 0.0 ? dy * W3[k] : 0.0; /* ReLU passes the gradient where active */
            }
            for (int j = 0; j < H; ++j) {
                gb2[j] += d2[j];
                for (int k = 0; k < H; ++k) g2[H * j + k] += d2[j] * h1r[k];
            }
            for (int k = 0; k < H; ++k) {
                double a = 0.0;
                for (int j = 0; j < H; ++j) a += W2[H * j + k] * d2[j];
                d1[k] = h1[k] > 0.0 ? a : 0.0;
            }
            for (int j = 0; j < H; ++j) {
                gb1[j] += d1[j];
                for (int k = 0; k < 3; ++k) g1[3 * j + k] += d1[j] * xi[k];
            }
        }
    }
    free(h1); free(h2); free(d2); free(d1);
    return n > 0 ? loss / (double)n : 0.0;
}

/* ------------------------------------------------------------------------------------
 * Stellar luminosity split (Sec. 7.2) and UV radiation pressure (App. C)
 * ---------------------------------------------------------------------------------- */
/* Lyman-continuum fraction of a black body at temperature T (eq. for gamma(T_X) in
 * Sec. 7.2): with x0 = h nu_LyC / (k T) = t_lyc / T and the Planck integral
 * I(x0) = int_x0^inf x^3 / (e^x - 1) dx, gamma = I(x0) / I(0), I(0) = pi^4 / 15.
 * x0 >= 2: I = sum_k e^{-k x0} (x0^3/k + 3 x0^2/k^2 + 6 x0/k^3 + 6/k^4) (term-wise
 * integration of the geometric series of 1/(e^x - 1)); x0 < 2: I = pi^4/15 - int_0^x0,
 * with x/(e^x - 1) = sum_n B_n x^n / n! (Bernoulli numbers, |x| < 2 pi) integrated
 * term by term: int_0^x0 = sum_n B_n x0^(n+3) / (n! (n+3)). */
double or_lyman_fraction(double T, double t_lyc) {
    if (!(T > 0.0)) return 0.0;
    const double x0 = t_lyc / T;
    const double I0 = pow(M_PI, 4) / 15.0;
    if (x0 >= 2.0) {
        double s = 0.0;
        for (int k = 1; k <= 200; ++k) {
            double e = exp(-k * x0);
            double term = e * (x0 * x0 * x0 / k + 3.0 * x0 * x0 / ((double)k * k) +
                               6.0 * x0 / ((double)k * k * k) + 6.0 / ((double)k * k * k * k));
            s += term;
            if (term < 1e-18 * s) break;
        }
        return s / I0;
    }
    /* Bernoulli numbers B_0 .. B_30 (B_1 = -1/2, odd ones beyond vanish) */
    static const double B[31] = {1.0, -0.5, 1.0 / 6, 0, -1.0 / 30, 0, 1.0 / 42, 0, -1.0 / 30, 0, 5.0 / 66, 0,
                                 -691.0 / 2730, 0, 7.0 / 6, 0, -3617.0 / 510, 0, 43867.0 / 798, 0,
                                 -174611.0 / 330, 0, 854513.0 / 138, 0, -236364091.0 / 2730, 0,
                                 8553103.0 / 6, 0, -23749461029.0 / 870, 0, 8615841276005.0 / 14322};
    double low = 0.0, fact = 1.0, pw = x0 * x0 * x0;
    for (int n = 0; n <= 30; ++n) {
        if (n > 0) fact *= n;
        low += B[n] * pw / (fact * (n + 3));
        pw *= x0;
    }
    return (I0 - low) / I0;
}

void or_luminosity_split(int n, const double *L_int, const double *L_acc, const double *r_star,
                         double f_fill, double sigma, double t_lyc, double *L_uv, double *L_ir) {
    for (int s = 0; s < n; ++s) {
        /* effective temperatures of the photosphere and of the accretion hot spots */
        double area = 4.0 * M_PI * r_star[s] * r_star[s];
        double T_int = pow(L_int[s] / (sigma * area), 0.25);
        double T_acc = pow(L_acc[s] / (f_fill * sigma * area), 0.25);
        double uv = or_lyman_fraction(T_int, t_lyc) * L_int[s] + or_lyman_fraction(T_acc, t_lyc) * L_acc[s];
        L_uv[s] = uv;
        L_ir[s] = L_int[s] + L_acc[s] - uv;
    }
}

/* App. C: momentum deposited per unit time and volume on dust (sigma_d n), neutral
 * hydrogen (sigma_H n_H0) and, through recombinations balanced by absorptions, ionised
 * hydrogen (alpha_B n_H+^2), for a photon number flux N of mean energy E along u; n =
 * rho / (mu m_H) hydrogen nuclei, n_H0 = (1 - x) n, n_H+ = x n.  a = total / rho. */
void or_uv_rad_pressure(int64_t n, const double *rho, const double *x_ion, const double *nph,
                        const double *uph, double e_ph, double sigma_d, double sigma_h, double alpha_b,
                        double mu_mh, double c, double *a, double *parts) {
    for (int64_t i = 0; i < n; ++i) {
        double nh = rho[i] / mu_mh, x = x_ion[i];
        double p = e_ph / c;
        double pd = sigma_d * nh * p * nph[i];
        double ph = sigma_h * (1.0 - x) * nh * p * nph[i];
        double pi = (x * nh) * (x * nh) * alpha_b * p;
        for (int k = 0; k < 3; ++k) a[3 * i + k] = (pd + ph + pi) * uph[3 * i + k] / rho[i];
        if (parts) { parts[3 * i] = pd; parts[3 * i + 1] = ph; parts[3 * i + 2] = pi; }
    }
}
