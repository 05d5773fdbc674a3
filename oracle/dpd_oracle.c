/*
 * dpd_oracle.c -- plain, slow, FP64 CPU reference of the DPD hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library under paper_1311_0402_amd/) never calls it and shares no code,
 * header, table or constant with it.
 *
 * Source: Tang & Karniadakis, "Accelerating Dissipative Particle Dynamics
 * Simulations on GPUs" (arXiv 1311.0402).  Every function names the passage
 * it follows.  Where the paper is silent the reading is stated inline and in
 * the design notes (readings A1-A25 of the hot-path scope).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA contraction,
 * so every fma() below is the only fused operation).
 *
 * Conventions: positions/velocities/forces are structure-of-arrays
 * double[3][n] (x row, y row, z row).  Tags are uint32, types uint8,
 * type-pair tables are dense row-major double[n_types * n_types].
 * Neighbour lists are CSR: off[n_rows + 1], idx[off[n_rows]], each row
 * ascending.  Functions return 0 (or a count >= 0) on success, < 0 on error.
 *
 * Pins (tests/test_oracle_pins.py): Philox against an independent library
 * engine; xi moments / symmetry; closed-form two-particle forces; brute-force
 * vs cell-list neighbour sets; Morton rank by sort vs by counting; Newton's
 * third law (momentum); ballistic motion; harmonic dimer period; k_BT from
 * the fluctuation-dissipation relation; Poiseuille parabola; finite
 * differences for the vector-Jacobian products.  No function here is parity
 * unpinned.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_TYPES 8

typedef struct orc_params {
    double box[3];      /* periodic box lengths L_x, L_y, L_z               */
    double r_c;         /* cutoff of Eqs (3)-(6)                             */
    double r_list;      /* neighbour radius r_c + skin                       */
    double s;           /* weight exponent of Eq (8)                         */
    double dt;          /* time step (enters F^R as dt^-1/2, Eq (5))         */
    double lambda;      /* Groot-Warren velocity-prediction factor           */
    int32_t n_types;
    double a[ORC_MAX_TYPES * ORC_MAX_TYPES];
    double gamma[ORC_MAX_TYPES * ORC_MAX_TYPES];
    double sigma[ORC_MAX_TYPES * ORC_MAX_TYPES];
    uint64_t seed;
    double body_g;      /* F_x += +g for y < body_split, -g otherwise        */
    double body_split;
    double bond_k;      /* harmonic bond F = -k (r - r0) e                   */
    double bond_r0;
    const int32_t* partner; /* int32[2 * n] by tag, -1 = none; NULL = no bonds */
} orc_params;

/* ------------------------------------------------------------------------ */
/* Random numbers (Sec. 3.5: one Gaussian per pair, regenerated in situ from */
/* particle tags, the time step and a global seed).  The hash is Philox4x32  */
/* with 10 rounds as defined by Salmon, Moraes, Dror & Shaw (SC'11,          */
/* "Parallel random numbers: as easy as 1, 2, 3").                           */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t mult0 = 0xD2511F53u, mult1 = 0xCD9E8D57u;   /* round multipliers */
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;   /* key schedule      */
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)mult0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)mult1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += weyl0;
        k1 += weyl1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

void orc_philox_batch(int64_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out)
{
    for (int64_t i = 0; i < n; ++i)
        orc_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

/* xi_ij: counter (min tag, max tag, low/high word of the step), key = the two
 * words of the seed; uniforms u1 = (w0 + 1/2) 2^-32 in (0,1), u2 = w1 2^-32;
 * first Box-Muller output sqrt(-2 ln u1) cos(2 pi u2) (Sec. 3.5, the z_1
 * form).  Symmetric in (t_i, t_j) by construction. */
double orc_xi(uint32_t ti, uint32_t tj, uint64_t step, uint64_t seed)
{
    uint32_t ctr[4], key[2], w[4];
    ctr[0] = ti < tj ? ti : tj;
    ctr[1] = ti < tj ? tj : ti;
    ctr[2] = (uint32_t)step;
    ctr[3] = (uint32_t)(step >> 32);
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    orc_philox4x32_10(ctr, key, w);
    double u1 = ((double)w[0] + 0.5) * 0x1p-32;
    double u2 = (double)w[1] * 0x1p-32;
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

void orc_xi_batch(int64_t n, const uint32_t* ti, const uint32_t* tj, uint64_t step,
                  uint64_t seed, double* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = orc_xi(ti[i], tj[i], step, seed);
}

/* ------------------------------------------------------------------------ */
/* Geometry: minimum-image separation r_ij = r_i - r_j (reading A1).         */
/* Subtract first, then shift by one box length.                             */
/* ------------------------------------------------------------------------ */

static double min_image(double d, double L)
{
    if (d > 0.5 * L) d = d - L;
    else if (d < -0.5 * L) d = d + L;
    return d;
}

static double separation(const double* x, int64_t n, int64_t i, int64_t j,
                         const double box[3], double d[3])
{
    for (int k = 0; k < 3; ++k) d[k] = min_image(x[k * n + i] - x[k * n + j], box[k]);
    return fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0]));
}

/* ------------------------------------------------------------------------ */
/* Cell grid and reordering (Sec. 3.2.2-3.2.3): cells of side >= r_list,     */
/* ordered along a Morton curve; particles of one cell get consecutive       */
/* indices.  Inside a cell the order is by tag (the paper's second Morton    */
/* level is replaced by this total order).                                   */
/* ------------------------------------------------------------------------ */

int orc_cell_grid(const double box[3], double r_list, int32_t nc[3])
{
    if (!(r_list > 0.0)) return -1;
    for (int k = 0; k < 3; ++k) {
        if (!(box[k] > 0.0)) return -1;
        double q = floor(box[k] / r_list);
        if (q > 1.0e6) return -1;
        int32_t m = (int32_t)q;
        /* margin: a cell must be wider than r_list by a relative 2^-40 */
        while (m > 0 && box[k] / (double)m < r_list * (1.0 + 0x1p-40)) --m;
        if (m < 3) return -1;
        nc[k] = m;
    }
    return 0;
}

static uint64_t morton3(uint32_t cx, uint32_t cy, uint32_t cz)
{
    uint64_t code = 0;
    for (int b = 0; b < 21; ++b) {
        code |= (uint64_t)((cx >> b) & 1u) << (3 * b);
        code |= (uint64_t)((cy >> b) & 1u) << (3 * b + 1);
        code |= (uint64_t)((cz >> b) & 1u) << (3 * b + 2);
    }
    return code;
}

typedef struct { uint64_t key; int64_t id; } orc_kv;

static int cmp_kv(const void* pa, const void* pb)
{
    const orc_kv* a = (const orc_kv*)pa;
    const orc_kv* b = (const orc_kv*)pb;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    if (a->id < b->id) return -1;
    if (a->id > b->id) return 1;
    return 0;
}

/* rank[cx + nc0*(cy + nc1*cz)] = position of the cell in ascending Morton code */
int orc_morton_rank_table(const int32_t nc[3], int32_t* rank)
{
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    orc_kv* kv = (orc_kv*)malloc(sizeof(orc_kv) * (size_t)ncell);
    if (!kv) return -1;
    for (int64_t c = 0; c < ncell; ++c) {
        uint32_t cx = (uint32_t)(c % nc[0]);
        uint32_t cy = (uint32_t)((c / nc[0]) % nc[1]);
        uint32_t cz = (uint32_t)(c / ((int64_t)nc[0] * nc[1]));
        kv[c].key = morton3(cx, cy, cz);
        kv[c].id = c;
    }
    qsort(kv, (size_t)ncell, sizeof(orc_kv), cmp_kv);
    for (int64_t r = 0; r < ncell; ++r) rank[kv[r].id] = (int32_t)r;
    free(kv);
    return 0;
}

static void cell_of(const double* x, int64_t n, int64_t i, const int32_t nc[3],
                    const double inv[3], int32_t c[3])
{
    for (int k = 0; k < 3; ++k) {
        int32_t ck = (int32_t)(x[k * n + i] * inv[k]);
        if (ck > nc[k] - 1) ck = nc[k] - 1;
        c[k] = ck;
    }
}

/* perm[new] = old index, sorted by (Morton rank of the particle's cell, tag).
 * cell_start (nullable, n_cells + 1 entries) gets the first new index of
 * every cell in rank order. */
int orc_reorder(int32_t n, const double* x, const uint32_t* tag, const double box[3],
                double r_list, int32_t* perm, int32_t* cell_start)
{
    int32_t nc[3];
    if (orc_cell_grid(box, r_list, nc)) return -1;
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int32_t* rank = (int32_t*)malloc(sizeof(int32_t) * (size_t)ncell);
    orc_kv* kv = (orc_kv*)malloc(sizeof(orc_kv) * (size_t)(n > 0 ? n : 1));
    if (!rank || !kv) { free(rank); free(kv); return -1; }
    orc_morton_rank_table(nc, rank);
    double inv[3];
    for (int k = 0; k < 3; ++k) inv[k] = (double)nc[k] / box[k];
    for (int64_t i = 0; i < n; ++i) {
        int32_t c[3];
        cell_of(x, n, i, nc, inv, c);
        int64_t lin = c[0] + (int64_t)nc[0] * (c[1] + (int64_t)nc[1] * c[2]);
        kv[i].key = ((uint64_t)(uint32_t)rank[lin] << 32) | (uint64_t)tag[i];
        kv[i].id = i;
    }
    qsort(kv, (size_t)n, sizeof(orc_kv), cmp_kv);
    for (int64_t q = 0; q < n; ++q) perm[q] = (int32_t)kv[q].id;
    if (cell_start) {
        for (int64_t r = 0; r <= ncell; ++r) cell_start[r] = 0;
        for (int64_t q = 0; q < n; ++q) cell_start[(kv[q].key >> 32) + 1] += 1;
        for (int64_t r = 0; r < ncell; ++r) cell_start[r + 1] += cell_start[r];
    }
    free(rank);
    free(kv);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Neighbour sets (Sec. 3.3.2; Algorithm 3's strict "<" test): j is a        */
/* neighbour of i iff j != i and |r_ij|^2 < r_list^2.  Rows ascend in j      */
/* (the paper's ordered list).  Brute force over all pairs.                  */
/* ------------------------------------------------------------------------ */

static void exclusive_scan(const int32_t* count, int64_t n, int64_t* off)
{
    off[0] = 0;
    for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + count[i];
}

/* Rows for the query particles q[0..nq) (q == NULL: all particles).
 * count[r] = row length; when list != NULL the rows are written back to back
 * (row r at sum(count[0..r))) provided the total fits in cap.
 * Returns the total, or -1 if it exceeds cap. */
int64_t orc_neighbors_brute(int32_t n, const double* x, const double box[3], double r_list,
                            int32_t nq, const int32_t* q, int32_t* count,
                            int32_t* list, int64_t cap)
{
    const double rl2 = r_list * r_list;
    if (q == NULL) nq = n;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int32_t r = 0; r < nq; ++r) {
        int64_t i = q ? q[r] : r;
        int32_t c = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            if (separation(x, n, i, j, box, d) < rl2) ++c;
        }
        count[r] = c;
    }
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * ((size_t)nq + 1));
    exclusive_scan(count, nq, off);
    int64_t total = off[nq];
    if (list) {
        if (total > cap) { free(off); return -1; }
        #pragma omp parallel for schedule(dynamic, 16)
        for (int32_t r = 0; r < nq; ++r) {
            int64_t i = q ? q[r] : r;
            int64_t w = off[r];
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double d[3];
                if (separation(x, n, i, j, box, d) < rl2) list[w++] = (int32_t)j;
            }
        }
    }
    free(off);
    return total;
}

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Same rows via a cell list (27 surrounding cells of side >= r_list), then
 * each row sorted ascending.  Exists for large systems; the pins require it
 * to equal orc_neighbors_brute exactly. */
static int64_t cells_rows(int32_t n, const double* x, const double box[3], double r_list,
                          int32_t* count, int32_t* list, int64_t cap, int counts_known)
{
    int32_t nc[3];
    if (orc_cell_grid(box, r_list, nc)) return -2;
    const double rl2 = r_list * r_list;
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    double inv[3];
    for (int k = 0; k < 3; ++k) inv[k] = (double)nc[k] / box[k];
    int32_t* pc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t* head = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
    int32_t* members = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncell);
    for (int64_t i = 0; i < n; ++i) {
        int32_t c[3];
        cell_of(x, n, i, nc, inv, c);
        pc[i] = c[0] + nc[0] * (c[1] + nc[1] * c[2]);
        head[pc[i] + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; ++c) head[c + 1] += head[c];
    for (int64_t c = 0; c < ncell; ++c) fill[c] = head[c];
    for (int64_t i = 0; i < n; ++i) members[fill[pc[i]]++] = (int32_t)i;

    for (int pass = counts_known ? 1 : 0; pass < 2; ++pass) {
        int64_t* off = NULL;
        if (pass == 1) {
            if (!list) break;
            off = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
            exclusive_scan(count, n, off);
            if (off[n] > cap) { free(off); free(pc); free(head); free(members); free(fill); return -1; }
        }
        #pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            int32_t ci[3];
            ci[0] = pc[i] % nc[0];
            ci[1] = (pc[i] / nc[0]) % nc[1];
            ci[2] = pc[i] / (nc[0] * nc[1]);
            int32_t c = 0;
            int64_t w = pass ? off[i] : 0;
            for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int32_t cx = (ci[0] + dx + nc[0]) % nc[0];
                int32_t cy = (ci[1] + dy + nc[1]) % nc[1];
                int32_t cz = (ci[2] + dz + nc[2]) % nc[2];
                int64_t cc = cx + (int64_t)nc[0] * (cy + (int64_t)nc[1] * cz);
                for (int64_t m = head[cc]; m < head[cc + 1]; ++m) {
                    int64_t j = members[m];
                    if (j == i) continue;
                    double d[3];
                    if (separation(x, n, i, j, box, d) < rl2) {
                        if (pass) list[w] = (int32_t)j;
                        ++w;
                        ++c;
                    }
                }
            }
            if (pass) qsort(list + off[i], (size_t)c, sizeof(int32_t), cmp_i32);
            else count[i] = c;
        }
        free(off);
    }
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) total += count[i];
    free(pc); free(head); free(members); free(fill);
    return total;
}

int64_t orc_neighbors_cells(int32_t n, const double* x, const double box[3], double r_list,
                            int32_t* count, int32_t* list, int64_t cap)
{
    return cells_rows(n, x, box, r_list, count, list, cap, 0);
}

/* ------------------------------------------------------------------------ */
/* Pair force, Eqs (2)-(8): F_ij = (a w_C - gamma w_D (e.v_ij)               */
/* + sigma w_R xi dt^-1/2) e_ij for |r_ij| < r_c, with w_C = 1 - r/r_c       */
/* (reading A2), w_R = w_C^s (Eq 8), w_D = w_R^2 (Eq 7).                     */
/* ------------------------------------------------------------------------ */

static void pair_force(const orc_params* p, const double d[3], double r2,
                       const double vij[3], int ti, int tj, uint32_t tagi, uint32_t tagj,
                       uint64_t step, double f[3], double* pe)
{
    double r = sqrt(r2);
    double e[3] = { d[0] / r, d[1] / r, d[2] / r };
    double wC = 1.0 - r / p->r_c;
    double wR = pow(wC, p->s);
    double wD = wR * wR;
    double ev = e[0] * vij[0] + e[1] * vij[1] + e[2] * vij[2];
    int tp = ti * p->n_types + tj;
    double xi = orc_xi(tagi, tagj, step, p->seed);
    double phi = p->a[tp] * wC - p->gamma[tp] * wD * ev + p->sigma[tp] * wR * xi / sqrt(p->dt);
    for (int k = 0; k < 3; ++k) f[k] = phi * e[k];
    /* conservative potential 1/2 a r_c w_C^2, half of it booked on each side */
    *pe = 0.25 * p->a[tp] * p->r_c * wC * wC;
}

static int32_t* make_idx_of_tag(int32_t n, const uint32_t* tag)
{
    int32_t* iot = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) iot[i] = -1;
    for (int64_t i = 0; i < n; ++i)
        if (tag[i] < (uint32_t)n) iot[tag[i]] = (int32_t)i;
    return iot;
}

/* Harmonic bond force on i from partner j: F = -k (r - r0) e (Sec. 4.5). */
static void bond_force(const orc_params* p, const double d[3], double r2, double f[3], double* pe)
{
    double r = sqrt(r2);
    double mag = -p->bond_k * (r - p->bond_r0);
    for (int k = 0; k < 3; ++k) f[k] = mag * d[k] / r;
    *pe = 0.25 * p->bond_k * (r - p->bond_r0) * (r - p->bond_r0);   /* half of 1/2 k (r-r0)^2 */
}

/* Forces on the query rows (q == NULL: all particles, nq ignored).
 * off/nb hold each row's neighbour candidates (any superset of the pairs
 * within r_c, e.g. the r_list rows); pairs with r^2 >= r_c^2 contribute 0.
 * v is the velocity entering F^D (the predicted velocity of the integrator).
 * f: double[3][nq]; pe (nullable): per-row potential energy (pairs + bonds,
 * halves); npair (nullable): per-row count of pairs inside r_c; scale
 * (nullable): per-row sum of the magnitudes of all added terms, the scale
 * of the summation-order rounding error.
 * Sums run in ascending neighbour order, then bonds, then the body force. */
int orc_forces(const orc_params* p, int32_t n, const double* x, const double* v,
               const uint32_t* tag, const uint8_t* type, int32_t nq, const int32_t* q,
               const int64_t* off, const int32_t* nb, uint64_t step,
               double* f, double* pe, int32_t* npair, double* scale)
{
    if (q == NULL) nq = n;
    const double rc2 = p->r_c * p->r_c;
    int32_t* iot = p->partner ? make_idx_of_tag(n, tag) : NULL;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int32_t r = 0; r < nq; ++r) {
        int64_t i = q ? q[r] : r;
        double fi[3] = { 0.0, 0.0, 0.0 };
        double pei = 0.0, sc = 0.0;
        int32_t np = 0;
        for (int64_t e = off[r]; e < off[r + 1]; ++e) {
            int64_t j = nb[e];
            double d[3];
            double r2 = separation(x, n, i, j, p->box, d);
            if (!(r2 < rc2)) continue;
            double vij[3];
            for (int k = 0; k < 3; ++k) vij[k] = v[k * n + i] - v[k * n + j];
            double fij[3], peij;
            pair_force(p, d, r2, vij, type[i], type[j], tag[i], tag[j], step, fij, &peij);
            for (int k = 0; k < 3; ++k) fi[k] += fij[k];
            sc += sqrt(fij[0] * fij[0] + fij[1] * fij[1] + fij[2] * fij[2]);
            pei += peij;
            ++np;
        }
        if (iot) {
            for (int b = 0; b < 2; ++b) {
                int32_t pt = p->partner[2 * (int64_t)tag[i] + b];
                if (pt < 0) continue;
                int64_t j = iot[pt];
                double d[3];
                double r2 = separation(x, n, i, j, p->box, d);
                double fb[3], peb;
                bond_force(p, d, r2, fb, &peb);
                for (int k = 0; k < 3; ++k) fi[k] += fb[k];
                sc += sqrt(fb[0] * fb[0] + fb[1] * fb[1] + fb[2] * fb[2]);
                pei += peb;
            }
        }
        if (p->body_g != 0.0) {
            fi[0] += (x[1 * n + i] < p->body_split) ? p->body_g : -p->body_g;
            sc += fabs(p->body_g);
        }
        for (int k = 0; k < 3; ++k) f[k * (int64_t)nq + r] = fi[k];
        if (pe) pe[r] = pei;
        if (npair) npair[r] = np;
        if (scale) scale[r] = sc;
    }
    free(iot);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Time step (Eq (1); Algorithm 1's integration phases 1 and 2; velocity     */
/* Verlet in the Groot-Warren form with prediction factor lambda).           */
/* State in: x_n, v_n, F_n.  Out: x_{n+1}, v_{n+1}, F_{n+1} = F(x_{n+1},     */
/* v~, n+1).  Particle order is kept (no reordering is needed for a          */
/* reference).  red[8]: P_x, P_y, P_z, sum |v|^2, PE, unique pairs, k_BT, 0. */
/* use_cells selects the cell-list neighbour search (equal sets, faster).    */
/* ------------------------------------------------------------------------ */

int orc_step(const orc_params* p, int32_t n, double* x, double* v, double* f,
             const uint32_t* tag, const uint8_t* type, uint64_t step_next,
             int use_cells, double* red)
{
    const double half_dt = 0.5 * p->dt;
    double* vh = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* vt = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    for (int k = 0; k < 3; ++k) {
        const double L = p->box[k];
        for (int64_t i = 0; i < n; ++i) {
            int64_t a = k * (int64_t)n + i;
            vh[a] = fma(half_dt, f[a], v[a]);                 /* phase 1: kick  */
            double xn = fma(p->dt, vh[a], x[a]);               /*          drift */
            if (xn < 0.0) xn = xn + L;                         /* periodic wrap  */
            if (xn >= L) xn = xn - L;
            x[a] = xn;
            vt[a] = (p->lambda == 0.5) ? vh[a] : fma(p->lambda * p->dt, f[a], v[a]);
        }
    }
    int32_t* count = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t total = use_cells ? orc_neighbors_cells(n, x, p->box, p->r_list, count, NULL, 0)
                              : orc_neighbors_brute(n, x, p->box, p->r_list, 0, NULL, count, NULL, 0);
    if (total < 0) { free(vh); free(vt); free(count); return -1; }
    int32_t* list = (int32_t*)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    if (use_cells) cells_rows(n, x, p->box, p->r_list, count, list, total, 1);
    else orc_neighbors_brute(n, x, p->box, p->r_list, 0, NULL, count, list, total);
    int64_t* off = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n + 1));
    exclusive_scan(count, n, off);
    double* pe = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int32_t* np = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    orc_forces(p, n, x, vt, tag, type, 0, NULL, off, list, step_next, f, pe, np, NULL);
    for (int k = 0; k < 3; ++k)
        for (int64_t i = 0; i < n; ++i) {
            int64_t a = k * (int64_t)n + i;
            v[a] = fma(half_dt, f[a], vh[a]);                 /* phase 2: kick  */
        }
    if (red) {
        double P[3] = { 0, 0, 0 }, v2 = 0, pesum = 0, pairs = 0;
        for (int64_t i = 0; i < n; ++i) {
            for (int k = 0; k < 3; ++k) {
                double vk = v[k * (int64_t)n + i];
                P[k] += vk;
                v2 += vk * vk;
            }
            pesum += pe[i];
            pairs += np[i];
        }
        double m2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            double mean = P[k] / n;
            for (int64_t i = 0; i < n; ++i) {
                double dv = v[k * (int64_t)n + i] - mean;
                m2 += dv * dv;
            }
        }
        red[0] = P[0]; red[1] = P[1]; red[2] = P[2];
        red[3] = v2;
        red[4] = pesum;
        red[5] = 0.5 * pairs;
        red[6] = m2 / (3.0 * (n - 1));        /* k_BT over 3(N-1) degrees of freedom */
        red[7] = 0.0;
    }
    free(vh); free(vt); free(count); free(list); free(off); free(pe); free(np);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Vector-Jacobian products of the deterministic forces (xi and the pair set */
/* held fixed; reading A20).  With F_i = sum_j f(r_ij, v_ij) and g = dL/dF:  */
/*   xbar_i = sum_j (df/dr_ij)^T (g_i - g_j),                                */
/*   vbar_i = sum_j (df/dv_ij)^T (g_i - g_j),                                */
/*   abar[t,u] = sum over unordered pairs of type {t,u} (g_i - g_j).df/da,   */
/*   gbar[t,u] likewise for gamma (a and gamma are symmetric parameters;     */
/*   both entries of an off-diagonal pair receive the same value).           */
/* f = phi e, phi = a w_C - gamma w_D (e.v) + sigma w_R xi / sqrt(dt):        */
/*   df/dr = dphi/dr e e^T + dphi/du e ((I - e e^T) v / r)^T                 */
/*           + phi (I - e e^T) / r,        u = e.v,                          */
/*   df/dv = dphi/du e e^T,  dphi/du = -gamma w_D.                           */
/* Bonds add  -k [e e^T + (r - r0)/r (I - e e^T)]  to df/dr.                 */
/* ------------------------------------------------------------------------ */

int orc_forces_vjp(const orc_params* p, int32_t n, const double* x, const double* v,
                   const uint32_t* tag, const uint8_t* type, const int64_t* off,
                   const int32_t* nb, uint64_t step, const double* g,
                   double* xbar, double* vbar, double* abar, double* gbar)
{
    const double rc2 = p->r_c * p->r_c;
    const int nt = p->n_types;
    const double s = p->s;
    int32_t* iot = p->partner ? make_idx_of_tag(n, tag) : NULL;
    double* pa = (double*)calloc((size_t)n * nt * nt, sizeof(double));
    double* pg = (double*)calloc((size_t)n * nt * nt, sizeof(double));
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double xb[3] = { 0, 0, 0 }, vb[3] = { 0, 0, 0 };
        for (int64_t e_ = off[i]; e_ < off[i + 1]; ++e_) {
            int64_t j = nb[e_];
            double d[3];
            double r2 = separation(x, n, i, j, p->box, d);
            if (!(r2 < rc2)) continue;
            double r = sqrt(r2);
            double e[3] = { d[0] / r, d[1] / r, d[2] / r };
            double vij[3], gij[3];
            for (int k = 0; k < 3; ++k) {
                vij[k] = v[k * (int64_t)n + i] - v[k * (int64_t)n + j];
                gij[k] = g[k * (int64_t)n + i] - g[k * (int64_t)n + j];
            }
            int tp = type[i] * nt + type[j];
            double A = p->a[tp], G = p->gamma[tp], S = p->sigma[tp];
            double wC = 1.0 - r / p->r_c;
            double wR = pow(wC, s);
            double wD = wR * wR;
            double dwC = -1.0 / p->r_c;
            double dwR = s * pow(wC, s - 1.0) * dwC;
            double dwD = 2.0 * s * pow(wC, 2.0 * s - 1.0) * dwC;
            double u = e[0] * vij[0] + e[1] * vij[1] + e[2] * vij[2];
            double xi = orc_xi(tag[i], tag[j], step, p->seed);
            double rdt = 1.0 / sqrt(p->dt);
            double phi = A * wC - G * wD * u + S * wR * xi * rdt;
            double dphi_dr = A * dwC - G * dwD * u + S * dwR * xi * rdt;
            double dphi_du = -G * wD;
            double eg = e[0] * gij[0] + e[1] * gij[1] + e[2] * gij[2];
            for (int k = 0; k < 3; ++k) {
                double perp_v = (vij[k] - u * e[k]) / r;     /* (I - e e^T) v / r */
                double perp_g = (gij[k] - eg * e[k]) / r;    /* (I - e e^T) g / r */
                xb[k] += dphi_dr * eg * e[k] + dphi_du * eg * perp_v + phi * perp_g;
                vb[k] += dphi_du * eg * e[k];
            }
            /* df/da = w_C e, df/dgamma = -w_D u e; each unordered pair is seen
             * twice (from i and from j) with equal value, hence the 1/2 */
            int ti = type[i], tj = type[j];
            int lo = ti < tj ? ti : tj, hi = ti < tj ? tj : ti;
            pa[i * nt * nt + lo * nt + hi] += 0.5 * wC * eg;
            pg[i * nt * nt + lo * nt + hi] += 0.5 * (-wD * u) * eg;
        }
        if (iot) {
            for (int b = 0; b < 2; ++b) {
                int32_t pt = p->partner[2 * (int64_t)tag[i] + b];
                if (pt < 0) continue;
                int64_t j = iot[pt];
                double d[3];
                double r2 = separation(x, n, i, j, p->box, d);
                double r = sqrt(r2);
                double e[3] = { d[0] / r, d[1] / r, d[2] / r };
                double gij[3];
                for (int k = 0; k < 3; ++k) gij[k] = g[k * (int64_t)n + i] - g[k * (int64_t)n + j];
                double eg = e[0] * gij[0] + e[1] * gij[1] + e[2] * gij[2];
                double tperp = (r - p->bond_r0) / r;
                for (int k = 0; k < 3; ++k)
                    xb[k] += -p->bond_k * (eg * e[k] + tperp * (gij[k] - eg * e[k]));
            }
        }
        for (int k = 0; k < 3; ++k) {
            xbar[k * (int64_t)n + i] = xb[k];
            vbar[k * (int64_t)n + i] = vb[k];
        }
    }
    for (int t = 0; t < nt * nt; ++t) { abar[t] = 0.0; gbar[t] = 0.0; }
    for (int64_t i = 0; i < n; ++i)
        for (int t = 0; t < nt * nt; ++t) {
            abar[t] += pa[i * nt * nt + t];
            gbar[t] += pg[i * nt * nt + t];
        }
    for (int t = 0; t < nt; ++t)
        for (int u = t + 1; u < nt; ++u) {
            abar[u * nt + t] = abar[t * nt + u];
            gbar[u * nt + t] = gbar[t * nt + u];
        }
    free(pa); free(pg); free(iot);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Several steps in a row (for the long statistical pins).  red: double      */
/* [n_steps][8] as in orc_step.  When prof != NULL, after step index          */
/* prof_from the velocity component prof_comp is averaged into nbins slabs   */
/* along axis prof_axis: prof[b] += v, prof_cnt[b] += 1.                     */
/* ------------------------------------------------------------------------ */
int orc_run(const orc_params* p, int32_t n, double* x, double* v, double* f,
            const uint32_t* tag, const uint8_t* type, uint64_t step0, int32_t n_steps,
            int use_cells, double* red, int32_t prof_axis, int32_t prof_comp, int32_t nbins,
            int32_t prof_from, double* prof, double* prof_cnt)
{
    for (int32_t s = 0; s < n_steps; ++s) {
        if (orc_step(p, n, x, v, f, tag, type, step0 + (uint64_t)s + 1, use_cells,
                     red ? red + 8 * (int64_t)s : NULL))
            return -1;
        if (prof && s >= prof_from) {
            const double L = p->box[prof_axis];
            for (int64_t i = 0; i < n; ++i) {
                int32_t b = (int32_t)(x[prof_axis * (int64_t)n + i] / L * nbins);
                if (b >= nbins) b = nbins - 1;
                prof[b] += v[prof_comp * (int64_t)n + i];
                prof_cnt[b] += 1.0;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Border determination for a spatial decomposition (Sec. 3.6, Algorithm 6): */
/* each processor keeps, for every neighbour, a send list of the local      */
/* particles whose copies that neighbour needs.  For the brick [lo, hi) and */
/* a halo of `width`, face f = 2 d + s (axis d; s = 0 the low face, s = 1   */
/* the high face) lists, in ascending index order, the particles with       */
/* x_d < lo_d + width (s = 0) or x_d >= hi_d - width (s = 1); only faces    */
/* selected in face_mask get a list.  off[7] receives the exclusive offsets */
/* of the six lists in idx (idx NULL: offsets only).  Returns the total.    */
/* ------------------------------------------------------------------------ */
int64_t orc_border_lists(int32_t n, const double* x, const double lo[3], const double hi[3], double width,
                         int32_t face_mask, int64_t* off, int32_t* idx)
{
    int64_t total = 0;
    for (int f = 0; f < 6; ++f) {
        const int d = f / 2, high = f % 2;
        off[f] = total;
        if (!((face_mask >> f) & 1)) continue;
        const double band = high ? hi[d] - width : lo[d] + width;
        for (int64_t i = 0; i < n; ++i) {
            const double xd = x[d * (int64_t)n + i];
            const int sent = high ? (xd >= band) : (xd < band);
            if (sent) {
                if (idx) idx[total] = (int32_t)i;
                ++total;
            }
        }
    }
    off[6] = total;
    return total;
}

/* The ghost record of each send-list entry: the particle's position moved  */
/* by its face's shift (the image the receiving neighbour sees; shift is    */
/* double[6][3]), its velocity, tag and type.  Records are written as        */
/* separate arrays: gx, gv double[3][total] (component-major), gtag, gtype.  */
void orc_border_pack(int32_t n, const double* x, const double* v, const uint32_t* tag, const uint8_t* type,
                     const int64_t* off, const int32_t* idx, const double* shift,
                     double* gx, double* gv, uint32_t* gtag, uint32_t* gtype)
{
    const int64_t total = off[6];
    for (int f = 0; f < 6; ++f)
        for (int64_t r = off[f]; r < off[f + 1]; ++r) {
            const int64_t j = idx[r];
            for (int d = 0; d < 3; ++d) {
                gx[d * total + r] = x[d * (int64_t)n + j] + shift[3 * f + d];
                gv[d * total + r] = v[d * (int64_t)n + j];
            }
            gtag[r] = tag[j];
            gtype[r] = type[j];
        }
}

/* ------------------------------------------------------------------------ */
/* The paper's alternative pair generator (Sec. 3.5, Algorithm 4), for the  */
/* A/B study only.  TEA: Wheeler & Needham, "TEA, a tiny encryption         */
/* algorithm" (Fast Software Encryption, 1994): each cycle adds the golden- */
/* ratio constant delta = 0x9E3779B9 to a running sum and updates the two   */
/* halves with shifts by 4 and 5, key words and the sum.  Readings (the     */
/* paper gives no key and no pair layout): keys (seed low, seed high, step  */
/* low, step high); a signature hashes (bit-reversed tag, the leading 11    */
/* mantissa bits of v_x, v_y, v_z interleaved bit by bit, x lowest, the     */
/* 33rd bit dropped) with 16 cycles and xors the halves; a pair hashes      */
/* (smaller signature, larger signature) with 4 cycles into two uniforms of */
/* the same Box-Muller form as orc_xi.                                       */
/* ------------------------------------------------------------------------ */

void orc_tea(int32_t rounds, uint32_t v[2], const uint32_t k[4])
{
    const uint32_t delta = 0x9E3779B9u;
    uint32_t y = v[0], z = v[1], sum = 0;
    for (int32_t r = 0; r < rounds; ++r) {
        sum += delta;
        y += ((z << 4) + k[0]) ^ (z + sum) ^ ((z >> 5) + k[1]);
        z += ((y << 4) + k[2]) ^ (y + sum) ^ ((y >> 5) + k[3]);
    }
    v[0] = y;
    v[1] = z;
}

static void tea_key_of(uint64_t seed, uint64_t step, uint32_t k[4])
{
    k[0] = (uint32_t)seed; k[1] = (uint32_t)(seed >> 32);
    k[2] = (uint32_t)step; k[3] = (uint32_t)(step >> 32);
}

/* the two words a signature hashes (before the 16 cycles) */
void orc_tea_sig_inputs(uint32_t tag, double vx, double vy, double vz, uint32_t out[2])
{
    uint32_t rev = 0;
    for (int b = 0; b < 32; ++b) rev |= ((tag >> b) & 1u) << (31 - b);
    const double comp[3] = { vx, vy, vz };
    uint32_t m[3];
    for (int c = 0; c < 3; ++c) {
        uint64_t bits;
        memcpy(&bits, &comp[c], sizeof(bits));
        m[c] = (uint32_t)((bits >> 41) & 0x7FFu);      /* mantissa bits 51 .. 41 */
    }
    uint32_t inter = 0;
    for (int b = 0; b < 11; ++b)
        for (int c = 0; c < 3; ++c) {
            const int pos = 3 * b + c;
            if (pos < 32) inter |= ((m[c] >> b) & 1u) << pos;
        }
    out[0] = rev;
    out[1] = inter;
}

void orc_tea_signatures(int32_t n, const uint32_t* tag, const double* v, uint64_t step, uint64_t seed,
                        uint32_t* sig)
{
    uint32_t k[4];
    tea_key_of(seed, step, k);
    for (int64_t i = 0; i < n; ++i) {
        uint32_t w[2];
        orc_tea_sig_inputs(tag[i], v[i], v[(int64_t)n + i], v[2 * (int64_t)n + i], w);
        orc_tea(16, w, k);
        sig[i] = w[0] ^ w[1];
    }
}

void orc_tea_xi_batch(int64_t n, const uint32_t* si, const uint32_t* sj, uint64_t step, uint64_t seed,
                      uint32_t* words, double* xi)
{
    uint32_t k[4];
    tea_key_of(seed, step, k);
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t w[2] = { si[i] < sj[i] ? si[i] : sj[i], si[i] < sj[i] ? sj[i] : si[i] };
        orc_tea(4, w, k);
        if (words) { words[2 * i] = w[0]; words[2 * i + 1] = w[1]; }
        const double u1 = ((double)w[0] + 0.5) / 4294967296.0;
        const double u2 = (double)w[1] / 4294967296.0;
        xi[i] = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
    }
}
