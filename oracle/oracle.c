/*
 * oracle.c -- plain, single-threaded FP64 reference of the geometric docking
 * hot path.  TEST INFRASTRUCTURE ONLY: it exists to check the GPU library and
 * must never be linked or called by the product path (only tests, the smoke
 * check and the benchmark's CPU-baseline leg use it).  It shares no source
 * with the GPU library.
 *
 * What it computes (paper: Gadioli et al., "Tunable Approximations to Control
 * Time-to-Solution in an HPC Molecular Docking Mini-App"):
 *
 *  - Overlap score, Eq. 1 (Section III-A): o = l / sum_i min_j d^2(L_i, P_j).
 *    Read on a lattice of spacing h anchored at the origin: every ligand atom
 *    and pocket point is snapped to its cell floor(x/h), and min_j d^2 becomes
 *    D(c) = min over occupied cells c' of |c - c'|^2 (integer, cell units).
 *    S = sum_i D(cell(X_i)) is the integer "overlap count"; o = l / (h^2 S)
 *    and smaller S ranks better.  D is evaluated by brute force over the
 *    occupied cells (memoised per cell), i.e. by its definition.
 *  - Feasibility ("CheckBumps", Alg. 1, Section III-B): a shape is infeasible
 *    when a pair of atoms more than 3 bonds apart comes closer than the clash
 *    distance (strict d^2 < clash_dist^2).  A sweep of one fragment tests the
 *    pairs that straddle the rotatable bond; the endpoint flag tests all.
 *  - MatchProbesShape with the five knobs, Alg. 2 (Section III-C): for each
 *    repetition, for each rotamer in list order, the left and then the right
 *    fragment is swept through its angle schedule (coarse step when the
 *    fragment's relative size is <= threshold; otherwise either the flat fine
 *    step, or the tile-peeling refinement of Eq. 2/3), and the best feasible
 *    angle is committed.
 *  - Rigid orientations: each run starts from a unit quaternion that rotates
 *    the ligand about its centroid and places the centroid at the pocket
 *    centroid; per orientation the endpoint (S, clash, chosen angles, pose)
 *    is recorded and the orientations are ranked by (clash, S, index).
 *
 * Numerical conventions (the GPU library reproduces the FP64 parts of these
 * formulas in the same operation order, so FP64 states agree bit for bit):
 *  - Angles are integer degrees; c = cos(deg * (pi/180)), s = sin(...) (libm).
 *  - Rotation about unit axis k by angle theta (right-hand rule):
 *      R = c I + s [k]x + (1-c) k k^T, written element by element below,
 *      Y = p + R (X - p), p = the moving fragment's own bond atom.
 *  - Axis k = (X_b - X_a) / |X_b - X_a| for both fragments of rotamer (a,b).
 *  - Compiled with -ffp-contract=off: no fused multiply-adds.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_GRAPH 2
#define ORC_ERR_ROTAMER 3
#define ORC_ERR_KNOB 4

static const double ORC_PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* Pocket: occupied cells and the squared-distance field D (Eq. 1 on a grid) */

typedef struct {
    double h;
    int n_points;
    double* pts;        /* n x 3, FP64 widening of the FP32 input */
    int n_occ;
    int64_t* occ;       /* unique occupied cells, n_occ x 3 */
    double centroid[3]; /* mean of the points, summed in input order */
    int64_t mlo[3], mdim[3];
    int64_t* memo;      /* D per cell of the memo box, -1 = not computed yet */
} orc_pocket;

static int64_t cell_of(double v, double h) { return (int64_t)floor(v / h); }

static int cmp_cell(const void* a, const void* b) {
    const int64_t* x = (const int64_t*)a;
    const int64_t* y = (const int64_t*)b;
    for (int k = 0; k < 3; k++) {
        if (x[k] < y[k]) return -1;
        if (x[k] > y[k]) return 1;
    }
    return 0;
}

orc_pocket* orc_pocket_new(const float* xyz, int n, double h) {
    if (n < 1 || !(h > 0)) return NULL;
    orc_pocket* P = (orc_pocket*)calloc(1, sizeof(orc_pocket));
    P->h = h;
    P->n_points = n;
    P->pts = (double*)malloc(sizeof(double) * 3 * n);
    int64_t* cells = (int64_t*)malloc(sizeof(int64_t) * 3 * n);
    double sx = 0, sy = 0, sz = 0;
    for (int i = 0; i < n; i++) {
        double x = (double)xyz[3 * i], y = (double)xyz[3 * i + 1], z = (double)xyz[3 * i + 2];
        P->pts[3 * i] = x; P->pts[3 * i + 1] = y; P->pts[3 * i + 2] = z;
        sx = sx + x; sy = sy + y; sz = sz + z;
        cells[3 * i] = cell_of(x, h); cells[3 * i + 1] = cell_of(y, h); cells[3 * i + 2] = cell_of(z, h);
    }
    P->centroid[0] = sx / (double)n; P->centroid[1] = sy / (double)n; P->centroid[2] = sz / (double)n;
    qsort(cells, n, sizeof(int64_t) * 3, cmp_cell);
    int m = 0;
    for (int i = 0; i < n; i++) {
        if (m > 0 && cmp_cell(cells + 3 * i, cells + 3 * (m - 1)) == 0) continue;
        memmove(cells + 3 * m, cells + 3 * i, sizeof(int64_t) * 3);
        m++;
    }
    P->n_occ = m;
    P->occ = cells;
    int64_t lo[3], hi[3];
    for (int k = 0; k < 3; k++) { lo[k] = cells[k]; hi[k] = cells[k]; }
    for (int i = 0; i < m; i++)
        for (int k = 0; k < 3; k++) {
            if (cells[3 * i + k] < lo[k]) lo[k] = cells[3 * i + k];
            if (cells[3 * i + k] > hi[k]) hi[k] = cells[3 * i + k];
        }
    const int64_t margin = 64;
    int64_t total = 1;
    for (int k = 0; k < 3; k++) {
        P->mlo[k] = lo[k] - margin;
        P->mdim[k] = hi[k] - lo[k] + 1 + 2 * margin;
        total *= P->mdim[k];
    }
    P->memo = (int64_t*)malloc(sizeof(int64_t) * total);
    for (int64_t i = 0; i < total; i++) P->memo[i] = -1;
    return P;
}

void orc_pocket_free(orc_pocket* P) {
    if (!P) return;
    free(P->pts); free(P->occ); free(P->memo); free(P);
}

void orc_pocket_centroid(const orc_pocket* P, double* c) { c[0] = P->centroid[0]; c[1] = P->centroid[1]; c[2] = P->centroid[2]; }
int orc_pocket_n_occ(const orc_pocket* P) { return P->n_occ; }
void orc_pocket_occ(const orc_pocket* P, int64_t* out) { memcpy(out, P->occ, sizeof(int64_t) * 3 * P->n_occ); }

/* D(c) = min over occupied cells o of |c - o|^2, by brute force. */
static int64_t D_brute(const orc_pocket* P, int64_t cx, int64_t cy, int64_t cz) {
    int64_t best = INT64_MAX;
    for (int i = 0; i < P->n_occ; i++) {
        int64_t dx = cx - P->occ[3 * i], dy = cy - P->occ[3 * i + 1], dz = cz - P->occ[3 * i + 2];
        int64_t d = dx * dx + dy * dy + dz * dz;
        if (d < best) best = d;
    }
    return best;
}

int64_t orc_D(orc_pocket* P, int64_t cx, int64_t cy, int64_t cz) {
    int64_t ix = cx - P->mlo[0], iy = cy - P->mlo[1], iz = cz - P->mlo[2];
    if (ix < 0 || iy < 0 || iz < 0 || ix >= P->mdim[0] || iy >= P->mdim[1] || iz >= P->mdim[2])
        return D_brute(P, cx, cy, cz);
    int64_t idx = (iz * P->mdim[1] + iy) * P->mdim[0] + ix;
    if (P->memo[idx] < 0) P->memo[idx] = D_brute(P, cx, cy, cz);
    return P->memo[idx];
}

/* S(X) = sum_i D(cell(X_i)) over the given FP64 coordinates (n x 3). */
int64_t orc_score_xyz(orc_pocket* P, int n, const double* X) {
    int64_t S = 0;
    for (int i = 0; i < n; i++)
        S += orc_D(P, cell_of(X[3 * i], P->h), cell_of(X[3 * i + 1], P->h), cell_of(X[3 * i + 2], P->h));
    return S;
}

/* ------------------------------------------------------------------------ */
/* Ligand topology: validation, bond-count distances, fragments              */

typedef struct {
    int l, nb, nr;
    const int* bonds;
    const int* rot;
    int* deg;
    int* dist;          /* l x l bond-count distances */
    unsigned char* left; /* nr x l: atom is in the left fragment of rotamer b */
} orc_topo;

static void topo_free(orc_topo* T) { free(T->deg); free(T->dist); free(T->left); }

/* BFS from src; if (ea,eb) >= 0 that edge is ignored.  dist[] gets -1 when unreachable. */
static void bfs(const orc_topo* T, int src, int ea, int eb, int* dist) {
    int l = T->l;
    int* queue = (int*)malloc(sizeof(int) * l);
    for (int i = 0; i < l; i++) dist[i] = -1;
    int qh = 0, qt = 0;
    dist[src] = 0;
    queue[qt++] = src;
    while (qh < qt) {
        int u = queue[qh++];
        for (int b = 0; b < T->nb; b++) {
            int a = T->bonds[2 * b], c = T->bonds[2 * b + 1], w;
            if (a == u) w = c; else if (c == u) w = a; else continue;
            if ((a == ea && c == eb) || (a == eb && c == ea)) continue;
            if (dist[w] < 0) { dist[w] = dist[u] + 1; queue[qt++] = w; }
        }
    }
    free(queue);
}

static int topo_build(orc_topo* T, int l, int nb, const int* bonds, int nr, const int* rot) {
    memset(T, 0, sizeof(*T));
    if (l < 1 || nb < 0 || nr < 0) return ORC_ERR_GRAPH;
    T->l = l; T->nb = nb; T->nr = nr; T->bonds = bonds; T->rot = rot;
    T->deg = (int*)calloc(l, sizeof(int));
    T->dist = (int*)malloc(sizeof(int) * l * l);
    T->left = (unsigned char*)calloc((size_t)(nr > 0 ? nr : 1) * l, 1);
    for (int b = 0; b < nb; b++) {
        int a = bonds[2 * b], c = bonds[2 * b + 1];
        if (a < 0 || c < 0 || a >= l || c >= l || a == c) return ORC_ERR_GRAPH;
        for (int e = 0; e < b; e++) {
            int a2 = bonds[2 * e], c2 = bonds[2 * e + 1];
            if ((a == a2 && c == c2) || (a == c2 && c == a2)) return ORC_ERR_GRAPH;
        }
        T->deg[a]++; T->deg[c]++;
    }
    for (int i = 0; i < l; i++) {
        bfs(T, i, -1, -1, T->dist + (size_t)i * l);
        for (int j = 0; j < l; j++)
            if (T->dist[(size_t)i * l + j] < 0) return ORC_ERR_GRAPH; /* disconnected */
    }
    int* d = (int*)malloc(sizeof(int) * l);
    for (int r = 0; r < nr; r++) {
        int a = rot[2 * r], c = rot[2 * r + 1];
        if (a < 0 || c < 0 || a >= l || c >= l || a == c) { free(d); return ORC_ERR_ROTAMER; }
        int is_bond = 0;
        for (int b = 0; b < nb; b++) {
            int x = bonds[2 * b], y = bonds[2 * b + 1];
            if ((x == a && y == c) || (x == c && y == a)) is_bond = 1;
        }
        if (!is_bond || T->deg[a] < 2 || T->deg[c] < 2) { free(d); return ORC_ERR_ROTAMER; }
        /* left = atoms reachable from a without using the bond (a,c) */
        bfs(T, a, a, c, d);
        if (d[c] >= 0) { free(d); return ORC_ERR_ROTAMER; } /* not a bridge */
        for (int i = 0; i < l; i++) T->left[(size_t)r * l + i] = d[i] >= 0;
    }
    free(d);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Knobs and angle schedules (Alg. 2, Eq. 2, Eq. 3)                           */

typedef struct {
    int hp_step, lp_step;  /* integer degrees, each a divisor of 360 */
    double threshold;      /* relative fragment size; <= threshold -> coarse step */
    int repetitions;
    int refine;            /* tile-peeling iterative refinement */
    double clash_dist;
    int clash_min_bonds;   /* pairs at >= this many bonds are checked */
} orc_knobs;

static int knobs_ok(const orc_knobs* k) {
    if (k->hp_step < 1 || k->hp_step > 360 || 360 % k->hp_step) return 0;
    if (k->lp_step < 1 || k->lp_step > 360 || 360 % k->lp_step) return 0;
    if (!(k->threshold >= 0.0 && k->threshold <= 1.0)) return 0;
    if (k->repetitions < 1) return 0;
    if (!(k->clash_dist >= 0.0)) return 0;
    if (k->clash_min_bonds < 1) return 0;
    return 1;
}

/* Tile size x for the peel/tile refinement: minimise Eq. 2, y = 360/x + x/hp,
 * over divisors x of 360 that are multiples of hp; ties go to the smaller x.
 * (Eq. 3's continuous optimum sqrt(360 hp) is generally not a divisor.) */
int orc_tile_size(int hp) {
    int best = -1, besty = 0;
    for (int x = hp; x <= 360; x += hp) {
        if (360 % x) continue;
        int y = 360 / x + x / hp;
        if (best < 0 || y < besty) { best = x; besty = y; }
    }
    return best;
}

/* Flat schedule {0, step, ..., 360-step}. */
static int flat_schedule(int step, int* out) {
    int n = 360 / step;
    for (int k = 0; k < n; k++) out[k] = k * step;
    return n;
}

/* Peel elements: the central element of each tile of size x. */
static int peel_schedule(int hp, int* out) {
    int x = orc_tile_size(hp);
    int off = (x / (2 * hp)) * hp;
    int n = 360 / x;
    for (int t = 0; t < n; t++) out[t] = t * x + off;
    return n;
}

/* Public helper for tests: mode 0 = coarse, 1 = flat fine, 2 = refinement
 * (returns the peel list; the tile list is t*x + k*hp, k < x/hp). */
int orc_side_mode(const orc_knobs* k, int side_size, int l) {
    double rel = (double)side_size / (double)l;
    if (rel <= k->threshold) return 0;
    return k->refine ? 2 : 1;
}

/* ------------------------------------------------------------------------ */
/* Rigid-body arithmetic                                                      */

static void axis_angle_matrix(const double k[3], int deg, double R[9]) {
    double rad = (double)deg * (ORC_PI / 180.0);
    double c = cos(rad), s = sin(rad), t = 1.0 - c;
    R[0] = t * k[0] * k[0] + c;        R[1] = t * k[0] * k[1] - s * k[2]; R[2] = t * k[0] * k[2] + s * k[1];
    R[3] = t * k[0] * k[1] + s * k[2]; R[4] = t * k[1] * k[1] + c;        R[5] = t * k[1] * k[2] - s * k[0];
    R[6] = t * k[0] * k[2] - s * k[1]; R[7] = t * k[1] * k[2] + s * k[0]; R[8] = t * k[2] * k[2] + c;
}

static void rotate_about(const double p[3], const double R[9], const double* x, double* y) {
    double d0 = x[0] - p[0], d1 = x[1] - p[1], d2 = x[2] - p[2];
    y[0] = p[0] + (R[0] * d0 + R[1] * d1 + R[2] * d2);
    y[1] = p[1] + (R[3] * d0 + R[4] * d1 + R[5] * d2);
    y[2] = p[2] + (R[6] * d0 + R[7] * d1 + R[8] * d2);
}

static void quat_matrix(const double* q, double R[9]) {
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Place the ligand: X = R(q) (x - c_L) + c_P. */
static void place(int l, const float* x, const float* y, const float* z, const double* q, const double cP[3],
                  double* X) {
    double sx = 0, sy = 0, sz = 0;
    for (int i = 0; i < l; i++) { sx = sx + (double)x[i]; sy = sy + (double)y[i]; sz = sz + (double)z[i]; }
    double cL[3] = {sx / (double)l, sy / (double)l, sz / (double)l};
    double R[9];
    quat_matrix(q, R);
    for (int i = 0; i < l; i++) {
        double d0 = (double)x[i] - cL[0], d1 = (double)y[i] - cL[1], d2 = (double)z[i] - cL[2];
        X[3 * i + 0] = (R[0] * d0 + R[1] * d1 + R[2] * d2) + cP[0];
        X[3 * i + 1] = (R[3] * d0 + R[4] * d1 + R[5] * d2) + cP[1];
        X[3 * i + 2] = (R[6] * d0 + R[7] * d1 + R[8] * d2) + cP[2];
    }
}

static double dist2(const double* a, const double* b) {
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return dx * dx + dy * dy + dz * dz;
}

/* Whole-ligand clash: any pair at >= min_bonds bonds with d^2 < cd2. */
static int clash_all(const orc_topo* T, const double* X, double cd2, int min_bonds) {
    for (int i = 0; i < T->l; i++)
        for (int j = i + 1; j < T->l; j++)
            if (T->dist[(size_t)i * T->l + j] >= min_bonds && dist2(X + 3 * i, X + 3 * j) < cd2) return 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One orientation: the greedy sweep of Alg. 2                                */

typedef struct {
    orc_pocket* P;
    const orc_topo* T;
    const orc_knobs* K;
    double cd2;
    double* Y;       /* candidate pose scratch, l x 3 */
    int64_t n_cand;  /* candidates evaluated */
} sweep_ctx;

/* Evaluate one candidate angle for the moving set; returns feasibility, S via *S. */
static int eval_candidate(sweep_ctx* C, const double* X, const unsigned char* moving, const double p[3],
                          const double k[3], int deg, int64_t* S) {
    int l = C->T->l;
    double R[9];
    axis_angle_matrix(k, deg, R);
    memcpy(C->Y, X, sizeof(double) * 3 * l);
    for (int i = 0; i < l; i++)
        if (moving[i]) rotate_about(p, R, X + 3 * i, C->Y + 3 * i);
    C->n_cand++;
    int feasible = 1;
    for (int i = 0; i < l && feasible; i++) {
        if (!moving[i]) continue;
        for (int j = 0; j < l; j++) {
            if (moving[j]) continue;
            if (C->T->dist[(size_t)i * l + j] < C->K->clash_min_bonds) continue;
            if (dist2(C->Y + 3 * i, C->Y + 3 * j) < C->cd2) { feasible = 0; break; }
        }
    }
    *S = orc_score_xyz(C->P, l, C->Y);
    return feasible;
}

/* Pick the best feasible angle among `angles`: lowest S, ties to the earliest
 * position; returns the position or -1 when no candidate is feasible. */
static int best_of(sweep_ctx* C, const double* X, const unsigned char* moving, const double p[3], const double k[3],
                   const int* angles, int n) {
    int best = -1;
    int64_t bestS = 0;
    for (int t = 0; t < n; t++) {
        int64_t S;
        int ok = eval_candidate(C, X, moving, p, k, angles[t], &S);
        if (ok && (best < 0 || S < bestS)) { best = t; bestS = S; }
    }
    return best;
}

/* The moving set of one side of rotamer r (left = the side of its first
 * atom), the pivot (that side's bond atom) and the unit axis a -> c from the
 * pose X; returns the side's atom count. */
static int side_frame(const orc_topo* T, const double* X, int r, int side, unsigned char* moving, double p[3],
                      double k[3]) {
    int l = T->l;
    int a = T->rot[2 * r], c = T->rot[2 * r + 1];
    int size = 0;
    for (int i = 0; i < l; i++) {
        int in_left = T->left[(size_t)r * l + i];
        moving[i] = side == 0 ? in_left : !in_left;
        size += moving[i];
    }
    const double* piv = X + 3 * (side == 0 ? a : c);
    p[0] = piv[0]; p[1] = piv[1]; p[2] = piv[2];
    double ax = X[3 * c] - X[3 * a], ay = X[3 * c + 1] - X[3 * a + 1], az = X[3 * c + 2] - X[3 * a + 2];
    double nrm = sqrt(ax * ax + ay * ay + az * az);
    k[0] = ax / nrm; k[1] = ay / nrm; k[2] = az / nrm;
    return size;
}

static int sweep_side(sweep_ctx* C, double* X, int r, int side) {
    const orc_topo* T = C->T;
    int l = T->l;
    unsigned char* moving = (unsigned char*)malloc(l);
    double p[3], k[3];
    int size = side_frame(T, X, r, side, moving, p, k);

    int angles[360];
    int theta = 0;
    int mode = orc_side_mode(C->K, size, l);
    if (mode == 0 || mode == 1) {
        int n = flat_schedule(mode == 0 ? C->K->lp_step : C->K->hp_step, angles);
        int b = best_of(C, X, moving, p, k, angles, n);
        theta = b < 0 ? 0 : angles[b];
    } else {
        int hp = C->K->hp_step, x = orc_tile_size(hp);
        int n = peel_schedule(hp, angles);
        int t = best_of(C, X, moving, p, k, angles, n);
        if (t < 0) t = 0;
        int m = x / hp;
        for (int j = 0; j < m; j++) angles[j] = t * x + j * hp;
        int b = best_of(C, X, moving, p, k, angles, m);
        theta = b < 0 ? 0 : angles[b];
    }
    if (theta != 0) {
        double R[9];
        axis_angle_matrix(k, theta, R);
        for (int i = 0; i < l; i++)
            if (moving[i]) {
                double y[3];
                rotate_about(p, R, X + 3 * i, y);
                X[3 * i] = y[0]; X[3 * i + 1] = y[1]; X[3 * i + 2] = y[2];
            }
    }
    free(moving);
    return theta;
}

/*
 * Dock one ligand in all given orientations.
 * Outputs per orientation o: S[o], clash[o], angles[o][rep][rot][side]
 * (int16 degrees, may be NULL), xyz[o][atom][3] (FP64, may be NULL).
 * *n_cand gets the number of evaluated candidate poses (sweep candidates plus
 * one endpoint evaluation per orientation).
 */
int orc_dock(orc_pocket* P, int l, const float* x, const float* y, const float* z, int nb, const int* bonds, int nr,
             const int* rot, const orc_knobs* K, int n_orient, const double* quats, int64_t* S, uint8_t* clash,
             int16_t* angles, double* xyz, int64_t* n_cand) {
    if (!P || !K || n_orient < 0) return ORC_ERR_ARG;
    if (!knobs_ok(K)) return ORC_ERR_KNOB;
    orc_topo T;
    int rc = topo_build(&T, l, nb, bonds, nr, rot);
    if (rc != ORC_OK) { topo_free(&T); return rc; }
    sweep_ctx C;
    C.P = P; C.T = &T; C.K = K;
    C.cd2 = K->clash_dist * K->clash_dist;
    C.Y = (double*)malloc(sizeof(double) * 3 * l);
    C.n_cand = 0;
    double* X = (double*)malloc(sizeof(double) * 3 * l);
    for (int o = 0; o < n_orient; o++) {
        place(l, x, y, z, quats + 4 * o, P->centroid, X);
        for (int rep = 0; rep < K->repetitions; rep++)
            for (int r = 0; r < nr; r++)
                for (int side = 0; side < 2; side++) {
                    int th = sweep_side(&C, X, r, side);
                    if (angles) angles[(((size_t)o * K->repetitions + rep) * nr + r) * 2 + side] = (int16_t)th;
                }
        S[o] = orc_score_xyz(P, l, X);
        clash[o] = (uint8_t)clash_all(&T, X, C.cd2, K->clash_min_bonds);
        C.n_cand++;
        if (xyz) memcpy(xyz + (size_t)o * 3 * l, X, sizeof(double) * 3 * l);
    }
    if (n_cand) *n_cand = C.n_cand;
    free(X); free(C.Y);
    topo_free(&T);
    return ORC_OK;
}

/* Rank orientations by (clash, S, index) ascending and keep the first k. */
static const int64_t* g_S;
static const uint8_t* g_clash;
static int cmp_rank(const void* a, const void* b) {
    int i = *(const int*)a, j = *(const int*)b;
    if (g_clash[i] != g_clash[j]) return g_clash[i] < g_clash[j] ? -1 : 1;
    if (g_S[i] != g_S[j]) return g_S[i] < g_S[j] ? -1 : 1;
    return i < j ? -1 : (i > j);
}
int orc_topk(int n, const int64_t* S, const uint8_t* clash, int k, int* out) {
    if (k < 0 || k > n) return ORC_ERR_KNOB;
    int* idx = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int i = 0; i < n; i++) idx[i] = i;
    g_S = S; g_clash = clash;
    qsort(idx, n, sizeof(int), cmp_rank);
    memcpy(out, idx, sizeof(int) * k);
    free(idx);
    return ORC_OK;
}

/*
 * Overlap landscape of one side of rotamer r (the peak analysis of Section
 * III-B): from the pose X (l x 3, FP64) the side is turned about the bond by
 * every multiple of `step` degrees in [0, 360), and each candidate is
 * evaluated as a sweep evaluates it: whole-ligand S and feasibility of the
 * straddling far pairs (strict).  S and feasible receive 360/step entries.
 * Returns the side's atom count (its bond atom included), or an error code
 * (negative).
 */
int orc_sweep_profile(orc_pocket* P, int l, int nb, const int* bonds, int nr, const int* rot, const double* X, int r,
                      int side, int step, double clash_dist, int clash_min_bonds, int64_t* S, uint8_t* feasible) {
    if (!P || !X || !S || !feasible || r < 0 || r >= nr || side < 0 || side > 1 || step < 1 || step > 360 ||
        360 % step != 0)
        return -ORC_ERR_ARG;
    orc_topo T;
    int rc = topo_build(&T, l, nb, bonds, nr, rot);
    if (rc != ORC_OK) { topo_free(&T); return -rc; }
    orc_knobs K;
    memset(&K, 0, sizeof(K));
    K.clash_min_bonds = clash_min_bonds;
    sweep_ctx C;
    C.P = P; C.T = &T; C.K = &K;
    C.cd2 = clash_dist * clash_dist;
    C.Y = (double*)malloc(sizeof(double) * 3 * l);
    C.n_cand = 0;
    unsigned char* moving = (unsigned char*)malloc(l);
    double p[3], k[3];
    int size = side_frame(&T, X, r, side, moving, p, k);
    for (int t = 0; t < 360 / step; t++) feasible[t] = (uint8_t)eval_candidate(&C, X, moving, p, k, t * step, S + t);
    free(moving);
    free(C.Y);
    topo_free(&T);
    return size;
}

/* Overlap o = l / (h^2 S); S = 0 gives +inf. */
double orc_overlap(int l, int64_t S, double h) { return (double)l / (h * h * (double)S); }

/*
 * Eq. 1 without the lattice: each atom's smallest squared distance to any
 * pocket point (the points' FP32 input widened to FP64), summed over the
 * atoms in index order.  The squared distance of one pair is dx^2 + dy^2 +
 * dz^2 formed as fma(dz, dz, fma(dy, dy, dx * dx)): the plain definition with
 * IEEE 754 fused multiply-add rounding.  X is l x 3 row-major FP64; min_d2
 * (optional) receives the per-atom minima.  Returns the sum, from which the
 * overlap is l / sum (+inf when the sum is 0).
 */
double orc_overlap_continuous(const orc_pocket* P, int l, const double* X, double* min_d2) {
    double sum = 0.0;
    for (int i = 0; i < l; i++) {
        double best = INFINITY;
        for (int j = 0; j < P->n_points; j++) {
            const double dx = X[3 * i] - P->pts[3 * j];
            const double dy = X[3 * i + 1] - P->pts[3 * j + 1];
            const double dz = X[3 * i + 2] - P->pts[3 * j + 2];
            best = fmin(best, fma(dz, dz, fma(dy, dy, dx * dx)));
        }
        if (min_d2) min_d2[i] = best;
        sum += best;
    }
    return sum;
}

/*
 * Exact score of given poses (FP32 coordinates widened to FP64): S and the
 * whole-ligand clash flag, for one ligand topology.
 */
int orc_score_poses(orc_pocket* P, int l, int nb, const int* bonds, int n_poses, const float* px, const float* py,
                    const float* pz, double clash_dist, int min_bonds, int64_t* S, uint8_t* clash) {
    orc_topo T;
    int rc = topo_build(&T, l, nb, bonds, 0, NULL);
    if (rc != ORC_OK) { topo_free(&T); return rc; }
    double* X = (double*)malloc(sizeof(double) * 3 * l);
    double cd2 = clash_dist * clash_dist;
    for (int p = 0; p < n_poses; p++) {
        for (int i = 0; i < l; i++) {
            X[3 * i] = (double)px[(size_t)p * l + i];
            X[3 * i + 1] = (double)py[(size_t)p * l + i];
            X[3 * i + 2] = (double)pz[(size_t)p * l + i];
        }
        S[p] = orc_score_xyz(P, l, X);
        clash[p] = (uint8_t)clash_all(&T, X, cd2, min_bonds);
    }
    free(X);
    topo_free(&T);
    return ORC_OK;
}

/* Bond-count distance matrix and left-fragment masks, for tests. */
int orc_topology(int l, int nb, const int* bonds, int nr, const int* rot, int* dist, uint8_t* left) {
    orc_topo T;
    int rc = topo_build(&T, l, nb, bonds, nr, rot);
    if (rc == ORC_OK) {
        if (dist) memcpy(dist, T.dist, sizeof(int) * l * l);
        if (left) memcpy(left, T.left, (size_t)nr * l);
    }
    topo_free(&T);
    return rc;
}

/* Rigid placement of one orientation (for tests): X = R(q)(x - c_L) + c_P. */
void orc_place(int l, const float* x, const float* y, const float* z, const double* q, const double* cP, double* X) {
    place(l, x, y, z, q, cP, X);
}

/*
 * Apply a list of fragment rotations (rotamer r, side 0=left/1=right, integer
 * degrees) to the FP64 pose X in order, with the same kinematics as a sweep
 * commit (for tests of the kinematic invariants).
 */
int orc_apply_torsions(int l, int nb, const int* bonds, int nr, const int* rot, double* X, int n_moves,
                       const int* moves) {
    orc_topo T;
    int rc = topo_build(&T, l, nb, bonds, nr, rot);
    if (rc != ORC_OK) { topo_free(&T); return rc; }
    for (int m = 0; m < n_moves; m++) {
        int r = moves[3 * m], side = moves[3 * m + 1], deg = moves[3 * m + 2];
        if (r < 0 || r >= nr) { topo_free(&T); return ORC_ERR_ARG; }
        int a = rot[2 * r], c = rot[2 * r + 1];
        double p[3], k[3], R[9];
        const double* piv = X + 3 * (side == 0 ? a : c);
        p[0] = piv[0]; p[1] = piv[1]; p[2] = piv[2];
        double ax = X[3 * c] - X[3 * a], ay = X[3 * c + 1] - X[3 * a + 1], az = X[3 * c + 2] - X[3 * a + 2];
        double nrm = sqrt(ax * ax + ay * ay + az * az);
        k[0] = ax / nrm; k[1] = ay / nrm; k[2] = az / nrm;
        axis_angle_matrix(k, deg, R);
        for (int i = 0; i < l; i++) {
            int in_left = T.left[(size_t)r * l + i];
            if ((side == 0) != (in_left != 0)) continue;
            double y[3];
            rotate_about(p, R, X + 3 * i, y);
            X[3 * i] = y[0]; X[3 * i + 1] = y[1]; X[3 * i + 2] = y[2];
        }
    }
    topo_free(&T);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Smoothed surrogate for pose refinement (a differentiable stand-in for the
 * overlap score, used only to propose refined poses; every refined pose is
 * scored again with the exact lattice score S and the bump rule).
 *
 *   rho(g)  = sum_j exp(-|g - P_j|^2 / (2 sigma^2)) over points with
 *             |g - P_j| <= cutoff, at lattice nodes g = bh * (i, j, k)
 *   rho~(x) = trilinear interpolation of rho in the lattice cell containing x
 *   F       = sum_i rho~(X_i)
 *   X(t, q, tau) = R(q/|q|) (FK_tau(X0) - c0) + c0 + t, c0 = mean of X0;
 *   FK_tau rotates, root first (bond distance of the rotamer's atom nearer to
 *   atom 0, ties in list order), the side of rotamer b that does not contain
 *   atom 0 by tau_b (radians, right-handed about near -> far atom) about its
 *   current axis.                                                            */

typedef struct {
    double sigma, cutoff, bh;
    int64_t lo[3], dim[3];
    double* memo; /* NaN = unknown */
} orc_blur;


orc_blur* orc_blur_new(const orc_pocket* P, double sigma, double cutoff, double bh) {
    orc_blur* B = (orc_blur*)calloc(1, sizeof(orc_blur));
    B->sigma = sigma; B->cutoff = cutoff; B->bh = bh;
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int i = 0; i < P->n_points; i++)
        for (int a = 0; a < 3; a++) {
            if (P->pts[3 * i + a] < mn[a]) mn[a] = P->pts[3 * i + a];
            if (P->pts[3 * i + a] > mx[a]) mx[a] = P->pts[3 * i + a];
        }
    int64_t total = 1;
    for (int a = 0; a < 3; a++) {
        B->lo[a] = (int64_t)floor((mn[a] - cutoff) / bh) - 2;
        B->dim[a] = (int64_t)ceil((mx[a] + cutoff) / bh) + 2 - B->lo[a] + 1;
        total *= B->dim[a];
    }
    B->memo = (double*)malloc(sizeof(double) * total);
    for (int64_t i = 0; i < total; i++) B->memo[i] = NAN;
    return B;
}

void orc_blur_free(orc_blur* B) {
    if (!B) return;
    free(B->memo);
    free(B);
}

/* rho at node (i,j,k) by its definition (sum over points in input order). */
double orc_rho_node(const orc_pocket* P, orc_blur* B, int64_t i, int64_t j, int64_t k) {
    int64_t ix = i - B->lo[0], iy = j - B->lo[1], iz = k - B->lo[2];
    int inside = ix >= 0 && iy >= 0 && iz >= 0 && ix < B->dim[0] && iy < B->dim[1] && iz < B->dim[2];
    if (!inside) return 0.0; /* farther than the cutoff from every point */
    int64_t idx = (iz * B->dim[1] + iy) * B->dim[0] + ix;
    if (!isnan(B->memo[idx])) return B->memo[idx];
    double g[3] = {B->bh * (double)i, B->bh * (double)j, B->bh * (double)k};
    double cut2 = B->cutoff * B->cutoff, inv2s2 = 1.0 / (2.0 * B->sigma * B->sigma);
    double s = 0.0;
    for (int p = 0; p < P->n_points; p++) {
        double d2 = dist2(g, P->pts + 3 * p);
        if (d2 <= cut2) s += exp(-d2 * inv2s2);
    }
    B->memo[idx] = s;
    return s;
}

/* Trilinear interpolation of rho at x and its gradient. */
double orc_rho_interp(const orc_pocket* P, orc_blur* B, const double* x, double* grad) {
    double u[3], f[3];
    int64_t c[3];
    for (int a = 0; a < 3; a++) {
        u[a] = x[a] / B->bh;
        c[a] = (int64_t)floor(u[a]);
        f[a] = u[a] - (double)c[a];
    }
    double v = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int dz = 0; dz < 2; dz++)
        for (int dy = 0; dy < 2; dy++)
            for (int dx = 0; dx < 2; dx++) {
                double r = orc_rho_node(P, B, c[0] + dx, c[1] + dy, c[2] + dz);
                double wx = dx ? f[0] : 1.0 - f[0], wy = dy ? f[1] : 1.0 - f[1], wz = dz ? f[2] : 1.0 - f[2];
                double sx = dx ? 1.0 : -1.0, sy = dy ? 1.0 : -1.0, sz = dz ? 1.0 : -1.0;
                v += wx * wy * wz * r;
                gx += sx * wy * wz * r;
                gy += wx * sy * wz * r;
                gz += wx * wy * sz * r;
            }
    if (grad) { grad[0] = gx / B->bh; grad[1] = gy / B->bh; grad[2] = gz / B->bh; }
    return v;
}

/* Torsion tree: rotamers in root-first order with near/far atoms and the
 * moving side (the side without atom 0). */
typedef struct {
    int nr;
    int* order;          /* root-first order of rotamer indices */
    int* near_atom;      /* per rotamer */
    int* far_atom;
    unsigned char* mov;  /* nr x l */
} orc_tree;

static void tree_free(orc_tree* T) { free(T->order); free(T->near_atom); free(T->far_atom); free(T->mov); }

static int tree_build(const orc_topo* T, orc_tree* R) {
    int l = T->l, nr = T->nr;
    R->nr = nr;
    R->order = (int*)malloc(sizeof(int) * (nr > 0 ? nr : 1));
    R->near_atom = (int*)malloc(sizeof(int) * (nr > 0 ? nr : 1));
    R->far_atom = (int*)malloc(sizeof(int) * (nr > 0 ? nr : 1));
    R->mov = (unsigned char*)calloc((size_t)(nr > 0 ? nr : 1) * l, 1);
    const int* d0 = T->dist; /* distances from atom 0 */
    for (int r = 0; r < nr; r++) {
        int a = T->rot[2 * r], c = T->rot[2 * r + 1];
        int root_left = T->left[(size_t)r * l + 0];
        R->near_atom[r] = root_left ? a : c;
        R->far_atom[r] = root_left ? c : a;
        for (int i = 0; i < l; i++) {
            int in_left = T->left[(size_t)r * l + i];
            R->mov[(size_t)r * l + i] = root_left ? !in_left : in_left;
        }
        R->order[r] = r;
    }
    /* stable insertion sort by the near atom's bond distance from atom 0 */
    for (int i = 1; i < nr; i++) {
        int v = R->order[i], j = i - 1;
        while (j >= 0 && d0[R->near_atom[R->order[j]]] > d0[R->near_atom[v]]) { R->order[j + 1] = R->order[j]; j--; }
        R->order[j + 1] = v;
    }
    return ORC_OK;
}

/* Rotate the moving set of rotamer r by angle (radians) about its current axis. */
static void fk_rotate(const orc_tree* R, int l, int r, double ang, double* X) {
    int na = R->near_atom[r], fa = R->far_atom[r];
    double k[3] = {X[3 * fa] - X[3 * na], X[3 * fa + 1] - X[3 * na + 1], X[3 * fa + 2] - X[3 * na + 2]};
    double nrm = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    k[0] /= nrm; k[1] /= nrm; k[2] /= nrm;
    double c = cos(ang), s = sin(ang), t = 1.0 - c;
    double M[9];
    M[0] = t * k[0] * k[0] + c;        M[1] = t * k[0] * k[1] - s * k[2]; M[2] = t * k[0] * k[2] + s * k[1];
    M[3] = t * k[0] * k[1] + s * k[2]; M[4] = t * k[1] * k[1] + c;        M[5] = t * k[1] * k[2] - s * k[0];
    M[6] = t * k[0] * k[2] - s * k[1]; M[7] = t * k[1] * k[2] + s * k[0]; M[8] = t * k[2] * k[2] + c;
    double p[3] = {X[3 * na], X[3 * na + 1], X[3 * na + 2]};
    for (int i = 0; i < l; i++)
        if (R->mov[(size_t)r * l + i]) {
            double y[3];
            rotate_about(p, M, X + 3 * i, y);
            X[3 * i] = y[0]; X[3 * i + 1] = y[1]; X[3 * i + 2] = y[2];
        }
}

/* Pose from parameters; Y gets FK_tau(X0) (before the rigid motion). */
static void pose_from_params(const orc_tree* R, int l, const double* X0, const double* c0, const double* prm,
                             double* Y, double* X) {
    memcpy(Y, X0, sizeof(double) * 3 * l);
    for (int k = 0; k < R->nr; k++) {
        int r = R->order[k];
        fk_rotate(R, l, r, prm[7 + r], Y);
    }
    double Rq[9];
    quat_matrix(prm + 3, Rq);
    for (int i = 0; i < l; i++) {
        double d0 = Y[3 * i] - c0[0], d1 = Y[3 * i + 1] - c0[1], d2 = Y[3 * i + 2] - c0[2];
        X[3 * i] = (Rq[0] * d0 + Rq[1] * d1 + Rq[2] * d2) + c0[0] + prm[0];
        X[3 * i + 1] = (Rq[3] * d0 + Rq[4] * d1 + Rq[5] * d2) + c0[1] + prm[1];
        X[3 * i + 2] = (Rq[6] * d0 + Rq[7] * d1 + Rq[8] * d2) + c0[2] + prm[2];
    }
}

/* d R(qhat) / d qhat_k for the unit-quaternion matrix of quat_matrix. */
static void dquat(const double* q, double D[4][9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double Dw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
    double Dx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
    double Dy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
    double Dz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
    memcpy(D[0], Dw, sizeof(Dw)); memcpy(D[1], Dx, sizeof(Dx)); memcpy(D[2], Dy, sizeof(Dy)); memcpy(D[3], Dz, sizeof(Dz));
}

/* Bump penalty of the clash-penalised surrogate (an extension beyond the
 * paper): pen = lam sum over pairs (i < j) at least minb bonds apart with
 * d^2 < cd2 of (cd2 - d^2)^2.  Returns pen and subtracts d pen / dX_i from
 * g (the gradient of F - pen). */
static double bump_penalty(const orc_topo* T, int l, const double* X, double lam, double cd2, int minb, double* g) {
    double pen = 0.0;
    for (int i = 0; i < l; i++)
        for (int j = i + 1; j < l; j++) {
            if (T->dist[(size_t)i * l + j] < minb) continue;
            double d[3] = {X[3 * i] - X[3 * j], X[3 * i + 1] - X[3 * j + 1], X[3 * i + 2] - X[3 * j + 2]};
            double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (d2 >= cd2) continue;
            double e = cd2 - d2;
            pen += e * e;
            /* d(e^2)/dX_i = -4 e d, so -lam d(e^2)/dX_i = 4 lam e d */
            for (int a = 0; a < 3; a++) {
                g[3 * i + a] += 4.0 * lam * e * d[a];
                g[3 * j + a] -= 4.0 * lam * e * d[a];
            }
        }
    return lam * pen;
}

/*
 * Surrogate value and analytic gradient.  prm = [t(3), q(4), tau(nr)];
 * grad (may be NULL) gets dF/dprm; X (may be NULL) the pose.  With lam > 0
 * the value is F - pen (bump_penalty above).
 */
static double surrogate_eval(const orc_pocket* P, orc_blur* B, const orc_tree* R, int l, const double* X0,
                             const double* c0, const double* prm, double* grad, double* Xout, const orc_topo* T,
                             double lam, double cd2, int minb) {
    double* Y = (double*)malloc(sizeof(double) * 3 * l);
    double* X = (double*)malloc(sizeof(double) * 3 * l);
    double* g = (double*)malloc(sizeof(double) * 3 * l);
    pose_from_params(R, l, X0, c0, prm, Y, X);
    double F = 0.0;
    for (int i = 0; i < l; i++) F += orc_rho_interp(P, B, X + 3 * i, g + 3 * i);
    if (lam > 0.0) F -= bump_penalty(T, l, X, lam, cd2, minb, g);
    if (grad) {
        int nr = R->nr;
        for (int k = 0; k < 7 + nr; k++) grad[k] = 0.0;
        for (int i = 0; i < l; i++)
            for (int a = 0; a < 3; a++) grad[a] += g[3 * i + a];
        /* quaternion: G = sum_i g_i (Y_i - c0)^T, dF/dqhat_k = <G, dR/dqhat_k> */
        double G[9] = {0};
        for (int i = 0; i < l; i++)
            for (int r = 0; r < 3; r++)
                for (int c = 0; c < 3; c++) G[3 * r + c] += g[3 * i + r] * (Y[3 * i + c] - c0[c]);
        const double* q = prm + 3;
        double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        double qh[4] = {q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn};
        double D[4][9], gqh[4];
        dquat(qh, D);
        for (int k = 0; k < 4; k++) {
            gqh[k] = 0.0;
            for (int e = 0; e < 9; e++) gqh[k] += G[e] * D[k][e];
        }
        double dot = qh[0] * gqh[0] + qh[1] * gqh[1] + qh[2] * gqh[2] + qh[3] * gqh[3];
        for (int k = 0; k < 4; k++) grad[3 + k] = (gqh[k] - qh[k] * dot) / qn;
        /* torsions: dF/dtau_b = K_b . sum_{i moving} (X_i - A_b) x g_i, final frame */
        for (int r = 0; r < nr; r++) {
            int na = R->near_atom[r], fa = R->far_atom[r];
            double K[3] = {X[3 * fa] - X[3 * na], X[3 * fa + 1] - X[3 * na + 1], X[3 * fa + 2] - X[3 * na + 2]};
            double nrm = sqrt(K[0] * K[0] + K[1] * K[1] + K[2] * K[2]);
            K[0] /= nrm; K[1] /= nrm; K[2] /= nrm;
            double tq[3] = {0, 0, 0};
            for (int i = 0; i < l; i++) {
                if (!R->mov[(size_t)r * l + i]) continue;
                double d[3] = {X[3 * i] - X[3 * na], X[3 * i + 1] - X[3 * na + 1], X[3 * i + 2] - X[3 * na + 2]};
                const double* gi = g + 3 * i;
                tq[0] += d[1] * gi[2] - d[2] * gi[1];
                tq[1] += d[2] * gi[0] - d[0] * gi[2];
                tq[2] += d[0] * gi[1] - d[1] * gi[0];
            }
            grad[7 + r] = K[0] * tq[0] + K[1] * tq[1] + K[2] * tq[2];
        }
    }
    if (Xout) memcpy(Xout, X, sizeof(double) * 3 * l);
    free(Y); free(X); free(g);
    return F;
}

static void centroid3(int l, const double* X, double* c) {
    double s[3] = {0, 0, 0};
    for (int i = 0; i < l; i++) { s[0] = s[0] + X[3 * i]; s[1] = s[1] + X[3 * i + 1]; s[2] = s[2] + X[3 * i + 2]; }
    c[0] = s[0] / (double)l; c[1] = s[1] / (double)l; c[2] = s[2] / (double)l;
}

/* Public: surrogate value, gradient and pose at given parameters. */
int orc_surrogate(orc_pocket* P, orc_blur* B, int l, int nb, const int* bonds, int nr, const int* rot,
                  const double* X0, const double* prm, double lam, double clash_dist, int clash_min_bonds, double* F,
                  double* grad, double* X) {
    orc_topo T;
    int rc = topo_build(&T, l, nb, bonds, nr, rot);
    if (rc != ORC_OK) { topo_free(&T); return rc; }
    orc_tree R;
    tree_build(&T, &R);
    double c0[3];
    centroid3(l, X0, c0);
    *F = surrogate_eval(P, B, &R, l, X0, c0, prm, grad, X, &T, lam, clash_dist * clash_dist, clash_min_bonds);
    tree_free(&R);
    topo_free(&T);
    return ORC_OK;
}

/*
 * Gradient ascent on F from t = 0, q = (1,0,0,0), tau = 0:
 *   dt = lr_t grad_t scaled down to |dt| <= max_dt;  q <- (q + lr_q grad_q)/|.|;
 *   tau_b += clamp(lr_tau grad_tau_b, -max_dtau, max_dtau).
 * Outputs the final parameters, pose and F of the final iterate.
 */
int orc_refine(orc_pocket* P, orc_blur* B, int l, int nb, const int* bonds, int nr, const int* rot, const double* X0,
               int steps, double lr_t, double lr_q, double lr_tau, double max_dt, double max_dtau, double lam,
               double clash_dist, int clash_min_bonds, double* prm_out, double* X_out, double* F_out) {
    const double cd2 = clash_dist * clash_dist;
    orc_topo T;
    int rc = topo_build(&T, l, nb, bonds, nr, rot);
    if (rc != ORC_OK) { topo_free(&T); return rc; }
    orc_tree R;
    tree_build(&T, &R);
    double c0[3];
    centroid3(l, X0, c0);
    int np = 7 + nr;
    double* prm = (double*)calloc(np, sizeof(double));
    double* grad = (double*)calloc(np, sizeof(double));
    prm[3] = 1.0;
    for (int s = 0; s < steps; s++) {
        surrogate_eval(P, B, &R, l, X0, c0, prm, grad, NULL, &T, lam, cd2, clash_min_bonds);
        double dt[3] = {lr_t * grad[0], lr_t * grad[1], lr_t * grad[2]};
        double n = sqrt(dt[0] * dt[0] + dt[1] * dt[1] + dt[2] * dt[2]);
        double sc = n > max_dt ? max_dt / n : 1.0;
        for (int a = 0; a < 3; a++) prm[a] += dt[a] * sc;
        double qn = 0.0;
        for (int k = 0; k < 4; k++) { prm[3 + k] += lr_q * grad[3 + k]; qn += prm[3 + k] * prm[3 + k]; }
        qn = sqrt(qn);
        for (int k = 0; k < 4; k++) prm[3 + k] /= qn;
        for (int r = 0; r < nr; r++) {
            double d = lr_tau * grad[7 + r];
            if (d > max_dtau) d = max_dtau;
            if (d < -max_dtau) d = -max_dtau;
            prm[7 + r] += d;
        }
    }
    *F_out = surrogate_eval(P, B, &R, l, X0, c0, prm, NULL, X_out, &T, lam, cd2, clash_min_bonds);
    memcpy(prm_out, prm, sizeof(double) * np);
    free(prm); free(grad);
    tree_free(&R);
    topo_free(&T);
    return ORC_OK;
}

/* Root-first order and moving sides of the torsion tree (for tests). */
int orc_torsion_tree(int l, int nb, const int* bonds, int nr, const int* rot, int* order, int* near_atom,
                     int* far_atom, uint8_t* mov) {
    orc_topo T;
    int rc = topo_build(&T, l, nb, bonds, nr, rot);
    if (rc != ORC_OK) { topo_free(&T); return rc; }
    orc_tree R;
    tree_build(&T, &R);
    memcpy(order, R.order, sizeof(int) * nr);
    memcpy(near_atom, R.near_atom, sizeof(int) * nr);
    memcpy(far_atom, R.far_atom, sizeof(int) * nr);
    memcpy(mov, R.mov, (size_t)nr * l);
    tree_free(&R);
    topo_free(&T);
    return ORC_OK;
}
