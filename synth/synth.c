/*
 * Seeded synthetic inputs for the geometric docking hot path.
 *
 * The paper evaluates on a private library of drug-like ligands (28-153
 * atoms, 2-53 rotatable bonds) and six PASS pockets (Section IV-A).  Neither
 * is available, so this module generates stand-ins with the same kind of
 * structure:
 *   - ligands: random trees of heavy atoms (valence cap 4) placed by NeRF
 *     with 1.5 A bonds and 109.5 +/- 3 degree bond angles, optionally fused
 *     to one rigid planar 3-6 membered ring; rotatable bonds are chosen among
 *     non-terminal bridges of the bond graph (Section II defines rotamers as
 *     bonds whose removal splits the ligand into two non-empty fragments);
 *   - pockets: points uniform in an ellipsoid (PASS sphere centres stand-in);
 *   - rigid orientations: uniform unit quaternions (Shoemake's method).
 *
 * This file holds none of the docking method's arithmetic: no scores, no
 * fragment rotations, no clash tests.  Every draw comes from SplitMix64
 * streams keyed by (seed, item index), so any item can be regenerated alone.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define SY_MAX_ATOMS 128

typedef struct { uint64_t s; } sy_rng;

static uint64_t sy_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint64_t sy_next(sy_rng* r) {
    r->s += 0x9E3779B97F4A7C15ull;
    return sy_mix(r->s);
}
/* uniform double in [0,1) with 53 random bits */
static double sy_u01(sy_rng* r) { return (double)(sy_next(r) >> 11) * (1.0 / 9007199254740992.0); }
/* uniform integer in [lo, hi] (inclusive) */
static int sy_int(sy_rng* r, int lo, int hi) {
    uint64_t span = (uint64_t)(hi - lo + 1);
    return lo + (int)(sy_next(r) % span);
}
static sy_rng sy_stream(uint64_t seed, uint64_t index, uint64_t salt) {
    sy_rng r;
    r.s = sy_mix(seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull) ^ sy_mix(index + 0xD1B54A32D192ED03ull * (salt + 1));
    return r;
}

static const double SY_PI = 3.14159265358979323846;

typedef struct { double x, y, z; } v3;
static v3 v3_sub(v3 a, v3 b) { v3 r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static v3 v3_add(v3 a, v3 b) { v3 r = {a.x + b.x, a.y + b.y, a.z + b.z}; return r; }
static v3 v3_scale(v3 a, double s) { v3 r = {a.x * s, a.y * s, a.z * s}; return r; }
static double v3_dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 v3_cross(v3 a, v3 b) {
    v3 r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    return r;
}
static v3 v3_unit(v3 a) { return v3_scale(a, 1.0 / sqrt(v3_dot(a, a))); }

/* NeRF: place D such that |CD| = r, angle(B,C,D) = theta, dihedral(A,B,C,D) = phi. */
static v3 nerf(v3 A, v3 B, v3 C, double r, double theta, double phi) {
    v3 bc = v3_unit(v3_sub(C, B));
    v3 n = v3_unit(v3_cross(v3_sub(B, A), bc));
    v3 m = v3_cross(n, bc);
    double d2x = -r * cos(theta), d2y = r * sin(theta) * cos(phi), d2z = r * sin(theta) * sin(phi);
    v3 d = v3_add(v3_add(v3_scale(bc, d2x), v3_scale(m, d2y)), v3_scale(n, d2z));
    return v3_add(C, d);
}

typedef struct {
    int n_atoms;
    int n_bonds;
    int n_rot;
    float x[SY_MAX_ATOMS], y[SY_MAX_ATOMS], z[SY_MAX_ATOMS];
    int bonds[2 * 2 * SY_MAX_ATOMS];
    int rot[2 * SY_MAX_ATOMS];
} sy_ligand;

/* Is edge (a,c) a bridge of the graph given as adjacency lists? */
static int sy_is_bridge(int n, const int* deg, int adj[][6], int a, int c) {
    int seen[SY_MAX_ATOMS], stack[SY_MAX_ATOMS], sp = 0;
    memset(seen, 0, sizeof(seen));
    seen[a] = 1;
    stack[sp++] = a;
    while (sp) {
        int u = stack[--sp];
        for (int k = 0; k < deg[u]; k++) {
            int w = adj[u][k];
            if ((u == a && w == c) || (u == c && w == a)) continue;
            if (!seen[w]) { seen[w] = 1; stack[sp++] = w; }
        }
    }
    (void)n;
    return !seen[c];
}

/*
 * Generate ligand `index` of the stream `seed`.
 * n_atoms ~ U[lmin,lmax], target rotatable bonds ~ U[bmin,bmax]; with
 * probability ring_frac the ligand carries one rigid ring of 3-6 atoms.
 */
static void sy_make_ligand(uint64_t seed, uint64_t index, int lmin, int lmax, int bmin, int bmax,
                           double ring_frac, sy_ligand* L) {
    sy_rng r = sy_stream(seed, index, 1);
    int n = sy_int(&r, lmin, lmax);
    int want_rot = sy_int(&r, bmin, bmax);
    int ring = 0;
    if (ring_frac > 0.0 && sy_u01(&r) < ring_frac) ring = sy_int(&r, 3, 6);
    if (ring > n) ring = 0;

    v3 pos[SY_MAX_ATOMS];
    int deg[SY_MAX_ATOMS], adj[SY_MAX_ATOMS][6], refp[SY_MAX_ATOMS], nchild[SY_MAX_ATOMS];
    double phi0[SY_MAX_ATOMS];
    memset(deg, 0, sizeof(deg));
    memset(nchild, 0, sizeof(nchild));
    int nb = 0;
    /* virtual reference atoms for the first placements: -1 -> VA, -2 -> VB */
    const v3 VA = {-1.5, 0.0, 0.0}, VB = {-2.0, 1.41, 0.0};
    int placed;

    if (ring) {
        /* regular planar k-gon with 1.5 A sides, centred at the origin */
        double R = 1.5 / (2.0 * sin(SY_PI / ring));
        for (int k = 0; k < ring; k++) {
            double a = 2.0 * SY_PI * k / ring;
            pos[k].x = R * cos(a); pos[k].y = R * sin(a); pos[k].z = 0.0;
            refp[k] = (k + 1) % ring;
            phi0[k] = sy_u01(&r) * 2.0 * SY_PI;
        }
        for (int k = 0; k < ring; k++) {
            int a = k, c = (k + 1) % ring;
            adj[a][deg[a]++] = c; adj[c][deg[c]++] = a;
            L->bonds[2 * nb] = a; L->bonds[2 * nb + 1] = c; nb++;
        }
        placed = ring;
    } else {
        pos[0].x = pos[0].y = pos[0].z = 0.0;
        refp[0] = -1;
        phi0[0] = sy_u01(&r) * 2.0 * SY_PI;
        placed = 1;
    }

    for (int i = placed; i < n; i++) {
        v3 best = {0, 0, 0};
        int best_p = -1;
        double best_min = -1.0;
        for (int attempt = 0; attempt < 24; attempt++) {
            /* random parent with free valence */
            int cand[SY_MAX_ATOMS], nc = 0;
            for (int j = 0; j < i; j++) if (deg[j] < 4) cand[nc++] = j;
            if (nc == 0) break;
            int p = cand[sy_int(&r, 0, nc - 1)];
            int g = refp[p];
            v3 Cp = pos[p];
            v3 Bg = g == -1 ? VA : pos[g];
            v3 Agg;
            if (g == -1) Agg = VB;
            else if (refp[g] == -1) Agg = VA;
            else Agg = pos[refp[g]];
            double theta = (109.5 + (sy_u01(&r) * 6.0 - 3.0)) * SY_PI / 180.0;
            double phi = phi0[p] + (double)(nchild[p] + attempt / 8) * (2.0 * SY_PI / 3.0);
            v3 cand_pos = nerf(Agg, Bg, Cp, 1.5, theta, phi);
            double dmin = 1e30;
            for (int j = 0; j < i; j++) {
                if (j == p) continue;
                v3 d = v3_sub(cand_pos, pos[j]);
                double dd = v3_dot(d, d);
                if (dd < dmin) dmin = dd;
            }
            if (dmin > best_min) { best_min = dmin; best = cand_pos; best_p = p; }
            if (dmin >= 2.2 * 2.2) break;
        }
        int p = best_p;
        pos[i] = best;
        refp[i] = p;
        phi0[i] = sy_u01(&r) * 2.0 * SY_PI;
        nchild[p]++;
        adj[p][deg[p]++] = i; adj[i][deg[i]++] = p;
        L->bonds[2 * nb] = p; L->bonds[2 * nb + 1] = i; nb++;
    }

    /* rotatable bonds: non-terminal bridges, chosen uniformly without replacement */
    int elig[2 * SY_MAX_ATOMS], ne = 0;
    for (int b = 0; b < nb; b++) {
        int a = L->bonds[2 * b], c = L->bonds[2 * b + 1];
        if (deg[a] < 2 || deg[c] < 2) continue;
        if (ring && !sy_is_bridge(n, deg, adj, a, c)) continue;
        elig[ne++] = b;
    }
    int nr = want_rot < ne ? want_rot : ne;
    for (int k = 0; k < nr; k++) {
        int j = sy_int(&r, k, ne - 1);
        int t = elig[k]; elig[k] = elig[j]; elig[j] = t;
        int a = L->bonds[2 * elig[k]], c = L->bonds[2 * elig[k] + 1];
        if (sy_next(&r) & 1) { int s = a; a = c; c = s; }
        L->rot[2 * k] = a; L->rot[2 * k + 1] = c;
    }

    L->n_atoms = n;
    L->n_bonds = nb;
    L->n_rot = nr;
    for (int i = 0; i < n; i++) {
        L->x[i] = (float)pos[i].x; L->y[i] = (float)pos[i].y; L->z[i] = (float)pos[i].z;
    }
}

/*
 * Generate ligands [first, first+count) of stream `seed` into CSR arrays.
 * Capacities: atoms count*lmax, bonds count*(lmax+1)*2 ints, rot count*lmax*2 ints.
 * Returns 0, or -1 if lmax exceeds the generator's atom limit.
 */
int sy_ligands(uint64_t seed, int64_t first, int count, int lmin, int lmax, int bmin, int bmax,
               double ring_frac, int* atom_off, float* x, float* y, float* z, int* bond_off, int* bonds,
               int* rot_off, int* rot) {
    if (lmax > SY_MAX_ATOMS || lmin < 2 || lmin > lmax || bmin < 0 || bmin > bmax) return -1;
    sy_ligand L;
    atom_off[0] = 0; bond_off[0] = 0; rot_off[0] = 0;
    for (int i = 0; i < count; i++) {
        sy_make_ligand(seed, (uint64_t)(first + i), lmin, lmax, bmin, bmax, ring_frac, &L);
        int ao = atom_off[i], bo = bond_off[i], ro = rot_off[i];
        memcpy(x + ao, L.x, sizeof(float) * L.n_atoms);
        memcpy(y + ao, L.y, sizeof(float) * L.n_atoms);
        memcpy(z + ao, L.z, sizeof(float) * L.n_atoms);
        memcpy(bonds + 2 * bo, L.bonds, sizeof(int) * 2 * L.n_bonds);
        memcpy(rot + 2 * ro, L.rot, sizeof(int) * 2 * L.n_rot);
        atom_off[i + 1] = ao + L.n_atoms;
        bond_off[i + 1] = bo + L.n_bonds;
        rot_off[i + 1] = ro + L.n_rot;
    }
    return 0;
}

/* n points uniform in the ellipsoid with semi-axes (ax,ay,az) centred at (cx,cy,cz). */
int sy_pocket(uint64_t seed, int n, double ax, double ay, double az, double cx, double cy, double cz,
              float* xyz) {
    if (n < 1 || ax <= 0 || ay <= 0 || az <= 0) return -1;
    sy_rng r = sy_stream(seed, 0, 2);
    for (int i = 0; i < n; i++) {
        double u, v, w;
        do {
            u = 2.0 * sy_u01(&r) - 1.0;
            v = 2.0 * sy_u01(&r) - 1.0;
            w = 2.0 * sy_u01(&r) - 1.0;
        } while (u * u + v * v + w * w > 1.0);
        xyz[3 * i + 0] = (float)(cx + ax * u);
        xyz[3 * i + 1] = (float)(cy + ay * v);
        xyz[3 * i + 2] = (float)(cz + az * w);
    }
    return 0;
}

/* n uniform unit quaternions (w,x,y,z), w >= 0, by Shoemake's subgroup method. */
int sy_quaternions(uint64_t seed, int n, double* q) {
    if (n < 0) return -1;
    sy_rng r = sy_stream(seed, 0, 3);
    for (int i = 0; i < n; i++) {
        double u1 = sy_u01(&r), u2 = sy_u01(&r), u3 = sy_u01(&r);
        double a = sqrt(1.0 - u1), b = sqrt(u1);
        double w = a * sin(2.0 * SY_PI * u2), x = a * cos(2.0 * SY_PI * u2);
        double y = b * sin(2.0 * SY_PI * u3), zz = b * cos(2.0 * SY_PI * u3);
        if (w < 0) { w = -w; x = -x; y = -y; zz = -zz; }
        q[4 * i + 0] = w; q[4 * i + 1] = x; q[4 * i + 2] = y; q[4 * i + 3] = zz;
    }
    return 0;
}
