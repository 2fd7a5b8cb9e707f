// Host runtime of libgd: argument validation, pocket set-up (occupancy and the
// exact squared distance transform), ligand preparation (bond distances,
// fragments, straddling pairs, angle schedules, work-queue order), device
// memory, HIP-graph capture of the batched form and the C ABI of gd.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <functional>
#include <limits>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "gd_internal.h"
#include "runtime.h"

namespace gd {

// The tilings the docking kernel is instantiated for.
bool tiling_supported(int waves_per_block, int angle_block, int pairs_per_lane) {
    auto in = [](int v, std::initializer_list<int> set) { return std::find(set.begin(), set.end(), v) != set.end(); };
    return in(waves_per_block, {1, 2, 4, 8}) && in(angle_block, {8, 16, 32}) && in(pairs_per_lane, {1, 2, 4, 8});
}

// --------------------------------------------------------------------------
// errors

static thread_local std::string g_last_error;

gd_status fail(gd_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

gd_status hip_fail(hipError_t e, const char* where) {
    return fail(e == hipErrorOutOfMemory ? GD_ERR_OOM : GD_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

void clear_error() { g_last_error.clear(); }
const char* last_error() { return g_last_error.c_str(); }

// --------------------------------------------------------------------------
// trig tables: cos/sin of integer degrees with the argument deg * (pi/180)

void trig_tables(double* c64, double* s64, float* c32, float* s32) {
    const double kPi = 3.14159265358979323846;
    for (int d = 0; d < 360; d++) {
        double rad = (double)d * (kPi / 180.0);
        c64[d] = cos(rad);
        s64[d] = sin(rad);
        c32[d] = (float)c64[d];
        s32[d] = (float)s64[d];
    }
}

// --------------------------------------------------------------------------
// device buffers

DevBuf::~DevBuf() { reset(); }
void DevBuf::reset() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}
hipError_t DevBuf::alloc(size_t n) {
    reset();
    if (n == 0) n = 16;
    hipError_t e = hipMalloc(&ptr, n);
    if (e == hipSuccess) bytes = n;
    else ptr = nullptr;
    return e;
}
hipError_t DevBuf::upload(const void* src, size_t n, hipStream_t s) {
    hipError_t e = alloc(n);
    if (e != hipSuccess) return e;
    if (n == 0) return hipSuccess;
    e = hipMemcpyAsync(ptr, src, n, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

// --------------------------------------------------------------------------
// pocket

static bool is_pow2(float h) {
    if (!(h > 0) || !std::isfinite(h)) return false;
    int e;
    double m = frexp((double)h, &e);
    return m == 0.5;
}

// One dimension of the separable squared distance transform (lower envelope
// of parabolas, Felzenszwalb & Huttenlocher); f and d hold exact integers.
static void dt1d(const double* f, int n, double* d, int* v, double* z) {
    int k = 0;
    v[0] = 0;
    z[0] = -1e300;
    z[1] = 1e300;
    for (int q = 1; q < n; q++) {
        double s = ((f[q] + (double)q * q) - (f[v[k]] + (double)v[k] * v[k])) / (2.0 * q - 2.0 * v[k]);
        while (s <= z[k]) {
            k--;
            s = ((f[q] + (double)q * q) - (f[v[k]] + (double)v[k] * v[k])) / (2.0 * q - 2.0 * v[k]);
        }
        k++;
        v[k] = q;
        z[k] = s;
        z[k + 1] = 1e300;
    }
    k = 0;
    for (int q = 0; q < n; q++) {
        while (z[k + 1] < q) k++;
        double dq = (double)(q - v[k]);
        d[q] = dq * dq + f[v[k]];
    }
}

gd_status create_pocket(const gd_pocket_desc* desc, hipStream_t stream, gd_pocket** out) {
    if (!desc || !out) return fail(GD_ERR_ARG, "gd_create_pocket: null argument");
    *out = nullptr;
    if (!desc->xyz || desc->n_points < 1) return fail(GD_ERR_ARG, "gd_create_pocket: need at least one point");
    if (!is_pow2(desc->grid_h)) return fail(GD_ERR_ARG, "gd_create_pocket: grid_h must be a power of two");
    if (!(desc->pad >= 0) || !std::isfinite(desc->pad) || desc->pad > 200)
        return fail(GD_ERR_ARG, "gd_create_pocket: pad must be in [0, 200]");
    const int n = desc->n_points;
    const double h = desc->grid_h, inv_h = 1.0 / h;
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    double sum[3] = {0, 0, 0};
    for (int i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) {
            double v = (double)desc->xyz[3 * i + a];
            if (!std::isfinite(v) || fabs(v) > 1e4)
                return fail(GD_ERR_ARG, "gd_create_pocket: point %d has a non-finite or huge coordinate", i);
            mn[a] = std::min(mn[a], v);
            mx[a] = std::max(mx[a], v);
        }
    for (int i = 0; i < n; i++) {
        sum[0] = sum[0] + (double)desc->xyz[3 * i];
        sum[1] = sum[1] + (double)desc->xyz[3 * i + 1];
        sum[2] = sum[2] + (double)desc->xyz[3 * i + 2];
    }
    std::unique_ptr<gd_pocket> P(new gd_pocket());
    for (int a = 0; a < 3; a++) P->centroid[a] = sum[a] / (double)n;
    int lo[3], dim[3];
    for (int a = 0; a < 3; a++) {
        lo[a] = (int)floor((mn[a] - desc->pad) * inv_h);
        int hi = (int)floor((mx[a] + desc->pad) * inv_h);
        dim[a] = hi - lo[a] + 1;
        if (dim[a] > 512) return fail(GD_ERR_CAPACITY, "gd_create_pocket: grid box exceeds 512 cells per axis");
    }
    // occupied cells
    std::vector<int32_t> cells(3 * (size_t)n);
    for (int i = 0; i < n; i++)
        for (int a = 0; a < 3; a++) cells[3 * i + a] = (int32_t)floor((double)desc->xyz[3 * i + a] * inv_h);
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        for (int k = 0; k < 3; k++)
            if (cells[3 * a + k] != cells[3 * b + k]) return cells[3 * a + k] < cells[3 * b + k];
        return false;
    });
    std::vector<int32_t> occ;
    for (int idx = 0; idx < n; idx++) {
        int i = order[idx];
        size_t m = occ.size() / 3;
        if (m > 0 && occ[3 * (m - 1)] == cells[3 * i] && occ[3 * (m - 1) + 1] == cells[3 * i + 1] &&
            occ[3 * (m - 1) + 2] == cells[3 * i + 2])
            continue;
        occ.push_back(cells[3 * i]);
        occ.push_back(cells[3 * i + 1]);
        occ.push_back(cells[3 * i + 2]);
    }
    const size_t total = (size_t)dim[0] * dim[1] * dim[2];
    if (total >= ((size_t)1 << 24)) return fail(GD_ERR_CAPACITY, "gd_create_pocket: grid box exceeds 2^24 cells");
    std::vector<double> g(total, 1e15);
    for (size_t m = 0; m < occ.size() / 3; m++) {
        int ix = occ[3 * m] - lo[0], iy = occ[3 * m + 1] - lo[1], iz = occ[3 * m + 2] - lo[2];
        g[((size_t)iz * dim[1] + iy) * dim[0] + ix] = 0.0;
    }
    {
        int nmax = std::max(dim[0], std::max(dim[1], dim[2]));
        std::vector<double> f(nmax), d(nmax), z(nmax + 1);
        std::vector<int> v(nmax);
        for (int iz = 0; iz < dim[2]; iz++)
            for (int iy = 0; iy < dim[1]; iy++) {
                double* row = &g[((size_t)iz * dim[1] + iy) * dim[0]];
                for (int ix = 0; ix < dim[0]; ix++) f[ix] = row[ix];
                dt1d(f.data(), dim[0], d.data(), v.data(), z.data());
                for (int ix = 0; ix < dim[0]; ix++) row[ix] = d[ix];
            }
        for (int iz = 0; iz < dim[2]; iz++)
            for (int ix = 0; ix < dim[0]; ix++) {
                for (int iy = 0; iy < dim[1]; iy++) f[iy] = g[((size_t)iz * dim[1] + iy) * dim[0] + ix];
                dt1d(f.data(), dim[1], d.data(), v.data(), z.data());
                for (int iy = 0; iy < dim[1]; iy++) g[((size_t)iz * dim[1] + iy) * dim[0] + ix] = d[iy];
            }
        for (int iy = 0; iy < dim[1]; iy++)
            for (int ix = 0; ix < dim[0]; ix++) {
                for (int iz = 0; iz < dim[2]; iz++) f[iz] = g[((size_t)iz * dim[1] + iy) * dim[0] + ix];
                dt1d(f.data(), dim[2], d.data(), v.data(), z.data());
                for (int iz = 0; iz < dim[2]; iz++) g[((size_t)iz * dim[1] + iy) * dim[0] + ix] = d[iz];
            }
    }
    std::vector<uint16_t> edt(total + 1, 0);  // + a zero sentinel cell read by masked lanes
    for (size_t i = 0; i < total; i++) {
        if (g[i] > 65535.0) return fail(GD_ERR_CAPACITY, "gd_create_pocket: distance grid value exceeds 65535");
        edt[i] = (uint16_t)g[i];
    }
    hipError_t e;
    if ((e = upload_trig_tables()) != hipSuccess) return hip_fail(e, "gd_create_pocket");
    if ((e = P->edt.upload(edt.data(), edt.size() * 2, stream)) != hipSuccess) return hip_fail(e, "gd_create_pocket");
    if ((e = P->occ.upload(occ.data(), occ.size() * 4, stream)) != hipSuccess) return hip_fail(e, "gd_create_pocket");
    {
        // raw points for the continuous overlap: FP64 planes padded with far points
        const int pad_n = (n + kOvUnroll - 1) / kOvUnroll * kOvUnroll;
        std::vector<double> pl((size_t)3 * pad_n, 1e150);
        for (int i = 0; i < n; i++)
            for (int a = 0; a < 3; a++) pl[(size_t)a * pad_n + i] = (double)desc->xyz[3 * i + a];
        if ((e = P->pts.upload(pl.data(), pl.size() * sizeof(double), stream)) != hipSuccess)
            return hip_fail(e, "gd_create_pocket");
        P->n_points = n;
        P->pts_pad = pad_n;
    }
    PocketDev& D = P->dev;
    D.edt = (const uint16_t*)P->edt.ptr;
    D.n_cells = (int32_t)total;
    D.occ = (const int32_t*)P->occ.ptr;
    D.n_occ = (int32_t)(occ.size() / 3);
    for (int a = 0; a < 3; a++) {
        D.lo[a] = lo[a];
        D.dim[a] = dim[a];
        D.cP[a] = P->centroid[a];
    }
    D.h = h;
    D.inv_h = inv_h;
    D.rho = nullptr;
    D.rho4 = nullptr;
    for (int a = 0; a < 3; a++) {
        D.blo[a] = 0;
        D.bdim[a] = 0;
    }
    D.bh = 0.f;
    D.inv_bh = 0.f;
    // blurred density grid for the refinement surrogate
    if (desc->blur_sigma > 0) {
        const double sg = desc->blur_sigma, bh = desc->blur_h, cut = (double)desc->blur_cutoff_sigmas * sg;
        if (!(bh > 0) || !(cut > 0) || !(desc->blur_pad >= 0))
            return fail(GD_ERR_ARG, "gd_create_pocket: bad density grid parameters");
        int blo[3], bdim[3];
        size_t btot = 1;
        for (int a = 0; a < 3; a++) {
            blo[a] = (int)floor((mn[a] - desc->blur_pad) / bh);
            int bhi = (int)ceil((mx[a] + desc->blur_pad) / bh);
            bdim[a] = bhi - blo[a] + 1;
            if (bdim[a] > 1024) return fail(GD_ERR_CAPACITY, "gd_create_pocket: density grid too large");
            btot *= bdim[a];
        }
        // the plain grid and its corner-packed copy (about 4x) stay within a few GiB
        if (btot > ((size_t)1 << 28)) return fail(GD_ERR_CAPACITY, "gd_create_pocket: density grid too large");
        std::vector<double> rho(btot, 0.0);
        const double cut2 = cut * cut, inv2s2 = 1.0 / (2.0 * sg * sg);
        const int reach = (int)ceil(cut / bh) + 1;
        for (int j = 0; j < n; j++) {
            double p[3] = {(double)desc->xyz[3 * j], (double)desc->xyz[3 * j + 1], (double)desc->xyz[3 * j + 2]};
            int c[3];
            for (int a = 0; a < 3; a++) c[a] = (int)floor(p[a] / bh) - blo[a];
            for (int iz = std::max(0, c[2] - reach); iz <= std::min(bdim[2] - 1, c[2] + reach); iz++)
                for (int iy = std::max(0, c[1] - reach); iy <= std::min(bdim[1] - 1, c[1] + reach); iy++)
                    for (int ix = std::max(0, c[0] - reach); ix <= std::min(bdim[0] - 1, c[0] + reach); ix++) {
                        double gx = bh * (double)(ix + blo[0]) - p[0];
                        double gy = bh * (double)(iy + blo[1]) - p[1];
                        double gz = bh * (double)(iz + blo[2]) - p[2];
                        double d2 = gx * gx + gy * gy + gz * gz;
                        if (d2 <= cut2) rho[((size_t)iz * bdim[1] + iy) * bdim[0] + ix] += exp(-d2 * inv2s2);
                    }
        }
        std::vector<float> rf(btot);
        for (size_t i = 0; i < btot; i++) rf[i] = (float)rho[i];
        if ((e = P->rho.upload(rf.data(), rf.size() * 4, stream)) != hipSuccess) return hip_fail(e, "gd_create_pocket");
        D.rho = (const float*)P->rho.ptr;
        // corner-packed copy for the trilinear gathers (see PocketDev::rho4)
        const int qx = bdim[0] + 1, qy = bdim[1] + 1, qz = bdim[2] + 2;
        std::vector<float> pk((size_t)qx * qy * qz * 4, 0.f);
        auto at = [&](int x, int y, int z) {
            return (x >= 0 && x < bdim[0] && y >= 0 && y < bdim[1] && z >= 0 && z < bdim[2])
                       ? rf[((size_t)z * bdim[1] + y) * bdim[0] + x]
                       : 0.f;
        };
        for (int z = -1; z <= bdim[2]; z++)
            for (int y = -1; y < bdim[1]; y++)
                for (int x = -1; x < bdim[0]; x++) {
                    float* o = &pk[4 * (((size_t)(z + 1) * qy + (y + 1)) * qx + (x + 1))];
                    o[0] = at(x, y, z);
                    o[1] = at(x + 1, y, z);
                    o[2] = at(x, y + 1, z);
                    o[3] = at(x + 1, y + 1, z);
                }
        if ((e = P->rho4.upload(pk.data(), pk.size() * 4, stream)) != hipSuccess)
            return hip_fail(e, "gd_create_pocket");
        D.rho4 = (const float4*)P->rho4.ptr;
        for (int a = 0; a < 3; a++) {
            D.blo[a] = blo[a];
            D.bdim[a] = bdim[a];
        }
        D.bh = (float)bh;
        D.inv_bh = (float)(1.0 / bh);
        P->blur_h = bh;
    }
    if ((e = P->devcopy.upload(&P->dev, sizeof(PocketDev), stream)) != hipSuccess) return hip_fail(e, "gd_create_pocket");
    *out = P.release();
    return GD_OK;
}

// --------------------------------------------------------------------------
// ligand preparation

int tile_size(int hp) {
    int best = -1, besty = 0;
    for (int x = hp; x <= 360; x += hp) {
        if (360 % x) continue;
        int y = 360 / x + x / hp;
        if (best < 0 || y < besty) {
            best = x;
            besty = y;
        }
    }
    return best;
}

static bool step_ok(int s) { return s >= 1 && s <= 360 && 360 % s == 0; }

gd_status validate_knobs(const gd_knobs* k) {
    if (!k) return fail(GD_ERR_ARG, "knobs: null");
    if (!step_ok(k->hp_step_deg)) return fail(GD_ERR_KNOB, "knobs: hp_step_deg must be an integer divisor of 360");
    if (!step_ok(k->lp_step_deg)) return fail(GD_ERR_KNOB, "knobs: lp_step_deg must be an integer divisor of 360");
    if (!(k->threshold >= 0.f && k->threshold <= 1.f)) return fail(GD_ERR_KNOB, "knobs: threshold outside [0, 1]");
    if (k->repetitions < 1 || k->repetitions > 64) return fail(GD_ERR_KNOB, "knobs: repetitions outside [1, 64]");
    if (k->n_orient < 1 || k->n_orient > 65535) return fail(GD_ERR_KNOB, "knobs: n_orient outside [1, 65535]");
    if (!k->quats) return fail(GD_ERR_ARG, "knobs: null quaternions");
    if (k->top_k < 1 || k->top_k > k->n_orient) return fail(GD_ERR_KNOB, "knobs: top_k outside [1, n_orient]");
    if (!(k->clash_dist >= 0.f) || !std::isfinite(k->clash_dist) || k->clash_dist > 100.f)
        return fail(GD_ERR_KNOB, "knobs: clash_dist outside [0, 100]");
    if (k->clash_min_bonds < 1 || k->clash_min_bonds > 255) return fail(GD_ERR_KNOB, "knobs: clash_min_bonds < 1");
    for (int o = 0; o < k->n_orient; o++) {
        const double* q = k->quats + 4 * (size_t)o;
        double nn = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
        if (!std::isfinite(nn) || !(fabs(sqrt(nn) - 1.0) < 1e-6))
            return fail(GD_ERR_KNOB, "knobs: quaternion %d is not a unit quaternion", o);
    }
    return GD_OK;
}

// Topology of one ligand: validation, bond-count distances, fragments.
struct Topo {
    int l = 0, nb = 0, nr = 0;
    std::vector<std::vector<int>> adj;
    std::vector<uint8_t> dist;  // l*l, saturated at 255
    std::vector<uint8_t> left;  // nr*l
};

static gd_status build_topo(const gd_ligands* L, int i, Topo& T) {
    const int a0 = L->atom_off[i], a1 = L->atom_off[i + 1];
    const int b0 = L->bond_off[i], b1 = L->bond_off[i + 1];
    const int r0 = L->rot_off[i], r1 = L->rot_off[i + 1];
    const int l = a1 - a0, nb = b1 - b0, nr = r1 - r0;
    if (l < 1 || nb < 0 || nr < 0) return fail(GD_ERR_GRAPH, "ligand %d: bad offsets", i);
    if (l > kMaxAtoms) return fail(GD_ERR_GRAPH, "ligand %d: %d atoms exceed the limit of %d", i, l, kMaxAtoms);
    if (nr > kMaxRot) return fail(GD_ERR_ROTAMER, "ligand %d: %d rotamers exceed the limit of %d", i, nr, kMaxRot);
    T.l = l;
    T.nb = nb;
    T.nr = nr;
    T.adj.assign(l, {});
    for (int a = a0; a < a1; a++) {
        float c[3] = {L->x[a], L->y[a], L->z[a]};
        for (float v : c)
            if (!std::isfinite(v) || fabsf(v) > 1e4f)
                return fail(GD_ERR_ARG, "ligand %d: non-finite or huge coordinate", i);
    }
    for (int b = 0; b < nb; b++) {
        int a = L->bonds[2 * (b0 + b)], c = L->bonds[2 * (b0 + b) + 1];
        if (a < 0 || c < 0 || a >= l || c >= l || a == c)
            return fail(GD_ERR_GRAPH, "ligand %d: bond %d has an invalid atom index", i, b);
        for (int w : T.adj[a])
            if (w == c) return fail(GD_ERR_GRAPH, "ligand %d: duplicate bond %d-%d", i, a, c);
        double bx = (double)L->x[a0 + a] - L->x[a0 + c], by = (double)L->y[a0 + a] - L->y[a0 + c],
               bz = (double)L->z[a0 + a] - L->z[a0 + c];
        if (!(bx * bx + by * by + bz * bz > 1e-6))
            return fail(GD_ERR_GRAPH, "ligand %d: bond %d-%d has zero length", i, a, c);
        T.adj[a].push_back(c);
        T.adj[c].push_back(a);
    }
    T.dist.assign((size_t)l * l, 255);
    std::vector<int> q(l);
    for (int s = 0; s < l; s++) {
        uint8_t* d = &T.dist[(size_t)s * l];
        int qh = 0, qt = 0;
        d[s] = 0;
        q[qt++] = s;
        while (qh < qt) {
            int u = q[qh++];
            for (int w : T.adj[u])
                if (d[w] == 255) {
                    d[w] = (uint8_t)std::min(254, d[u] + 1);
                    q[qt++] = w;
                }
        }
        if (qt != l) return fail(GD_ERR_GRAPH, "ligand %d: bond graph is disconnected", i);
    }
    T.left.assign((size_t)std::max(nr, 1) * l, 0);
    for (int r = 0; r < nr; r++) {
        int a = L->rot[2 * (r0 + r)], c = L->rot[2 * (r0 + r) + 1];
        if (a < 0 || c < 0 || a >= l || c >= l || a == c)
            return fail(GD_ERR_ROTAMER, "ligand %d: rotamer %d has an invalid atom index", i, r);
        bool bond = false;
        for (int w : T.adj[a]) bond |= w == c;
        if (!bond) return fail(GD_ERR_ROTAMER, "ligand %d: rotamer %d (%d-%d) is not a bond", i, r, a, c);
        if (T.adj[a].size() < 2 || T.adj[c].size() < 2)
            return fail(GD_ERR_ROTAMER, "ligand %d: rotamer %d (%d-%d) has a terminal atom", i, r, a, c);
        uint8_t* m = &T.left[(size_t)r * l];
        int qh = 0, qt = 0;
        m[a] = 1;
        q[qt++] = a;
        while (qh < qt) {
            int u = q[qh++];
            for (int w : T.adj[u]) {
                if ((u == a && w == c) || (u == c && w == a)) continue;
                if (!m[w]) {
                    m[w] = 1;
                    q[qt++] = w;
                }
            }
        }
        if (m[c]) return fail(GD_ERR_ROTAMER, "ligand %d: rotamer %d (%d-%d) is not a bridge", i, r, a, c);
    }
    return GD_OK;
}

gd_status validate_ligands_struct(const gd_ligands* L) {
    if (!L) return fail(GD_ERR_ARG, "ligands: null");
    if (L->n_ligands < 1) return fail(GD_ERR_ARG, "ligands: n_ligands < 1");
    if (!L->atom_off || !L->x || !L->y || !L->z || !L->bond_off || !L->rot_off)
        return fail(GD_ERR_ARG, "ligands: null array");
    for (int i = 0; i < L->n_ligands; i++) {
        if (L->atom_off[i + 1] < L->atom_off[i] || L->bond_off[i + 1] < L->bond_off[i] ||
            L->rot_off[i + 1] < L->rot_off[i])
            return fail(GD_ERR_ARG, "ligands: offsets not ascending at %d", i);
    }
    if (L->atom_off[0] != 0 || L->bond_off[0] != 0 || L->rot_off[0] != 0)
        return fail(GD_ERR_ARG, "ligands: offsets must start at 0");
    if (L->bond_off[L->n_ligands] > 0 && !L->bonds) return fail(GD_ERR_ARG, "ligands: null bonds");
    if (L->rot_off[L->n_ligands] > 0 && !L->rot) return fail(GD_ERR_ARG, "ligands: null rotamers");
    return GD_OK;
}

// Per-ligand host product of the preparation.
struct LigPrep {
    gd_status st = GD_OK;
    std::string err;
    LigMeta meta{};
    std::vector<RotInfo> rot;
    std::vector<uint16_t> pairs, efar;
    std::vector<uint8_t> mv;
    double cost = 0;
    double flops = 0, bytes = 0;  // direct-evaluation work per orientation
    int nmax = 1;
    int64_t n_pairs = 0;
};

static void prep_one(const gd_ligands* L, const gd_knobs* K, int i, bool topo_only, int minb, LigPrep& out) {
    Topo T;
    gd_status st = build_topo(L, i, T);
    if (st != GD_OK) {
        out.st = st;
        out.err = last_error();
        return;
    }
    const int l = T.l, nr = T.nr;
    const int a0 = L->atom_off[i];
    const int r0 = L->rot_off[i];
    double sx = 0, sy = 0, sz = 0;
    for (int a = 0; a < l; a++) {
        sx = sx + (double)L->x[a0 + a];
        sy = sy + (double)L->y[a0 + a];
        sz = sz + (double)L->z[a0 + a];
    }
    LigMeta& M = out.meta;
    M.cL[0] = sx / (double)l;
    M.cL[1] = sy / (double)l;
    M.cL[2] = sz / (double)l;
    M.atom_off = a0;
    M.l = l;
    M.nr = nr;
    for (int a = 0; a < l; a++)
        for (int b = a + 1; b < l; b++)
            if (T.dist[(size_t)a * l + b] >= minb) out.efar.push_back((uint16_t)(a | (b << 8)));
    if (topo_only) return;
    int64_t cand = 0;
    double cost = 0;
    for (int r = 0; r < nr; r++) {
        RotInfo ri{};
        ri.a = L->rot[2 * (r0 + r)];
        ri.c = L->rot[2 * (r0 + r) + 1];
        const uint8_t* m = &T.left[(size_t)r * l];
        ri.pair_off = (int32_t)out.pairs.size();
        for (int a = 0; a < l; a++) {
            if (!m[a]) continue;
            for (int b = 0; b < l; b++)
                if (!m[b] && T.dist[(size_t)a * l + b] >= minb) out.pairs.push_back((uint16_t)(a | (b << 8)));
        }
        ri.n_pairs = (int32_t)out.pairs.size() - ri.pair_off;
        // each side's moving atoms farthest from the bond axis first (in the
        // input conformation): a candidate's partial sum then tends to reach
        // the sweep's bound in fewer steps (S is an integer sum, so the order
        // does not change any result)
        const double ax = (double)L->x[a0 + ri.c] - L->x[a0 + ri.a], ay = (double)L->y[a0 + ri.c] - L->y[a0 + ri.a],
                     az = (double)L->z[a0 + ri.c] - L->z[a0 + ri.a];
        const double an = std::sqrt(ax * ax + ay * ay + az * az);
        auto radial = [&](int a) {
            const double ux = (double)L->x[a0 + a] - L->x[a0 + ri.a], uy = (double)L->y[a0 + a] - L->y[a0 + ri.a],
                         uz = (double)L->z[a0 + a] - L->z[a0 + ri.a];
            const double cx = uy * az - uz * ay, cy = uz * ax - ux * az, cz = ux * ay - uy * ax;
            return an > 0 ? std::sqrt(cx * cx + cy * cy + cz * cz) / an : 0.0;
        };
        for (int side = 0; side < 2; side++) {
            ri.mv_off[side] = (int32_t)out.mv.size();
            std::vector<std::pair<double, int>> order;
            for (int a = 0; a < l; a++)
                if ((m[a] != 0) == (side == 0)) order.push_back({-radial(a), a});
            std::stable_sort(order.begin(), order.end(),
                             [](const std::pair<double, int>& p, const std::pair<double, int>& q) { return p.first < q.first; });
            for (const auto& e : order) out.mv.push_back((uint8_t)e.second);
            ri.n_mv[side] = (int32_t)out.mv.size() - ri.mv_off[side];
            double rel = (double)ri.n_mv[side] / (double)l;
            if (rel <= (double)K->threshold) {
                ri.mode[side] = kFlat;
                ri.step[side] = K->lp_step_deg;
                ri.n_cand[side] = 360 / K->lp_step_deg;
                out.nmax = std::max(out.nmax, ri.n_cand[side]);
            } else if (K->enable_refinement) {
                int hp = K->hp_step_deg, x = tile_size(hp);
                ri.mode[side] = kPeel;
                ri.step[side] = hp;
                ri.tile[side] = x;
                ri.off[side] = (x / (2 * hp)) * hp;
                ri.n_cand[side] = 360 / x + x / hp;
                out.nmax = std::max(out.nmax, std::max(360 / x, x / hp));
            } else {
                ri.mode[side] = kFlat;
                ri.step[side] = K->hp_step_deg;
                ri.n_cand[side] = 360 / K->hp_step_deg;
                out.nmax = std::max(out.nmax, ri.n_cand[side]);
            }
            cand += ri.n_cand[side];
            cost += (double)ri.n_cand[side] * (ri.n_mv[side] + 0.5 * ri.n_pairs + 8);
            out.flops += (double)ri.n_cand[side] * (24.0 * ri.n_mv[side] + 8.0 * ri.n_pairs);
            out.bytes += (double)ri.n_cand[side] * 2.0 * ri.n_mv[side];
        }
        out.n_pairs += ri.n_pairs;
        out.rot.push_back(ri);
    }
    M.cand_per_orient = cand * K->repetitions + 1;
    out.cost = cost * K->repetitions + l;
    out.flops = out.flops * K->repetitions + 3.0 * l + 8.0 * (double)out.efar.size();
    out.bytes = out.bytes * K->repetitions + 2.0 * l;
}

static gd_status prep_all(const gd_ligands* L, const gd_knobs* K, bool topo_only, int minb,
                         std::vector<LigPrep>& preps) {
    const int n = L->n_ligands;
    preps.assign(n, LigPrep());
    unsigned hw = std::thread::hardware_concurrency();
    int nt = (int)std::min<unsigned>(hw ? hw : 4, 16);
    if (n < 64) nt = 1;
    std::atomic<int> next(0);
    auto work = [&]() {
        for (;;) {
            int i0 = next.fetch_add(64);
            if (i0 >= n) break;
            for (int i = i0; i < std::min(n, i0 + 64); i++) prep_one(L, K, i, topo_only, minb, preps[i]);
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; t++) th.emplace_back(work);
    work();
    for (auto& t : th) t.join();
    for (int i = 0; i < n; i++)
        if (preps[i].st != GD_OK) return fail(preps[i].st, "%s", preps[i].err.c_str());
    return GD_OK;
}

gd_status prepare_topology(const gd_ligands* L, int min_bonds, TopoHost& T) {
    gd_status st;
    if ((st = validate_ligands_struct(L)) != GD_OK) return st;
    if (min_bonds < 1 || min_bonds > 255) return fail(GD_ERR_ARG, "clash_min_bonds outside [1, 255]");
    std::vector<LigPrep> preps;
    if ((st = prep_all(L, nullptr, true, min_bonds, preps)) != GD_OK) return st;
    const int n = L->n_ligands;
    T.n_atoms.resize(n);
    T.far_off.resize(n);
    T.n_far.resize(n);
    T.efar.clear();
    for (int i = 0; i < n; i++) {
        T.n_atoms[i] = preps[i].meta.l;
        T.far_off[i] = (int32_t)T.efar.size();
        T.n_far[i] = (int32_t)preps[i].efar.size();
        T.efar.insert(T.efar.end(), preps[i].efar.begin(), preps[i].efar.end());
    }
    return GD_OK;
}

gd_status prepare_tree(const gd_ligands* L, TreeHost& out) {
    gd_status st;
    if ((st = validate_ligands_struct(L)) != GD_OK) return st;
    const int n = L->n_ligands;
    out.n_atoms.resize(n);
    out.nr.resize(n);
    out.tree_off.resize(n);
    out.tree.clear();
    out.mask.clear();
    for (int i = 0; i < n; i++) {
        Topo T;
        if ((st = build_topo(L, i, T)) != GD_OK) return st;
        const int l = T.l, nr = T.nr, r0 = L->rot_off[i];
        out.n_atoms[i] = l;
        out.nr[i] = nr;
        out.tree_off[i] = (int32_t)(out.tree.size() / 4);
        std::vector<int> order(nr), near(nr), far(nr);
        for (int r = 0; r < nr; r++) {
            int a = L->rot[2 * (r0 + r)], c = L->rot[2 * (r0 + r) + 1];
            bool root_left = T.left[(size_t)r * l + 0] != 0;
            near[r] = root_left ? a : c;
            far[r] = root_left ? c : a;
            order[r] = r;
        }
        // root first: by the bond distance of the near atom from atom 0
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return T.dist[near[x]] < T.dist[near[y]]; });
        for (int e = 0; e < nr; e++) {
            int r = order[e];
            out.tree.insert(out.tree.end(), {near[r], far[r], r, 0});
            bool root_left = T.left[(size_t)r * l + 0] != 0;
            uint32_t w[4] = {0, 0, 0, 0};
            for (int a = 0; a < l; a++) {
                bool in_left = T.left[(size_t)r * l + a] != 0;
                if (root_left != in_left) w[a >> 5] |= 1u << (a & 31);
            }
            out.mask.insert(out.mask.end(), w, w + 4);
        }
    }
    return GD_OK;
}

static void quat_matrix(const double* q, double* R) {
    double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z);       R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);       R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);       R[7] = 2.0 * (y * z + w * x);       R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// --------------------------------------------------------------------------
// ligand descriptors in device memory

bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // unknown (pageable host) pointers are reported as an error
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

gd_status ligands_on_host(const gd_ligands* L, hipStream_t s, HostLigands& H, const gd_ligands** out,
                          const char* who) {
    *out = L;
    if (!L) return fail(GD_ERR_ARG, "%s: null ligands", who);
    if (L->on_device == 0) return GD_OK;
    if (L->on_device != 1) return fail(GD_ERR_ARG, "%s: on_device must be 0 or 1", who);
    const int n = L->n_ligands;
    if (n < 1) return fail(GD_ERR_ARG, "%s: n_ligands < 1", who);
    const void* arrs[] = {L->atom_off, L->x, L->y, L->z, L->bond_off, L->rot_off};
    for (const void* a : arrs)
        if (!is_device_ptr(a)) return fail(GD_ERR_ARG, "%s: on_device is set but an array is not device memory", who);
    hipError_t e;
    auto get = [&](auto& vec, const auto* src, size_t count) -> hipError_t {
        vec.resize(std::max<size_t>(count, 1));
        if (count == 0) return hipSuccess;
        return hipMemcpyAsync(vec.data(), src, count * sizeof(vec[0]), hipMemcpyDeviceToHost, s);
    };
    if ((e = get(H.atom_off, L->atom_off, n + 1)) != hipSuccess || (e = get(H.bond_off, L->bond_off, n + 1)) != hipSuccess ||
        (e = get(H.rot_off, L->rot_off, n + 1)) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, who);
    // the offsets size the other copies: check them first
    for (int i = 0; i < n; i++)
        if (H.atom_off[i + 1] < H.atom_off[i] || H.bond_off[i + 1] < H.bond_off[i] || H.rot_off[i + 1] < H.rot_off[i])
            return fail(GD_ERR_ARG, "ligands: offsets not ascending at %d", i);
    if (H.atom_off[0] != 0 || H.bond_off[0] != 0 || H.rot_off[0] != 0)
        return fail(GD_ERR_ARG, "ligands: offsets must start at 0");
    const size_t na = (size_t)H.atom_off[n], nb = (size_t)H.bond_off[n], nr = (size_t)H.rot_off[n];
    if ((nb > 0 && !is_device_ptr(L->bonds)) || (nr > 0 && !is_device_ptr(L->rot)))
        return fail(GD_ERR_ARG, "%s: on_device is set but an array is not device memory", who);
    if ((e = get(H.x, L->x, na)) != hipSuccess || (e = get(H.y, L->y, na)) != hipSuccess ||
        (e = get(H.z, L->z, na)) != hipSuccess || (e = get(H.bonds, L->bonds, 2 * nb)) != hipSuccess ||
        (e = get(H.rot, L->rot, 2 * nr)) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
        return hip_fail(e, who);
    H.view = gd_ligands{n, H.atom_off.data(), H.x.data(), H.y.data(), H.z.data(), H.bond_off.data(),
                        nb ? H.bonds.data() : nullptr, H.rot_off.data(), nr ? H.rot.data() : nullptr, 0};
    *out = &H.view;
    return GD_OK;
}

// --------------------------------------------------------------------------
// batch preparation: host tables, then device copies

// Host product of a batch preparation: the tables the kernels read, the
// scalar fields of the device view (pointers unset) and the sizes of the
// per-call device scratch.
struct HostBatch {
    std::vector<LigMeta> meta;
    std::vector<RotInfo> rot;
    std::vector<uint16_t> pairs, efar;
    std::vector<uint8_t> mv;
    std::vector<double> qmat;
    std::vector<int32_t> items;
    int64_t n_keys = 0, n_ang = 0;
    int atoms = 0, nmax = 1;
    BatchDev dev{};
    gd_batch_info info{};
    Tiling tiling;
};

static gd_status prepare_host(const gd_pocket* pocket, const gd_ligands* L, const gd_knobs* K, const char* who,
                              HostBatch& H) {
    gd_status st;
    if ((st = validate_ligands_struct(L)) != GD_OK) return st;
    if ((st = validate_knobs(K)) != GD_OK) return st;
    std::vector<LigPrep> preps;
    if ((st = prep_all(L, K, false, K->clash_min_bonds, preps)) != GD_OK) return st;
    const int n = L->n_ligands, no = K->n_orient;
    H.meta.resize(n);
    int lmax = 1, rmax = 0, nmax = 1;
    int64_t key_off = 0, ang_off = 0, poses = 0, npairs = 0;
    double flops = 0, bytes = 0;
    for (int i = 0; i < n; i++) {
        LigPrep& p = preps[i];
        LigMeta m = p.meta;
        m.rot_off = (int32_t)H.rot.size();
        for (RotInfo ri : p.rot) {
            ri.pair_off += (int32_t)H.pairs.size();
            ri.mv_off[0] += (int32_t)H.mv.size();
            ri.mv_off[1] += (int32_t)H.mv.size();
            H.rot.push_back(ri);
        }
        m.far_off = (int32_t)H.efar.size();
        m.n_far = (int32_t)p.efar.size();
        H.pairs.insert(H.pairs.end(), p.pairs.begin(), p.pairs.end());
        H.mv.insert(H.mv.end(), p.mv.begin(), p.mv.end());
        H.efar.insert(H.efar.end(), p.efar.begin(), p.efar.end());
        m.key_off = key_off;
        if (ang_off > (int64_t)std::numeric_limits<int32_t>::max())
            return fail(GD_ERR_CAPACITY, "%s: angle records exceed 2^31 entries; split the batch", who);
        m.ang_off = (int32_t)ang_off;
        key_off += no;
        ang_off += (int64_t)no * K->repetitions * m.nr * 2;
        poses += m.cand_per_orient * no;
        npairs += p.n_pairs;
        flops += p.flops * no;
        bytes += p.bytes * no;
        lmax = std::max(lmax, m.l);
        rmax = std::max(rmax, m.nr);
        nmax = std::max(nmax, p.nmax);
        H.meta[i] = m;
    }
    if (H.pairs.size() > (size_t)std::numeric_limits<int32_t>::max() ||
        H.efar.size() > (size_t)std::numeric_limits<int32_t>::max())
        return fail(GD_ERR_CAPACITY, "%s: pair lists exceed 2^31 entries; split the batch", who);
    // rotation matrices of the orientations
    H.qmat.resize(9 * (size_t)no);
    for (int o = 0; o < no; o++) quat_matrix(K->quats + 4 * (size_t)o, &H.qmat[9 * (size_t)o]);
    // work queue: (ligand, orientation block), costliest ligands first
    const int opi = std::max(1, std::min(no, 8));
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return preps[a].cost > preps[b].cost; });
    for (int idx = 0; idx < n; idx++)
        for (int o0 = 0; o0 < no; o0 += opi) {
            H.items.push_back(order[idx]);
            H.items.push_back(o0);
        }
    H.atoms = L->atom_off[n];
    H.n_keys = key_off;
    H.n_ang = std::max<int64_t>(ang_off, 1);
    H.nmax = nmax;
    BatchDev& D = H.dev;
    D.n_lig = n;
    D.n_orient = no;
    D.reps = K->repetitions;
    D.top_k = K->top_k;
    D.lmax = lmax;
    D.rmax = std::max(rmax, 1);
    const double cd = (double)K->clash_dist;
    D.cd2 = cd * cd;
    D.cd2f = (float)D.cd2;
    D.n_items = (int32_t)(H.items.size() / 2);
    D.orient_per_item = opi;
    gd_batch_info& I = H.info;
    I.n_ligands = n;
    I.max_atoms = lmax;
    I.max_rot = D.rmax;
    I.repetitions = K->repetitions;
    I.top_k = K->top_k;
    I.n_orient = no;
    I.poses_expected = poses;
    I.n_pairs_total = npairs;
    I.n_atoms_total = H.atoms;
    I.algo_flops = flops;
    I.algo_bytes = bytes;
    while (H.tiling.waves_per_block > 1 && dock_lds_bytes(lmax, nmax, H.tiling.waves_per_block) > lds_limit_per_block())
        H.tiling.waves_per_block /= 2;
    if (const char* env = getenv("GD_TILING")) {
        int w, nb, ppl;
        if (sscanf(env, "%d,%d,%d", &w, &nb, &ppl) == 3 && tiling_supported(w, nb, ppl)) {
            H.tiling.waves_per_block = w;
            H.tiling.angle_block = nb;
            H.tiling.pairs_per_lane = ppl;
        }
    }
    (void)pocket;
    return GD_OK;
}

gd_status prepare_batch(const gd_pocket* pocket, const gd_ligands* L0, const gd_knobs* K, hipStream_t stream,
                        gd_batch** out) {
    const char* who = "gd_prepare_batch";
    if (!pocket || !out) return fail(GD_ERR_ARG, "%s: null argument", who);
    *out = nullptr;
    gd_status st;
    HostLigands HL;
    const gd_ligands* L = nullptr;
    if ((st = ligands_on_host(L0, stream, HL, &L, who)) != GD_OK) return st;
    HostBatch H;
    if ((st = prepare_host(pocket, L, K, who, H)) != GD_OK) return st;
    std::unique_ptr<gd_batch> B(new gd_batch());
    hipError_t e;
#define UP(buf, vec)                                                                                      \
    if ((e = B->buf.upload((vec).data(), (vec).size() * sizeof((vec)[0]), stream)) != hipSuccess)         \
        return hip_fail(e, who);
    UP(lig, H.meta);
    UP(rot, H.rot);
    UP(pairs, H.pairs);
    UP(mv, H.mv);
    UP(efar, H.efar);
    UP(qmat, H.qmat);
    UP(items, H.items);
#undef UP
    const size_t cb = sizeof(float) * (size_t)H.atoms;
    if (L0->on_device) {
        // device to device: the batch outlives the caller's arrays
        DevBuf* dst[3] = {&B->x, &B->y, &B->z};
        const float* src[3] = {L0->x, L0->y, L0->z};
        for (int c = 0; c < 3; c++) {
            if ((e = dst[c]->alloc(cb)) != hipSuccess ||
                (cb && (e = hipMemcpyAsync(dst[c]->ptr, src[c], cb, hipMemcpyDeviceToDevice, stream)) != hipSuccess))
                return hip_fail(e, who);
        }
        if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(e, who);
    } else {
        if ((e = B->x.upload(L->x, cb, stream)) != hipSuccess || (e = B->y.upload(L->y, cb, stream)) != hipSuccess ||
            (e = B->z.upload(L->z, cb, stream)) != hipSuccess)
            return hip_fail(e, who);
    }
    if ((e = B->keys.alloc(sizeof(uint64_t) * (size_t)H.n_keys)) != hipSuccess ||
        (e = B->ang.alloc(sizeof(uint16_t) * (size_t)H.n_ang)) != hipSuccess || (e = B->head.alloc(64)) != hipSuccess ||
        (e = B->counters.alloc(sizeof(int64_t) * GD_N_COUNTERS)) != hipSuccess)
        return hip_fail(e, who);
    BatchDev& D = B->dev;
    D = H.dev;
    D.lig = (const LigMeta*)B->lig.ptr;
    D.rot = (const RotInfo*)B->rot.ptr;
    D.x = (const float*)B->x.ptr;
    D.y = (const float*)B->y.ptr;
    D.z = (const float*)B->z.ptr;
    D.pairs = (const uint16_t*)B->pairs.ptr;
    D.mv = (const uint8_t*)B->mv.ptr;
    D.efar = (const uint16_t*)B->efar.ptr;
    D.qmat = (const double*)B->qmat.ptr;
    D.keys = (uint64_t*)B->keys.ptr;
    D.ang = (uint16_t*)B->ang.ptr;
    D.items = (const int32_t*)B->items.ptr;
    D.head = (int32_t*)B->head.ptr;
    D.counters = (unsigned long long*)B->counters.ptr;
    B->nmax = H.nmax;
    B->info = H.info;
    B->h = pocket->dev.h;
    B->tiling = H.tiling;
    if ((e = B->devcopy.upload(&B->dev, sizeof(BatchDev), stream)) != hipSuccess) return hip_fail(e, who);
    *out = B.release();
    return GD_OK;
}

// The two stages of a docking call: queue reset + docking kernel, then top-k
// and pose replay.
static hipError_t enqueue_dock(const gd_pocket* P, const BatchDev& D, const BatchDev* Ddev, const Tiling& t, int nmax,
                               gd_mode mode, hipStream_t s, unsigned long long* counters) {
    DockLaunch L{(const PocketDev*)P->devcopy.ptr, Ddev, counters, D.lmax, nmax};
    hipError_t e;
    if ((e = launch_reset(D.head, L.counters, s)) != hipSuccess) return e;
    if (mode == GD_BATCHED) {
        int grid = persistent_grid(t, D.lmax, nmax, D.n_items);
        return launch_dock(L, t, true, 0, grid, s);
    }
    const int grid = (D.n_orient + t.waves_per_block - 1) / t.waves_per_block;
    for (int i = 0; i < D.n_lig; i++)
        if ((e = launch_dock(L, t, false, i, grid, s)) != hipSuccess) return e;
    return hipSuccess;
}

static hipError_t enqueue_post(const gd_pocket* P, const BatchDev& D, double h, int nmax, hipStream_t s,
                               gd_pose_rec* out, uint16_t* angles, float* pose_xyz) {
    hipError_t e;
    if ((e = launch_topk(D, out, angles, h, s)) != hipSuccess) return e;
    if (pose_xyz)
        if ((e = launch_replay(P->dev, D, out, pose_xyz, nmax, s)) != hipSuccess) return e;
    return hipSuccess;
}

static hipError_t enqueue_dock_stage(const gd_pocket* P, gd_batch* B, gd_mode mode, hipStream_t s, int64_t* counters) {
    return enqueue_dock(P, B->dev, (const BatchDev*)B->devcopy.ptr, B->tiling, B->nmax, mode, s,
                        counters ? (unsigned long long*)counters : B->dev.counters);
}

static hipError_t enqueue_post_stage(const gd_pocket* P, gd_batch* B, hipStream_t s, gd_pose_rec* out,
                                     uint16_t* angles, float* pose_xyz) {
    return enqueue_post(P, B->dev, B->h, B->nmax, s, out, angles, pose_xyz);
}

static hipError_t capture(hipStream_t s, hipGraphExec_t* exec, const std::function<hipError_t()>& body) {
    hipGraph_t g;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = body();
    e = hipStreamEndCapture(s, &g);
    if (le != hipSuccess) return le;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    return e;
}

static hipError_t timing_mark(gd_batch* B, hipStream_t s, bool start) {
    if (!B->timing) return hipSuccess;
    int slot = (B->ring_head) % gd_batch::kRing;
    hipEvent_t* ev = start ? &B->ev0[slot] : &B->ev1[slot];
    if (!*ev) {
        hipError_t e = hipEventCreate(ev);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(*ev, s);
    if (e == hipSuccess && !start) {
        B->ring_head = (B->ring_head + 1) % gd_batch::kRing;
        B->ring_count = std::min(B->ring_count + 1, gd_batch::kRing);
    }
    return e;
}

gd_status dock_prepared(const gd_pocket* P, gd_batch* B, gd_mode mode, hipStream_t s, gd_pose_rec* out,
                        uint16_t* angles, float* pose_xyz, int64_t* counters) {
    if (!P || !B || !out) return fail(GD_ERR_ARG, "gd_dock_prepared: null argument");
    if (mode != GD_PER_LIGAND && mode != GD_BATCHED) return fail(GD_ERR_ARG, "gd_dock_prepared: bad mode");
    size_t lds = dock_lds_bytes(B->dev.lmax, B->nmax, B->tiling.waves_per_block);
    if (lds > lds_limit_per_block())
        return fail(GD_ERR_CAPACITY, "gd_dock_prepared: tiling needs %zu B of LDS per block, the device allows %zu",
                    lds, lds_limit_per_block());
    hipError_t e;
    const bool use_graph = mode == GD_BATCHED && s != nullptr && !getenv("GD_NO_GRAPH");
    if (!use_graph) {
        if ((e = timing_mark(B, s, true)) != hipSuccess || (e = enqueue_dock_stage(P, B, mode, s, counters)) != hipSuccess ||
            (e = timing_mark(B, s, false)) != hipSuccess || (e = enqueue_post_stage(P, B, s, out, angles, pose_xyz)) != hipSuccess)
            return hip_fail(e, "gd_dock_prepared");
        return GD_OK;
    }
    GraphKey key{P, out, angles, pose_xyz, counters, B->tiling.waves_per_block, B->tiling.angle_block,
                 B->tiling.pairs_per_lane};
    if (!B->graph_dock || !B->graph_post || !(B->graph_key == key)) {
        if (B->graph_dock) (void)hipGraphExecDestroy(B->graph_dock);
        if (B->graph_post) (void)hipGraphExecDestroy(B->graph_post);
        B->graph_dock = B->graph_post = nullptr;
        if ((e = capture(s, &B->graph_dock, [&]() { return enqueue_dock_stage(P, B, mode, s, counters); })) !=
            hipSuccess)
            return hip_fail(e, "gd_dock_prepared: graph capture");
        if ((e = capture(s, &B->graph_post, [&]() { return enqueue_post_stage(P, B, s, out, angles, pose_xyz); })) !=
            hipSuccess)
            return hip_fail(e, "gd_dock_prepared: graph capture");
        B->graph_key = key;
    }
    if ((e = timing_mark(B, s, true)) != hipSuccess || (e = hipGraphLaunch(B->graph_dock, s)) != hipSuccess ||
        (e = timing_mark(B, s, false)) != hipSuccess || (e = hipGraphLaunch(B->graph_post, s)) != hipSuccess)
        return hip_fail(e, "gd_dock_prepared: graph launch");
    return GD_OK;
}

// --------------------------------------------------------------------------
// pinned staging buffers for the asynchronous uploads of gd_dock_batch

namespace {
struct Staging {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;  // recorded on the stream after the copy out of the buffer
    int device = -1;
    int state = 0;              // 0 idle, 1 held by a call, 2 copy in flight
};
std::mutex g_stage_mu;
std::vector<Staging*> g_stage;  // kept for reuse until the process ends
}  // namespace

// A pinned host buffer of at least n bytes, held by the caller until
// stage_release; idle buffers too small for the request are freed.
static hipError_t stage_acquire(size_t n, Staging** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(g_stage_mu);
    Staging* pick = nullptr;
    for (Staging* st : g_stage) {
        if (st->device != dev) continue;
        if (st->state == 2) {
            hipError_t q = hipEventQuery(st->done);
            if (q == hipErrorNotReady) {
                (void)hipGetLastError();
                continue;
            }
            if (q != hipSuccess) return q;
            st->state = 0;
        }
        if (st->state == 0 && st->cap >= n && (!pick || st->cap < pick->cap)) pick = st;
    }
    if (!pick) {
        for (auto it = g_stage.begin(); it != g_stage.end();) {
            Staging* st = *it;
            if (st->device == dev && st->state == 0 && st->cap < n) {
                (void)hipHostFree(st->host);
                (void)hipEventDestroy(st->done);
                delete st;
                it = g_stage.erase(it);
            } else {
                ++it;
            }
        }
        std::unique_ptr<Staging> st(new Staging());
        st->cap = std::max<size_t>(n, (size_t)1 << 20);
        if ((e = hipHostMalloc(&st->host, st->cap, hipHostMallocDefault)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&st->done, hipEventDisableTiming)) != hipSuccess) {
            (void)hipHostFree(st->host);
            return e;
        }
        st->device = dev;
        pick = st.release();
        g_stage.push_back(pick);
    }
    pick->state = 1;
    *out = pick;
    return hipSuccess;
}

// Give the buffer back: after the copy enqueued on s (copied = true) or at once.
static hipError_t stage_release(Staging* st, hipStream_t s, bool copied) {
    std::lock_guard<std::mutex> lock(g_stage_mu);
    if (!copied) {
        st->state = 0;
        return hipSuccess;
    }
    hipError_t e = hipEventRecord(st->done, s);
    st->state = e == hipSuccess ? 2 : 0;
    return e;
}

hipError_t upload_async(void* dev, const void* host, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    Staging* st = nullptr;
    hipError_t e = stage_acquire(n, &st);
    if (e != hipSuccess) return e;
    memcpy(st->host, host, n);
    e = hipMemcpyAsync(dev, st->host, n, hipMemcpyHostToDevice, s);
    const hipError_t r = stage_release(st, s, e == hipSuccess);
    return e != hipSuccess ? e : r;
}

gd_status dock_batch(const gd_pocket* P, const gd_ligands* L0, const gd_knobs* K, gd_mode mode, hipStream_t s,
                     gd_pose_rec* out, uint16_t* angles, float* pose_xyz, int64_t* counters) {
    const char* who = "gd_dock_batch";
    if (!P || !out) return fail(GD_ERR_ARG, "%s: null argument", who);
    if (mode != GD_PER_LIGAND && mode != GD_BATCHED) return fail(GD_ERR_ARG, "%s: bad mode", who);
    gd_status st;
    HostLigands HL;
    const gd_ligands* L = nullptr;
    if ((st = ligands_on_host(L0, s, HL, &L, who)) != GD_OK) return st;
    HostBatch H;
    if ((st = prepare_host(P, L, K, who, H)) != GD_OK) return st;
    const BatchDev& D0 = H.dev;
    const size_t lds = dock_lds_bytes(D0.lmax, H.nmax, H.tiling.waves_per_block);
    if (lds > lds_limit_per_block())
        return fail(GD_ERR_CAPACITY, "%s: the batch needs %zu B of LDS per block, the device allows %zu", who, lds,
                    lds_limit_per_block());
    // outputs in device memory are written in place, host outputs through device scratch
    const size_t n_rec = (size_t)D0.n_lig * D0.top_k;
    const size_t b_out = n_rec * sizeof(gd_pose_rec), b_ang = n_rec * D0.reps * D0.rmax * 2 * sizeof(uint16_t),
                 b_xyz = n_rec * D0.lmax * 3 * sizeof(float), b_cnt = GD_N_COUNTERS * sizeof(int64_t);
    void* user[4] = {out, angles, pose_xyz, counters};
    const size_t ubytes[4] = {b_out, b_ang, b_xyz, b_cnt};
    bool via_host[4];
    bool sync = false;
    for (int k = 0; k < 4; k++) {
        via_host[k] = user[k] && !is_device_ptr(user[k]);
        sync |= via_host[k];
    }
    // one stream-ordered arena: the staged tables first (one copy), then scratch
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t at = off;
        off += (b + 255) & ~(size_t)255;
        return at;
    };
    const size_t o_lig = take(H.meta.size() * sizeof(LigMeta)), o_rot = take(H.rot.size() * sizeof(RotInfo)),
                 o_pairs = take(H.pairs.size() * 2), o_mv = take(H.mv.size()), o_efar = take(H.efar.size() * 2),
                 o_qmat = take(H.qmat.size() * 8), o_items = take(H.items.size() * 4);
    const size_t cb = sizeof(float) * (size_t)H.atoms;
    const bool own_xyz = L0->on_device == 0;
    const size_t o_x = own_xyz ? take(cb) : 0, o_y = own_xyz ? take(cb) : 0, o_z = own_xyz ? take(cb) : 0;
    const size_t o_dev = take(sizeof(BatchDev));
    const size_t staged = off;
    const size_t o_keys = take(sizeof(uint64_t) * (size_t)H.n_keys), o_ang = take(sizeof(uint16_t) * (size_t)H.n_ang),
                 o_head = take(64), o_cnt = take(b_cnt);
    size_t o_user[4];
    for (int k = 0; k < 4; k++) o_user[k] = via_host[k] ? take(ubytes[k]) : 0;
    char* arena = nullptr;
    hipError_t e = hipMallocAsync((void**)&arena, off, s);
    if (e != hipSuccess) return hip_fail(e, who);
    Staging* stg = nullptr;
    bool copied = false;
    auto bail = [&](hipError_t err) {
        if (stg) (void)stage_release(stg, s, copied);
        (void)hipFreeAsync(arena, s);
        return hip_fail(err, who);
    };
    if ((e = stage_acquire(staged, &stg)) != hipSuccess) return bail(e);
    char* hs = (char*)stg->host;
    auto put = [&](size_t at, const void* src, size_t b) {
        if (b) memcpy(hs + at, src, b);
    };
    put(o_lig, H.meta.data(), H.meta.size() * sizeof(LigMeta));
    put(o_rot, H.rot.data(), H.rot.size() * sizeof(RotInfo));
    put(o_pairs, H.pairs.data(), H.pairs.size() * 2);
    put(o_mv, H.mv.data(), H.mv.size());
    put(o_efar, H.efar.data(), H.efar.size() * 2);
    put(o_qmat, H.qmat.data(), H.qmat.size() * 8);
    put(o_items, H.items.data(), H.items.size() * 4);
    if (own_xyz) {
        put(o_x, L->x, cb);
        put(o_y, L->y, cb);
        put(o_z, L->z, cb);
    }
    BatchDev D = D0;
    D.lig = (const LigMeta*)(arena + o_lig);
    D.rot = (const RotInfo*)(arena + o_rot);
    D.pairs = (const uint16_t*)(arena + o_pairs);
    D.mv = (const uint8_t*)(arena + o_mv);
    D.efar = (const uint16_t*)(arena + o_efar);
    D.qmat = (const double*)(arena + o_qmat);
    D.items = (const int32_t*)(arena + o_items);
    D.x = own_xyz ? (const float*)(arena + o_x) : L0->x;  // device inputs are read in place
    D.y = own_xyz ? (const float*)(arena + o_y) : L0->y;
    D.z = own_xyz ? (const float*)(arena + o_z) : L0->z;
    D.keys = (uint64_t*)(arena + o_keys);
    D.ang = (uint16_t*)(arena + o_ang);
    D.head = (int32_t*)(arena + o_head);
    D.counters = (unsigned long long*)(arena + o_cnt);
    put(o_dev, &D, sizeof(BatchDev));
    if ((e = hipMemcpyAsync(arena, hs, staged, hipMemcpyHostToDevice, s)) != hipSuccess) return bail(e);
    copied = true;
    e = stage_release(stg, s, true);
    stg = nullptr;
    if (e != hipSuccess) return bail(e);
    void* dst[4];
    for (int k = 0; k < 4; k++) dst[k] = via_host[k] ? (void*)(arena + o_user[k]) : user[k];
    if ((e = enqueue_dock(P, D, (const BatchDev*)(arena + o_dev), H.tiling, H.nmax, mode, s,
                          dst[3] ? (unsigned long long*)dst[3] : D.counters)) != hipSuccess ||
        (e = enqueue_post(P, D, P->dev.h, H.nmax, s, (gd_pose_rec*)dst[0], (uint16_t*)dst[1], (float*)dst[2])) !=
            hipSuccess)
        return bail(e);
    for (int k = 0; k < 4; k++)
        if (via_host[k] && (e = hipMemcpyAsync(user[k], dst[k], ubytes[k], hipMemcpyDeviceToHost, s)) != hipSuccess)
            return bail(e);
    if ((e = hipFreeAsync(arena, s)) != hipSuccess) return hip_fail(e, who);
    if (sync && (e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, who);
    return GD_OK;
}

}  // namespace gd

gd_batch::~gd_batch() {
    if (graph_dock) (void)hipGraphExecDestroy(graph_dock);
    if (graph_post) (void)hipGraphExecDestroy(graph_post);
    for (int i = 0; i < kRing; i++) {
        if (ev0[i]) (void)hipEventDestroy(ev0[i]);
        if (ev1[i]) (void)hipEventDestroy(ev1[i]);
    }
}

// ----------------------------------------------------------------------------
// C ABI

using namespace gd;

extern "C" {

const char* gd_last_error(void) { return last_error(); }

gd_status gd_create_pocket(const gd_pocket_desc* desc, void* stream, gd_pocket** out) {
    clear_error();
    return create_pocket(desc, (hipStream_t)stream, out);
}

gd_status gd_destroy_pocket(gd_pocket* pocket) {
    clear_error();
    delete pocket;
    return GD_OK;
}

gd_status gd_pocket_get_info(const gd_pocket* P, gd_pocket_info* info) {
    clear_error();
    if (!P || !info) return fail(GD_ERR_ARG, "gd_pocket_get_info: null argument");
    for (int a = 0; a < 3; a++) {
        info->box_lo[a] = P->dev.lo[a];
        info->box_dim[a] = P->dev.dim[a];
        info->centroid[a] = P->centroid[a];
        info->blur_lo[a] = P->dev.blo[a];
        info->blur_dim[a] = P->dev.bdim[a];
    }
    info->n_occupied = P->dev.n_occ;
    info->grid_h = (float)P->dev.h;
    info->blur_h = (float)P->blur_h;
    return GD_OK;
}

gd_status gd_pocket_read_grid(const gd_pocket* P, uint16_t* host_out) {
    clear_error();
    if (!P || !host_out) return fail(GD_ERR_ARG, "gd_pocket_read_grid: null argument");
    hipError_t e = hipMemcpy(host_out, P->edt.ptr, (size_t)P->dev.n_cells * sizeof(uint16_t), hipMemcpyDeviceToHost);
    return e == hipSuccess ? GD_OK : hip_fail(e, "gd_pocket_read_grid");
}

gd_status gd_pocket_read_density(const gd_pocket* P, float* host_out) {
    clear_error();
    if (!P || !host_out) return fail(GD_ERR_ARG, "gd_pocket_read_density: null argument");
    if (!P->rho.ptr) return fail(GD_ERR_ARG, "gd_pocket_read_density: pocket has no density grid");
    hipError_t e = hipMemcpy(host_out, P->rho.ptr, P->rho.bytes, hipMemcpyDeviceToHost);
    return e == hipSuccess ? GD_OK : hip_fail(e, "gd_pocket_read_density");
}

gd_status gd_prepare_batch(const gd_pocket* pocket, const gd_ligands* ligands, const gd_knobs* knobs, void* stream,
                           gd_batch** out) {
    clear_error();
    return prepare_batch(pocket, ligands, knobs, (hipStream_t)stream, out);
}

gd_status gd_destroy_batch(gd_batch* batch) {
    clear_error();
    delete batch;
    return GD_OK;
}

gd_status gd_batch_get_info(const gd_batch* B, gd_batch_info* info) {
    clear_error();
    if (!B || !info) return fail(GD_ERR_ARG, "gd_batch_get_info: null argument");
    *info = B->info;
    return GD_OK;
}

gd_status gd_batch_enable_timing(gd_batch* B, int32_t enable) {
    clear_error();
    if (!B) return fail(GD_ERR_ARG, "gd_batch_enable_timing: null batch");
    B->timing = enable != 0;
    B->ring_head = B->ring_count = 0;
    return GD_OK;
}

gd_status gd_batch_read_timing(gd_batch* B, float* ms_out, int32_t max_n, int32_t* n_out) {
    clear_error();
    if (!B || !n_out || (max_n > 0 && !ms_out)) return fail(GD_ERR_ARG, "gd_batch_read_timing: null argument");
    int n = std::min(B->ring_count, std::max(max_n, 0));
    int first = (B->ring_head - B->ring_count + gd_batch::kRing) % gd_batch::kRing;
    first = (first + (B->ring_count - n)) % gd_batch::kRing;
    for (int k = 0; k < n; k++) {
        int slot = (first + k) % gd_batch::kRing;
        hipError_t e = hipEventSynchronize(B->ev1[slot]);
        if (e != hipSuccess) return hip_fail(e, "gd_batch_read_timing");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, B->ev0[slot], B->ev1[slot]);
        if (e != hipSuccess) return hip_fail(e, "gd_batch_read_timing");
        ms_out[k] = ms;
    }
    *n_out = n;
    B->ring_head = B->ring_count = 0;
    return GD_OK;
}

gd_status gd_batch_set_tiling(gd_batch* B, const gd_tiling* t) {
    clear_error();
    if (!B || !t) return fail(GD_ERR_ARG, "gd_batch_set_tiling: null argument");
    if (!tiling_supported(t->waves_per_block, t->angle_block, t->pairs_per_lane))
        return fail(GD_ERR_ARG, "gd_batch_set_tiling: unsupported tiling");
    B->tiling.waves_per_block = t->waves_per_block;
    B->tiling.angle_block = t->angle_block;
    B->tiling.pairs_per_lane = t->pairs_per_lane;
    return GD_OK;
}

gd_status gd_batch_get_tiling(const gd_batch* B, gd_tiling* t) {
    clear_error();
    if (!B || !t) return fail(GD_ERR_ARG, "gd_batch_get_tiling: null argument");
    t->waves_per_block = B->tiling.waves_per_block;
    t->angle_block = B->tiling.angle_block;
    t->pairs_per_lane = B->tiling.pairs_per_lane;
    return GD_OK;
}

gd_status gd_dock_prepared(const gd_pocket* pocket, gd_batch* batch, gd_mode mode, void* stream, gd_pose_rec* out,
                           uint16_t* angles, float* pose_xyz, int64_t* counters) {
    clear_error();
    return dock_prepared(pocket, batch, mode, (hipStream_t)stream, out, angles, pose_xyz, counters);
}

gd_status gd_dock_batch(const gd_pocket* pocket, const gd_ligands* ligands, const gd_knobs* knobs, gd_mode mode,
                        void* stream, gd_pose_rec* out, uint16_t* angles, float* pose_xyz, int64_t* counters) {
    clear_error();
    return dock_batch(pocket, ligands, knobs, mode, (hipStream_t)stream, out, angles, pose_xyz, counters);
}

}  // extern "C"
