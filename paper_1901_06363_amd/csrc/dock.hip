// Docking kernels for gfx950: the greedy fragment sweep of Alg. 2 (Section
// III-C) over rigid orientations, scored with Eq. 1 on the integer distance
// grid, with the bump test of Section III-B, plus the top-k reduction and the
// replay of the selected poses.
//
// One wavefront docks one (ligand, orientation).  The state that must agree
// with an FP64 evaluation bit for bit (placement, fragment axes, committed
// rotations, endpoint score and bumps) is kept in FP64 in LDS and computed
// with the textbook formulas in a fixed operation order:
//   rotation about unit axis k by angle t: R = cos t I + sin t [k]x + (1 - cos t) k k^T
//   applied as Y = p + R (X - p), p = the moving fragment's own bond atom;
//   cos/sin of integer degrees come from libm tables built on the host.
// The candidate angles of one sweep are evaluated in FP32 with a cheaper,
// algebraically equivalent form:
//   atom position   Y(t) = P0 + cos t U + sin t V        (cell units)
//   pair distance   d^2(t) = A + B cos t + C sin t
// with P0 = p + (k.u)k, U = u - (k.u)k, V = k x u, u = X_moving - p, and
// A = |u|^2 + |v|^2 - 2(k.u)(k.v), B = -2(u.v - (k.u)(k.v)), C = -2 v.(k x u),
// v = X_fixed - p.  Every FP32 decision carries a rounding-error bound; a cell
// index or bump decision within that bound of a boundary is marked uncertain,
// and any uncertain candidate that could still win the sweep is re-evaluated
// with the FP64 formulas above, so the chosen angle equals the FP64 choice.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gd_internal.h"
#include "device_common.h"

namespace gd {

__constant__ double c_cos64[360];
__constant__ double c_sin64[360];
__constant__ float c_cos32[360];
__constant__ float c_sin32[360];

// --------------------------------------------------------------------------
// FP64 kinematics (same formulas and operation order everywhere)

struct Mat3 {
    double m[9];
};

__device__ __forceinline__ Mat3 axis_angle(double kx, double ky, double kz, int deg) {
    double c = c_cos64[deg], s = c_sin64[deg], t = 1.0 - c;
    Mat3 R;
    R.m[0] = t * kx * kx + c;      R.m[1] = t * kx * ky - s * kz; R.m[2] = t * kx * kz + s * ky;
    R.m[3] = t * kx * ky + s * kz; R.m[4] = t * ky * ky + c;      R.m[5] = t * ky * kz - s * kx;
    R.m[6] = t * kx * kz - s * ky; R.m[7] = t * ky * kz + s * kx; R.m[8] = t * kz * kz + c;
    return R;
}

__device__ __forceinline__ void rotate_about(double px, double py, double pz, const Mat3& R, double x, double y,
                                             double z, double& ox, double& oy, double& oz) {
    double d0 = x - px, d1 = y - py, d2 = z - pz;
    ox = px + (R.m[0] * d0 + R.m[1] * d1 + R.m[2] * d2);
    oy = py + (R.m[3] * d0 + R.m[4] * d1 + R.m[5] * d2);
    oz = pz + (R.m[6] * d0 + R.m[7] * d1 + R.m[8] * d2);
}

// --------------------------------------------------------------------------
// per-wave LDS

struct WaveLds {
    double* X;     // [3][lp] FP64 master coordinates (x, y, z planes)
    double* AD;    // [8][lp] per-atom sweep data: u (3), k.u, k x u (3), |u|^2
    float* MV;     // [9][lp] moving atoms: P0 (3), U (3), V (3) in cell units
    int* Slo;      // [nmax]
    int* Shi;      // [nmax]
    uint8_t* st;   // [nmax] bit0: certain bump, bit1: possible bump
};

__host__ __device__ inline int lds_pitch(int lmax) { return (lmax + 1) & ~1; }
__host__ __device__ inline size_t wave_lds_bytes(int lmax, int nmax) {
    int lp = lds_pitch(lmax);
    size_t b = sizeof(double) * 3 * lp + sizeof(double) * 8 * lp + sizeof(float) * 9 * lp +
               sizeof(int) * 2 * nmax + ((nmax + 15) & ~15);
    return (b + 15) & ~(size_t)15;
}

__host__ __device__ inline size_t replay_lds_bytes(int lmax) { return sizeof(double) * 3 * lds_pitch(lmax); }

__device__ inline WaveLds carve(char* base, int lmax, int nmax) {
    int lp = lds_pitch(lmax);
    WaveLds W;
    W.X = (double*)base;
    W.AD = W.X + 3 * lp;
    W.MV = (float*)(W.AD + 8 * lp);
    W.Slo = (int*)(W.MV + 9 * lp);
    W.Shi = W.Slo + nmax;
    W.st = (uint8_t*)(W.Shi + nmax);
    return W;
}

struct Acc {
    long long poses = 0, fallback = 0, sweeps = 0;
    int oob = 0;
};

// State of the sweep in progress (wave-uniform values).
struct Sweep {
    const uint8_t* mvl;       // moving atoms
    const uint16_t* pairs;    // straddling far pairs (left | right << 8)
    int m, npairs, side, l, lp;
    double kx, ky, kz, px, py, pz;
    float gcell;              // guard for cell decisions (cell units)
    float thr_lo, thr_hi;     // bump thresholds on FP32 d^2
};

// --------------------------------------------------------------------------
// FP64 evaluation of one candidate of the current sweep: S over the moving
// atoms and feasibility over the straddling far pairs.

__device__ bool eval_fp64(const PocketDev& P, const BatchDev& B, const Sweep& sw, const WaveLds& W, int deg,
                          int& S_out, Acc& acc) {
    const int lane = lane_id();
    const Mat3 R = axis_angle(sw.kx, sw.ky, sw.kz, deg);
    const double* Xx = W.X;
    const double* Xy = W.X + sw.lp;
    const double* Xz = W.X + 2 * sw.lp;
    int S = 0;
    for (int j = lane; j < sw.m; j += kWave) {
        int i = sw.mvl[j];
        double yx, yy, yz;
        rotate_about(sw.px, sw.py, sw.pz, R, Xx[i], Xy[i], Xz[i], yx, yy, yz);
        S += D_exact(P, yx, yy, yz, acc.oob);
    }
    S = wave_sum(S);
    bool clash = false;
    for (int q = lane; q < sw.npairs; q += kWave) {
        uint16_t pr = sw.pairs[q];
        int li = pr & 0xff, ri = pr >> 8;
        int mv = sw.side == 0 ? li : ri, fx = sw.side == 0 ? ri : li;
        double yx, yy, yz;
        rotate_about(sw.px, sw.py, sw.pz, R, Xx[mv], Xy[mv], Xz[mv], yx, yy, yz);
        clash |= dist2(yx, yy, yz, Xx[fx], Xy[fx], Xz[fx]) < B.cd2;
    }
    clash = __ballot(clash) != 0;
    S_out = S;
    acc.fallback++;
    return !clash;
}

// FP32 contribution of one candidate atom with an interval for cells within
// the guard of a face.
__device__ __forceinline__ void atom_cell_score(const PocketDev& P, float yx, float yy, float yz, float g, int& slo,
                                                int& shi, int& oob) {
    float fx = floorf(yx), fy = floorf(yy), fz = floorf(yz);
    float rx = yx - fx, ry = yy - fy, rz = yz - fz;  // exact in FP32
    int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    float lim = 0.5f - g;
    bool ux = fabsf(rx - 0.5f) > lim, uy = fabsf(ry - 0.5f) > lim, uz = fabsf(rz - 0.5f) > lim;
    if (!(ux | uy | uz)) {
        int d = D_box(P, ix, iy, iz, oob);
        slo += d;
        shi += d;
        return;
    }
    // a coordinate within the guard of a face: the true cell is one of two per
    // uncertain axis; take the range of D over those cells
    int ax = ux ? (rx < 0.5f ? -1 : 1) : 0, ay = uy ? (ry < 0.5f ? -1 : 1) : 0, az = uz ? (rz < 0.5f ? -1 : 1) : 0;
    int lo = 0x7fffffff, hi = 0;
    for (int dz = 0; dz <= (az != 0); dz++)
        for (int dy = 0; dy <= (ay != 0); dy++)
            for (int dx = 0; dx <= (ax != 0); dx++) {
                int d = D_box(P, ix + dx * ax, iy + dy * ay, iz + dz * az, oob);
                lo = d < lo ? d : lo;
                hi = d > hi ? d : hi;
            }
    slo += lo;
    shi += hi;
}

// Evaluate the candidate angles base + k*stride (k < n) of the current sweep;
// returns the winning position (lowest S among feasible candidates, earliest
// on ties) or -1 when none is feasible.
template <int NB, int PPL>
__device__ int eval_candidates(const PocketDev& P, const BatchDev& B, const Sweep& sw, const WaveLds& W, int base,
                               int stride, int n, Acc& acc) {
    const int lane = lane_id();
    constexpr int G = kWave / NB;
    const int lp = sw.lp;
    acc.poses += n;

    // ---- score pass: lanes = (angle within block, atom group)
    for (int kb = 0; kb < n; kb += NB) {
        const int k = kb + (lane & (NB - 1));
        const int g = lane / NB;
        int slo = 0, shi = 0;
        if (k < n) {
            const int deg = base + k * stride;
            const float c = c_cos32[deg], s = c_sin32[deg];
            for (int j = g; j < sw.m; j += G) {
                const float* mv = W.MV + j;
                float yx = fmaf(s, mv[6 * lp], fmaf(c, mv[3 * lp], mv[0]));
                float yy = fmaf(s, mv[7 * lp], fmaf(c, mv[4 * lp], mv[lp]));
                float yz = fmaf(s, mv[8 * lp], fmaf(c, mv[5 * lp], mv[2 * lp]));
                atom_cell_score(P, yx, yy, yz, sw.gcell, slo, shi, acc.oob);
            }
        }
#pragma unroll
        for (int o = NB; o < kWave; o <<= 1) {
            slo += __shfl_xor(slo, o);
            shi += __shfl_xor(shi, o);
        }
        if (lane < NB && k < n) {
            W.Slo[k] = slo;
            W.Shi[k] = shi;
        }
    }

    // ---- bump pass: lanes = straddling pairs, loop over angles of a word
    const double* ux = W.AD;
    const double* uy = W.AD + lp;
    const double* uz = W.AD + 2 * lp;
    const double* ku = W.AD + 3 * lp;
    const double* wx = W.AD + 4 * lp;
    const double* wy = W.AD + 5 * lp;
    const double* wz = W.AD + 6 * lp;
    const double* uu = W.AD + 7 * lp;
    for (int w0 = 0; w0 < n; w0 += kWave) {
        const int nw = min(kWave, n - w0);
        float cl = 0.f, sl = 0.f;
        if (lane < nw) {
            int deg = base + (w0 + lane) * stride;
            cl = c_cos32[deg];
            sl = c_sin32[deg];
        }
        uint64_t cert = 0, maybe = 0;
        for (int q0 = 0; q0 < sw.npairs; q0 += kWave * PPL) {
            float A[PPL], Bc[PPL], Cs[PPL];
#pragma unroll
            for (int t = 0; t < PPL; t++) {
                const int q = q0 + t * kWave + lane;
                if (q < sw.npairs) {
                    uint16_t pr = sw.pairs[q];
                    int li = pr & 0xff, ri = pr >> 8;
                    int m = sw.side == 0 ? li : ri, f = sw.side == 0 ? ri : li;
                    double kk = ku[m] * ku[f];
                    double uv = ux[m] * ux[f] + uy[m] * uy[f] + uz[m] * uz[f];
                    double vw = ux[f] * wx[m] + uy[f] * wy[m] + uz[f] * wz[m];
                    A[t] = (float)(uu[m] + uu[f] - 2.0 * kk);
                    Bc[t] = (float)(-2.0 * (uv - kk));
                    Cs[t] = (float)(-2.0 * vw);
                } else {
                    A[t] = 3.0e38f;
                    Bc[t] = 0.f;
                    Cs[t] = 0.f;
                }
            }
            for (int k = 0; k < nw; k++) {
                const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(cl), k));
                const float s = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(sl), k));
                float d = fmaf(Cs[0], s, fmaf(Bc[0], c, A[0]));
#pragma unroll
                for (int t = 1; t < PPL; t++) d = fminf(d, fmaf(Cs[t], s, fmaf(Bc[t], c, A[t])));
                if (__ballot(d < sw.thr_lo)) cert |= 1ull << k;
                if (__ballot(d < sw.thr_hi)) maybe |= 1ull << k;
            }
        }
        if (lane < nw) W.st[w0 + lane] = (uint8_t)(((cert >> lane) & 1) | (((maybe >> lane) & 1) << 1));
    }
    wave_sync();

    // ---- decision: best certain candidate, then resolve uncertain contenders
    uint64_t best = ~0ull;
    for (int k0 = 0; k0 < n; k0 += kWave) {
        const int k = k0 + lane;
        if (k < n) {
            int lo = W.Slo[k], hi = W.Shi[k];
            if (!(W.st[k] & 2) && lo == hi) {
                uint64_t key = ((uint64_t)(uint32_t)lo << 16) | (uint64_t)k;
                best = key < best ? key : best;
            }
        }
    }
    best = wave_min_u64(best);
    for (int k0 = 0; k0 < n; k0 += kWave) {
        const int k = k0 + lane;
        bool need = false;
        if (k < n) {
            int st = W.st[k], lo = W.Slo[k], hi = W.Shi[k];
            uint64_t key = ((uint64_t)(uint32_t)lo << 16) | (uint64_t)k;
            need = !(st & 1) && ((st & 2) || lo != hi) && key < best;
        }
        uint64_t mask = __ballot(need);
        while (mask) {
            const int bit = __builtin_ctzll(mask);
            mask &= mask - 1;
            const int kk = k0 + bit;
            int S;
            if (eval_fp64(P, B, sw, W, base + kk * stride, S, acc)) {
                uint64_t key = ((uint64_t)(uint32_t)S << 16) | (uint64_t)kk;
                best = key < best ? key : best;
            }
        }
    }
    wave_sync();
    return best == ~0ull ? -1 : (int)(best & 0xffff);
}

// Prepare one fragment sweep: FP64 axis and pivot, per-atom pair data and the
// FP32 moving-atom coefficients, plus the rounding guards of this sweep.
__device__ void sweep_setup(const PocketDev& P, const BatchDev& B, const LigMeta& L, const RotInfo& ri, int side,
                            const WaveLds& W, Sweep& sw) {
    const int lane = lane_id();
    const int lp = lds_pitch(B.lmax);
    const double* Xx = W.X;
    const double* Xy = W.X + lp;
    const double* Xz = W.X + 2 * lp;
    sw.lp = lp;
    sw.l = L.l;
    sw.side = side;
    sw.mvl = B.mv + ri.mv_off[side];
    sw.m = ri.n_mv[side];
    sw.pairs = B.pairs + ri.pair_off;
    sw.npairs = ri.n_pairs;
    const int a = ri.a, c = ri.c;
    double ax = Xx[c] - Xx[a], ay = Xy[c] - Xy[a], az = Xz[c] - Xz[a];
    double nrm = sqrt(ax * ax + ay * ay + az * az);
    sw.kx = ax / nrm;
    sw.ky = ay / nrm;
    sw.kz = az / nrm;
    const int piv = side == 0 ? a : c;
    sw.px = Xx[piv];
    sw.py = Xy[piv];
    sw.pz = Xz[piv];
    wave_sync();

    double r2max = 0.0;
    for (int i = lane; i < L.l; i += kWave) {
        double ux = Xx[i] - sw.px, uy = Xy[i] - sw.py, uz = Xz[i] - sw.pz;
        double ku = sw.kx * ux + sw.ky * uy + sw.kz * uz;
        double uu = ux * ux + uy * uy + uz * uz;
        W.AD[i] = ux;
        W.AD[lp + i] = uy;
        W.AD[2 * lp + i] = uz;
        W.AD[3 * lp + i] = ku;
        W.AD[4 * lp + i] = sw.ky * uz - sw.kz * uy;
        W.AD[5 * lp + i] = sw.kz * ux - sw.kx * uz;
        W.AD[6 * lp + i] = sw.kx * uy - sw.ky * ux;
        W.AD[7 * lp + i] = uu;
        r2max = fmax(r2max, uu);
    }
    double amax = 0.0, umax = 0.0;
    const double ih = P.inv_h;
    for (int j = lane; j < sw.m; j += kWave) {
        int i = sw.mvl[j];
        double ux = Xx[i] - sw.px, uy = Xy[i] - sw.py, uz = Xz[i] - sw.pz;
        double ku = sw.kx * ux + sw.ky * uy + sw.kz * uz;
        double ax0 = (sw.px + ku * sw.kx) * ih - (double)P.lo[0];
        double ay0 = (sw.py + ku * sw.ky) * ih - (double)P.lo[1];
        double az0 = (sw.pz + ku * sw.kz) * ih - (double)P.lo[2];
        double Ux = (ux - ku * sw.kx) * ih, Uy = (uy - ku * sw.ky) * ih, Uz = (uz - ku * sw.kz) * ih;
        double Vx = (sw.ky * uz - sw.kz * uy) * ih, Vy = (sw.kz * ux - sw.kx * uz) * ih,
               Vz = (sw.kx * uy - sw.ky * ux) * ih;
        float* mv = W.MV + j;
        mv[0] = (float)ax0;
        mv[lp] = (float)ay0;
        mv[2 * lp] = (float)az0;
        mv[3 * lp] = (float)Ux;
        mv[4 * lp] = (float)Uy;
        mv[5 * lp] = (float)Uz;
        mv[6 * lp] = (float)Vx;
        mv[7 * lp] = (float)Vy;
        mv[8 * lp] = (float)Vz;
        amax = fmax(amax, fmax(fabs(ax0), fmax(fabs(ay0), fabs(az0))));
        umax = fmax(umax, fmax(fabs(Ux), fmax(fabs(Uy), fmax(fabs(Uz), fmax(fabs(Vx), fmax(fabs(Vy), fabs(Vz)))))));
    }
    r2max = wave_max(r2max);
    amax = wave_max(amax);
    umax = wave_max(umax);
    // FP32 error of Y = fma(s, V, fma(c, U, P0)) from FP64 P0, U, V:
    //   <= u (3|P0| + 4|U| + 3|V|), u = 2^-24; doubled for safety.
    const double u32 = 1.0 / 16777216.0;
    sw.gcell = (float)(2.0 * u32 * (3.0 * amax + 7.0 * umax) + 1e-6);
    // FP32 error of d^2 = fma(C, s, fma(B, c, A)) with |A| <= 4R^2, |B|,|C| <= 2R^2
    //   (A, B, C rounded from FP64): <= u (3|A| + 4|B| + 3|C|) as for Y above,
    //   from the evaluation, i.e. <= 26 u R^2 in all; doubled for safety.
    double gc = 2.0 * u32 * 26.0 * r2max + 1e-6;
    sw.thr_lo = (float)(B.cd2 - gc);
    sw.thr_hi = (float)(B.cd2 + gc);
    wave_sync();
}

// Apply the chosen rotation to the moving fragment in FP64.
__device__ void commit(const Sweep& sw, const WaveLds& W, int deg) {
    if (deg == 0) return;
    const int lane = lane_id();
    const Mat3 R = axis_angle(sw.kx, sw.ky, sw.kz, deg);
    double* Xx = W.X;
    double* Xy = W.X + sw.lp;
    double* Xz = W.X + 2 * sw.lp;
    for (int j = lane; j < sw.m; j += kWave) {
        int i = sw.mvl[j];
        double ox, oy, oz;
        rotate_about(sw.px, sw.py, sw.pz, R, Xx[i], Xy[i], Xz[i], ox, oy, oz);
        Xx[i] = ox;
        Xy[i] = oy;
        Xz[i] = oz;
    }
    wave_sync();
}

// Rigid placement X = R(q)(x - c_L) + c_P.
__device__ void place(const PocketDev& P, const BatchDev& B, const LigMeta& L, int o, const WaveLds& W) {
    const int lane = lane_id();
    const int lp = lds_pitch(B.lmax);
    const double* R = B.qmat + 9 * (size_t)o;
    for (int i = lane; i < L.l; i += kWave) {
        double d0 = (double)B.x[L.atom_off + i] - L.cL[0];
        double d1 = (double)B.y[L.atom_off + i] - L.cL[1];
        double d2 = (double)B.z[L.atom_off + i] - L.cL[2];
        W.X[i] = (R[0] * d0 + R[1] * d1 + R[2] * d2) + P.cP[0];
        W.X[lp + i] = (R[3] * d0 + R[4] * d1 + R[5] * d2) + P.cP[1];
        W.X[2 * lp + i] = (R[6] * d0 + R[7] * d1 + R[8] * d2) + P.cP[2];
    }
    wave_sync();
}

// Whole-ligand endpoint: exact S and bump flag from the FP64 pose.
__device__ void endpoint(const PocketDev& P, const BatchDev& B, const LigMeta& L, const WaveLds& W, int& S,
                         bool& clash, Acc& acc) {
    const int lane = lane_id();
    const int lp = lds_pitch(B.lmax);
    const double* Xx = W.X;
    const double* Xy = W.X + lp;
    const double* Xz = W.X + 2 * lp;
    int s = 0;
    for (int i = lane; i < L.l; i += kWave) s += D_exact(P, Xx[i], Xy[i], Xz[i], acc.oob);
    S = wave_sum(s);
    bool c = false;
    const uint16_t* fp = B.efar + L.far_off;
    for (int q = lane; q < L.n_far; q += kWave) {
        uint16_t pr = fp[q];
        int i = pr & 0xff, j = pr >> 8;
        c |= dist2(Xx[i], Xy[i], Xz[i], Xx[j], Xy[j], Xz[j]) < B.cd2;
    }
    clash = __ballot(c) != 0;
    acc.poses += 1;
}

// The greedy sweep of one orientation (Alg. 2).
template <int NB, int PPL>
__device__ void dock_orientation(const PocketDev& P, const BatchDev& B, int lig, int o, const WaveLds& W, Acc& acc) {
    const LigMeta L = B.lig[lig];
    place(P, B, L, o, W);
    const int nrec = B.reps * L.nr * 2;
    uint16_t* ang = B.ang + L.ang_off + (size_t)o * nrec;
    for (int rep = 0; rep < B.reps; rep++) {
        for (int r = 0; r < L.nr; r++) {
            const RotInfo ri = B.rot[L.rot_off + r];
            for (int side = 0; side < 2; side++) {
                Sweep sw;
                sweep_setup(P, B, L, ri, side, W, sw);
                int deg;
                if (ri.mode[side] == kFlat) {
                    const int st = ri.step[side];
                    int k = eval_candidates<NB, PPL>(P, B, sw, W, 0, st, 360 / st, acc);
                    deg = k < 0 ? 0 : k * st;
                } else {
                    const int hp = ri.step[side], x = ri.tile[side];
                    int t = eval_candidates<NB, PPL>(P, B, sw, W, ri.off[side], x, 360 / x, acc);
                    if (t < 0) t = 0;
                    int k = eval_candidates<NB, PPL>(P, B, sw, W, t * x, hp, x / hp, acc);
                    deg = k < 0 ? 0 : t * x + k * hp;
                }
                commit(sw, W, deg);
                acc.sweeps++;
                if (lane_id() == 0) ang[(rep * L.nr + r) * 2 + side] = (uint16_t)deg;
            }
        }
    }
    int S;
    bool clash;
    endpoint(P, B, L, W, S, clash, acc);
    if (lane_id() == 0)
        B.keys[L.key_off + o] = ((uint64_t)clash << 63) | ((uint64_t)(uint32_t)S << 32) | (uint64_t)(uint32_t)o;
}

__device__ void flush(const BatchDev& B, Acc& acc) {
    int oob = wave_sum(acc.oob);
    if (lane_id() == 0 && B.counters) {
        atomicAdd(B.counters + GD_CNT_POSES, (unsigned long long)acc.poses);
        atomicAdd(B.counters + GD_CNT_FALLBACK, (unsigned long long)acc.fallback);
        atomicAdd(B.counters + GD_CNT_OOB, (unsigned long long)oob);
        atomicAdd(B.counters + GD_CNT_SWEEPS, (unsigned long long)acc.sweeps);
    }
    acc = Acc();
}

// Per-ligand form: one launch per ligand, one wave per orientation.
template <int NB, int PPL>
__global__ void __launch_bounds__(512) dock_ligand_kernel(PocketDev P, BatchDev B, int lig, int nmax) {
    extern __shared__ __align__(16) char smem[];
    const int wave = threadIdx.x / kWave;
    const WaveLds W = carve(smem + wave * wave_lds_bytes(B.lmax, nmax), B.lmax, nmax);
    const int o = blockIdx.x * (blockDim.x / kWave) + wave;
    Acc acc;
    if (o < B.n_orient) dock_orientation<NB, PPL>(P, B, lig, o, W, acc);
    flush(B, acc);
}

// Batched form: a persistent grid; every wave pops (ligand, orientation
// block) items from the device queue until it is empty.
template <int NB, int PPL>
__global__ void __launch_bounds__(512) dock_persistent_kernel(PocketDev P, BatchDev B, int nmax) {
    extern __shared__ __align__(16) char smem[];
    const int wave = threadIdx.x / kWave;
    const WaveLds W = carve(smem + wave * wave_lds_bytes(B.lmax, nmax), B.lmax, nmax);
    Acc acc;
    for (;;) {
        int item = 0;
        if (lane_id() == 0) item = atomicAdd(B.head, 1);
        item = __shfl(item, 0);
        if (item >= B.n_items) break;
        const int lig = B.items[2 * item], o0 = B.items[2 * item + 1];
        const int o1 = min(o0 + B.orient_per_item, B.n_orient);
        for (int o = o0; o < o1; o++) dock_orientation<NB, PPL>(P, B, lig, o, W, acc);
    }
    flush(B, acc);
}

__global__ void reset_kernel(int* head, unsigned long long* counters) {
    if (threadIdx.x == 0) *head = 0;
    if (counters && threadIdx.x < GD_N_COUNTERS) counters[threadIdx.x] = 0;
}

// Top-k per ligand by repeated minimum extraction over the endpoint keys
// (keys are unique: the orientation index is part of the key).
__global__ void __launch_bounds__(256) topk_kernel(BatchDev B, gd_pose_rec* out, uint16_t* ang_out, int rmax,
                                                   double h) {
    const int lig = blockIdx.x;
    const LigMeta L = B.lig[lig];
    const uint64_t* keys = B.keys + L.key_off;
    __shared__ uint64_t red[256 / kWave];
    __shared__ uint64_t sel;
    uint64_t prev = 0;
    bool first = true;
    const int nrec = B.reps * L.nr * 2;
    for (int r = 0; r < B.top_k; r++) {
        uint64_t m = ~0ull;
        for (int o = threadIdx.x; o < B.n_orient; o += blockDim.x) {
            uint64_t k = keys[o];
            if ((first || k > prev) && k < m) m = k;
        }
        m = wave_min_u64(m);
        if (lane_id() == 0) red[threadIdx.x / kWave] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint64_t v = red[0];
            for (int w = 1; w < (int)(blockDim.x / kWave); w++) v = red[w] < v ? red[w] : v;
            sel = v;
        }
        __syncthreads();
        const uint64_t k = sel;
        const int o = (int)(k & 0xffffffffu);
        const int S = (int)((k >> 32) & 0x7fffffff);
        if (threadIdx.x == 0) {
            gd_pose_rec rec;
            rec.orient = o;
            rec.S = S;
            rec.clash = (int)(k >> 63);
            rec.n_atoms = L.l;
            rec.overlap = (double)L.l / (h * h * (double)S);
            out[(size_t)lig * B.top_k + r] = rec;
        }
        if (ang_out) {
            const int per = B.reps * rmax * 2;
            uint16_t* dst = ang_out + ((size_t)lig * B.top_k + r) * per;
            const uint16_t* src = B.ang + L.ang_off + (size_t)o * nrec;
            for (int e = threadIdx.x; e < per; e += blockDim.x) {
                int rep = e / (rmax * 2), rr = (e / 2) % rmax, side = e & 1;
                dst[e] = rr < L.nr ? src[(rep * L.nr + rr) * 2 + side] : 0;
            }
        }
        prev = k;
        first = false;
        __syncthreads();
    }
}

// Rebuild the selected poses from their recorded angles (same FP64 placement
// and commits as the sweep) and write them as FP32.
__global__ void __launch_bounds__(256) replay_kernel(PocketDev P, BatchDev B, const gd_pose_rec* recs, float* xyz,
                                                     int nmax) {
    extern __shared__ __align__(16) char smem[];
    const int wave = threadIdx.x / kWave;
    const int idx = blockIdx.x * (blockDim.x / kWave) + wave;
    if (idx >= B.n_lig * B.top_k) return;
    const int lig = idx / B.top_k;
    WaveLds W{};
    W.X = (double*)(smem + wave * replay_lds_bytes(B.lmax));
    const LigMeta L = B.lig[lig];
    const int o = recs[idx].orient;
    place(P, B, L, o, W);
    const int nrec = B.reps * L.nr * 2;
    const uint16_t* ang = B.ang + L.ang_off + (size_t)o * nrec;
    for (int rep = 0; rep < B.reps; rep++)
        for (int r = 0; r < L.nr; r++) {
            const RotInfo ri = B.rot[L.rot_off + r];
            for (int side = 0; side < 2; side++) {
                Sweep sw;
                const int lp = lds_pitch(B.lmax);
                sw.lp = lp;
                sw.side = side;
                sw.mvl = B.mv + ri.mv_off[side];
                sw.m = ri.n_mv[side];
                const double* Xx = W.X;
                const double* Xy = W.X + lp;
                const double* Xz = W.X + 2 * lp;
                double ax = Xx[ri.c] - Xx[ri.a], ay = Xy[ri.c] - Xy[ri.a], az = Xz[ri.c] - Xz[ri.a];
                double nrm = sqrt(ax * ax + ay * ay + az * az);
                sw.kx = ax / nrm;
                sw.ky = ay / nrm;
                sw.kz = az / nrm;
                const int piv = side == 0 ? ri.a : ri.c;
                sw.px = Xx[piv];
                sw.py = Xy[piv];
                sw.pz = Xz[piv];
                wave_sync();
                commit(sw, W, ang[(rep * L.nr + r) * 2 + side]);
            }
        }
    const int lp = lds_pitch(B.lmax);
    float* dst = xyz + (size_t)idx * B.lmax * 3;
    for (int i = lane_id(); i < B.lmax; i += kWave) {
        bool in = i < L.l;
        dst[3 * i + 0] = in ? (float)W.X[i] : 0.f;
        dst[3 * i + 1] = in ? (float)W.X[lp + i] : 0.f;
        dst[3 * i + 2] = in ? (float)W.X[2 * lp + i] : 0.f;
    }
}

// --------------------------------------------------------------------------
// host-side launchers

hipError_t upload_trig_tables() {
    static bool done = false;
    if (done) return hipSuccess;
    double c64[360], s64[360];
    float c32[360], s32[360];
    trig_tables(c64, s64, c32, s32);
    hipError_t e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_cos64), c64, sizeof(c64))) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_sin64), s64, sizeof(s64))) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_cos32), c32, sizeof(c32))) != hipSuccess) return e;
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_sin32), s32, sizeof(s32))) != hipSuccess) return e;
    done = true;
    return hipSuccess;
}

size_t dock_lds_bytes(int lmax, int nmax, int waves) { return wave_lds_bytes(lmax, nmax) * waves; }

template <int NB, int PPL>
static hipError_t launch_dock_t(const PocketDev& P, const BatchDev& B, int nmax, int waves, bool persistent,
                                int lig, int grid, hipStream_t s) {
    size_t lds = dock_lds_bytes(B.lmax, nmax, waves);
    if (persistent)
        hipLaunchKernelGGL((dock_persistent_kernel<NB, PPL>), dim3(grid), dim3(waves * kWave), lds, s, P, B, nmax);
    else
        hipLaunchKernelGGL((dock_ligand_kernel<NB, PPL>), dim3(grid), dim3(waves * kWave), lds, s, P, B, lig, nmax);
    return hipGetLastError();
}

template <int NB>
static hipError_t launch_dock_nb(const PocketDev& P, const BatchDev& B, int nmax, const Tiling& t, bool persistent,
                                 int lig, int grid, hipStream_t s) {
    switch (t.pairs_per_lane) {
        case 1: return launch_dock_t<NB, 1>(P, B, nmax, t.waves_per_block, persistent, lig, grid, s);
        case 2: return launch_dock_t<NB, 2>(P, B, nmax, t.waves_per_block, persistent, lig, grid, s);
        case 4: return launch_dock_t<NB, 4>(P, B, nmax, t.waves_per_block, persistent, lig, grid, s);
        case 8: return launch_dock_t<NB, 8>(P, B, nmax, t.waves_per_block, persistent, lig, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dock(const PocketDev& P, const BatchDev& B, int nmax, const Tiling& t, bool persistent, int lig,
                       int grid, hipStream_t s) {
    switch (t.angle_block) {
        case 4: return launch_dock_nb<4>(P, B, nmax, t, persistent, lig, grid, s);
        case 8: return launch_dock_nb<8>(P, B, nmax, t, persistent, lig, grid, s);
        case 16: return launch_dock_nb<16>(P, B, nmax, t, persistent, lig, grid, s);
        case 32: return launch_dock_nb<32>(P, B, nmax, t, persistent, lig, grid, s);
        default: return hipErrorInvalidValue;
    }
}

size_t lds_limit_per_block() {
    static size_t lim = 0;
    if (!lim) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) lim = prop.sharedMemPerBlock;
        if (!lim) lim = 64 * 1024;
    }
    return lim;
}

int persistent_grid(const Tiling& t, int lmax, int nmax, int n_items) {
    // one resident block per slot the LDS budget allows on each CU
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    (void)hipGetDeviceProperties(&prop, dev);
    size_t lds = dock_lds_bytes(lmax, nmax, t.waves_per_block);
    int per_cu_lds = (int)(prop.maxSharedMemoryPerMultiProcessor / (lds > 0 ? lds : 1));
    int per_cu_waves = 32 / t.waves_per_block;  // 8 waves per SIMD
    int per_cu = per_cu_lds < per_cu_waves ? per_cu_lds : per_cu_waves;
    if (per_cu < 1) per_cu = 1;
    long long g = (long long)per_cu * prop.multiProcessorCount;
    long long need = ((long long)n_items + t.waves_per_block - 1) / t.waves_per_block;
    if (g > need) g = need;
    return (int)(g < 1 ? 1 : g);
}

hipError_t launch_reset(int* head, unsigned long long* counters, hipStream_t s) {
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, head, counters);
    return hipGetLastError();
}

hipError_t launch_topk(const BatchDev& B, gd_pose_rec* out, uint16_t* ang_out, double h, hipStream_t s) {
    hipLaunchKernelGGL(topk_kernel, dim3(B.n_lig), dim3(256), 0, s, B, out, ang_out, B.rmax, h);
    return hipGetLastError();
}

hipError_t launch_replay(const PocketDev& P, const BatchDev& B, const gd_pose_rec* recs, float* xyz, int nmax,
                         hipStream_t s) {
    const int waves = 4;
    int n = B.n_lig * B.top_k;
    size_t lds = replay_lds_bytes(B.lmax) * waves;
    hipLaunchKernelGGL(replay_kernel, dim3((n + waves - 1) / waves), dim3(waves * kWave), lds, s, P, B, recs, xyz,
                       nmax);
    return hipGetLastError();
}

}  // namespace gd
