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
// v = X_fixed - p.  Over a full turn d^2 never drops below A - sqrt(B^2 + C^2),
// so pairs that cannot bump at any angle are dropped once per sweep.  Every
// FP32 decision carries a rounding-error bound; a cell index or bump decision
// within that bound of a boundary is marked uncertain, and any uncertain
// candidate that could still win the sweep is re-evaluated with the FP64
// formulas above, so the chosen angle equals the FP64 choice.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "gd_internal.h"

namespace gd {

__constant__ double c_cos64[360];
__constant__ double c_sin64[360];
// FP32 roundings of the same tables, cos then sin, read with per-lane
// indices (once per angle block, outside the atom loops) from global memory
__device__ float c_trig32[720];

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

// LDS (address space 3) views of the per-wave working set: 32-bit addresses
// and LDS-only memory instructions.
typedef __attribute__((address_space(3))) double lds_double;
typedef __attribute__((address_space(3))) float lds_float;
typedef float f4 __attribute__((ext_vector_type(4)));  // plain 16-byte vector (copyable from LDS)
typedef __attribute__((address_space(3))) f4 lds_float4;
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) f2 lds_float2;

__device__ __forceinline__ f4 mk4(float a, float b, float c, float d) {
    f4 v;
    v.x = a;
    v.y = b;
    v.z = c;
    v.w = d;
    return v;
}
typedef __attribute__((address_space(3))) int lds_int;
typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(3))) uint16_t lds_u16;

constexpr int kSurvCap = 128;  // straddling pairs that can still bump in one sweep (LDS list)
constexpr int kMvPad = 16;     // sentinel rows after the moving list (cover one step of the score pass)

// The per-wave slice is sized for the batch's largest ligand and decides how
// many waves fit a CU, so the moving-atom rows are packed to 36 bytes (no
// padding lane) and the survivors' coefficients to 12 bytes.
struct WaveLds {
    lds_double* X;     // [3][lp] FP64 master coordinates (x, y, z planes)
    lds_double* SW;    // [8] FP64 axis k (3), pivot p (3) and |X_c - X_a| of the sweep in progress
    lds_float4* AD;    // [lmax][2] per-atom sweep data: (u, k.u), (k x u, |u|^2), u = X - p (A); set-up only
    // moving atoms in cell units, rows [0, m) then sentinel rows, written after
    // the prune over the memory of AD: P0 = (a.x, a.y, a.z), U = (a.w, b.x,
    // b.y), V = (b.z, b.w, c)
    lds_float4* MVa;   // [lmax + kMvPad]
    lds_float4* MVb;   // [lmax + kMvPad]
    lds_float* MVc;    // [lmax + kMvPad]
    lds_int* Slo;      // [nmax] lower bound of each candidate's S over the moving atoms
    lds_int* Shi;      // [nmax] upper bound
    lds_u16* surv_pr;  // [kSurvCap] the surviving pairs (left | right << 8)
    lds_u8* st;        // [nmax] bit0: certain bump, bit1: possible bump
    lds_float* survA;  // [kSurvCap] A of d^2 = A + 2B cos + 2C sin for the pairs that survive the prune
    lds_float2* survBC;  // [kSurvCap] (B, C)
};

// FP64 plane pitch: even, so that the FP32 arrays after the planes stay 16-byte aligned
__host__ __device__ inline int lds_pitch(int lmax) { return (lmax + 1) & ~1; }
__host__ __device__ inline int mv_rows(int lmax) { return lmax + kMvPad; }
// the moving-atom rows over the per-atom data, rounded to 16 bytes
__host__ __device__ inline size_t mv_region_bytes(int lmax) {
    const size_t rows = (size_t)mv_rows(lmax) * (2 * sizeof(f4) + sizeof(float));
    const size_t ad = (size_t)lmax * 2 * sizeof(f4);
    return ((rows > ad ? rows : ad) + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t wave_lds_bytes(int lmax, int nmax) {
    const int lp = lds_pitch(lmax);
    const int np = (nmax + 15) & ~15;
    size_t b = sizeof(double) * 3 * lp + sizeof(double) * 8 + mv_region_bytes(lmax) +
               (sizeof(f2) + sizeof(float)) * kSurvCap + sizeof(int) * 2 * np + np + sizeof(uint16_t) * kSurvCap;
    return (b + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t replay_lds_bytes(int lmax) {
    return sizeof(double) * 3 * lds_pitch(lmax) + sizeof(double) * 8;
}

__device__ inline WaveLds carve(char* base, int lmax, int nmax) {
    const int lp = lds_pitch(lmax), R = mv_rows(lmax);
    const int np = (nmax + 15) & ~15;
    WaveLds W;
    W.X = (lds_double*)base;
    W.SW = W.X + 3 * lp;
    char* region = (char*)(W.SW + 8);
    W.AD = (lds_float4*)region;
    W.MVa = (lds_float4*)region;
    W.MVb = W.MVa + R;
    W.MVc = (lds_float*)(W.MVb + R);
    W.survBC = (lds_float2*)(region + mv_region_bytes(lmax));
    W.survA = (lds_float*)(W.survBC + kSurvCap);
    W.Slo = (lds_int*)(W.survA + kSurvCap);
    W.Shi = W.Slo + np;
    W.st = (lds_u8*)(W.Shi + np);
    W.surv_pr = (lds_u16*)(W.st + np);
    return W;
}

struct Acc {
    long long poses = 0, fallback = 0, sweeps = 0;
    int oob = 0;
};

// Wave-uniform state of the sweep in progress used by the FP32 passes.
struct Sweep {
    const uint8_t* mvl;       // moving atoms
    const uint16_t* pairs;    // straddling far pairs (left | right << 8)
    int m, npairs, side, lp;
    float gface;              // a lookup is certain when every coordinate is within gface of its cell centre
    float thr_lo, thr_hi;     // bump thresholds on FP32 d^2
    int nsurv;                // pairs that can bump at some angle of this sweep
    bool pruned;              // survivors listed in LDS (else test every pair)
    bool inside;              // every moving atom stays inside the grid box at every angle
};

// --------------------------------------------------------------------------
// FP64 evaluation of one candidate of the current sweep: S over the moving
// atoms and feasibility over the straddling far pairs.

// Kept out of line (it runs for a small fraction of candidates); every
// argument is a value or a pointer so that nothing of the caller's state has
// to live in scratch memory.  Returns S (< 2^38: at most 128 atoms of
// D < 2^31) in the low 40 bits, feasibility in bit 40 and this lane's count
// of out-of-box lookups from bit 41.
__device__ __noinline__ uint64_t eval_fp64(const PocketDev* Pp, const lds_double* X, const lds_double* SWp, int lp,
                                           const uint8_t* mvl, int m, const uint16_t* pairs, int npairs, int side,
                                           double cd2, int deg) {
    const PocketDev& P = *Pp;
    const int lane = lane_id();
    const double kx = uniform_d(SWp[0]), ky = uniform_d(SWp[1]), kz = uniform_d(SWp[2]);
    const double px = uniform_d(SWp[3]), py = uniform_d(SWp[4]), pz = uniform_d(SWp[5]);
    const Mat3 R = axis_angle(kx, ky, kz, deg);
    const lds_double* Xx = X;
    const lds_double* Xy = X + lp;
    const lds_double* Xz = X + 2 * lp;
    long long S = 0;
    int oob = 0;
    for (int j = lane; j < m; j += kWave) {
        int i = ldg(mvl + j);
        double yx, yy, yz;
        rotate_about(px, py, pz, R, Xx[i], Xy[i], Xz[i], yx, yy, yz);
        S += D_exact(P, yx, yy, yz, oob);
    }
    S = wave_sum64(S);
    bool clash = false;
    for (int q = lane; q < npairs; q += kWave) {
        uint16_t pr = ldg(pairs + q);
        int li = pr & 0xff, ri = pr >> 8;
        int mv = side == 0 ? li : ri, fx = side == 0 ? ri : li;
        double yx, yy, yz;
        rotate_about(px, py, pz, R, Xx[mv], Xy[mv], Xz[mv], yx, yy, yz);
        clash |= dist2(yx, yy, yz, Xx[fx], Xy[fx], Xz[fx]) < cd2;
    }
    clash = __ballot(clash) != 0;
    return (uint64_t)S | ((uint64_t)(!clash) << 40) | ((uint64_t)(uint32_t)oob << 41);
}

// An atom within the guard of a cell face, or outside the tabulated grid,
// widens its candidate's S range to [S of the other atoms, unbounded]; such a
// candidate is re-evaluated in FP64 if it can still win its sweep.
constexpr int kOpenHi = 0x20000000;

// FP32 coefficients of d^2(theta) = A + 2 B cos(theta) + 2 C sin(theta) for a
// straddling pair (li on the left, ri on the right) in the frame of the
// current sweep, from the per-atom data u = X - p, z = k.u, k x u and
// rho = |k x u| (axial and radial coordinates about the rotamer's axis):
//   A = (z_l - z_r)^2 + rho_l^2 + rho_r^2  (= |u_l|^2 + |u_r|^2 - 2 z_l z_r),
//   B = z_l z_r - u_l.u_r,
//   C = -(k x u_l).u_r when the left side turns; turning the right side
//   instead flips the sign of C (csign = -1 left, +1 right).
__device__ __forceinline__ f4 pair_coeffs_from(f4 ul, f4 wl, f4 ur, f4 wr, float csign) {
    const float dz = ul.w - ur.w;
    const float A = fmaf(dz, dz, fmaf(wl.w, wl.w, wr.w * wr.w));
    const float uv = fmaf(ul.z, ur.z, fmaf(ul.y, ur.y, ul.x * ur.x));
    const float vw = fmaf(ur.z, wl.z, fmaf(ur.y, wl.y, ur.x * wl.x));
    return mk4(A, fmaf(ul.w, ur.w, -uv), csign * vw, 0.f);
}

__device__ __forceinline__ f4 pair_coeffs(const WaveLds& W, uint32_t pr, float csign) {
    const int li = pr & 0xff, ri = pr >> 8;
    return pair_coeffs_from(W.AD[2 * li], W.AD[2 * li + 1], W.AD[2 * ri], W.AD[2 * ri + 1], csign);
}

// Per-atom sweep data of atom i (the values the set-up stores in W.AD):
// (u, z) and (k x u, rho) with u = X_i - p, z = k.u and rho = |k x u|.  u, z
// and k x u are formed in FP64 and rounded once to FP32; rho is the FP32 norm
// of the rounded k x u (v_sqrt_f32, 1 ulp), within 5 u rho of the exact one
// (u = 2^-24).
struct Frame {
    double kx, ky, kz, px, py, pz;
};

__device__ __forceinline__ void atom_data(const WaveLds& W, int lp, const Frame& f, int i, f4& a0, f4& a1) {
    const double ux = W.X[i] - f.px, uy = W.X[lp + i] - f.py, uz = W.X[2 * lp + i] - f.pz;
    const double ku = fma(f.kz, uz, fma(f.ky, uy, f.kx * ux));
    const float wx = (float)fma(f.ky, uz, -f.kz * uy), wy = (float)fma(f.kz, ux, -f.kx * uz),
                wz = (float)fma(f.kx, uy, -f.ky * ux);
    const float rho = __builtin_amdgcn_sqrtf(fmaf(wz, wz, fmaf(wy, wy, wx * wx)));
    a0 = mk4((float)ux, (float)uy, (float)uz, (float)ku);
    a1 = mk4(wx, wy, wz, rho);
}

// K pairs per lane starting at q0 (lanes = straddling pairs), then for each
// of the nw angles of the word (c2 = 2 cos, s2 = 2 sin per lane) a certain /
// possible bump bit.  Used when more pairs survive the prune than the LDS list
// holds (rare).
template <int K>
__device__ __forceinline__ void bump_block(const Sweep& sw, const WaveLds& W, int q0, int nq, int nw, float c2,
                                           float s2, uint64_t& cert, uint64_t& maybe) {
    const int lane = lane_id();
    const float csign = sw.side == 0 ? -1.f : 1.f;
    // W.AD has been overwritten by the moving-atom rows: rebuild the per-atom
    // data of both atoms from the FP64 masters (the same values)
    const Frame fr{uniform_d(W.SW[0]), uniform_d(W.SW[1]), uniform_d(W.SW[2]),
                   uniform_d(W.SW[3]), uniform_d(W.SW[4]), uniform_d(W.SW[5])};
    f4 e[K];
#pragma unroll
    for (int t = 0; t < K; t++) {
        const int q = q0 + t * kWave + lane;
        e[t] = mk4(3.0e38f, 0.f, 0.f, 0.f);
        if (q < nq) {
            const uint32_t pr = ldg(sw.pairs + q);
            f4 ul, wl, ur, wr;
            atom_data(W, sw.lp, fr, pr & 0xff, ul, wl);
            atom_data(W, sw.lp, fr, pr >> 8, ur, wr);
            e[t] = pair_coeffs_from(ul, wl, ur, wr, csign);
        }
    }
    for (int k = 0; k < nw; k++) {
        const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c2), k));
        const float s = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(s2), k));
        float d = fmaf(e[0].z, s, fmaf(e[0].y, c, e[0].x));
#pragma unroll
        for (int t = 1; t < K; t++) d = fminf(d, fmaf(e[t].z, s, fmaf(e[t].y, c, e[t].x)));
        if (__ballot(d < sw.thr_lo)) cert |= 1ull << k;
        if (__ballot(d < sw.thr_hi)) maybe |= 1ull << k;
    }
}

// Eight pairs per lane do not fit the inlined register budget: that block
// runs out of line, with values and pointers as arguments (no record of the
// caller's in memory), and returns its bits.
struct BumpBits {
    uint64_t cert, maybe;
};
template <int K>
__device__ __noinline__ BumpBits bump_block_far(const uint16_t* pairs, int side, int lp, float thr_lo, float thr_hi,
                                                const lds_double* X, const lds_double* SW, const lds_float4* AD,
                                                int q0, int nq, int nw, float c2, float s2) {
    Sweep sw;
    sw.pairs = pairs;
    sw.side = side;
    sw.lp = lp;
    sw.thr_lo = thr_lo;
    sw.thr_hi = thr_hi;
    WaveLds W;
    W.X = (lds_double*)X;
    W.SW = (lds_double*)SW;
    W.AD = (lds_float4*)AD;
    BumpBits b{0, 0};
    bump_block<K>(sw, W, q0, nq, nw, c2, s2, b.cert, b.maybe);
    return b;
}

// Score pass over the candidate angles base + k*stride (k < n).  Lanes are
// (k0 < NB, atom group g < G = 64/NB); a block covers up to KANG*NB angles
// and a lane scores the angles kb + k0 + NB*a (a < KANG) over the atoms g,
// g + G, ... of the moving list, KATU atoms per step, so each atom's
// coefficients are read from LDS once for up to KANG angles and KATU*KANG
// distance-grid gathers are in flight.  (NB, KANG, KATU) = (8, 4, 1),
// (16, 2, 2) or (32, 1, 4): up to 32 angles per block and 8 atoms per step
// over the groups.  The moving list is followed by kMvPad rows
// whose position is the zero sentinel cell (certain, D = 0), so every lane
// runs the same steps (a wave-uniform loop) with no end-of-list masking; an
// atom whose cell is not certain reads the sentinel too and marks its
// candidate uncertain (a ballot mask in scalar registers).  Positions are
// relative to the centre of the box's first cell, so an atom's cell is its
// position rounded to the nearest integers and the lookup is certain when
// every coordinate lies within gface of that integer (one max3 of absolute
// differences and one compare).  With BOX the grid bounds are tested per
// atom, otherwise the sweep set-up has proven that every moving atom stays
// inside the box.  Writes W.Slo / W.Shi per candidate.
template <int NB>
__device__ __forceinline__ uint32_t fold_groups(uint64_t m) {
    // OR together the bits of lanes k0 + NB*g over g: result bit k0
#pragma unroll
    for (int sh = 32; sh >= NB; sh >>= 1) m |= m >> sh;
    return (uint32_t)m & (uint32_t)((1ull << NB) - 1);
}

// Sum over the lanes k0 + NB*g (g < 64/NB) in every lane: swaps of rows of
// eight lanes (DPP rotate by 8 within a row of 16), then of rows of 16 and 32
// lanes (the gfx950 permlane swaps: the two outputs together hold a lane's
// value and its partner's, whichever output holds which).
template <int NB>
__device__ __forceinline__ int group_sum(int v) {
    static_assert(NB >= 4 && NB <= 32, "angle blocks of 4, 8, 16 or 32");
    if (NB == 4) v += __builtin_amdgcn_update_dpp(0, v, 0x124, 0xf, 0xf, false);  // row_ror:4
    if (NB <= 8) v += __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, false);  // row_ror:8
    if (NB <= 16) {
        const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        v = (int)p[0] + (int)p[1];
    }
    const auto q = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (int)q[0] + (int)q[1];
}

template <int NB, int KANG, int KATU, bool BOX>
__device__ __forceinline__ void score_blocks(const PocketDev& P, const Sweep& sw, const WaveLds& W, const float* trig,
                                             int base, int stride, int kfirst, int n, int T) {
    constexpr int G = kWave / NB;
    static_assert(G * KATU <= kMvPad + 1, "sentinel rows must cover a step");
    const int lane = lane_id();
    const int k0 = lane & (NB - 1), g = lane / NB;
    const float fnx = (float)P.dim[0], fny = (float)P.dim[1], fnz = (float)P.dim[2];
    // byte offsets 2 * (z nx ny + y nx + x) in FP32: every partial result is an
    // even integer below 2^25, hence exact
    const float fsy2 = 2.f * fnx, fsz2 = 2.f * fnx * fny;
    const float fsent2 = 2.f * (float)P.n_cells;
    const float thr = sw.gface;
    const int m = sw.m;
    const __attribute__((address_space(1))) char* edt = (const __attribute__((address_space(1))) char*)P.edt;
    for (int kb = kfirst; kb < n; kb += NB * KANG) {
        const int A = min(KANG, (n - kb + NB - 1) / NB);
        float c[KANG], s[KANG];
#pragma unroll
        for (int a = 0; a < KANG; a++) {
            const int k = kb + k0 + NB * a;
            const int deg = base + (((a < A) & (k < n)) ? k : 0) * stride;
            c[a] = ldg(trig + deg);
            s[a] = ldg(trig + 360 + deg);
        }
        int sum[KANG];
        uint64_t badm[KANG];
        bool alive[KANG];
#pragma unroll
        for (int a = 0; a < KANG; a++) {
            sum[a] = 0;
            badm[a] = 0;
            alive[a] = true;
        }
        // byte offsets of the KATU x KANG lookups of the step at row j0 (the
        // sentinel's for an uncertain cell, whose candidate is flagged)
        uint32_t off[KATU][KANG];
        auto offsets = [&](int j0) {
#pragma unroll
            for (int t = 0; t < KATU; t++) {
                const int r = j0 + g + t * G;  // at most m + KATU * G - 2: within the sentinel rows
                const f4 ra = W.MVa[r], rb = W.MVb[r];
                const float rc = W.MVc[r];
                const bool live = BOX ? (r < m) : true;
#pragma unroll
                for (int a = 0; a < KANG; a++) {
                    off[t][a] = 0;
                    if (a < A) {
                        const float yx = fmaf(s[a], rb.z, fmaf(c[a], ra.w, ra.x));
                        const float yy = fmaf(s[a], rb.w, fmaf(c[a], rb.x, ra.y));
                        const float yz = fmaf(s[a], rc, fmaf(c[a], rb.y, ra.z));
                        // nearest integers (ties to even: a tie is never certain); the
                        // differences are exact
                        const float fx = __builtin_rintf(yx), fy = __builtin_rintf(yy), fz = __builtin_rintf(yz);
                        const float e = fmaxf(fmaxf(fabsf(yx - fx), fabsf(yy - fy)), fabsf(yz - fz));
                        bool sure = e <= thr;
                        if (BOX)
                            sure = sure & (fx >= 0.f) & (fx < fnx) & (fy >= 0.f) & (fy < fny) & (fz >= 0.f) &
                                   (fz < fnz);
                        badm[a] |= __ballot(live & !sure);
                        const float fi2 = fmaf(fz, fsz2, fmaf(fy, fsy2, fx + fx));
                        off[t][a] = (uint32_t)((live & sure & alive[a]) ? fi2 : fsent2);
                    }
                }
            }
        };
        // software pipeline: the gathers of a step are in flight while the
        // next step's offsets are computed (an empty list reads only sentinel rows)
        offsets(0);
        for (int j0 = 0; j0 < m; j0 += KATU * G) {
            int v[KATU][KANG];
#pragma unroll
            for (int t = 0; t < KATU; t++)
#pragma unroll
                for (int a = 0; a < KANG; a++)
                    v[t][a] = a < A ? (int)*(const __attribute__((address_space(1))) uint16_t*)(edt + off[t][a]) : 0;
            if (j0 + KATU * G < m) offsets(j0 + KATU * G);
#pragma unroll
            for (int a = 0; a < KANG; a++) {
#pragma unroll
                for (int t = 0; t < KATU; t++) sum[a] += v[t][a];
                // a candidate stops once its partial sum over all atom groups
                // reaches the bound (every lane of the candidate agrees)
                if (T != 0x7fffffff)
                    alive[a] = alive[a] & ((group_sum<NB>(sum[a]) < T) | (kb + k0 + NB * a == 0));
            }
        }
        // sum the groups of each angle across lanes; uncertain flags folded from the ballots
#pragma unroll
        for (int a = 0; a < KANG; a++)
            if (a < A) {
                const int tot = group_sum<NB>(sum[a]);
                const uint32_t badbits = fold_groups<NB>(badm[a] | __ballot(!alive[a]));
                const int k = kb + NB * a + lane;
                if (lane < NB && k < n) {
                    W.Slo[k] = tot;
                    W.Shi[k] = ((badbits >> lane) & 1u) ? kOpenHi : tot;
                }
            }
    }
}

// A remainder of at most four angles in one block of 4 angles x 16 atom
// groups (out of line, so that the wide pass keeps its registers).
// Its arguments are values and pointers only, so that no record of the
// caller's has to be placed in scratch memory for the call.
__device__ __noinline__ void score_tail4(const PocketDev* Pp, const lds_float4* MVa, const lds_float4* MVb,
                                        const lds_float* MVc, lds_int* Slo, lds_int* Shi, float gface, int m,
                                        const float* trig, int base, int stride, int kfirst, int n, int T) {
    Sweep sw;
    sw.gface = gface;
    sw.m = m;
    WaveLds W;
    W.MVa = (lds_float4*)MVa;
    W.MVb = (lds_float4*)MVb;
    W.MVc = (lds_float*)MVc;
    W.Slo = Slo;
    W.Shi = Shi;
    score_blocks<4, 1, 1, false>(*Pp, sw, W, trig, base, stride, kfirst, n, T);
}

template <int NB, bool BOX>
__device__ __forceinline__ void score_pass(const PocketDev& P, const Sweep& sw, const WaveLds& W, const float* trig,
                                           int base, int stride, int n, int T) {
    constexpr int KANG = NB == 8 ? 4 : NB == 16 ? 2 : 1;
    constexpr int KATU = NB == 8 ? 1 : NB == 16 ? 2 : 4;
    const int r = n % (NB * KANG);
    const int wide = (BOX || r > 4 || r == 0) ? n : n - r;
    score_blocks<NB, KANG, KATU, BOX>(P, sw, W, trig, base, stride, 0, wide, T);
    if (!BOX && wide < n)
        score_tail4(&P, W.MVa, W.MVb, W.MVc, W.Slo, W.Shi, sw.gface, sw.m, trig, base, stride, wide, n, T);
    wave_sync();
}

// Evaluate the candidate angles base + k*stride (k < n) of the current sweep;
// returns the winning position (lowest S among feasible candidates, earliest
// on ties) or -1 when none is feasible.
template <int NB, int PPL>
__device__ int eval_candidates(const PocketDev& P, const BatchDev& B, const Sweep& sw, const WaveLds& W,
                               const float* trig, int base, int stride, int n, Acc& acc) {
    const int lane = lane_id();
    constexpr int G = kWave / NB;
    acc.poses += n;


    // ---- bump pass.  After a successful prune: lanes = candidate angles (64
    // per word), each takes the minimum of d^2 = A + 2B cos + 2C sin over the
    // survivors' coefficients (broadcast from LDS); a certain bump is
    // min < cd^2 - guard, a possible one min < cd^2 + guard.  Otherwise (more
    // survivors than the LDS list holds): lanes = straddling pairs, looping
    // over the angles of the word.
    if (sw.pruned) {
        const int ns = sw.nsurv;
        for (int w0 = 0; w0 < n; w0 += kWave) {
            const int k = w0 + lane;
            const int deg = base + (k < n ? k : 0) * stride;
            const float c = 2.f * ldg(trig + deg), s = 2.f * ldg(trig + 360 + deg);
            float d = 3.0e38f;
            // four survivors from one 16-byte broadcast read of A and two of
            // (B, C) (the lists are 16-byte aligned); eight per step, so that
            // six reads are in flight before the arithmetic
            auto four = [&](int q0) {
                const f4 a = *(const lds_float4*)(W.survA + q0);
                const f4 b0 = *(const lds_float4*)(W.survBC + q0), b1 = *(const lds_float4*)(W.survBC + q0 + 2);
                const float e0 = fmaf(b0.y, s, fmaf(b0.x, c, a.x));
                const float e1 = fmaf(b0.w, s, fmaf(b0.z, c, a.y));
                const float e2 = fmaf(b1.y, s, fmaf(b1.x, c, a.z));
                const float e3 = fmaf(b1.w, s, fmaf(b1.z, c, a.w));
                return fminf(fminf(e0, e1), fminf(e2, e3));
            };
            int q = 0;
            for (; q + 7 < ns; q += 8) d = fminf(d, fminf(four(q), four(q + 4)));
            if (q + 3 < ns) {
                d = fminf(d, four(q));
                q += 4;
            }
            for (; q < ns; q++) {
                const f2 e = W.survBC[q];
                d = fminf(d, fmaf(e.y, s, fmaf(e.x, c, W.survA[q])));
            }
            if (k < n) W.st[k] = (uint8_t)((d < sw.thr_lo ? 1 : 0) | (d < sw.thr_hi ? 2 : 0));
        }
    } else {
        for (int w0 = 0; w0 < n; w0 += kWave) {
            const int nw = min(kWave, n - w0);
            float cl = 0.f, sl = 0.f;
            if (lane < nw) {
                int deg = base + (w0 + lane) * stride;
                cl = 2.f * ldg(trig + deg);
                sl = 2.f * ldg(trig + 360 + deg);
            }
            uint64_t cert = 0, maybe = 0;
            const int nq = sw.npairs;
            int q0 = 0;
            if (PPL > 4) {
                for (; nq - q0 > kWave * (PPL - 1); q0 += kWave * PPL) {
                    const BumpBits b = bump_block_far<PPL>(sw.pairs, sw.side, sw.lp, sw.thr_lo, sw.thr_hi, W.X, W.SW,
                                                           W.AD, q0, nq, nw, cl, sl);
                    cert |= b.cert;
                    maybe |= b.maybe;
                }
            } else if (PPL > 1) {
                for (; nq - q0 > kWave * (PPL - 1); q0 += kWave * PPL)
                    bump_block<PPL>(sw, W, q0, nq, nw, cl, sl, cert, maybe);
            }
            for (; q0 < nq; q0 += kWave) bump_block<1>(sw, W, q0, nq, nw, cl, sl, cert, maybe);
            if (lane < nw) W.st[w0 + lane] = (uint8_t)(((cert >> lane) & 1) | (((maybe >> lane) & 1) << 1));
        }
    }
    wave_sync();

    // ---- score pass.  A schedule starting at angle 0 has the unturned
    // fragment as its first candidate: when its S is certain and it cannot
    // bump, no other candidate whose partial sum reaches that S can win (ties
    // go to the earlier position), so such candidates stop gathering and keep
    // their partial sum as a lower bound (their upper bound left open).  The
    // extra pass that scores the unturned fragment is skipped on sweeps of at
    // most 8 candidates.
    int T = 0x7fffffff;
    if (base == 0 && sw.inside && n > 8) {
        int s0 = 0;
        bool ok = true;
        for (int j = lane; j < sw.m; j += kWave) {
            const f4 ra = W.MVa[j], rb = W.MVb[j];
            const float yx = ra.x + ra.w, yy = ra.y + rb.x, yz = ra.z + rb.y;
            const float fx = __builtin_rintf(yx), fy = __builtin_rintf(yy), fz = __builtin_rintf(yz);
            const float e = fmaxf(fmaxf(fabsf(yx - fx), fabsf(yy - fy)), fabsf(yz - fz));
            ok = ok & (e <= sw.gface);
            const float fi = fmaf(fz, (float)P.dim[0] * (float)P.dim[1], fmaf(fy, (float)P.dim[0], fx));
            s0 += ok ? (int)P.edt[(uint32_t)fi] : 0;
        }
        s0 = wave_sum(s0);
        if (__ballot(!ok) == 0 && W.st[0] == 0) T = s0;
    }
    if (sw.inside)
        score_pass<NB, false>(P, sw, W, trig, base, stride, n, T);
    else
        score_pass<NB, true>(P, sw, W, trig, base, stride, n, T);

    // ---- decision: key = S << 9 | position (a schedule has at most 360
    // positions).  The certain candidates' S comes from in-box cells only (at
    // most 128 moving atoms of D <= 65535, below 2^23), so their keys fit 32
    // bits; an FP64 re-evaluation may score atoms far outside the box (S below
    // 2^38), so the running best is a 64-bit key.  The lowest certain key
    // first, then the uncertain contenders whose lower bound could still win,
    // re-evaluated in FP64 in position order.
    static_assert(kMaxAtoms * 65535 < (1 << 23), "in-box moving-atom S must fit 23 bits");
    uint32_t best32 = 0xffffffffu;
    for (int k0 = 0; k0 < n; k0 += kWave) {
        const int k = k0 + lane;
        if (k < n) {
            const int lo = W.Slo[k], hi = W.Shi[k];
            if (!(W.st[k] & 2) && lo == hi) best32 = min(best32, ((uint32_t)lo << 9) | (uint32_t)k);
        }
    }
    best32 = wave_min_u32(best32);
    const uint64_t kNone = ~0ull;
    uint64_t best = best32 == 0xffffffffu ? kNone : (uint64_t)best32;
    for (int k0 = 0; k0 < n; k0 += kWave) {
        const int k = k0 + lane;
        bool need = false;
        if (k < n) {
            const int st = W.st[k], lo = W.Slo[k], hi = W.Shi[k];
            need = !(st & 1) && ((st & 2) || lo != hi) && ((((uint64_t)(uint32_t)lo) << 9) | (uint64_t)k) < best;
        }
        uint64_t mask = __ballot(need);
        while (mask) {
            const int bit = __builtin_ctzll(mask);
            mask &= mask - 1;
            const int kk = k0 + bit;
            const uint64_t r = eval_fp64(&P, W.X, W.SW, sw.lp, sw.mvl, sw.m, sw.pairs, sw.npairs, sw.side, B.cd2,
                                         base + kk * stride);
            acc.fallback++;
            acc.oob += (int)(r >> 41);
            const uint64_t S = r & ((1ull << 40) - 1);
            if ((r >> 40) & 1) best = min(best, (S << 9) | (uint64_t)kk);
        }
    }
    wave_sync();
    return best == kNone ? -1 : (int)(best & 511u);
}

// Axis k = (X_c - X_a)/|X_c - X_a| and pivot of one fragment sweep (FP64,
// stored in W.SW), from the current master coordinates.  The right side of a
// rotamer follows its left side: the left commit leaves X_a exactly in place
// (p + R 0 = p) and does not move X_c, so the axis in W.SW is already the
// bit-exact result and only the pivot changes (keep_axis).
// Lanes 0-2 hold one component each, so the three divisions are one.
__device__ __forceinline__ void sweep_axis(const WaveLds& W, int lp, int a, int c, int piv, bool keep_axis) {
    const int lane = lane_id_here();
    const int comp = lane < 3 ? lane : 0;
    if (!keep_axis) {
        const double d = W.X[comp * lp + c] - W.X[comp * lp + a];
        const double ax = readlane_d(d, 0), ay = readlane_d(d, 1), az = readlane_d(d, 2);
        const double nrm = sqrt(ax * ax + ay * ay + az * az);
        const double k = d / nrm;
        if (lane < 3) W.SW[lane] = k;
        if (lane == 0) W.SW[6] = nrm;
    }
    if (lane < 3) W.SW[3 + lane] = W.X[comp * lp + piv];
    wave_sync();
}

// Prepare one fragment sweep: axis and pivot, per-atom pair data, FP32
// moving-atom coefficients, the rounding guards, and the pair prune.
// One side of a rotamer, read field by field so that no copy of the record
// is indexed by the side number (which would place it in scratch memory).
struct SideInfo {
    int a, c, piv, pair_off, n_pairs, mv_off, n_mv, mode, step, tile, off;
};

__device__ __forceinline__ SideInfo side_info(const RotInfo* rp, int side) {
    SideInfo si;
    si.a = ldc(&rp->a);
    si.c = ldc(&rp->c);
    si.piv = side == 0 ? si.a : si.c;
    si.pair_off = ldc(&rp->pair_off);
    si.n_pairs = ldc(&rp->n_pairs);
    si.mv_off = ldc(rp->mv_off + side);
    si.n_mv = ldc(rp->n_mv + side);
    si.mode = ldc(rp->mode + side);
    si.step = ldc(rp->step + side);
    si.tile = ldc(rp->tile + side);
    si.off = ldc(rp->off + side);
    return si;
}

__device__ __forceinline__ void sweep_setup(const PocketDev& P, const BatchDev& B, const LigMeta& L,
                                         const SideInfo& ri, int side, int left_nsurv, const WaveLds& W,
                                         Sweep& sw) {
    const int lane = lane_id();
    const int lp = lds_pitch(B.lmax);
    const lds_double* Xx = W.X;
    const lds_double* Xy = W.X + lp;
    const lds_double* Xz = W.X + 2 * lp;
    sw.lp = lp;
    sw.side = side;
    sw.mvl = B.mv + ri.mv_off;
    sw.m = ri.n_mv;
    sw.pairs = B.pairs + ri.pair_off;
    sw.npairs = ri.n_pairs;
    sweep_axis(W, lp, ri.a, ri.c, ri.piv, side == 1);
    const double kx = uniform_d(W.SW[0]), ky = uniform_d(W.SW[1]), kz = uniform_d(W.SW[2]);
    const double px = uniform_d(W.SW[3]), py = uniform_d(W.SW[4]), pz = uniform_d(W.SW[5]);

    // per-atom data of every atom, for the prune and the pair coefficients
    const Frame fr{kx, ky, kz, px, py, pz};
    float r2max = 0.f;
    for (int i = lane; i < L.l; i += kWave) {
        f4 a0, a1;
        atom_data(W, lp, fr, i, a0, a1);
        W.AD[2 * i] = a0;
        W.AD[2 * i + 1] = a1;
        r2max = fmaxf(r2max, fmaf(a0.w, a0.w, a1.w * a1.w));  // |u|^2 = z^2 + rho^2
    }
    r2max = wave_maxf(r2max);
    // Rounding guards (u = 2^-24), each doubled for safety and with the maxima
    // rounded up by 1 %:
    //  cell: Y = fma(s, V, fma(c, U, P0)) from P0, U, V rounded once from FP64
    //        deviates by <= u (3|P0| + 4|U| + 3|V|) cell units;
    //  bump: with every per-atom value within 5 u R of its exact one (|u| <=
    //        R), A = dz^2 + rho_l^2 + rho_r^2, 2B and 2C formed in FP32 carry
    //        <= 45, 18 and 10 u R^2; their evaluation with the rounded cos/sin
    //        adds <= u (3|A| + 4|2B| + 3|2C|) <= 26 u R^2: 99 u R^2 in all.
    const double u32 = 1.0 / 16777216.0;
    const double gc = 2.0 * u32 * 100.0 * 1.01 * (double)r2max + 1e-6;
    sw.thr_lo = (float)(B.cd2 - gc);
    sw.thr_hi = (float)(B.cd2 + gc);
    wave_sync();
    // Prune: over a full turn the pair's smallest d^2, A - 2 sqrt(B^2 + C^2),
    // is the squared distance of the two atoms in the (axial, radial) plane,
    // (z_l - z_r)^2 + (rho_l - rho_r)^2 (the radial parts' dot and cross
    // products are B and C); a pair for which it clears the bump distance by
    // more than twice the guard never bumps.
    //
    // It depends only on the two atoms' radial and axial coordinates about the
    // rotamer's axis, which neither the left commit nor the change of pivot
    // along the axis alters, so the right sweep reuses the left sweep's
    // survivors (left_nsurv >= 0) and only recomputes their coefficients.  For
    // that the left prune clears twice the larger of its own guard and a bound
    // on the right one (R_right <= R_left + |X_c - X_a|): the computed squared
    // distance errs by <= 44 u R^2, less than half a guard, and an evaluation
    // by half a guard, so an excluded pair stays above cd^2 + guard at every
    // angle of either sweep.
    const float csign = side == 0 ? -1.f : 1.f;
    int nsurv = 0;
    if (left_nsurv >= 0) {
        nsurv = left_nsurv;
    } else {
        double gp = gc;
        if (side == 0) {
            const double Rr = sqrt(1.01 * (double)r2max) + uniform_d(W.SW[6]);
            gp = fmax(gp, 2.0 * u32 * 100.0 * 1.01 * Rr * Rr + 1e-6);
        }
        const float T = (float)(B.cd2 + 2.0 * gp);
        const lds_float* zr = (const lds_float*)W.AD;  // z of atom i at 8 i + 3, rho at 8 i + 7
        for (int q0 = 0; q0 < sw.npairs; q0 += 4 * kWave) {
            uint16_t prs[4];
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const int q = q0 + t * kWave + lane;
                prs[t] = q < sw.npairs ? ldg(sw.pairs + q) : (uint16_t)0;
            }
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const int q = q0 + t * kWave + lane;
                const int li = prs[t] & 0xff, ri = prs[t] >> 8;
                const float dz = zr[8 * li + 3] - zr[8 * ri + 3], dr = zr[8 * li + 7] - zr[8 * ri + 7];
                const bool keep = (q < sw.npairs) & (fmaf(dz, dz, dr * dr) < T);
                const uint64_t mk = __ballot(keep);
                const int pos = nsurv + __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0));
                if (keep && pos < kSurvCap) W.surv_pr[pos] = prs[t];
                nsurv += __popcll(mk);
            }
        }
        wave_sync();
    }
    // coefficients of the survivors in this sweep's frame
    for (int q = lane; q < min(nsurv, kSurvCap); q += kWave) {
        const f4 e = pair_coeffs(W, W.surv_pr[q], csign);
        W.survA[q] = e.x;
        W.survBC[q] = f2{e.y, e.z};
    }
    sw.nsurv = nsurv;
    sw.pruned = nsurv <= kSurvCap;
    // moving-atom rows for the score pass, over the memory of the per-atom data
    // (no longer read: the prune and the coefficients are done).  Cell units
    // relative to the centre of the box's first cell: P0 = (p + z k) / h - lo
    // - 1/2, U = (u - z k) / h, V = (k x u) / h; the cell of a position is its
    // nearest integer point.
    wave_sync();
    const double ih = P.inv_h;
    const double kxh = kx * ih, kyh = ky * ih, kzh = kz * ih;  // exact: h is a power of two
    const double qx = px * ih - ((double)P.lo[0] + 0.5), qy = py * ih - ((double)P.lo[1] + 0.5),
                 qz = pz * ih - ((double)P.lo[2] + 0.5);
    const float ex = (float)P.dim[0] - 0.51f, ey = (float)P.dim[1] - 0.51f, ez = (float)P.dim[2] - 0.51f;
    float gterm = 0.f;
    bool outside = false;
    for (int j = lane; j < sw.m; j += kWave) {
        const int i = ldg(sw.mvl + j);
        const double ux = Xx[i] - px, uy = Xy[i] - py, uz = Xz[i] - pz;
        const double ku = fma(kz, uz, fma(ky, uy, kx * ux));
        const float ax0 = (float)fma(ku, kxh, qx), ay0 = (float)fma(ku, kyh, qy), az0 = (float)fma(ku, kzh, qz);
        const float Ux = (float)fma(-ku, kxh, ux * ih), Uy = (float)fma(-ku, kyh, uy * ih),
                    Uz = (float)fma(-ku, kzh, uz * ih);
        const float Vx = (float)fma(kyh, uz, -kzh * uy), Vy = (float)fma(kzh, ux, -kxh * uz),
                    Vz = (float)fma(kxh, uy, -kyh * ux);
        W.MVa[j] = mk4(ax0, ay0, az0, Ux);
        W.MVb[j] = mk4(Uy, Uz, Vx, Vy);
        W.MVc[j] = Vz;
        // the atom's circle lies in the ball of radius |U| (= |V|) about P0:
        // keep that ball 0.01 cell inside the box on every side, [-0.49,
        // dim - 0.51] about the first cell's centre (the FP32 test errs by far
        // less than the margin)
        const float r = __builtin_amdgcn_sqrtf(fmaf(Uz, Uz, fmaf(Uy, Uy, Ux * Ux)));
        const float lo = fminf(fminf(ax0, ay0), az0) - r;
        const float hi = fmaxf(fmaxf(ax0 - ex, ay0 - ey), az0 - ez) + r;
        outside |= !((lo >= -0.49f) & (hi <= 0.f));
        // components of U and V are at most r
        gterm = fmaxf(gterm, fmaf(3.f, fmaxf(fmaxf(fabsf(ax0), fabsf(ay0)), fabsf(az0)), 7.f * r));
    }
    sw.inside = __ballot(outside) == 0;
    gterm = wave_maxf(gterm);
    // sentinel rows after the list: U = V = 0 at the centre of cell (0, 0, nz),
    // whose linear index is the zero sentinel cell
    // (the values are formed here: kept from the kernel's start they would
    // hold four registers across the inner loops)
    const int lane_s = lane_id_here();
    if (lane_s < kMvPad) {
        const float z = zero_here();
        W.MVa[sw.m + lane_s] = mk4(z, z, z + (float)P.dim[2], z);
        W.MVb[sw.m + lane_s] = mk4(z, z, z, z);
        W.MVc[sw.m + lane_s] = z;
    }
    // a lookup is certain when each coordinate is more than the guard away from
    // a cell face, i.e. within 1/2 - guard of the cell centre; the FP32
    // threshold is rounded down
    const double face = 0.5 - (2.0 * u32 * 1.01 * (double)gterm + 1e-6);
    float tf = (float)face;
    if ((double)tf > face) tf = __int_as_float(__float_as_int(tf) - 1);
    sw.gface = tf;

    wave_sync();
}

// Apply the chosen rotation to the moving fragment in FP64.
__device__ __forceinline__ void commit(const uint8_t* mvl, int m, const WaveLds& W, int lp, int deg) {
    if (deg == 0) return;
    const int lane = lane_id();
    const double kx = uniform_d(W.SW[0]), ky = uniform_d(W.SW[1]), kz = uniform_d(W.SW[2]);
    const double px = uniform_d(W.SW[3]), py = uniform_d(W.SW[4]), pz = uniform_d(W.SW[5]);
    const Mat3 R = axis_angle(kx, ky, kz, deg);
    lds_double* Xx = W.X;
    lds_double* Xy = W.X + lp;
    lds_double* Xz = W.X + 2 * lp;
    for (int j = lane; j < m; j += kWave) {
        int i = mvl[j];
        double ox, oy, oz;
        rotate_about(px, py, pz, R, Xx[i], Xy[i], Xz[i], ox, oy, oz);
        Xx[i] = ox;
        Xy[i] = oy;
        Xz[i] = oz;
    }
    wave_sync();
}

// Rigid placement X = R(q)(x - c_L) + c_P.
__device__ void place(const PocketDev& P, const BatchDev& B, const LigMeta& L, int o, const WaveLds& W) {
    const int lane = lane_id_here();
    const int lp = lds_pitch(B.lmax);
    const __attribute__((address_space(4))) double* R = (const __attribute__((address_space(4))) double*)(B.qmat + 9 * (size_t)o);
    for (int i = lane; i < L.l; i += kWave) {
        double d0 = (double)ldg(B.x + L.atom_off + i) - L.cL[0];
        double d1 = (double)ldg(B.y + L.atom_off + i) - L.cL[1];
        double d2 = (double)ldg(B.z + L.atom_off + i) - L.cL[2];
        W.X[i] = (R[0] * d0 + R[1] * d1 + R[2] * d2) + P.cP[0];
        W.X[lp + i] = (R[3] * d0 + R[4] * d1 + R[5] * d2) + P.cP[1];
        W.X[2 * lp + i] = (R[6] * d0 + R[7] * d1 + R[8] * d2) + P.cP[2];
    }
    wave_sync();
}

// Whole-ligand endpoint: exact S and bump flag from the FP64 pose.
__device__ __forceinline__ void endpoint(const PocketDev& P, const BatchDev& B, const LigMeta& L, const WaveLds& W,
                                      int& S, bool& clash, Acc& acc) {
    const int lane = lane_id();
    const int lp = lds_pitch(B.lmax);
    const lds_double* Xx = W.X;
    const lds_double* Xy = W.X + lp;
    const lds_double* Xz = W.X + 2 * lp;
    long long s = 0;
    for (int i = lane; i < L.l; i += kWave) s += D_exact(P, Xx[i], Xy[i], Xz[i], acc.oob);
    S = sat_S(wave_sum64(s));
    // whole-ligand bump flag: any far pair closer than the bump distance (the
    // scan stops at the first word of pairs that holds one)
    const uint16_t* fp = B.efar + L.far_off;
    clash = false;
    // four pairs per lane per step (their reads in flight together)
    for (int q0 = 0; q0 < L.n_far && !clash; q0 += 4 * kWave) {
        uint16_t pr[4];
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int q = q0 + t * kWave + lane;
            pr[t] = q < L.n_far ? ldg(fp + q) : (uint16_t)0xffff;
        }
        bool c = false;
#pragma unroll
        for (int t = 0; t < 4; t++)
            if (pr[t] != 0xffff) {
                const int i = pr[t] & 0xff, j = pr[t] >> 8;
                c |= dist2(Xx[i], Xy[i], Xz[i], Xx[j], Xy[j], Xz[j]) < B.cd2;
            }
        clash = __ballot(c) != 0;
    }
    acc.poses += 1;
}

// The greedy sweep of one orientation (Alg. 2).
// Outputs of a work item (orientations o0 .. o0 + n - 1 of one ligand), held
// in registers until they fill whole runs of memory: the chosen angles one
// per lane (record q of the item in lane q mod 64, stored 64 at a time; an
// item's records are contiguous), the keys one per lane (stored at the end).
struct ItemOut {
    int angv = 0, q = 0;
    uint64_t keyv = 0;
};

template <int NB, int PPL>
__device__ void dock_orientation(const PocketDev& P, const BatchDev& B, int lig, int o, int o0, int n_item,
                                 const WaveLds& W, const float* trig, Acc& acc, ItemOut& out) {
    const LigMeta L = ldc_record(B.lig + lig);
    place(P, B, L, o, W);
    const int nrec = B.reps * L.nr * 2;
    const int total = n_item * nrec;
    for (int rep = 0; rep < B.reps; rep++) {
        for (int r = 0; r < L.nr; r++) {
            const RotInfo* rp = B.rot + L.rot_off + r;
            int left_nsurv = -1;
            for (int side = 0; side < 2; side++) {
                const SideInfo ri = side_info(rp, side);
                Sweep sw;
                sweep_setup(P, B, L, ri, side, left_nsurv, W, sw);
                left_nsurv = sw.pruned ? sw.nsurv : -1;
                int deg;
                if (ri.mode == kFlat) {
                    const int st = ri.step;
                    int k = eval_candidates<NB, PPL>(P, B, sw, W, trig, 0, st, 360 / st, acc);
                    deg = k < 0 ? 0 : k * st;
                } else {
                    const int hp = ri.step, x = ri.tile;
                    int t = eval_candidates<NB, PPL>(P, B, sw, W, trig, ri.off, x, 360 / x, acc);
                    if (t < 0) t = 0;
                    int k = eval_candidates<NB, PPL>(P, B, sw, W, trig, t * x, hp, x / hp, acc);
                    deg = k < 0 ? 0 : t * x + k * hp;
                }
                commit(sw.mvl, sw.m, W, sw.lp, deg);
                acc.sweeps++;
                const int ql = out.q & (kWave - 1);
                out.angv = lane_id() == ql ? deg : out.angv;
                if (ql == kWave - 1 || out.q == total - 1) {
                    uint16_t* dst = B.ang + L.ang_off + (size_t)o0 * nrec + (out.q - ql);
                    if (lane_id() <= ql) dst[lane_id()] = (uint16_t)out.angv;
                }
                out.q++;
            }
        }
    }
    int S;
    bool clash;
    endpoint(P, B, L, W, S, clash, acc);
    const uint64_t key = ((uint64_t)clash << 63) | ((uint64_t)(uint32_t)S << 32) | (uint64_t)(uint32_t)o;
    out.keyv = lane_id() == o - o0 ? key : out.keyv;
    if (o - o0 == n_item - 1 && lane_id() < n_item) B.keys[L.key_off + o0 + lane_id()] = out.keyv;
}

__device__ void flush(unsigned long long* counters, Acc& acc) {
    int oob = wave_sum(acc.oob);
    if (lane_id() == 0 && counters) {
        atomicAdd(counters + GD_CNT_POSES, (unsigned long long)acc.poses);
        atomicAdd(counters + GD_CNT_FALLBACK, (unsigned long long)acc.fallback);
        atomicAdd(counters + GD_CNT_OOB, (unsigned long long)oob);
        atomicAdd(counters + GD_CNT_SWEEPS, (unsigned long long)acc.sweeps);
    }
    acc = Acc();
}

// Per-ligand form: one launch per ligand, one wave per orientation.
template <int NB, int PPL>
// Register budget: the per-ligand form at >= 3 waves per SIMD (<= 168 VGPRs),
// the persistent form at >= 4 (<= 128 VGPRs, a few spills outside the inner
// loops); with 2-wave blocks the LDS slices then admit 4 waves per SIMD for
// ligands of up to 80 atoms.
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3))) dock_ligand_kernel(const PocketDev* __restrict__ Pp,
                                                          const BatchDev* __restrict__ Bp,
                                                          unsigned long long* counters, int lig, int nmax) {
    const PocketDev& P = *Pp;
    const BatchDev& B = *Bp;
    extern __shared__ __align__(16) char smem[];
    const int wave = uniform(threadIdx.x / kWave);
    const WaveLds W = carve(smem + wave * wave_lds_bytes(B.lmax, nmax), B.lmax, nmax);
    const int o = uniform(blockIdx.x * (blockDim.x / kWave) + wave);
    Acc acc;
    if (o < B.n_orient) {
        ItemOut out;
        dock_orientation<NB, PPL>(P, B, lig, o, o, 1, W, c_trig32, acc, out);
    }
    flush(counters, acc);
}

// Batched form: a persistent grid; every wave pops (ligand, orientation
// block) items from the device queue until it is empty.
template <int NB, int PPL>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) dock_persistent_kernel(const PocketDev* __restrict__ Pp,
                                                              const BatchDev* __restrict__ Bp,
                                                              unsigned long long* counters, int nmax) {
    const PocketDev& P = *Pp;
    const BatchDev& B = *Bp;
    extern __shared__ __align__(16) char smem[];
    const int wave = uniform(threadIdx.x / kWave);
    const WaveLds W = carve(smem + wave * wave_lds_bytes(B.lmax, nmax), B.lmax, nmax);
    Acc acc;
    for (;;) {
        int item = 0;
        if (lane_id() == 0) item = atomicAdd(B.head, 1);
        item = uniform(item);  // lane 0 took the item and is the first active lane
        if (item >= B.n_items) break;
        const int lig = ldc(B.items + 2 * item), o0 = ldc(B.items + 2 * item + 1);
        const int o1 = min(o0 + B.orient_per_item, B.n_orient);
        // at most 8 orientations per item (one key per lane)
        ItemOut out;
        for (int o = o0; o < o1; o++) dock_orientation<NB, PPL>(P, B, lig, o, o0, o1 - o0, W, c_trig32, acc, out);
    }
    flush(counters, acc);
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
    const LigMeta L = ldg_record(B.lig + lig);
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
    const int wave = uniform(threadIdx.x / kWave);
    const int idx = blockIdx.x * (blockDim.x / kWave) + wave;
    if (idx >= B.n_lig * B.top_k) return;
    const int lig = idx / B.top_k;
    WaveLds W{};
    const int lp = lds_pitch(B.lmax);
    W.X = (lds_double*)(smem + wave * replay_lds_bytes(B.lmax));
    W.SW = W.X + 3 * lp;
    const LigMeta L = ldg_record(B.lig + lig);
    const int o = recs[idx].orient;
    place(P, B, L, o, W);
    const int nrec = B.reps * L.nr * 2;
    const uint16_t* ang = B.ang + L.ang_off + (size_t)o * nrec;
    for (int rep = 0; rep < B.reps; rep++)
        for (int r = 0; r < L.nr; r++) {
            const RotInfo* rp = B.rot + L.rot_off + r;
            for (int side = 0; side < 2; side++) {
                const SideInfo ri = side_info(rp, side);
                sweep_axis(W, lp, ri.a, ri.c, ri.piv, side == 1);
                commit(B.mv + ri.mv_off, ri.n_mv, W, lp, ang[(rep * L.nr + r) * 2 + side]);
            }
        }
    float* dst = xyz + (size_t)idx * B.lmax * 3;
    for (int i = lane_id(); i < B.lmax; i += kWave) {
        bool in = i < L.l;
        dst[3 * i + 0] = in ? (float)W.X[i] : 0.f;
        dst[3 * i + 1] = in ? (float)W.X[lp + i] : 0.f;
        dst[3 * i + 2] = in ? (float)W.X[2 * lp + i] : 0.f;
    }
}

// Overlap landscape of every rotamer side at each ranked pose (the peak
// analysis of Section III-B).  The pose is rebuilt in FP64 as the replay does;
// then each side of each rotamer is turned about its bond from that pose by
// every multiple of `step` degrees and evaluated as a sweep's FP64 path does:
// whole-ligand S (the turned side's S plus that of the atoms that stay) and
// the straddling pairs' feasibility.  One wave per ranked pose; a record whose
// orientation or stored angles are out of range (no docking call before)
// yields zeros.
__global__ void __launch_bounds__(256) profile_kernel(const PocketDev* Pp, BatchDev B, const gd_pose_rec* recs,
                                                      int step, int32_t* S_out, uint8_t* f_out, int32_t* size_out) {
    extern __shared__ __align__(16) char smem[];
    const int wave = uniform(threadIdx.x / kWave);
    const int idx = blockIdx.x * (blockDim.x / kWave) + wave;
    if (idx >= B.n_lig * B.top_k) return;
    const int lane = lane_id();
    const int lig = idx / B.top_k;
    const int nang = 360 / step;
    WaveLds W{};
    const int lp = lds_pitch(B.lmax);
    W.X = (lds_double*)(smem + wave * replay_lds_bytes(B.lmax));
    W.SW = W.X + 3 * lp;
    const LigMeta L = ldg_record(B.lig + lig);
    const int o = recs[idx].orient;
    const int nrec = B.reps * L.nr * 2;
    bool ok = o >= 0 && o < B.n_orient;
    const uint16_t* ang = B.ang + L.ang_off + (size_t)(ok ? o : 0) * nrec;
    for (int q = 0; q < nrec && ok; q++) ok = ang[q] < 360;
    if (ok) {
        place(*Pp, B, L, o, W);
        for (int rep = 0; rep < B.reps; rep++)
            for (int r = 0; r < L.nr; r++) {
                const RotInfo* rp = B.rot + L.rot_off + r;
                for (int side = 0; side < 2; side++) {
                    const SideInfo ri = side_info(rp, side);
                    sweep_axis(W, lp, ri.a, ri.c, ri.piv, side == 1);
                    commit(B.mv + ri.mv_off, ri.n_mv, W, lp, ang[(rep * L.nr + r) * 2 + side]);
                }
            }
    }
    for (int r = 0; r < B.rmax; r++)
        for (int side = 0; side < 2; side++) {
            const size_t row = ((size_t)idx * B.rmax + r) * 2 + side;
            int32_t* So = S_out + row * nang;
            uint8_t* fo = f_out + row * nang;
            if (!ok || r >= L.nr) {
                for (int t = lane; t < nang; t += kWave) {
                    So[t] = 0;
                    fo[t] = 0;
                }
                if (lane == 0) size_out[row] = 0;
                continue;
            }
            const SideInfo si = side_info(B.rot + L.rot_off + r, side);
            sweep_axis(W, lp, si.a, si.c, si.piv, false);
            const uint8_t* mvl = B.mv + si.mv_off;
            int oob = 0;
            long long s_all = 0, s_mv = 0;
            for (int i = lane; i < L.l; i += kWave) s_all += D_exact(*Pp, W.X[i], W.X[lp + i], W.X[2 * lp + i], oob);
            for (int j = lane; j < si.n_mv; j += kWave) {
                const int i = ldg(mvl + j);
                s_mv += D_exact(*Pp, W.X[i], W.X[lp + i], W.X[2 * lp + i], oob);
            }
            const long long s_fixed = wave_sum64(s_all) - wave_sum64(s_mv);
            for (int t = 0; t < nang; t++) {
                const uint64_t v = eval_fp64(Pp, W.X, W.SW, lp, mvl, si.n_mv, B.pairs + si.pair_off, si.n_pairs, side,
                                             B.cd2, t * step);
                if (lane == 0) {
                    So[t] = sat_S(s_fixed + (long long)(v & ((1ull << 40) - 1)));
                    fo[t] = (uint8_t)((v >> 40) & 1);
                }
            }
            if (lane == 0) size_out[row] = si.n_mv;
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
    float t32[720];
    for (int d = 0; d < 360; d++) {
        t32[d] = c32[d];
        t32[360 + d] = s32[d];
    }
    if ((e = hipMemcpyToSymbol(HIP_SYMBOL(c_trig32), t32, sizeof(t32))) != hipSuccess) return e;
    done = true;
    return hipSuccess;
}

size_t dock_lds_bytes(int lmax, int nmax, int waves) { return wave_lds_bytes(lmax, nmax) * waves; }

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

template <int NB, int PPL>
static hipError_t launch_dock_t(const DockLaunch& L, int waves, bool persistent, int lig, int grid, hipStream_t s) {
    size_t lds = dock_lds_bytes(L.lmax, L.nmax, waves);
    if (persistent)
        hipLaunchKernelGGL((dock_persistent_kernel<NB, PPL>), dim3(grid), dim3(waves * kWave), lds, s, L.P, L.B,
                           L.counters, L.nmax);
    else
        hipLaunchKernelGGL((dock_ligand_kernel<NB, PPL>), dim3(grid), dim3(waves * kWave), lds, s, L.P, L.B,
                           L.counters, lig, L.nmax);
    return hipGetLastError();
}

template <int NB>
static hipError_t launch_dock_nb(const DockLaunch& L, const Tiling& t, bool persistent, int lig, int grid,
                                 hipStream_t s) {
    switch (t.pairs_per_lane) {
        case 1: return launch_dock_t<NB, 1>(L, t.waves_per_block, persistent, lig, grid, s);
        case 2: return launch_dock_t<NB, 2>(L, t.waves_per_block, persistent, lig, grid, s);
        case 4: return launch_dock_t<NB, 4>(L, t.waves_per_block, persistent, lig, grid, s);
        case 8: return launch_dock_t<NB, 8>(L, t.waves_per_block, persistent, lig, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dock(const DockLaunch& L, const Tiling& t, bool persistent, int lig, int grid, hipStream_t s) {
    switch (t.angle_block) {
        case 8: return launch_dock_nb<8>(L, t, persistent, lig, grid, s);
        case 16: return launch_dock_nb<16>(L, t, persistent, lig, grid, s);
        case 32: return launch_dock_nb<32>(L, t, persistent, lig, grid, s);
        default: return hipErrorInvalidValue;
    }
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

hipError_t launch_profile(const PocketDev* Pd, const BatchDev& B, const gd_pose_rec* recs, int step, int32_t* S_out,
                          uint8_t* f_out, int32_t* size_out, hipStream_t s) {
    const int waves = 4;
    const int n = B.n_lig * B.top_k;
    const size_t lds = replay_lds_bytes(B.lmax) * waves;
    hipLaunchKernelGGL(profile_kernel, dim3((n + waves - 1) / waves), dim3(waves * kWave), lds, s, Pd, B, recs, step,
                       S_out, f_out, size_out);
    return hipGetLastError();
}

}  // namespace gd
