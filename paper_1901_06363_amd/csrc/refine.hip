// Pose refinement on a smoothed pocket density, in FP32.
//
//   rho(g)  = sum_j exp(-|g - P_j|^2 / (2 sigma^2)) (cut off) on the lattice
//             bh * (i, j, k), tabulated on the host
//   rho~(x) = trilinear interpolation of rho in the cell containing x
//   F       = sum_i rho~(X_i)
//   X(t, q, tau) = R(q/|q|) (FK_tau(X0) - c0) + c0 + t
// FK_tau rotates, root (atom 0) first, the side of every rotamer that does not
// hold atom 0 by tau_b about its current axis (near -> far atom, right-handed).
//
// Backward pass (no stored activations: the pose is recomputed), with
// o = c0 + t the centre of the rigid rotation and g_i = grad rho~(X_i):
//   dF/dt     = sum_i g_i
//   dF/dq     = (I - qh qh^T)/|q| * d(omega)/dqh . T,  T = sum_i (X_i - o) x g_i
//   dF/dtau_b = K_b . sum_{i moving} (X_i - A_b) x g_i
//             = sum_{i moving} K_b . ((X_i - o) x g_i) - (K_b x (A_b - o)) . g_i
// (final-frame axis K_b through A_b).  Lever arms are taken from o, so the sums
// do not cancel for poses far from the coordinate origin.
//
// One wavefront per pose.  A ligand of at most 64 atoms has one atom per lane
// (one slot); a larger one two (atom i in lane i % 64 of slot i / 64).  The
// per-rotamer gradient terms are summed eight rotamers at a time by one
// transposed reduction, and the final-frame axes are formed one rotamer per
// lane.  Internally torsions are kept in tree order (root first).
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "gd_internal.h"

// The refinement is compared with the FP64 oracle within a tolerance, not bit
// for bit: let the compiler fuse multiply-adds here (the library is otherwise
// built without contraction, which the docking kernel's rounding guards need).
#pragma clang fp contract(fast)

namespace gd {

constexpr int kSlotsMax = kMaxAtoms / kWave;  // atom slots per lane for the largest ligands
static_assert(kSlotsMax == 2, "one or two atom slots per lane");
static_assert(kMaxRot <= kWave, "one torsion per lane");

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

__device__ __forceinline__ float rlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Sum over the wavefront, the total in every lane, without LDS: a butterfly
// of DPP lane permutations (lane ^ 1, lane ^ 2, the two quads of a half row,
// the two halves of a row) and then the gfx950 permlane swaps of rows of 16
// and halves of the wave (the two outputs of a swap hold a lane's value and
// its partner's).
__device__ __forceinline__ float wsum(float v) {
    v += dpp_f<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f<0x141>(v);  // row_half_mirror
    v += dpp_f<0x128>(v);  // row_ror:8
    const auto p = __builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(v), false, false);
    v = __int_as_float((int)p[0]) + __int_as_float((int)p[1]);
    const auto q = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false);
    return __int_as_float((int)q[0]) + __int_as_float((int)q[1]);
}

// Wave totals of eight values at once (a transposed butterfly): afterwards a
// lane whose index has bits 5, 4, 3 equal to (b5, b4, b3) holds the total of
// value 4 b5 + 2 b4 + b3.  A permlane swap of two registers sends half of each
// to the partner lanes, so every stage halves the values a lane carries:
// 32-lane halves (8 -> 4 values), 16-lane rows (4 -> 2), 8-lane halves of a
// row (2 -> 1), then a plain butterfly within groups of eight lanes.
__device__ __forceinline__ float wsum8(const float v[8]) {
    float w[4], x[2];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const auto p = __builtin_amdgcn_permlane32_swap(__float_as_int(v[j]), __float_as_int(v[j + 4]), false, false);
        w[j] = __int_as_float((int)p[0]) + __int_as_float((int)p[1]);
    }
#pragma unroll
    for (int j = 0; j < 2; j++) {
        const auto p = __builtin_amdgcn_permlane16_swap(__float_as_int(w[j]), __float_as_int(w[j + 2]), false, false);
        x[j] = __int_as_float((int)p[0]) + __int_as_float((int)p[1]);
    }
    const bool hi = (lane_id() & 8) != 0;
    float y = (hi ? x[1] : x[0]) + dpp_f<0x128>(hi ? x[0] : x[1]);  // row_ror:8 = lane ^ 8 within a row
    y += dpp_f<0xB1>(y);
    y += dpp_f<0x4E>(y);
    y += dpp_f<0x141>(y);
    return y;
}

// The lane of wsum8's output that holds value j.
__device__ __forceinline__ int wsum8_lane(int j) { return ((j >> 2) & 1) * 32 + ((j >> 1) & 1) * 16 + (j & 1) * 8; }

// Coordinate a of a wave-uniform atom index held in the per-lane slots.
template <int NS>
__device__ __forceinline__ float atom_at(const float Y[NS][3], int i, int a) {
    if (NS == 1) return rlane(Y[0][a], i);
    const float lo = rlane(Y[0][a], i & 63);
    const float hi = rlane(Y[NS - 1][a], i & 63);
    return i < kWave ? lo : hi;
}

// Trilinear density and its gradient; corners outside the tabulated box are 0
// (every node beyond the box lies farther than the cutoff from the points).
// The cell's eight corners are two 16-byte nodes of the corner-packed grid;
// a cell with no corner in the box reads nothing.
__device__ __forceinline__ float rho_tri(const PocketDev& P, float x, float y, float z, float& gx, float& gy,
                                         float& gz) {
    float ux = x * P.inv_bh, uy = y * P.inv_bh, uz = z * P.inv_bh;
    float fx0 = floorf(ux), fy0 = floorf(uy), fz0 = floorf(uz);
    float fx = ux - fx0, fy = uy - fy0, fz = uz - fz0;
    int ix = (int)fx0 - P.blo[0], iy = (int)fy0 - P.blo[1], iz = (int)fz0 - P.blo[2];
    float4 lo = make_float4(0.f, 0.f, 0.f, 0.f), hi = lo;
    // at most 1024 nodes per axis (checked at pocket creation): the index fits 32 bits
    if ((unsigned)(ix + 1) <= (unsigned)P.bdim[0] && (unsigned)(iy + 1) <= (unsigned)P.bdim[1] &&
        (unsigned)(iz + 1) <= (unsigned)P.bdim[2]) {
        const int qx = P.bdim[0] + 1, qxy = qx * (P.bdim[1] + 1);
        const int n0 = (iz + 1) * qxy + (iy + 1) * qx + (ix + 1);
        lo = P.rho4[n0];
        hi = P.rho4[n0 + qxy];
    }
    const float r[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    float ax = 1.f - fx, ay = 1.f - fy, az = 1.f - fz;
    // interpolate along x, then y, then z
    float r00 = ax * r[0] + fx * r[1], r10 = ax * r[2] + fx * r[3];
    float r01 = ax * r[4] + fx * r[5], r11 = ax * r[6] + fx * r[7];
    float d00 = r[1] - r[0], d10 = r[3] - r[2], d01 = r[5] - r[4], d11 = r[7] - r[6];
    float r0 = ay * r00 + fy * r10, r1 = ay * r01 + fy * r11;
    gx = (az * (ay * d00 + fy * d10) + fz * (ay * d01 + fy * d11)) * P.inv_bh;
    gy = (az * (r10 - r00) + fz * (r11 - r01)) * P.inv_bh;
    gz = (r1 - r0) * P.inv_bh;
    return az * r0 + fz * r1;
}

__device__ __forceinline__ void quat_mat(const float* q, float* R) {
    const float in = 1.f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    float w = q[0] * in, x = q[1] * in, y = q[2] * in, z = q[3] * in;
    R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z);       R[2] = 2.f * (x * z + w * y);
    R[3] = 2.f * (x * y + w * z);       R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
    R[6] = 2.f * (x * z - w * y);       R[7] = 2.f * (y * z + w * x);       R[8] = 1.f - 2.f * (x * x + y * y);
}

// Per-wave state of one pose.
template <int NS>
struct PoseState {
    int l, nr, tree0, lig;
    float x0[NS][3];  // input pose (this lane's atoms)
    float c0[3];      // centroid of the input pose
    uint64_t mv[NS];  // bit e: this lane's atom moves with tree entry e (root-first order)
};

// Atom count of a pose's ligand (picks the slot form before load_pose).
__device__ __forceinline__ int pose_atoms(const TreeDev& T, const PoseDev& X, int pose) {
    return __builtin_amdgcn_readfirstlane(T.n_atoms[X.pose_lig[pose]]);
}

template <int NS>
__device__ void load_pose(const TreeDev& T, const PoseDev& X, int pose, PoseState<NS>& S) {
    const int lane = lane_id();
    const int lig = X.pose_lig[pose], off = X.pose_off[pose];
    S.l = T.n_atoms[lig];
    S.lig = lig;
    S.nr = T.nr[lig];
    S.tree0 = T.tree_off[lig];
    float s[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < NS; k++) {
        int i = lane + k * kWave;
        bool in = i < S.l;
        S.x0[k][0] = in ? X.px[off + i] : 0.f;
        S.x0[k][1] = in ? X.py[off + i] : 0.f;
        S.x0[k][2] = in ? X.pz[off + i] : 0.f;
        s[0] += S.x0[k][0];
        s[1] += S.x0[k][1];
        s[2] += S.x0[k][2];
    }
    for (int a = 0; a < 3; a++) S.c0[a] = wsum(s[a]) / (float)S.l;
#pragma unroll
    for (int k = 0; k < NS; k++) {
        const int i = lane + k * kWave;
        uint64_t b = 0;
        for (int e = 0; e < S.nr; e++) {
            const uint32_t* mk = T.tmask + 4 * (size_t)(S.tree0 + e);
            if (i < S.l && ((mk[i >> 5] >> (i & 31)) & 1u)) b |= 1ull << e;
        }
        S.mv[k] = b;
    }
}

// Forward kinematics + rigid motion; Ys gets FK_tau(X0) for this lane's
// atoms, Xf the final pose.  tau (tree order, this wave's LDS); with axes the
// pivot and unit axis of every tree entry in the torsion frame are stored
// there (6 floats per entry).
template <int NS>
__device__ void pose_forward(const TreeDev& T, const PoseState<NS>& S, const float* t, const float* q, const float* tau,
                             float* axes, float Ys[NS][3], float Xf[NS][3], float Rq[9]) {
#pragma unroll
    for (int k = 0; k < NS; k++)
        for (int a = 0; a < 3; a++) Ys[k][a] = S.x0[k][a];
    // lane e holds sin/cos of tree entry e; each edge reads its pair with a
    // uniform readlane instead of evaluating it
    float s_lane = 0.f, c_lane = 1.f;
    if (lane_id() < S.nr) sincosf(tau[lane_id()], &s_lane, &c_lane);
    for (int e = 0; e < S.nr; e++) {
        const int4 te = T.tree[S.tree0 + e];
        const int ia = __builtin_amdgcn_readfirstlane(te.x), ib = __builtin_amdgcn_readfirstlane(te.y);
        const float px = atom_at<NS>(Ys, ia, 0), py = atom_at<NS>(Ys, ia, 1), pz = atom_at<NS>(Ys, ia, 2);
        float kx = atom_at<NS>(Ys, ib, 0) - px, ky = atom_at<NS>(Ys, ib, 1) - py, kz = atom_at<NS>(Ys, ib, 2) - pz;
        const float inv = rsqrtf(kx * kx + ky * ky + kz * kz);
        kx *= inv;
        ky *= inv;
        kz *= inv;
        if (axes && lane_id() == 0) {
            float* ax = axes + 6 * e;
            ax[0] = px;
            ax[1] = py;
            ax[2] = pz;
            ax[3] = kx;
            ax[4] = ky;
            ax[5] = kz;
        }
        const float s = rlane(s_lane, e), c = rlane(c_lane, e);
        float tt = 1.f - c;
        float R[9] = {tt * kx * kx + c,      tt * kx * ky - s * kz, tt * kx * kz + s * ky,
                      tt * kx * ky + s * kz, tt * ky * ky + c,      tt * ky * kz - s * kx,
                      tt * kx * kz - s * ky, tt * ky * kz + s * kx, tt * kz * kz + c};
#pragma unroll
        for (int k = 0; k < NS; k++) {
            if ((S.mv[k] >> e) & 1) {
                float d0 = Ys[k][0] - px, d1 = Ys[k][1] - py, d2 = Ys[k][2] - pz;
                Ys[k][0] = px + (R[0] * d0 + R[1] * d1 + R[2] * d2);
                Ys[k][1] = py + (R[3] * d0 + R[4] * d1 + R[5] * d2);
                Ys[k][2] = pz + (R[6] * d0 + R[7] * d1 + R[8] * d2);
            }
        }
    }
    quat_mat(q, Rq);
#pragma unroll
    for (int k = 0; k < NS; k++) {
        float d0 = Ys[k][0] - S.c0[0], d1 = Ys[k][1] - S.c0[1], d2 = Ys[k][2] - S.c0[2];
        Xf[k][0] = (Rq[0] * d0 + Rq[1] * d1 + Rq[2] * d2) + S.c0[0] + t[0];
        Xf[k][1] = (Rq[3] * d0 + Rq[4] * d1 + Rq[5] * d2) + S.c0[1] + t[1];
        Xf[k][2] = (Rq[6] * d0 + Rq[7] * d1 + Rq[8] * d2) + S.c0[2] + t[2];
    }
}

// Bump penalty of the clash-penalised surrogate: subtracts clash_weight *
// (cd2 - d^2)^2 over the ligand's far pairs closer than the bump distance from
// F (lane partial) and, with GRAD, its derivative from the per-atom gradients
// g.  Atoms go through this wave's LDS (xs, gs: 3 floats per atom); lanes own
// pairs and add their gradient contributions with LDS atomics.
template <bool GRAD, int NS>
__device__ void bump_penalty(const Penalty pen, const PoseState<NS>& S, const float Xf[NS][3], float g[NS][3],
                             float& F, float* xs, float* gs) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < NS; k++) {
        const int i = lane + k * kWave;
        if (i < S.l)
            for (int a = 0; a < 3; a++) {
                xs[3 * i + a] = Xf[k][a];
                gs[3 * i + a] = 0.f;
            }
    }
    wave_sync();
    const uint16_t* fp = pen.efar + pen.far_off[S.lig];
    const int nf = pen.n_far[S.lig];
    float e2 = 0.f;
    for (int q = lane; q < nf; q += kWave) {
        const uint32_t pr = fp[q];
        const int i = pr & 0xff, j = pr >> 8;
        const float dx = xs[3 * i] - xs[3 * j], dy = xs[3 * i + 1] - xs[3 * j + 1], dz = xs[3 * i + 2] - xs[3 * j + 2];
        const float d2 = dx * dx + dy * dy + dz * dz;
        if (d2 < pen.cd2) {
            const float e = pen.cd2 - d2;
            e2 += e * e;
            if (GRAD) {
                // -w d(e^2)/dX_i = 4 w e (X_i - X_j), the opposite for X_j
                const float c = 4.f * pen.w * e;
                atomicAdd(&gs[3 * i], c * dx);
                atomicAdd(&gs[3 * i + 1], c * dy);
                atomicAdd(&gs[3 * i + 2], c * dz);
                atomicAdd(&gs[3 * j], -c * dx);
                atomicAdd(&gs[3 * j + 1], -c * dy);
                atomicAdd(&gs[3 * j + 2], -c * dz);
            }
        }
    }
    F -= pen.w * e2;
    if (GRAD) {
        wave_sync();
#pragma unroll
        for (int k = 0; k < NS; k++) {
            const int i = lane + k * kWave;
            if (i < S.l)
                for (int a = 0; a < 3; a++) g[k][a] += gs[3 * i + a];
        }
    }
    wave_sync();
}

// LDS of one wave: torsions and their gradient (tree order), the torsion-frame
// pivot and axis of every tree entry (6 floats), the final-frame axis K and
// K x (A - o) of every entry (8 floats, two 16-byte rows), and with the bump
// penalty the atoms and their gradients (3 floats per atom).
struct WaveBuf {
    float* tau;
    float* gtau;
    float* axes;
    float* kax;
    float* xs;
    float* gs;
};

// F and (optionally) dF/d(t, q, tau) at the given parameters; only
// lane-uniform values are returned, gtau in the wave's LDS.  With pen.w > 0 F
// is the clash-penalised surrogate.  WANT_F = false skips the value's sum
// (the ascent needs only the gradient).
template <bool GRAD, int NS, bool WANT_F = true>
__device__ float surrogate_eval(const PocketDev& P, const TreeDev& T, const PoseState<NS>& S, const float* t,
                                const float* q, const WaveBuf& W, float* gt, float* gq, float Xout[NS][3],
                                const Penalty pen = Penalty{}) {
    const int lane = lane_id();
    float Ys[NS][3], Xf[NS][3], g[NS][3], Rq[9];
    pose_forward<NS>(T, S, t, q, W.tau, GRAD ? W.axes : nullptr, Ys, Xf, Rq);
    float F = 0.f;
#pragma unroll
    for (int k = 0; k < NS; k++) {
        int i = lane + k * kWave;
        if (i < S.l) {
            F += rho_tri(P, Xf[k][0], Xf[k][1], Xf[k][2], g[k][0], g[k][1], g[k][2]);
        } else {
            g[k][0] = g[k][1] = g[k][2] = 0.f;
        }
        if (Xout)
            for (int a = 0; a < 3; a++) Xout[k][a] = Xf[k][a];
    }
    if (pen.w > 0.f) bump_penalty<GRAD, NS>(pen, S, Xf, g, F, W.xs, W.gs);
    if (!GRAD) return wsum(F);
    // lever arms from the centre of the rigid rotation
    const float ox = S.c0[0] + t[0], oy = S.c0[1] + t[1], oz = S.c0[2] + t[2];
    float xg[NS][3];
#pragma unroll
    for (int k = 0; k < NS; k++) {
        const float rx = Xf[k][0] - ox, ry = Xf[k][1] - oy, rz = Xf[k][2] - oz;
        xg[k][0] = ry * g[k][2] - rz * g[k][1];
        xg[k][1] = rz * g[k][0] - rx * g[k][2];
        xg[k][2] = rx * g[k][1] - ry * g[k][0];
    }
    // the rigid-body sums in one transposed reduction: sum g (3), the torque (3), F
    float tq[3];
    {
        float v[8];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            v[a] = g[0][a];
            v[3 + a] = xg[0][a];
#pragma unroll
            for (int k = 1; k < NS; k++) {
                v[a] += g[k][a];
                v[3 + a] += xg[k][a];
            }
        }
        v[6] = WANT_F ? F : 0.f;
        v[7] = 0.f;
        const float r = wsum8(v);
        for (int a = 0; a < 3; a++) {
            gt[a] = rlane(r, wsum8_lane(a));
            tq[a] = rlane(r, wsum8_lane(3 + a));
        }
        if (WANT_F) F = rlane(r, wsum8_lane(6));
    }
    // quaternion: a tangent change dq of the unit quaternion (w, v) turns the
    // pose by omega = 2 (w dv - dw v + v x dv) about o, so dF = omega . T;
    // divided by |q| for the unnormalised parameter
    {
        const float in = 1.f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const float w = q[0] * in, x = q[1] * in, y = q[2] * in, z = q[3] * in;
        gq[0] = -2.f * (tq[0] * x + tq[1] * y + tq[2] * z) * in;
        gq[1] = 2.f * (w * tq[0] + (tq[1] * z - tq[2] * y)) * in;
        gq[2] = 2.f * (w * tq[1] + (tq[2] * x - tq[0] * z)) * in;
        gq[3] = 2.f * (w * tq[2] + (tq[0] * y - tq[1] * x)) * in;
    }
    // torsions: lane e carries tree entry e's pivot and axis into the final
    // frame, K = Rq k and A - o = Rq (p - c0), and keeps K and K x (A - o)
    wave_sync();
    if (lane < S.nr) {
        const float* axe = W.axes + 6 * lane;
        const float d0 = axe[0] - S.c0[0], d1 = axe[1] - S.c0[1], d2 = axe[2] - S.c0[2];
        const float ax = Rq[0] * d0 + Rq[1] * d1 + Rq[2] * d2;
        const float ay = Rq[3] * d0 + Rq[4] * d1 + Rq[5] * d2;
        const float az = Rq[6] * d0 + Rq[7] * d1 + Rq[8] * d2;
        const float kx = Rq[0] * axe[3] + Rq[1] * axe[4] + Rq[2] * axe[5];
        const float ky = Rq[3] * axe[3] + Rq[4] * axe[4] + Rq[5] * axe[5];
        const float kz = Rq[6] * axe[3] + Rq[7] * axe[4] + Rq[8] * axe[5];
        float* kr = W.kax + 8 * lane;
        kr[0] = kx;
        kr[1] = ky;
        kr[2] = kz;
        kr[4] = ky * az - kz * ay;
        kr[5] = kz * ax - kx * az;
        kr[6] = kx * ay - ky * ax;
    }
    wave_sync();
    // per atom K . ((X - o) x g) - (K x (A - o)) . g over the entries that
    // move it, eight entries per transposed reduction
    for (int e0 = 0; e0 < S.nr; e0 += 8) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            v[j] = 0.f;
            const int e = e0 + j;
            if (e < S.nr) {
                const float* kr = W.kax + 8 * e;
                const float kx = kr[0], ky = kr[1], kz = kr[2], cx = kr[4], cy = kr[5], cz = kr[6];
#pragma unroll
                for (int k = 0; k < NS; k++) {
                    const float term = (kx * xg[k][0] + ky * xg[k][1] + kz * xg[k][2]) -
                                       (cx * g[k][0] + cy * g[k][1] + cz * g[k][2]);
                    v[j] += ((S.mv[k] >> e) & 1) ? term : 0.f;
                }
            }
        }
        const float r = wsum8(v);
        const int j = ((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1);
        if ((lane & 7) == 0 && e0 + j < S.nr) W.gtau[e0 + j] = r;
    }
    wave_sync();
    return F;
}

// ---------------------------------------------------------------------------

// One pose of the surrogate kernel in the slot form NS: F, or its gradient
// scaled by dF.
template <bool PEN, int NS>
__device__ void surrogate_pose(const PocketDev& P, const TreeDev& T, const PoseDev& X, int pose, const float* t,
                               const float* q, const float* tau, int tau_stride, const float* dF, float* F_out,
                               float* dt_out, float* dq_out, float* dtau_out, const Penalty& pen, const WaveBuf& W) {
    const int lane = lane_id();
    PoseState<NS> S;
    load_pose<NS>(T, X, pose, S);
    const float* tp = t + 3 * (size_t)pose;
    const float* qp = q + 4 * (size_t)pose;
    // torsions into tree order
    int rot_e = 0;
    if (lane < S.nr) {
        rot_e = T.tree[S.tree0 + lane].z;
        W.tau[lane] = tau[(size_t)tau_stride * pose + rot_e];
    }
    wave_sync();
    if (!dF) {
        float F = surrogate_eval<false, NS>(P, T, S, tp, qp, W, nullptr, nullptr, nullptr, pen);
        if (lane == 0) F_out[pose] = F;
        return;
    }
    float gt[3], gq[4];
    float F = surrogate_eval<true, NS>(P, T, S, tp, qp, W, gt, gq, nullptr, pen);
    const float up = dF[pose];
    if (lane == 0) {
        if (F_out) F_out[pose] = F;
        for (int a = 0; a < 3; a++) dt_out[3 * (size_t)pose + a] = up * gt[a];
        for (int a = 0; a < 4; a++) dq_out[4 * (size_t)pose + a] = up * gq[a];
    }
    for (int r = lane; r < tau_stride; r += kWave)
        if (r >= S.nr) dtau_out[(size_t)tau_stride * pose + r] = 0.f;
    if (lane < S.nr) dtau_out[(size_t)tau_stride * pose + rot_e] = up * W.gtau[lane];
}

template <bool PEN>
__global__ void __launch_bounds__(256) surrogate_kernel(PocketDev P, TreeDev T, PoseDev X, int n_poses,
                                                        const float* t, const float* q, const float* tau,
                                                        int tau_stride, const float* dF, float* F_out, float* dt_out,
                                                        float* dq_out, float* dtau_out, Penalty pen_in) {
    __shared__ float tau_all[4][kMaxRot], gtau_all[4][kMaxRot], axes_all[4][6 * kMaxRot];
    __shared__ __align__(16) float kax_all[4][8 * kMaxRot];
    __shared__ float pen_x[4][PEN ? 3 * kMaxAtoms : 1], pen_g[4][PEN ? 3 * kMaxAtoms : 1];
    const Penalty pen = PEN ? pen_in : Penalty{};
    const int wave = threadIdx.x / kWave;
    const int pose = blockIdx.x * 4 + wave;
    if (pose >= n_poses) return;
    const WaveBuf W{tau_all[wave], gtau_all[wave], axes_all[wave], kax_all[wave], pen_x[wave], pen_g[wave]};
    if (pose_atoms(T, X, pose) <= kWave)
        surrogate_pose<PEN, 1>(P, T, X, pose, t, q, tau, tau_stride, dF, F_out, dt_out, dq_out, dtau_out, pen, W);
    else
        surrogate_pose<PEN, 2>(P, T, X, pose, t, q, tau, tau_stride, dF, F_out, dt_out, dq_out, dtau_out, pen, W);
}

// The whole ascent of one pose in one wavefront (slot form NS): parameters
// stay in registers; the final pose is written to (rx, ry, rz).
template <bool PEN, int NS>
__device__ void refine_pose(const PocketDev& P, const TreeDev& T, const PoseDev& X, int pose, const RefineParams& rp,
                            float* rx, float* ry, float* rz, float* F_out, const WaveBuf& W) {
    const int lane = lane_id();
    PoseState<NS> S;
    load_pose<NS>(T, X, pose, S);
    const Penalty pen = PEN ? Penalty{rp.clash_weight, rp.cd2, rp.efar, rp.far_off, rp.n_far} : Penalty{};
    float t[3] = {0.f, 0.f, 0.f}, q[4] = {1.f, 0.f, 0.f, 0.f};
    float gt[3], gq[4];
    for (int r = lane; r < kMaxRot; r += kWave) W.tau[r] = W.gtau[r] = 0.f;
    wave_sync();
    for (int s = 0; s < rp.steps; s++) {
        surrogate_eval<true, NS, false>(P, T, S, t, q, W, gt, gq, nullptr, pen);
        float dt[3] = {rp.lr_t * gt[0], rp.lr_t * gt[1], rp.lr_t * gt[2]};
        float n = sqrtf(dt[0] * dt[0] + dt[1] * dt[1] + dt[2] * dt[2]);
        float sc = n > rp.max_dt ? rp.max_dt / n : 1.f;
        for (int a = 0; a < 3; a++) t[a] += dt[a] * sc;
        float qn = 0.f;
        for (int a = 0; a < 4; a++) {
            q[a] += rp.lr_q * gq[a];
            qn += q[a] * q[a];
        }
        qn = 1.f / sqrtf(qn);
        for (int a = 0; a < 4; a++) q[a] *= qn;
        if (lane < S.nr) W.tau[lane] += fminf(fmaxf(rp.lr_tau * W.gtau[lane], -rp.max_dtau), rp.max_dtau);
        wave_sync();
    }
    float Xf[NS][3];
    float F = surrogate_eval<false, NS>(P, T, S, t, q, W, nullptr, nullptr, Xf, pen);
    const int off = X.pose_off[pose];
#pragma unroll
    for (int k = 0; k < NS; k++) {
        int i = lane + k * kWave;
        if (i < S.l) {
            rx[off + i] = Xf[k][0];
            ry[off + i] = Xf[k][1];
            rz[off + i] = Xf[k][2];
        }
    }
    if (lane == 0) F_out[pose] = F;
}

// PEN: the clash-penalised surrogate (its own instance, so that the plain one
// keeps its registers and LDS).
template <bool PEN>
__global__ void __launch_bounds__(256) refine_kernel(PocketDev P, TreeDev T, PoseDev X, int n_poses, RefineParams rp,
                                                     float* rx, float* ry, float* rz, float* F_out) {
    __shared__ float tau_all[4][kMaxRot], gtau_all[4][kMaxRot], axes_all[4][6 * kMaxRot];
    __shared__ __align__(16) float kax_all[4][8 * kMaxRot];
    __shared__ float pen_x[4][PEN ? 3 * kMaxAtoms : 1], pen_g[4][PEN ? 3 * kMaxAtoms : 1];
    const int wave = threadIdx.x / kWave;
    const int pose = blockIdx.x * 4 + wave;
    if (pose >= n_poses) return;
    const WaveBuf W{tau_all[wave], gtau_all[wave], axes_all[wave], kax_all[wave], pen_x[wave], pen_g[wave]};
    if (pose_atoms(T, X, pose) <= kWave)
        refine_pose<PEN, 1>(P, T, X, pose, rp, rx, ry, rz, F_out, W);
    else
        refine_pose<PEN, 2>(P, T, X, pose, rp, rx, ry, rz, F_out, W);
}

// Keep the refined pose iff it is bump-free and strictly improves S.
__global__ void __launch_bounds__(256) accept_kernel(PoseDev X, int n_poses, const int32_t* n_atoms, const float* rx,
                                                     const float* ry, const float* rz, const int32_t* S_in,
                                                     const int32_t* S_ref, const uint8_t* c_ref, float* px, float* py,
                                                     float* pz, int32_t* S_out, uint8_t* clash_out, uint8_t* accepted,
                                                     const uint8_t* c_in) {
    const int wave = threadIdx.x / kWave;
    const int pose = blockIdx.x * 4 + wave;
    if (pose >= n_poses) return;
    const bool acc = !c_ref[pose] && S_ref[pose] < S_in[pose];
    const int off = X.pose_off[pose], l = n_atoms[X.pose_lig[pose]];
    if (acc)
        for (int i = lane_id(); i < l; i += kWave) {
            px[off + i] = rx[off + i];
            py[off + i] = ry[off + i];
            pz[off + i] = rz[off + i];
        }
    if (lane_id() == 0) {
        accepted[pose] = acc;
        S_out[pose] = acc ? S_ref[pose] : S_in[pose];
        clash_out[pose] = acc ? c_ref[pose] : c_in[pose];
    }
}

hipError_t launch_surrogate(const PocketDev& P, const TreeDev& T, const PoseDev& X, int n_poses, const float* t,
                            const float* q, const float* tau, int tau_stride, const float* dF, float* F_out,
                            float* dt_out, float* dq_out, float* dtau_out, const Penalty& pen, int lmax,
                            hipStream_t s) {
    (void)lmax;
    if (n_poses <= 0) return hipSuccess;
    if (pen.w > 0.f)
        hipLaunchKernelGGL(surrogate_kernel<true>, dim3((n_poses + 3) / 4), dim3(256), 0, s, P, T, X, n_poses, t, q,
                           tau, tau_stride, dF, F_out, dt_out, dq_out, dtau_out, pen);
    else
        hipLaunchKernelGGL(surrogate_kernel<false>, dim3((n_poses + 3) / 4), dim3(256), 0, s, P, T, X, n_poses, t, q,
                           tau, tau_stride, dF, F_out, dt_out, dq_out, dtau_out, pen);
    return hipGetLastError();
}

hipError_t launch_refine(const PocketDev& P, const TreeDev& T, const PoseDev& X, int n_poses,
                         const RefineParams& rp, float* rx, float* ry, float* rz, float* F_out, int lmax,
                         hipStream_t s) {
    (void)lmax;
    if (n_poses <= 0) return hipSuccess;
    if (rp.clash_weight > 0.f)
        hipLaunchKernelGGL(refine_kernel<true>, dim3((n_poses + 3) / 4), dim3(256), 0, s, P, T, X, n_poses, rp, rx, ry,
                           rz, F_out);
    else
        hipLaunchKernelGGL(refine_kernel<false>, dim3((n_poses + 3) / 4), dim3(256), 0, s, P, T, X, n_poses, rp, rx,
                           ry, rz, F_out);
    return hipGetLastError();
}

hipError_t launch_accept(const PoseDev& X, int n_poses, const int32_t* n_atoms, const float* rx, const float* ry,
                         const float* rz, const int32_t* S_in, const int32_t* S_ref, const uint8_t* c_ref,
                         float* px, float* py, float* pz, int32_t* S_out, uint8_t* clash_out, uint8_t* accepted,
                         const uint8_t* c_in, hipStream_t s) {
    if (n_poses <= 0) return hipSuccess;
    hipLaunchKernelGGL(accept_kernel, dim3((n_poses + 3) / 4), dim3(256), 0, s, X, n_poses, n_atoms, rx, ry, rz,
                       S_in, S_ref, c_ref, px, py, pz, S_out, clash_out, accepted, c_in);
    return hipGetLastError();
}

}  // namespace gd
