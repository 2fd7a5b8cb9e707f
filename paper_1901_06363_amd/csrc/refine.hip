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
// Backward pass (no stored activations: the pose is recomputed):
//   dF/dt     = sum_i g_i,               g_i = grad rho~(X_i)
//   dF/dq     = (I - qh qh^T)/|q| * <G, dR/dqh>,  G = sum_i g_i (Y_i - c0)^T
//   dF/dtau_b = K_b . sum_{i moving} (X_i - A_b) x g_i
//             = K_b . (sum x_i x g_i - A_b x sum g_i)   (final-frame axis K_b, A_b)
// One wavefront per pose; each lane holds two atoms (ligands of <= 128 atoms).
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "gd_internal.h"

// The refinement is compared with the FP64 oracle within a tolerance, not bit
// for bit: let the compiler fuse multiply-adds here (the library is otherwise
// built without contraction, which the docking kernel's rounding guards need).
#pragma clang fp contract(fast)

namespace gd {

constexpr int kSlots = kMaxAtoms / kWave;  // atoms per lane

// Sum over the wavefront, the total in every lane, without LDS: a butterfly
// of DPP lane permutations (lane ^ 1, lane ^ 2, the two quads of a half row,
// the two halves of a row) and then the gfx950 permlane swaps of rows of 16
// and halves of the wave (the two outputs of a swap hold a lane's value and
// its partner's).
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

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

// Coordinate of a wave-uniform atom index held in the per-lane slots (atom i
// lives in lane i % 64 of slot i / 64).
__device__ __forceinline__ float atom_at(const float Y[kSlots][3], int i, int a) {
    static_assert(kSlots == 2, "two atom slots per lane");
    const float lo = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(Y[0][a]), i & 63));
    const float hi = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(Y[1][a]), i & 63));
    return i < kWave ? lo : hi;
}

// Trilinear density and its gradient; corners outside the tabulated box are 0
// (every node beyond the box lies farther than the cutoff from the points).
__device__ __forceinline__ float rho_tri(const PocketDev& P, float x, float y, float z, float& gx, float& gy,
                                         float& gz) {
    float ux = x * P.inv_bh, uy = y * P.inv_bh, uz = z * P.inv_bh;
    float fx0 = floorf(ux), fy0 = floorf(uy), fz0 = floorf(uz);
    float fx = ux - fx0, fy = uy - fy0, fz = uz - fz0;
    int ix = (int)fx0 - P.blo[0], iy = (int)fy0 - P.blo[1], iz = (int)fz0 - P.blo[2];
    float r[8];
#pragma unroll
    for (int c = 0; c < 8; c++) {
        int jx = ix + (c & 1), jy = iy + ((c >> 1) & 1), jz = iz + (c >> 2);
        bool in = (unsigned)jx < (unsigned)P.bdim[0] && (unsigned)jy < (unsigned)P.bdim[1] &&
                  (unsigned)jz < (unsigned)P.bdim[2];
        // at most 1024 nodes per axis (checked at pocket creation): the index fits 32 bits
        r[c] = in ? P.rho[(jz * P.bdim[1] + jy) * P.bdim[0] + jx] : 0.f;
    }
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
struct PoseState {
    int l, nr, tree0, lig;
    float x0[kSlots][3];  // input pose (this lane's atoms)
    float c0[3];          // centroid of the input pose
    uint64_t mv[kSlots];  // bit e: this lane's atom moves with rotamer e (root-first order)
};

__device__ void load_pose(const TreeDev& T, const PoseDev& X, int pose, PoseState& S) {
    const int lane = lane_id();
    const int lig = X.pose_lig[pose], off = X.pose_off[pose];
    S.l = T.n_atoms[lig];
    S.lig = lig;
    S.nr = T.nr[lig];
    S.tree0 = T.tree_off[lig];
    float s[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < kSlots; k++) {
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
    for (int k = 0; k < kSlots; k++) {
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
// atoms, Xf the final pose.
__device__ void pose_forward(const TreeDev& T, const PoseState& S, const float* t, const float* q, const float* tau,
                             float* axes, float Ys[kSlots][3], float Xf[kSlots][3], float Rq[9]) {
#pragma unroll
    for (int k = 0; k < kSlots; k++)
        for (int a = 0; a < 3; a++) Ys[k][a] = S.x0[k][a];
    // Lane r holds sin/cos of torsion r (one torsion per lane at most); each
    // edge reads its pair with a uniform readlane instead of evaluating it.
    static_assert(kMaxRot <= kWave, "one torsion per lane");
    float s_lane = 0.f, c_lane = 1.f;
    if (lane_id() < S.nr) sincosf(tau[lane_id()], &s_lane, &c_lane);
    for (int e = 0; e < S.nr; e++) {
        const int4 te = T.tree[S.tree0 + e];
        const int ia = __builtin_amdgcn_readfirstlane(te.x), ib = __builtin_amdgcn_readfirstlane(te.y);
        const float px = atom_at(Ys, ia, 0), py = atom_at(Ys, ia, 1), pz = atom_at(Ys, ia, 2);
        float kx = atom_at(Ys, ib, 0) - px, ky = atom_at(Ys, ib, 1) - py, kz = atom_at(Ys, ib, 2) - pz;
        const float inv = rsqrtf(kx * kx + ky * ky + kz * kz);
        kx *= inv;
        ky *= inv;
        kz *= inv;
        if (axes && lane_id() == 0) {
            float* ax = axes + 6 * te.z;
            ax[0] = px;
            ax[1] = py;
            ax[2] = pz;
            ax[3] = kx;
            ax[4] = ky;
            ax[5] = kz;
        }
        const int rz = __builtin_amdgcn_readfirstlane(te.z);
        const float s = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(s_lane), rz));
        const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c_lane), rz));
        float tt = 1.f - c;
        float R[9] = {tt * kx * kx + c,      tt * kx * ky - s * kz, tt * kx * kz + s * ky,
                      tt * kx * ky + s * kz, tt * ky * ky + c,      tt * ky * kz - s * kx,
                      tt * kx * kz - s * ky, tt * ky * kz + s * kx, tt * kz * kz + c};
#pragma unroll
        for (int k = 0; k < kSlots; k++) {
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
    for (int k = 0; k < kSlots; k++) {
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
template <bool GRAD>
__device__ void bump_penalty(const Penalty pen, const PoseState& S, const float Xf[kSlots][3], float g[kSlots][3],
                             float& F, float* xs, float* gs) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < kSlots; k++) {
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
        for (int k = 0; k < kSlots; k++) {
            const int i = lane + k * kWave;
            if (i < S.l)
                for (int a = 0; a < 3; a++) g[k][a] += gs[3 * i + a];
        }
    }
    wave_sync();
}

// F and (optionally) dF/d(t, q, tau) at the given parameters.  tau, gtau and
// axes (6 floats per rotamer: pivot and unit axis in the torsion frame) are
// this wave's LDS arrays indexed by rotamer (list order); only lane-uniform
// values are returned.  With pen.w > 0 F is the clash-penalised surrogate;
// xs and gs are then this wave's LDS scratch (3 floats per atom).
template <bool GRAD>
__device__ float surrogate_eval(const PocketDev& P, const TreeDev& T, const PoseState& S, const float* t,
                                const float* q, const float* tau, float* axes, float* gt, float* gq, float* gtau,
                                float Xout[kSlots][3], const Penalty pen = Penalty{}, float* xs = nullptr,
                                float* gs = nullptr) {
    const int lane = lane_id();
    float Ys[kSlots][3], Xf[kSlots][3], g[kSlots][3], Rq[9];
    pose_forward(T, S, t, q, tau, GRAD ? axes : nullptr, Ys, Xf, Rq);
    float F = 0.f;
#pragma unroll
    for (int k = 0; k < kSlots; k++) {
        int i = lane + k * kWave;
        if (i < S.l) {
            F += rho_tri(P, Xf[k][0], Xf[k][1], Xf[k][2], g[k][0], g[k][1], g[k][2]);
        } else {
            g[k][0] = g[k][1] = g[k][2] = 0.f;
        }
        if (Xout)
            for (int a = 0; a < 3; a++) Xout[k][a] = Xf[k][a];
    }
    if (pen.w > 0.f) bump_penalty<GRAD>(pen, S, Xf, g, F, xs, gs);
    F = wsum(F);
    if (!GRAD) return F;
    // translation
    for (int a = 0; a < 3; a++) gt[a] = wsum(g[0][a] + g[1][a]);
    // x x g per atom, for the quaternion and the torsions
    float xg[kSlots][3];
#pragma unroll
    for (int k = 0; k < kSlots; k++) {
        xg[k][0] = Xf[k][1] * g[k][2] - Xf[k][2] * g[k][1];
        xg[k][1] = Xf[k][2] * g[k][0] - Xf[k][0] * g[k][2];
        xg[k][2] = Xf[k][0] * g[k][1] - Xf[k][1] * g[k][0];
    }
    // quaternion: a tangent change dq of the unit quaternion (w, v) turns the
    // pose by omega = 2 (w dv - dw v + v x dv) about c0 + t, so dF = omega . tau
    // with the torque tau = sum (X - c0 - t) x g; divided by |q| for the
    // unnormalised parameter
    {
        float sx[3];
        for (int a = 0; a < 3; a++) sx[a] = wsum(xg[0][a] + xg[1][a]);
        const float ox = S.c0[0] + t[0], oy = S.c0[1] + t[1], oz = S.c0[2] + t[2];
        const float tx = sx[0] - (oy * gt[2] - oz * gt[1]);
        const float ty = sx[1] - (oz * gt[0] - ox * gt[2]);
        const float tz = sx[2] - (ox * gt[1] - oy * gt[0]);
        const float in = 1.f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const float w = q[0] * in, x = q[1] * in, y = q[2] * in, z = q[3] * in;
        gq[0] = -2.f * (tx * x + ty * y + tz * z) * in;
        gq[1] = 2.f * (w * tx + (ty * z - tz * y)) * in;
        gq[2] = 2.f * (w * ty + (tz * x - tx * z)) * in;
        gq[3] = 2.f * (w * tz + (tx * y - ty * x)) * in;
    }
    // torsions, in the final frame: K . sum over the moving atoms of
    // (x_i - A) x g_i, with the pivot A and axis K of the forward pass carried
    // into the final frame.  Per atom that is K . (x_i x g_i) - (K x A) . g_i,
    // so each lane forms its atoms' scalar terms and one wave sum per rotamer
    // finishes the job.
    wave_sync();
    for (int e = 0; e < S.nr; e++) {
        const int4 te = T.tree[S.tree0 + e];
        const float* axe = axes + 6 * te.z;
        const float d0 = axe[0] - S.c0[0], d1 = axe[1] - S.c0[1], d2 = axe[2] - S.c0[2];
        const float ax = (Rq[0] * d0 + Rq[1] * d1 + Rq[2] * d2) + S.c0[0] + t[0];
        const float ay = (Rq[3] * d0 + Rq[4] * d1 + Rq[5] * d2) + S.c0[1] + t[1];
        const float az = (Rq[6] * d0 + Rq[7] * d1 + Rq[8] * d2) + S.c0[2] + t[2];
        const float kx = Rq[0] * axe[3] + Rq[1] * axe[4] + Rq[2] * axe[5];
        const float ky = Rq[3] * axe[3] + Rq[4] * axe[4] + Rq[5] * axe[5];
        const float kz = Rq[6] * axe[3] + Rq[7] * axe[4] + Rq[8] * axe[5];
        const float cx = ky * az - kz * ay, cy = kz * ax - kx * az, cz = kx * ay - ky * ax;  // K x A
        float v = 0.f;
#pragma unroll
        for (int k = 0; k < kSlots; k++) {
            const float term = (kx * xg[k][0] + ky * xg[k][1] + kz * xg[k][2]) -
                               (cx * g[k][0] + cy * g[k][1] + cz * g[k][2]);
            v += ((S.mv[k] >> e) & 1) ? term : 0.f;
        }
        v = wsum(v);
        if (lane == 0) gtau[te.z] = v;
    }
    wave_sync();
    return F;
}

// ---------------------------------------------------------------------------

template <bool PEN>
__global__ void __launch_bounds__(256) surrogate_kernel(PocketDev P, TreeDev T, PoseDev X, int n_poses,
                                                        const float* t, const float* q, const float* tau,
                                                        int tau_stride, const float* dF, float* F_out, float* dt_out,
                                                        float* dq_out, float* dtau_out, Penalty pen_in) {
    __shared__ float tau_all[4][kMaxRot], gtau_all[4][kMaxRot], axes_all[4][6 * kMaxRot];
    __shared__ float pen_x[4][PEN ? 3 * kMaxAtoms : 1], pen_g[4][PEN ? 3 * kMaxAtoms : 1];
    const Penalty pen = PEN ? pen_in : Penalty{};
    const int wave = threadIdx.x / kWave;
    const int pose = blockIdx.x * 4 + wave;
    if (pose >= n_poses) return;
    const int lane = lane_id();
    float* tau_l = tau_all[wave];
    float* gtau = gtau_all[wave];
    PoseState S;
    load_pose(T, X, pose, S);
    const float* tp = t + 3 * (size_t)pose;
    const float* qp = q + 4 * (size_t)pose;
    for (int r = lane; r < kMaxRot; r += kWave) {
        tau_l[r] = r < S.nr ? tau[(size_t)tau_stride * pose + r] : 0.f;
        gtau[r] = 0.f;
    }
    wave_sync();
    if (!dF) {
        float F = surrogate_eval<false>(P, T, S, tp, qp, tau_l, nullptr, nullptr, nullptr, nullptr, nullptr, pen,
                                        pen_x[wave], pen_g[wave]);
        if (lane == 0) F_out[pose] = F;
        return;
    }
    float gt[3], gq[4];
    float F = surrogate_eval<true>(P, T, S, tp, qp, tau_l, axes_all[wave], gt, gq, gtau, nullptr, pen, pen_x[wave],
                                   pen_g[wave]);
    const float up = dF[pose];
    if (lane == 0) {
        if (F_out) F_out[pose] = F;
        for (int a = 0; a < 3; a++) dt_out[3 * (size_t)pose + a] = up * gt[a];
        for (int a = 0; a < 4; a++) dq_out[4 * (size_t)pose + a] = up * gq[a];
    }
    for (int r = lane; r < tau_stride; r += kWave)
        dtau_out[(size_t)tau_stride * pose + r] = r < S.nr ? up * gtau[r] : 0.f;
}

// The whole ascent of one pose in one wavefront: parameters stay in
// registers; the final pose is written to (rx, ry, rz).  PEN: the
// clash-penalised surrogate (its own instance, so that the plain one keeps its
// registers and LDS).
template <bool PEN>
__global__ void __launch_bounds__(256) refine_kernel(PocketDev P, TreeDev T, PoseDev X, int n_poses, RefineParams rp,
                                                     float* rx, float* ry, float* rz, float* F_out) {
    __shared__ float tau_all[4][kMaxRot], gtau_all[4][kMaxRot], axes_all[4][6 * kMaxRot];
    __shared__ float pen_x[4][PEN ? 3 * kMaxAtoms : 1], pen_g[4][PEN ? 3 * kMaxAtoms : 1];
    const int wave = threadIdx.x / kWave;
    const int pose = blockIdx.x * 4 + wave;
    if (pose >= n_poses) return;
    const int lane = lane_id();
    float* tau = tau_all[wave];
    float* gtau = gtau_all[wave];
    PoseState S;
    load_pose(T, X, pose, S);
    const Penalty pen = PEN ? Penalty{rp.clash_weight, rp.cd2, rp.efar, rp.far_off, rp.n_far} : Penalty{};
    float t[3] = {0.f, 0.f, 0.f}, q[4] = {1.f, 0.f, 0.f, 0.f};
    float gt[3], gq[4];
    for (int r = lane; r < kMaxRot; r += kWave) tau[r] = gtau[r] = 0.f;
    wave_sync();
    for (int s = 0; s < rp.steps; s++) {
        surrogate_eval<true>(P, T, S, t, q, tau, axes_all[wave], gt, gq, gtau, nullptr, pen, pen_x[wave],
                             pen_g[wave]);
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
        for (int r = lane; r < S.nr; r += kWave)
            tau[r] += fminf(fmaxf(rp.lr_tau * gtau[r], -rp.max_dtau), rp.max_dtau);
        wave_sync();
    }
    float Xf[kSlots][3];
    float F = surrogate_eval<false>(P, T, S, t, q, tau, nullptr, nullptr, nullptr, nullptr, Xf, pen, pen_x[wave],
                                    pen_g[wave]);
    const int off = X.pose_off[pose];
    for (int k = 0; k < kSlots; k++) {
        int i = lane_id() + k * kWave;
        if (i < S.l) {
            rx[off + i] = Xf[k][0];
            ry[off + i] = Xf[k][1];
            rz[off + i] = Xf[k][2];
        }
    }
    if (lane_id() == 0) F_out[pose] = F;
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
