// C ABI of the density-surrogate refinement: forward, backward and the fused
// ascent with exact rescoring and acceptance.
#include <hip/hip_runtime.h>
#include <math.h>

#include <vector>

#include "gd_internal.h"
#include "runtime.h"

namespace gd {

// Validated device views shared by the three calls.
struct SurrogateCall {
    TreeHost tree;
    std::vector<int32_t> lig, off;
    TreeDev T{};
    PoseDev X{};
    int lmax = 0, rmax = 0;
};

static gd_status setup(const gd_pocket* P, const gd_ligands* topo, int32_t n_poses, const int32_t* pose_lig,
                       const float* px, const float* py, const float* pz, AsyncScratch& A, SurrogateCall& C,
                       const char* who) {
    if (!P || !topo) return fail(GD_ERR_ARG, "%s: null argument", who);
    if (!P->dev.rho) return fail(GD_ERR_ARG, "%s: the pocket was created without a density grid (blur_sigma = 0)", who);
    if (n_poses > 0 && (!px || !py || !pz)) return fail(GD_ERR_ARG, "%s: null coordinates", who);
    gd_status st;
    if ((st = prepare_tree(topo, C.tree)) != GD_OK) return st;
    if ((st = pose_layout(topo, n_poses, pose_lig, C.tree.n_atoms, C.lig, C.off)) != GD_OK) return st;
    for (int p = 0; p < n_poses; p++) {
        C.lmax = std::max(C.lmax, C.tree.n_atoms[C.lig[p]]);
        C.rmax = std::max(C.rmax, C.tree.nr[C.lig[p]]);
    }
    if (n_poses == 0) return GD_OK;
    hipError_t e;
    const int32_t* tree_ptr = nullptr;
    if ((e = A.put(C.tree.n_atoms, &C.T.n_atoms)) != hipSuccess || (e = A.put(C.tree.nr, &C.T.nr)) != hipSuccess ||
        (e = A.put(C.tree.tree_off, &C.T.tree_off)) != hipSuccess || (e = A.put(C.tree.tree, &tree_ptr)) != hipSuccess ||
        (e = A.put(C.tree.mask, &C.T.tmask)) != hipSuccess || (e = A.put(C.lig, &C.X.pose_lig)) != hipSuccess ||
        (e = A.put(C.off, &C.X.pose_off)) != hipSuccess)
        return hip_fail(e, who);
    C.T.tree = (const int4*)tree_ptr;
    C.X.px = px;
    C.X.py = py;
    C.X.pz = pz;
    return GD_OK;
}

gd_status surrogate(const gd_pocket* P, const gd_ligands* topo0, int32_t n_poses, const int32_t* pose_lig,
                    const float* px, const float* py, const float* pz, const float* t, const float* q,
                    const float* tau, int32_t tau_stride, const gd_bump_penalty* pb, const float* dF, hipStream_t s,
                    float* F_out, float* dt_out, float* dq_out, float* dtau_out, const char* who) {
    if (n_poses > 0 && (!t || !q || (!tau && tau_stride > 0))) return fail(GD_ERR_ARG, "%s: null parameters", who);
    if (dF ? (!dt_out || !dq_out || (tau_stride > 0 && !dtau_out)) : !F_out)
        return fail(GD_ERR_ARG, "%s: null output", who);
    HostLigands HL;
    const gd_ligands* topo = nullptr;
    gd_status st = ligands_on_host(topo0, s, HL, &topo, who);
    if (st != GD_OK) return st;
    AsyncScratch A(s);
    SurrogateCall C;
    st = setup(P, topo, n_poses, pose_lig, px, py, pz, A, C, who);
    if (st != GD_OK) return st;
    if (tau_stride < C.rmax) return fail(GD_ERR_ARG, "%s: tau_stride %d < rotamers %d", who, tau_stride, C.rmax);
    Penalty pen{};
    TopoHost TH;
    if (pb && pb->weight != 0.f) {
        if (!(pb->weight > 0.f) || !std::isfinite(pb->weight) || !(pb->clash_dist >= 0.f) || pb->clash_dist > 100.f)
            return fail(GD_ERR_ARG, "%s: bad bump penalty", who);
        if ((st = prepare_topology(topo, pb->clash_min_bonds, TH)) != GD_OK) return st;
        if (n_poses > 0) {
            hipError_t e;
            if ((e = A.put(TH.far_off, &pen.far_off)) != hipSuccess || (e = A.put(TH.n_far, &pen.n_far)) != hipSuccess ||
                (e = A.put(TH.efar, &pen.efar)) != hipSuccess)
                return hip_fail(e, who);
        }
        pen.w = pb->weight;
        pen.cd2 = (float)((double)pb->clash_dist * (double)pb->clash_dist);
    }
    if (n_poses == 0) return GD_OK;
    static const float zero = 0.f;
    const float* tau_ok = tau ? tau : &zero;
    hipError_t e = launch_surrogate(P->dev, C.T, C.X, n_poses, t, q, tau_ok, tau_stride, dF, F_out, dt_out, dq_out,
                                    dtau_out, pen, C.lmax, s);
    return e == hipSuccess ? GD_OK : hip_fail(e, who);
}

gd_status refine(const gd_pocket* P, const gd_ligands* topo0, int32_t n_poses, const int32_t* pose_lig, float* px,
                 float* py, float* pz, const gd_refine_opts* o, float clash_dist, int32_t min_bonds, hipStream_t s,
                 float* F_out, int32_t* S_out, uint8_t* clash_out, uint8_t* accepted_out, float* rx_out,
                 float* ry_out, float* rz_out) {
    const char* who = "gd_refine";
    if (!o || !F_out || !S_out || !clash_out || !accepted_out) return fail(GD_ERR_ARG, "%s: null argument", who);
    if (o->steps < 0 || !(o->max_dt >= 0) || !(o->max_dtau >= 0) || !std::isfinite(o->lr_t) ||
        !std::isfinite(o->lr_q) || !std::isfinite(o->lr_tau))
        return fail(GD_ERR_ARG, "%s: bad options", who);
    if (!(clash_dist >= 0.f) || clash_dist > 100.f) return fail(GD_ERR_ARG, "%s: bad clash_dist", who);
    if (!(o->clash_weight >= 0.f) || !std::isfinite(o->clash_weight))
        return fail(GD_ERR_ARG, "%s: clash_weight must be finite and >= 0", who);
    HostLigands HL;
    const gd_ligands* topo = nullptr;
    gd_status st = ligands_on_host(topo0, s, HL, &topo, who);
    if (st != GD_OK) return st;
    AsyncScratch A(s);
    SurrogateCall C;
    st = setup(P, topo, n_poses, pose_lig, px, py, pz, A, C, who);
    if (st != GD_OK) return st;
    TopoHost TH;
    if ((st = prepare_topology(topo, min_bonds, TH)) != GD_OK) return st;
    if (n_poses == 0) return GD_OK;
    size_t atoms = 0;
    for (int p = 0; p < n_poses; p++) atoms += C.tree.n_atoms[C.lig[p]];
    hipError_t e;
    ScoreDev SD{};
    void *rx = rx_out, *ry = ry_out, *rz = rz_out, *S_in, *c_in, *S_ref, *c_ref;
    if ((e = A.put(TH.n_atoms, &SD.n_atoms)) != hipSuccess || (e = A.put(TH.far_off, &SD.far_off)) != hipSuccess ||
        (e = A.put(TH.n_far, &SD.n_far)) != hipSuccess || (e = A.put(TH.efar, &SD.efar)) != hipSuccess ||
        (e = rx_out ? hipSuccess : A.scratch(atoms * 4, &rx)) != hipSuccess ||
        (e = ry_out ? hipSuccess : A.scratch(atoms * 4, &ry)) != hipSuccess ||
        (e = rz_out ? hipSuccess : A.scratch(atoms * 4, &rz)) != hipSuccess ||
        (e = A.scratch(n_poses * 4, &S_in)) != hipSuccess ||
        (e = A.scratch(n_poses, &c_in)) != hipSuccess || (e = A.scratch(n_poses * 4, &S_ref)) != hipSuccess ||
        (e = A.scratch(n_poses, &c_ref)) != hipSuccess)
        return hip_fail(e, who);
    SD.pose_lig = C.X.pose_lig;
    SD.pose_off = C.X.pose_off;
    const double cd = (double)clash_dist;
    // exact score of the input poses
    SD.px = px;
    SD.py = py;
    SD.pz = pz;
    if ((e = launch_score(P->dev, SD, n_poses, cd * cd, (int32_t*)S_in, (uint8_t*)c_in, s)) != hipSuccess)
        return hip_fail(e, who);
    RefineParams rp{o->steps, o->lr_t, o->lr_q, o->lr_tau, o->max_dt, o->max_dtau, o->clash_weight,
                    (float)(cd * cd), SD.efar, SD.far_off, SD.n_far};
    struct Events {  // optional timing of the ascent kernel
        hipEvent_t ev[2] = {nullptr, nullptr};
        ~Events() {
            for (hipEvent_t x : ev)
                if (x) (void)hipEventDestroy(x);
        }
    } T;
    if (o->kernel_ms && ((e = hipEventCreate(&T.ev[0])) != hipSuccess || (e = hipEventCreate(&T.ev[1])) != hipSuccess ||
                         (e = hipEventRecord(T.ev[0], s)) != hipSuccess))
        return hip_fail(e, who);
    e = launch_refine(P->dev, C.T, C.X, n_poses, rp, (float*)rx, (float*)ry, (float*)rz, F_out, C.lmax, s);
    if (e == hipSuccess && o->kernel_ms) e = hipEventRecord(T.ev[1], s);
    if (e != hipSuccess) return hip_fail(e, who);
    // exact score of the refined poses, then acceptance
    SD.px = (const float*)rx;
    SD.py = (const float*)ry;
    SD.pz = (const float*)rz;
    if ((e = launch_score(P->dev, SD, n_poses, cd * cd, (int32_t*)S_ref, (uint8_t*)c_ref, s)) != hipSuccess)
        return hip_fail(e, who);
    if ((e = launch_accept(C.X, n_poses, C.T.n_atoms, (const float*)rx, (const float*)ry, (const float*)rz,
                           (const int32_t*)S_in, (const int32_t*)S_ref, (const uint8_t*)c_ref, px, py, pz, S_out,
                           clash_out, accepted_out, (const uint8_t*)c_in, s)) != hipSuccess)
        return hip_fail(e, who);
    if (o->kernel_ms) {
        float ms = 0.f;
        if ((e = hipEventSynchronize(T.ev[1])) == hipSuccess) e = hipEventElapsedTime(&ms, T.ev[0], T.ev[1]);
        if (e != hipSuccess) return hip_fail(e, who);
        *o->kernel_ms = ms;
    }
    return GD_OK;
}

}  // namespace gd

using namespace gd;

extern "C" {

gd_status gd_surrogate_fwd(const gd_pocket* pocket, const gd_ligands* topo, int32_t n_poses, const int32_t* pose_lig,
                           const float* px, const float* py, const float* pz, const float* t, const float* q,
                           const float* tau, int32_t tau_stride, const gd_bump_penalty* penalty, void* stream,
                           float* F_out) {
    clear_error();
    return surrogate(pocket, topo, n_poses, pose_lig, px, py, pz, t, q, tau, tau_stride, penalty, nullptr,
                     (hipStream_t)stream, F_out, nullptr, nullptr, nullptr, "gd_surrogate_fwd");
}

gd_status gd_surrogate_bwd(const gd_pocket* pocket, const gd_ligands* topo, int32_t n_poses, const int32_t* pose_lig,
                           const float* px, const float* py, const float* pz, const float* t, const float* q,
                           const float* tau, int32_t tau_stride, const gd_bump_penalty* penalty, const float* dF,
                           void* stream, float* dt_out, float* dq_out, float* dtau_out) {
    clear_error();
    if (!dF) return fail(GD_ERR_ARG, "gd_surrogate_bwd: null dF");
    return surrogate(pocket, topo, n_poses, pose_lig, px, py, pz, t, q, tau, tau_stride, penalty, dF,
                     (hipStream_t)stream, nullptr, dt_out, dq_out, dtau_out, "gd_surrogate_bwd");
}

gd_status gd_refine(const gd_pocket* pocket, const gd_ligands* topo, int32_t n_poses, const int32_t* pose_lig,
                    float* px, float* py, float* pz, const gd_refine_opts* opts, float clash_dist,
                    int32_t clash_min_bonds, void* stream, float* F_out, int32_t* S_out, uint8_t* clash_out,
                    uint8_t* accepted_out, float* rx_out, float* ry_out, float* rz_out) {
    clear_error();
    return refine(pocket, topo, n_poses, pose_lig, px, py, pz, opts, clash_dist, clash_min_bonds, (hipStream_t)stream,
                  F_out, S_out, clash_out, accepted_out, rx_out, ry_out, rz_out);
}

}  // extern "C"
