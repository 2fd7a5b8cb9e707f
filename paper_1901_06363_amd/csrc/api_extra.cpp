// C ABI: exact pose scoring and the kernel-tiling autotuner.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "gd_internal.h"
#include "runtime.h"

namespace gd {

// Validates the pose list against the topology and fills the CSR offsets.
gd_status pose_layout(const gd_ligands* topo, int32_t n_poses, const int32_t* pose_lig,
                      const std::vector<int32_t>& n_atoms, std::vector<int32_t>& lig, std::vector<int32_t>& off) {
    if (n_poses < 0) return fail(GD_ERR_ARG, "n_poses < 0");
    if (n_poses > 0 && !pose_lig) return fail(GD_ERR_ARG, "null pose_lig");
    lig.assign(pose_lig, pose_lig + n_poses);
    off.resize(n_poses);
    int64_t o = 0;
    for (int p = 0; p < n_poses; p++) {
        if (lig[p] < 0 || lig[p] >= topo->n_ligands) return fail(GD_ERR_ARG, "pose %d: ligand index out of range", p);
        off[p] = (int32_t)o;
        o += n_atoms[lig[p]];
        if (o > (int64_t)INT32_MAX) return fail(GD_ERR_CAPACITY, "more than 2^31 pose atoms");
    }
    return GD_OK;
}

gd_status score_poses(const gd_pocket* P, const gd_ligands* topo0, int32_t n_poses, const int32_t* pose_lig,
                      const float* px, const float* py, const float* pz, float clash_dist, int32_t min_bonds,
                      hipStream_t s, int32_t* S_out, uint8_t* clash_out) {
    if (!P || !topo0 || !S_out || !clash_out) return fail(GD_ERR_ARG, "gd_score_poses: null argument");
    if (n_poses > 0 && (!px || !py || !pz)) return fail(GD_ERR_ARG, "gd_score_poses: null coordinates");
    if (!(clash_dist >= 0.f) || clash_dist > 100.f) return fail(GD_ERR_ARG, "gd_score_poses: bad clash_dist");
    TopoHost T;
    gd_status st;
    HostLigands HL;
    const gd_ligands* topo = nullptr;
    if ((st = ligands_on_host(topo0, s, HL, &topo, "gd_score_poses")) != GD_OK) return st;
    if ((st = prepare_topology(topo, min_bonds, T)) != GD_OK) return st;
    std::vector<int32_t> lig, off;
    if ((st = pose_layout(topo, n_poses, pose_lig, T.n_atoms, lig, off)) != GD_OK) return st;
    if (n_poses == 0) return GD_OK;
    AsyncScratch A(s);
    ScoreDev D;
    hipError_t e;
    if ((e = A.put(lig, &D.pose_lig)) != hipSuccess || (e = A.put(off, &D.pose_off)) != hipSuccess ||
        (e = A.put(T.n_atoms, &D.n_atoms)) != hipSuccess || (e = A.put(T.far_off, &D.far_off)) != hipSuccess ||
        (e = A.put(T.n_far, &D.n_far)) != hipSuccess || (e = A.put(T.efar, &D.efar)) != hipSuccess)
        return hip_fail(e, "gd_score_poses");
    D.px = px;
    D.py = py;
    D.pz = pz;
    const double cd = (double)clash_dist;
    if ((e = launch_score(P->dev, D, n_poses, cd * cd, S_out, clash_out, s)) != hipSuccess)
        return hip_fail(e, "gd_score_poses");
    return GD_OK;
}

// The same scoring with the call's tables staged in the library's static
// device scratch (no device allocation).  The host tables are packed into one
// buffer at 16-byte aligned offsets and copied with one stream-ordered copy.
gd_status score_poses_noalloc(const gd_pocket* P, const gd_ligands* topo0, int32_t n_poses, const int32_t* pose_lig,
                              const float* px, const float* py, const float* pz, float clash_dist, int32_t min_bonds,
                              hipStream_t s, int32_t* S_out, uint8_t* clash_out) {
    const char* who = "gd_score_poses_noalloc";
    if (!P || !topo0 || !S_out || !clash_out) return fail(GD_ERR_ARG, "%s: null argument", who);
    if (n_poses > 0 && (!px || !py || !pz)) return fail(GD_ERR_ARG, "%s: null coordinates", who);
    if (!(clash_dist >= 0.f) || clash_dist > 100.f) return fail(GD_ERR_ARG, "%s: bad clash_dist", who);
    TopoHost T;
    gd_status st;
    HostLigands HL;
    const gd_ligands* topo = nullptr;
    if ((st = ligands_on_host(topo0, s, HL, &topo, who)) != GD_OK) return st;
    if ((st = prepare_topology(topo, min_bonds, T)) != GD_OK) return st;
    std::vector<int32_t> lig, off;
    if ((st = pose_layout(topo, n_poses, pose_lig, T.n_atoms, lig, off)) != GD_OK) return st;
    if (n_poses == 0) return GD_OK;
    auto al = [](size_t b) { return (b + 15) & ~(size_t)15; };
    const size_t b_lig = al(lig.size() * 4), b_off = al(off.size() * 4), b_nat = al(T.n_atoms.size() * 4),
                 b_foff = al(T.far_off.size() * 4), b_nfar = al(T.n_far.size() * 4), b_efar = al(T.efar.size() * 2);
    const size_t total = b_lig + b_off + b_nat + b_foff + b_nfar + b_efar;
    if (total > kNoAllocScratch)
        return fail(GD_ERR_CAPACITY, "%s: the call's tables take %zu bytes, the scratch holds %zu", who, total,
                    (size_t)kNoAllocScratch);
    void* base = nullptr;
    hipError_t e = noalloc_scratch(&base);
    if (e != hipSuccess) return hip_fail(e, who);
    std::vector<uint8_t> host(total, 0);
    size_t o = 0;
    auto put = [&](const void* src, size_t n, size_t span) {
        if (n) memcpy(host.data() + o, src, n);
        const size_t at = o;
        o += span;
        return (const void*)((const uint8_t*)base + at);
    };
    ScoreDev D;
    D.pose_lig = (const int32_t*)put(lig.data(), lig.size() * 4, b_lig);
    D.pose_off = (const int32_t*)put(off.data(), off.size() * 4, b_off);
    D.n_atoms = (const int32_t*)put(T.n_atoms.data(), T.n_atoms.size() * 4, b_nat);
    D.far_off = (const int32_t*)put(T.far_off.data(), T.far_off.size() * 4, b_foff);
    D.n_far = (const int32_t*)put(T.n_far.data(), T.n_far.size() * 4, b_nfar);
    D.efar = (const uint16_t*)put(T.efar.data(), T.efar.size() * 2, b_efar);
    D.px = px;
    D.py = py;
    D.pz = pz;
    if ((e = hipMemcpyAsync(base, host.data(), total, hipMemcpyHostToDevice, s)) != hipSuccess) return hip_fail(e, who);
    const double cd = (double)clash_dist;
    if ((e = launch_score(P->dev, D, n_poses, cd * cd, S_out, clash_out, s)) != hipSuccess) return hip_fail(e, who);
    return GD_OK;
}

// --------------------------------------------------------------------------
// autotuner

static std::string tune_key(const gd_pocket* P, const gd_batch* B) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    (void)hipGetDeviceProperties(&prop, dev);
    std::ostringstream k;
    int lbin = (B->dev.lmax + 31) / 32;
    k << prop.gcnArchName << "|box" << P->dev.dim[0] << "x" << P->dev.dim[1] << "x" << P->dev.dim[2] << "|n"
      << B->nmax << "|l" << lbin << "|r" << B->dev.reps;
    std::string s = k.str();
    for (char& c : s)
        if (c == ' ') c = '_';
    return s;
}

static bool cache_lookup(const char* path, const std::string& key, Tiling& t) {
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        Tiling c;
        if (is >> k >> c.waves_per_block >> c.angle_block >> c.pairs_per_lane && k == key) {
            t = c;
            found = true;
        }
    }
    return found;
}

static void cache_store(const char* path, const std::string& key, const Tiling& t) {
    if (!path) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << t.waves_per_block << " " << t.angle_block << " " << t.pairs_per_lane << "\n";
}

gd_status autotune(const gd_pocket* P, gd_batch* B, hipStream_t s, int reps, const char* cache, gd_tiling* chosen) {
    if (!P || !B) return fail(GD_ERR_ARG, "gd_batch_autotune: null argument");
    if (reps < 1) reps = 1;
    const std::string key = tune_key(P, B);
    Tiling best = B->tiling;
    if (!cache_lookup(cache, key, best)) {
        // a strided sample of the work queue keeps the LPT mix of costs; 16
        // items per resident wave, so that a run measures throughput rather
        // than the latency of its costliest item
        std::vector<int32_t> items(2 * (size_t)B->dev.n_items);
        hipError_t e = hipMemcpy(items.data(), B->dev.items, items.size() * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "gd_batch_autotune");
        int dev = 0;
        (void)hipGetDevice(&dev);
        hipDeviceProp_t prop;
        (void)hipGetDeviceProperties(&prop, dev);
        const int want = 16 * 16 * std::max(1, prop.multiProcessorCount);
        int stride = std::max(1, B->dev.n_items / want);
        std::vector<int32_t> sample;
        for (int i = 0; i < B->dev.n_items; i += stride) {
            sample.push_back(items[2 * i]);
            sample.push_back(items[2 * i + 1]);
        }
        DevBuf sb;
        if ((e = sb.upload(sample.data(), sample.size() * 4, s)) != hipSuccess) return hip_fail(e, "gd_batch_autotune");
        BatchDev D = B->dev;
        D.items = (const int32_t*)sb.ptr;
        D.n_items = (int32_t)(sample.size() / 2);
        DevBuf dcopy;
        if ((e = dcopy.upload(&D, sizeof(BatchDev), s)) != hipSuccess) return hip_fail(e, "gd_batch_autotune");
        DockLaunch L{(const PocketDev*)P->devcopy.ptr, (const BatchDev*)dcopy.ptr, D.counters, D.lmax, B->nmax};
        hipEvent_t e0, e1;
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        float best_ms = 1e30f;
        for (int w : {2, 4, 8})
            for (int nb : {8, 16, 32})
                for (int ppl : {2, 4, 8}) {
                    Tiling t;
                    t.waves_per_block = w;
                    t.angle_block = nb;
                    t.pairs_per_lane = ppl;
                    if (dock_lds_bytes(D.lmax, B->nmax, w) > lds_limit_per_block()) continue;
                    int grid = persistent_grid(t, D.lmax, B->nmax, D.n_items);
                    float tot = 0.f;
                    bool ok = true;
                    for (int r = 0; r <= reps && ok; r++) {  // first run warms up
                        ok &= launch_reset(D.head, D.counters, s) == hipSuccess;
                        (void)hipEventRecord(e0, s);
                        ok &= launch_dock(L, t, true, 0, grid, s) == hipSuccess;
                        (void)hipEventRecord(e1, s);
                        ok &= hipEventSynchronize(e1) == hipSuccess;
                        float ms = 0.f;
                        (void)hipEventElapsedTime(&ms, e0, e1);
                        if (r > 0) tot += ms;
                    }
                    if (!ok) continue;
                    if (tot < best_ms) {
                        best_ms = tot;
                        best = t;
                    }
                }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (best_ms < 1e30f) cache_store(cache, key, best);
    }
    B->tiling = best;
    if (chosen) {
        chosen->waves_per_block = best.waves_per_block;
        chosen->angle_block = best.angle_block;
        chosen->pairs_per_lane = best.pairs_per_lane;
    }
    return GD_OK;
}

}  // namespace gd

using namespace gd;

extern "C" {

gd_status gd_score_poses(const gd_pocket* pocket, const gd_ligands* topo, int32_t n_poses, const int32_t* pose_lig,
                         const float* px, const float* py, const float* pz, float clash_dist, int32_t clash_min_bonds,
                         void* stream, int32_t* S_out, uint8_t* clash_out) {
    clear_error();
    return score_poses(pocket, topo, n_poses, pose_lig, px, py, pz, clash_dist, clash_min_bonds, (hipStream_t)stream,
                       S_out, clash_out);
}

gd_status gd_score_poses_noalloc(const gd_pocket* pocket, const gd_ligands* topo, int32_t n_poses,
                                 const int32_t* pose_lig, const float* px, const float* py, const float* pz,
                                 float clash_dist, int32_t clash_min_bonds, void* stream, int32_t* S_out,
                                 uint8_t* clash_out) {
    clear_error();
    return score_poses_noalloc(pocket, topo, n_poses, pose_lig, px, py, pz, clash_dist, clash_min_bonds,
                               (hipStream_t)stream, S_out, clash_out);
}

gd_status gd_overlap_continuous(const gd_pocket* pocket, int32_t n_poses, const int32_t* pose_off, int64_t n_atoms,
                                const float* px, const float* py, const float* pz, void* stream, double* min_d2_out,
                                double* sum_out, double* overlap_out) {
    clear_error();
    if (!pocket) return fail(GD_ERR_ARG, "gd_overlap_continuous: null pocket");
    if (n_poses < 0 || n_atoms < 0) return fail(GD_ERR_ARG, "gd_overlap_continuous: negative size");
    if (n_atoms > (int64_t)INT32_MAX)
        return fail(GD_ERR_CAPACITY, "gd_overlap_continuous: more atoms than int32 offsets address");
    if (n_poses == 0) return GD_OK;
    if (!pose_off || !sum_out) return fail(GD_ERR_ARG, "gd_overlap_continuous: null pose offsets or sums");
    if (n_atoms > 0 && (!px || !py || !pz || !min_d2_out))
        return fail(GD_ERR_ARG, "gd_overlap_continuous: null coordinates or minima");
    hipError_t e = launch_overlap((const double*)pocket->pts.ptr, pocket->pts_pad, pocket->pts_pad, pose_off, n_poses,
                                  px, py, pz, n_atoms, min_d2_out, sum_out, overlap_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gd_overlap_continuous");
    return GD_OK;
}

gd_status gd_sweep_profile(const gd_pocket* pocket, const gd_batch* batch, const gd_pose_rec* recs, int32_t step,
                           void* stream, int32_t* S_out, uint8_t* feasible_out, int32_t* side_size_out) {
    clear_error();
    if (!pocket || !batch || !recs || !S_out || !feasible_out || !side_size_out)
        return fail(GD_ERR_ARG, "gd_sweep_profile: null argument");
    if (step < 1 || step > 360 || 360 % step != 0)
        return fail(GD_ERR_KNOB, "gd_sweep_profile: step must be an integer divisor of 360");
    hipError_t e = launch_profile((const PocketDev*)pocket->devcopy.ptr, batch->dev, recs, step, S_out, feasible_out,
                                  side_size_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gd_sweep_profile");
    return GD_OK;
}

gd_status gd_batch_autotune(const gd_pocket* pocket, gd_batch* batch, void* stream, int32_t reps,
                            const char* cache_path, gd_tiling* chosen) {
    clear_error();
    return autotune(pocket, batch, (hipStream_t)stream, reps, cache_path, chosen);
}

}  // extern "C"
