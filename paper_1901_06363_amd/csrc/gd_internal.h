// Internal data layout shared by the host runtime and the HIP kernels.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/gd.h"

namespace gd {

constexpr int kWave = 64;
constexpr int kMaxAtoms = GD_MAX_ATOMS;
constexpr int kMaxRot = GD_MAX_ROT;
constexpr int kMaxSched = 360;  // longest angle schedule (1-degree steps)

// Sweep schedule of one fragment (Alg. 2): flat list {k*step} or tile peeling.
enum SchedMode : int32_t { kFlat = 0, kPeel = 1 };

struct alignas(16) RotInfo {
    int32_t a, c;             // bond atoms; a is on the left side
    int32_t pair_off;         // first straddling far pair (global index)
    int32_t n_pairs;
    int32_t mv_off[2];        // moving-atom lists of the left / right sweep
    int32_t n_mv[2];
    int32_t mode[2];          // kFlat or kPeel per side
    int32_t step[2];          // flat: step; peel: fine step hp
    int32_t tile[2];          // peel: tile size x
    int32_t off[2];           // peel: offset of the central element
    int32_t n_cand[2];        // candidates of this side per repetition
};

struct alignas(16) LigMeta {
    double cL[3];             // ligand centroid (input order sum / l)
    int32_t atom_off;         // into the SoA coordinate arrays
    int32_t l;                // atoms
    int32_t nr;               // rotamers
    int32_t rot_off;          // into RotInfo
    int32_t far_off;          // endpoint far pairs (i<j), packed i | j<<8
    int32_t n_far;
    int32_t ang_off;          // per-orientation angle records of this ligand
    int32_t pad0;
    int64_t key_off;          // first endpoint key of this ligand
    int64_t cand_per_orient;  // closed-form candidates per orientation
};

// Device view of a pocket.
struct PocketDev {
    const uint16_t* edt;      // D on the box, x fastest, then one zero sentinel cell
    int32_t n_cells;          // cells of the box (= index of the sentinel), < 2^24
    const int32_t* occ;       // occupied cells (global lattice), 3 per cell
    int32_t n_occ;
    int32_t lo[3];            // box origin (lattice index)
    int32_t dim[3];
    double h, inv_h;
    double cP[3];
    // density grid
    const float* rho;
    int32_t blo[3], bdim[3];
    float bh, inv_bh;
    // the same grid corner-packed: node (x, y, z), x in [-1, bdim0), y in
    // [-1, bdim1), z in [-1, bdim2], holds rho at (x, y), (x+1, y), (x, y+1),
    // (x+1, y+1) of layer z (0 outside the box), x fastest, so a trilinear
    // cell is two 16-byte loads
    const float4* rho4;
};

// Kernel-visible view of a prepared batch.
struct BatchDev {
    const LigMeta* lig;
    const RotInfo* rot;
    const float* x;
    const float* y;
    const float* z;
    const uint16_t* pairs;    // straddling far pairs: left atom | right atom << 8
    const uint8_t* mv;        // moving-atom lists
    const uint16_t* efar;     // whole-ligand far pairs
    const double* qmat;       // n_orient x 9 rotation matrices of the orientations
    int32_t n_lig, n_orient, reps, top_k;
    int32_t lmax, rmax;
    double cd2;               // clash distance squared (FP64, as the oracle)
    float cd2f;
    // outputs of the sweep stage
    uint64_t* keys;           // per (ligand, orientation): clash<<63 | S<<32 | orient
    uint16_t* ang;            // per (ligand, orientation): reps*nr*2 chosen angles
    // work queue of the batched form
    const int32_t* items;     // (ligand, first orientation) pairs in LPT order
    int32_t n_items, orient_per_item;
    int32_t* head;            // queue head (reset before each launch)
    unsigned long long* counters;
};

// Kernel-visible view of poses to score (CSR by pose).
struct ScoreDev {
    const int32_t* pose_lig;  // ligand of each pose
    const int32_t* pose_off;  // first coordinate row of each pose
    const int32_t* n_atoms;   // per ligand
    const int32_t* far_off;   // per ligand, into efar
    const int32_t* n_far;
    const uint16_t* efar;     // far pairs i<j, packed i | j<<8
    const float* px;
    const float* py;
    const float* pz;
};

// Torsion trees of a ligand set for the refinement (rotamers root first).
struct TreeDev {
    const int32_t* n_atoms;   // per ligand
    const int32_t* nr;        // per ligand
    const int32_t* tree_off;  // per ligand, first tree entry
    const int4* tree;         // per entry: near atom, far atom, rotamer index, 0
    const uint32_t* tmask;    // per entry: 128-bit moving-side mask (4 words)
};

// Poses and their parameters for the surrogate kernels.
struct PoseDev {
    const int32_t* pose_lig;
    const int32_t* pose_off;
    const float* px;
    const float* py;
    const float* pz;
};

struct Tiling {
    int waves_per_block = 2;
    int angle_block = 32;
    int pairs_per_lane = 4;
};

// Trig tables of integer degrees (libm, FP64, and their FP32 roundings).
void trig_tables(double* c64, double* s64, float* c32, float* s32);

}  // namespace gd

#include <hip/hip_runtime.h>

namespace gd {
// launchers (dock.hip)
hipError_t upload_trig_tables();
size_t dock_lds_bytes(int lmax, int nmax, int waves);
size_t lds_limit_per_block();
// Device copies of the pocket and batch views plus what the host needs to size a launch.
struct DockLaunch {
    const PocketDev* P;
    const BatchDev* B;
    unsigned long long* counters;
    int lmax, nmax;
};
hipError_t launch_dock(const DockLaunch& L, const Tiling& t, bool persistent, int lig, int grid, hipStream_t s);
int persistent_grid(const Tiling& t, int lmax, int nmax, int n_items);
hipError_t launch_reset(int* head, unsigned long long* counters, hipStream_t s);
hipError_t launch_topk(const BatchDev& B, gd_pose_rec* out, uint16_t* ang_out, double h, hipStream_t s);
hipError_t launch_score(const PocketDev& P, const ScoreDev& S, int n_poses, double cd2, int32_t* S_out,
                        uint8_t* clash_out, hipStream_t s);
// Allocation-free scoring: the static device scratch of GD_NOALLOC_SCRATCH_BYTES
// and its address on the current device (score.hip).
constexpr size_t kNoAllocScratch = GD_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch(void** out);
// Bump penalty of the clash-penalised surrogate: w * sum over the ligand's far
// pairs (from far_off) with d^2 < cd2 of (cd2 - d^2)^2; w = 0: none.
struct Penalty {
    float w, cd2;
    const uint16_t* efar;
    const int32_t* far_off;
    const int32_t* n_far;
};
struct RefineParams {
    int steps;
    float lr_t, lr_q, lr_tau, max_dt, max_dtau;
    // clash-penalised surrogate: F - clash_weight * sum over whole-ligand far
    // pairs with d^2 < cd2 of (cd2 - d^2)^2 (no penalty when clash_weight = 0)
    float clash_weight, cd2;
    const uint16_t* efar;    // far pairs i | j << 8, per ligand from far_off
    const int32_t* far_off;
    const int32_t* n_far;
};
hipError_t launch_surrogate(const PocketDev& P, const TreeDev& T, const PoseDev& X, int n_poses, const float* t,
                            const float* q, const float* tau, int tau_stride, const float* dF, float* F_out,
                            float* dt_out, float* dq_out, float* dtau_out, const Penalty& pen, int lmax,
                            hipStream_t s);
hipError_t launch_refine(const PocketDev& P, const TreeDev& T, const PoseDev& X, int n_poses,
                         const RefineParams& rp, float* rx, float* ry, float* rz, float* F_out, int lmax,
                         hipStream_t s);
hipError_t launch_accept(const PoseDev& X, int n_poses, const int32_t* n_atoms, const float* rx, const float* ry,
                         const float* rz, const int32_t* S_in, const int32_t* S_ref, const uint8_t* c_ref,
                         float* px, float* py, float* pz, int32_t* S_out, uint8_t* clash_out, uint8_t* accepted,
                         const uint8_t* c_in, hipStream_t s);
hipError_t launch_replay(const PocketDev& P, const BatchDev& B, const gd_pose_rec* recs, float* xyz, int nmax,
                         hipStream_t s);
hipError_t launch_profile(const PocketDev* Pd, const BatchDev& B, const gd_pose_rec* recs, int step, int32_t* S_out,
                          uint8_t* f_out, int32_t* size_out, hipStream_t s);
// continuous Eq. 1: pocket points as three FP64 planes of `pitch`, padded to
// n_pad (a multiple of kOvUnroll) with far points
constexpr int kOvUnroll = 16;
hipError_t launch_overlap(const double* pts, int n_pad, int pitch, const int32_t* pose_off, int n_poses,
                          const float* px, const float* py, const float* pz, int64_t n_atoms, double* min_out,
                          double* sum_out, double* o_out, hipStream_t s);

}  // namespace gd
