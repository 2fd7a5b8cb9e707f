/*
 * gd.h -- C ABI of the MI355X geometric docking library (libgd.so).
 *
 * The library docks ligands into a protein pocket with the geometric method
 * of Gadioli et al., "Tunable Approximations to Control Time-to-Solution in
 * an HPC Molecular Docking Mini-App": for every ligand it enumerates rigid
 * orientations in the pocket, sweeps each rotatable bond greedily under the
 * paper's five tunable knobs (Alg. 2, Section III-C), scores every candidate
 * pose with the overlap score (Eq. 1, Section III-A) evaluated exactly on an
 * integer pocket distance grid, rejects intramolecular bumps, and reduces the
 * orientations to the best poses per ligand.  A differentiable refinement on
 * a Gaussian-blurred pocket density is provided next to the discrete search.
 *
 * Conventions for every call:
 *  - Every call returns gd_status; nothing throws across the ABI.  On a
 *    non-OK status gd_last_error() returns a thread-local message and no
 *    output has been written.  Validation happens before any device work.
 *  - Host inputs (ligands, quaternions, pocket points) are borrowed for the
 *    duration of the call only and copied to library-owned device memory.
 *  - Outputs marked "device" are caller-allocated device buffers of the
 *    documented size.  Work is enqueued on `stream` (a hipStream_t, NULL =
 *    the default stream) and the call returns without waiting unless noted.
 *  - Objects (gd_pocket, gd_batch) belong to the caller and are released with
 *    their destroy call.  A pocket is immutable after creation and may be
 *    shared read-only by concurrent calls; one gd_batch must not be used by
 *    two calls at the same time.
 *  - Lengths are in Angstrom, angles in integer degrees.
 */
#ifndef GD_H
#define GD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GD_OK = 0,
    GD_ERR_ARG = 1,      /* null pointer, negative size, bad descriptor field        */
    GD_ERR_GRAPH = 2,    /* bond index out of range, self/duplicate bond, disconnected
                            graph, more than GD_MAX_ATOMS atoms                       */
    GD_ERR_ROTAMER = 3,  /* rotamer is not a bond, not a bridge, or has a terminal end */
    GD_ERR_KNOB = 4,     /* step not an integer divisor of 360, threshold outside [0,1],
                            repetitions < 1, top_k outside [1, n_orient], bad quaternion */
    GD_ERR_OOM = 5,      /* device or host allocation failed                          */
    GD_ERR_HIP = 6,      /* HIP runtime error (message carries the HIP error string)  */
    GD_ERR_CAPACITY = 7  /* input exceeds a documented limit (grid size, counts)       */
} gd_status;

#define GD_MAX_ATOMS 128   /* atoms per ligand */
#define GD_MAX_ROT 64      /* rotatable bonds per ligand */

/* Message for the last non-OK status on the calling thread ("" if none). */
const char* gd_last_error(void);

/* ------------------------------------------------------------------------ */
/* Pocket                                                                    */

typedef struct gd_pocket gd_pocket;

typedef struct {
    const float* xyz;         /* host, n_points x 3 row-major: PASS sphere centres
                                 (Section III-A), the pocket point cloud P of Eq. 1 */
    int32_t n_points;         /* >= 1 */
    float grid_h;             /* lattice spacing h for Eq. 1, a power of two (0.5) */
    float pad;                /* margin around the points' bounding box covered by the
                                 tabulated distance grid (12.0); atoms outside it are
                                 scored exactly by a slower path                      */
    float blur_sigma;         /* Gaussian width for the refinement density; 0 = none */
    float blur_h;             /* lattice spacing of the density grid (0.375)         */
    float blur_cutoff_sigmas; /* density terms beyond this many sigma are dropped (4) */
    float blur_pad;           /* margin of the density grid (8.0)                    */
} gd_pocket_desc;

/*
 * Build the pocket on the device: the occupied cells floor(P_j / h), the exact
 * integer squared distance D(c) = min over occupied c' of |c - c'|^2 on the
 * padded box (uint16), the pocket centroid (FP64, points summed in input
 * order), and optionally the blurred density grid.  Synchronous.
 * Errors: GD_ERR_ARG (null, n_points < 1, h not a power of two, negative pad),
 * GD_ERR_CAPACITY (more than 512 cells per axis or 2^24 cells in all, or D would
 * exceed 65535; a density grid of more than 1024 nodes per axis or 2^28 in all).
 */
gd_status gd_create_pocket(const gd_pocket_desc* desc, void* stream, gd_pocket** out);
gd_status gd_destroy_pocket(gd_pocket* pocket);

typedef struct {
    int32_t box_lo[3];     /* lattice index of the first cell of the distance grid */
    int32_t box_dim[3];    /* cells per axis                                        */
    int32_t n_occupied;    /* distinct occupied cells                               */
    double centroid[3];    /* pocket centroid                                       */
    float grid_h;
    int32_t blur_lo[3];    /* density grid: first node index (node = blur_h * index) */
    int32_t blur_dim[3];   /* nodes per axis; 0 when no density grid was built      */
    float blur_h;
} gd_pocket_info;

gd_status gd_pocket_get_info(const gd_pocket* pocket, gd_pocket_info* info);
/* Copy the distance grid to host: box_dim[0]*box_dim[1]*box_dim[2] uint16, x fastest. */
gd_status gd_pocket_read_grid(const gd_pocket* pocket, uint16_t* host_out);
/* Copy the density grid to host: blur_dim[0]*blur_dim[1]*blur_dim[2] float, x fastest. */
gd_status gd_pocket_read_density(const gd_pocket* pocket, float* host_out);

/* ------------------------------------------------------------------------ */
/* Ligands and knobs                                                         */

/*
 * A ragged batch in CSR form with ligand-local atom indices: the ligand
 * database of Section III-A.  Atoms, bond graph and rotamers as in Section
 * II: a rotamer is a bond whose removal splits the ligand into two non-empty
 * fragments.  For rotamer (a,b) the "left" fragment is the side of a; the
 * list order is the sweep order.
 *
 * on_device = 0: the arrays are host memory, read during the call only.
 * on_device = 1: the arrays are device memory of the current device (for
 * instance a chunk already resident in HBM).  Validation and preparation run
 * on the host, so a call first copies the arrays to host memory on its stream,
 * after the stream's earlier work (that copy waits for it); the docking
 * kernels then read the coordinates in place: gd_dock_batch uses the
 * caller's arrays until its work on the stream has completed,
 * gd_prepare_batch copies them device to device into the batch.  Other
 * values: GD_ERR_ARG.  Zero-initialising the struct gives host arrays.
 */
typedef struct {
    int32_t n_ligands;
    const int32_t* atom_off;  /* n_ligands+1 */
    const float* x;           /* atom coordinates, structure of arrays */
    const float* y;
    const float* z;
    const int32_t* bond_off;  /* n_ligands+1 */
    const int32_t* bonds;     /* 2 per bond */
    const int32_t* rot_off;   /* n_ligands+1 */
    const int32_t* rot;       /* 2 per rotamer: (a, b) */
    int32_t on_device;        /* 0: host arrays, 1: device arrays (see above) */
} gd_ligands;

/*
 * The five knobs of Alg. 2 (Section III-C) plus the rigid orientations, the
 * size of the per-ligand result and the bump rule.
 */
typedef struct {
    int32_t hp_step_deg;       /* high-precision step, integer divisor of 360           */
    int32_t lp_step_deg;       /* low-precision step, integer divisor of 360            */
    float threshold;           /* fragments with relative size <= threshold use lp      */
    int32_t repetitions;       /* >= 1: passes over the rotamer list                    */
    int32_t enable_refinement; /* tile peeling (Eq. 2/3) for fragments above threshold  */
    int32_t n_orient;          /* rigid orientations, 1..65535                          */
    const double* quats;       /* host, n_orient x 4 unit quaternions (w,x,y,z)         */
    int32_t top_k;             /* poses kept per ligand, 1..n_orient                     */
    float clash_dist;          /* bump distance (2.0): infeasible if d < clash_dist     */
    int32_t clash_min_bonds;   /* only pairs at least this many bonds apart bump (4)    */
} gd_knobs;

/* One ranked pose of a ligand. */
typedef struct {
    int32_t orient;   /* orientation index */
    int32_t S;        /* integer overlap count: sum over atoms of D(cell(atom)) */
    int32_t clash;    /* 1 if any pair >= clash_min_bonds apart is closer than clash_dist */
    int32_t n_atoms;
    double overlap;   /* Eq. 1 on the lattice: n_atoms / (h^2 S), +inf when S = 0 */
} gd_pose_rec;

typedef enum {
    GD_PER_LIGAND = 0, /* one kernel launch per ligand                               */
    GD_BATCHED = 1     /* one persistent launch over a device work queue, captured as
                          a HIP graph and replayed on later calls                     */
} gd_mode;

/* Counters written by a docking call (device int64[GD_N_COUNTERS]). */
enum {
    GD_CNT_POSES = 0,      /* candidate poses scored (knob-determined)          */
    GD_CNT_FALLBACK = 1,   /* candidates re-evaluated in FP64 near a boundary   */
    GD_CNT_OOB = 2,        /* exact (FP64) atom lookups outside the grid box    */
    GD_CNT_SWEEPS = 3,     /* fragment sweeps performed                         */
    GD_N_COUNTERS = 4
};

/* ------------------------------------------------------------------------ */
/* Docking                                                                   */

typedef struct gd_batch gd_batch;

/*
 * Validate and prepare a ligand batch for one pocket and knob setting: bond
 * distances, fragments, the pairs each sweep must check, angle schedules and
 * the work queue order, all copied to the device.  Synchronous on `stream`.
 * Errors: GD_ERR_GRAPH, GD_ERR_ROTAMER, GD_ERR_KNOB, GD_ERR_ARG, GD_ERR_OOM.
 */
gd_status gd_prepare_batch(const gd_pocket* pocket, const gd_ligands* ligands, const gd_knobs* knobs,
                           void* stream, gd_batch** out);
gd_status gd_destroy_batch(gd_batch* batch);

typedef struct {
    int32_t n_ligands, max_atoms, max_rot, repetitions, top_k, n_orient;
    int64_t poses_expected; /* closed-form candidate count of one docking call    */
    int64_t n_pairs_total;  /* straddling far pairs summed over rotamers            */
    int64_t n_atoms_total;  /* atoms summed over ligands                            */
    double algo_flops;      /* direct-evaluation work of one docking call: per
                               candidate 24 flop per moving atom (rotation about
                               the pivot and cell index) + 8 flop per straddling
                               far pair; per endpoint 3 per atom + 8 per far pair */
    double algo_bytes;      /* distance-grid bytes gathered: 2 per atom lookup    */
} gd_batch_info;
gd_status gd_batch_get_info(const gd_batch* batch, gd_batch_info* info);

/*
 * Kernel timing: when enabled, every docking call of the batch brackets its
 * docking kernel with a pair of HIP events on the call's stream (kept in a
 * ring of the last 256 calls).  gd_batch_read_timing waits for the recorded
 * events and writes up to max_n durations in milliseconds, oldest first,
 * returning their number in *n_out; reading clears the ring.
 */
gd_status gd_batch_enable_timing(gd_batch* batch, int32_t enable);
gd_status gd_batch_read_timing(gd_batch* batch, float* ms_out, int32_t max_n, int32_t* n_out);

/*
 * Dock a prepared batch (Alg. 2 per orientation, then top-k per ligand).
 * Outputs (device, caller-allocated):
 *   out       n_ligands * top_k gd_pose_rec, rank order (clash, S, orient) ascending
 *   angles    n_ligands * top_k * repetitions * max_rot * 2 uint16 (chosen angle of
 *             each fragment sweep: [rep][rotamer][left,right]); may be NULL
 *   pose_xyz  n_ligands * top_k * max_atoms * 3 float (final pose, atom-major xyz;
 *             rows beyond a ligand's atom count are zero); may be NULL
 *   counters  GD_N_COUNTERS int64, overwritten; may be NULL
 * Asynchronous on `stream`.
 */
gd_status gd_dock_prepared(const gd_pocket* pocket, gd_batch* batch, gd_mode mode, void* stream,
                           gd_pose_rec* out, uint16_t* angles, float* pose_xyz, int64_t* counters);

/*
 * Prepare and dock a batch in one call (Alg. 2 per orientation, then top-k
 * per ligand), outputs as for gd_dock_prepared.  When every given output is
 * device memory the call is asynchronous on `stream`: it validates and
 * prepares on the host, enqueues the upload of the batch tables (from pinned
 * staging buffers the library keeps for reuse), the docking kernels and the
 * outputs, and returns; the batch tables live in a stream-ordered allocation
 * freed on the stream after the last kernel.  Host inputs may be reused when
 * the call returns; device inputs (on_device) and the outputs belong to the
 * stream's work until it completes.  When any output is host memory the
 * results go through device scratch and the call returns after they have
 * been copied to the host (synchronous).  Errors as gd_prepare_batch and
 * gd_dock_prepared, reported before any device work.
 */
gd_status gd_dock_batch(const gd_pocket* pocket, const gd_ligands* ligands, const gd_knobs* knobs, gd_mode mode,
                        void* stream, gd_pose_rec* out, uint16_t* angles, float* pose_xyz, int64_t* counters);

/*
 * Kernel tiling of the docking kernel.  waves_per_block: 1,2,4,8; angle_block:
 * candidate poses scored side by side per wavefront pass (8, 16, 32);
 * pairs_per_lane: straddling pairs each lane holds while sweeping the
 * angles (1, 2, 4, 8).  Results do not depend on the tiling.
 */
typedef struct {
    int32_t waves_per_block, angle_block, pairs_per_lane;
} gd_tiling;
gd_status gd_batch_set_tiling(gd_batch* batch, const gd_tiling* tiling);
gd_status gd_batch_get_tiling(const gd_batch* batch, gd_tiling* tiling);
/*
 * Time every tiling on a sample of the batch (HIP events, `reps` runs each)
 * and keep the fastest; the choice is cached per device, pocket grid size and
 * knob setting in the file named by cache_path (may be NULL).  Synchronous.
 */
gd_status gd_batch_autotune(const gd_pocket* pocket, gd_batch* batch, void* stream, int32_t reps,
                            const char* cache_path, gd_tiling* chosen);

/* ------------------------------------------------------------------------ */
/* Exact scoring of given poses                                              */

/*
 * Score poses exactly: S = sum_i D(floor(x_i / h)) (Eq. 1 on the lattice) and
 * the whole-ligand bump flag.  Pose p belongs to ligand pose_lig[p] (host) of
 * `topo` (its bonds define the bump pairs); its coordinates are rows
 * pose_off[p] .. pose_off[p] + n_atoms-1 of px/py/pz, where pose_off is the
 * running sum of the poses' atom counts (device arrays).  Outputs device
 * int32 S_out[n_poses], uint8 clash_out[n_poses].  Asynchronous.
 */
gd_status gd_score_poses(const gd_pocket* pocket, const gd_ligands* topo, int32_t n_poses, const int32_t* pose_lig,
                         const float* px, const float* py, const float* pz, float clash_dist,
                         int32_t clash_min_bonds, void* stream, int32_t* S_out, uint8_t* clash_out);

/*
 * gd_score_poses for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation).
 * Same arguments, outputs and errors as gd_score_poses, plus
 * GD_ERR_CAPACITY when the call's tables exceed GD_NOALLOC_SCRATCH_BYTES.
 * The per-call tables (each pose's ligand and first row, the ligands' atom
 * counts and far-pair lists, about 8 bytes per pose plus 12 per ligand plus
 * 2 per far pair) are copied from host memory into a static device buffer of
 * GD_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs on
 * until the process ends; the call makes no device allocation (host-side
 * validation uses ordinary host memory).  Every call on one device uses that
 * device's buffer, which keeps the last call's contents: calls that overlap
 * on one device (several host threads, or a stream running a call while
 * another call is enqueued on a different stream) race on it and must be
 * serialised by the caller.  The copy and the scoring kernel are enqueued on
 * `stream`.
 */
#define GD_NOALLOC_SCRATCH_BYTES (16u << 20)
gd_status gd_score_poses_noalloc(const gd_pocket* pocket, const gd_ligands* topo, int32_t n_poses,
                                 const int32_t* pose_lig, const float* px, const float* py, const float* pz,
                                 float clash_dist, int32_t clash_min_bonds, void* stream, int32_t* S_out,
                                 uint8_t* clash_out);

/* ------------------------------------------------------------------------ */
/* Overlap landscapes (peak analysis)                                        */

/*
 * The overlap landscape of every rotamer side at each ranked pose of the
 * last gd_dock_prepared call on `batch` (the peak analysis of Section III-B):
 * the pose is rebuilt in FP64 from that call's stored angles, then each side
 * of each rotamer is turned about its bond from the pose by t * step degrees,
 * t = 0 .. 360/step - 1, and evaluated exactly as a sweep's FP64 path does:
 * the whole-ligand S (Eq. 1 on the lattice) and the feasibility of the
 * straddling far pairs (strict d < clash_dist).
 *   recs           device, the n_ligands * top_k records that call wrote
 *   S_out          device int32[n_ligands * top_k * max_rot * 2 * (360/step)],
 *                  index ((pose * max_rot + r) * 2 + side) * (360/step) + t
 *   feasible_out   device uint8, same layout (1 = feasible)
 *   side_size_out  device int32[n_ligands * top_k * max_rot * 2]: atoms of
 *                  the turned side (its bond atom included)
 * Rotamers beyond a ligand's own count, and records whose orientation or
 * stored angles are out of range (the batch was never docked), give zeros.
 * The pocket must be the one the batch was docked against.  Asynchronous.
 * Errors: GD_ERR_ARG (null argument), GD_ERR_KNOB (step not an integer
 * divisor of 360), GD_ERR_HIP.
 */
gd_status gd_sweep_profile(const gd_pocket* pocket, const gd_batch* batch, const gd_pose_rec* recs, int32_t step,
                           void* stream, int32_t* S_out, uint8_t* feasible_out, int32_t* side_size_out);

/* ------------------------------------------------------------------------ */
/* Continuous overlap (Eq. 1 without the lattice)                            */

/*
 * Eq. 1 (Section III-A) on the pocket's raw points: for every atom the
 * smallest squared distance to any of the points given to gd_create_pocket,
 * then for every pose the sum over its atoms in index order and the overlap
 * o = l / sum.  FP64 throughout: coordinates are the FP32 inputs widened, one
 * pair's squared distance is fma(dz, dz, fma(dy, dy, dx * dx)).  Brute force
 * over all points, O(l p) per pose, like the paper's overlap measure.
 *   pose_off     device int32[n_poses + 1]: pose p owns atom rows
 *                pose_off[p] .. pose_off[p + 1] - 1; must start at 0, not
 *                decrease and end at n_atoms (not checked: a device array;
 *                offsets outside [0, n_atoms] are clamped, never read past)
 *   px, py, pz   device float[n_atoms], the poses' atoms in that order
 *   min_d2_out   device double[n_atoms]: per-atom minima (A^2); also the
 *                input of the per-pose sums, so it is required
 *   sum_out      device double[n_poses]: sum of the pose's minima
 *   overlap_out  device double[n_poses] or NULL: l / sum (+inf when the sum
 *                is 0, NaN for an empty pose)
 * Caller-owned buffers; nothing is allocated.  Asynchronous on `stream`.
 * Errors: GD_ERR_ARG (null pocket, negative sizes, null arrays when there is
 * work), GD_ERR_CAPACITY (n_atoms > 2^31 - 1, beyond int32 offsets),
 * GD_ERR_HIP (launch failure).
 * n_poses = 0 is a no-op.
 */
gd_status gd_overlap_continuous(const gd_pocket* pocket, int32_t n_poses, const int32_t* pose_off, int64_t n_atoms,
                                const float* px, const float* py, const float* pz, void* stream,
                                double* min_d2_out, double* sum_out, double* overlap_out);

/* ------------------------------------------------------------------------ */
/* Differentiable refinement on the blurred density                          */

/*
 * The surrogate F(t, q, tau) = sum_i rho~(X_i) where rho~ is the trilinear
 * interpolation of rho(g) = sum_j exp(-|g - P_j|^2 / (2 sigma^2)) (cutoff) on
 * the density lattice, and X = R(q/|q|) (FK_tau(X0) - c0) + c0 + t: X0 is the
 * pose being refined, c0 its centroid, FK_tau rotates, root (atom 0) first,
 * the side of every rotamer not containing atom 0 by tau_b about its current
 * axis.  Parameters per pose: t[3], q[4], tau[max_rot] (device float arrays,
 * rows of n_poses).  X0 as in gd_score_poses.
 */
typedef struct {
    int32_t steps;      /* ascent steps (50)                                      */
    float lr_t;         /* translation step per unit gradient (A per unit)        */
    float lr_q;         /* quaternion step                                        */
    float lr_tau;       /* torsion step (radians per unit gradient)               */
    float max_dt;       /* cap on |delta t| per step (A)                          */
    float max_dtau;     /* cap on |delta tau_b| per step (radians)                */
    float* kernel_ms;   /* host, may be NULL: when set, gd_refine times the ascent
                           kernel with HIP events on `stream`, waits for it and
                           stores its duration (ms) here                          */
    float clash_weight; /* >= 0; 0 = the plain surrogate.  Otherwise the ascent
                           climbs F - clash_weight * sum over the ligand's pairs
                           at least clash_min_bonds apart with d < clash_dist of
                           (clash_dist^2 - d^2)^2 (a bump penalty, beyond the
                           paper); F_out is then that penalised value         */
} gd_refine_opts;

/*
 * Optional bump penalty of the surrogate (an extension beyond the paper):
 * F - weight * sum over the ligand's atom pairs at least clash_min_bonds bonds
 * apart with d < clash_dist of (clash_dist^2 - d^2)^2.  NULL or weight 0: the
 * plain surrogate.  Errors: GD_ERR_ARG for a negative or non-finite weight or
 * a clash_dist outside [0, 100].
 */
typedef struct {
    float weight;
    float clash_dist;
    int32_t clash_min_bonds;
} gd_bump_penalty;

gd_status gd_surrogate_fwd(const gd_pocket* pocket, const gd_ligands* topo, int32_t n_poses, const int32_t* pose_lig,
                           const float* px, const float* py, const float* pz, const float* t, const float* q,
                           const float* tau, int32_t tau_stride, const gd_bump_penalty* penalty, void* stream,
                           float* F_out);
gd_status gd_surrogate_bwd(const gd_pocket* pocket, const gd_ligands* topo, int32_t n_poses, const int32_t* pose_lig,
                           const float* px, const float* py, const float* pz, const float* t, const float* q,
                           const float* tau, int32_t tau_stride, const gd_bump_penalty* penalty, const float* dF,
                           void* stream, float* dt_out, float* dq_out, float* dtau_out);

/*
 * Refine poses by `steps` ascent steps on F, then rate each refined pose with
 * the exact discrete score: accepted iff bump-free and S_refined < S_input.
 * px/py/pz are updated in place with the refined pose where accepted (the
 * input pose is kept otherwise).  Outputs (device): F_out[n_poses] surrogate
 * of the final iterate, S_out/clash_out of the returned pose, accepted_out,
 * and optionally (rx_out, ry_out, rz_out, may be NULL) the final iterate of
 * every pose in the layout of px/py/pz.
 */
gd_status gd_refine(const gd_pocket* pocket, const gd_ligands* topo, int32_t n_poses, const int32_t* pose_lig,
                    float* px, float* py, float* pz, const gd_refine_opts* opts, float clash_dist,
                    int32_t clash_min_bonds, void* stream, float* F_out, int32_t* S_out, uint8_t* clash_out,
                    uint8_t* accepted_out, float* rx_out, float* ry_out, float* rz_out);

#ifdef __cplusplus
}
#endif
#endif /* GD_H */
