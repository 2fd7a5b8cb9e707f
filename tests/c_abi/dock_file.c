/*
 * Docking through the C ABI alone (no Python): reads one small input file,
 * creates the pocket, docks every ligand of the file in the batched mode and
 * prints the ranked poses.  Then docks again from device-resident ligand
 * arrays (on_device = 1) on a stream of its own, asynchronously, and reports
 * whether the ranked poses are identical.
 *
 * Input (little endian): int32 n_points, float32[3 n_points] points,
 * int32 n_ligands, int32 atom_off[n+1], float32 x, y, z[atoms],
 * int32 bond_off[n+1], int32 bonds[2 bonds], int32 rot_off[n+1],
 * int32 rot[2 rotamers], int32 n_orient, float64 quats[4 n_orient],
 * int32 hp_step, int32 top_k.
 * Output: one line per ranked pose, "ligand rank orient S clash overlap",
 * then "device-resident inputs identical <0|1>", then "poses <candidate poses scored>".
 *
 * Build: gcc -I<repo>/include -I/opt/rocm/include -D__HIP_PLATFORM_AMD__
 *        dock_file.c -L<lib dir> -lgd -L/opt/rocm/lib -lamdhip64
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "gd.h"

static void* take(FILE* f, size_t n) {
    void* p = malloc(n ? n : 1);
    if (!p || fread(p, 1, n, f) != n) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

static int32_t take_i32(FILE* f) {
    int32_t* p = (int32_t*)take(f, 4);
    int32_t v = *p;
    free(p);
    return v;
}

#define CHECK_GD(x)                                                     \
    do {                                                                \
        gd_status s_ = (x);                                             \
        if (s_ != GD_OK) {                                              \
            fprintf(stderr, "%s failed: %d %s\n", #x, (int)s_, gd_last_error()); \
            return 1;                                                   \
        }                                                               \
    } while (0)

#define CHECK_HIP(x)                                                    \
    do {                                                                \
        hipError_t e_ = (x);                                            \
        if (e_ != hipSuccess) {                                         \
            fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_)); \
            return 1;                                                   \
        }                                                               \
    } while (0)

/* a device copy of a host array (at least 4 bytes allocated); 0 on success */
static int to_device(void** dst, const void* src, size_t bytes) {
    hipError_t e = hipMalloc(dst, bytes ? bytes : 4);
    if (e == hipSuccess && bytes) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) fprintf(stderr, "device copy failed: %s\n", hipGetErrorString(e));
    return e != hipSuccess;
}

int main(int argc, char** argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s input.bin\n", argv[0]);
        return 2;
    }
    FILE* f = fopen(argv[1], "rb");
    if (!f) {
        perror("input");
        return 2;
    }
    const int32_t np = take_i32(f);
    float* pts = (float*)take(f, sizeof(float) * 3 * (size_t)np);
    const int32_t n = take_i32(f);
    int32_t* atom_off = (int32_t*)take(f, sizeof(int32_t) * (size_t)(n + 1));
    const int32_t na = atom_off[n];
    float* x = (float*)take(f, sizeof(float) * (size_t)na);
    float* y = (float*)take(f, sizeof(float) * (size_t)na);
    float* z = (float*)take(f, sizeof(float) * (size_t)na);
    int32_t* bond_off = (int32_t*)take(f, sizeof(int32_t) * (size_t)(n + 1));
    int32_t* bonds = (int32_t*)take(f, sizeof(int32_t) * 2 * (size_t)bond_off[n]);
    int32_t* rot_off = (int32_t*)take(f, sizeof(int32_t) * (size_t)(n + 1));
    int32_t* rot = (int32_t*)take(f, sizeof(int32_t) * 2 * (size_t)rot_off[n]);
    const int32_t no = take_i32(f);
    double* quats = (double*)take(f, sizeof(double) * 4 * (size_t)no);
    const int32_t hp = take_i32(f);
    const int32_t top_k = take_i32(f);
    fclose(f);

    gd_pocket_desc pd = {pts, np, 0.5f, 12.0f, 0.0f, 0.375f, 4.0f, 8.0f};
    gd_pocket* pocket = NULL;
    CHECK_GD(gd_create_pocket(&pd, NULL, &pocket));
    gd_ligands L = {n, atom_off, x, y, z, bond_off, bonds, rot_off, rot};
    gd_knobs K = {hp, hp, 0.0f, 1, 0, no, quats, top_k, 2.0f, 4};

    /* device outputs: the ranked records and the counters (angles and
       coordinates are optional and not asked for) */
    const size_t n_rec = (size_t)n * (size_t)top_k;
    gd_pose_rec* d_out = NULL;
    int64_t* d_cnt = NULL;
    CHECK_HIP(hipMalloc((void**)&d_out, sizeof(gd_pose_rec) * n_rec));
    CHECK_HIP(hipMalloc((void**)&d_cnt, sizeof(int64_t) * GD_N_COUNTERS));
    CHECK_GD(gd_dock_batch(pocket, &L, &K, GD_BATCHED, NULL, d_out, NULL, NULL, d_cnt));
    CHECK_HIP(hipDeviceSynchronize());

    gd_pose_rec* out = (gd_pose_rec*)malloc(sizeof(gd_pose_rec) * n_rec);
    int64_t cnt[GD_N_COUNTERS];
    CHECK_HIP(hipMemcpy(out, d_out, sizeof(gd_pose_rec) * n_rec, hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(cnt, d_cnt, sizeof(cnt), hipMemcpyDeviceToHost));
    for (int i = 0; i < n; i++)
        for (int k = 0; k < top_k; k++) {
            const gd_pose_rec* r = out + (size_t)i * top_k + k;
            printf("%d %d %d %d %d %.17g\n", i, k, r->orient, r->S, r->clash, r->overlap);
        }

    /* the same ligands from device memory, on a stream of its own */
    int32_t *d_atom_off, *d_bond_off, *d_bonds, *d_rot_off, *d_rot;
    float *d_x, *d_y, *d_z;
    const size_t nb = (size_t)bond_off[n], nr = (size_t)rot_off[n];
    if (to_device((void**)&d_atom_off, atom_off, sizeof(int32_t) * (size_t)(n + 1)) ||
        to_device((void**)&d_x, x, sizeof(float) * (size_t)na) || to_device((void**)&d_y, y, sizeof(float) * (size_t)na) ||
        to_device((void**)&d_z, z, sizeof(float) * (size_t)na) ||
        to_device((void**)&d_bond_off, bond_off, sizeof(int32_t) * (size_t)(n + 1)) ||
        to_device((void**)&d_bonds, bonds, sizeof(int32_t) * 2 * nb) ||
        to_device((void**)&d_rot_off, rot_off, sizeof(int32_t) * (size_t)(n + 1)) ||
        to_device((void**)&d_rot, rot, sizeof(int32_t) * 2 * nr))
        return 1;
    gd_ligands DL = {n, d_atom_off, d_x, d_y, d_z, d_bond_off, d_bonds, d_rot_off, d_rot, 1};
    hipStream_t st;
    CHECK_HIP(hipStreamCreate(&st));
    gd_pose_rec* d_out2 = NULL;
    CHECK_HIP(hipMalloc((void**)&d_out2, sizeof(gd_pose_rec) * n_rec));
    CHECK_GD(gd_dock_batch(pocket, &DL, &K, GD_BATCHED, (void*)st, d_out2, NULL, NULL, NULL));
    CHECK_HIP(hipStreamSynchronize(st));
    gd_pose_rec* out2 = (gd_pose_rec*)malloc(sizeof(gd_pose_rec) * n_rec);
    CHECK_HIP(hipMemcpy(out2, d_out2, sizeof(gd_pose_rec) * n_rec, hipMemcpyDeviceToHost));
    int same = 1;
    for (size_t r = 0; r < n_rec; r++)
        same &= out[r].orient == out2[r].orient && out[r].S == out2[r].S && out[r].clash == out2[r].clash &&
                out[r].n_atoms == out2[r].n_atoms && out[r].overlap == out2[r].overlap;
    printf("device-resident inputs identical %d\n", same);
    printf("poses %lld\n", (long long)cnt[GD_CNT_POSES]);
    (void)hipFree(d_out2);
    (void)hipFree(d_atom_off); (void)hipFree(d_x); (void)hipFree(d_y); (void)hipFree(d_z);
    (void)hipFree(d_bond_off); (void)hipFree(d_bonds); (void)hipFree(d_rot_off); (void)hipFree(d_rot);
    CHECK_HIP(hipStreamDestroy(st));
    free(out2);

    (void)hipFree(d_out);
    (void)hipFree(d_cnt);
    CHECK_GD(gd_destroy_pocket(pocket));
    free(out); free(pts); free(atom_off); free(x); free(y); free(z); free(bond_off); free(bonds); free(rot_off);
    free(rot); free(quats);
    return 0;
}
