// Host-side objects behind the opaque handles of gd.h.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "gd_internal.h"

namespace gd {

// Owned device allocation.
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf();
    void reset();
    hipError_t alloc(size_t n);
    hipError_t upload(const void* src, size_t n, hipStream_t s);  // synchronous
};

struct GraphKey {
    const void* pocket;
    const void* out;
    const void* angles;
    const void* xyz;
    const void* counters;
    int w, nb, ppl;
    bool operator==(const GraphKey& o) const {
        return pocket == o.pocket && out == o.out && angles == o.angles && xyz == o.xyz && counters == o.counters &&
               w == o.w && nb == o.nb && ppl == o.ppl;
    }
};

gd_status fail(gd_status st, const char* fmt, ...);
gd_status hip_fail(hipError_t e, const char* where);
void clear_error();
const char* last_error();
int tile_size(int hp);
bool tiling_supported(int waves_per_block, int angle_block, int pairs_per_lane);

// Host topology of a ligand set for scoring: atom counts and far pairs.
struct TopoHost {
    std::vector<int32_t> n_atoms, far_off, n_far;
    std::vector<uint16_t> efar;
};
gd_status prepare_topology(const gd_ligands* L, int min_bonds, TopoHost& T);

// Host torsion trees for the refinement: per ligand the rotamers root first.
struct TreeHost {
    std::vector<int32_t> n_atoms, nr, tree_off;
    std::vector<int32_t> tree;   // 4 per entry: near, far, rotamer index, 0
    std::vector<uint32_t> mask;  // 4 words per entry
};
gd_status prepare_tree(const gd_ligands* L, TreeHost& out);
gd_status validate_ligands_struct(const gd_ligands* L);

// Host view of a ligand descriptor.  Host arrays (on_device = 0) are used as
// they are; device arrays are copied to host vectors on `s` (after the
// stream's earlier work) for the host-side validation and preparation.
struct HostLigands {
    gd_ligands view{};
    std::vector<int32_t> atom_off, bond_off, bonds, rot_off, rot;
    std::vector<float> x, y, z;
};
gd_status ligands_on_host(const gd_ligands* L, hipStream_t s, HostLigands& H, const gd_ligands** out,
                          const char* who);
// True when p is device (or managed) memory of the HIP runtime.
bool is_device_ptr(const void* p);

// Copy n bytes of host memory to device memory on s through one of the
// library's pinned staging buffers: the call returns once the bytes are in the
// staging buffer, without waiting for earlier work on s (a copy from pageable
// memory would).
hipError_t upload_async(void* dev, const void* host, size_t n, hipStream_t s);

// Stream-ordered device copies of small host arrays, released after the call.
struct AsyncScratch {
    hipStream_t s;
    std::vector<void*> ptrs;
    explicit AsyncScratch(hipStream_t st) : s(st) {}
    ~AsyncScratch() {
        for (void* p : ptrs) (void)hipFreeAsync(p, s);
    }
    template <class T>
    hipError_t put(const std::vector<T>& v, const T** out) {
        void* p = nullptr;
        size_t n = std::max<size_t>(v.size() * sizeof(T), 16);
        hipError_t e = hipMallocAsync(&p, n, s);
        if (e != hipSuccess) return e;
        ptrs.push_back(p);
        if (!v.empty()) {
            e = upload_async(p, v.data(), v.size() * sizeof(T), s);
            if (e != hipSuccess) return e;
        }
        *out = (const T*)p;
        return hipSuccess;
    }
    hipError_t scratch(size_t bytes, void** out) {
        hipError_t e = hipMallocAsync(out, std::max<size_t>(bytes, 16), s);
        if (e == hipSuccess) ptrs.push_back(*out);
        return e;
    }
};

gd_status pose_layout(const gd_ligands* topo, int32_t n_poses, const int32_t* pose_lig,
                      const std::vector<int32_t>& n_atoms, std::vector<int32_t>& lig, std::vector<int32_t>& off);

}  // namespace gd

struct gd_pocket {
    gd::PocketDev dev{};
    gd::DevBuf edt, occ, rho, rho4, devcopy;
    gd::DevBuf pts;          // FP64 planes x, y, z of the raw points (continuous Eq. 1)
    int n_points = 0, pts_pad = 0;
    double centroid[3] = {0, 0, 0};
    double blur_h = 0;
};

struct gd_batch {
    gd::BatchDev dev{};
    gd::DevBuf lig, rot, x, y, z, pairs, mv, efar, qmat, items, keys, ang, head, counters, devcopy;
    gd_batch_info info{};
    gd::Tiling tiling;
    int nmax = 1;
    double h = 0.5;
    hipGraphExec_t graph_dock = nullptr;   // queue reset + docking kernel
    hipGraphExec_t graph_post = nullptr;   // top-k + pose replay
    gd::GraphKey graph_key{};
    static constexpr int kRing = 256;
    bool timing = false;
    hipEvent_t ev0[kRing] = {}, ev1[kRing] = {};
    int ring_head = 0, ring_count = 0;
    ~gd_batch();
};
