// The plan: everything derived once from a problem's geometry (grid, sphere
// maps, kinetic factors, twiddles, D-block tables) plus the work space the
// kernels use. Built by plan.cpp, read by every module.
#pragma once

#include <cstdint>
#include <memory>
#include <vector>

#include "common.hpp"

namespace apw {

// Per-k device tables for the sphere <-> grid maps.
//
// The local term works plane by plane: plane s holds the sphere points whose
// first Miller index is m1 = m1min + s. For plane s:
//   points  [pt_off[s], pt_off[s+1])  with  pt_g   = index in the k's sphere order,
//                                           pt_pos = LDS slot perm2(i2) * N3 + perm3(i3)
//   rows    [row_off[s], row_off[s+1]) with row_list = slot row perm2(i2) of every z column
// where i = m mod N and perm is the digit-permuted slot of the LDS transform.
struct KTables {
    int npw = 0;
    int64_t pw_off = 0;          // sum of npw over the previous k-points
    const int *pt_off = nullptr;
    const int *pt_g = nullptr;
    const int *pt_pos = nullptr;
    const int *row_off = nullptr;
    const int *row_list = nullptr;
    const double *kin = nullptr;   // |k+G|^2 in sphere order
    const float *kin32 = nullptr;
};

// The same tables as device-resident descriptors, one per k-point, so a single
// launch can cover several k-points.
struct KDesc {
    const int *pt_off;
    const int *pt_g;
    const int *pt_pos;
    const int *row_off;
    const int *row_list;
    const double *kin;
    int64_t pw_off;
    int npw;
    int pad;
};

struct DeviceBuffer {
    void *ptr = nullptr;
    size_t bytes = 0;
    ~DeviceBuffer();
    int ensure(size_t n);   // grow (never shrink); contents are not preserved
    template <typename T> T *as() const { return static_cast<T *>(ptr); }
};

struct Plan {
    ~Plan();   // waits for the device before its buffers are freed
    // geometry
    double lattice[9];
    double recip[9];
    int N1 = 0, N2 = 0, N3 = 0;
    int64_t N = 0;
    int nslab = 0, m1min = 0;
    int max_rows = 0;              // most z-column rows in any plane of any k-point
    int nk = 0;
    std::vector<int> npw;
    std::vector<int64_t> pw_off;   // [nk+1]
    int64_t npw_total = 0;
    int max_npw = 0;
    std::vector<KTables> k;
    int nproj = 0, natom = 0;
    std::vector<int> proj_atom_offset;

    // device tables
    DeviceBuffer tables;          // all int/double geometry tables, one allocation
    DeviceBuffer kdesc_buf;       // KDesc[nk]
    const KDesc *kdesc = nullptr;
    const int *row_to_slab = nullptr;     // [N1]: slab index of LDS row perm1(i1), or -1
    const void *tw64[3] = {nullptr, nullptr, nullptr};   // per axis, cx<double>[N_i]
    const void *tw32[3] = {nullptr, nullptr, nullptr};   // per axis, cx<float>[N_i]
    // D application: for projector i, its atom block [blk_lo[i], blk_lo[i]+blk_n[i]) and
    // the offset of that block in dmat.
    const int *proj_blk_lo = nullptr;
    const int *proj_blk_n = nullptr;
    const int *proj_blk_doff = nullptr;
    int64_t dmat_len = 0;

    // reduced-precision copies of operator data (refreshed unless STATIC)
    DeviceBuffer vloc32;
    DeviceBuffer beta32;      // complex64 beta
    DeviceBuffer betabf;      // packed bf16 beta per k, rows padded to bf16_ld(npw_k)
    DeviceBuffer betabfT;     // packed bf16 beta transposed per k: [npw_k][bf16_ld(nproj)]
    DeviceBuffer psibf;       // packed bf16 psi of one k-point (MIXED_BF16 projection)
    DeviceBuffer qbf;         // packed bf16 Q = D P of one band batch (MIXED_BF16 accumulation)
    const void *vloc32_src = nullptr, *beta32_src = nullptr, *betabf_src = nullptr;

    // work space
    DeviceBuffer slab;        // [band_batch][nslab][N2][N3] complex
    DeviceBuffer slab2;       // second slab (adjoint: planes of dY)
    DeviceBuffer gemm_part;   // split-K partial sums
    DeviceBuffer proj;        // P = B^H psi  [nb][nproj] complex128 (or complex64)
    DeviceBuffer projq;       // Q = D P
    DeviceBuffer proj2;       // second projection (backward)
    DeviceBuffer projq2;
    DeviceBuffer gradv_part;  // band-group partial sums of grad V
    DeviceBuffer tmp_io;      // precision staging
    DeviceBuffer cheb[3];     // Chebyshev recurrence: two polynomial terms and H applied to one
    DeviceBuffer force_tab;   // nonlocal force: (k+G) [npw_total][3] float64, then atom offsets [natom+1]
    bool force_tab_ready = false;
    DeviceBuffer force_stack; // [4 nproj][npw_k] complex128: beta, (k+G)_x beta, (k+G)_y beta, (k+G)_z beta
};

// Global tuning knobs (abacus_pw_set_tuning); 0 selects the library default.
extern int g_band_batch;    // bands per local-term batch
extern int g_splitk_chunk;  // K chunk of the split-K projection GEMM
extern int g_yz_bands;      // bands per y-z plane work-group
extern int g_x_bands;       // bands per x-pass work-group
extern int g_yz_mode;       // plane kernels: 0 auto, 1 full plane in LDS, 2 compact rows
extern int g_overlap;       // projector GEMMs beside the local term: 0 default (off), 1 on, 2 off
extern int g_yz_threads;    // threads per work-group of the compact-row plane kernels: 0 default, 256 or 1024

// Looks up or builds the plan for a problem (validates it on build; the
// operator checks read V and D on `st`, after the caller's earlier work on it).
// The caller holds the returned reference for the duration of its call, so a
// plan evicted by another thread meanwhile stays alive until then.
int get_plan(const abacus_pw_problem *p, hipStream_t st, std::shared_ptr<Plan> &out);

// Host-side checks of a problem that do not need a plan.
int validate_problem_shallow(const abacus_pw_problem *p);

}  // namespace apw
