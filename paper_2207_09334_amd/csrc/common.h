// Internal helpers shared by the host sources of the library (error reporting, sizes).
#pragma once

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdarg>
#include <string>
#include <thread>
#include <vector>

#include "cronos.h"

namespace cronos {

// Runs fn(begin, end) over [0, n) split into contiguous chunks on up to 16 host threads.
// Each chunk must write only its own outputs, so results do not depend on the thread count.
template <typename F>
void parallel_for(int64_t n, F fn, int64_t min_chunk = 1024) {
    unsigned hw = std::thread::hardware_concurrency();
    int64_t t = std::min<int64_t>(hw ? hw : 1, 16);
    t = std::min<int64_t>(t, (n + min_chunk - 1) / min_chunk);
    if (t <= 1) {
        fn((int64_t)0, n);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (n + t - 1) / t;
    for (int64_t k = 0; k < t; ++k) {
        int64_t b = k * chunk, e = std::min<int64_t>(n, b + chunk);
        if (b < e) th.emplace_back(fn, b, e);
    }
    for (auto& x : th) x.join();
}

// Sets the calling thread's last-error text and returns the status.
cronos_status fail(cronos_status st, const char* fmt, ...);
void clear_error();

// Symmetric tridiagonal eigenvalues (tridiag.cpp): T has diagonal a[0..k) and off-diagonal
// b[0..k-1) (b2 = squares).  sturm_count = eigenvalues below x; tridiag_eigenvalue = the
// index-th smallest by bisection in [lo, hi]; eigvec_last_component = |last entry| of the
// unit eigenvector for an eigenvalue approximation theta (inverse iteration).
int64_t sturm_count(const double* a, const double* b2, int64_t k, double x, double tiny);
void gershgorin(const double* a, const double* b, int64_t k, double* lo, double* hi);
double tridiag_eigenvalue(const double* a, const double* b2, int64_t k, int64_t index, double lo, double hi,
                          double tiny);
double eigvec_last_component(const double* a, const double* b, int64_t k, double theta, double tiny);

// Masses per 64-lane slice: one wavefront owns one slice, one lane per mass.
constexpr int kSlice = 64;
// Default masses per workgroup (4 wavefronts).
constexpr int kDefaultBlock = 256;
// Marker of a passive (not actuated) incidence in the 16-bit group array.
constexpr uint16_t kPassive = 0xFFFF;

// Host-side renumbering, CSR incidence list and the sliced device layout built from it.
struct Layout {
    int64_t n = 0, s = 0;
    int32_t nb = 1;
    std::vector<int64_t> body_off;      // [nb+1]
    std::vector<int32_t> perm, inv;     // new->input, input->new
    std::vector<int32_t> ends;          // [2S] new endpoints (min, max), sorted
    std::vector<int32_t> spring_perm;   // new spring -> input spring
    std::vector<int64_t> row_ptr;       // [N+1]
    std::vector<int32_t> col, sid;      // [2S]

    // sliced layout: workgroup b covers masses [b*block, (b+1)*block) and stages their
    // positions plus its halo in LDS; lane t of the workgroup owns mass b*block +
    // lane_mass[b*block + t]; slice s covers lanes [64 s, 64 s + 64).
    int32_t block = kDefaultBlock;
    int64_t nblk = 0, nslice = 0;
    std::vector<uint16_t> lane_mass;    // [nblk*block] mass (offset from the block base) each lane
                                        // owns: a block's masses sorted by decreasing degree, so
                                        // a 64-lane slice holds masses of similar degree
    std::vector<int32_t> slice_ptr;     // [nslice+1] first entry of each slice (slices = lanes)
    std::vector<uint16_t> nbr_local;    // [entries] LDS slot of the neighbour
    std::vector<int32_t> entry_csr;     // [entries] CSR position, -1 = padding
    std::vector<int32_t> halo_ptr;      // [nblk+1]
    std::vector<int32_t> halo_idx;      // halo masses of each workgroup (new indices)
    int32_t max_halo = 0;
};

// Builds everything in Layout (renumbering, CSR, slices, halos).  Validates the springs.
cronos_status build_layout(int64_t n, int32_t nb, const int64_t* body_offset, const double* x,
                           const int32_t* grid, int64_t s, const int32_t* ends, int32_t block,
                           Layout& out);
cronos_status check_layout(const Layout& lay);

}  // namespace cronos

struct cronos_layout_t {
    cronos::Layout lay;
};
