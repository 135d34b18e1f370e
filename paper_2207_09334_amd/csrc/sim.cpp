// Simulation handle: validation, renumbering, device upload, step enqueueing (plain launches
// or HIP graphs of several steps), state read-back, force evaluation and diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <unordered_map>

#include "common.h"
#include "kernels.h"

namespace cronos {

namespace {
thread_local std::string g_err;
}

cronos_status fail(cronos_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

void clear_error() { g_err.clear(); }

}  // namespace cronos

using cronos::fail;

extern "C" const char* cronos_last_error(void) { return cronos::g_err.c_str(); }
extern "C" const char* cronos_version(void) { return "cronos-gfx950 0.1"; }

namespace {

// Step graphs: for each parity of the position buffers, one HIP graph of 2^j steps for
// j < kGraphLevels (1 .. 128 steps); a call of n steps launches n's binary decomposition from
// the largest level down, so consecutive launches of a graph run without the ~8 us the device
// leaves between two graphs more than once per 128 steps.
constexpr int kGraphLevels = 8;
constexpr int kResidentSteps = 4096;  // steps per launch of the resident form

#define HIP_TRY(expr)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(CRONOS_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

}  // namespace

// Device buffers of a differentiable rollout (checkpoints, one recomputed segment, adjoints).
struct RolloutBuffers {
    int64_t n0 = 0, T = 0;
    int32_t K = 0, nseg = 0;
    bool valid = false;
    float4* ck_x = nullptr;   // [nseg][N]
    float* ck_v = nullptr;    // [nseg][3N]
    // two segment buffers: the reverse sweep of one segment runs while the next one (earlier in
    // time) is recomputed into the other, on a second stream
    float4* seg_x[2] = {nullptr, nullptr};  // [K+1][N]
    float* seg_v[2] = {nullptr, nullptr};   // [K+1][3N]
    float* seg_vs[2] = {nullptr, nullptr};  // [K][3N]
    float* seg_f[2] = {nullptr, nullptr};   // [K][n_factor + 1] actuation factors of the segment's steps
    hipStream_t side = nullptr;             // the recompute's stream (default priority)
    hipEvent_t ev[5] = {};                  // fork, recomputed[2], reversed[2]
    float* lossw = nullptr;   // [3N]
    float4* w[2] = {nullptr, nullptr};    // [N] adjoint force terms, alternating by reversed step
    float* xb[2] = {nullptr, nullptr};
    float* vb[2] = {nullptr, nullptr};
    float* xbl[2] = {nullptr, nullptr};   // [3N] x_bar before the spring sum, alternating as w
    double2* sens = nullptr;  // [entries] each actuated entry's sensitivity, summed over the reversed steps
    // the entries of each actuation group (CSR, entry order), for the per-group sums on the device
    int32_t* grp_ptr = nullptr;      // [n_factor + 1]
    int32_t* grp_entries = nullptr;  // [actuated entries]
    double2* gsum = nullptr;         // [n_factor]
    size_t cap_seg = 0, cap_ck = 0;
};

struct cronos_sim_t {
    cronos::Layout lay;
    cronos::DeviceArrays d;
    cronos::StepParams p{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int cur = 0;
    int64_t step = 0;
    int32_t nb = 1, n_groups = 0;
    double dt = 0.0, omega = 0.0;
    unsigned long long cycles = 0;       // frac(f dt) * 2^64: period fraction per step
    bool actuated = false, use_graph = true;
    double plain_step_us = 0.0;          // step time with plain launches, measured at creation
    bool verlet = false;                 // integrator of eqs. (5)-(6): first step kicks dt / 2
    bool half_kick = false;              // the next step is Verlet's first
    hipGraphExec_t graph[2][kGraphLevels] = {};   // [parity][level]: 2^level steps
    std::vector<float> inv_m;            // new order
    std::vector<uint16_t> h_grp;         // per entry factor index (actuated sims), for the adjoint reduction
    std::vector<double> h_phase, h_amp;  // actuation parameters last set
    double origin[3] = {0.0, 0.0, 0.0};  // absolute position = device position + origin
    double rest_max = 0.0;               // longest nominal rest length
    RolloutBuffers ro;
    float4* h_x = nullptr;               // pinned staging
    float* h_v = nullptr;
    float* h_f = nullptr;
    double* h_diag = nullptr;
};

namespace {

void free_device(cronos_sim_t* s) {
    cronos::DeviceArrays& d = s->d;
    void* ptrs[] = {d.narrow, d.packed, d.table, d.blk_groups, d.sp_rec, d.sp_grp, d.sp_ptr, d.x[0], d.x[1], d.v[0], d.v[1], d.mass, d.fext, d.lane_mass, d.slice_ptr, d.nbr, d.kl, d.grp, d.halo_ptr,
                    d.halo_idx, d.phase, d.amp, d.factor, d.step_ctr, d.chunks, d.body_chunk, d.chunk_part,
                    d.body_out, d.fout, d.grid_halo, d.grid_org, d.grid_k, d.grid_tab};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (auto& per : s->graph)
        for (auto& g : per)
            if (g) (void)hipGraphExecDestroy(g);
    RolloutBuffers& r = s->ro;
    for (hipEvent_t e : r.ev)
        if (e) (void)hipEventDestroy(e);
    if (r.side) (void)hipStreamDestroy(r.side);
    void* rp[] = {r.seg_f[0], r.seg_f[1], r.ck_x, r.ck_v, r.seg_x[0], r.seg_x[1], r.seg_v[0], r.seg_v[1], r.seg_vs[0],
                  r.seg_vs[1], r.lossw, r.w[0], r.w[1], r.xb[0], r.xb[1], r.vb[0], r.vb[1],
                  r.xbl[0], r.xbl[1], r.sens, r.grp_ptr, r.grp_entries, r.gsum};
    for (void* p : rp)
        if (p) (void)hipFree(p);
    if (s->h_x) (void)hipHostFree(s->h_x);
    if (s->h_v) (void)hipHostFree(s->h_v);
    if (s->h_f) (void)hipHostFree(s->h_f);
    if (s->h_diag) (void)hipHostFree(s->h_diag);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
}

template <typename T>
cronos_status upload(T** dst, const T* src, size_t count) {
    if (count == 0) count = 1;
    if (hipMalloc((void**)dst, count * sizeof(T)) != hipSuccess) return fail(CRONOS_ENOMEM, "device allocation of %zu bytes failed", count * sizeof(T));
    if (src) HIP_TRY(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
    return CRONOS_OK;
}

#define TRY(expr)                                \
    do {                                         \
        cronos_status st_ = (expr);              \
        if (st_ != CRONOS_OK) return st_;        \
    } while (0)

// Structured-box form (see step_grid_kernel): host arrays of a system that is a full grid of
// masses in aligned 8 x 8 x 8 Morton blocks with all 26 neighbour springs, passive, rest
// length fixed per direction and k fixed per (boundary class, direction).  Returns false
// (and builds nothing) when the system is not of that shape.
struct GridHost {
    int32_t dim[3] = {0, 0, 0};
    std::vector<int32_t> halo;   // [nblk][488]
    std::vector<int4> org;       // [nblk]
    std::vector<float> kcls;     // [27][26]
    std::vector<uint32_t> tab;   // [512] lane: tile cell | lx << 10 | ly << 13 | lz << 16; [488] halo slot's cell
    float kin[3] = {}, l0[3] = {};   // per direction kind: 1, 2 or 3 non-zero offsets
};

// Direction index of a neighbour offset (dx, dy, dz) in {-1, 0, 1}^3 \ 0: (dz, dy, dx)
// lexicographic, the order of the device's sum; the opposite direction is 25 - index.
inline int grid_direction(int dx, int dy, int dz) {
    const int e = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
    return e < 13 ? e : e - 1;
}

bool detect_grid(const cronos_desc& d, const cronos::Layout& L, GridHost& G) {
    constexpr int E = 8, B = E * E * E;
    if (!d.grid || L.nb != 1 || L.block != B || d.group) return false;
    const int64_t n = L.n, s = L.s;
    if (n % B) return false;
    int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], d.grid[3 * i + c]);
            hi[c] = std::max(hi[c], d.grid[3 * i + c]);
        }
    int64_t cells = 1;
    for (int c = 0; c < 3; ++c) {
        G.dim[c] = hi[c] - lo[c] + 1;
        if (G.dim[c] < E || G.dim[c] % E) return false;
        cells *= G.dim[c];
    }
    if (cells != n) return false;
    const int nx = G.dim[0], ny = G.dim[1], nz = G.dim[2];
    auto cell_of = [&](int32_t o, int c) { return d.grid[3 * (int64_t)o + c] - lo[c]; };
    // every block is an aligned cube in Morton order: local index t holds (x, y, z) from its
    // interleaved bits
    std::vector<int32_t> at((size_t)n, -1);   // grid cell -> new index
    const int64_t nblk = n / B;
    G.org.assign((size_t)nblk, make_int4(0, 0, 0, 0));
    for (int64_t b = 0; b < nblk; ++b) {
        const int32_t o0 = L.perm[b * B];
        const int x0 = cell_of(o0, 0), y0 = cell_of(o0, 1), z0 = cell_of(o0, 2);
        if (x0 % E || y0 % E || z0 % E) return false;
        G.org[b] = make_int4(x0, y0, z0, 0);
        for (int t = 0; t < B; ++t) {
            const int lx = (t & 1) | ((t >> 2) & 2) | ((t >> 4) & 4);
            const int ly = ((t >> 1) & 1) | ((t >> 3) & 2) | ((t >> 5) & 4);
            const int lz = ((t >> 2) & 1) | ((t >> 4) & 2) | ((t >> 6) & 4);
            const int32_t o = L.perm[b * B + t];
            const int x = cell_of(o, 0), y = cell_of(o, 1), z = cell_of(o, 2);
            if (x != x0 + lx || y != y0 + ly || z != z0 + lz) return false;
            int32_t& slot = at[((int64_t)z * ny + y) * nx + x];
            if (slot >= 0) return false;
            slot = (int32_t)(b * B + t);
        }
    }
    // springs: exactly the pairs of grid neighbours, each once
    int64_t expected = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx)
                if (grid_direction(dx, dy, dz) < 13 && (dx || dy || dz))
                    expected += (int64_t)(nx - std::abs(dx)) * (ny - std::abs(dy)) * (nz - std::abs(dz));
    if (s != expected) return false;
    auto cls = [&](int x, int y, int z) {
        return (x == 0 ? 0 : x == nx - 1 ? 2 : 1) + 3 * (y == 0 ? 0 : y == ny - 1 ? 2 : 1) +
               9 * (z == 0 ? 0 : z == nz - 1 ? 2 : 1);
    };
    std::vector<uint32_t> seen((size_t)n, 0u);   // per input mass: directions met
    std::vector<float> kc(27 * 26, -1.0f);
    float l0d[26];
    bool l0set[26] = {};
    auto put = [&](float& slot, float v) {
        if (slot < 0.0f) slot = v;
        return slot == v;
    };
    for (int64_t q = 0; q < s; ++q) {
        const int32_t i = d.ends[2 * q], j = d.ends[2 * q + 1];
        const int xi = cell_of(i, 0), yi = cell_of(i, 1), zi = cell_of(i, 2);
        const int xj = cell_of(j, 0), yj = cell_of(j, 1), zj = cell_of(j, 2);
        const int dx = xj - xi, dy = yj - yi, dz = zj - zi;
        if (std::abs(dx) > 1 || std::abs(dy) > 1 || std::abs(dz) > 1 || !(dx || dy || dz)) return false;
        const int di = grid_direction(dx, dy, dz), dj = 25 - di;
        if ((seen[i] >> di) & 1u) return false;
        if ((seen[j] >> dj) & 1u) return false;
        seen[i] |= 1u << di;
        seen[j] |= 1u << dj;
        const float k = (float)d.k[q], l0 = (float)d.rest[q];
        if (!put(kc[26 * cls(xi, yi, zi) + di], k) || !put(kc[26 * cls(xj, yj, zj) + dj], k)) return false;
        for (int dd : {di, dj}) {
            if (!l0set[dd]) {
                l0d[dd] = l0;
                l0set[dd] = true;
            } else if (l0d[dd] != l0) {
                return false;
            }
        }
    }
    for (int dd = 0; dd < 26; ++dd)
        if (!l0set[dd]) return false;
    for (float& k : kc)
        if (k < 0.0f) k = 0.0f;   // a direction leaving the box: no spring
    G.kcls = kc;
    // rest length, and interior k, the same for every direction of a kind
    bool kind_set[3] = {};
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!(dx || dy || dz)) continue;
                const int dd = grid_direction(dx, dy, dz), kind = (dx != 0) + (dy != 0) + (dz != 0) - 1;
                const float kin = kc[26 * 13 + dd];
                if (!kind_set[kind]) {
                    kind_set[kind] = true;
                    G.kin[kind] = kin;
                    G.l0[kind] = l0d[dd];
                } else if (G.kin[kind] != kin || G.l0[kind] != l0d[dd]) {
                    return false;
                }
            }
    // the kernel's per-lane and per-halo-slot tile cells: lane t holds the block's mass t,
    // whose local coordinates are the de-interleaved bits of t (x from bits 0, 3, 6; y from
    // 1, 4, 7; z from 2, 5, 8); halo slots in the order of the halo lists below
    auto cell_at = [](int cx, int cy, int cz) { return (uint32_t)((cz * 10 + cy) * 10 + cx); };
    G.tab.clear();
    for (int t = 0; t < 512; ++t) {
        const int lx = (t & 1) | ((t >> 2) & 2) | ((t >> 4) & 4);
        const int ly = ((t >> 1) & 1) | ((t >> 3) & 2) | ((t >> 5) & 4);
        const int lz = ((t >> 2) & 1) | ((t >> 4) & 2) | ((t >> 6) & 4);
        G.tab.push_back(cell_at(lx + 1, ly + 1, lz + 1) | (uint32_t)lx << 10 | (uint32_t)ly << 13 | (uint32_t)lz << 16);
    }
    for (int cz : {0, 9})
        for (int cy = 0; cy < 10; ++cy)
            for (int cx = 0; cx < 10; ++cx) G.tab.push_back(cell_at(cx, cy, cz));
    for (int cz = 1; cz <= 8; ++cz) {
        for (int cy : {0, 9})
            for (int cx = 0; cx < 10; ++cx) G.tab.push_back(cell_at(cx, cy, cz));
        for (int cy = 1; cy <= 8; ++cy)
            for (int cx : {0, 9}) G.tab.push_back(cell_at(cx, cy, cz));
    }
    // halo cells of every block's 10 x 10 x 10 tile, in the same enumeration
    G.halo.assign((size_t)nblk * 488, -1);
    cronos::parallel_for(nblk, [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
            int h = 0;
            auto add = [&](int cx, int cy, int cz) {
                const int x = G.org[b].x + cx - 1, y = G.org[b].y + cy - 1, z = G.org[b].z + cz - 1;
                int32_t g = -1;
                if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz) g = at[((int64_t)z * ny + y) * nx + x];
                G.halo[(size_t)b * 488 + h++] = g;
            };
            for (int cz : {0, 9})
                for (int cy = 0; cy < 10; ++cy)
                    for (int cx = 0; cx < 10; ++cx) add(cx, cy, cz);
            for (int cz = 1; cz <= 8; ++cz) {
                for (int cy : {0, 9})
                    for (int cx = 0; cx < 10; ++cx) add(cx, cy, cz);
                for (int cy = 1; cy <= 8; ++cy)
                    for (int cx : {0, 9}) add(cx, cy, cz);
            }
        }
    }, 16);
    return true;
}

// Largest natural frequency of the rest-state system (springs k n n^T plus the contact
// plane's k_g on z) among free masses.  Gershgorin first; if that bound is not conclusive,
// power iteration on M^-1/2 K M^-1/2.
double omega_max(const cronos::Layout& L, const cronos_desc& d, const std::vector<double>& xn,
                 const std::vector<double>& mn, const std::vector<uint8_t>& pin, const std::vector<double>& ks,
                 bool& conclusive_gersh, double dt) {
    const int64_t n = L.n, s = L.s;
    std::vector<double> nx(3 * s), gq(s);
    cronos::parallel_for(s, [&](int64_t q0, int64_t q1) {
        for (int64_t q = q0; q < q1; ++q) {
            int32_t a = L.ends[2 * q], b = L.ends[2 * q + 1];
            double dv[3], len2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                dv[c] = xn[3 * b + c] - xn[3 * a + c];
                len2 += dv[c] * dv[c];
            }
            double len = std::sqrt(len2);
            double l1 = 0.0, mx = 0.0;
            for (int c = 0; c < 3; ++c) {
                nx[3 * q + c] = len > 0 ? dv[c] / len : 0.0;
                l1 += std::fabs(nx[3 * q + c]);
                mx = std::max(mx, std::fabs(nx[3 * q + c]));
            }
            gq[q] = 2.0 * ks[q] * mx * l1;
        }
    }, 1 << 16);
    // row sums over each mass's incidence list (the CSR), then the largest bound
    double kg = d.ground ? d.ground_k : 0.0;
    std::vector<double> part(64, 0.0);
    const int64_t per = (n + 63) / 64;
    cronos::parallel_for(64, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c)
            for (int64_t i = c * per; i < std::min(n, (c + 1) * per); ++i) {
                if (pin[i]) continue;
                double r = 0.0;
                for (int64_t p = L.row_ptr[i]; p < L.row_ptr[i + 1]; ++p) r += gq[L.sid[p]];
                part[c] = std::max(part[c], (r + kg) / mn[i]);
            }
    }, 1);
    double gersh = 0.0;
    for (double v : part) gersh = std::max(gersh, v);
    conclusive_gersh = std::sqrt(gersh) * dt < 2.0;
    if (conclusive_gersh) return std::sqrt(gersh);
    // power iteration on B = M^-1/2 K M^-1/2 over free DOFs:
    // (B u)_i = s_i sum_q k_q n_q n_q . (s_i u_i - s_j u_j) + [z] k_g / m_i u_i,  s = m^-1/2,
    // one mass per task over its incidence list; dot products in 64 fixed chunks
    std::vector<double> u(3 * n), w(3 * n), sm(n);
    for (int64_t i = 0; i < n; ++i) sm[i] = 1.0 / std::sqrt(mn[i]);
    for (int64_t i = 0; i < 3 * n; ++i) u[i] = pin[i / 3] ? 0.0 : 1.0 + 0.37 * std::sin(0.91 * (double)i);
    auto chunked = [&](auto body) {
        std::vector<double> acc(64, 0.0);
        cronos::parallel_for(64, [&](int64_t c0, int64_t c1) {
            for (int64_t c = c0; c < c1; ++c)
                for (int64_t i = c * per; i < std::min(n, (c + 1) * per); ++i) acc[c] += body(i);
        }, 1);
        double t = 0.0;
        for (double v : acc) t += v;
        return t;
    };
    double lam = 0.0;
    for (int it = 0; it < 400; ++it) {
        double nrm = std::sqrt(chunked([&](int64_t i) {
            return u[3 * i] * u[3 * i] + u[3 * i + 1] * u[3 * i + 1] + u[3 * i + 2] * u[3 * i + 2];
        }));
        if (nrm == 0.0) break;
        for (double& v : u) v /= nrm;
        const double lam_new = chunked([&](int64_t i) {
            double wi[3] = {0.0, 0.0, 0.0};
            if (!pin[i]) {
                for (int64_t p = L.row_ptr[i]; p < L.row_ptr[i + 1]; ++p) {
                    const int64_t q = L.sid[p], j = L.col[p];
                    const double* nq = &nx[3 * q];
                    double proj = 0.0;
                    for (int c = 0; c < 3; ++c) proj += nq[c] * (sm[i] * u[3 * i + c] - sm[j] * u[3 * j + c]);
                    for (int c = 0; c < 3; ++c) wi[c] += ks[q] * proj * nq[c];
                }
                for (int c = 0; c < 3; ++c) wi[c] *= sm[i];
                wi[2] += kg / mn[i] * u[3 * i + 2];
            }
            for (int c = 0; c < 3; ++c) w[3 * i + c] = wi[c];
            return u[3 * i] * wi[0] + u[3 * i + 1] * wi[1] + u[3 * i + 2] * wi[2];  // Rayleigh quotient
        });
        if (it > 20 && std::fabs(lam_new - lam) <= 1e-7 * std::fabs(lam_new)) {
            lam = lam_new;
            break;
        }
        lam = lam_new;
        u.swap(w);
    }
    return std::sqrt(std::max(lam, 0.0));
}

// One step's launches from buffer set s->cur into the other one (s->cur is not flipped).
cronos_status enqueue_one(cronos_sim_t* s) {
    if (s->actuated && !cronos::fused_actuation(s->d))
        HIP_TRY(cronos::launch_actuation(s->d, s->cycles, 1, s->stream, -1, nullptr, s->cur));
    HIP_TRY(cronos::launch_step(s->d, s->cur, s->p, s->stream));
    return CRONOS_OK;
}

cronos_status enqueue_plain(cronos_sim_t* s, int64_t n) {
    for (int64_t k = 0; k < n; ++k) {
        TRY(enqueue_one(s));
        s->cur ^= 1;
    }
    return CRONOS_OK;
}

// Graphs or plain launches for cronos_step, and for the actuated one-lane table form whether
// velocities and the new state pass through LDS in mass order (DeviceArrays::stage_io).
//
// A graph submits its launches for a fraction of the host time that one launch per kernel
// costs, which is what a step shorter than that host time needs; but each graph launch takes
// tens of microseconds before its first kernel starts, and once the device is the slower side
// plain launches run no slower.  The step time with plain launches is measured here, on the
// simulation's stream: the launches repeat one step from the current buffers (positions,
// velocities, step counter) into the other set, which the next real step overwrites anyway,
// so the state is unchanged.  Steps of at least kPlainStepUs keep plain launches, unless
// CRONOS_GRAPH or CRONOS_NO_GRAPH decides.
//
// Staging the state through LDS turns scattered accesses into contiguous ones at the price of
// two barriers: it pays where the step streams from HBM, i.e. where the step's compulsory
// bytes exceed the 256 MiB of the MI355X's Infinity Cache (measured on random-walk
// populations: 10.5 M masses 318 -> 298 us, 2.4 M masses 76.0 -> 74.1 us, 0.45 M masses 15.9
// -> 17.0 us).  Repeating one step at a fixed parity cannot time it (the rewritten output
// buffer stays in the cache), so the rule is by size; CRONOS_STAGED_IO / CRONOS_DIRECT_IO
// decide otherwise.
constexpr double kPlainStepUs = 12.0;
constexpr double kCacheBytes = 256.0 * 1024 * 1024;
constexpr int kModeTimedSteps = 8;

// Mean time of kModeTimedSteps plain launches of one step at a fixed parity, after one untimed.
cronos_status time_plain_steps(cronos_sim_t* s, double* us) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(CRONOS_EDEVICE, "create: hipEventCreate failed");
    }
    cronos_status st = enqueue_one(s);   // untimed: first launch of each kernel
    if (st == CRONOS_OK && hipEventRecord(e0, s->stream) != hipSuccess) st = CRONOS_EDEVICE;
    for (int k = 0; k < kModeTimedSteps && st == CRONOS_OK; ++k) st = enqueue_one(s);
    if (st == CRONOS_OK && hipEventRecord(e1, s->stream) != hipSuccess) st = CRONOS_EDEVICE;
    float ms = 0.0f;
    if (st == CRONOS_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = CRONOS_EDEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == CRONOS_EDEVICE) return fail(CRONOS_EDEVICE, "create: timing the plain launches failed");
    if (st != CRONOS_OK) return st;
    *us = 1e3 * (double)ms / kModeTimedSteps;
    return CRONOS_OK;
}

cronos_status choose_launch_mode(cronos_sim_t* s, uint32_t flags) {
    if (s->d.resident) return CRONOS_OK;
    // the staged variant exists for the actuated 32-bit table form with one lane per mass
    const bool stage_form = s->actuated && s->d.packed && !s->d.narrow && !s->d.sp_rec && !s->d.grid &&
                            s->d.lanes == 1;
    if (stage_form && !(flags & CRONOS_DIRECT_IO)) {
        // compulsory bytes per step: x (float4) and v (3 floats) read and written, 4 B per entry
        const double bytes = (double)s->d.n * 56.0 + 4.0 * (double)s->lay.slice_ptr.back();
        s->d.stage_io = (flags & CRONOS_STAGED_IO) || bytes > kCacheBytes ? 1 : 0;
    }
    if (!s->use_graph || !s->stream) return CRONOS_OK;
    double t = 0.0;
    TRY(time_plain_steps(s, &t));
    s->plain_step_us = t;
    if (!(flags & CRONOS_GRAPH) && t >= kPlainStepUs) s->use_graph = false;
    return CRONOS_OK;
}

// Captures 2^level launches starting from position buffer `par` as one HIP graph (if not
// already held).  Capture only records the launches; nothing runs.
cronos_status ensure_graph(cronos_sim_t* s, int par, int level) {
    if (s->graph[par][level]) return CRONOS_OK;
    hipGraph_t g = nullptr;
    const int cur0 = s->cur;
    s->cur = par;
    HIP_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    cronos_status st = enqueue_plain(s, (int64_t)1 << level);
    hipError_t e = hipStreamEndCapture(s->stream, &g);
    s->cur = cur0;
    if (st != CRONOS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(CRONOS_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&s->graph[par][level], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        s->graph[par][level] = nullptr;
        return fail(CRONOS_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return CRONOS_OK;
}

// Every level's graph for both parities, built ahead of the first cronos_step (at creation and
// whenever the parameters they capture change), so that no step call pays for capture and
// instantiation.
cronos_status prepare_graphs(cronos_sim_t* s) {
    if (!s->use_graph || !s->stream || s->d.resident) return CRONOS_OK;
    for (int par = 0; par < 2; ++par)
        for (int level = 0; level < kGraphLevels; ++level) TRY(ensure_graph(s, par, level));
    return CRONOS_OK;
}

void drop_graphs(cronos_sim_t* s) {
    for (auto& per : s->graph)
        for (auto& g : per)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
}

// ---- autotuner cache: (arch, log2 N, log2 S, actuated, contact) -> launch configuration
std::mutex g_tune_mu;
std::map<std::string, cronos_tune> g_tune;
bool g_tune_loaded = false;

int ilog2(int64_t v) {
    int r = 0;
    while (v > 1) {
        v >>= 1;
        ++r;
    }
    return r;
}

std::string tune_key(const cronos_desc& d) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, d.device) != hipSuccess) return std::string();
    std::ostringstream k;
    std::string arch(prop.gcnArchName);
    arch = arch.substr(0, arch.find(':'));
    k << arch << "/" << ilog2(d.n_masses) << "/" << ilog2(std::max<int64_t>(d.n_springs, 1)) << "/"
      << (d.group ? 1 : 0) << "/" << (d.ground ? 1 : 0);
    return k.str();
}

void load_tune_cache_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("CRONOS_TUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string key;
    cronos_tune t{};
    while (f >> key >> t.block_masses >> t.batch >> t.persistent >> t.lanes_per_mass >> t.us_per_step >> t.us_default)
        g_tune[key] = t;
}

bool lookup_tune(const std::string& key, cronos_tune* t) {
    if (key.empty()) return false;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache_locked();
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *t = it->second;
    return true;
}

void store_tune(const std::string& key, const cronos_tune& t) {
    if (key.empty()) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_tune_cache_locked();
    g_tune[key] = t;
    if (const char* path = std::getenv("CRONOS_TUNE_CACHE")) {
        std::ofstream f(path, std::ios::app);
        f << key << " " << t.block_masses << " " << t.batch << " " << t.persistent << " " << t.lanes_per_mass << " "
          << t.us_per_step << " " << t.us_default << "\n";
    }
}

}  // namespace

extern "C" cronos_status cronos_create(const cronos_desc* d, cronos_sim* out) {
    cronos::clear_error();
    if (!d || !out) return fail(CRONOS_EINVAL, "create: NULL argument");
    *out = nullptr;
    const int64_t n = d->n_masses, s = d->n_springs;
    if (n < 1) return fail(CRONOS_EINVAL, "create: n_masses < 1");
    if (s < 0) return fail(CRONOS_EINVAL, "create: n_springs < 0");
    if (!d->x0 || !d->mass) return fail(CRONOS_EINVAL, "create: x0 and mass are required");
    if (s > 0 && (!d->ends || !d->k || !d->rest)) return fail(CRONOS_EINVAL, "create: ends, k, rest are required");
    if (!(d->dt > 0.0) || !std::isfinite(d->dt)) return fail(CRONOS_EINVAL, "create: dt must be > 0");
    if (!(d->damping >= 0.0 && d->damping < 1.0)) return fail(CRONOS_EINVAL, "create: damping must be in [0, 1)");
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(d->gravity[c])) return fail(CRONOS_EINVAL, "create: gravity not finite");
    if (d->ground && (!std::isfinite(d->ground_z) || !(d->ground_k >= 0.0) || !(d->ground_mu >= 0.0)))
        return fail(CRONOS_EINVAL, "create: bad contact plane parameters");
    for (int64_t i = 0; i < n; ++i) {
        if (!(d->mass[i] > 0.0) || !std::isfinite(d->mass[i])) return fail(CRONOS_EINVAL, "create: mass %lld not > 0", (long long)i);
        for (int c = 0; c < 3; ++c) {
            if (!std::isfinite(d->x0[3 * i + c])) return fail(CRONOS_EINVAL, "create: x0 not finite");
            if (d->v0 && !std::isfinite(d->v0[3 * i + c])) return fail(CRONOS_EINVAL, "create: v0 not finite");
            if (d->fext && !std::isfinite(d->fext[3 * i + c])) return fail(CRONOS_EINVAL, "create: fext not finite");
        }
    }
    for (int64_t q = 0; q < s; ++q) {
        if (!(d->k[q] >= 0.0) || !std::isfinite(d->k[q])) return fail(CRONOS_EINVAL, "create: k[%lld] invalid", (long long)q);
        if (!(d->rest[q] > 0.0) || !std::isfinite(d->rest[q])) return fail(CRONOS_EINVAL, "create: rest[%lld] invalid", (long long)q);
        if (d->group && (d->group[q] < -1 || d->group[q] >= d->n_groups))
            return fail(CRONOS_EINVAL, "create: group[%lld] out of range", (long long)q);
    }
    if (d->group && ((int64_t)std::max(d->n_bodies, 1) * d->n_groups >= 65535 || d->n_groups < 1))
        return fail(CRONOS_EINVAL, "create: n_bodies * n_groups must be in [1, 65535)");
    if (d->batch != 0 && d->batch != 2 && d->batch != 4 && d->batch != 8)
        return fail(CRONOS_EINVAL, "create: batch must be 0, 2, 4 or 8");
    if (d->persistent < -1 || d->persistent > 1) return fail(CRONOS_EINVAL, "create: persistent must be -1, 0 or 1");
    if (d->lanes_per_mass != 0 && d->lanes_per_mass != 1 && d->lanes_per_mass != 2 && d->lanes_per_mass != 4)
        return fail(CRONOS_EINVAL, "create: lanes_per_mass must be 0, 1, 2 or 4");

    // launch configuration: explicit values win, then a cached tuning result, then defaults
    int32_t block = d->block_masses, batch = d->batch, persistent = d->persistent, lanes = d->lanes_per_mass;
    if (block == 0 || batch == 0 || persistent == 0 || lanes == 0) {
        cronos_tune t{};
        if (d->n_masses >= 1 && lookup_tune(tune_key(*d), &t)) {
            // lanes per mass were tuned together with the workgroup size: taken only with it
            if (lanes == 0 && block == 0) lanes = t.lanes_per_mass;
            if (block == 0) block = t.block_masses;
            if (batch == 0) batch = t.batch;
            if (persistent == 0) persistent = t.persistent;
        }
    }
    // untuned default for a system too small to fill the chip with one lane per mass: 4 lanes
    // and small workgroups (the autotuner's choice on the quadruped, cubes and beams of 13k to
    // 64k masses and populations of 38k and 97k masses: 12-28% faster than 256-mass workgroups
    // with one lane; at 320k and 446k masses it keeps one lane)
    constexpr int64_t kSmallSystem = 131072;
    const uint32_t no_lanes = CRONOS_NO_TABLE | CRONOS_SPLIT | CRONOS_RESIDENT;
    if (block == 0 && lanes == 0 && n < kSmallSystem && !(d->flags & no_lanes)) {
        lanes = 4;
        block = n < 32768 ? 64 : 128;
    }
    if (batch == 0) batch = 4;
    if (persistent < 0) persistent = 0;
    if (lanes < 1) lanes = 1;
    if (lanes > 1 && block != 0 && block * lanes > 1024)
        return fail(CRONOS_EINVAL, "create: block_masses * lanes_per_mass must be at most 1024");
    if (lanes > 1 && block == 0) block = 1024 / lanes < 256 ? 1024 / lanes : 256;
    // the resident form holds the whole system in one workgroup
    if ((d->flags & CRONOS_RESIDENT) && n <= 1024 && (block == 0 || block < n))
        block = (int32_t)std::max<int64_t>(cronos::kSlice, (n + cronos::kSlice - 1) / cronos::kSlice * cronos::kSlice);
    if (block == 0) {
        // untuned default: 512-mass workgroups for a system large enough to give every CU a
        // block (measured faster on the 640k-mass cantilever, the best-candidate bar and the
        // 10.5M-mass actuated population: 294 against 298 us), else 256
        block = n >= 512 * 256 ? 512 : 256;
    }

    auto* sim = new (std::nothrow) cronos_sim_t;
    if (!sim) return fail(CRONOS_ENOMEM, "create: out of memory");
    cronos_status st;
    try {
        st = cronos::build_layout(n, std::max(d->n_bodies, 1), d->body_offset, d->x0, d->grid, s, d->ends, block,
                                  sim->lay);
    } catch (const std::bad_alloc&) {
        st = fail(CRONOS_ENOMEM, "create: out of memory");
    }
    if (st != CRONOS_OK) {
        delete sim;
        return st;
    }
    if ((d->flags & CRONOS_CHECK_LAYOUT) && (st = cronos::check_layout(sim->lay)) != CRONOS_OK) {
        delete sim;
        return st;
    }
    const cronos::Layout& L = sim->lay;
    sim->nb = L.nb;
    sim->n_groups = d->group ? d->n_groups : 0;
    sim->actuated = d->group != nullptr;
    sim->dt = d->dt;
    sim->device = d->device;
    sim->use_graph = !(d->flags & CRONOS_NO_GRAPH);
    if ((d->flags & CRONOS_NO_GRAPH) && (d->flags & CRONOS_GRAPH)) {
        delete sim;
        return fail(CRONOS_EINVAL, "create: CRONOS_GRAPH and CRONOS_NO_GRAPH together");
    }
    if ((d->flags & CRONOS_STAGED_IO) && (d->flags & CRONOS_DIRECT_IO)) {
        delete sim;
        return fail(CRONOS_EINVAL, "create: CRONOS_STAGED_IO and CRONOS_DIRECT_IO together");
    }

    // ---- host arrays in the new order
    std::vector<double> xn(3 * n), mn(n), ks(s);
    std::vector<uint8_t> pin(n);
    for (int64_t i = 0; i < n; ++i) {
        int32_t o = L.perm[i];
        for (int c = 0; c < 3; ++c) xn[3 * i + c] = d->x0[3 * o + c];
        mn[i] = d->mass[o];
        pin[i] = d->pinned ? (d->pinned[o] != 0) : 0;
    }
    for (int64_t q = 0; q < s; ++q) ks[q] = d->k[L.spring_perm[q]];
    if (!(d->flags & CRONOS_ALLOW_UNSTABLE)) {
        bool by_gersh = false;
        double w = omega_max(L, *d, xn, mn, pin, ks, by_gersh, d->dt);
        if (w * d->dt >= 2.0) {
            delete sim;
            return fail(CRONOS_EUNSTABLE, "create: largest natural frequency %.6g rad/s times dt = %.4g >= 2: "
                        "symplectic Euler diverges (set CRONOS_ALLOW_UNSTABLE to override)", w, w * d->dt);
        }
    }

    // Device coordinates: shifted so every mass starts at least `delta` (a power of two of at
    // least twice the fast-path threshold) above zero on each axis, which lets nearly every
    // wavefront take plain differences.  With the contact plane z is not shifted (the plane
    // stays at device z = ground_z): penetrations of micrometres need the fine resolution FP32
    // has near zero; wavefronts near z = 0 take exact differences in z.
    {
        double rest_max = 0.0;
        for (int64_t q = 0; q < s; ++q) rest_max = std::max(rest_max, d->rest[q]);
        sim->rest_max = rest_max;
        double delta = 1.0;
        while (delta < 8.0 * rest_max) delta *= 2.0;
        while (delta > 16.0 * rest_max && rest_max > 0.0) delta *= 0.5;
        for (int c = 0; c < 3; ++c) {
            double lo = xn[c];
            for (int64_t i = 0; i < n; ++i) lo = std::min(lo, xn[3 * i + c]);
            sim->origin[c] = ((d->ground && c == 2) || (d->flags & CRONOS_NO_SHIFT)) ? 0.0 : lo - delta;
        }
    }
    std::vector<float4> hx(n);
    std::vector<float> hv(3 * n, 0.0f), hm(n), hf;
    sim->inv_m.resize(n);
    for (int64_t i = 0; i < n; ++i) {
        int32_t o = L.perm[i];
        float im = pin[i] ? 0.0f : (float)(1.0 / mn[i]);
        sim->inv_m[i] = im;
        hx[i] = make_float4((float)(xn[3 * i] - sim->origin[0]), (float)(xn[3 * i + 1] - sim->origin[1]),
                            (float)(xn[3 * i + 2] - sim->origin[2]), im);
        if (d->v0 && !pin[i])
            for (int c = 0; c < 3; ++c) hv[3 * i + c] = (float)d->v0[3 * o + c];
        hm[i] = (float)mn[i];
    }
    if (d->fext) {
        hf.resize(3 * n);
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < 3; ++c) hf[3 * i + c] = (float)d->fext[3 * L.perm[i] + c];
    }
    const int64_t entries = L.slice_ptr.back();
    std::vector<float2> hkl(entries);
    std::vector<uint16_t> hg;
    const int32_t n_factor = sim->nb * sim->n_groups;
    if (sim->actuated) hg.assign(entries, (uint16_t)n_factor);
    std::vector<int32_t> spring_body;
    if (sim->actuated) {
        spring_body.resize(s);
        int32_t b = 0;
        for (int64_t q = 0; q < s; ++q) {
            int32_t a = L.ends[2 * q];
            while (a >= L.body_off[b + 1]) ++b;
            while (a < L.body_off[b]) --b;
            spring_body[q] = b;
        }
    }
    cronos::parallel_for(entries, [&](int64_t e0, int64_t e1) {
        for (int64_t e = e0; e < e1; ++e) {
            int32_t pos = L.entry_csr[e];
            if (pos < 0) {
                hkl[e] = make_float2(0.0f, 0.0f);
                continue;
            }
            int32_t sn = L.sid[pos], si = L.spring_perm[sn];
            hkl[e] = make_float2((float)d->k[si], (float)d->rest[si]);
            if (sim->actuated && d->group[si] >= 0) hg[e] = (uint16_t)(spring_body[sn] * sim->n_groups + d->group[si]);
        }
    }, 1 << 16);

    // compact entry stream: the distinct (k, L0) pairs (in order of first use) and one 32-bit
    // word per entry.  Actuated: LDS slot (13 bits) | pair index (9 bits) | 1 + the spring's
    // actuation factor index relative to the first one its workgroup uses (10 bits; 0 =
    // passive).  Passive: slot << 19 | pair index << 4 (byte offsets for the kernel).  Not used
    // when a field would overflow; the explicit per-entry stream then serves.
    constexpr int kSlotBits = 13, kTypeBits = 9, kGroupBits = 10;
    std::vector<float2> htable;
    std::vector<uint32_t> hpacked;
    std::vector<int2> hblk_groups;
    int32_t max_local_groups = 0;
    if (!(d->flags & CRONOS_NO_TABLE) && (L.block + L.max_halo) <= (1 << kSlotBits)) {
        const int64_t spb = L.block / cronos::kSlice;
        auto key_of = [&](int64_t e) {
            uint32_t kb, lb;
            std::memcpy(&kb, &hkl[e].x, 4);
            std::memcpy(&lb, &hkl[e].y, 4);
            return ((uint64_t)kb << 32) | lb;
        };
        // distinct pairs of each workgroup in order of first use, then numbered in workgroup
        // order: the same numbering as one sequential pass over the entries
        std::vector<std::vector<uint64_t>> firsts(L.nblk);
        std::atomic<bool> ok{true};
        if (sim->actuated) hblk_groups.assign(L.nblk, make_int2(0, 0));
        cronos::parallel_for(L.nblk, [&](int64_t b0, int64_t b1) {
            std::unordered_map<uint64_t, char> seen;
            for (int64_t b = b0; b < b1; ++b) {
                seen.clear();
                int lo = 1 << 30, hi = -1;
                for (int64_t e = L.slice_ptr[b * spb]; e < L.slice_ptr[(b + 1) * spb]; ++e) {
                    const uint64_t key = key_of(e);
                    if (seen.emplace(key, 0).second) firsts[b].push_back(key);
                    if (sim->actuated && hg[e] < n_factor) {
                        lo = std::min<int>(lo, hg[e]);
                        hi = std::max<int>(hi, hg[e]);
                    }
                }
                if (hi >= 0) {
                    hblk_groups[b] = make_int2(lo, hi - lo + 1);
                    if (hi - lo + 1 >= (1 << kGroupBits)) ok = false;
                }
            }
        }, 16);
        std::unordered_map<uint64_t, uint32_t> index;
        for (int64_t b = 0; b < L.nblk && ok; ++b) {
            for (uint64_t key : firsts[b])
                if (index.find(key) == index.end()) {
                    if ((int)htable.size() >= (1 << kTypeBits)) {
                        ok = false;
                        break;
                    }
                    index.emplace(key, (uint32_t)htable.size());
                    float2 c;
                    const uint32_t kb = (uint32_t)(key >> 32), lb = (uint32_t)key;
                    std::memcpy(&c.x, &kb, 4);
                    std::memcpy(&c.y, &lb, 4);
                    htable.push_back(c);
                }
            if (sim->actuated) max_local_groups = std::max(max_local_groups, hblk_groups[b].y);
        }
        if (ok) {
            hpacked.resize(entries);
            cronos::parallel_for(L.nblk, [&](int64_t b0, int64_t b1) {
                for (int64_t b = b0; b < b1; ++b)
                    for (int64_t e = L.slice_ptr[b * spb]; e < L.slice_ptr[(b + 1) * spb]; ++e) {
                        const uint32_t id = index.find(key_of(e))->second;
                        uint32_t lg = 0;
                        if (sim->actuated && hg[e] < n_factor) lg = (uint32_t)(hg[e] - hblk_groups[b].x + 1);
                        hpacked[e] = sim->actuated ? (uint32_t)L.nbr_local[e] | (id << kSlotBits) | (lg << (kSlotBits + kTypeBits))
                                                   : ((uint32_t)L.nbr_local[e] << 19) | (id << 4);
                    }
            }, 16);
        } else {
            htable.clear();
            hblk_groups.clear();
            max_local_groups = 0;
        }
    }

    // split form: per workgroup, one record per spring with an end among its masses (in mass
    // order, then incidence order; a spring between two of its masses is recorded by the end
    // with the lower slot) and, per entry, the neighbour slot | record index << 13; padding
    // entries point at the record count, whose factor the kernel sets to zero.  Needs the
    // compact form, first-end slots below 1024 and the factors within LDS.
    std::vector<uint32_t> hsplit, hsp_rec;
    std::vector<uint16_t> hsp_grp;
    std::vector<int32_t> hsp_ptr;
    int32_t max_sp = 0;
    if (!htable.empty() && (d->flags & CRONOS_SPLIT) && L.block <= 1024) {
        const int64_t spb = L.block / cronos::kSlice;
        auto type_of = [&](int64_t e) -> uint32_t {
            return sim->actuated ? (hpacked[e] >> kSlotBits) & ((1u << kTypeBits) - 1u) : (hpacked[e] >> 4) & ((1u << kTypeBits) - 1u);
        };
        std::vector<std::vector<uint32_t>> rec(L.nblk);
        std::vector<std::vector<uint16_t>> rgrp(sim->actuated ? L.nblk : 0);
        hsplit.resize(entries);
        std::atomic<bool> ok{true}, consistent{true};
        cronos::parallel_for(L.nblk, [&](int64_t b0, int64_t b1) {
            std::vector<int32_t> lane_of(L.block);
            std::unordered_map<int32_t, uint32_t> first;
            for (int64_t b = b0; b < b1; ++b) {
                const int64_t base = b * L.block;
                for (int l = 0; l < L.block; ++l) lane_of[L.lane_mass[base + l]] = l;
                first.clear();
                std::vector<uint32_t>& R = rec[b];
                for (int pass = 0; pass < 2; ++pass)
                    for (int m = 0; m < L.block; ++m) {
                        const int64_t i = base + m;
                        const int l = lane_of[m];
                        const int64_t sl = (base + l) / cronos::kSlice;
                        const int64_t w = (L.slice_ptr[sl + 1] - L.slice_ptr[sl]) / cronos::kSlice;
                        const int64_t deg = i < n ? L.row_ptr[i + 1] - L.row_ptr[i] : 0;
                        for (int64_t r = 0; r < w; ++r) {
                            const int64_t e = L.slice_ptr[sl] + r * cronos::kSlice + (l % cronos::kSlice);
                            const uint32_t slot = L.nbr_local[e];
                            if (r >= deg) continue;  // padding, resolved once the count is known
                            const int32_t sn = L.sid[L.entry_csr[e]];
                            const bool producer = slot >= (uint32_t)L.block || (uint32_t)m < slot;
                            if (pass == 0 && producer) {
                                const uint32_t type = type_of(e);
                                first.emplace(sn, (uint32_t)R.size());
                                R.push_back((uint32_t)m | (slot << 10) | (type << 23));
                                if (sim->actuated) rgrp[b].push_back((uint16_t)(hpacked[e] >> (kSlotBits + kTypeBits)));  // local factor
                            } else if (pass == 1) {
                                auto it = first.find(sn);
                                if (it == first.end()) {
                                    consistent = false;
                                    continue;
                                }
                                hsplit[e] = slot | (it->second << kSlotBits);
                            }
                        }
                    }
                if (R.size() >= (size_t(1) << (32 - kSlotBits))) ok = false;
                // padding entries: record count (zero factor); then every entry is checked
                // against its record: same two ends, parameter pair and actuation factor
                const uint32_t n_sp = (uint32_t)R.size();
                for (int64_t sl = base / cronos::kSlice; sl < base / cronos::kSlice + spb; ++sl)
                    for (int64_t e = L.slice_ptr[sl]; e < L.slice_ptr[sl + 1]; ++e) {
                        const uint32_t own = L.lane_mass[sl * cronos::kSlice + (e - L.slice_ptr[sl]) % cronos::kSlice];
                        const uint32_t slot = L.nbr_local[e];
                        if (L.entry_csr[e] < 0) {
                            hsplit[e] = slot | (n_sp << kSlotBits);
                            continue;
                        }
                        const uint32_t j = hsplit[e] >> kSlotBits;
                        if ((hsplit[e] & ((1u << kSlotBits) - 1u)) != slot || j >= n_sp) {
                            consistent = false;
                            continue;
                        }
                        const uint32_t ra = R[j] & 1023u, rb = (R[j] >> 10) & 8191u, rt = R[j] >> 23;
                        const bool ends = (ra == own && rb == slot) || (ra == slot && rb == own);
                        const bool type = rt == type_of(e);
                        const bool grp = !sim->actuated || rgrp[b][j] == (hpacked[e] >> (kSlotBits + kTypeBits));
                        if (!ends || !type || !grp || rb >= (uint32_t)(L.block + L.max_halo)) consistent = false;
                    }
            }
        }, 16);
        if (!consistent) {
            delete sim;
            return fail(CRONOS_EINVAL, "create: internal error: split incidence form inconsistent");
        }
        hsp_ptr.assign(L.nblk + 1, 0);
        for (int64_t b = 0; b < L.nblk; ++b) {
            hsp_ptr[b + 1] = hsp_ptr[b] + (int32_t)rec[b].size();
            max_sp = std::max<int32_t>(max_sp, (int32_t)rec[b].size());
        }
        const size_t lds = (size_t)cronos::table_base(L.block + L.max_halo) + htable.size() * sizeof(float4) +
                           (size_t)(max_local_groups + 1) * sizeof(float) + (size_t)(max_sp + 1) * sizeof(float);
        if (ok && lds <= 160 * 1024) {
            hsp_rec.reserve(hsp_ptr[L.nblk]);
            for (auto& R : rec) hsp_rec.insert(hsp_rec.end(), R.begin(), R.end());
            if (sim->actuated) {
                hsp_grp.reserve(hsp_ptr[L.nblk]);
                for (auto& G : rgrp) hsp_grp.insert(hsp_grp.end(), G.begin(), G.end());
            }
        } else {
            hsplit.clear();
            hsp_ptr.clear();
            max_sp = 0;
        }
    }

    // diagnostics chunks: workgroup blocks split at body boundaries
    std::vector<int4> chunks;
    std::vector<int32_t> body_chunk(sim->nb + 1, 0);
    {
        int32_t b = 0;
        for (int64_t blk = 0; blk < L.nblk; ++blk) {
            int64_t m0 = blk * L.block, m1 = std::min<int64_t>(n, m0 + L.block);
            while (m0 < m1) {
                while (m0 >= L.body_off[b + 1]) {
                    ++b;
                    body_chunk[b] = (int32_t)chunks.size();
                }
                int64_t e = std::min<int64_t>(m1, L.body_off[b + 1]);
                chunks.push_back(make_int4((int)blk, (int)m0, (int)e, b));
                m0 = e;
            }
        }
        for (int32_t bb = b + 1; bb <= sim->nb; ++bb) body_chunk[bb] = (int32_t)chunks.size();
    }

    // ---- structured-box form
    GridHost gridh;
    const uint32_t no_grid = CRONOS_NO_GRID | CRONOS_NO_TABLE | CRONOS_SPLIT | CRONOS_WIDE_ENTRIES | CRONOS_RESIDENT;
    const bool use_grid = lanes == 1 && !(d->flags & no_grid) && detect_grid(*d, L, gridh);

    // ---- device
    cronos::DeviceArrays& D = sim->d;
    D.n = n;
    D.block = L.block;
    D.nblk = L.nblk;
    D.nslice = L.nslice;
    D.lds_slots = L.block + L.max_halo;
    D.nb = sim->nb;
    D.batch = batch;
    D.lanes = lanes;
    D.n_factor = n_factor;
    D.n_chunks = (int32_t)chunks.size();
    if (hipSetDevice(d->device) != hipSuccess) {
        delete sim;
        return fail(CRONOS_EDEVICE, "create: hipSetDevice(%d) failed", d->device);
    }
    {
        size_t static_lds = 0;
        if (cronos::step_static_lds(&static_lds) != hipSuccess || static_lds != 0) {
            delete sim;
            return fail(CRONOS_EDEVICE, "create: step kernels must not use static LDS (%zu bytes)", static_lds);
        }
    }
    if ((size_t)D.lds_slots * sizeof(float4) > 160 * 1024) {
        delete sim;
        return fail(CRONOS_EINVAL, "create: workgroup halo needs %zu bytes of LDS", (size_t)D.lds_slots * sizeof(float4));
    }
    st = [&]() -> cronos_status {
        if (d->stream) {
            sim->stream = (hipStream_t)d->stream;
        } else {
            HIP_TRY(hipStreamCreateWithFlags(&sim->stream, hipStreamNonBlocking));
            sim->own_stream = true;
        }
        TRY(upload(&D.x[0], hx.data(), n));
        TRY(upload<float4>(&D.x[1], nullptr, n));
        TRY(upload(&D.v[0], hv.data(), 3 * n));
        TRY(upload<float>(&D.v[1], nullptr, 3 * n));
        TRY(upload(&D.mass, hm.data(), n));
        if (d->fext) TRY(upload(&D.fext, hf.data(), 3 * n));
        TRY(upload(&D.lane_mass, L.lane_mass.data(), L.lane_mass.size()));
        TRY(upload(&D.slice_ptr, L.slice_ptr.data(), L.slice_ptr.size()));
        TRY(upload(&D.nbr, L.nbr_local.data(), entries));
        TRY(upload(&D.kl, hkl.data(), entries));
        if (!hsp_rec.empty()) {
            TRY(upload(&D.packed, hsplit.data(), entries));
            TRY(upload(&D.sp_rec, hsp_rec.data(), hsp_rec.size()));
            TRY(upload(&D.sp_ptr, hsp_ptr.data(), hsp_ptr.size()));
            if (sim->actuated) TRY(upload(&D.sp_grp, hsp_grp.data(), hsp_grp.size()));
            D.max_sp = max_sp;
        }
        if (!htable.empty()) {
            // passive simulations whose LDS slots and pair indices fit in 16 bits together take
            // 16-bit entries (slot << tb | pair index): half the bytes of the entry stream
            const bool resident = (d->flags & CRONOS_RESIDENT) && L.nblk == 1 && hsp_rec.empty();
            std::vector<uint16_t> hnarrow;
            if (!sim->actuated && hsp_rec.empty() && !resident && !(d->flags & CRONOS_WIDE_ENTRIES)) {
                int sb = 1;
                while ((1 << sb) < L.block + L.max_halo) ++sb;
                const int tb = std::min(16 - sb, (int)kTypeBits);
                if (tb >= 1 && (int64_t)htable.size() <= (int64_t)1 << tb) {
                    hnarrow.resize(entries);
                    cronos::parallel_for(entries, [&](int64_t e0, int64_t e1) {
                        for (int64_t e = e0; e < e1; ++e) {
                            const uint32_t q = hpacked[e];
                            hnarrow[e] = (uint16_t)(((q >> 19) << tb) | ((q >> 4) & ((1u << kTypeBits) - 1u)));
                        }
                    });
                    D.narrow_tb = tb;
                }
            }
            if (!hnarrow.empty()) TRY(upload(&D.narrow, hnarrow.data(), entries));
            else if (hsp_rec.empty()) TRY(upload(&D.packed, hpacked.data(), entries));
            std::vector<float4> tab(htable.size());
            for (size_t q = 0; q < htable.size(); ++q) {
                // (k, L0, L0^2 exactly, as an FP64 value in the last two words)
                const float l0 = htable[q].y;
                const double sq = (double)l0 * (double)l0;
                float w[2];
                std::memcpy(w, &sq, sizeof sq);
                tab[q] = make_float4(htable[q].x, l0, w[0], w[1]);
            }
            TRY(upload(&D.table, tab.data(), tab.size()));
            D.n_table = (int32_t)htable.size();
            D.resident = (d->flags & CRONOS_RESIDENT) && L.nblk == 1 && hsp_rec.empty() ? 1 : 0;
            if (sim->actuated) TRY(upload(&D.blk_groups, hblk_groups.data(), hblk_groups.size()));
            D.max_local_groups = max_local_groups;
            if (D.resident && D.packed) {
                // the resident form keeps the entries in LDS as well when they fit beside the
                // positions, the (k, L0) table and the factors
                int dev = 0, cap = 0;
                HIP_TRY(hipGetDevice(&dev));
                HIP_TRY(hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
                if (cronos::step_lds_bytes(D) + (size_t)entries * sizeof(uint32_t) <= (size_t)cap)
                    D.resident_staged = (int32_t)entries;
            }
        }
        if (sim->actuated) TRY(upload(&D.grp, hg.data(), entries));
        TRY(upload(&D.halo_ptr, L.halo_ptr.data(), L.halo_ptr.size()));
        TRY(upload(&D.halo_idx, L.halo_idx.data(), L.halo_idx.size()));
        std::vector<float> ones(n_factor + 1, 1.0f);
        std::vector<float> zeros(std::max<int32_t>(n_factor, 1), 0.0f);
        TRY(upload(&D.factor, ones.data(), ones.size()));
        TRY(upload(&D.phase, zeros.data(), zeros.size()));
        TRY(upload(&D.amp, zeros.data(), zeros.size()));
        const long long zeros2[2] = {0, 0};
        TRY(upload(&D.step_ctr, zeros2, 2));
        TRY(upload(&D.chunks, chunks.data(), chunks.size()));
        TRY(upload(&D.body_chunk, body_chunk.data(), body_chunk.size()));
        TRY(upload<double>(&D.chunk_part, nullptr, chunks.size() * cronos::kDiagFields));
        TRY(upload<double>(&D.body_out, nullptr, (size_t)sim->nb * cronos::kDiagFields));
        TRY(upload<float>(&D.fout, nullptr, 3 * n));
        if (use_grid) {
            TRY(upload(&D.grid_halo, gridh.halo.data(), gridh.halo.size()));
            TRY(upload(&D.grid_org, gridh.org.data(), gridh.org.size()));
            TRY(upload(&D.grid_k, gridh.kcls.data(), gridh.kcls.size()));
            TRY(upload(&D.grid_tab, gridh.tab.data(), gridh.tab.size()));
            for (int c = 0; c < 3; ++c) D.grid_dim[c] = gridh.dim[c];
            for (int q = 0; q < 3; ++q) {
                D.grid_kin[q] = gridh.kin[q];
                D.grid_l0[q] = gridh.l0[q];
            }
            D.grid = 1;
        }
        HIP_TRY(hipDeviceSynchronize());
        return CRONOS_OK;
    }();
    if (st != CRONOS_OK) {
        free_device(sim);
        delete sim;
        return st;
    }
    cronos::StepParams& P = sim->p;
    P.dt = (float)d->dt;
    P.dtv = P.dt;
    sim->verlet = (d->flags & CRONOS_VERLET) != 0;
    sim->half_kick = sim->verlet;
    P.damp = (float)(1.0 - d->damping);
    P.gx = (float)d->gravity[0];
    P.gy = (float)d->gravity[1];
    P.gz = (float)d->gravity[2];
    P.ground = d->ground ? 1 : 0;
    P.ground_z = (float)(d->ground_z - sim->origin[2]);
    P.ground_k = (float)d->ground_k;
    P.ground_mu = (float)d->ground_mu;
    P.exact = (d->flags & CRONOS_FAST_DIFF) ? 0 : 1;
    P.safe = (float)(4.0 * sim->rest_max);
    P.ox = sim->origin[0];
    P.oy = sim->origin[1];
    P.oz = sim->origin[2];
    // several lanes per mass exist for the compact table forms, one workgroup per block
    if (D.lanes > 1 && (D.resident || D.sp_rec || !(D.packed || D.narrow))) D.lanes = 1;
    if (D.lanes > 1 || D.grid) persistent = 0;
    if (persistent > 0) {
        int g = 0;
        hipError_t e = cronos::persistent_grid(D, P.exact, &g);
        if (e != hipSuccess) {
            free_device(sim);
            delete sim;
            return fail(CRONOS_EDEVICE, "create: occupancy query failed: %s", hipGetErrorString(e));
        }
        D.persistent_groups = g;
    }
    if (sim->actuated) sim->h_grp = std::move(hg);
    // the Morton-order host copies are only needed at creation
    sim->lay.nbr_local.clear();
    sim->lay.nbr_local.shrink_to_fit();
    sim->lay.entry_csr.clear();
    sim->lay.entry_csr.shrink_to_fit();
    if ((st = choose_launch_mode(sim, d->flags)) != CRONOS_OK || (st = prepare_graphs(sim)) != CRONOS_OK) {
        free_device(sim);
        delete sim;
        return st;
    }
    *out = sim;
    return CRONOS_OK;
}

extern "C" void cronos_destroy(cronos_sim sim) {
    if (!sim) return;
    (void)hipSetDevice(sim->device);
    if (sim->stream) (void)hipStreamSynchronize(sim->stream);
    free_device(sim);
    delete sim;
}

extern "C" cronos_status cronos_set_actuation(cronos_sim sim, const double* phase, const double* amp, double freq_hz) {
    cronos::clear_error();
    if (!sim) return fail(CRONOS_EINVAL, "set_actuation: NULL handle");
    if (!sim->actuated) return fail(CRONOS_EINVAL, "set_actuation: simulation has no actuation groups");
    if (!phase || !amp || !std::isfinite(freq_hz)) return fail(CRONOS_EINVAL, "set_actuation: bad arguments");
    const size_t m = (size_t)sim->d.n_factor;
    for (size_t g = 0; g < m; ++g)
        if (!std::isfinite(phase[g]) || !std::isfinite(amp[g])) return fail(CRONOS_EINVAL, "set_actuation: non-finite value");
    HIP_TRY(hipSetDevice(sim->device));
    HIP_TRY(hipStreamSynchronize(sim->stream));
    std::vector<float> ph(phase, phase + m), am(amp, amp + m);
    HIP_TRY(hipMemcpy(sim->d.phase, ph.data(), m * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(sim->d.amp, am.data(), m * sizeof(float), hipMemcpyHostToDevice));
    sim->omega = 2.0 * M_PI * freq_hz;
    {
        const double c = freq_hz * sim->dt;
        sim->cycles = (unsigned long long)std::ldexp(c - std::floor(c), 64);
        sim->p.cycles = sim->cycles;   // the fused step computes its factors from it
    }
    double amax = 0.0;
    for (size_t g = 0; g < m; ++g) amax = std::max(amax, std::fabs(amp[g]));
    sim->p.safe = (float)(4.0 * sim->rest_max * (1.0 + amax));
    drop_graphs(sim);             // graphs captured the old parameters

    sim->h_phase.assign(phase, phase + m);
    sim->h_amp.assign(amp, amp + m);
    return prepare_graphs(sim);
}

extern "C" cronos_status cronos_step(cronos_sim sim, int64_t n_steps) {
    cronos::clear_error();
    if (!sim) return fail(CRONOS_EINVAL, "step: NULL handle");
    if (n_steps < 0) return fail(CRONOS_EINVAL, "step: n_steps < 0");
    HIP_TRY(hipSetDevice(sim->device));
    int64_t left = n_steps;
    if (sim->d.resident) {
        // one launch runs up to kResidentSteps steps inside a single workgroup
        float dtv0 = sim->half_kick ? 0.5f * sim->p.dt : sim->p.dtv;
        while (left > 0) {
            const int k = (int)std::min<int64_t>(left, kResidentSteps);
            HIP_TRY(cronos::launch_resident(sim->d, sim->cur, sim->p, dtv0, sim->cycles, k, sim->stream));
            sim->cur ^= 1;
            left -= k;
            dtv0 = sim->p.dtv;
        }
        if (n_steps > 0) sim->half_kick = false;
        sim->step += n_steps;
        return CRONOS_OK;
    }
    if (sim->half_kick && left > 0) {
        // Verlet's first step (eq. (5)) kicks the velocity for dt / 2; the steps after it are
        // eq. (6), which in velocity form is the same kernel with a full kick
        sim->p.dtv = 0.5f * sim->p.dt;
        const cronos_status st = enqueue_plain(sim, 1);
        sim->p.dtv = sim->p.dt;
        if (st != CRONOS_OK) return st;
        sim->half_kick = false;
        --left;
    }
    if (sim->use_graph && sim->stream) {
        while (left > 0) {
            int level = kGraphLevels - 1;
            while (((int64_t)1 << level) > left) --level;
            TRY(ensure_graph(sim, sim->cur, level));
            HIP_TRY(hipGraphLaunch(sim->graph[sim->cur][level], sim->stream));
            if (level == 0) sim->cur ^= 1;   // an odd number of steps flips the buffers
            left -= (int64_t)1 << level;
        }
    }
    TRY(enqueue_plain(sim, left));
    sim->step += n_steps;
    return CRONOS_OK;
}

extern "C" cronos_status cronos_read_state(cronos_sim sim, double* x, double* v, int64_t* step) {
    cronos::clear_error();
    if (!sim) return fail(CRONOS_EINVAL, "read_state: NULL handle");
    const int64_t n = sim->d.n;
    HIP_TRY(hipSetDevice(sim->device));
    if (!sim->h_x) HIP_TRY(hipHostMalloc((void**)&sim->h_x, n * sizeof(float4), 0));
    if (!sim->h_v) HIP_TRY(hipHostMalloc((void**)&sim->h_v, 3 * n * sizeof(float), 0));
    if (x) HIP_TRY(hipMemcpyAsync(sim->h_x, sim->d.x[sim->cur], n * sizeof(float4), hipMemcpyDeviceToHost, sim->stream));
    if (v) HIP_TRY(hipMemcpyAsync(sim->h_v, sim->d.v[sim->cur], 3 * n * sizeof(float), hipMemcpyDeviceToHost, sim->stream));
    HIP_TRY(hipStreamSynchronize(sim->stream));
    const cronos::Layout& L = sim->lay;
    for (int64_t i = 0; i < n; ++i) {
        int32_t o = L.perm[i];
        if (x) {
            x[3 * o + 0] = (double)sim->h_x[i].x + sim->origin[0];
            x[3 * o + 1] = (double)sim->h_x[i].y + sim->origin[1];
            x[3 * o + 2] = (double)sim->h_x[i].z + sim->origin[2];
        }
        if (v)
            for (int c = 0; c < 3; ++c) v[3 * o + c] = sim->h_v[3 * i + c];
    }
    if (step) *step = sim->step;
    return CRONOS_OK;
}

extern "C" cronos_status cronos_set_state(cronos_sim sim, const double* x, const double* v, int64_t step) {
    cronos::clear_error();
    if (!sim) return fail(CRONOS_EINVAL, "set_state: NULL handle");
    if (step < 0) return fail(CRONOS_EINVAL, "set_state: step < 0");
    const int64_t n = sim->d.n;
    const cronos::Layout& L = sim->lay;
    HIP_TRY(hipSetDevice(sim->device));
    HIP_TRY(hipStreamSynchronize(sim->stream));
    if (x) {
        std::vector<float4> hx(n);
        for (int64_t i = 0; i < n; ++i) {
            int32_t o = L.perm[i];
            for (int c = 0; c < 3; ++c)
                if (!std::isfinite(x[3 * o + c])) return fail(CRONOS_EINVAL, "set_state: non-finite x");
            hx[i] = make_float4((float)(x[3 * o] - sim->origin[0]), (float)(x[3 * o + 1] - sim->origin[1]),
                                (float)(x[3 * o + 2] - sim->origin[2]), sim->inv_m[i]);
        }
        HIP_TRY(hipMemcpy(sim->d.x[sim->cur], hx.data(), n * sizeof(float4), hipMemcpyHostToDevice));
    }
    if (v) {
        std::vector<float> hv(3 * n);
        for (int64_t i = 0; i < n; ++i) {
            int32_t o = L.perm[i];
            for (int c = 0; c < 3; ++c) hv[3 * i + c] = sim->inv_m[i] == 0.0f ? 0.0f : (float)v[3 * o + c];
        }
        HIP_TRY(hipMemcpy(sim->d.v[sim->cur], hv.data(), 3 * n * sizeof(float), hipMemcpyHostToDevice));
    }
    long long ctr = step;
    HIP_TRY(hipMemcpy(sim->d.step_ctr + sim->cur, &ctr, sizeof ctr, hipMemcpyHostToDevice));
    sim->step = step;
    sim->half_kick = sim->verlet;   // Verlet restarts from (x_0, v_0): eq. (5)
    return CRONOS_OK;
}

extern "C" cronos_status cronos_eval_forces(cronos_sim sim, double* f) {
    cronos::clear_error();
    if (!sim || !f) return fail(CRONOS_EINVAL, "eval_forces: NULL argument");
    const int64_t n = sim->d.n;
    HIP_TRY(hipSetDevice(sim->device));
    if (sim->actuated) HIP_TRY(cronos::launch_actuation(sim->d, sim->cycles, 0, sim->stream, -1, nullptr, sim->cur));
    HIP_TRY(cronos::launch_forces(sim->d, sim->cur, sim->p, sim->stream));
    if (!sim->h_f) HIP_TRY(hipHostMalloc((void**)&sim->h_f, 3 * n * sizeof(float), 0));
    HIP_TRY(hipMemcpyAsync(sim->h_f, sim->d.fout, 3 * n * sizeof(float), hipMemcpyDeviceToHost, sim->stream));
    HIP_TRY(hipStreamSynchronize(sim->stream));
    for (int64_t i = 0; i < n; ++i) {
        int32_t o = sim->lay.perm[i];
        for (int c = 0; c < 3; ++c) f[3 * o + c] = sim->h_f[3 * i + c];
    }
    return CRONOS_OK;
}

namespace {

// Ritz values of the Lanczos tridiagonal matrix T_k with their error estimates.  Values whose
// residual intervals overlap are copies of one eigenvalue (the "ghosts" that plain Lanczos
// produces once an eigenvalue has converged) and are merged, keeping the smallest residual.
struct RitzCluster {
    double theta, err, floor;  // floor: the error that FP64 arithmetic on T cannot go below
};

std::vector<RitzCluster> ritz_clusters(const std::vector<double>& a, const std::vector<double>& b, int64_t k,
                                       int64_t count) {
    std::vector<double> b2(k > 1 ? k - 1 : 1);
    for (int64_t i = 0; i + 1 < k; ++i) b2[i] = b[i] * b[i];
    double lo, hi;
    cronos::gershgorin(a.data(), b.data(), k, &lo, &hi);
    const double norm = std::max(std::fabs(lo), std::fabs(hi));
    const double tiny_count = 1e-300, tiny_solve = 1e-15 * std::max(norm, 1e-300);
    const double beta_k = b[k - 1];  // norm of the next Lanczos residual
    std::vector<double> th(count), r(count);
    double lower = lo;
    for (int64_t j = 0; j < count; ++j) {
        th[j] = cronos::tridiag_eigenvalue(a.data(), b2.data(), k, j, lower, hi, tiny_count);
        lower = std::max(lo, th[j] - 4e-16 * norm);
        r[j] = std::fabs(beta_k) * cronos::eigvec_last_component(a.data(), b.data(), k, th[j], tiny_solve);
    }
    std::vector<RitzCluster> out;
    std::vector<double> out_r;
    for (int64_t j = 0; j < count; ++j) {
        if (!out.empty() && th[j] - out.back().theta <= r[j] + out_r.back() + 8e-16 * norm) {
            if (r[j] < out_r.back()) {
                out.back().theta = th[j];
                out_r.back() = r[j];
            }
            continue;
        }
        out.push_back({th[j], 0.0, 0.0});
        out_r.push_back(r[j]);
    }
    // error bound min(r, r^2 / gap), gap to the neighbouring clusters; never below what the
    // FP64 arithmetic on T itself resolves
    const double floor = 8e-16 * norm;
    for (size_t c = 0; c < out.size(); ++c) {
        double gap = 1e300;
        if (c > 0) gap = std::min(gap, out[c].theta - out[c - 1].theta);
        if (c + 1 < out.size()) gap = std::min(gap, out[c + 1].theta - out[c].theta);
        const double rr = out_r[c];
        out[c].err = std::max(std::min(rr, rr * rr / gap), floor);
        out[c].floor = floor;
    }
    // the last cluster's upper neighbour is unknown: only its residual bounds it
    if (!out.empty()) out.back().err = std::max(out_r.back(), floor);
    return out;
}

}  // namespace

namespace {

cronos_status check_modes_args(cronos_sim sim, int32_t n_modes, int32_t max_iter, double tol, const double* omega,
                               const int32_t* n_found) {
    if (!sim || !omega || !n_found) return fail(CRONOS_EINVAL, "natural_frequencies: NULL argument");
    if (n_modes < 1 || n_modes > 32) return fail(CRONOS_EINVAL, "natural_frequencies: n_modes must be in [1, 32]");
    if (max_iter < 2 * n_modes + 8 || max_iter > (1 << 24))
        return fail(CRONOS_EINVAL, "natural_frequencies: max_iter must be in [2 n_modes + 8, 2^24]");
    if (!(tol > 0.0 && tol < 1.0)) return fail(CRONOS_EINVAL, "natural_frequencies: tol must be in (0, 1)");
    return CRONOS_OK;
}

// The Lanczos iteration of cronos_natural_frequencies on workspace m (every buffer of
// ModesBuffers sized for sim and max_iter).
cronos_status lanczos_frequencies(cronos_sim sim, cronos::ModesBuffers& m, int32_t n_modes, int32_t max_iter, double tol,
                                  uint64_t seed, double* omega, int32_t* n_found, int32_t* iterations) {
    const int64_t n = sim->d.n;
    if (sim->actuated) HIP_TRY(cronos::launch_actuation(sim->d, sim->cycles, 0, sim->stream, -1, nullptr, sim->cur));
    HIP_TRY(cronos::launch_modes_init(sim->d, sim->cur, m, seed, sim->stream));
    std::vector<double> ha(max_iter), hb(max_iter);
    int32_t k = 0, next = std::min<int32_t>(max_iter, std::max<int32_t>(64, 4 * n_modes + 16));
    int32_t found = 0;
    std::vector<double> best;
    while (true) {
        for (; k < next; ++k) HIP_TRY(cronos::launch_modes_iteration(sim->d, sim->cur, sim->p, m, k, sim->stream));
        HIP_TRY(hipMemcpyAsync(ha.data(), m.alpha, k * sizeof(double), hipMemcpyDeviceToHost, sim->stream));
        HIP_TRY(hipMemcpyAsync(hb.data(), m.beta, k * sizeof(double), hipMemcpyDeviceToHost, sim->stream));
        HIP_TRY(hipStreamSynchronize(sim->stream));
        for (int32_t i = 0; i < k; ++i)
            if (!std::isfinite(ha[i]) || !std::isfinite(hb[i]))
                return fail(CRONOS_ESTATE, "natural_frequencies: non-finite Lanczos coefficient at step %d", i);
        const int64_t count = std::min<int64_t>(k, 2 * n_modes + 8);
        std::vector<RitzCluster> cl = ritz_clusters(ha, hb, k, count);
        // the converged prefix: every cluster up to it has an error within tol
        int32_t conv = 0;
        for (const RitzCluster& c : cl) {
            if (c.err > tol * std::fabs(c.theta) && c.err > c.floor && !(hb[k - 1] == 0.0)) break;
            ++conv;
        }
        found = std::min<int32_t>(conv, n_modes);
        best.clear();
        for (int32_t c = 0; c < found; ++c) best.push_back(cl[c].theta);
        const bool exhausted = hb[k - 1] <= 1e-14 * std::fabs(ha[0]) || k >= std::min<int64_t>(max_iter, 3 * n);
        if (found >= n_modes || exhausted || k >= max_iter) break;
        next = (int32_t)std::min<int64_t>(max_iter, (int64_t)k + std::max<int64_t>(256, k / 4));
    }
    for (int32_t c = 0; c < n_modes; ++c) {
        const double t = c < found ? best[c] : 0.0;
        omega[c] = t >= 0.0 ? std::sqrt(t) : -std::sqrt(-t);
    }
    *n_found = found;
    if (iterations) *iterations = k;
    return CRONOS_OK;
}

}  // namespace

extern "C" cronos_status cronos_natural_frequencies(cronos_sim sim, int32_t n_modes, int32_t max_iter, double tol,
                                                    uint64_t seed, double* omega, int32_t* n_found,
                                                    int32_t* iterations) {
    cronos::clear_error();
    TRY(check_modes_args(sim, n_modes, max_iter, tol, omega, n_found));
    const int64_t n = sim->d.n;
    HIP_TRY(hipSetDevice(sim->device));
    cronos::ModesBuffers m;
    const int64_t nu = (n + 255) / 256;
    std::vector<void*> owned;
    auto alloc = [&](double** p, size_t count) -> cronos_status {
        if (hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(double)) != hipSuccess)
            return fail(CRONOS_ENOMEM, "natural_frequencies: device allocation of %zu doubles failed", count);
        owned.push_back(*p);
        return CRONOS_OK;
    };
    auto run = [&]() -> cronos_status {
        TRY(alloc(&m.ism, n));
        TRY(alloc(&m.q[0], 3 * n));
        TRY(alloc(&m.q[1], 3 * n));
        TRY(alloc(&m.y, 3 * n));
        TRY(alloc(&m.part_a, sim->d.nblk));
        TRY(alloc(&m.part_u, nu));
        TRY(alloc(&m.alpha, max_iter));
        TRY(alloc(&m.beta, max_iter));
        return lanczos_frequencies(sim, m, n_modes, max_iter, tol, seed, omega, n_found, iterations);
    };
    const cronos_status st = run();
    (void)hipStreamSynchronize(sim->stream);
    for (void* p : owned) (void)hipFree(p);
    return st;
}

extern "C" cronos_status cronos_natural_frequencies_noalloc(cronos_sim sim, int32_t n_modes, int32_t max_iter,
                                                            double tol, uint64_t seed, double* omega,
                                                            int32_t* n_found, int32_t* iterations) {
    cronos::clear_error();
    TRY(check_modes_args(sim, n_modes, max_iter, tol, omega, n_found));
    const int64_t n = sim->d.n;
    HIP_TRY(hipSetDevice(sim->device));
    double* base = nullptr;
    HIP_TRY(cronos::modes_scratch(sim->device, &base));
    // carve the fixed workspace: every buffer starts on a 256-byte boundary
    const int64_t counts[8] = {n, 3 * n, 3 * n, 3 * n, sim->d.nblk, (n + 255) / 256, max_iter, max_iter};
    int64_t off[8], used = 0;
    for (int b = 0; b < 8; ++b) {
        off[b] = used;
        used += (std::max<int64_t>(counts[b], 1) + 31) / 32 * 32;
    }
    if (used > (int64_t)cronos::kModesScratchDoubles)
        return fail(CRONOS_EINVAL,
                    "natural_frequencies_noalloc: %lld masses and max_iter %d need %lld doubles of workspace; the "
                    "fixed workspace holds %zu",
                    (long long)n, max_iter, (long long)used, cronos::kModesScratchDoubles);
    cronos::ModesBuffers m;
    m.ism = base + off[0];
    m.q[0] = base + off[1];
    m.q[1] = base + off[2];
    m.y = base + off[3];
    m.part_a = base + off[4];
    m.part_u = base + off[5];
    m.alpha = base + off[6];
    m.beta = base + off[7];
    const cronos_status st = lanczos_frequencies(sim, m, n_modes, max_iter, tol, seed, omega, n_found, iterations);
    (void)hipStreamSynchronize(sim->stream);
    return st;
}

extern "C" cronos_status cronos_diagnostics(cronos_sim sim, cronos_diag* out) {
    cronos::clear_error();
    if (!sim || !out) return fail(CRONOS_EINVAL, "diagnostics: NULL argument");
    HIP_TRY(hipSetDevice(sim->device));
    const int nb = sim->nb;
    if (sim->actuated) HIP_TRY(cronos::launch_actuation(sim->d, sim->cycles, 0, sim->stream, -1, nullptr, sim->cur));
    HIP_TRY(cronos::launch_diagnostics(sim->d, sim->cur, sim->p, sim->stream));
    if (!sim->h_diag) HIP_TRY(hipHostMalloc((void**)&sim->h_diag, (size_t)nb * cronos::kDiagFields * sizeof(double), 0));
    HIP_TRY(hipMemcpyAsync(sim->h_diag, sim->d.body_out, (size_t)nb * cronos::kDiagFields * sizeof(double),
                           hipMemcpyDeviceToHost, sim->stream));
    HIP_TRY(hipStreamSynchronize(sim->stream));
    bool bad = false;
    for (int b = 0; b < nb; ++b) {
        const double* q = sim->h_diag + (size_t)b * cronos::kDiagFields;
        cronos_diag& o = out[b];
        std::memset(&o, 0, sizeof o);
        o.ke = q[0];
        o.pe_spring = q[1];
        o.pe_grav = q[2];
        o.pe_contact = q[3];
        o.mass = q[10];
        for (int c = 0; c < 3; ++c) {
            o.p[c] = q[4 + c];
            o.com[c] = q[7 + c] / q[10];
            o.bbox_max[c] = q[11 + c];
            o.bbox_min[c] = q[14 + c];
        }
        o.step = sim->step;
        o.nonfinite = q[17] > 0.0 || !std::isfinite(q[0]) || !std::isfinite(q[1]);
        bad = bad || o.nonfinite;
    }
    if (bad) return fail(CRONOS_ESTATE, "diagnostics: non-finite state");
    return CRONOS_OK;
}

extern "C" cronos_status cronos_info(cronos_sim sim, int64_t* n_masses, int64_t* n_springs, int32_t* n_bodies,
                                     int32_t* block_masses, int64_t* step) {
    if (!sim) return fail(CRONOS_EINVAL, "info: NULL handle");
    if (n_masses) *n_masses = sim->lay.n;
    if (n_springs) *n_springs = sim->lay.s;
    if (n_bodies) *n_bodies = sim->nb;
    if (block_masses) *block_masses = sim->lay.block;
    if (step) *step = sim->step;
    return CRONOS_OK;
}

namespace {

template <typename T>
cronos_status ensure(T** p, size_t count) {
    if (*p) return CRONOS_OK;
    if (hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess)
        return fail(CRONOS_ENOMEM, "device allocation of %zu bytes failed", count * sizeof(T));
    return CRONOS_OK;
}

template <typename T>
void release(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

}  // namespace

namespace {

// The actuated entries of each actuation group in entry order (CSR over groups), read by the
// device's per-group sums of the adjoint's sensitivities.
cronos_status build_group_lists(cronos_sim_t* sim) {
    RolloutBuffers& R = sim->ro;
    const int32_t G = sim->d.n_factor;
    const int64_t entries = sim->lay.slice_ptr.back();
    std::vector<int32_t> ptr((size_t)G + 1, 0);
    for (int64_t e = 0; e < entries; ++e)
        if (sim->h_grp[e] < G) ++ptr[(size_t)sim->h_grp[e] + 1];
    for (int32_t g = 0; g < G; ++g) ptr[(size_t)g + 1] += ptr[(size_t)g];
    std::vector<int32_t> idx((size_t)ptr[(size_t)G]), fill(ptr.begin(), ptr.end() - 1);
    for (int64_t e = 0; e < entries; ++e)
        if (sim->h_grp[e] < G) idx[(size_t)fill[sim->h_grp[e]]++] = (int32_t)e;
    TRY(ensure(&R.grp_entries, idx.size()));
    TRY(ensure(&R.gsum, (size_t)std::max(G, 1)));
    if (!idx.empty()) HIP_TRY(hipMemcpy(R.grp_entries, idx.data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    TRY(ensure(&R.grp_ptr, ptr.size()));
    HIP_TRY(hipMemcpy(R.grp_ptr, ptr.data(), ptr.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    return CRONOS_OK;
}

}  // namespace

extern "C" cronos_status cronos_rollout(cronos_sim sim, int64_t n_steps, int32_t ckpt_every, const double* loss_w,
                                        double* loss) {
    cronos::clear_error();
    if (!sim || !loss_w || !loss) return fail(CRONOS_EINVAL, "rollout: NULL argument");
    if (n_steps < 0 || ckpt_every < 1) return fail(CRONOS_EINVAL, "rollout: need n_steps >= 0 and ckpt_every >= 1");
    if (sim->verlet) return fail(CRONOS_EINVAL, "rollout: the adjoint is of the symplectic Euler step, not Verlet");
    const int64_t n = sim->d.n;
    RolloutBuffers& R = sim->ro;
    HIP_TRY(hipSetDevice(sim->device));
    const int32_t K = (int32_t)std::min<int64_t>(ckpt_every, std::max<int64_t>(n_steps, 1));
    const int32_t nseg = (int32_t)((n_steps + K - 1) / K);
    if (R.cap_seg < (size_t)K || R.cap_ck < (size_t)nseg) {
        HIP_TRY(hipStreamSynchronize(sim->stream));
        release(R.ck_x);
        release(R.ck_v);
        for (int q = 0; q < 2; ++q) {
            release(R.seg_x[q]);
            release(R.seg_v[q]);
            release(R.seg_vs[q]);
            release(R.seg_f[q]);
        }
        R.cap_seg = std::max<size_t>(R.cap_seg, (size_t)K);
        R.cap_ck = std::max<size_t>(R.cap_ck, (size_t)std::max(nseg, 1));
    }
    TRY(ensure(&R.ck_x, R.cap_ck * n));
    TRY(ensure(&R.ck_v, R.cap_ck * 3 * n));
    for (int q = 0; q < 2; ++q) {
        TRY(ensure(&R.seg_x[q], (R.cap_seg + 1) * n));
        TRY(ensure(&R.seg_v[q], (R.cap_seg + 1) * 3 * n));
        TRY(ensure(&R.seg_vs[q], R.cap_seg * 3 * n));
        TRY(ensure(&R.seg_f[q], R.cap_seg * (size_t)(sim->d.n_factor + 1)));
    }
    if (!R.side) HIP_TRY(hipStreamCreateWithFlags(&R.side, hipStreamNonBlocking));
    for (hipEvent_t& e : R.ev)
        if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    TRY(ensure(&R.lossw, 3 * n));
    for (int q = 0; q < 2; ++q) {
        TRY(ensure(&R.w[q], n));
        TRY(ensure(&R.xb[q], 3 * n));
        TRY(ensure(&R.vb[q], 3 * n));
        TRY(ensure(&R.xbl[q], 3 * n));
    }
    TRY(ensure(&R.sens, (size_t)sim->lay.slice_ptr.back()));
    if (sim->actuated && !R.grp_ptr) TRY(build_group_lists(sim));
    // loss weights in the device order (FP32)
    std::vector<float> hw(3 * n);
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) hw[3 * i + c] = (float)loss_w[3 * sim->lay.perm[i] + c];
    HIP_TRY(hipStreamSynchronize(sim->stream));
    HIP_TRY(hipMemcpy(R.lossw, hw.data(), 3 * n * sizeof(float), hipMemcpyHostToDevice));
    R.n0 = sim->step;
    R.T = n_steps;
    R.K = K;
    R.nseg = nseg;
    for (int32_t c = 0; c < nseg; ++c) {
        HIP_TRY(hipMemcpyAsync(R.ck_x + (size_t)c * n, sim->d.x[sim->cur], n * sizeof(float4), hipMemcpyDeviceToDevice,
                               sim->stream));
        HIP_TRY(hipMemcpyAsync(R.ck_v + (size_t)c * 3 * n, sim->d.v[sim->cur], 3 * n * sizeof(float),
                               hipMemcpyDeviceToDevice, sim->stream));
        TRY(cronos_step(sim, std::min<int64_t>(K, n_steps - (int64_t)c * K)));
    }
    std::vector<double> xT(3 * n);
    TRY(cronos_read_state(sim, xT.data(), nullptr, nullptr));
    double L = 0.0;
    for (int64_t i = 0; i < 3 * n; ++i) L += loss_w[i] * xT[i];
    *loss = L;
    R.valid = true;
    return CRONOS_OK;
}

namespace {

// Enqueues the reverse sweep of the recorded rollout on the simulation's stream: for each
// segment from the last, restore its checkpoint, recompute its states forward (keeping v* and
// each step's actuation factors), then run the adjoint of each of its steps backwards.  The
// recompute runs one segment ahead on a second stream, into the other segment buffer, so it
// overlaps the adjoint kernels (both are small launches on bodies of this size); events
// order the two.  No host synchronisation and no memsets, so it can be captured in a HIP
// graph (the second stream joins the capture through the first event).
cronos_status enqueue_reverse_sweep(cronos_sim_t* sim) {
    RolloutBuffers& R = sim->ro;
    const int64_t n = sim->d.n;
    const cronos::DeviceArrays& D = sim->d;
    hipStream_t st = sim->stream;
    const size_t fs = (size_t)D.n_factor + 1;
    hipEvent_t fork = R.ev[0], *done_fwd = R.ev + 1, *done_rev = R.ev + 3;
    // segment c into buffer c & 1 on the side stream: restore its checkpoint, recompute its
    // states forward keeping v* and each step's actuation factors
    auto recompute = [&](int32_t c) -> cronos_status {
        const int p = c & 1;
        const int64_t nc = R.n0 + (int64_t)c * R.K;
        const int32_t steps = (int32_t)std::min<int64_t>(R.K, R.T - (int64_t)c * R.K);
        HIP_TRY(hipMemcpyAsync(R.seg_x[p], R.ck_x + (size_t)c * n, n * sizeof(float4), hipMemcpyDeviceToDevice, R.side));
        HIP_TRY(hipMemcpyAsync(R.seg_v[p], R.ck_v + (size_t)c * 3 * n, 3 * n * sizeof(float), hipMemcpyDeviceToDevice,
                               R.side));
        if (sim->actuated)
            HIP_TRY(cronos::launch_actuation_steps(D, sim->cycles, nc, steps, R.seg_f[p], (long long)fs, R.side));
        for (int32_t k = 0; k < steps; ++k) {
            float* fk = sim->actuated ? R.seg_f[p] + (size_t)k * fs : nullptr;
            HIP_TRY(cronos::launch_step_io(D, R.seg_x[p] + (size_t)k * n, R.seg_v[p] + (size_t)k * 3 * n,
                                           R.seg_x[p] + (size_t)(k + 1) * n, R.seg_v[p] + (size_t)(k + 1) * 3 * n,
                                           R.seg_vs[p] + (size_t)k * 3 * n, sim->p, R.side, fk));
        }
        HIP_TRY(hipEventRecord(done_fwd[p], R.side));
        return CRONOS_OK;
    };
    // the side stream starts after what the main stream holds (and joins a capture this way)
    HIP_TRY(hipEventRecord(fork, st));
    HIP_TRY(hipStreamWaitEvent(R.side, fork, 0));
    TRY(recompute(R.nseg - 1));
    int cur = 0, wc = 0;
    for (int32_t c = R.nseg - 1; c >= 0; --c) {
        const int p = c & 1;
        const int64_t nc = R.n0 + (int64_t)c * R.K;
        const int32_t steps = (int32_t)std::min<int64_t>(R.K, R.T - (int64_t)c * R.K);
        if (c > 0) {
            // the earlier segment's buffer was last read by the reverse sweep of segment c + 1
            if (c + 1 < R.nseg) HIP_TRY(hipStreamWaitEvent(R.side, done_rev[(c - 1) & 1], 0));
            TRY(recompute(c - 1));
        }
        HIP_TRY(hipStreamWaitEvent(st, done_fwd[p], 0));
        // the segment's last step: adj_local on its own; every later adj_local (of step k - 1)
        // runs at the end of the gather of step k, while the segment's states are at hand
        const int32_t last = steps - 1;
        HIP_TRY(cronos::launch_adj_local(D, R.seg_x[p] + (size_t)last * n, R.seg_vs[p] + (size_t)last * 3 * n,
                                         R.xb[cur], R.vb[cur], R.w[wc], R.vb[cur ^ 1], R.xbl[wc], sim->p, st));
        for (int32_t k = last; k >= 0; --k) {
            const double t = (double)(nc + k) * sim->dt;
            cronos::AdjNext nx;
            if (k > 0) {
                nx.x = R.seg_x[p] + (size_t)(k - 1) * n;
                nx.vstar = R.seg_vs[p] + (size_t)(k - 1) * 3 * n;
                nx.vb1 = R.vb[cur ^ 1];
                nx.w = R.w[wc ^ 1];
                nx.vb0 = R.vb[cur];
                nx.xbl = R.xbl[wc ^ 1];
            }
            HIP_TRY(cronos::launch_adj_gather(D, R.seg_x[p] + (size_t)k * n, R.w[wc], R.xbl[wc], R.xb[cur ^ 1], R.sens,
                                              std::cos(sim->omega * t), std::sin(sim->omega * t), st,
                                              sim->actuated ? R.seg_f[p] + (size_t)k * fs : nullptr, sim->p, nx));
            cur ^= 1;
            if (k > 0) wc ^= 1;
        }
        HIP_TRY(hipEventRecord(done_rev[p], st));
    }
    return CRONOS_OK;
}

}  // namespace

extern "C" cronos_status cronos_rollout_backward(cronos_sim sim, double* dphase, double* damp, double* dx0,
                                                 double* dv0) {
    cronos::clear_error();
    if (!sim) return fail(CRONOS_EINVAL, "rollout_backward: NULL handle");
    RolloutBuffers& R = sim->ro;
    if (!R.valid) return fail(CRONOS_EINVAL, "rollout_backward: no rollout recorded");
    const int64_t n = sim->d.n;
    const int64_t entries = sim->lay.slice_ptr.back();
    hipStream_t st = sim->stream;
    HIP_TRY(hipSetDevice(sim->device));
    HIP_TRY(hipMemcpyAsync(R.xb[0], R.lossw, 3 * n * sizeof(float), hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemsetAsync(R.vb[0], 0, 3 * n * sizeof(float), st));
    HIP_TRY(hipMemsetAsync(R.sens, 0, (size_t)entries * sizeof(double2), st));
    // the reverse sweep flips the adjoint buffers once per step
    const int cur = (int)(R.T & 1);
    // plain launches on the two streams: captured as one HIP graph the same sweep ran its
    // recompute and adjoint branches one after the other (quadruped, 2000 steps: 26.3-27.3 ms
    // against 20.7 ms)
    TRY(enqueue_reverse_sweep(sim));
    // per-group sums of the actuation sensitivities (FP64), then the chain rule to phase and amplitude
    const int32_t G = sim->d.n_factor;
    if ((dphase || damp) && G > 0 && sim->actuated) {
        // per group: the sum of its entries' sensitivities, in a fixed order on the device
        std::vector<double> sp(G, 0.0), sq(G, 0.0);
        HIP_TRY(cronos::launch_adj_group_sums(R.sens, R.grp_ptr, R.grp_entries, G, R.gsum, st));
        std::vector<double2> hs(G);
        HIP_TRY(hipMemcpyAsync(hs.data(), R.gsum, (size_t)G * sizeof(double2), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int32_t g = 0; g < G; ++g) {
            sp[g] = hs[g].x;
            sq[g] = hs[g].y;
        }
        for (int32_t g = 0; g < G; ++g) {
            const double ph = sim->h_phase.empty() ? 0.0 : sim->h_phase[g];
            const double am = sim->h_amp.empty() ? 0.0 : sim->h_amp[g];
            if (dphase) dphase[g] = am * (sp[g] * std::cos(ph) - sq[g] * std::sin(ph));
            if (damp) damp[g] = sq[g] * std::cos(ph) + sp[g] * std::sin(ph);
        }
    } else {
        for (int32_t g = 0; g < G; ++g) {
            if (dphase) dphase[g] = 0.0;
            if (damp) damp[g] = 0.0;
        }
    }
    if (dx0 || dv0) {
        std::vector<float> hx(3 * n), hv(3 * n);
        HIP_TRY(hipMemcpyAsync(hx.data(), R.xb[cur], 3 * n * sizeof(float), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(hv.data(), R.vb[cur], 3 * n * sizeof(float), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < 3; ++c) {
                if (dx0) dx0[3 * sim->lay.perm[i] + c] = hx[3 * i + c];
                if (dv0) dv0[3 * sim->lay.perm[i] + c] = hv[3 * i + c];
            }
    }
    HIP_TRY(hipStreamSynchronize(st));
    return CRONOS_OK;
}

extern "C" cronos_status cronos_launch_config(cronos_sim sim, int32_t* block_masses, int32_t* batch,
                                              int32_t* persistent_groups, int32_t* step_form,
                                              int32_t* lanes_per_mass) {
    if (!sim) return fail(CRONOS_EINVAL, "launch_config: NULL handle");
    if (block_masses) *block_masses = sim->lay.block;
    if (batch) *batch = sim->d.batch;
    if (persistent_groups) *persistent_groups = sim->d.persistent_groups;
    if (lanes_per_mass) *lanes_per_mass = sim->d.lanes;
    if (step_form)
        *step_form = sim->d.grid ? CRONOS_FORM_GRID
                     : sim->d.resident ? CRONOS_FORM_RESIDENT
                     : sim->d.sp_rec ? CRONOS_FORM_SPLIT
                     : sim->d.narrow ? CRONOS_FORM_NARROW
                     : sim->d.packed ? CRONOS_FORM_TABLE
                                     : CRONOS_FORM_EXPLICIT;
    return CRONOS_OK;
}

extern "C" cronos_status cronos_launch_mode(cronos_sim sim, int32_t* graphs, double* plain_step_us, int32_t* staged_io) {
    if (!sim) return fail(CRONOS_EINVAL, "launch_mode: NULL handle");
    if (graphs) *graphs = sim->use_graph && sim->stream && !sim->d.resident ? 1 : 0;
    if (plain_step_us) *plain_step_us = sim->plain_step_us;
    if (staged_io) *staged_io = sim->d.stage_io;
    return CRONOS_OK;
}

extern "C" cronos_status cronos_autotune(const cronos_desc* d, int32_t n_steps, cronos_tune* out) {
    cronos::clear_error();
    if (!d || !out || n_steps < 1) return fail(CRONOS_EINVAL, "autotune: bad arguments");
    cronos_tune best{};
    best.us_per_step = 1e300;
    best.us_default = 0.0;
    const int blocks[] = {64, 128, 256, 512, 1024};
    const int batches[] = {2, 4, 8};
    for (int blk : blocks) {
        cronos_desc dd = *d;
        dd.block_masses = blk;
        dd.batch = 4;
        dd.persistent = -1;
        dd.lanes_per_mass = 1;
        dd.flags |= CRONOS_ALLOW_UNSTABLE;   // checked once by the caller's own create
        cronos_sim sim = nullptr;
        cronos_status st = cronos_create(&dd, &sim);
        if (st == CRONOS_EINVAL && blk != 256) continue;   // e.g. a halo too large for this size
        if (st != CRONOS_OK) return st;
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            cronos_destroy(sim);
            return fail(CRONOS_EDEVICE, "autotune: hipEventCreate failed");
        }
        int pgrid = 0;
        if (cronos::persistent_grid(sim->d, sim->p.exact, &pgrid) != hipSuccess) pgrid = 0;
        // configurations: (batch, persistent) with one lane per mass, then 2 and 4 lanes per
        // mass (table forms, one workgroup per block; batch does not apply)
        const bool lanes_ok = !sim->d.resident && !sim->d.sp_rec && (sim->d.packed || sim->d.narrow);
        std::vector<std::array<int, 3>> cfgs;
        for (int bt : batches)
            for (int pers = 0; pers < 2; ++pers)
                if (!pers || pgrid > 0) cfgs.push_back({bt, pers, 1});
        for (int ln : {2, 4})
            if (lanes_ok && blk * ln <= 1024) cfgs.push_back({4, 0, ln});
        if (sim->d.grid) cfgs.assign(1, {4, 0, 1});   // the structured-box form has no such choices
        for (const auto& cfg : cfgs) {
            const int bt = cfg[0], pers = cfg[1], ln = cfg[2];
            {
                sim->d.batch = bt;
                sim->d.persistent_groups = pers ? pgrid : 0;
                sim->d.lanes = ln;
                sim->use_graph = false;
                // warm up and time on the simulation's stream; the state evolves, which is
                // harmless for timing (the tuner's simulation is discarded)
                cronos_status s2 = enqueue_plain(sim, 3);
                if (s2 == CRONOS_OK && hipEventRecord(e0, sim->stream) != hipSuccess) s2 = CRONOS_EDEVICE;
                if (s2 == CRONOS_OK) s2 = enqueue_plain(sim, n_steps);
                if (s2 == CRONOS_OK && hipEventRecord(e1, sim->stream) != hipSuccess) s2 = CRONOS_EDEVICE;
                float ms = 0.0f;
                if (s2 == CRONOS_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    s2 = CRONOS_EDEVICE;
                if (s2 != CRONOS_OK) {
                    (void)hipEventDestroy(e0);
                    (void)hipEventDestroy(e1);
                    cronos_destroy(sim);
                    return s2 == CRONOS_EDEVICE ? fail(CRONOS_EDEVICE, "autotune: timing failed") : s2;
                }
                const double us = 1e3 * (double)ms / n_steps;
                if (blk == 256 && bt == 4 && !pers && ln == 1) best.us_default = us;
                if (us < best.us_per_step) {
                    best.us_per_step = us;
                    best.block_masses = blk;
                    best.batch = bt;
                    best.persistent = pers;
                    best.lanes_per_mass = ln;
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        cronos_destroy(sim);
    }
    if (best.block_masses == 0) return fail(CRONOS_EDEVICE, "autotune: no configuration could be timed");
    store_tune(tune_key(*d), best);
    *out = best;
    return CRONOS_OK;
}

extern "C" cronos_status cronos_get_layout(cronos_sim sim, int32_t* perm, int64_t* row_ptr, int32_t* col,
                                           int32_t* sid, int32_t* spring_perm) {
    if (!sim) return fail(CRONOS_EINVAL, "get_layout: NULL handle");
    const cronos::Layout& L = sim->lay;
    if (perm) std::memcpy(perm, L.perm.data(), L.n * sizeof(int32_t));
    if (row_ptr) std::memcpy(row_ptr, L.row_ptr.data(), (L.n + 1) * sizeof(int64_t));
    if (col) std::memcpy(col, L.col.data(), 2 * L.s * sizeof(int32_t));
    if (sid) std::memcpy(sid, L.sid.data(), 2 * L.s * sizeof(int32_t));
    if (spring_perm) std::memcpy(spring_perm, L.spring_perm.data(), L.s * sizeof(int32_t));
    return CRONOS_OK;
}
