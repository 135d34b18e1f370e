// Space-filling-curve renumbering, per-mass incidence CSR and the sliced device layout.
//
// Section "GPU Implementation" stores the mass->spring connectivity a second time so that a
// per-mass pass can visit each mass's springs; Algorithm 1 then sums each mass's spring
// forces.  Here that per-mass list is a CSR over a Morton renumbering (neighbours of a mass
// are mostly nearby in memory), sliced for the GPU:
//   * slice = 64 lanes = one wavefront, one lane per mass; within a workgroup the lanes take
//     the masses in order of decreasing degree, so a slice holds masses of similar degree; the
//     slice's entries are stored column-major (entry r of lane l at slice_ptr[s] + 64 r + l)
//     and padded to the slice's largest degree with entries that contribute exactly zero;
//   * workgroup = `block` consecutive masses; it stages the positions of its own masses and
//     of its halo (neighbours outside the block, ascending) in LDS, and every entry names its
//     neighbour by that 16-bit LDS slot.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>

#include "common.h"

namespace cronos {

namespace {

inline uint64_t spread3(uint64_t v) {
    // bit b of v -> bit 3b (21 bits)
    uint64_t r = 0;
    for (int b = 0; b < 21; ++b) r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

inline uint64_t morton(uint64_t qx, uint64_t qy, uint64_t qz) {
    return spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
}

}  // namespace

cronos_status build_layout(int64_t n, int32_t nb, const int64_t* body_offset, const double* x,
                           const int32_t* grid, int64_t s, const int32_t* ends, int32_t block,
                           Layout& L) {
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(CRONOS_EINVAL, "layout: n_masses out of range");
    if (s < 0 || 2 * s >= (int64_t(1) << 31)) return fail(CRONOS_EINVAL, "layout: n_springs out of range");
    if (nb < 1) return fail(CRONOS_EINVAL, "layout: n_bodies < 1");
    if (nb > 1 && !body_offset) return fail(CRONOS_EINVAL, "layout: body_offset required");
    if (!x && !grid) return fail(CRONOS_EINVAL, "layout: positions or grid required");
    if (s > 0 && !ends) return fail(CRONOS_EINVAL, "layout: ends required");
    if (block == 0) block = kDefaultBlock;
    if (block < kSlice || block > 1024 || block % kSlice) return fail(CRONOS_EINVAL, "layout: bad block_masses");

    L = Layout();
    L.n = n;
    L.s = s;
    L.nb = nb;
    L.block = block;
    L.body_off.resize(nb + 1);
    for (int32_t b = 0; b <= nb; ++b) L.body_off[b] = body_offset ? body_offset[b] : (b ? n : 0);
    if (L.body_off[0] != 0 || L.body_off[nb] != n) return fail(CRONOS_EINVAL, "layout: body_offset must span [0, n)");
    for (int32_t b = 0; b < nb; ++b)
        if (L.body_off[b + 1] <= L.body_off[b]) return fail(CRONOS_EINVAL, "layout: empty or decreasing body");

    // ---- Morton keys and the stable (body, key, index) order (bodies in parallel)
    std::vector<uint64_t> key(n);
    std::vector<int> body_err(nb, 0);
    L.perm.resize(n);
    parallel_for(nb, [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
            int64_t a0 = L.body_off[b], a1 = L.body_off[b + 1];
            if (grid) {
                int64_t mn[3] = {INT64_MAX, INT64_MAX, INT64_MAX};
                for (int64_t i = a0; i < a1; ++i)
                    for (int c = 0; c < 3; ++c) mn[c] = std::min<int64_t>(mn[c], grid[3 * i + c]);
                for (int64_t i = a0; i < a1; ++i) {
                    uint64_t q[3];
                    for (int c = 0; c < 3; ++c) {
                        int64_t dd = (int64_t)grid[3 * i + c] - mn[c];
                        if (dd >= (int64_t(1) << 21)) body_err[b] = 1;
                        q[c] = (uint64_t)dd & ((1ull << 21) - 1);
                    }
                    key[i] = morton(q[0], q[1], q[2]);
                }
            } else {
                double lo[3], hi[3];
                for (int c = 0; c < 3; ++c) lo[c] = hi[c] = x[3 * a0 + c];
                for (int64_t i = a0; i < a1; ++i)
                    for (int c = 0; c < 3; ++c) {
                        double v = x[3 * i + c];
                        if (!std::isfinite(v)) body_err[b] = 2;
                        lo[c] = std::min(lo[c], v);
                        hi[c] = std::max(hi[c], v);
                    }
                double ext = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
                for (int64_t i = a0; i < a1; ++i) {
                    uint64_t q[3] = {0, 0, 0};
                    if (ext > 0.0 && !body_err[b]) {
                        double scale = 1048576.0 / ext;
                        for (int c = 0; c < 3; ++c) {
                            double t = (x[3 * i + c] - lo[c]) * scale;
                            int64_t qi = (int64_t)std::floor(t);
                            q[c] = (uint64_t)std::min<int64_t>(qi, 1048575);
                        }
                    }
                    key[i] = morton(q[0], q[1], q[2]);
                }
            }
            for (int64_t i = a0; i < a1; ++i) L.perm[i] = (int32_t)i;
            std::sort(L.perm.begin() + a0, L.perm.begin() + a1,
                      [&](int32_t p, int32_t q) { return key[p] != key[q] ? key[p] < key[q] : p < q; });
        }
    }, 1);
    for (int32_t b = 0; b < nb; ++b) {
        if (body_err[b] == 1) return fail(CRONOS_EINVAL, "layout: grid extent exceeds 2^21");
        if (body_err[b] == 2) return fail(CRONOS_EINVAL, "layout: non-finite position");
    }
    L.inv.resize(n);
    for (int64_t i = 0; i < n; ++i) L.inv[L.perm[i]] = (int32_t)i;

    // body of each input mass
    std::vector<int32_t> body_of(n);
    for (int32_t b = 0; b < nb; ++b)
        for (int64_t i = L.body_off[b]; i < L.body_off[b + 1]; ++i) body_of[i] = b;

    // ---- springs: validate, renumber, CSR by counting sort on the row
    std::vector<int64_t> deg(n + 1, 0);
    for (int64_t q = 0; q < s; ++q) {
        int32_t a = ends[2 * q], b = ends[2 * q + 1];
        if (a < 0 || b < 0 || a >= n || b >= n) return fail(CRONOS_EINVAL, "layout: spring %lld end out of range", (long long)q);
        if (a == b) return fail(CRONOS_EINVAL, "layout: spring %lld joins a mass to itself", (long long)q);
        if (body_of[a] != body_of[b]) return fail(CRONOS_EINVAL, "layout: spring %lld joins two bodies", (long long)q);
        deg[L.inv[a] + 1]++;
        deg[L.inv[b] + 1]++;
    }
    L.row_ptr.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) L.row_ptr[i + 1] = L.row_ptr[i] + deg[i + 1];
    L.col.assign(2 * s, 0);
    std::vector<int32_t> in_spring(2 * s);
    {
        std::vector<int64_t> fill(L.row_ptr.begin(), L.row_ptr.end() - 1);
        for (int64_t q = 0; q < s; ++q) {
            int32_t a = L.inv[ends[2 * q]], b = L.inv[ends[2 * q + 1]];
            L.col[fill[a]] = b;
            in_spring[fill[a]++] = (int32_t)q;
            L.col[fill[b]] = a;
            in_spring[fill[b]++] = (int32_t)q;
        }
    }
    // sort each row by neighbour (rows in parallel); reject duplicate springs
    {
        std::vector<int> dup_found(1, 0);
        std::vector<int64_t> dup_flags((n + 4095) / 4096, 0);
        parallel_for((n + 4095) / 4096, [&](int64_t c0, int64_t c1) {
            std::vector<std::pair<int32_t, int32_t>> tmp;
            for (int64_t c = c0; c < c1; ++c)
                for (int64_t i = c * 4096; i < std::min<int64_t>(n, (c + 1) * 4096); ++i) {
                    int64_t r0 = L.row_ptr[i], r1 = L.row_ptr[i + 1];
                    tmp.resize(r1 - r0);
                    for (int64_t r = r0; r < r1; ++r) tmp[r - r0] = {L.col[r], in_spring[r]};
                    std::sort(tmp.begin(), tmp.end());
                    for (int64_t r = r0; r < r1; ++r) {
                        L.col[r] = tmp[r - r0].first;
                        in_spring[r] = tmp[r - r0].second;
                        if (r > r0 && L.col[r] == L.col[r - 1]) dup_flags[c] = 1;
                    }
                }
        }, 1);
        for (int64_t f : dup_flags)
            if (f) return fail(CRONOS_EINVAL, "layout: duplicate spring");
    }
    // new spring numbering: rows in order, entries with neighbour > row
    L.sid.assign(2 * s, -1);
    L.ends.resize(2 * s);
    L.spring_perm.resize(s);
    std::vector<int32_t> new_of_input(s, -1);
    int32_t next = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t r = L.row_ptr[i]; r < L.row_ptr[i + 1]; ++r)
            if (L.col[r] > i) {
                L.sid[r] = next;
                L.ends[2 * next] = (int32_t)i;
                L.ends[2 * next + 1] = L.col[r];
                L.spring_perm[next] = in_spring[r];
                new_of_input[in_spring[r]] = next;
                ++next;
            }
    parallel_for(2 * s, [&](int64_t r0, int64_t r1) {
        for (int64_t r = r0; r < r1; ++r)
            if (L.sid[r] < 0) L.sid[r] = new_of_input[in_spring[r]];
    });

    // ---- sliced layout and halos (blocks in parallel; concatenation in block order)
    L.nslice = (L.nblk = (n + block - 1) / block) * (block / kSlice);
    L.lane_mass.assign(L.nblk * block, 0);
    std::vector<std::vector<int32_t>> halos(L.nblk);
    parallel_for(L.nblk, [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
            int64_t base = b * block, end = std::min<int64_t>(n, base + block);
            uint16_t* lm = &L.lane_mass[base];
            for (int t = 0; t < block; ++t) lm[t] = (uint16_t)t;
            auto deg_of = [&](int t) -> int64_t {
                int64_t i = base + t;
                return i < n ? L.row_ptr[i + 1] - L.row_ptr[i] : -1;
            };
            std::stable_sort(lm, lm + block, [&](uint16_t p, uint16_t q) { return deg_of(p) > deg_of(q); });
            std::vector<int32_t>& halo = halos[b];
            for (int64_t i = base; i < end; ++i)
                for (int64_t r = L.row_ptr[i]; r < L.row_ptr[i + 1]; ++r)
                    if (L.col[r] < base || L.col[r] >= end) halo.push_back(L.col[r]);
            std::sort(halo.begin(), halo.end());
            halo.erase(std::unique(halo.begin(), halo.end()), halo.end());
        }
    }, 64);
    auto lane_deg = [&](int64_t lane_global) -> int64_t {
        int64_t b = lane_global / block;
        int64_t i = b * block + L.lane_mass[lane_global];
        return i < n ? L.row_ptr[i + 1] - L.row_ptr[i] : 0;
    };
    std::vector<int64_t> width(L.nslice, 0);
    parallel_for(L.nslice, [&](int64_t s0, int64_t s1) {
        for (int64_t sl = s0; sl < s1; ++sl)
            for (int64_t l = sl * kSlice; l < (sl + 1) * kSlice; ++l) width[sl] = std::max<int64_t>(width[sl], lane_deg(l));
    });
    L.slice_ptr.assign(L.nslice + 1, 0);
    for (int64_t sl = 0; sl < L.nslice; ++sl) {
        int64_t next_ptr = (int64_t)L.slice_ptr[sl] + width[sl] * kSlice;
        if (next_ptr >= (int64_t(1) << 31)) return fail(CRONOS_EINVAL, "layout: too many incidence entries");
        L.slice_ptr[sl + 1] = (int32_t)next_ptr;
    }
    L.halo_ptr.assign(L.nblk + 1, 0);
    L.max_halo = 0;
    for (int64_t b = 0; b < L.nblk; ++b) {
        if ((int64_t)halos[b].size() + block > 65535) return fail(CRONOS_EINVAL, "layout: halo too large for 16-bit slots");
        L.max_halo = std::max<int32_t>(L.max_halo, (int32_t)halos[b].size());
        int64_t next = (int64_t)L.halo_ptr[b] + (int64_t)halos[b].size();
        if (next >= (int64_t(1) << 31)) return fail(CRONOS_EINVAL, "layout: halo lists too long");
        L.halo_ptr[b + 1] = (int32_t)next;
    }
    L.halo_idx.resize(L.halo_ptr[L.nblk]);
    const int64_t entries = L.slice_ptr[L.nslice];
    L.nbr_local.assign(entries, 0);
    L.entry_csr.assign(entries, -1);
    parallel_for(L.nblk, [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
            const std::vector<int32_t>& halo = halos[b];
            std::copy(halo.begin(), halo.end(), L.halo_idx.begin() + L.halo_ptr[b]);
            int64_t base = b * block, end = std::min<int64_t>(n, base + block);
            for (int64_t sl = base / kSlice; sl < (base + block) / kSlice; ++sl) {
                int64_t w = (L.slice_ptr[sl + 1] - L.slice_ptr[sl]) / kSlice;
                for (int lane = 0; lane < kSlice; ++lane) {
                    int64_t own = L.lane_mass[sl * kSlice + lane];
                    int64_t i = base + own;
                    int64_t d = i < n ? L.row_ptr[i + 1] - L.row_ptr[i] : 0;
                    for (int64_t r = 0; r < w; ++r) {
                        int64_t e = L.slice_ptr[sl] + r * kSlice + lane;
                        if (r < d) {
                            int64_t pos = L.row_ptr[i] + r;
                            int32_t j = L.col[pos];
                            int64_t slot;
                            if (j >= base && j < end) slot = j - base;
                            else slot = block + (std::lower_bound(halo.begin(), halo.end(), j) - halo.begin());
                            L.nbr_local[e] = (uint16_t)slot;
                            L.entry_csr[e] = (int32_t)pos;
                        } else {
                            L.nbr_local[e] = (uint16_t)own;   // self: zero-length, contributes 0
                            L.entry_csr[e] = -1;
                        }
                    }
                }
            }
        }
    }, 64);
    return CRONOS_OK;
}

cronos_status check_layout(const Layout& L) {
    for (int64_t b = 0; b < L.nblk; ++b) {
        int64_t base = b * L.block, end = std::min<int64_t>(L.n, base + L.block);
        int64_t h0 = L.halo_ptr[b], h1 = L.halo_ptr[b + 1];
        std::vector<uint8_t> seen(L.block, 0);
        for (int t = 0; t < L.block; ++t) {
            int own = L.lane_mass[base + t];
            if (own >= L.block || seen[own]) return fail(CRONOS_EINVAL, "layout check: lane map of block %lld is not a permutation", (long long)b);
            seen[own] = 1;
        }
        for (int64_t sl = base / kSlice; sl < (base + L.block) / kSlice; ++sl) {
            int64_t w = (L.slice_ptr[sl + 1] - L.slice_ptr[sl]) / kSlice;
            for (int lane = 0; lane < kSlice; ++lane) {
                int64_t own = L.lane_mass[sl * kSlice + lane];
                int64_t i = base + own;
                int64_t d = i < L.n ? L.row_ptr[i + 1] - L.row_ptr[i] : 0;
                for (int64_t r = 0; r < w; ++r) {
                    int64_t e = L.slice_ptr[sl] + r * kSlice + lane;
                    int64_t slot = L.nbr_local[e];
                    int64_t j = slot < L.block ? base + slot : (slot - L.block < h1 - h0 ? L.halo_idx[h0 + slot - L.block] : -1);
                    if (r < d) {
                        int64_t pos = L.row_ptr[i] + r;
                        if (L.entry_csr[e] != pos || j != L.col[pos])
                            return fail(CRONOS_EINVAL, "layout check: entry %lld decodes wrong", (long long)e);
                    } else if (L.entry_csr[e] != -1 || j != i) {
                        return fail(CRONOS_EINVAL, "layout check: padding entry %lld not self", (long long)e);
                    }
                }
            }
        }
        for (int64_t h = h0; h < h1; ++h) {
            int32_t j = L.halo_idx[h];
            if (j >= base && j < end) return fail(CRONOS_EINVAL, "layout check: halo holds an own mass");
            if (h > h0 && L.halo_idx[h - 1] >= j) return fail(CRONOS_EINVAL, "layout check: halo not ascending");
        }
    }
    return CRONOS_OK;
}

}  // namespace cronos

using cronos::fail;

extern "C" cronos_status cronos_layout_build(int64_t n, int32_t nb, const int64_t* body_offset, const double* x,
                                             const int32_t* grid, int64_t s, const int32_t* ends,
                                             int32_t block, cronos_layout* out) {
    cronos::clear_error();
    if (!out) return fail(CRONOS_EINVAL, "layout: NULL out");
    *out = nullptr;
    auto* h = new (std::nothrow) cronos_layout_t;
    if (!h) return fail(CRONOS_ENOMEM, "layout: out of memory");
    cronos_status st;
    try {
        st = cronos::build_layout(n, nb, body_offset, x, grid, s, ends, block, h->lay);
    } catch (const std::bad_alloc&) {
        st = fail(CRONOS_ENOMEM, "layout: out of memory");
    }
    if (st != CRONOS_OK) {
        delete h;
        return st;
    }
    *out = h;
    return CRONOS_OK;
}

extern "C" cronos_status cronos_layout_get(cronos_layout h, int32_t* perm, int64_t* row_ptr, int32_t* col,
                                           int32_t* sid, int32_t* spring_perm) {
    if (!h) return fail(CRONOS_EINVAL, "layout: NULL handle");
    const cronos::Layout& L = h->lay;
    if (perm) std::memcpy(perm, L.perm.data(), L.n * sizeof(int32_t));
    if (row_ptr) std::memcpy(row_ptr, L.row_ptr.data(), (L.n + 1) * sizeof(int64_t));
    if (col) std::memcpy(col, L.col.data(), 2 * L.s * sizeof(int32_t));
    if (sid) std::memcpy(sid, L.sid.data(), 2 * L.s * sizeof(int32_t));
    if (spring_perm) std::memcpy(spring_perm, L.spring_perm.data(), L.s * sizeof(int32_t));
    return CRONOS_OK;
}

extern "C" cronos_status cronos_layout_check(cronos_layout h) {
    if (!h) return fail(CRONOS_EINVAL, "layout: NULL handle");
    return cronos::check_layout(h->lay);
}

extern "C" cronos_status cronos_layout_stats(cronos_layout h, int64_t* sell_entries, int64_t* halo_entries,
                                             int32_t* max_halo) {
    if (!h) return fail(CRONOS_EINVAL, "layout: NULL handle");
    if (sell_entries) *sell_entries = h->lay.slice_ptr.empty() ? 0 : h->lay.slice_ptr.back();
    if (halo_entries) *halo_entries = (int64_t)h->lay.halo_idx.size();
    if (max_halo) *max_halo = h->lay.max_halo;
    return CRONOS_OK;
}

extern "C" void cronos_layout_destroy(cronos_layout h) { delete h; }
