// Voxel lattice -> masses and springs (section "Generating a Lattice", voxel-grid variant).
//
// Nodes are the distinct corners of the occupied voxels, numbered per body in (z, y, x)
// order of their integer coordinate.  Every voxel links its 8 corners pairwise: 12 edges,
// 12 face diagonals, 4 long diagonals (the lattice figure of that section); a link shared by
// several voxels is one spring.  Parameters: uniform or lumped mass, uniform or per-voxel
// assembled stiffness, nominal rest lengths a * sqrt(number of differing coordinates).
// All floating-point values are formed with the same operations in the same order as the
// plain definition, so results are reproducible bit for bit (compiled without contraction).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "common.h"

namespace {

struct Body {
    std::vector<int32_t> coords;   // [n][3]
    std::vector<double> x, mass;
    std::vector<uint8_t> pinned;
    std::vector<int32_t> ends;     // [s][2]
    std::vector<double> k, rest;
    std::vector<int16_t> group;
};

inline uint64_t pack(int64_t x, int64_t y, int64_t z) {
    const int64_t off = int64_t(1) << 20;
    return (uint64_t(z + off) << 42) | (uint64_t(y + off) << 21) | uint64_t(x + off);
}

const int kCorner[8][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {1, 1, 0},
                           {0, 0, 1}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}};

cronos_status build_body(const cronos_lattice_desc& d, int64_t v0, int64_t v1, Body& out) {
    const int64_t nv = v1 - v0;
    if (nv <= 0) return cronos::fail(CRONOS_EINVAL, "lattice: empty body");
    // canonical voxel order: (z, y, x)
    std::vector<std::pair<uint64_t, int64_t>> vk(nv);
    for (int64_t i = 0; i < nv; ++i) {
        const int32_t* c = d.voxels + 3 * (v0 + i);
        for (int a = 0; a < 3; ++a)
            if (c[a] <= -(1 << 20) + 1 || c[a] >= (1 << 20) - 1)
                return cronos::fail(CRONOS_EINVAL, "lattice: voxel coordinate out of range");
        vk[i] = {pack(c[0], c[1], c[2]), v0 + i};
    }
    std::sort(vk.begin(), vk.end());
    for (int64_t i = 1; i < nv; ++i)
        if (vk[i].first == vk[i - 1].first) return cronos::fail(CRONOS_EINVAL, "lattice: duplicate voxel");

    // corners -> distinct nodes in canonical order
    std::vector<uint64_t> ck(8 * nv);
    for (int64_t i = 0; i < nv; ++i) {
        const int32_t* c = d.voxels + 3 * vk[i].second;
        for (int q = 0; q < 8; ++q)
            ck[8 * i + q] = pack(c[0] + kCorner[q][0], c[1] + kCorner[q][1], c[2] + kCorner[q][2]);
    }
    std::vector<uint64_t> nodes(ck);
    std::sort(nodes.begin(), nodes.end());
    nodes.erase(std::unique(nodes.begin(), nodes.end()), nodes.end());
    const int64_t nn = (int64_t)nodes.size();
    if (nn >= (int64_t(1) << 31)) return cronos::fail(CRONOS_EINVAL, "lattice: too many nodes");
    std::vector<int32_t> cnode(8 * nv);
    for (int64_t i = 0; i < 8 * nv; ++i)
        cnode[i] = (int32_t)(std::lower_bound(nodes.begin(), nodes.end(), ck[i]) - nodes.begin());

    out.coords.resize(3 * nn);
    const int64_t off = int64_t(1) << 20, m21 = (int64_t(1) << 21) - 1;
    for (int64_t i = 0; i < nn; ++i) {
        out.coords[3 * i + 0] = (int32_t)((int64_t)(nodes[i] & m21) - off);
        out.coords[3 * i + 1] = (int32_t)((int64_t)((nodes[i] >> 21) & m21) - off);
        out.coords[3 * i + 2] = (int32_t)((int64_t)(nodes[i] >> 42) - off);
    }

    // links in (voxel, corner pair) order -> springs sorted by (lo, hi)
    struct Link { uint64_t key; int64_t voxel; int type; };
    std::vector<Link> links;
    links.reserve(28 * nv);
    for (int64_t i = 0; i < nv; ++i)
        for (int c1 = 0; c1 < 8; ++c1)
            for (int c2 = c1 + 1; c2 < 8; ++c2) {
                int32_t a = cnode[8 * i + c1], b = cnode[8 * i + c2];
                int32_t lo = std::min(a, b), hi = std::max(a, b);
                int type = (kCorner[c1][0] != kCorner[c2][0]) + (kCorner[c1][1] != kCorner[c2][1]) +
                           (kCorner[c1][2] != kCorner[c2][2]);
                links.push_back({(uint64_t(lo) << 32) | uint64_t(hi), i, type});
            }
    // stable: keeps (voxel, pair) order among equal keys -> the assembly sums in voxel order
    std::stable_sort(links.begin(), links.end(), [](const Link& p, const Link& q) { return p.key < q.key; });

    const int32_t* vmat = d.material;
    const int32_t* vgrp = d.group;
    const double weight[4] = {0.0, 0.25, 0.5, 1.0};
    size_t L = links.size();
    for (size_t a = 0; a < L;) {
        size_t b = a;
        while (b < L && links[b].key == links[a].key) ++b;
        int32_t lo = int32_t(links[a].key >> 32), hi = int32_t(links[a].key & 0xffffffffu);
        out.ends.push_back(lo);
        out.ends.push_back(hi);
        int type = links[a].type;
        out.rest.push_back(d.spacing * std::sqrt((double)type));
        double kk;
        if (d.k_mode == CRONOS_K_UNIFORM) {
            kk = d.k_uniform;
        } else {
            kk = 0.0;
            for (size_t q = a; q < b; ++q) {
                int32_t m = vmat ? vmat[vk[links[q].voxel].second] : 0;
                kk = kk + d.material_k[m] * weight[type];
            }
        }
        out.k.push_back(kk);
        int16_t g = -1;
        if (vgrp) {
            int64_t best = -1;
            for (size_t q = a; q < b; ++q) {
                int32_t gv = vgrp[vk[links[q].voxel].second];
                if (gv >= 0 && (best < 0 || links[q].voxel < best)) best = links[q].voxel;
            }
            if (best >= 0) g = (int16_t)vgrp[vk[best].second];
        }
        out.group.push_back(g);
        a = b;
    }

    out.mass.assign(nn, 0.0);
    if (d.mass_mode == CRONOS_MASS_UNIFORM) {
        for (int64_t i = 0; i < nn; ++i) out.mass[i] = d.mass_value;
    } else {
        const double m_corner = d.density * d.spacing * d.spacing * d.spacing / 8.0;
        std::vector<int64_t> count(nn, 0);
        for (int64_t i = 0; i < 8 * nv; ++i) count[cnode[i]]++;
        for (int64_t i = 0; i < nn; ++i) out.mass[i] = (double)count[i] * m_corner;
    }
    out.x.resize(3 * nn);
    for (int64_t i = 0; i < nn; ++i)
        for (int a = 0; a < 3; ++a) {
            double p = d.spacing * (double)out.coords[3 * i + a];
            out.x[3 * i + a] = d.origin[a] + p;
        }
    out.pinned.assign(nn, 0);
    if (d.pin_axis >= 0) {
        int32_t mn = out.coords[d.pin_axis];
        for (int64_t i = 0; i < nn; ++i) mn = std::min(mn, out.coords[3 * i + d.pin_axis]);
        for (int64_t i = 0; i < nn; ++i) out.pinned[i] = (out.coords[3 * i + d.pin_axis] - mn) == d.pin_index;
    }
    return CRONOS_OK;
}

}  // namespace

struct cronos_lattice_t {
    std::vector<Body> bodies;
    int64_t n = 0, s = 0;
};

extern "C" cronos_status cronos_lattice_build(const cronos_lattice_desc* d, cronos_lattice* out) {
    cronos::clear_error();
    if (!d || !out) return cronos::fail(CRONOS_EINVAL, "lattice: NULL argument");
    *out = nullptr;
    if (d->n_bodies < 1 || d->n_voxels < 1 || !d->voxels)
        return cronos::fail(CRONOS_EINVAL, "lattice: need >= 1 body and voxels");
    if (d->n_bodies > 1 && !d->body_voxel_offset)
        return cronos::fail(CRONOS_EINVAL, "lattice: body_voxel_offset required for several bodies");
    if (!(d->spacing > 0.0) || !std::isfinite(d->spacing)) return cronos::fail(CRONOS_EINVAL, "lattice: spacing must be > 0");
    if (d->mass_mode != CRONOS_MASS_UNIFORM && d->mass_mode != CRONOS_MASS_LUMPED)
        return cronos::fail(CRONOS_EINVAL, "lattice: bad mass_mode");
    if (d->k_mode != CRONOS_K_UNIFORM && d->k_mode != CRONOS_K_ASSEMBLY)
        return cronos::fail(CRONOS_EINVAL, "lattice: bad k_mode");
    if (d->k_mode == CRONOS_K_ASSEMBLY && (d->n_materials < 1 || !d->material_k))
        return cronos::fail(CRONOS_EINVAL, "lattice: assembly needs material_k");
    if (d->pin_axis < -1 || d->pin_axis > 2) return cronos::fail(CRONOS_EINVAL, "lattice: bad pin_axis");
    if (d->material) {
        for (int64_t i = 0; i < d->n_voxels; ++i)
            if (d->material[i] < 0 || (d->k_mode == CRONOS_K_ASSEMBLY && d->material[i] >= d->n_materials))
                return cronos::fail(CRONOS_EINVAL, "lattice: material index out of range");
    }
    if (d->group) {
        for (int64_t i = 0; i < d->n_voxels; ++i)
            if (d->group[i] < -1 || d->group[i] > 32767) return cronos::fail(CRONOS_EINVAL, "lattice: group out of range");
    }
    for (int32_t b = 0; b < d->n_bodies; ++b) {
        int64_t v0 = d->body_voxel_offset ? d->body_voxel_offset[b] : 0;
        int64_t v1 = d->body_voxel_offset ? d->body_voxel_offset[b + 1] : d->n_voxels;
        if (v0 < 0 || v1 > d->n_voxels || v1 < v0) return cronos::fail(CRONOS_EINVAL, "lattice: bad body_voxel_offset");
    }
    auto* lat = new (std::nothrow) cronos_lattice_t;
    if (!lat) return cronos::fail(CRONOS_ENOMEM, "lattice: out of memory");
    // bodies are independent: build them on several host threads, report the first failure
    std::vector<cronos_status> status(d->n_bodies, CRONOS_OK);
    std::vector<std::string> errors(d->n_bodies);
    try {
        lat->bodies.resize(d->n_bodies);
        cronos::parallel_for(d->n_bodies, [&](int64_t b0, int64_t b1) {
            for (int64_t b = b0; b < b1; ++b) {
                int64_t v0 = d->body_voxel_offset ? d->body_voxel_offset[b] : 0;
                int64_t v1 = d->body_voxel_offset ? d->body_voxel_offset[b + 1] : d->n_voxels;
                try {
                    status[b] = build_body(*d, v0, v1, lat->bodies[b]);
                } catch (const std::bad_alloc&) {
                    status[b] = CRONOS_ENOMEM;
                }
                if (status[b] != CRONOS_OK) errors[b] = cronos_last_error();
            }
        }, 1);
    } catch (const std::bad_alloc&) {
        delete lat;
        return cronos::fail(CRONOS_ENOMEM, "lattice: out of memory");
    }
    for (int32_t b = 0; b < d->n_bodies; ++b) {
        if (status[b] != CRONOS_OK) {
            delete lat;
            return cronos::fail(status[b], "%s (body %d)", errors[b].empty() ? "lattice: out of memory" : errors[b].c_str(), b);
        }
        lat->n += (int64_t)lat->bodies[b].mass.size();
        lat->s += (int64_t)lat->bodies[b].k.size();
    }
    if (lat->n >= (int64_t(1) << 31)) {
        delete lat;
        return cronos::fail(CRONOS_EINVAL, "lattice: more than 2^31 masses");
    }
    *out = lat;
    return CRONOS_OK;
}

extern "C" cronos_status cronos_lattice_sizes(cronos_lattice lat, int64_t* n, int64_t* s) {
    if (!lat) return cronos::fail(CRONOS_EINVAL, "lattice: NULL handle");
    if (n) *n = lat->n;
    if (s) *s = lat->s;
    return CRONOS_OK;
}

extern "C" cronos_status cronos_lattice_export(cronos_lattice lat, int32_t* coords, double* x, double* mass,
                                               uint8_t* pinned, int64_t* body_offset, int32_t* ends,
                                               double* k, double* rest, int16_t* group) {
    if (!lat) return cronos::fail(CRONOS_EINVAL, "lattice: NULL handle");
    int64_t no = 0, so = 0;
    if (body_offset) body_offset[0] = 0;
    for (size_t b = 0; b < lat->bodies.size(); ++b) {
        const Body& B = lat->bodies[b];
        int64_t nn = (int64_t)B.mass.size(), ns = (int64_t)B.k.size();
        if (coords) std::memcpy(coords + 3 * no, B.coords.data(), 3 * nn * sizeof(int32_t));
        if (x) std::memcpy(x + 3 * no, B.x.data(), 3 * nn * sizeof(double));
        if (mass) std::memcpy(mass + no, B.mass.data(), nn * sizeof(double));
        if (pinned) std::memcpy(pinned + no, B.pinned.data(), nn);
        if (ends)
            for (int64_t i = 0; i < 2 * ns; ++i) ends[2 * so + i] = B.ends[i] + (int32_t)no;
        if (k) std::memcpy(k + so, B.k.data(), ns * sizeof(double));
        if (rest) std::memcpy(rest + so, B.rest.data(), ns * sizeof(double));
        if (group) std::memcpy(group + so, B.group.data(), ns * sizeof(int16_t));
        no += nn;
        so += ns;
        if (body_offset) body_offset[b + 1] = no;
    }
    return CRONOS_OK;
}

extern "C" void cronos_lattice_destroy(cronos_lattice lat) { delete lat; }
