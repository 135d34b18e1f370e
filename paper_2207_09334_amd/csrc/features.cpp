// Surrogate input features of a voxel robot: 32 morphology descriptors followed by the
// actuation parameters as (A_g cos phi_g, A_g sin phi_g) per group.
//
// Morphology (lengths in metres, voxel centres c relative to the body's minimum corner):
//   0 log(node count)  1 log(voxel count)  2-4 extent per axis  5-7 fraction of materials 0,1,2
//   8-10 centre of voxel centres minus bbox centre  11-16 second moments about that centre
//   (xx, yy, zz, xy, xz, yz)  17 fraction of voxels in the bottom layer  18-25 8-bin histogram
//   of voxel height  26 actuated fraction  27 mean log10 of voxel stiffness  28-30 stiffness-
//   weighted centre minus centre  31 fraction of voxel faces on the surface.
#include <algorithm>
#include <cmath>
#include <new>

#include "common.h"

namespace {

inline uint64_t pack(int64_t x, int64_t y, int64_t z) {
    const int64_t off = int64_t(1) << 20;
    return (uint64_t(z + off) << 42) | (uint64_t(y + off) << 21) | uint64_t(x + off);
}

void body_features(const int32_t* vox, const int32_t* mat, const int32_t* grp, int64_t nv, int32_t n_materials,
                   const double* material_k, double a, double* f) {
    int64_t mn[3], mx[3];
    for (int c = 0; c < 3; ++c) mn[c] = mx[c] = vox[c];
    for (int64_t i = 0; i < nv; ++i)
        for (int c = 0; c < 3; ++c) {
            mn[c] = std::min<int64_t>(mn[c], vox[3 * i + c]);
            mx[c] = std::max<int64_t>(mx[c], vox[3 * i + c]);
        }
    std::vector<uint64_t> keys(nv), corners(8 * nv);
    for (int64_t i = 0; i < nv; ++i) {
        const int32_t* v = vox + 3 * i;
        keys[i] = pack(v[0], v[1], v[2]);
        for (int q = 0; q < 8; ++q) corners[8 * i + q] = pack(v[0] + (q & 1), v[1] + ((q >> 1) & 1), v[2] + ((q >> 2) & 1));
    }
    std::sort(keys.begin(), keys.end());
    std::sort(corners.begin(), corners.end());
    const int64_t nodes = std::unique(corners.begin(), corners.end()) - corners.begin();

    double ext[3], com[3] = {0, 0, 0}, frac[3] = {0, 0, 0}, kc[3] = {0, 0, 0};
    double ksum = 0.0, logk = 0.0, bottom = 0.0, actuated = 0.0, hist[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = 0; c < 3; ++c) ext[c] = (double)(mx[c] - mn[c] + 1) * a;
    const int64_t nz = mx[2] - mn[2] + 1;
    for (int64_t i = 0; i < nv; ++i) {
        const int32_t* v = vox + 3 * i;
        const int m = mat ? mat[i] : 0;
        const double k = material_k && m < n_materials ? material_k[m] : 1.0;
        if (m >= 0 && m < 3) frac[m] += 1.0;
        for (int c = 0; c < 3; ++c) {
            const double ctr = ((double)(v[c] - mn[c]) + 0.5) * a;
            com[c] += ctr;
            kc[c] += k * ctr;
        }
        ksum += k;
        logk += std::log10(k);
        if (v[2] == mn[2]) bottom += 1.0;
        if (grp && grp[i] >= 0) actuated += 1.0;
        hist[std::min<int64_t>(7, (8 * (int64_t)(v[2] - mn[2])) / nz)] += 1.0;
    }
    const double inv = 1.0 / (double)nv;
    for (int c = 0; c < 3; ++c) com[c] *= inv;
    double mom[6] = {0, 0, 0, 0, 0, 0};
    int64_t exposed = 0;
    const int dir[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    for (int64_t i = 0; i < nv; ++i) {
        const int32_t* v = vox + 3 * i;
        double d[3];
        for (int c = 0; c < 3; ++c) d[c] = ((double)(v[c] - mn[c]) + 0.5) * a - com[c];
        mom[0] += d[0] * d[0];
        mom[1] += d[1] * d[1];
        mom[2] += d[2] * d[2];
        mom[3] += d[0] * d[1];
        mom[4] += d[0] * d[2];
        mom[5] += d[1] * d[2];
        for (auto& o : dir)
            if (!std::binary_search(keys.begin(), keys.end(), pack(v[0] + o[0], v[1] + o[1], v[2] + o[2]))) ++exposed;
    }
    f[0] = std::log((double)nodes);
    f[1] = std::log((double)nv);
    for (int c = 0; c < 3; ++c) f[2 + c] = ext[c];
    for (int c = 0; c < 3; ++c) f[5 + c] = frac[c] * inv;
    for (int c = 0; c < 3; ++c) f[8 + c] = com[c] - 0.5 * ext[c];
    for (int c = 0; c < 6; ++c) f[11 + c] = mom[c] * inv;
    f[17] = bottom * inv;
    for (int b = 0; b < 8; ++b) f[18 + b] = hist[b] * inv;
    f[26] = actuated * inv;
    f[27] = logk * inv;
    for (int c = 0; c < 3; ++c) f[28 + c] = kc[c] / ksum - com[c];
    f[31] = (double)exposed / (6.0 * (double)nv);
}

}  // namespace

extern "C" cronos_status cronos_features(int32_t n_bodies, const int64_t* body_voxel_offset, const int32_t* voxels,
                                         const int32_t* material, const int32_t* group, int32_t n_materials,
                                         const double* material_k, double spacing, int32_t n_groups,
                                         const double* phase, const double* amp, double* out) {
    cronos::clear_error();
    if (n_bodies < 1 || !voxels || !out || !(spacing > 0.0) || n_groups < 0)
        return cronos::fail(CRONOS_EINVAL, "features: bad arguments");
    if (n_bodies > 1 && !body_voxel_offset) return cronos::fail(CRONOS_EINVAL, "features: body_voxel_offset required");
    if (n_groups > 0 && (!phase || !amp)) return cronos::fail(CRONOS_EINVAL, "features: phase and amp required");
    for (int32_t b = 0; b < n_bodies; ++b) {
        const int64_t v0 = body_voxel_offset ? body_voxel_offset[b] : 0;
        const int64_t v1 = body_voxel_offset ? body_voxel_offset[b + 1] : -1;
        if (body_voxel_offset && v1 <= v0) return cronos::fail(CRONOS_EINVAL, "features: empty body %d", b);
    }
    if (!body_voxel_offset) return cronos::fail(CRONOS_EINVAL, "features: body_voxel_offset required");
    const int width = 32 + 2 * n_groups;
    try {
        cronos::parallel_for(n_bodies, [&](int64_t b0, int64_t b1) {
            for (int64_t b = b0; b < b1; ++b) {
                const int64_t v0 = body_voxel_offset[b], v1 = body_voxel_offset[b + 1];
                double* f = out + b * width;
                body_features(voxels + 3 * v0, material ? material + v0 : nullptr, group ? group + v0 : nullptr, v1 - v0,
                              n_materials, material_k, spacing, f);
                for (int g = 0; g < n_groups; ++g) {
                    const double A = amp[b * n_groups + g], ph = phase[b * n_groups + g];
                    f[32 + 2 * g] = A * std::cos(ph);
                    f[33 + 2 * g] = A * std::sin(ph);
                }
            }
        }, 8);
    } catch (const std::bad_alloc&) {
        return cronos::fail(CRONOS_ENOMEM, "features: out of memory");
    }
    return CRONOS_OK;
}

extern "C" cronos_status cronos_candidate_features(int64_t n_cand, const int32_t* body_of, int32_t n_bodies,
                                                   const double* morph, int32_t n_groups, const double* phase,
                                                   const double* amp, double* out) {
    cronos::clear_error();
    if (n_cand < 0 || n_bodies < 1 || !body_of || !morph || !out || n_groups < 0 || (n_groups && (!phase || !amp)))
        return cronos::fail(CRONOS_EINVAL, "candidate_features: bad arguments");
    for (int64_t c = 0; c < n_cand; ++c)
        if (body_of[c] < 0 || body_of[c] >= n_bodies) return cronos::fail(CRONOS_EINVAL, "candidate_features: bad body index");
    const int width = 32 + 2 * n_groups;
    cronos::parallel_for(n_cand, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c) {
            double* f = out + c * width;
            const double* m = morph + (int64_t)body_of[c] * 32;
            for (int q = 0; q < 32; ++q) f[q] = m[q];
            for (int g = 0; g < n_groups; ++g) {
                const double A = amp[c * n_groups + g], ph = phase[c * n_groups + g];
                f[32 + 2 * g] = A * std::cos(ph);
                f[33 + 2 * g] = A * std::sin(ph);
            }
        }
    }, 4096);
    return CRONOS_OK;
}
