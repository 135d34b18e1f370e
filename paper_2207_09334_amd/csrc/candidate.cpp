// Quasi-uniform lattices by best-candidate sampling (section "Generating a Lattice": Mitchell's
// best-candidate algorithm with k nearest neighbours) and distance-cutoff springs.
//
// Random draws: the counter hash h(seed, stream, keys...) = SplitMix64 chained over the keys
// (Steele, Lea & Flood, OOPSLA 2014), uniform = top 53 bits * 2^-53; candidate c of point p
// has coordinate a = size[a] * uniform(h(seed, 8, p, c, a)).
//
// Nearest-neighbour queries use a uniform grid of the placed points (cell ~ the expected point
// spacing), searched in growing cubic shells until no unvisited cell can hold a point nearer
// than the current k-th; the result is the exact k nearest, so the choice is the same as a
// brute-force search computing the same distances in the same order.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "common.h"

namespace {

constexpr uint64_t kStreamCandidate = 8;

inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

inline double uniform01(uint64_t seed, uint64_t p, uint64_t c, uint64_t a) {
    uint64_t z = splitmix64(seed);
    z = splitmix64(z ^ kStreamCandidate);
    z = splitmix64(z ^ p);
    z = splitmix64(z ^ c);
    z = splitmix64(z ^ a);
    return (double)(z >> 11) * 0x1p-53;
}

inline double dist(const double* a, const double* b) {
    const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return std::sqrt(dx * dx + dy * dy + dz * dz);
}

struct Grid {
    double h;
    int64_t dim[3];
    std::vector<std::vector<int64_t>> cells;
    Grid(const double size[3], double cell) : h(cell) {
        for (int a = 0; a < 3; ++a) dim[a] = std::max<int64_t>(1, (int64_t)std::ceil(size[a] / cell));
        cells.resize((size_t)(dim[0] * dim[1] * dim[2]));
    }
    int64_t coord(double v, int a) const {
        return std::min<int64_t>(dim[a] - 1, std::max<int64_t>(0, (int64_t)std::floor(v / h)));
    }
    std::vector<int64_t>& at(int64_t x, int64_t y, int64_t z) { return cells[(size_t)((z * dim[1] + y) * dim[0] + x)]; }
};

// Sum, in ascending order, of the distances from q to its k nearest points (k <= placed).
double knn_score(Grid& g, const double* pts, const double* q, int k, std::vector<double>& best) {
    best.clear();
    const int64_t c[3] = {g.coord(q[0], 0), g.coord(q[1], 1), g.coord(q[2], 2)};
    const int64_t maxr = std::max({g.dim[0], g.dim[1], g.dim[2]});
    for (int64_t r = 0; r <= maxr; ++r) {
        // stop once the k-th best is no farther than any point of shell r can be
        if ((int)best.size() == k && best.back() <= (double)(r - 1) * g.h) break;
        for (int64_t z = c[2] - r; z <= c[2] + r; ++z) {
            if (z < 0 || z >= g.dim[2]) continue;
            for (int64_t y = c[1] - r; y <= c[1] + r; ++y) {
                if (y < 0 || y >= g.dim[1]) continue;
                for (int64_t x = c[0] - r; x <= c[0] + r; ++x) {
                    if (x < 0 || x >= g.dim[0]) continue;
                    if (std::max({std::llabs(x - c[0]), std::llabs(y - c[1]), std::llabs(z - c[2])}) != r) continue;
                    for (int64_t j : g.at(x, y, z)) {
                        const double d = dist(q, pts + 3 * j);
                        if ((int)best.size() < k) {
                            best.insert(std::upper_bound(best.begin(), best.end(), d), d);
                        } else if (d < best.back()) {
                            best.pop_back();
                            best.insert(std::upper_bound(best.begin(), best.end(), d), d);
                        }
                    }
                }
            }
        }
    }
    double s = 0.0;
    for (double d : best) s += d;
    return s;
}

}  // namespace

extern "C" cronos_status cronos_candidate_points(const double* size, int64_t n_points, int32_t n_candidates,
                                                 int32_t k_nn, uint64_t seed, double* points) {
    cronos::clear_error();
    if (!size || !points || n_points < 1 || n_candidates < 1 || k_nn < 1 || k_nn > 64)
        return cronos::fail(CRONOS_EINVAL, "candidate_points: bad arguments");
    for (int a = 0; a < 3; ++a)
        if (!(size[a] > 0.0) || !std::isfinite(size[a])) return cronos::fail(CRONOS_EINVAL, "candidate_points: bad size");
    try {
        // the grid's cell follows the spacing of the points placed so far: rebuilt whenever
        // their number has doubled, so a query visits O(1) cells at every stage
        const double volume = size[0] * size[1] * size[2];
        auto build = [&](int64_t placed) {
            Grid g(size, std::cbrt(volume / (double)std::max<int64_t>(placed, k_nn)));
            for (int64_t j = 0; j < placed; ++j)
                g.at(g.coord(points[3 * j], 0), g.coord(points[3 * j + 1], 1), g.coord(points[3 * j + 2], 2)).push_back(j);
            return g;
        };
        std::vector<double> best;
        best.reserve(k_nn + 1);
        for (int a = 0; a < 3; ++a) points[a] = size[a] * uniform01(seed, 0, 0, (uint64_t)a);
        Grid g = build(1);
        int64_t next_build = 2 * std::max<int64_t>(k_nn, 1);
        for (int64_t p = 1; p < n_points; ++p) {
            if (p >= next_build) {
                g = build(p);
                next_build = 2 * p;
            }
            const int k = (int)std::min<int64_t>(k_nn, p);
            double top = -1.0, q[3], pick[3] = {0.0, 0.0, 0.0};
            for (int32_t c = 0; c < n_candidates; ++c) {
                for (int a = 0; a < 3; ++a) q[a] = size[a] * uniform01(seed, (uint64_t)p, (uint64_t)c, (uint64_t)a);
                const double sc = knn_score(g, points, q, k, best);
                if (sc > top) {  // strict: ties keep the lowest candidate index
                    top = sc;
                    pick[0] = q[0];
                    pick[1] = q[1];
                    pick[2] = q[2];
                }
            }
            for (int a = 0; a < 3; ++a) points[3 * p + a] = pick[a];
            g.at(g.coord(pick[0], 0), g.coord(pick[1], 1), g.coord(pick[2], 2)).push_back(p);
        }
    } catch (const std::bad_alloc&) {
        return cronos::fail(CRONOS_ENOMEM, "candidate_points: out of memory");
    }
    return CRONOS_OK;
}

extern "C" cronos_status cronos_cutoff_springs(int64_t n_points, const double* points, double cutoff,
                                               int64_t max_springs, int32_t* ends, int64_t* n_springs) {
    cronos::clear_error();
    if (n_points < 1 || n_points >= (int64_t(1) << 31) || !points || !n_springs || !(cutoff > 0.0) ||
        (max_springs > 0 && !ends))
        return cronos::fail(CRONOS_EINVAL, "cutoff_springs: bad arguments");
    try {
        double lo[3], hi[3];
        for (int a = 0; a < 3; ++a) lo[a] = hi[a] = points[a];
        for (int64_t i = 0; i < n_points; ++i)
            for (int a = 0; a < 3; ++a) {
                if (!std::isfinite(points[3 * i + a])) return cronos::fail(CRONOS_EINVAL, "cutoff_springs: non-finite point");
                lo[a] = std::min(lo[a], points[3 * i + a]);
                hi[a] = std::max(hi[a], points[3 * i + a]);
            }
        const double size[3] = {hi[0] - lo[0] + cutoff, hi[1] - lo[1] + cutoff, hi[2] - lo[2] + cutoff};
        Grid g(size, cutoff);
        std::vector<double> rel(3 * (size_t)n_points);
        for (int64_t i = 0; i < n_points; ++i) {
            for (int a = 0; a < 3; ++a) rel[3 * i + a] = points[3 * i + a] - lo[a];
            g.at(g.coord(rel[3 * i], 0), g.coord(rel[3 * i + 1], 1), g.coord(rel[3 * i + 2], 2)).push_back(i);
        }
        const double c2 = cutoff * cutoff;
        // per point i, the partners j > i within the cutoff, in increasing j
        std::vector<std::vector<int32_t>> nb(n_points);
        cronos::parallel_for(n_points, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) {
                const double* pi = points + 3 * i;
                const int64_t c[3] = {g.coord(rel[3 * i], 0), g.coord(rel[3 * i + 1], 1), g.coord(rel[3 * i + 2], 2)};
                for (int64_t z = std::max<int64_t>(0, c[2] - 1); z <= std::min(g.dim[2] - 1, c[2] + 1); ++z)
                    for (int64_t y = std::max<int64_t>(0, c[1] - 1); y <= std::min(g.dim[1] - 1, c[1] + 1); ++y)
                        for (int64_t x = std::max<int64_t>(0, c[0] - 1); x <= std::min(g.dim[0] - 1, c[0] + 1); ++x)
                            for (int64_t j : g.at(x, y, z)) {
                                if (j <= i) continue;
                                const double* pj = points + 3 * j;
                                const double dx = pi[0] - pj[0], dy = pi[1] - pj[1], dz = pi[2] - pj[2];
                                if (dx * dx + dy * dy + dz * dz <= c2) nb[i].push_back((int32_t)j);
                            }
                std::sort(nb[i].begin(), nb[i].end());
            }
        }, 1024);
        int64_t s = 0;
        for (int64_t i = 0; i < n_points; ++i) {
            for (int32_t j : nb[i]) {
                if (s < max_springs) {
                    ends[2 * s] = (int32_t)i;
                    ends[2 * s + 1] = j;
                }
                ++s;
            }
        }
        *n_springs = s;
        if (s > max_springs && max_springs > 0)
            return cronos::fail(CRONOS_EINVAL, "cutoff_springs: %lld springs exceed max_springs", (long long)s);
    } catch (const std::bad_alloc&) {
        return cronos::fail(CRONOS_ENOMEM, "cutoff_springs: out of memory");
    }
    return CRONOS_OK;
}

extern "C" cronos_status cronos_point_params(int64_t n_points, const double* points, int64_t n_springs,
                                             const int32_t* ends, double k_ref, double length_ref,
                                             double mass_per_point, int32_t pin_axis, double pin_below, double* k,
                                             double* rest, double* mass, uint8_t* pinned) {
    cronos::clear_error();
    if (n_points < 1 || !points || n_springs < 0 || (n_springs > 0 && !ends) || !(k_ref > 0.0) ||
        !(length_ref > 0.0) || !(mass_per_point > 0.0) || pin_axis < -1 || pin_axis > 2 ||
        !std::isfinite(k_ref * length_ref) || !std::isfinite(mass_per_point))
        return cronos::fail(CRONOS_EINVAL, "point_params: bad arguments");
    for (int64_t s = 0; s < n_springs; ++s) {
        const int64_t i = ends[2 * s], j = ends[2 * s + 1];
        if (i < 0 || j < 0 || i >= n_points || j >= n_points || i == j)
            return cronos::fail(CRONOS_EINVAL, "point_params: spring %lld has bad ends", (long long)s);
        const double dx = points[3 * j] - points[3 * i], dy = points[3 * j + 1] - points[3 * i + 1],
                     dz = points[3 * j + 2] - points[3 * i + 2];
        // the spring's initial length is its rest length; its stiffness scales inversely to it
        const double len = std::sqrt((dx * dx + dy * dy) + dz * dz);
        if (!(len > 0.0) || !std::isfinite(len))
            return cronos::fail(CRONOS_EINVAL, "point_params: spring %lld has zero or non-finite length", (long long)s);
        if (rest) rest[s] = len;
        if (k) k[s] = (k_ref * length_ref) / len;
    }
    for (int64_t i = 0; i < n_points; ++i) {
        if (mass) mass[i] = mass_per_point;
        if (pinned) pinned[i] = pin_axis >= 0 && points[3 * i + pin_axis] < pin_below ? 1 : 0;
    }
    return CRONOS_OK;
}
