// Eigenvalues of the symmetric tridiagonal matrices that the Lanczos iterations of
// cronos_natural_frequencies build: Sturm-sequence bisection for the smallest ones and
// inverse iteration for the last component of their eigenvectors (the Lanczos residual).
#include <cmath>

#include "common.h"

namespace cronos {

// Number of eigenvalues of T below x (T: diagonal a[0..k), off-diagonal b[0..k-1), b2 = b^2).
// The ratios of the LDL^T factorisation of T - x I count the negative pivots; a zero pivot
// is replaced by a tiny one, which moves x by far less than the bisection tolerance.
int64_t sturm_count(const double* a, const double* b2, int64_t k, double x, double tiny) {
    int64_t count = 0;
    double q = a[0] - x;
    for (int64_t i = 0;; ++i) {
        if (std::fabs(q) < tiny) q = -tiny;
        if (q < 0.0) ++count;
        if (i + 1 == k) break;
        q = (a[i + 1] - x) - b2[i] / q;
    }
    return count;
}

// Gershgorin interval [lo, hi] holding every eigenvalue of T.
void gershgorin(const double* a, const double* b, int64_t k, double* lo, double* hi) {
    double l = a[0], h = a[0];
    for (int64_t i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
        l = std::min(l, a[i] - r);
        h = std::max(h, a[i] + r);
    }
    *lo = l;
    *hi = h;
}

// The index-th smallest eigenvalue (0-based) of T by bisection within [lo, hi].
double tridiag_eigenvalue(const double* a, const double* b2, int64_t k, int64_t index, double lo, double hi,
                          double tiny) {
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;  // interval at one ulp
        if (sturm_count(a, b2, k, mid, tiny) > index) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// |last component| of the unit eigenvector of T for the eigenvalue approximation theta: two
// steps of inverse iteration, (T - theta I) z = z_prev solved by Gaussian elimination with
// partial pivoting (the band then has two super-diagonals).
double eigvec_last_component(const double* a, const double* b, int64_t k, double theta, double tiny) {
    if (k == 1) return 1.0;
    std::vector<double> dd(k), dl(k - 1), du(k - 1), du2(k > 2 ? k - 2 : 1, 0.0), z(k, 1.0 / std::sqrt((double)k));
    std::vector<char> swapped(k - 1, 0);
    for (int64_t i = 0; i < k; ++i) dd[i] = a[i] - theta;
    for (int64_t i = 0; i + 1 < k; ++i) dl[i] = du[i] = b[i];
    for (int64_t i = 0; i + 1 < k; ++i) {
        if (std::fabs(dd[i]) >= std::fabs(dl[i])) {
            if (std::fabs(dd[i]) < tiny) dd[i] = tiny;
            const double m = dl[i] / dd[i];
            dl[i] = m;
            dd[i + 1] -= m * du[i];
            if (i + 2 < k) du2[i] = 0.0;
        } else {
            const double m = dd[i] / dl[i];
            dd[i] = dl[i];
            dl[i] = m;
            const double t = du[i];
            du[i] = dd[i + 1];
            dd[i + 1] = t - m * dd[i + 1];
            if (i + 2 < k) {
                du2[i] = du[i + 1];
                du[i + 1] = -m * du[i + 1];
            }
            swapped[i] = 1;
        }
    }
    if (std::fabs(dd[k - 1]) < tiny) dd[k - 1] = tiny;
    for (int rep = 0; rep < 2; ++rep) {
        // forward: apply the row swaps and multipliers (L^-1 P)
        for (int64_t i = 0; i + 1 < k; ++i) {
            if (swapped[i]) std::swap(z[i], z[i + 1]);
            z[i + 1] -= dl[i] * z[i];
        }
        // back substitution with U (diagonal dd, super-diagonals du, du2)
        z[k - 1] /= dd[k - 1];
        z[k - 2] = (z[k - 2] - du[k - 2] * z[k - 1]) / dd[k - 2];
        for (int64_t i = k - 3; i >= 0; --i) z[i] = (z[i] - du[i] * z[i + 1] - du2[i] * z[i + 2]) / dd[i];
        double nrm = 0.0, big = 0.0;
        for (int64_t i = 0; i < k; ++i) big = std::max(big, std::fabs(z[i]));
        if (!(big > 0.0) || !std::isfinite(big)) return 1.0;
        for (int64_t i = 0; i < k; ++i) {
            z[i] /= big;
            nrm += z[i] * z[i];
        }
        nrm = std::sqrt(nrm);
        for (int64_t i = 0; i < k; ++i) z[i] /= nrm;
    }
    return std::fabs(z[k - 1]);
}

}  // namespace cronos

extern "C" cronos_status cronos_tridiag_smallest(int64_t k, const double* a, const double* b, int64_t count,
                                                 double* theta, double* last) {
    cronos::clear_error();
    if (k < 1 || count < 1 || count > k) return cronos::fail(CRONOS_EINVAL, "tridiag_smallest: need 1 <= count <= k");
    if (!a || !theta || (k > 1 && !b)) return cronos::fail(CRONOS_EINVAL, "tridiag_smallest: NULL argument");
    for (int64_t i = 0; i < k; ++i)
        if (!std::isfinite(a[i]) || (i + 1 < k && !std::isfinite(b[i])))
            return cronos::fail(CRONOS_EINVAL, "tridiag_smallest: non-finite entry");
    const double zero = 0.0;
    const double* bb = k > 1 ? b : &zero;
    std::vector<double> b2(k > 1 ? k - 1 : 1, 0.0);
    for (int64_t i = 0; i + 1 < k; ++i) b2[i] = bb[i] * bb[i];
    double lo, hi;
    cronos::gershgorin(a, bb, k, &lo, &hi);
    const double norm = std::max({std::fabs(lo), std::fabs(hi), 1e-300});
    double lower = lo;
    for (int64_t j = 0; j < count; ++j) {
        theta[j] = cronos::tridiag_eigenvalue(a, b2.data(), k, j, lower, hi, 1e-300);
        lower = std::max(lo, theta[j] - 4e-16 * norm);
        if (last) last[j] = cronos::eigvec_last_component(a, bb, k, theta[j], 1e-15 * norm);
    }
    return CRONOS_OK;
}
