// dense.hpp - small dense complex linear algebra on the host for the outer solver's
// restarts (matrices of order <= 17): least squares through Givens QR, LU solves, and a
// complex Schur decomposition with eigenvalues reordered by modulus. Column-major
// storage: element (i, j) of an n-row matrix is a[i + n * j].
#pragma once
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace sapdd {
namespace dense {

typedef std::complex<double> cd;

// Unitary rotation [[c, s], [-conj(s), c]] (c real) with G [a; b] = [r; 0].
inline void givens(cd a, cd b, double &c, cd &s) {
    const double na = std::abs(a), nb = std::abs(b);
    if (nb == 0.0) {
        c = 1.0;
        s = 0.0;
        return;
    }
    if (na == 0.0) {
        c = 0.0;
        s = std::conj(b) / nb;
        return;
    }
    const double r = std::hypot(na, nb);
    c = na / r;
    s = (a / na) * std::conj(b) / r;
}

// min |c - H y| for an nr x nc matrix H (nr >= nc, any structure) by Givens QR. y gets
// nc entries; returns the residual norm |c - H y|. H and c are taken by value.
inline double lstsq(int nr, int nc, std::vector<cd> h, std::vector<cd> c, std::vector<cd> &y) {
    for (int j = 0; j < nc; ++j)
        for (int i = j + 1; i < nr; ++i) {
            if (h[i + nr * j] == 0.0) continue;
            double cs;
            cd sn;
            givens(h[j + nr * j], h[i + nr * j], cs, sn);
            for (int q = j; q < nc; ++q) {
                const cd a = h[j + nr * q], b = h[i + nr * q];
                h[j + nr * q] = cs * a + sn * b;
                h[i + nr * q] = -std::conj(sn) * a + cs * b;
            }
            const cd a = c[j], b = c[i];
            c[j] = cs * a + sn * b;
            c[i] = -std::conj(sn) * a + cs * b;
        }
    y.assign(nc, 0.0);
    for (int j = nc - 1; j >= 0; --j) {
        cd t = c[j];
        for (int q = j + 1; q < nc; ++q) t -= h[j + nr * q] * y[q];
        const cd d = h[j + nr * j];
        y[j] = d != 0.0 ? t / d : 0.0;
    }
    double r = 0;
    for (int i = nc; i < nr; ++i) r += std::norm(c[i]);
    return std::sqrt(r);
}

// Solve A x = b (n x n) by LU with partial pivoting; false if A is singular.
inline bool solve(int n, std::vector<cd> a, std::vector<cd> &b) {
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (std::abs(a[i + n * k]) > std::abs(a[p + n * k])) p = i;
        if (a[p + n * k] == 0.0) return false;
        if (p != k) {
            for (int q = 0; q < n; ++q) std::swap(a[k + n * q], a[p + n * q]);
            std::swap(b[k], b[p]);
        }
        for (int i = k + 1; i < n; ++i) {
            const cd f = a[i + n * k] / a[k + n * k];
            if (f == 0.0) continue;
            for (int q = k; q < n; ++q) a[i + n * q] -= f * a[k + n * q];
            b[i] -= f * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        cd t = b[k];
        for (int q = k + 1; q < n; ++q) t -= a[k + n * q] * b[q];
        b[k] = t / a[k + n * k];
    }
    return true;
}

// Apply the rotation to rows (i, i + 1) of t (columns c0..n-1) from the left as G^H and
// to columns (i, i + 1) of t (rows 0..r1) and of q from the right as G, G = [[c, s],
// [-conj(s), c]]^H... written out: the similarity t <- G^H t G with G's first column
// (c, -conj(s))^H.
inline void rotate_similarity(int n, std::vector<cd> &t, std::vector<cd> &q, int i, double c, cd s, int c0,
                              int r1) {
    // rows: [x; y] <- [c x + s y; -conj(s) x + c y]
    for (int col = c0; col < n; ++col) {
        const cd x = t[i + n * col], y = t[i + 1 + n * col];
        t[i + n * col] = c * x + s * y;
        t[i + 1 + n * col] = -std::conj(s) * x + c * y;
    }
    // columns: [x, y] <- [c x + conj(s) y, -s x + c y] (the inverse rotation on the right)
    for (int row = 0; row <= r1; ++row) {
        const cd x = t[row + n * i], y = t[row + n * (i + 1)];
        t[row + n * i] = c * x + std::conj(s) * y;
        t[row + n * (i + 1)] = -s * x + c * y;
    }
    for (int row = 0; row < n; ++row) {
        const cd x = q[row + n * i], y = q[row + n * (i + 1)];
        q[row + n * i] = c * x + std::conj(s) * y;
        q[row + n * (i + 1)] = -s * x + c * y;
    }
}

// Complex Schur form a = q t q^H (t upper triangular, q unitary) with the eigenvalues on
// the diagonal of t in ascending modulus. a is overwritten by t. Householder reduction to
// Hessenberg form, then shifted QR steps (Wilkinson shift, Givens rotations) with
// deflation at negligible subdiagonal entries, then adjacent swaps of diagonal entries
// (each a rotation that takes the second eigenvector of a 2x2 triangle to the front).
// Returns false if the QR iteration does not converge.
inline bool schur_sorted(int n, std::vector<cd> &a, std::vector<cd> &q) {
    q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) q[i + n * i] = 1.0;
    // Hessenberg reduction
    for (int k = 0; k + 2 < n; ++k) {
        double alpha2 = 0;
        for (int i = k + 1; i < n; ++i) alpha2 += std::norm(a[i + n * k]);
        const double alpha = std::sqrt(alpha2);
        if (alpha == 0.0) continue;
        const cd x0 = a[k + 1 + n * k];
        const cd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1.0);
        std::vector<cd> v(n, 0.0);
        v[k + 1] = x0 + ph * alpha;
        for (int i = k + 2; i < n; ++i) v[i] = a[i + n * k];
        double vn2 = 0;
        for (int i = k + 1; i < n; ++i) vn2 += std::norm(v[i]);
        if (vn2 == 0.0) continue;
        // a <- (1 - 2 v v^H / |v|^2) a (1 - 2 v v^H / |v|^2), q <- q (1 - 2 v v^H / |v|^2)
        for (int col = 0; col < n; ++col) {
            cd d = 0;
            for (int i = k + 1; i < n; ++i) d += std::conj(v[i]) * a[i + n * col];
            d *= 2.0 / vn2;
            for (int i = k + 1; i < n; ++i) a[i + n * col] -= v[i] * d;
        }
        for (int row = 0; row < n; ++row) {
            cd d = 0;
            for (int i = k + 1; i < n; ++i) d += a[row + n * i] * v[i];
            d *= 2.0 / vn2;
            for (int i = k + 1; i < n; ++i) a[row + n * i] -= d * std::conj(v[i]);
            cd e = 0;
            for (int i = k + 1; i < n; ++i) e += q[row + n * i] * v[i];
            e *= 2.0 / vn2;
            for (int i = k + 1; i < n; ++i) q[row + n * i] -= e * std::conj(v[i]);
        }
        for (int i = k + 2; i < n; ++i) a[i + n * k] = 0.0;
    }
    // shifted QR on the active window [lo, hi]
    const double eps = 2.220446049250313e-16;
    int hi = n - 1, iter = 0;
    while (hi > 0) {
        if (++iter > 100 * n) return false;
        int lo = hi;
        while (lo > 0) {
            const double sub = std::abs(a[lo + n * (lo - 1)]);
            if (sub <= eps * (std::abs(a[lo + n * lo]) + std::abs(a[lo - 1 + n * (lo - 1)]))) {
                a[lo + n * (lo - 1)] = 0.0;
                break;
            }
            --lo;
        }
        if (lo == hi) {
            --hi;
            continue;
        }
        // Wilkinson shift from the trailing 2x2 block of the window
        const cd p = a[hi - 1 + n * (hi - 1)], r = a[hi - 1 + n * hi], s2 = a[hi + n * (hi - 1)],
                 u = a[hi + n * hi];
        const cd tr = p + u, det = p * u - r * s2;
        const cd disc = std::sqrt(tr * tr / 4.0 - det);
        const cd l1 = tr / 2.0 + disc, l2 = tr / 2.0 - disc;
        cd mu = std::abs(l1 - u) < std::abs(l2 - u) ? l1 : l2;
        if (iter % 11 == 10) mu += std::abs(a[hi + n * (hi - 1)]);  // exceptional shift
        // explicit QR step on the window: t - mu = G^H R, t <- R G + mu, as a chain of
        // similarity rotations (chasing the bulge from the first rotation)
        for (int i = lo; i < hi; ++i) {
            cd x, y;
            if (i == lo) {
                x = a[lo + n * lo] - mu;
                y = a[lo + 1 + n * lo];
            } else {
                x = a[i + n * (i - 1)];
                y = a[i + 1 + n * (i - 1)];
            }
            double c;
            cd s;
            givens(x, y, c, s);
            rotate_similarity(n, a, q, i, c, s, i == lo ? lo : i - 1, std::min(i + 2, hi));
            if (i > lo) a[i + 1 + n * (i - 1)] = 0.0;
        }
    }
    for (int j = 0; j < n; ++j)
        for (int i = j + 1; i < n; ++i) a[i + n * j] = 0.0;
    // bubble the eigenvalues into ascending modulus
    for (int pass = 0; pass < n; ++pass) {
        bool swapped = false;
        for (int i = 0; i + 1 < n; ++i) {
            const cd ta = a[i + n * i], tb = a[i + 1 + n * (i + 1)], tt = a[i + n * (i + 1)];
            if (!(std::abs(tb) < std::abs(ta))) continue;
            // eigenvector of tb in the 2x2 triangle: (tt, tb - ta)
            double c;
            cd s;
            givens(tt, tb - ta, c, s);
            // the rotation whose first column is that vector: G = [[c, -s]; [conj(s), c]]^...
            // applied as the similarity with G^H rows = [[c, s]; [-conj(s), c]]
            rotate_similarity(n, a, q, i, c, s, i, std::min(i + 1, n - 1));
            a[i + 1 + n * i] = 0.0;
            swapped = true;
        }
        if (!swapped) break;
    }
    return true;
}

}  // namespace dense
}  // namespace sapdd
