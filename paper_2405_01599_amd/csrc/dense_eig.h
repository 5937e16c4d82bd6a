// Small dense eigenvalue routines for the restarted Arnoldi driver (host
// code, matrices of order <= 64, row-major, element (i, j) at i * n + j).
//
//   schur      real Schur form of an upper Hessenberg matrix by the Francis
//              double-shift QR iteration (Golub and Van Loan, Algorithms
//              7.5.1-7.5.2): H = Z T Z^T, T quasi-upper-triangular with 2 x 2
//              blocks only for complex conjugate pairs (a block with real
//              eigenvalues is split by a rotation).
//   ritz_vec   eigenvector of T for one of its eigenvalues, by back
//              substitution in complex arithmetic.
//   qr_shift1  one implicit single-shift QR step on a Hessenberg matrix
//   qr_shift2  one implicit double-shift QR step (shifts mu, conj(mu)) given
//              s = mu + conj(mu) and t = mu * conj(mu)
// The QR steps are the exact-shift filter of the implicitly restarted
// Arnoldi method (Sorensen 1992): H <- Q^T H Q, Q accumulated.
#pragma once
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace xab {
namespace dense {

using cplx = std::complex<double>;
constexpr double kEps = 2.220446049250313e-16;

// Householder vector for (x, y, z): (I - beta v v^T)(x, y, z)^T = (alpha, 0, 0).
struct House3 {
    double v[3] = {0, 0, 0}, beta = 0;
    House3(double x, double y, double z) {
        const double nr = std::sqrt(x * x + y * y + z * z);
        if (nr == 0.0) return;
        const double alpha = x >= 0 ? -nr : nr;
        v[0] = x - alpha;
        v[1] = y;
        v[2] = z;
        const double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        beta = vv > 0 ? 2.0 / vv : 0.0;
    }
};

// Rows r0, r0+1, r0+2 (or r0, r0+1 when len = 2) of a, columns c0 .. c1-1:
// a <- (I - beta v v^T) a.
inline void house_left(int n, std::vector<double> &a, const double *v, double beta, int len, int r0, int c0,
                       int c1) {
    if (beta == 0.0) return;
    for (int j = c0; j < c1; ++j) {
        double s = 0.0;
        for (int q = 0; q < len; ++q) s += v[q] * a[(size_t)(r0 + q) * n + j];
        s *= beta;
        for (int q = 0; q < len; ++q) a[(size_t)(r0 + q) * n + j] -= s * v[q];
    }
}

// Columns c0 .. c0+len-1 of rows r0 .. r1-1: a <- a (I - beta v v^T).
inline void house_right(int n, std::vector<double> &a, const double *v, double beta, int len, int c0, int r0,
                        int r1) {
    if (beta == 0.0) return;
    for (int i = r0; i < r1; ++i) {
        double s = 0.0;
        for (int q = 0; q < len; ++q) s += a[(size_t)i * n + c0 + q] * v[q];
        s *= beta;
        for (int q = 0; q < len; ++q) a[(size_t)i * n + c0 + q] -= s * v[q];
    }
}

// One Francis double-shift step on the active window [l, hi] of the
// Hessenberg matrix h (order n), shifts the roots of z^2 - s z + t; the
// similarity is applied to whole rows and columns and accumulated in z.
inline void francis_step(int n, std::vector<double> &h, std::vector<double> &zm, int l, int hi, double s,
                         double t) {
    auto H = [&](int i, int j) -> double & { return h[(size_t)i * n + j]; };
    double x = H(l, l) * H(l, l) + H(l, l + 1) * H(l + 1, l) - s * H(l, l) + t;
    double y = H(l + 1, l) * (H(l, l) + H(l + 1, l + 1) - s);
    double z = l + 2 <= hi ? H(l + 1, l) * H(l + 2, l + 1) : 0.0;
    for (int k = l; k <= hi - 2; ++k) {
        House3 P(x, y, z);
        const int c0 = std::max(k - 1, l);
        house_left(n, h, P.v, P.beta, 3, k, c0, n);
        house_right(n, h, P.v, P.beta, 3, k, 0, std::min(k + 4, hi + 1));
        house_right(n, zm, P.v, P.beta, 3, k, 0, n);
        if (k > l) H(k + 1, k - 1) = H(k + 2, k - 1) = 0.0;  // the bulge column is annihilated
        x = H(k + 1, k);
        y = H(k + 2, k);
        if (k < hi - 2) z = H(k + 3, k);
    }
    // last 2-vector reflector on rows hi-1, hi
    const double nr = std::hypot(x, y);
    if (nr != 0.0) {
        const double alpha = x >= 0 ? -nr : nr;
        double v[2] = {x - alpha, y};
        const double vv = v[0] * v[0] + v[1] * v[1];
        const double beta = vv > 0 ? 2.0 / vv : 0.0;
        house_left(n, h, v, beta, 2, hi - 1, std::max(hi - 2, l), n);
        house_right(n, h, v, beta, 2, hi - 1, 0, hi + 1);
        house_right(n, zm, v, beta, 2, hi - 1, 0, n);
        if (hi - 2 >= l) H(hi, hi - 2) = 0.0;
    }
}

// Real Schur form of the upper Hessenberg h (order n, overwritten by T);
// zm is multiplied on the right by every transformation (pass the
// identity to get Z).  wr, wi: the eigenvalues in diagonal order, a
// complex pair as (re, +im), (re, -im).  false if an eigenvalue needed more
// than 30 n iterations.
inline bool schur(int n, std::vector<double> &h, std::vector<double> &zm, std::vector<double> &wr,
                  std::vector<double> &wi) {
    auto H = [&](int i, int j) -> double & { return h[(size_t)i * n + j]; };
    wr.assign(n, 0.0);
    wi.assign(n, 0.0);
    double norm = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = std::max(i - 1, 0); j < n; ++j) norm += std::fabs(H(i, j));
    int hi = n - 1, its = 0, total = 0;
    while (hi >= 0) {
        int l = hi;
        for (; l > 0; --l) {
            double s = std::fabs(H(l - 1, l - 1)) + std::fabs(H(l, l));
            if (s == 0.0) s = norm;
            if (std::fabs(H(l, l - 1)) <= kEps * s) {
                H(l, l - 1) = 0.0;
                break;
            }
        }
        if (l == hi) {  // 1 x 1 block
            wr[hi] = H(hi, hi);
            wi[hi] = 0.0;
            --hi;
            its = 0;
            continue;
        }
        if (l == hi - 1) {  // 2 x 2 block
            const int na = hi - 1;
            const double a = H(na, na), b = H(na, hi), c = H(hi, na), d = H(hi, hi);
            const double p = 0.5 * (a - d), q = p * p + b * c;
            if (q >= 0.0) {
                // real pair: eigenvalues d + zz and d - bc / zz; a rotation
                // makes the block upper triangular
                double zz = std::sqrt(q);
                zz = p >= 0.0 ? p + zz : p - zz;
                wr[na] = d + zz;
                wr[hi] = zz != 0.0 ? d - b * c / zz : wr[na];
                const double sx = std::fabs(c) + std::fabs(zz);
                double pr = c / sx, qr = zz / sx;
                const double r = std::hypot(pr, qr);
                pr /= r;
                qr /= r;
                for (int j = na; j < n; ++j) {  // rows na, hi
                    const double t0 = H(na, j);
                    H(na, j) = qr * t0 + pr * H(hi, j);
                    H(hi, j) = qr * H(hi, j) - pr * t0;
                }
                for (int i = 0; i <= hi; ++i) {  // columns na, hi
                    const double t0 = H(i, na);
                    H(i, na) = qr * t0 + pr * H(i, hi);
                    H(i, hi) = qr * H(i, hi) - pr * t0;
                }
                for (int i = 0; i < n; ++i) {
                    const double t0 = zm[(size_t)i * n + na];
                    zm[(size_t)i * n + na] = qr * t0 + pr * zm[(size_t)i * n + hi];
                    zm[(size_t)i * n + hi] = qr * zm[(size_t)i * n + hi] - pr * t0;
                }
                H(hi, na) = 0.0;
                wr[na] = H(na, na);  // the rotated diagonal, in diagonal order
                wr[hi] = H(hi, hi);
            } else {
                wr[na] = wr[hi] = d + p;
                wi[na] = std::sqrt(-q);
                wi[hi] = -wi[na];
            }
            hi -= 2;
            its = 0;
            continue;
        }
        if (++total > 30 * n) return false;
        double s, t;
        if (its == 10 || its == 20) {  // exceptional shift
            const double e = std::fabs(H(hi, hi - 1)) + std::fabs(H(hi - 1, hi - 2));
            s = 1.5 * e;
            t = e * e;
        } else {
            s = H(hi - 1, hi - 1) + H(hi, hi);
            t = H(hi - 1, hi - 1) * H(hi, hi) - H(hi - 1, hi) * H(hi, hi - 1);
        }
        ++its;
        francis_step(n, h, zm, l, hi, s, t);
    }
    return true;
}

// Eigenvector x (length n) of the quasi-triangular t for the eigenvalue at
// diagonal position p: the real one of a 1 x 1 block, or (for a 2 x 2 block
// starting at p) the one with positive imaginary part.  Back substitution
// in complex arithmetic; tiny pivots are replaced by eps * ||t||.
inline void ritz_vec(int n, const std::vector<double> &t, int p, std::vector<cplx> &x) {
    auto T = [&](int i, int j) { return t[(size_t)i * n + j]; };
    double tn = 0.0;
    for (double v : t) tn = std::max(tn, std::fabs(v));
    const double small = std::max(kEps * tn, 1e-300);
    x.assign(n, cplx(0.0, 0.0));
    const bool pair = p + 1 < n && T(p + 1, p) != 0.0;
    cplx lam;
    int i;
    if (!pair) {
        lam = T(p, p);
        x[p] = 1.0;
        i = p - 1;
    } else {
        const double a = T(p, p), b = T(p, p + 1), c = T(p + 1, p), d = T(p + 1, p + 1);
        const double pp = 0.5 * (a - d), q = pp * pp + b * c;  // q < 0 for a pair
        lam = cplx(d + pp, std::sqrt(std::max(-q, 0.0)));
        // (a - lam) x0 + b x1 = 0
        if (std::abs(b) >= std::abs(c)) {
            x[p] = b;
            x[p + 1] = lam - a;
        } else {
            x[p] = lam - d;
            x[p + 1] = c;
        }
        i = p - 1;
    }
    while (i >= 0) {
        const bool blk = i >= 1 && T(i, i - 1) != 0.0;
        if (!blk) {
            cplx rhs = 0.0;
            for (int j = i + 1; j < n; ++j) rhs -= T(i, j) * x[j];
            cplx den = T(i, i) - lam;
            if (std::abs(den) < small) den = small;
            x[i] = rhs / den;
            --i;
        } else {
            cplx r0 = 0.0, r1 = 0.0;
            for (int j = i + 1; j < n; ++j) {
                r0 -= T(i - 1, j) * x[j];
                r1 -= T(i, j) * x[j];
            }
            const cplx a = T(i - 1, i - 1) - lam, b = T(i - 1, i), c = T(i, i - 1), d = T(i, i) - lam;
            cplx det = a * d - b * c;
            if (std::abs(det) < small * small) det = small * small;
            x[i - 1] = (r0 * d - b * r1) / det;
            x[i] = (a * r1 - c * r0) / det;
            i -= 2;
        }
        double mx = 0.0;
        for (const cplx &v : x) mx = std::max(mx, std::abs(v));
        if (mx > 1e100)
            for (cplx &v : x) v /= mx;
    }
}

// One implicit single-shift QR step with shift mu on the Hessenberg h
// (order n): a Givens chase; h <- Q^T h Q, q <- q Q.
inline void qr_shift1(int n, std::vector<double> &h, std::vector<double> &q, double mu) {
    auto H = [&](int i, int j) -> double & { return h[(size_t)i * n + j]; };
    double x = H(0, 0) - mu, y = H(1, 0);
    for (int k = 0; k <= n - 2; ++k) {
        const double r = std::hypot(x, y);
        const double c = r == 0.0 ? 1.0 : x / r, s = r == 0.0 ? 0.0 : y / r;
        for (int j = std::max(k - 1, 0); j < n; ++j) {  // rows k, k+1
            const double a = H(k, j), b = H(k + 1, j);
            H(k, j) = c * a + s * b;
            H(k + 1, j) = -s * a + c * b;
        }
        for (int i = 0; i <= std::min(k + 2, n - 1); ++i) {  // columns k, k+1
            const double a = H(i, k), b = H(i, k + 1);
            H(i, k) = c * a + s * b;
            H(i, k + 1) = -s * a + c * b;
        }
        for (int i = 0; i < n; ++i) {
            const double a = q[(size_t)i * n + k], b = q[(size_t)i * n + k + 1];
            q[(size_t)i * n + k] = c * a + s * b;
            q[(size_t)i * n + k + 1] = -s * a + c * b;
        }
        if (k > 0) H(k + 1, k - 1) = 0.0;
        if (k < n - 2) {
            x = H(k + 1, k);
            y = H(k + 2, k);
        }
    }
}

// One implicit double-shift QR step (shifts the roots of z^2 - s z + t).
inline void qr_shift2(int n, std::vector<double> &h, std::vector<double> &q, double s, double t) {
    francis_step(n, h, q, 0, n - 1, s, t);
}

}  // namespace dense
}  // namespace xab
