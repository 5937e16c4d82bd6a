// C shim over the library's host-side dense eigenvalue routines, built by
// tests/test_host_dense_eig.py with g++ (no GPU code involved).
#include "../../paper_2405_01599_amd/csrc/dense_eig.h"

#include <cstring>

extern "C" {

// h: n x n row-major Hessenberg in, T out; z: Z out; wr, wi: eigenvalues
int shim_schur(int n, double *h, double *z, double *wr, double *wi) {
    std::vector<double> H(h, h + (size_t)n * n), Z((size_t)n * n, 0.0), R, I;
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    const bool ok = xab::dense::schur(n, H, Z, R, I);
    memcpy(h, H.data(), sizeof(double) * n * n);
    memcpy(z, Z.data(), sizeof(double) * n * n);
    memcpy(wr, R.data(), sizeof(double) * n);
    memcpy(wi, I.data(), sizeof(double) * n);
    return ok ? 0 : 1;
}

// eigenvector of the quasi-triangular t at position p: xr, xi (length n)
void shim_ritz_vec(int n, const double *t, int p, double *xr, double *xi) {
    std::vector<double> T(t, t + (size_t)n * n);
    std::vector<xab::dense::cplx> x;
    xab::dense::ritz_vec(n, T, p, x);
    for (int i = 0; i < n; ++i) {
        xr[i] = x[i].real();
        xi[i] = x[i].imag();
    }
}

// one implicit QR step: kind 1 (shift s) or 2 (s, t); h and q (n x n) in place
void shim_qr_shift(int n, double *h, double *q, int kind, double s, double t) {
    std::vector<double> H(h, h + (size_t)n * n), Q(q, q + (size_t)n * n);
    if (kind == 1) xab::dense::qr_shift1(n, H, Q, s);
    else xab::dense::qr_shift2(n, H, Q, s, t);
    memcpy(h, H.data(), sizeof(double) * n * n);
    memcpy(q, Q.data(), sizeof(double) * n * n);
}
}
