// Host build of the one-lane-per-matrix Hermitian eigensolver (eig_ql.h) for
// the CPU tests: reads [count][N][N] complex double, takes the Hermitian part,
// writes eigenvalues [count][N] (ascending) and eigenvectors [count][N][N]
// complex (column c for eigenvalue c), the layout the device kernel writes.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>
#define __host__
#define __device__
#define __forceinline__ inline
#include "../../paper_2002_02045_amd/csrc/eig_ql.h"
struct HostMath {
    static double rsqrt(double x) { return 1.0 / std::sqrt(x); }
    static double rcp(double x) { return 1.0 / x; }
    static bool any(bool b) { return b; }
};
template <int N, int C>
void store_cols(const ephx::HermLane<N>& s, const int* rk, double* v) {
    if constexpr (C < N) {
        double xr[N], xi[N];
        ephx::herm_eigenvector<N, C>(s, ephx::ReflInRegs<N>{s}, xr, xi);
        for (int i = 0; i < N; ++i) { v[(i * N + rk[C]) * 2] = xr[i]; v[(i * N + rk[C]) * 2 + 1] = xi[i]; }
        store_cols<N, C + 1>(s, rk, v);
    }
}
template <int N>
void run(long count, const double* A, double* w, double* v) {
    using namespace ephx;
    for (long t = 0; t < count; ++t) {
        HermLane<N> s;
        const double* a = A + t * N * N * 2;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j <= i; ++j) {
                s.ar[i][j] = 0.5 * (a[2 * (i * N + j)] + a[2 * (j * N + i)]);
                s.ai[i][j] = 0.5 * (a[2 * (i * N + j) + 1] - a[2 * (j * N + i) + 1]);
            }
        herm_tridiagonalize<HostMath, N>(s);
        tridiag_ql<HostMath, N>(s);
        int rk[N];
        eig_ranks<N>(s.d, rk);
        for (int c = 0; c < N; ++c) w[t * N + rk[c]] = s.d[c];
        store_cols<N, 0>(s, rk, v + t * N * N * 2);
    }
}
int main(int argc, char** argv) {
    int n = atoi(argv[1]);
    long count = atol(argv[2]);
    std::vector<double> A(count * n * n * 2), w(count * n), v(count * n * n * 2);
    FILE* f = fopen(argv[3], "rb");
    if (fread(A.data(), 8, A.size(), f) != A.size()) return 1;
    fclose(f);
    switch (n) {
        case 1: run<1>(count, A.data(), w.data(), v.data()); break;
        case 2: run<2>(count, A.data(), w.data(), v.data()); break;
        case 3: run<3>(count, A.data(), w.data(), v.data()); break;
        case 4: run<4>(count, A.data(), w.data(), v.data()); break;
        case 5: run<5>(count, A.data(), w.data(), v.data()); break;
        case 6: run<6>(count, A.data(), w.data(), v.data()); break;
        case 7: run<7>(count, A.data(), w.data(), v.data()); break;
        case 8: run<8>(count, A.data(), w.data(), v.data()); break;
    }
    f = fopen(argv[4], "wb");
    fwrite(w.data(), 8, w.size(), f);
    fwrite(v.data(), 8, v.size(), f);
    fclose(f);
    return 0;
}
