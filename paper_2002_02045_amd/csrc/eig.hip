// Batched Hermitian eigensolvers in FP64 for the small matrices of the method:
// H(k) and H(k+q) (n = Nw, Eq. wannier_3) and D(q) (n = 3 nat, Eq. IFC2).
//
// n <= 8: one matrix per lane, 64 per wavefront: Householder reduction to a
// real tridiagonal matrix, implicit QL with Wilkinson shifts, eigenvectors
// U = Q Z (eig_ql.h).  About 240 VALU instructions per 8 x 8 matrix against
// about 950 for cyclic Jacobi with one lane per row, which it replaces.
//
// 8 < n <= 128: one workgroup per matrix, cyclic Jacobi with plane rotations
// applied to disjoint pairs in parallel (Golub & Van Loan, "Matrix
// Computations", Sec. 8.5, in its complex Hermitian form).  For a pair (p, q),
// p < q, with a_pq = |a_pq| e^{i phi}:
//   th = (a_qq - a_pp)/(2|a_pq|), t = sgn(th)/(|th| + sqrt(th^2 + 1)),
//   c = 1/sqrt(1 + t^2), s = t c, J_pq = s e^{i phi}, J_qp = -s e^{-i phi},
// and A <- J^dag A J, V <- V J.  Sweeps run until the off-diagonal Frobenius
// norm is below 1e-15 of the matrix norm.
//
// Both sort the eigenpairs ascending, ties by index.
#include "internal.h"
#include "eig_ql.h"

namespace ephx {
namespace {

// 1/b and 1/sqrt(x) from the hardware estimates refined by two Newton steps
// each (quadratic convergence from the estimate's ~1e-8 relative error to the
// last bits); any nonzero b, any positive normal x.
__device__ __forceinline__ double recip(double b) {
    double y = __builtin_amdgcn_rcp(b);
    y = y * fma(-b, y, 2.0);
    return y * fma(-b, y, 2.0);
}
__device__ __forceinline__ double rsqrt1(double x) {
    const double h = 0.5 * x;
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-h * y, y, 1.5);
    return y * fma(-h * y, y, 1.5);
}

// Device arithmetic of the one-lane-per-matrix solver (eig_ql.h): the
// refined inverse square root and reciprocal above (any positive x; any
// nonzero b), and the wavefront vote that keeps a QL iteration running while
// any lane's block is unreduced.
struct LaneMath {
    static __device__ __forceinline__ double rsqrt(double x) { return rsqrt1(x); }
    static __device__ __forceinline__ double rcp(double b) { return recip(b); }
    static __device__ __forceinline__ bool any(bool p) { return __any(p); }
};

template <int N, int C>
__device__ __forceinline__ void store_lane_vectors(const HermLane<N>& s, const int (&rk)[N], double* out) {
    if constexpr (C < N) {
        double xr[N], xi[N];
        herm_eigenvector<N, C>(s, xr, xi);
#pragma unroll
        for (int i = 0; i < N; ++i) *reinterpret_cast<double2*>(out + (i * N + rk[C]) * 2) = double2{xr[i], xi[i]};
        store_lane_vectors<N, C + 1>(s, rk, out);
    }
}

// One matrix per lane (n <= 8): Householder tridiagonalisation, implicit QL,
// eigenvectors U = Q Z (eig_ql.h).  PK selects the packed Hermitian input, else the Hermitian part of a complex
// n x n matrix is taken; eigenvalues ascending, ties by index, eigenvector c
// in column c of evecs[slot] (row-major complex n x n).
template <typename Tin, int N, bool PK = false>
__global__ __launch_bounds__(256) void k_eig_lane(int batch, const Tin* __restrict__ A, long strideA,
                                                  double* __restrict__ evals, double* __restrict__ evecs) {
    const long slot = (long)blockIdx.x * 256 + threadIdx.x;
    const bool valid = slot < batch;
    HermLane<N> s;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double re = 0.0, im = 0.0;
            if (valid && PK) {
                const Tin* ab = A + slot * strideA;
                re = (double)ab[j * N + i];
                im = i == j ? 0.0 : -(double)ab[i * N + j];
            } else if (valid) {
                const Tin* ab = A + slot * strideA * 2;
                const double xr = (double)ab[2 * (i * N + j)], xi = (double)ab[2 * (i * N + j) + 1];
                const double yr = (double)ab[2 * (j * N + i)], yi = (double)ab[2 * (j * N + i) + 1];
                re = 0.5 * (xr + yr);
                im = i == j ? 0.0 : 0.5 * (xi - yi);
            }
            s.ar[i][j] = re;
            s.ai[i][j] = im;
        }
    herm_tridiagonalize<LaneMath, N>(s);
    tridiag_ql<LaneMath, N>(s);
    int rk[N];
    eig_ranks<N>(s.d, rk);
    if (!valid) return;
#pragma unroll
    for (int c = 0; c < N; ++c) evals[slot * N + rk[c]] = s.d[c];
    if (evecs != nullptr) store_lane_vectors<N, 0>(s, rk, evecs + slot * N * N * 2);
}

// Larger matrices (8 < n <= 128, e.g. H(k) of a 64-function model, D(q) of a
// 40-atom cell): one 256-thread workgroup per matrix, the Jacobi rotations of
// the header, with the n/2 disjoint rotations of a round (circle-method
// ordering) applied by all threads at once.  For n <= 64 (k_eig_wg) A and V
// live in LDS (2 x 65 KB, rows padded by one element) and a round is a column
// pass and a row pass, three barriers apart; above, see k_eig_wg_packed.  The
// rotation parameters of a round go through LDS.
constexpr int kWgMax = 128;
constexpr int kWgLds = 64;     // largest order kept in LDS with its eigenvectors

__device__ __forceinline__ int circle_index(int pos, int r, int ne) {
    return pos == 0 ? 0 : (pos - 1 + r) % (ne - 1) + 1;
}

__global__ __launch_bounds__(256) void k_eig_wg(int n, double* __restrict__ A, long strideA, double* __restrict__ evals,
                                                double* __restrict__ evecs) {
    __shared__ int pp[kWgMax / 2], qq[kWgMax / 2];
    __shared__ double rc[kWgMax / 2], rsr[kWgMax / 2], rsi[kWgMax / 2];
    __shared__ double red[2][256];
    __shared__ double dg[kWgMax];
    __shared__ int rk[kWgMax];
    // in LDS the rows are padded by one complex element, so that a column
    // (stride ld) walks across the banks instead of hitting one
    __shared__ double sbuf[4 * kWgLds * (kWgLds + 1)];
    const int tid = threadIdx.x;
    const long mi = blockIdx.x;
    double* ga = A + mi * strideA * 2;
    double* gv = evecs != nullptr ? evecs + mi * (long)n * n * 2 : nullptr;
    const int ld = n + 1;   // complex elements per row of a and v
    double* a = sbuf;
    double* v = gv ? sbuf + 2 * kWgLds * (kWgLds + 1) : nullptr;
    const int nn = n * n;
    // Hermitian part 0.5 (A + A^dag), V = I
    for (int e = tid; e < nn; e += 256) {
        const int i = e / n, j = e % n;
        if (i < j) {
            const double xr = 0.5 * (ga[2 * e] + ga[2 * (j * n + i)]);
            const double xi = 0.5 * (ga[2 * e + 1] - ga[2 * (j * n + i) + 1]);
            a[2 * (i * ld + j)] = xr;
            a[2 * (i * ld + j) + 1] = xi;
            a[2 * (j * ld + i)] = xr;
            a[2 * (j * ld + i) + 1] = -xi;
        } else if (i == j) {
            a[2 * (i * ld + i)] = ga[2 * e];
            a[2 * (i * ld + i) + 1] = 0.0;
        }
        if (v) {
            v[2 * (i * ld + j)] = i == j ? 1.0 : 0.0;
            v[2 * (i * ld + j) + 1] = 0.0;
        }
    }
    __syncthreads();
    const int ne = n + (n & 1), np = ne / 2;
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < nn; e += 256) {
            const int i = e / n, j = e % n;
            const double m2 = a[2 * (i * ld + j)] * a[2 * (i * ld + j)] + a[2 * (i * ld + j) + 1] * a[2 * (i * ld + j) + 1];
            tot += m2;
            off += (i != j) ? m2 : 0.0;
        }
        red[0][tid] = off;
        red[1][tid] = tot;
        __syncthreads();
        for (int w = 128; w >= 1; w >>= 1) {
            if (tid < w) {
                red[0][tid] += red[0][tid + w];
                red[1][tid] += red[1][tid + w];
            }
            __syncthreads();
        }
        const bool done = !(red[0][0] > 1e-30 * red[1][0]);
        __syncthreads();
        if (done) break;
        for (int r = 0; r < ne - 1; ++r) {
            if (tid < np) {
                const int i1 = circle_index(tid, r, ne), i2 = circle_index(ne - 1 - tid, r, ne);
                const int p = i1 < i2 ? i1 : i2, q = i1 < i2 ? i2 : i1;
                double c = 1.0, sr = 0.0, si = 0.0;
                if (q < n) {
                    const double apr = a[2 * (p * ld + q)], api = a[2 * (p * ld + q) + 1];
                    const double m2 = apr * apr + api * api;
                    if (m2 > 0.0) {
                        // t/|a_pq| and se as in the wavefront solver
                        const double d = a[2 * (q * ld + q)] - a[2 * (p * ld + p)];
                        const double tm = (d >= 0.0 ? 2.0 : -2.0) * recip(fabs(d) + sqrt(fma(d, d, 4.0 * m2)));
                        c = rsqrt1(fma(tm * tm, m2, 1.0));
                        const double w = tm * c;
                        sr = w * apr;
                        si = w * api;
                    }
                }
                pp[tid] = p;
                qq[tid] = q < n ? q : p;   // a dummy partner never rotates
                rc[tid] = c;
                rsr[tid] = sr;
                rsi[tid] = si;
            }
            __syncthreads();
            // columns: (AJ)_{.p} = c A_.p - conj(se) A_.q ; (AJ)_{.q} = se A_.p + c A_.q ; V likewise
            for (int e = tid; e < np * n; e += 256) {
                const int k = e / n, i = e % n;
                const int p = pp[k], q = qq[k];
                if (p == q) continue;
                const double c = rc[k], sr = rsr[k], si = rsi[k];
                double* x = a + 2 * (i * ld + p);
                double* y = a + 2 * (i * ld + q);
                const double xr = x[0], xi = x[1], yr = y[0], yi = y[1];
                x[0] = c * xr - (sr * yr + si * yi);
                x[1] = c * xi - (sr * yi - si * yr);
                y[0] = (sr * xr - si * xi) + c * yr;
                y[1] = (sr * xi + si * xr) + c * yi;
                if (v) {
                    double* u = v + 2 * (i * ld + p);
                    double* w = v + 2 * (i * ld + q);
                    const double ur = u[0], ui = u[1], wr = w[0], wi = w[1];
                    u[0] = c * ur - (sr * wr + si * wi);
                    u[1] = c * ui - (sr * wi - si * wr);
                    w[0] = (sr * ur - si * ui) + c * wr;
                    w[1] = (sr * ui + si * ur) + c * wi;
                }
            }
            __syncthreads();
            // rows: (J^dag A)_{p.} = c A_p. - se A_q. ; (J^dag A)_{q.} = conj(se) A_p. + c A_q.
            for (int e = tid; e < np * n; e += 256) {
                const int k = e / n, j = e % n;
                const int p = pp[k], q = qq[k];
                if (p == q) continue;
                const double c = rc[k], sr = rsr[k], si = rsi[k];
                double* x = a + 2 * (p * ld + j);
                double* y = a + 2 * (q * ld + j);
                const double xr = x[0], xi = x[1], yr = y[0], yi = y[1];
                x[0] = c * xr - (sr * yr - si * yi);
                x[1] = c * xi - (sr * yi + si * yr);
                y[0] = (sr * xr + si * xi) + c * yr;
                y[1] = (sr * xi - si * xr) + c * yi;
            }
            __syncthreads();
        }
    }
    // sort ascending, ties by index
    for (int i = tid; i < n; i += 256) dg[i] = a[2 * (i * ld + i)];
    __syncthreads();
    for (int i = tid; i < n; i += 256) {
        int r = 0;
        for (int m = 0; m < n; ++m) r += (dg[m] < dg[i] || (dg[m] == dg[i] && m < i)) ? 1 : 0;
        rk[i] = r;
        evals[mi * n + r] = dg[i];
    }
    __syncthreads();
    if (gv) {
        // columns of V go to their ranks directly
        for (int e = tid; e < nn; e += 256) {
            const int i = e / n, c = e % n;
            gv[2 * (i * n + rk[c])] = v[2 * (i * ld + c)];
            gv[2 * (i * n + rk[c]) + 1] = v[2 * (i * ld + c) + 1];
        }
    }
}

// Orders above the LDS range of k_eig_wg (64 < n <= 128): A is kept in LDS in
// the packed Hermitian form (n*n reals, P[i][j] = Re A_ij for i <= j and Im A_ji
// for i > j: 131 KB at n = 128) and each round applies J^dag A J at once, block
// by block: the rows of pair a and the columns of pair b form a 2 x 2 block B,
// and its new value is J_a^dag B J_b (the same column-then-row arithmetic as
// the two-phase update), so only the blocks with a <= b are formed and the
// rest follows by Hermiticity.  The eigenvectors accumulate transposed, V^T,
// in A's global storage (the input is overwritten), so that the column update
// V J of a round walks contiguous memory.
__global__ __launch_bounds__(256) void k_eig_wg_packed(int n, double* __restrict__ A, long strideA,
                                                       double* __restrict__ evals, double* __restrict__ evecs) {
    __shared__ double P[kWgMax * kWgMax];
    __shared__ int pp[kWgMax / 2], qq[kWgMax / 2];
    __shared__ double rc[kWgMax / 2], rsr[kWgMax / 2], rsi[kWgMax / 2];
    __shared__ double red[2][256];
    __shared__ double dg[kWgMax];
    __shared__ int rk[kWgMax];
    const int tid = threadIdx.x;
    const long mi = blockIdx.x;
    double* ga = A + mi * strideA * 2;
    const bool want_v = evecs != nullptr;
    const int nn = n * n;
    // packed Hermitian part 0.5 (A + A^dag)
    for (int e = tid; e < nn; e += 256) {
        const int i = e / n, j = e % n;
        if (i < j) {
            P[i * n + j] = 0.5 * (ga[2 * e] + ga[2 * (j * n + i)]);
            P[j * n + i] = 0.5 * (ga[2 * e + 1] - ga[2 * (j * n + i) + 1]);
        } else if (i == j) {
            P[i * n + i] = ga[2 * e];
        }
    }
    __syncthreads();
    // V^T = I over A's storage (read complete above)
    if (want_v)
        for (int e = tid; e < nn; e += 256) {
            ga[2 * e] = (e / n == e % n) ? 1.0 : 0.0;
            ga[2 * e + 1] = 0.0;
        }
    // element (i, j), i != j, of the Hermitian matrix from the packed form
    auto get = [&](int i, int j, double& re, double& im) {
        if (i < j) {
            re = P[i * n + j];
            im = P[j * n + i];
        } else {
            re = P[j * n + i];
            im = -P[i * n + j];
        }
    };
    auto put = [&](int i, int j, double re, double im) {
        if (i < j) {
            P[i * n + j] = re;
            P[j * n + i] = im;
        } else {
            P[j * n + i] = re;
            P[i * n + j] = -im;
        }
    };
    const int ne = n + (n & 1), np = ne / 2;
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int e = tid; e < nn; e += 256) {
            const int i = e / n, j = e % n;
            if (i == j) {
                tot += P[e] * P[e];
            } else if (i < j) {
                const double m2 = 2.0 * (P[e] * P[e] + P[j * n + i] * P[j * n + i]);
                tot += m2;
                off += m2;
            }
        }
        red[0][tid] = off;
        red[1][tid] = tot;
        __syncthreads();
        for (int w = 128; w >= 1; w >>= 1) {
            if (tid < w) {
                red[0][tid] += red[0][tid + w];
                red[1][tid] += red[1][tid + w];
            }
            __syncthreads();
        }
        const bool done = !(red[0][0] > 1e-30 * red[1][0]);
        __syncthreads();
        if (done) break;
        for (int r = 0; r < ne - 1; ++r) {
            if (tid < np) {
                const int i1 = circle_index(tid, r, ne), i2 = circle_index(ne - 1 - tid, r, ne);
                const int p = i1 < i2 ? i1 : i2, q = i1 < i2 ? i2 : i1;
                double c = 1.0, sr = 0.0, si = 0.0;
                if (q < n) {
                    const double apr = P[p * n + q], api = P[q * n + p];
                    const double m2 = apr * apr + api * api;
                    if (m2 > 0.0) {
                        const double d = P[q * n + q] - P[p * n + p];
                        const double tm = (d >= 0.0 ? 2.0 : -2.0) * recip(fabs(d) + sqrt(fma(d, d, 4.0 * m2)));
                        c = rsqrt1(fma(tm * tm, m2, 1.0));
                        const double w = tm * c;
                        sr = w * apr;
                        si = w * api;
                    }
                }
                pp[tid] = p;
                qq[tid] = q < n ? q : p;   // a dummy partner never rotates
                rc[tid] = c;
                rsr[tid] = sr;
                rsi[tid] = si;
            }
            __syncthreads();
            // blocks (a, b), a <= b: B' = J_a^dag B J_b with J = [[c, se], [-conj(se), c]]
            for (int t = tid; t < np * np; t += 256) {
                const int a = t / np, b = t % np;
                if (a > b) continue;
                const int ra[2] = {pp[a], qq[a]}, cb[2] = {pp[b], qq[b]};
                const int nr = ra[1] != ra[0] ? 2 : 1, nc = cb[1] != cb[0] ? 2 : 1;
                double br_[2][2], bi_[2][2];
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y) {
                        const int i = ra[x], j = cb[y];
                        if (i == j) {
                            br_[x][y] = P[i * n + i];
                            bi_[x][y] = 0.0;
                        } else {
                            get(i, j, br_[x][y], bi_[x][y]);
                        }
                    }
                // T = B J_b: T_.p = c B_.p - conj(s) B_.q ; T_.q = s B_.p + c B_.q
                const double cb_ = rc[b], sbr = rsr[b], sbi = rsi[b];
                double tr[2][2], ti[2][2];
#pragma unroll
                for (int x = 0; x < 2; ++x) {
                    const double ur = br_[x][0], ui = bi_[x][0], wr = br_[x][1], wi = bi_[x][1];
                    tr[x][0] = cb_ * ur - (sbr * wr + sbi * wi);
                    ti[x][0] = cb_ * ui - (sbr * wi - sbi * wr);
                    tr[x][1] = (sbr * ur - sbi * ui) + cb_ * wr;
                    ti[x][1] = (sbr * ui + sbi * ur) + cb_ * wi;
                }
                // B' = J_a^dag T: B'_p. = c T_p. - s T_q. ; B'_q. = conj(s) T_p. + c T_q.
                const double ca = rc[a], sar = rsr[a], sai = rsi[a];
                double orr[2][2], oi[2][2];
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    const double xr = tr[0][y], xi = ti[0][y], yr = tr[1][y], yi = ti[1][y];
                    orr[0][y] = ca * xr - (sar * yr - sai * yi);
                    oi[0][y] = ca * xi - (sar * yi + sai * yr);
                    orr[1][y] = (sar * xr + sai * xi) + ca * yr;
                    oi[1][y] = (sar * xi - sai * xr) + ca * yi;
                }
                if (a == b) {
                    // Hermitian diagonal block: two real diagonal entries, one pair
                    P[ra[0] * n + ra[0]] = orr[0][0];
                    if (nr == 2) {
                        P[ra[1] * n + ra[1]] = orr[1][1];
                        put(ra[0], ra[1], orr[0][1], oi[0][1]);
                    }
                } else {
                    for (int x = 0; x < nr; ++x)
                        for (int y = 0; y < nc; ++y) put(ra[x], cb[y], orr[x][y], oi[x][y]);
                }
            }
            // V <- V J on V^T: rows p, q of V^T, contiguous over i
            if (want_v)
                for (int t = tid; t < np * n; t += 256) {
                    const int b = t / n, i = t % n;
                    const int p = pp[b], q = qq[b];
                    if (p == q) continue;
                    const double c = rc[b], sr = rsr[b], si = rsi[b];
                    double* u = ga + 2 * ((long)p * n + i);
                    double* w = ga + 2 * ((long)q * n + i);
                    const double ur = u[0], ui = u[1], wr = w[0], wi = w[1];
                    u[0] = c * ur - (sr * wr + si * wi);
                    u[1] = c * ui - (sr * wi - si * wr);
                    w[0] = (sr * ur - si * ui) + c * wr;
                    w[1] = (sr * ui + si * ur) + c * wi;
                }
            __syncthreads();
        }
    }
    // sort ascending, ties by index
    for (int i = tid; i < n; i += 256) dg[i] = P[i * n + i];
    __syncthreads();
    for (int i = tid; i < n; i += 256) {
        int r = 0;
        for (int m = 0; m < n; ++m) r += (dg[m] < dg[i] || (dg[m] == dg[i] && m < i)) ? 1 : 0;
        rk[i] = r;
        evals[mi * n + r] = dg[i];
    }
    __syncthreads();
    if (want_v) {
        // column c of V (row c of V^T) goes to column rank(c) of the output
        double* gv = evecs + mi * (long)n * n * 2;
        for (int e = tid; e < nn; e += 256) {
            const int c = e / n, i = e % n;
            gv[2 * (i * n + rk[c])] = ga[2 * e];
            gv[2 * (i * n + rk[c]) + 1] = ga[2 * e + 1];
        }
    }
}

__global__ void k_phonon_omega(long count, double* lam) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const double w2 = kHbar2AmuA2 * lam[t];
    lam[t] = (w2 >= 0.0 ? 1.0 : -1.0) * sqrt(fabs(w2));
}

template <typename Tin, bool PK = false>
void launch_eig(int batch, int n, const Tin* A, long strideA, double* evals, double* evecs, hipStream_t st) {
    dim3 grid((unsigned)(((long)batch + 255) / 256));
    switch (n) {
#define EPHX_EIG_CASE(NN) \
    case NN:                                                                                                \
        hipLaunchKernelGGL((k_eig_lane<Tin, NN, PK>), grid, dim3(256), 0, st, batch, A, strideA, evals, evecs); \
        break;
        EPHX_EIG_CASE(1)
        EPHX_EIG_CASE(2)
        EPHX_EIG_CASE(3)
        EPHX_EIG_CASE(4)
        EPHX_EIG_CASE(5)
        EPHX_EIG_CASE(6)
        EPHX_EIG_CASE(7)
        EPHX_EIG_CASE(8)
#undef EPHX_EIG_CASE
        default: throw Error{-6, "eig_herm: matrix order above 8 is not supported in this build"};
    }
}

}  // namespace

void eig_herm(int batch, int n, void* A, int a_f32, long strideA, double* evals, double* evecs, hipStream_t st) {
    if (batch <= 0) return;
    if (n < 1 || n > kWgMax) throw Error{-6, "eig_herm: matrix order above 128 is not supported"};
    if (n > kEigMax) {
        if (a_f32) throw Error{-1, "eig_herm: matrices above order 8 must be FP64"};
        if (n <= kWgLds)
            hipLaunchKernelGGL(k_eig_wg, dim3((unsigned)batch), dim3(256), 0, st, n, (double*)A, strideA, evals,
                               evecs);
        else
            hipLaunchKernelGGL(k_eig_wg_packed, dim3((unsigned)batch), dim3(256), 0, st, n, (double*)A, strideA, evals,
                               evecs);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) throw Error{-3, std::string("eig_herm: ") + hipGetErrorString(e)};
        return;
    }
    if (a_f32)
        launch_eig(batch, n, (const float*)A, strideA, evals, evecs, st);
    else
        launch_eig(batch, n, (const double*)A, strideA, evals, evecs, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{-3, std::string("eig_herm: ") + hipGetErrorString(e)};
}

void eig_herm_packed(int batch, int n, const double* P, long strideP, double* evals, double* evecs, hipStream_t st) {
    if (batch <= 0) return;
    if (n < 1 || n > kEigMax) throw Error{-6, "eig_herm_packed: matrix order must be 1..8"};
    if (strideP < (long)n * n) throw Error{-1, "eig_herm_packed: stride below n*n"};
    launch_eig<double, true>(batch, n, P, strideP, evals, evecs, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{-3, std::string("eig_herm_packed: ") + hipGetErrorString(e)};
}

void phonon_omega(long count, double* lam, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_phonon_omega, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, lam);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{-3, std::string("phonon_omega: ") + hipGetErrorString(e)};
}

}  // namespace ephx
