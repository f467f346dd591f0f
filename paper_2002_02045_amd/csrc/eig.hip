// Batched Hermitian eigensolver in FP64 for the small matrices of the method:
// H(k) and H(k+q) (n = Nw, Eq. wannier_3) and D(q) (n = 3 nat, Eq. IFC2).
//
// Cyclic Jacobi with plane rotations applied to disjoint pairs in parallel
// (Golub & Van Loan, "Matrix Computations", Sec. 8.5, in its complex Hermitian
// form).  For a pair (p, q), p < q, with a_pq = |a_pq| e^{i phi}:
//   th = (a_qq - a_pp)/(2|a_pq|), t = sgn(th)/(|th| + sqrt(th^2 + 1)),
//   c = 1/sqrt(1 + t^2), s = t c, J_pq = s e^{i phi}, J_qp = -s e^{-i phi},
// and A <- J^dag A J, V <- V J.
//
// Layout: one lane per matrix row, R = 2^ceil(log2 n) lanes per matrix (rows
// and columns beyond n are zero and never rotate), 64/R matrices per
// wavefront.  Round m = 1..R-1 of a sweep pairs row i with row i^m; over a
// sweep every pair meets once.  Lane i keeps its row in lane-relative order:
// register d holds column i^d (the diagonal is register 0).  Then every
// exchange between lanes is "read register e of lane i^x" with x and e fixed
// at compile time: XOR 1, 2, 3 by DPP quad permutes and XOR 7 by the DPP
// half-row mirror inside the VALU, XOR 4..6 by the LDS crossbar's bit-mask
// swizzle (no memory access).  Sweeps run until the off-diagonal Frobenius norm of
// every matrix in the wavefront is below 1e-15 of its norm; eigenpairs are
// then sorted ascending.
#include <type_traits>

#include "internal.h"

namespace ephx {
namespace {

// value of lane (lane ^ X) within each group of 8 lanes
template <int X>
__device__ __forceinline__ int xlane(int v) {
    static_assert(X >= 0 && X < 8, "lane offset");
    constexpr int kQuad = X == 1 ? 0xB1 : (X == 2 ? 0x4E : 0x1B);   // XOR 1, 2, 3
    constexpr int kMirror = 0x141;                                                      // lane -> 7 - lane
    // every lane has a source under these permutations, so the destination is
    // written in full (bound_ctrl set: no "old" value has to be placed first);
    // the callers run with every lane of the wavefront active
    if (X == 0) return v;
    if (X <= 3) return __builtin_amdgcn_update_dpp(0, v, kQuad, 0xF, 0xF, true);
    if (X == 7) return __builtin_amdgcn_update_dpp(0, v, kMirror, 0xF, 0xF, true);
    // XOR 4..6 would take two DPP moves; the LDS crossbar's bit-mask swizzle
    // (lane ^ X within groups of 32, no memory access) does it in one
    // instruction outside the VALU, which this solver keeps busy
    return __builtin_amdgcn_ds_swizzle(v, 0x1F | (X << 10));
}
template <int X>
__device__ __forceinline__ double xlane(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = xlane<X>((int)(b & 0xffffffffLL)), hi = xlane<X>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

struct Cx {
    double r, i;
};

// 1/b and 1/sqrt(x) from the hardware estimates refined by two Newton steps
// each (quadratic convergence from the estimate's ~1e-8 relative error to the
// last bits); b > 0, x >= 1 where they are used.
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

// Columns c1 = i^D (register D) and c2 = i^D^M (register E = D^M) form one pair
// of the round, rotated with the parameters of lane i^D's pair.  With X_p, X_q
// the columns of the pair (p < q),
//   (XJ)_{.p} = c X_p - conj(se) X_q ,   (XJ)_{.q} = c X_q + se X_p ,
// so each register is updated as  x_D <- c x_D + s_D x_E,  x_E <- c x_E + s_E x_D
// with s = -conj(se) for the p column and s = se for the q column: the two
// differ only in the sign of the real part, so no operand is selected.
template <int R, int M, int D>
__device__ __forceinline__ void column_pair(int i, Cx (&a)[R], Cx (&v)[R], double c, double sr, double si) {
    constexpr int E = D ^ M;
    constexpr int kTop = M >= 4 ? 4 : (M >= 2 ? 2 : 1);   // highest bit of M
    const double cc = xlane<D>(c), s_r = xlane<D>(sr), s_i = xlane<D>(si);
    const bool d_is_p = ((i ^ D) & kTop) == 0;
    const double rd = d_is_p ? -s_r : s_r;   // real part of s_D; s_E has -rd
    const Cx xd = a[D], xe = a[E];
    a[D] = Cx{fma(cc, xd.r, fma(rd, xe.r, -s_i * xe.i)), fma(cc, xd.i, fma(rd, xe.i, s_i * xe.r))};
    a[E] = Cx{fma(cc, xe.r, fma(-rd, xd.r, -s_i * xd.i)), fma(cc, xe.i, fma(-rd, xd.i, s_i * xd.r))};
    const Cx yd = v[D], ye = v[E];
    v[D] = Cx{fma(cc, yd.r, fma(rd, ye.r, -s_i * ye.i)), fma(cc, yd.i, fma(rd, ye.i, s_i * ye.r))};
    v[E] = Cx{fma(cc, ye.r, fma(-rd, yd.r, -s_i * yd.i)), fma(cc, ye.i, fma(-rd, yd.i, s_i * yd.r))};
}

template <int R, int M, int D>
__device__ __forceinline__ void column_pairs(int i, Cx (&a)[R], Cx (&v)[R], double c, double sr, double si) {
    if constexpr (D < R) {
        if constexpr (D < (D ^ M)) column_pair<R, M, D>(i, a, v, c, sr, si);
        column_pairs<R, M, D + 1>(i, a, v, c, sr, si);
    }
}

template <int R, int M, int D>
__device__ __forceinline__ void fetch_partner_row(const Cx (&a)[R], Cx (&q)[R]) {
    // partner row i^M, column i^D sits in the partner's register D^M
    if constexpr (D < R) {
        q[D].r = xlane<M>(a[D ^ M].r);
        q[D].i = xlane<M>(a[D ^ M].i);
        fetch_partner_row<R, M, D + 1>(a, q);
    }
}

template <int R, int M>
__device__ __forceinline__ void jacobi_round(int i, Cx (&a)[R], Cx (&v)[R]) {
    // rotation of the pair (i, i^M), evaluated by its lower lane and copied
    const bool lower = i < (i ^ M);
    const double dself = a[0].r;
    const double dpart = xlane<M>(a[0].r);
    // t and s of the header, divided by |a_pq| so that neither |a_pq| nor the
    // phase needs its own root or quotient: with d = a_qq - a_pp and
    // m2 = |a_pq|^2, t/|a_pq| = 2 sgn(d)/(|d| + sqrt(d^2 + 4 m2)) and
    // se = (t/|a_pq|) c a_pq
    const double apr = a[M].r, api = a[M].i;   // A[i][i^M]
    const double m2 = apr * apr + api * api;
    const double d = dpart - dself;
    const double tm = (d >= 0.0 ? 2.0 : -2.0) * recip(fabs(d) + sqrt(fma(d, d, 4.0 * m2)));
    const double c0 = rsqrt1(fma(tm * tm, m2, 1.0));
    const double w = tm * c0;
    const bool rot = m2 > 0.0;
    double c = rot ? c0 : 1.0;
    double sr = rot ? w * apr : 0.0;
    double si = rot ? w * api : 0.0;
    const double cp = xlane<M>(c), srp = xlane<M>(sr), sip = xlane<M>(si);
    c = lower ? c : cp;
    sr = lower ? sr : srp;
    si = lower ? si : sip;
    // column rotations A J and V J for every pair of the round
    column_pairs<R, M, 0>(i, a, v, c, sr, si);
    // row rotation J^dag A with the partner row: lower row p <- c A_p - se A_q,
    // upper row q <- c A_q + conj(se) A_p, i.e. a <- c a + t q with
    // t = (-sr, -si) or (sr, -si)
    Cx q[R];
    fetch_partner_row<R, M, 0>(a, q);
    const double tr = lower ? -sr : sr;
#pragma unroll
    for (int d = 0; d < R; ++d)
        a[d] = Cx{fma(c, a[d].r, fma(tr, q[d].r, si * q[d].i)), fma(c, a[d].i, fma(tr, q[d].i, -si * q[d].r))};
}

template <int R, int M>
__device__ __forceinline__ void jacobi_sweep(int i, Cx (&a)[R], Cx (&v)[R]) {
    if constexpr (M < R) {
        jacobi_round<R, M>(i, a, v);
        jacobi_sweep<R, M + 1>(i, a, v);
    }
}

template <int R, int X>
__device__ __forceinline__ double group_sum(double x) {
    if constexpr (X < R) return group_sum<R, 2 * X>(x + xlane<X>(x));
    return x;
}

template <int R, int E>
__device__ __forceinline__ void rank_step(int i, int n, double d, int& rk) {
    if constexpr (E < R) {
        const double de = xlane<E>(d);
        const int j = i ^ E;
        rk += (E != 0 && j < n && (de < d || (de == d && j < i))) ? 1 : 0;
        rank_step<R, E + 1>(i, n, d, rk);
    }
}

template <int R, int E, typename F>
__device__ __forceinline__ void for_offsets(F&& f) {
    if constexpr (E < R) {
        f(std::integral_constant<int, E>{});
        for_offsets<R, E + 1>(f);
    }
}

// PK = false: A holds n*n complex entries per matrix (stride strideA complex
// elements) and the Hermitian part 0.5 (A + A^dag) is taken.  PK = true: A
// holds the packed Hermitian form, n*n reals per matrix (stride strideA reals)
// with P[i][j] = Re X_ij for i <= j and P[i][j] = Im X_ji for i > j.
template <typename Tin, int N, bool PK = false>
__global__ __launch_bounds__(256) void k_eig_rows(int batch, const Tin* __restrict__ A, long strideA,
                                                  double* __restrict__ evals, double* __restrict__ evecs) {
    constexpr int R = N <= 1 ? 1 : (N <= 2 ? 2 : (N <= 4 ? 4 : 8));
    const int lane = threadIdx.x & 63;
    const long slot = ((long)blockIdx.x * 256 + threadIdx.x) / R;
    const int i = lane % R;
    const bool valid = slot < batch;
    const bool act = valid && i < N;
    Cx a[R], v[R];
#pragma unroll
    for (int d = 0; d < R; ++d) {
        a[d] = Cx{0.0, 0.0};
        v[d] = Cx{d == 0 ? 1.0 : 0.0, 0.0};
    }
    if (act && PK) {
        const Tin* ab = A + slot * strideA;
#pragma unroll
        for (int d = 0; d < R; ++d) {
            const int j = i ^ d;
            if (j < N) {
                const int lo = i < j ? i : j, hi = i < j ? j : i;
                const double re = (double)ab[lo * N + hi];
                const double im = d == 0 ? 0.0 : (i < j ? 1.0 : -1.0) * (double)ab[hi * N + lo];
                a[d] = Cx{re, im};
            }
        }
    } else if (act) {
        const Tin* ab = A + slot * strideA * 2;
#pragma unroll
        for (int d = 0; d < R; ++d) {
            const int j = i ^ d;
            if (j < N) {
                // Hermitian part 0.5 (A + A^dag)
                const double xr = (double)ab[2 * (i * N + j)], xi = (double)ab[2 * (i * N + j) + 1];
                const double yr = (double)ab[2 * (j * N + i)], yi = (double)ab[2 * (j * N + i) + 1];
                a[d] = Cx{0.5 * (xr + yr), 0.5 * (xi - yi)};
            }
        }
    }
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, tot = 0.0;
#pragma unroll
        for (int d = 0; d < R; ++d) {
            const double m2 = a[d].r * a[d].r + a[d].i * a[d].i;
            tot += m2;
            off += d != 0 ? m2 : 0.0;
        }
        off = group_sum<R, 1>(off);
        tot = group_sum<R, 1>(tot);
        const bool done = !(off > 1e-30 * tot);
        if (__all(done)) break;
        jacobi_sweep<R, 1>(i, a, v);
    }
    // sort ascending, ties by index
    const double dv = a[0].r;
    int rk = 0;
    rank_step<R, 0>(i, N, dv, rk);
    if (act) evals[slot * N + rk] = dv;
    if (evecs != nullptr) {
        // V[i][c] with c = i^e sits in register e; its column goes to rank(c)
        for_offsets<R, 0>([&](auto ec) {
            constexpr int E = decltype(ec)::value;
            const int rc = xlane<E>(rk);
            const int c = i ^ E;
            if (act && c < N) {
                const long off = ((slot * N + i) * N + rc) * 2;
                evecs[off] = v[E].r;
                evecs[off + 1] = v[E].i;
            }
        });
    }
}

// Larger matrices (8 < n <= 128, e.g. H(k) of a 64-function model, D(q) of a
// 40-atom cell): one 256-thread workgroup per matrix, the same rotations and
// convergence test, with the n/2 disjoint rotations of a round (circle-method
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
    const int R = n <= 1 ? 1 : (n <= 2 ? 2 : (n <= 4 ? 4 : 8));
    const long threads = (long)batch * R;
    dim3 grid((unsigned)((threads + 255) / 256));
    switch (n) {
#define EPHX_EIG_CASE(NN) \
    case NN:                                                                                                \
        hipLaunchKernelGGL((k_eig_rows<Tin, NN, PK>), grid, dim3(256), 0, st, batch, A, strideA, evals, evecs); \
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
