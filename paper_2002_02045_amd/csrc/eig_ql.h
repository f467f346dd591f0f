// One Hermitian eigenproblem of order N <= 8 per lane, in FP64:
// Householder reduction to a real symmetric tridiagonal T = Q^H A Q, the
// implicit QL iteration with Wilkinson shifts on T = Z L Z^T, and the
// eigenvectors U = Q Z (Golub & Van Loan, "Matrix Computations", Secs. 8.3.1
// and 8.3.5; the reflectors in the form H = I - tau v v^H with a real image
// beta e_1, as LAPACK's zlarfg/zhetd2 define them).
//
// The outer indices (reflector j, QL block start l) are template parameters
// and every other loop has constant bounds, so all array indices are
// compile-time constants: the matrix, the reflectors and Z stay in registers.
// The QL sweep over rows i = m-1 .. l of the active block [l, m] (m found at
// run time) runs over all compile-time rows under a per-lane predicate, so
// lanes holding different matrices execute the same instructions.  MathT
// supplies rsqrt(x), rcp(x) and any(pred) (a wavefront vote on the device,
// the value itself on the host).
#pragma once

namespace ephx {

template <int N>
struct HermLane {
    // lower triangle of A (i >= j) on input; after the reduction, the
    // reflector vectors below the subdiagonal (leading 1 implicit)
    double ar[N][N], ai[N][N];
    double taur[N], taui[N];
    double d[N], e[N];  // T: d diagonal, e[i] couples i and i+1 (e[N-1] = 0)
    double z[N][N];     // eigenvectors of T, column c belongs to d[c]
};

// reflector j: H_j^H A[j+1.., j] = beta e_1, then A <- H_j^H A H_j on the
// trailing block
template <class MathT, int N, int J>
__host__ __device__ __forceinline__ void herm_reflect(HermLane<N>& s) {
    if constexpr (J < N - 1) {
        constexpr int L = N - 1 - J;
        const double alr = s.ar[J + 1][J], ali = s.ai[J + 1][J];
        double xn2 = 0.0;
#pragma unroll
        for (int i = J + 2; i < N; ++i) xn2 = fma(s.ar[i][J], s.ar[i][J], fma(s.ai[i][J], s.ai[i][J], xn2));
        const bool ident = xn2 == 0.0 && ali == 0.0;
        const double nrm2 = alr * alr + ali * ali + xn2;
        const double nrm = nrm2 * MathT::rsqrt(ident ? 1.0 : nrm2);
        const double beta = ident ? alr : (alr >= 0.0 ? -nrm : nrm);
        const double ib = MathT::rcp(ident ? 1.0 : beta);
        const double tr = ident ? 0.0 : (beta - alr) * ib, ti = ident ? 0.0 : -ali * ib;
        // v = x / (alpha - beta) below its leading 1
        const double dr = alr - beta, di = ali;
        const double den = MathT::rcp(ident ? 1.0 : dr * dr + di * di);
        const double sr = ident ? 1.0 : dr * den, si = ident ? 0.0 : -di * den;
        double vr[L], vi[L], pr[L], pi[L];
        vr[0] = 1.0;
        vi[0] = 0.0;
#pragma unroll
        for (int a = 1; a < L; ++a) {
            const double xr = s.ar[J + 1 + a][J], xi = s.ai[J + 1 + a][J];
            vr[a] = xr * sr - xi * si;
            vi[a] = xr * si + xi * sr;
            s.ar[J + 1 + a][J] = vr[a];
            s.ai[J + 1 + a][J] = vi[a];
        }
        s.taur[J] = tr;
        s.taui[J] = ti;
        s.e[J] = beta;
        // p = tau A v, w = p - (1/2) tau (p^H v) v, A -= v w^H + w v^H
#pragma unroll
        for (int a = 0; a < L; ++a) {
            double yr = 0.0, yi = 0.0;
#pragma unroll
            for (int b = 0; b < L; ++b) {
                const int ia = J + 1 + a, ibb = J + 1 + b;
                const double mr = a >= b ? s.ar[ia][ibb] : s.ar[ibb][ia];
                const double mi = a > b ? s.ai[ia][ibb] : (a == b ? 0.0 : -s.ai[ibb][ia]);
                yr = fma(mr, vr[b], fma(-mi, vi[b], yr));
                yi = fma(mr, vi[b], fma(mi, vr[b], yi));
            }
            pr[a] = tr * yr - ti * yi;
            pi[a] = tr * yi + ti * yr;
        }
        double hr = 0.0, hi = 0.0;   // p^H v
#pragma unroll
        for (int a = 0; a < L; ++a) {
            hr = fma(pr[a], vr[a], fma(pi[a], vi[a], hr));
            hi = fma(pr[a], vi[a], fma(-pi[a], vr[a], hi));
        }
        const double kr = -0.5 * (tr * hr - ti * hi), ki = -0.5 * (tr * hi + ti * hr);
#pragma unroll
        for (int a = 0; a < L; ++a) {
            const double wr = pr[a] + kr * vr[a] - ki * vi[a];
            const double wi = pi[a] + kr * vi[a] + ki * vr[a];
            pr[a] = wr;
            pi[a] = wi;
        }
#pragma unroll
        for (int a = 0; a < L; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                // minus v_a conj(w_b) + w_a conj(v_b), as FMAs into the entry
                double& xr = s.ar[J + 1 + a][J + 1 + b];
                xr = fma(-vr[a], pr[b], fma(-vi[a], pi[b], fma(-pr[a], vr[b], fma(-pi[a], vi[b], xr))));
                if (a != b) {
                    double& xi = s.ai[J + 1 + a][J + 1 + b];
                    xi = fma(-vi[a], pr[b], fma(vr[a], pi[b], fma(-pi[a], vr[b], fma(pr[a], vi[b], xi))));
                }
            }
        herm_reflect<MathT, N, J + 1>(s);
    }
}

template <class MathT, int N>
__host__ __device__ __forceinline__ void herm_tridiagonalize(HermLane<N>& s) {
    herm_reflect<MathT, N, 0>(s);
#pragma unroll
    for (int i = 0; i < N; ++i) s.d[i] = s.ar[i][i];
    s.e[N - 1] = 0.0;
}

// Implicit QL iterations deflating row l; e[m] counts as zero once
// |e[m]| <= 2^-53 (|d[m]| + |d[m+1]|).  Every update is a select on the
// lane's predicates, and the sweep's rotations reach Z after the sweep, one
// row of Z at a time: written so, the compiler keeps one copy of Z and no
// copies of it at the joins of the predicated code.
template <class MathT, int N, int L>
__host__ __device__ __forceinline__ void ql_deflate(double (&d)[N], double (&e)[N], double (&z)[N][N], int max_iter) {
    if constexpr (L < N - 1) {
        for (int it = 0; it < max_iter; ++it) {
            int m = N - 1;
#pragma unroll
            for (int mm = N - 2; mm >= L; --mm)
                m = fabs(e[mm]) <= 1.1102230246251565e-16 * (fabs(d[mm]) + fabs(d[mm + 1])) ? mm : m;
            const bool act = m != L;
            if (!MathT::any(act)) break;
            double dm = d[N - 1];
#pragma unroll
            for (int mm = L; mm < N - 1; ++mm) dm = m == mm ? d[mm] : dm;
            // Wilkinson shift from the leading 2x2 block of [L, m]
            const double el = act ? e[L] : 1.0;
            double g = (d[L + 1] - d[L]) * MathT::rcp(2.0 * el);
            const double r = (g * g + 1.0) * MathT::rsqrt(g * g + 1.0);
            g = dm - d[L] + el * MathT::rcp(g + (g >= 0.0 ? r : -r));
            double sn = 1.0, cs = 1.0, p = 0.0;
            double zs[N - 1], zc[N - 1];
            bool brk = false;
#pragma unroll
            for (int i = N - 2; i >= L; --i) {
                const bool on = act && i < m && !brk;
                const double f = sn * e[i], b = cs * e[i];
                const double r2 = f * f + g * g;
                const bool zero = on && r2 == 0.0;
                const bool upd = on && !zero;
                // a lane that does not update (r2 = 0 among them, where ir is
                // infinite) discards all that ir feeds through the selects
                // below, so the inverse root waits on nothing but r2
                const double ir = MathT::rsqrt(r2);
                const double s1 = f * ir, c1 = g * ir;
                const double g1 = d[i + 1] - p;
                const double q1 = (d[i] - g1) * s1 + 2.0 * c1 * b;
                const double p1 = s1 * q1;
                e[i + 1] = upd ? r2 * ir : e[i + 1];
                d[i + 1] = upd ? g1 + p1 : (zero ? d[i + 1] - p : d[i + 1]);
                sn = upd ? s1 : sn;
                cs = upd ? c1 : cs;
                p = upd ? p1 : p;
                g = upd ? c1 * q1 - b : g;
                brk = brk || zero;
                zs[i] = upd ? s1 : 0.0;
                zc[i] = upd ? c1 : 1.0;
            }
            // the sweep's rotations applied to the rows of Z, one row at a time
#pragma unroll
            for (int k = 0; k < N; ++k)
#pragma unroll
                for (int i = N - 2; i >= L; --i) {
                    const double zf = z[k][i + 1];
                    z[k][i + 1] = zs[i] * z[k][i] + zc[i] * zf;
                    z[k][i] = zc[i] * z[k][i] - zs[i] * zf;
                }
            const bool fin = act && !brk;
            d[L] = fin ? d[L] - p : d[L];
            e[L] = fin ? g : e[L];
            // e[m] is zero after the sweep, completed or cut short
#pragma unroll
            for (int mm = L + 1; mm < N; ++mm) e[mm] = act && m == mm ? 0.0 : e[mm];
        }
        ql_deflate<MathT, N, L + 1>(d, e, z, max_iter);
    }
}

template <class MathT, int N>
__host__ __device__ __forceinline__ void tridiag_ql(HermLane<N>& s, int max_iter = 60) {
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int c = 0; c < N; ++c) s.z[r][c] = r == c ? 1.0 : 0.0;
    ql_deflate<MathT, N, 0>(s.d, s.e, s.z, max_iter);
}

// Where the back-transform reads reflector J's entries (i >= J+2): the lane's
// registers by default; a caller may move some reflectors elsewhere (the
// device solver keeps the first ones in LDS while QL runs).
template <int N>
struct ReflInRegs {
    const HermLane<N>& s;
    __host__ __device__ __forceinline__ double re(int i, int j) const { return s.ar[i][j]; }
    __host__ __device__ __forceinline__ double im(int i, int j) const { return s.ai[i][j]; }
};

// Column C of U = Q Z, Q = H_0 H_1 ... H_{N-2}: reflector J applied to rows
// J+1 .. after the reflectors above it.  Columns are independent, so a caller
// forms and stores them one at a time.
template <int N, int J, class RS>
__host__ __device__ __forceinline__ void herm_back_step(const HermLane<N>& s, const RS& rs, double (&xr)[N],
                                                        double (&xi)[N]) {
    if constexpr (J >= 0) {
        const double tr = s.taur[J], ti = s.taui[J];
        // y = v^H x
        double yr = xr[J + 1], yi = xi[J + 1];
#pragma unroll
        for (int i = J + 2; i < N; ++i) {
            const double vr = rs.re(i, J), vi = rs.im(i, J);
            yr = fma(vr, xr[i], fma(vi, xi[i], yr));
            yi = fma(vr, xi[i], fma(-vi, xr[i], yi));
        }
        // x -= tau v y
        const double tyr = tr * yr - ti * yi, tyi = tr * yi + ti * yr;
        xr[J + 1] -= tyr;
        xi[J + 1] -= tyi;
#pragma unroll
        for (int i = J + 2; i < N; ++i) {
            const double vr = rs.re(i, J), vi = rs.im(i, J);
            xr[i] = fma(-vr, tyr, fma(vi, tyi, xr[i]));
            xi[i] = fma(-vr, tyi, fma(-vi, tyr, xi[i]));
        }
        herm_back_step<N, J - 1>(s, rs, xr, xi);
    }
}

template <int N, int C, class RS>
__host__ __device__ __forceinline__ void herm_eigenvector(const HermLane<N>& s, const RS& rs, double (&xr)[N],
                                                          double (&xi)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        xr[i] = s.z[i][C];
        xi[i] = 0.0;
    }
    herm_back_step<N, N - 2>(s, rs, xr, xi);
}

// rank of each eigenvalue in ascending order, ties by index
template <int N>
__host__ __device__ __forceinline__ void eig_ranks(const double (&d)[N], int (&rk)[N]) {
#pragma unroll
    for (int c = 0; c < N; ++c) {
        int r = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) r += (d[k] < d[c] || (d[k] == d[c] && k < c)) ? 1 : 0;
        rk[c] = r;
    }
}

}  // namespace ephx
