// Batched Hermitian eigensolvers in FP64 for the small matrices of the method:
// H(k) and H(k+q) (n = Nw, Eq. wannier_3) and D(q) (n = 3 nat, Eq. IFC2).
//
// n <= 8: one matrix per lane, 64 per wavefront: Householder reduction to a
// real tridiagonal matrix, implicit QL with Wilkinson shifts, eigenvectors
// U = Q Z (eig_ql.h).  About 240 VALU instructions per 8 x 8 matrix against
// about 950 for cyclic Jacobi with one lane per row, which it replaces.
//
// 8 < n <= 128: the same three steps with one wavefront per matrix (the
// reduction and QL) and one workgroup per matrix for U = Q Z (k_eig_tql,
// k_eig_tqlv), in place of cyclic Jacobi with one workgroup per matrix (5x
// faster at n = 64, 4x at n = 120).
//
// Both sort the eigenpairs ascending, ties by index.
#include "internal.h"
#include "eig_ql.h"

namespace ephx {
namespace {

// 1/b and 1/sqrt(x) from the hardware estimates (relative error below 6e-8,
// measured) and one third-order correction each: with e the estimate's
// residual, 1/b = r / (1 - e), e = 1 - b r, and 1/sqrt(x) = y (1 - e)^(-1/2),
// e = 1 - x y^2, truncated after e^2 (the dropped terms are below 1e-21
// relative).  Any nonzero b, any positive normal x; within 2 ulp (measured),
// as two Newton steps, with three dependent operations after the estimate
// instead of four (1/b) and four instead of six (1/sqrt(x)): the QL rotation
// chain, one inverse root per rotation, is latency-bound.
__device__ __forceinline__ double recip(double b) {
    const double r = __builtin_amdgcn_rcp(b);
    const double e = fma(-b, r, 1.0);
    return fma(r, fma(e, e, e), r);
}
__device__ __forceinline__ double rsqrt1(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
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

// column C of U to its ranked column: row-major (entry (i, c) at i N + c), or
// column-major when cm (at c N + i: the column is one contiguous 16 N bytes,
// whole cache lines, where the row-major stores land 16 N bytes apart and
// leave lines half written)
template <int N, int C, class RS>
__device__ __forceinline__ void store_lane_vectors(const HermLane<N>& s, const RS& rs, const int (&rk)[N],
                                                   double* out, int cm) {
    if constexpr (C < N) {
        double xr[N], xi[N];
        herm_eigenvector<N, C>(s, rs, xr, xi);
#pragma unroll
        for (int i = 0; i < N; ++i)
            *reinterpret_cast<double2*>(out + (cm ? rk[C] * N + i : i * N + rk[C]) * 2) = double2{xr[i], xi[i]};
        // the next column reads the reflectors in LDS again rather than
        // holding them in registers across columns
        __asm__ volatile("" ::: "memory");
        store_lane_vectors<N, C + 1>(s, rs, rk, out, cm);
    }
}

// The 8 x 8 solver keeps reflectors 0..3 (18 complex entries, 288 bytes per
// lane) in LDS from the end of the reduction to the back-transform, entry e
// of lane t at [e][t].  Its registers then stay under 256 and two 256-lane
// workgroups (72 KB of LDS each) share a CU: two waves per SIMD, one issuing
// while the other waits on the QL rotation chain.  (Parked in global memory
// instead, the reflectors of the resident waves did not stay in L2.)
constexpr int kReflLds = 4;
template <int N>
constexpr int refl_lds_entries() {
    int c = 0;
    for (int j = 0; j < kReflLds && j < N - 2; ++j) c += N - 2 - j;
    return c;
}
__host__ __device__ constexpr int refl_entry(int n, int i, int j) { return j * (n - 2) - j * (j - 1) / 2 + (i - j - 2); }

template <int N>
struct ReflInLds {
    const HermLane<N>& s;
    const double2* lds;
    int t;
    __device__ __forceinline__ double re(int i, int j) const {
        return j < kReflLds ? lds[refl_entry(N, i, j) * 256 + t].x : s.ar[i][j];
    }
    __device__ __forceinline__ double im(int i, int j) const {
        return j < kReflLds ? lds[refl_entry(N, i, j) * 256 + t].y : s.ai[i][j];
    }
};

// One matrix per lane (n <= 8): Householder tridiagonalisation, implicit QL,
// eigenvectors U = Q Z (eig_ql.h).  PK selects the packed Hermitian input, else the Hermitian part of a complex
// n x n matrix is taken; eigenvalues ascending, ties by index, eigenvector c
// in column c of evecs[slot] (row-major complex n x n).
template <typename Tin, int N, bool PK = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(N == 8 ? 2 : 1))) void k_eig_lane(
    int batch, const Tin* __restrict__ A, long strideA, double* __restrict__ evals, double* __restrict__ evecs,
    int cm) {
    constexpr bool LR = N == 8;
    constexpr int NE = LR ? refl_lds_entries<N>() : 1;
    __shared__ double2 rl[NE * 256];
    const int tid = threadIdx.x;
    const long slot = (long)blockIdx.x * 256 + tid;
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
    if constexpr (LR) {
#pragma unroll
        for (int j = 0; j < kReflLds; ++j)
#pragma unroll
            for (int i = j + 2; i < N; ++i) rl[refl_entry(N, i, j) * 256 + tid] = double2{s.ar[i][j], s.ai[i][j]};
        // the entries are read back from LDS, not kept in registers
        __asm__ volatile("" ::: "memory");
    }
    tridiag_ql<LaneMath, N>(s);
    int rk[N];
    eig_ranks<N>(s.d, rk);
    if (!valid) return;
#pragma unroll
    for (int c = 0; c < N; ++c) evals[slot * N + rk[c]] = s.d[c];
    if (evecs == nullptr) return;
    if constexpr (LR)
        store_lane_vectors<N, 0>(s, ReflInLds<N>{s, rl, tid}, rk, evecs + slot * N * N * 2, cm);
    else
        store_lane_vectors<N, 0>(s, ReflInRegs<N>{s}, rk, evecs + slot * N * N * 2, cm);
}

constexpr int kWgMax = 128;   // largest order of the wavefront solver

// 8 < n <= 128 by Householder reduction and implicit QL (the one-lane solver's
// steps, spread over a wavefront), in two kernels.
//
// k_eig_tql: one wavefront per matrix, lane l owning rows l and l + 64.  The
// lower triangle of A is held in LDS (packed, complex); reflector j is formed
// from column j (a wavefront sum for the norm), p = tau A v row by row, the
// rank-2 update row by row, as in herm_reflect.  The reflectors and their tau
// go to the matrix's own slot of A (which the call overwrites), the same LDS
// then holds Z^T for the implicit QL on (d, e): the rotation chain is
// wavefront-uniform (every lane computes it), with the next d, e and Z entries
// read ahead of their use and the just-rotated Z entry carried in registers,
// so a rotation costs its arithmetic plus one LDS read and one write per row.
// The eigenvalues are ranked (ascending, ties by index) and Z's columns written
// to the slot in rank order.
//
// k_eig_tqlv: U = Q Z, one 256-thread workgroup per matrix, TPC threads per
// column of Z holding 16 rows each; a reflector's inner product is summed over
// the column's threads by lane exchanges.
//
// Slot of matrix mi (2 n^2 doubles of A): [0, n^2) Z^T in rank order,
// [n^2, n^2 + 2(n-1)) tau, then reflector j's entries i = j+2 .. n-1 at
// j(n-2) - j(j-1)/2 + (i - j - 2) (complex).
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}
__device__ __forceinline__ int tri_idx(int i, int m) { return i * (i + 1) / 2 + m; }
__device__ __forceinline__ int refl_base(int n, int j) { return j * (n - 2) - j * (j - 1) / 2; }

template <int R>
__global__ __launch_bounds__(64) void k_eig_tql(int n, double* __restrict__ A, long strideA,
                                                double* __restrict__ evals) {
    constexpr int NMAX = 64 * R;
    constexpr int REG = NMAX * (NMAX + 1);   // doubles: packed lower triangle (complex), later Z^T
    __shared__ __attribute__((aligned(16))) double lds[REG + 4 * NMAX];
    __shared__ double dd[NMAX], ee[NMAX];
    __shared__ int rk[NMAX];
    double2* a = reinterpret_cast<double2*>(lds);
    double2* vv = reinterpret_cast<double2*>(lds + REG);
    double2* ww = vv + NMAX;
    const int l = threadIdx.x;
    const long mi = blockIdx.x;
    double* ga = A + mi * strideA * 2;
    const long nn = (long)n * n;
    // Hermitian part 0.5 (A + A^dag), lower triangle
    for (int i = 0; i < n; ++i)
        for (int m = l; m <= i; m += 64) {
            const double xr = ga[2 * (i * n + m)], xi = ga[2 * (i * n + m) + 1];
            const double yr = ga[2 * (m * n + i)], yi = ga[2 * (m * n + i) + 1];
            a[tri_idx(i, m)] = i == m ? double2{xr, 0.0} : double2{0.5 * (xr + yr), 0.5 * (xi - yi)};
        }
    __syncthreads();
    // reflector j: H_j^H A[j+1.., j] = beta e_1, A <- H_j^H A H_j on the trailing block
    for (int j = 0; j < n - 1; ++j) {
        const double2 al = a[tri_idx(j + 1, j)];
        double xn2 = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = l + 64 * r;
            if (i >= j + 2 && i < n) {
                const double2 x = a[tri_idx(i, j)];
                xn2 = fma(x.x, x.x, fma(x.y, x.y, xn2));
            }
        }
        xn2 = wave_sum(xn2);
        const bool ident = xn2 == 0.0 && al.y == 0.0;
        const double nrm2 = al.x * al.x + al.y * al.y + xn2;
        const double nrm = nrm2 * rsqrt1(ident ? 1.0 : nrm2);
        const double beta = ident ? al.x : (al.x >= 0.0 ? -nrm : nrm);
        const double ib = recip(ident ? 1.0 : beta);
        const double tr = ident ? 0.0 : (beta - al.x) * ib, ti = ident ? 0.0 : -al.y * ib;
        const double dr = al.x - beta, di = al.y;
        const double den = recip(ident ? 1.0 : dr * dr + di * di);
        const double sr = ident ? 1.0 : dr * den, si = ident ? 0.0 : -di * den;
        double2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = l + 64 * r;
            v[r] = double2{0.0, 0.0};
            if (i == j + 1) v[r] = double2{1.0, 0.0};
            if (i >= j + 2 && i < n) {
                const double2 x = a[tri_idx(i, j)];
                v[r] = double2{x.x * sr - x.y * si, x.x * si + x.y * sr};
                a[tri_idx(i, j)] = v[r];
                const long q = nn + 2 * (n - 1) + 2 * (refl_base(n, j) + (i - j - 2));
                ga[q] = v[r].x;
                ga[q + 1] = v[r].y;
            }
            if (i >= j + 1 && i < n) vv[i] = v[r];
        }
        if (l == 0) {
            ga[nn + 2 * j] = tr;
            ga[nn + 2 * j + 1] = ti;
            ee[j] = beta;
        }
        __syncthreads();
        // p = tau A v on the trailing block, row by row
        double2 p[R];
        double hr = 0.0, hi = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = l + 64 * r;
            p[r] = double2{0.0, 0.0};
            if (i >= j + 1 && i < n) {
                double yr = 0.0, yi = 0.0;
                for (int m = j + 1; m < n; ++m) {
                    double mr, mim;
                    if (m <= i) {
                        const double2 t = a[tri_idx(i, m)];
                        mr = t.x;
                        mim = m == i ? 0.0 : t.y;
                    } else {
                        const double2 t = a[tri_idx(m, i)];
                        mr = t.x;
                        mim = -t.y;
                    }
                    const double2 vm = vv[m];
                    yr = fma(mr, vm.x, fma(-mim, vm.y, yr));
                    yi = fma(mr, vm.y, fma(mim, vm.x, yi));
                }
                p[r] = double2{tr * yr - ti * yi, tr * yi + ti * yr};
                hr = fma(p[r].x, v[r].x, fma(p[r].y, v[r].y, hr));
                hi = fma(p[r].x, v[r].y, fma(-p[r].y, v[r].x, hi));
            }
        }
        hr = wave_sum(hr);
        hi = wave_sum(hi);
        const double kr = -0.5 * (tr * hr - ti * hi), ki = -0.5 * (tr * hi + ti * hr);
        double2 w[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = l + 64 * r;
            w[r] = double2{p[r].x + kr * v[r].x - ki * v[r].y, p[r].y + kr * v[r].y + ki * v[r].x};
            if (i >= j + 1 && i < n) ww[i] = w[r];
        }
        __syncthreads();
        // A -= v w^H + w v^H on the lower triangle of the trailing block
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = l + 64 * r;
            if (i >= j + 1 && i < n) {
                for (int m = j + 1; m <= i; ++m) {
                    // minus v_i conj(w_m) + w_i conj(v_m), as FMAs into the entry
                    const double2 vm = vv[m], wm = ww[m];
                    double2 t = a[tri_idx(i, m)];
                    t.x = fma(-v[r].x, wm.x, fma(-v[r].y, wm.y, fma(-w[r].x, vm.x, fma(-w[r].y, vm.y, t.x))));
                    if (m != i)
                        t.y = fma(-v[r].y, wm.x, fma(v[r].x, wm.y, fma(-w[r].y, vm.x, fma(w[r].x, vm.y, t.y))));
                    a[tri_idx(i, m)] = t;
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = l + 64 * r;
        if (i < n) dd[i] = a[tri_idx(i, i)].x;
    }
    if (l == 0) ee[n - 1] = 0.0;
    __syncthreads();
    // Z^T = I in the same LDS
    double* zt = lds;
    for (long e = l; e < nn; e += 64) zt[e] = (e / n == e % n) ? 1.0 : 0.0;
    __syncthreads();
    // implicit QL with Wilkinson shifts, deflating row L; e[m] counts as zero
    // once |e[m]| <= 2^-53 (|d[m]| + |d[m+1]|)
    for (int L = 0; L < n - 1; ++L) {
        for (int it = 0; it < 60; ++it) {
            int m = n - 1;
#pragma unroll
            for (int r = R - 1; r >= 0; --r) {
                const int mm = L + l + 64 * r;
                const bool neg = mm < n - 1 && fabs(ee[mm]) <= 1.1102230246251565e-16 * (fabs(dd[mm]) + fabs(dd[mm + 1]));
                const unsigned long long bal = __ballot(neg);
                if (bal) m = L + 64 * r + __builtin_ctzll(bal);
            }
            if (m == L) break;
            const double el = ee[L], dL = dd[L];
            double g = (dd[L + 1] - dL) * recip(2.0 * el);
            const double r0 = (g * g + 1.0) * rsqrt1(g * g + 1.0);
            g = dd[m] - dL + el * recip(g + (g >= 0.0 ? r0 : -r0));
            double s = 1.0, c = 1.0, p = 0.0;
            bool brk = false;
            // carried along the sweep: d[i+1] and, per row, Z[k][i+1]
            double di1 = dd[m];
            double zc[R], zn[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int k = l + 64 * r;
                zc[r] = k < n ? zt[(long)m * n + k] : 0.0;
                zn[r] = k < n ? zt[(long)(m - 1) * n + k] : 0.0;
            }
            double ei = ee[m - 1], di = dd[m - 1];
            int i = m - 1;
            for (; i >= L; --i) {
                // the next rotation's operands, read ahead
                const double ein = i > L ? ee[i - 1] : 0.0, din = i > L ? dd[i - 1] : 0.0;
                double znn[R];
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int k = l + 64 * r;
                    znn[r] = (i > L && k < n) ? zt[(long)(i - 1) * n + k] : 0.0;
                }
                const double f = s * ei, b = c * ei;
                const double r2 = f * f + g * g;
                if (r2 == 0.0) {
                    dd[i + 1] = di1 - p;
                    brk = true;
                    break;
                }
                const double ir = rsqrt1(r2);
                ee[i + 1] = r2 * ir;
                s = f * ir;
                c = g * ir;
                const double g1 = di1 - p;
                const double q1 = (di - g1) * s + 2.0 * c * b;
                p = s * q1;
                dd[i + 1] = g1 + p;
                g = c * q1 - b;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int k = l + 64 * r;
                    const double zf = zc[r];
                    if (k < n) zt[(long)(i + 1) * n + k] = s * zn[r] + c * zf;
                    zc[r] = c * zn[r] - s * zf;
                    zn[r] = znn[r];
                }
                di1 = di;
                ei = ein;
                di = din;
            }
            // Z[k][i+1] as carried (the sweep's last rotated entry, or the
            // untouched one where the sweep stopped)
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int k = l + 64 * r;
                if (k < n) zt[(long)(i + 1) * n + k] = zc[r];
            }
            if (!brk) {
                dd[L] = dd[L] - p;
                ee[L] = g;
            }
            ee[m] = 0.0;
            __syncthreads();
        }
    }
    __syncthreads();
    // ranks (ascending, ties by index), eigenvalues, Z^T rows in rank order
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int c = l + 64 * r;
        if (c < n) {
            const double dc = dd[c];
            int k = 0;
            for (int m = 0; m < n; ++m) k += (dd[m] < dc || (dd[m] == dc && m < c)) ? 1 : 0;
            rk[c] = k;
            evals[mi * n + k] = dc;
        }
    }
    __syncthreads();
    for (int c = 0; c < n; ++c) {
        const long dst = (long)rk[c] * n;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k = l + 64 * r;
            if (k < n) ga[dst + k] = zt[(long)c * n + k];
        }
    }
}

// U = Q Z from the slot k_eig_tql leaves (see there); TPC threads per column,
// 16 rows each (n <= 16 TPC).
template <int TPC>
__global__ __launch_bounds__(256) void k_eig_tqlv(int n, const double* __restrict__ A, long strideA,
                                                  double* __restrict__ evecs) {
    constexpr int RPT = 16, CPP = 256 / TPC, NMAX = RPT * TPC;
    __shared__ __attribute__((aligned(16))) double lds[NMAX * NMAX - NMAX];
    const int tid = threadIdx.x;
    const long mi = blockIdx.x;
    const double* ga = A + mi * strideA * 2;
    const long nn = (long)n * n;
    const int cnt = n * n - n;   // tau and the reflectors
    for (int e = tid; e < cnt; e += 256) lds[e] = ga[nn + e];
    __syncthreads();
    const double2* tau = reinterpret_cast<const double2*>(lds);
    const double2* refl = reinterpret_cast<const double2*>(lds + 2 * (n - 1));
    double* gv = evecs + mi * nn * 2;
    const int tc = tid / TPC, rb = tid % TPC;
    for (int c0 = 0; c0 < n; c0 += CPP) {
        const int c = c0 + tc;
        const bool cv = c < n;
        double xr[RPT], xi[RPT];
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = rb * RPT + r;
            xr[r] = (cv && i < n) ? ga[(long)c * n + i] : 0.0;
            xi[r] = 0.0;
        }
        for (int j = n - 2; j >= 0; --j) {
            const double2 t = tau[j];
            const int base = refl_base(n, j) - j - 2;
            double yr = 0.0, yi = 0.0;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = rb * RPT + r;
                if (i == j + 1) {
                    yr += xr[r];
                    yi += xi[r];
                } else if (i >= j + 2 && i < n) {
                    const double2 v = refl[base + i];
                    yr = fma(v.x, xr[r], fma(v.y, xi[r], yr));
                    yi = fma(v.x, xi[r], fma(-v.y, xr[r], yi));
                }
            }
#pragma unroll
            for (int o = 1; o < TPC; o <<= 1) {
                yr += __shfl_xor(yr, o, 64);
                yi += __shfl_xor(yi, o, 64);
            }
            const double tyr = t.x * yr - t.y * yi, tyi = t.x * yi + t.y * yr;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = rb * RPT + r;
                if (i == j + 1) {
                    xr[r] -= tyr;
                    xi[r] -= tyi;
                } else if (i >= j + 2 && i < n) {
                    const double2 v = refl[base + i];
                    xr[r] = fma(-v.x, tyr, fma(v.y, tyi, xr[r]));
                    xi[r] = fma(-v.x, tyi, fma(-v.y, tyr, xi[r]));
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = rb * RPT + r;
            if (cv && i < n) *reinterpret_cast<double2*>(gv + ((long)i * n + c) * 2) = double2{xr[r], xi[r]};
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
void launch_eig(int batch, int n, const Tin* A, long strideA, double* evals, double* evecs, int cm, hipStream_t st) {
    dim3 grid((unsigned)(((long)batch + 255) / 256));
    switch (n) {
#define EPHX_EIG_CASE(NN) \
    case NN:                                                                                                \
        hipLaunchKernelGGL((k_eig_lane<Tin, NN, PK>), grid, dim3(256), 0, st, batch, A, strideA, evals, evecs, cm); \
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
        if (n <= 64) {
            hipLaunchKernelGGL(k_eig_tql<1>, dim3((unsigned)batch), dim3(64), 0, st, n, (double*)A, strideA, evals);
            if (evecs)
                hipLaunchKernelGGL(k_eig_tqlv<4>, dim3((unsigned)batch), dim3(256), 0, st, n, (const double*)A,
                                   strideA, evecs);
        } else {
            hipLaunchKernelGGL(k_eig_tql<2>, dim3((unsigned)batch), dim3(64), 0, st, n, (double*)A, strideA, evals);
            if (evecs)
                hipLaunchKernelGGL(k_eig_tqlv<8>, dim3((unsigned)batch), dim3(256), 0, st, n, (const double*)A,
                                   strideA, evecs);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) throw Error{-3, std::string("eig_herm: ") + hipGetErrorString(e)};
        return;
    }
    if (a_f32)
        launch_eig(batch, n, (const float*)A, strideA, evals, evecs, 0, st);
    else
        launch_eig(batch, n, (const double*)A, strideA, evals, evecs, 0, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{-3, std::string("eig_herm: ") + hipGetErrorString(e)};
}

void eig_herm_packed(int batch, int n, const double* P, long strideP, double* evals, double* evecs, int evecs_cm,
                     hipStream_t st) {
    if (batch <= 0) return;
    if (n < 1 || n > kEigMax) throw Error{-6, "eig_herm_packed: matrix order must be 1..8"};
    if (strideP < (long)n * n) throw Error{-1, "eig_herm_packed: stride below n*n"};
    launch_eig<double, true>(batch, n, P, strideP, evals, evecs, evecs_cm, st);
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
