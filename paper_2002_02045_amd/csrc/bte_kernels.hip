// Boltzmann-equation kernels on grid states (paper Sec. 2.1 and 4.3).
//
// Pair table.  For states s = (k_s, n_s) and t = (k_t, n_t) on one grid,
// q = k_t - k_s and the table holds G[nu][s][t] = 1/2(|g(s->t)|^2 + |g(t->s)|^2).
//
// Collision integral in matrix form.  With Delta = e_s - e_t and the mode sum
// done once when parameters are set,
//   P_st = sum_nu s_nu G[nu][s][t] [ delta(Delta - hw)(N+1) + delta(Delta + hw) N ],
// Eq. e_ph_scattering becomes (using G_st = G_ts, omega(-q) = omega(q) and the
// evenness of the Gaussian)
//   I_s = -(2 pi/hbar)(1/N_q) [ f_s sum_t P_st (1 - f_t) - (1 - f_s) sum_t P_ts f_t ],
// so one pass over P (row sums and column sums together) evaluates I for any
// f: 4 S^2 bytes instead of the 4 S^2 3nat bytes of the per-mode table.
//
// Streaming pass.  A 256-thread workgroup owns a 1024-column tile and a run of
// rows sized so that the whole grid is resident at once; its four waves take
// the rows in turn, each lane holding 16 columns (four 16-byte nontemporal
// loads per row, one instruction reading 1 KB contiguously).  Row sums are
// reduced across the wave with shuffles, column sums stay in registers and are
// combined across the four waves through LDS at the end.  Partials go to
// rowp[a][col tile][row] and colp[b][row tile][col] and are reduced in a fixed
// order by the finishing kernel (no atomics; results are deterministic).
#include <algorithm>
#include <atomic>

#include "internal.h"

namespace ephx {
namespace {

inline void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{-3, std::string(what) + ": " + hipGetErrorString(e)};
}

template <typename T>
struct cx {
    T x, y;
};
template <typename T>
__device__ __forceinline__ cx<T> ldc(const T* p, long i) {
    return {p[2 * i], p[2 * i + 1]};
}
template <typename T>
__device__ __forceinline__ cx<T> ldcd(const double* p, long i) {
    return {(T)p[2 * i], (T)p[2 * i + 1]};
}
template <typename T>
__device__ __forceinline__ void cfma(cx<T>& acc, cx<T> a, cx<T> b) {
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
template <typename T>
__device__ __forceinline__ void cjfma(cx<T>& acc, cx<T> a, cx<T> b) {
    acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
}

__device__ __forceinline__ long grid_q(const int32_t* kc, int s, int t, int n1, int n2, int n3) {
    int a = kc[3 * t] - kc[3 * s], b = kc[3 * t + 1] - kc[3 * s + 1], c = kc[3 * t + 2] - kc[3 * s + 2];
    a += a < 0 ? n1 : 0;
    b += b < 0 ? n2 : 0;
    c += c < 0 ? n3 : 0;
    return ((long)a * n2 + b) * n3 + c;
}

// One thread per (source s in chunk, target t): rotation with conj(U(k_t))[:, n_t],
// mode projection with e(q)/sqrt(M) and sqrt(hbar^2/(2 M omega)), |g|^2 (FP32).
__global__ void k_pair_epilogue_f32(PairEpilogue e, long ld) {
    const int z = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= e.S) return;
    const int s = e.s_off + z;
    const int nw = e.nw, nm = e.nm;
    const long iq = grid_q(e.kc, s, t, e.n1, e.n2, e.n3);
    const float* gp = reinterpret_cast<const float*>(e.gw) + ((long)z * e.S + t) * nm * nw * 2;
    const int bt = e.band[t];
    const double* ut = e.ut + (long)t * nw * nw * 2;
    cx<float> gh[kMaxModes];
    for (int x = 0; x < nm; ++x) {
        cx<float> a = {0, 0};
        for (int i = 0; i < nw; ++i) cjfma(a, ldcd<float>(ut, (long)i * nw + bt), ldc(gp, (long)x * nw + i));
        gh[x] = a;
    }
    if (e.lr != nullptr) {
        const double* us = e.us + (long)s * nw * nw * 2;
        const int bs = e.band[s];
        cx<float> ov = {0, 0};
        for (int i = 0; i < nw; ++i) cjfma(ov, ldcd<float>(ut, (long)i * nw + bt), ldcd<float>(us, (long)i * nw + bs));
        for (int x = 0; x < nm; ++x) cfma(gh[x], ldcd<float>(e.lr, iq * nm + x), ov);
    }
    for (int nu = 0; nu < nm; ++nu) {
        const double om = e.omega[iq * nm + nu];
        float g2 = 0.f;
        if (om > e.omega_cut) {
            cx<float> g = {0, 0};
            for (int x = 0; x < nm; ++x) {
                cx<float> ev = ldcd<float>(e.evec, (iq * nm + x) * nm + nu);
                ev.x *= (float)e.minv[x];
                ev.y *= (float)e.minv[x];
                cfma(g, ev, gh[x]);
            }
            const float amp2 = (float)(kHbar2AmuA2 / (2.0 * om));
            g2 = amp2 * (g.x * g.x + g.y * g.y);
        }
        e.g2raw[((long)nu * e.S + s) * ld + t] = g2;
    }
}

// FP64 variant writing a double table
__global__ void k_pair_epilogue_f64(PairEpilogue e, long ld, double* g2out) {
    const int z = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= e.S) return;
    const int s = e.s_off + z;
    const int nw = e.nw, nm = e.nm;
    const long iq = grid_q(e.kc, s, t, e.n1, e.n2, e.n3);
    const double* gp = reinterpret_cast<const double*>(e.gw) + ((long)z * e.S + t) * nm * nw * 2;
    const int bt = e.band[t];
    const double* ut = e.ut + (long)t * nw * nw * 2;
    cx<double> gh[kMaxModes];
    for (int x = 0; x < nm; ++x) {
        cx<double> a = {0, 0};
        for (int i = 0; i < nw; ++i) cjfma(a, ldc(ut, (long)i * nw + bt), ldc(gp, (long)x * nw + i));
        gh[x] = a;
    }
    if (e.lr != nullptr) {
        const double* us = e.us + (long)s * nw * nw * 2;
        const int bs = e.band[s];
        cx<double> ov = {0, 0};
        for (int i = 0; i < nw; ++i) cjfma(ov, ldc(ut, (long)i * nw + bt), ldc(us, (long)i * nw + bs));
        for (int x = 0; x < nm; ++x) cfma(gh[x], ldc(e.lr, iq * nm + x), ov);
    }
    for (int nu = 0; nu < nm; ++nu) {
        const double om = e.omega[iq * nm + nu];
        double g2 = 0.0;
        if (om > e.omega_cut) {
            cx<double> g = {0, 0};
            for (int x = 0; x < nm; ++x) {
                cx<double> ev = ldc(e.evec, (iq * nm + x) * nm + nu);
                ev.x *= e.minv[x];
                ev.y *= e.minv[x];
                cfma(g, ev, gh[x]);
            }
            const double amp = sqrt(kHbar2AmuA2 / (2.0 * om));
            g2 = amp * amp * (g.x * g.x + g.y * g.y);
        }
        g2out[((long)nu * e.S + s) * ld + t] = g2;
    }
}

// G <- (G + G^T)/2 per mode, in place, 32x32 tiles with i <= j
template <typename T>
__global__ void k_symmetrise(int S, long ld, T* g) {
    __shared__ T a[32][33], b[32][33];
    const int nu = blockIdx.z;
    const int bi = blockIdx.y, bj = blockIdx.x;
    if (bi > bj) return;
    T* gn = g + (long)nu * S * ld;
    const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int i = bi * 32 + r, j = bj * 32 + tx;
        a[r][tx] = (i < S && j < S) ? gn[(long)i * ld + j] : (T)0;
        const int i2 = bj * 32 + r, j2 = bi * 32 + tx;
        b[r][tx] = (i2 < S && j2 < S) ? gn[(long)i2 * ld + j2] : (T)0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int i = bi * 32 + r, j = bj * 32 + tx;
        if (i < S && j < S) gn[(long)i * ld + j] = (T)0.5 * (a[r][tx] + b[tx][r]);
        const int i2 = bj * 32 + r, j2 = bi * 32 + tx;
        if (i2 < S && j2 < S) gn[(long)i2 * ld + j2] = (T)0.5 * (b[r][tx] + a[tx][r]);
    }
}

// P[s][t] = sum_nu scale_nu G[nu][s][t] w_nu(s,t) with
//   collision:  w = delta(D - hw)(N+1) + delta(D + hw) N
//   transport:  w = (2 pi/hbar)[delta(D - hw)(1 + N - f0_t) + delta(D + hw)(N + f0_t)]
// Pairs with |D| > dcut (> 0: at least the largest phonon energy + 6 sigma, so
// both delta arguments of every mode lie beyond the cut) are written as the
// exact zero the sum gives, without evaluating it.
template <typename T, bool TRANSPORT>
__global__ void k_build_matrix(int S, int nm, long ld, const T* __restrict__ g2, const int32_t* __restrict__ kc,
                               int n1, int n2, int n3, const double* __restrict__ omega,
                               const double* __restrict__ eps, double temp, double mu, double sigma,
                               double omega_cut, const double* __restrict__ scale,
                               const int32_t* __restrict__ perm, T* __restrict__ out, double dcut) {
    // 1-D grid of 256-column chunks, rows padded to a multiple of 8.  Blocks are
    // dealt to the 8 XCDs in turn, so every chunk of row i lands on XCD i % 8
    // and the gathered reads of G[.][perm[i]][.] share that XCD's L2.
    const int nch = (S + 255) / 256;
    const long b = blockIdx.x;
    const long local = b >> 3;
    const int i = (int)(local / nch) * 8 + (int)(b & 7);
    const int j = (int)(local % nch) * 256 + threadIdx.x;
    if (i >= S || j >= S) return;
    const int s = perm ? perm[i] : i, t = perm ? perm[j] : j;
    const long iq = grid_q(kc, s, t, n1, n2, n3);
    const double d = eps[s] - eps[t];
    if (dcut > 0.0 && fabs(d) > dcut) {
        out[(long)i * ld + j] = (T)0;
        return;
    }
    const double kt = kBoltzEv * temp;
    const double is = 1.0 / sigma, nrm = 1.0 / (sqrt(kPi) * sigma);
    double f0t = 0.0;
    if (TRANSPORT) f0t = 1.0 / (exp((eps[t] - mu) / kt) + 1.0);
    double acc = 0.0;
    for (int nu = 0; nu < nm; ++nu) {
        const double om = omega[iq * nm + nu];
        if (!(om > omega_cut)) continue;
        const double nb = 1.0 / expm1(om / kt);
        const double x1 = (d - om) * is, x2 = (d + om) * is;
        const double de = x1 * x1 > kDeltaCut2 ? 0.0 : nrm * exp(-x1 * x1);
        const double da = x2 * x2 > kDeltaCut2 ? 0.0 : nrm * exp(-x2 * x2);
        const double w = TRANSPORT ? (de * (1.0 + nb - f0t) + da * (nb + f0t)) : (de * (nb + 1.0) + da * nb);
        acc += scale[nu] * (double)g2[((long)nu * S + s) * ld + t] * w;
    }
    out[(long)i * ld + j] = (T)(TRANSPORT ? acc * (2.0 * kPi / kHbarEvFs) : acc);
}

// ---------------------------------------------------------------- streaming pass
// A block owns a column tile of kTC columns (kCPL per lane) and a run of rpb
// rows; its four waves take the rows of the run in turn.  rpb is chosen on the
// host so that the whole grid is resident at once (one wave of blocks): a
// second, partly filled wave of blocks would leave HBM idle at the end.
constexpr int kTC = kStreamTileCols; // columns per tile
constexpr int kCPL = kTC / 64;    // columns per lane (16)

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
    typedef float4 type;
};
template <>
struct Vec4<double> {
    typedef double4 type;
};

// Nontemporal loads: the matrix is streamed once per pass and is far larger
// than the caches, so its lines should not evict the reused vectors x, y.
__device__ __forceinline__ float4 ld_stream(const float* p) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 t = __builtin_nontemporal_load(reinterpret_cast<const v4*>(p));
    return make_float4(t.x, t.y, t.z, t.w);
}
__device__ __forceinline__ double4 ld_stream(const double* p) {
    typedef double v2 __attribute__((ext_vector_type(2)));
    const v2 a = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    const v2 b = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p + 2));
    return make_double4(a.x, a.y, b.x, b.y);
}

template <typename T>
__device__ __forceinline__ void load_row(const T* __restrict__ P, long ld, int r, bool ok, int c0, int lane,
                                         typename Vec4<T>::type (&v)[4]) {
    const T* row = P + (long)r * ld + c0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int c = 4 * (lane + 64 * j);
        if (ok && c0 + c < ld) {
            v[j] = ld_stream(row + c);
        } else {
            v[j].x = v[j].y = v[j].z = v[j].w = (T)0;
        }
    }
}

// one row of the tile: NA row sums (reduced over the wavefront) and NB column
// accumulations, all in FP64
template <typename T, int NA, int NB>
__device__ __forceinline__ void stream_row(int S, int r, int lane, int ct, int n_ct,
                                           const typename Vec4<T>::type (&v)[4], const double (&xv)[NA > 0 ? NA : 1][kCPL],
                                           double (&cacc)[NB > 0 ? NB : 1][kCPL], const VecPtrs& yb,
                                           double* __restrict__ rowp) {
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        double sa = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            sa = fma((double)v[j].x, xv[a][4 * j], sa);
            sa = fma((double)v[j].y, xv[a][4 * j + 1], sa);
            sa = fma((double)v[j].z, xv[a][4 * j + 2], sa);
            sa = fma((double)v[j].w, xv[a][4 * j + 3], sa);
        }
        for (int w = 32; w >= 1; w >>= 1) sa += __shfl_xor(sa, w, 64);
        if (lane == 0) rowp[((long)a * n_ct + ct) * S + r] = sa;
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const double yr = yb.p[b][r];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            cacc[b][4 * j] = fma((double)v[j].x, yr, cacc[b][4 * j]);
            cacc[b][4 * j + 1] = fma((double)v[j].y, yr, cacc[b][4 * j + 1]);
            cacc[b][4 * j + 2] = fma((double)v[j].z, yr, cacc[b][4 * j + 2]);
            cacc[b][4 * j + 3] = fma((double)v[j].w, yr, cacc[b][4 * j + 3]);
        }
    }
}

// Two register sets X, Y alternate: while one row is reduced the other's loads
// are in flight, and no register copy has to wait on an outstanding load.
// Everything here is in matrix order (vectors gathered beforehand).  Block b
// takes tile tiles[b]; blocks from n_live on hold tiles of exact zeros and only
// write zero partials.
template <typename T, int NA, int NB>
__global__ __launch_bounds__(256) void k_stream(int S, long ld, const T* __restrict__ P, VecPtrs xa, VecPtrs yb,
                                                double* __restrict__ rowp, double* __restrict__ colp, int n_ct,
                                                int n_rt, int rpb, const int32_t* __restrict__ tiles, int n_live) {
    __shared__ double cred[NB > 0 ? NB : 1][kTC];
    const int ct = tiles[2 * blockIdx.x], rt = tiles[2 * blockIdx.x + 1];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int c0 = ct * kTC;
    const int r_beg = rt * rpb;
    const int r_end = min(S, r_beg + rpb);
    if ((int)blockIdx.x >= n_live) {
        for (int r = r_beg + tid; r < r_end; r += 256)
#pragma unroll
            for (int a = 0; a < NA; ++a) rowp[((long)a * n_ct + ct) * S + r] = 0.0;
        for (int c = tid; c < kTC; c += 256)
            if (c0 + c < S)
#pragma unroll
                for (int b = 0; b < NB; ++b) colp[((long)b * n_rt + rt) * S + c0 + c] = 0.0;
        return;
    }
    // lane columns: c0 + 4*(lane + 64*j) + u, j = 0..3, u = 0..3
    double xv[NA > 0 ? NA : 1][kCPL];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = c0 + 4 * (lane + 64 * j) + u;
                xv[a][4 * j + u] = c < S ? xa.p[a][c] : 0.0;
            }
    double cacc[NB > 0 ? NB : 1][kCPL];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < kCPL; ++i) cacc[b][i] = 0.0;
    int r = r_beg + wave;
    typename Vec4<T>::type X[4], Y[4];
    load_row(P, ld, r, r < r_end, c0, lane, X);
    load_row(P, ld, r + 4, r + 4 < r_end, c0, lane, Y);
    for (; r < r_end; r += 8) {
        stream_row<T, NA, NB>(S, r, lane, ct, n_ct, X, xv, cacc, yb, rowp);
        load_row(P, ld, r + 8, r + 8 < r_end, c0, lane, X);
        if (r + 4 < r_end) stream_row<T, NA, NB>(S, r + 4, lane, ct, n_ct, Y, xv, cacc, yb, rowp);
        load_row(P, ld, r + 12, r + 12 < r_end, c0, lane, Y);
    }
    if (NB > 0) {
        // combine the four waves' column sums in a fixed order
        for (int w = 0; w < 4; ++w) {
            if (wave == w) {
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int c = 4 * (lane + 64 * j) + u;
                            cred[b][c] = (w == 0 ? 0.0 : cred[b][c]) + cacc[b][4 * j + u];
                        }
            }
            __syncthreads();
        }
        for (int b = 0; b < NB; ++b)
            for (int c = tid; c < kTC; c += 256)
                if (c0 + c < S) colp[((long)b * n_rt + rt) * S + c0 + c] = cred[b][c];
    }
}

// f_bar_u = -c [ lam_u (R0_u + C0_u) - C1_u - R1_u ]
__global__ void k_vjp_finish(int S, int n_ct, int n_rt, const double* __restrict__ rowp,
                             const double* __restrict__ colp, const double* __restrict__ lam, double c,
                             double* __restrict__ fbar) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= S) return;
    double r0 = 0.0, r1 = 0.0, c0 = 0.0, c1 = 0.0;
    for (int ct = 0; ct < n_ct; ++ct) {
        r0 += rowp[(long)ct * S + u];
        r1 += rowp[((long)n_ct + ct) * S + u];
    }
    for (int rt = 0; rt < n_rt; ++rt) {
        c0 += colp[(long)rt * S + u];
        c1 += colp[((long)n_rt + rt) * S + u];
    }
    fbar[u] = -c * (lam[u] * (r0 + c0) - c1 - r1);
}

// s_bar_nu = (acc ? s_bar_nu : 0) - c sum_j sum_s f_js (lam_js R1_js - R2_js)
// over ns pairs (f_j, lam_j), with R1_j = P^nu (1 - f_j), R2_j = P^nu (lam_j (1 - f_j))
// (state order; r[2 (nu ns + j)] and the next row), P^nu the collision matrix
// of mode nu alone at unit scale: the derivative of sum_j lam_j^T I[f_j] with
// respect to the mode scale s_nu.  One block per mode; fixed summation order.
__global__ void k_mode_finish(int S, int ns, const double* __restrict__ r, VecPtrs f, VecPtrs lam, double c,
                              double* __restrict__ sbar, int accumulate) {
    __shared__ double red[256];
    const int nu = blockIdx.x;
    double* out = sbar + nu;
    double acc = 0.0;
    for (int j = 0; j < ns; ++j) {
        const double* r1 = r + (long)2 * (nu * ns + j) * S;
        const double* r2 = r1 + S;
        const double* fj = f.p[j];
        const double* lj = lam.p[j];
        for (int s = threadIdx.x; s < S; s += 256) acc += fj[s] * (lj[s] * r1[s] - r2[s]);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (accumulate ? *out : 0.0) - c * red[0];
}

// ITA update: F[s][a] = F0[s][a] + tau_s/N_q * sum_ct rowp[a][ct][s]; also gamma from a ones pass
__global__ void k_ita_gamma(int S, int n_ct, const double* __restrict__ rowp, double n_q, const double* __restrict__ vel,
                            double* __restrict__ tau, double* __restrict__ f0, double* __restrict__ f) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    double g = 0.0;
    for (int ct = 0; ct < n_ct; ++ct) g += rowp[(long)ct * S + s];
    const double ts = n_q / g;
    tau[s] = ts;
    for (int a = 0; a < 3; ++a) {
        f0[(long)a * S + s] = ts * vel[3 * s + a];
        f[(long)a * S + s] = ts * vel[3 * s + a];
    }
}

// With chg != nullptr, also max_{s,a} |F_new - F_prev| and max_{s,a} |F_new|
// into chg[0], chg[1] (bit patterns of non-negative doubles, which atomicMax
// orders like the values; cleared by the caller).
__global__ void k_ita_update(int S, int n_ct, const double* __restrict__ rowp, double n_q, const double* __restrict__ tau,
                             const double* __restrict__ f0, double* __restrict__ f, const double* __restrict__ fprev,
                             unsigned long long* __restrict__ chg) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    double dmax = 0.0, amax = 0.0;
    if (s < S) {
        for (int a = 0; a < 3; ++a) {
            double r = 0.0;
            for (int ct = 0; ct < n_ct; ++ct) r += rowp[((long)a * n_ct + ct) * S + s];
            const double v = f0[(long)a * S + s] + tau[s] / n_q * r;
            f[(long)a * S + s] = v;
            if (chg) {
                dmax = fmax(dmax, fabs(v - fprev[(long)a * S + s]));
                amax = fmax(amax, fabs(v));
            }
        }
    }
    if (!chg) return;
    __shared__ double red[2][256];
    red[0][threadIdx.x] = dmax;
    red[1][threadIdx.x] = amax;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + w]);
            red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&chg[0], (unsigned long long)__double_as_longlong(red[0][0]));
        atomicMax(&chg[1], (unsigned long long)__double_as_longlong(red[1][0]));
    }
}

// mu_ab = 0.1 sum_s v^a F^b f0(1-f0)/(kT) / sum_s f0, one block; also F out as [S][3]
__global__ void k_mobility(int S, const double* __restrict__ eps, const double* __restrict__ vel,
                           const double* __restrict__ f, double mu, double temp, double* __restrict__ fout,
                           double* __restrict__ mob) {
    __shared__ double red[10][256];
    const double kt = kBoltzEv * temp;
    double acc[10];
    for (int i = 0; i < 10; ++i) acc[i] = 0.0;
    for (int s = threadIdx.x; s < S; s += 256) {
        const double f0 = 1.0 / (exp((eps[s] - mu) / kt) + 1.0);
        const double w = f0 * (1.0 - f0) / kt;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) acc[3 * a + b] += vel[3 * s + a] * f[(long)b * S + s] * w;
        acc[9] += f0;
        if (fout)
            for (int b = 0; b < 3; ++b) fout[3 * s + b] = f[(long)b * S + s];
    }
    for (int i = 0; i < 10; ++i) red[i][threadIdx.x] = acc[i];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int i = 0; i < 10; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 9 && mob) mob[threadIdx.x] = 0.1 * red[threadIdx.x][0] / red[9][0];
}

// ---------------------------------------------------------------- mobility adjoint
// Reverse of the iteration (Eqs. BTE_iter, cond) for L = sum_ab lam_ab mu_ab, with
//   F^{i+1} = tau (v + (1/N_q) W F^i),  F^0 = tau v,  tau_s = N_q / sum_t W_st.
// F and its adjoint are stored [3][S].

// F_bar_b(s) = 0.1 sum_a lam_ab v^a_s f0_s (1 - f0_s)/kT / sum_t f0_t  (one block)
__global__ void k_mob_seed(int S, const double* __restrict__ eps, const double* __restrict__ vel,
                           const double* __restrict__ lam, double mu, double temp, double* __restrict__ fbar) {
    __shared__ double red[256];
    const double kt = kBoltzEv * temp;
    double a = 0.0;
    for (int s = threadIdx.x; s < S; s += 256) a += 1.0 / (exp((eps[s] - mu) / kt) + 1.0);
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double tot = red[0];
    for (int s = threadIdx.x; s < S; s += 256) {
        const double f0 = 1.0 / (exp((eps[s] - mu) / kt) + 1.0);
        const double w = 0.1 * f0 * (1.0 - f0) / kt / tot;
        for (int b = 0; b < 3; ++b) {
            double c = 0.0;
            for (int a2 = 0; a2 < 3; ++a2) c += lam[3 * a2 + b] * vel[3 * s + a2];
            fbar[(long)b * S + s] = w * c;
        }
    }
}

// step i (F^{i+1} = tau u^i): tau_bar += sum_b Fbar^{i+1}_b F^{i+1}_b / tau ; ubar^i = tau Fbar^{i+1}
__global__ void k_ita_adj_step(int S, const double* __restrict__ tau, const double* __restrict__ fbar,
                               const double* __restrict__ fnext, double* __restrict__ taubar,
                               double* __restrict__ ubar, int first) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    double tb = first ? 0.0 : taubar[s];
    for (int b = 0; b < 3; ++b) {
        const long o = (long)b * S + s;
        tb += fbar[o] * fnext[o] / tau[s];
        ubar[o] = tau[s] * fbar[o];
    }
    taubar[s] = tb;
}

// Fbar^i_t = (1/N_q) sum_s W_st ubar^i_s from the column partials of one pass
__global__ void k_ita_adj_cols(int S, int n_rt, const double* __restrict__ colp, double n_q, double* __restrict__ fbar) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S) return;
    for (int b = 0; b < 3; ++b) {
        double c = 0.0;
        for (int rt = 0; rt < n_rt; ++rt) c += colp[((long)b * n_rt + rt) * S + t];
        fbar[(long)b * S + t] = c / n_q;
    }
}

// F^0 = tau v: tau_bar += sum_b Fbar^0_b v_b ; Gamma_bar = -tau^2 tau_bar, so that
// W_bar_st gets Gamma_bar_s / N_q from the row sum
__global__ void k_ita_adj_final(int S, const double* __restrict__ tau, const double* __restrict__ fbar0,
                                const double* __restrict__ vel, const double* __restrict__ taubar, int first,
                                double* __restrict__ gbar) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    double tb = first ? 0.0 : taubar[s];
    for (int b = 0; b < 3; ++b) tb += fbar0[(long)b * S + s] * vel[3 * s + b];
    gbar[s] = -tau[s] * tau[s] * tb;
}

// transport weight of one mode for the transition s -> t (Delta = e_s - e_t),
// the same expression as the transport matrix uses
__device__ __forceinline__ double transport_weight(double d, double om, double f0t, double kt, double is, double nrm,
                                                   double omega_cut) {
    if (!(om > omega_cut)) return 0.0;
    const double nb = 1.0 / expm1(om / kt);
    const double x1 = (d - om) * is, x2 = (d + om) * is;
    const double de = x1 * x1 > kDeltaCut2 ? 0.0 : nrm * exp(-x1 * x1);
    const double da = x2 * x2 > kDeltaCut2 ? 0.0 : nrm * exp(-x2 * x2);
    return de * (1.0 + nb - f0t) + da * (nb + f0t);
}

// One thread per (source s in chunk, target t).  W_bar_st = (1/N_q)(sum_h ubar_h(s) F_h(t)
// + Gamma_bar_s); dL/d|g_nu(s->t)|^2 = 1/2 (2 pi/hbar)(w_nu(s,t) W_bar_st + w_nu(t,s) W_bar_ts)
// (the table holds the symmetrised G); g_nu(s->t) is recomputed from the FP64
// Rp contraction exactly as the table epilogue forms it, and the adjoint of
// |g|^2 -> mode projection -> band rotation gives the Rp-contraction adjoint
// g'W_bar[x][i] = U(k_t)[i][n_t] sum_nu amp minv_x conj(e_x,nu) 2 c_nu g_nu.
__global__ void k_pair_adjoint(PairAdjoint e) {
    const int z = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= e.S) return;
    const int s = e.s_off + z;
    const int S = e.S, nw = e.nw, nm = e.nm;
    double wst = e.gamma_bar[s], wts = e.gamma_bar[t];
    for (int h = 0; h < e.n_hist; ++h) {
        wst = fma(e.ubar[(long)h * S + s], e.fhist[(long)h * S + t], wst);
        wts = fma(e.ubar[(long)h * S + t], e.fhist[(long)h * S + s], wts);
    }
    wst /= e.n_q;
    wts /= e.n_q;
    const long iq = grid_q(e.kc, s, t, e.n1, e.n2, e.n3);
    const long iqr = grid_q(e.kc, t, s, e.n1, e.n2, e.n3);
    const double kt = kBoltzEv * e.temp;
    const double is = 1.0 / e.sigma, nrm = 1.0 / (sqrt(kPi) * e.sigma);
    const double f0s = 1.0 / (exp((e.eps[s] - e.mu) / kt) + 1.0);
    const double f0t = 1.0 / (exp((e.eps[t] - e.mu) / kt) + 1.0);
    const double d = e.eps[s] - e.eps[t];
    const double* gp = e.gw + ((long)z * S + t) * nm * nw * 2;
    const int bt = e.band[t];
    const double* ut = e.ut + (long)t * nw * nw * 2;
    cx<double> gh[kMaxModes], gb[kMaxModes];
    for (int x = 0; x < nm; ++x) {
        cx<double> a = {0, 0};
        for (int i = 0; i < nw; ++i) cjfma(a, ldc(ut, (long)i * nw + bt), ldc(gp, (long)x * nw + i));
        gh[x] = a;
        gb[x] = {0, 0};
    }
    if (e.lr != nullptr) {
        const double* us = e.us + (long)s * nw * nw * 2;
        const int bs = e.band[s];
        cx<double> ov = {0, 0};
        for (int i = 0; i < nw; ++i) cjfma(ov, ldc(ut, (long)i * nw + bt), ldc(us, (long)i * nw + bs));
        for (int x = 0; x < nm; ++x) cfma(gh[x], ldc(e.lr, iq * nm + x), ov);
    }
    const double pref = 0.5 * (2.0 * kPi / kHbarEvFs);
    for (int nu = 0; nu < nm; ++nu) {
        const double om = e.omega[iq * nm + nu];
        if (!(om > e.omega_cut_table)) continue;
        const double c = pref * (transport_weight(d, om, f0t, kt, is, nrm, e.omega_cut) * wst +
                                 transport_weight(-d, e.omega[iqr * nm + nu], f0s, kt, is, nrm, e.omega_cut) * wts);
        const double amp = sqrt(kHbar2AmuA2 / (2.0 * om));
        cx<double> g = {0, 0};
        for (int x = 0; x < nm; ++x) {
            cx<double> ev = ldc(e.evec, (iq * nm + x) * nm + nu);
            ev.x *= e.minv[x];
            ev.y *= e.minv[x];
            cfma(g, ev, gh[x]);
        }
        // gbar_nu = 2 c g_nu (amp folded in twice: once in g, once in the adjoint)
        const double sc = 2.0 * c * amp * amp;
        const cx<double> gbn = {sc * g.x, sc * g.y};
        for (int x = 0; x < nm; ++x) {
            cx<double> ev = ldc(e.evec, (iq * nm + x) * nm + nu);
            ev.x *= e.minv[x];
            ev.y *= e.minv[x];
            cjfma(gb[x], ev, gbn);
        }
    }
    double* out = e.gw_bar + ((long)z * S + t) * nm * nw * 2;
    for (int x = 0; x < nm; ++x)
        for (int i = 0; i < nw; ++i) {
            const cx<double> u = ldc(ut, (long)i * nw + bt);
            out[2 * ((long)x * nw + i)] = u.x * gb[x].x - u.y * gb[x].y;
            out[2 * ((long)x * nw + i) + 1] = u.x * gb[x].y + u.y * gb[x].x;
        }
}

// Adjoint of g'(s)[p][x][i] = sum_j g(s)[p][x][i][j] U(k_s)[j][n_s], with the
// phase exp(2 pi i k_s . Rp_p) that turns a sum over exp(-2 pi i k_t . Rp) into
// one over exp(-2 pi i (k_t - k_s) . Rp):
//   out[z][p][x][i][j] = exp(2 pi i k_s . Rp_p) in[z][p][x][i] conj(U(k_s)[j][n_s])
__global__ void k_apply_u_column_adj(int nrp, int nm, int nw, int s_off, const double* __restrict__ in,
                                     const double* __restrict__ ks, const int32_t* __restrict__ rp,
                                     const double* __restrict__ us, const int32_t* __restrict__ band,
                                     double* __restrict__ out) {
    const int z = blockIdx.y;
    const int s = s_off + z;
    const long per = (long)nrp * nm * nw * nw;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per) return;
    const int j = (int)(idx % nw);
    const long pxi = idx / nw;
    const int p = (int)(pxi / ((long)nm * nw));
    double arg = ks[3 * s] * rp[3 * p] + ks[3 * s + 1] * rp[3 * p + 1] + ks[3 * s + 2] * rp[3 * p + 2];
    arg -= rint(arg);
    double sn, cs;
    sincospi(2.0 * arg, &sn, &cs);
    const cx<double> a = ldc(in, (long)z * nrp * nm * nw + pxi);
    const cx<double> u = ldc(us, ((long)s * nw + j) * nw + band[s]);
    // (cs + i sn) a conj(u)
    const double ar = cs * a.x - sn * a.y, ai = cs * a.y + sn * a.x;
    out[2 * ((long)z * per + idx)] = ar * u.x + ai * u.y;
    out[2 * ((long)z * per + idx) + 1] = ai * u.x - ar * u.y;
}

__global__ void k_axpy_copy(int S, const double* __restrict__ x, double a, const double* __restrict__ y,
                            double* __restrict__ out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < S) out[s] = x[s] + a * (y ? y[s] : 0.0);
}

// out = sum_i c_i v_i (v_i may be the same array as out); terms with null v are skipped
__global__ void k_lincomb(int S, Lincomb lc, double* __restrict__ out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    double acc = lc.c0;
    for (int i = 0; i < lc.n; ++i) acc += lc.c[i] * lc.v[i][s];
    out[s] = acc;
}

// out0 = 1 - f, out1 = lam (1 - f), out2 = lam f (out1/out2 skipped when lam is null)
__global__ void k_occ_vectors(int S, const double* __restrict__ f, const double* __restrict__ lam, double* __restrict__ o0,
                              double* __restrict__ o1, double* __restrict__ o2) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const double fs = f[s];
    o0[s] = 1.0 - fs;
    if (lam) {
        o1[s] = lam[s] * (1.0 - fs);
        o2[s] = lam[s] * fs;
    }
}

__global__ void k_fill(long n, double v, double* out) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

// ---------------------------------------------------------------- mode-scale gradient over a panel of stages
// For J stages (f_j, lam_j), the mode-scale gradient of the collision integral
// summed over the stages is
//   s_bar_nu = -c sum_j sum_st P^nu_st f_js (1 - f_jt)(lam_js - lam_jt)
//            = -c sum_st P^nu_st M_st,   M = A B^T - C D^T,
// with the rows a_j = f_j lam_j, c_j = f_j and the columns b_j = 1 - f_j,
// d_j = lam_j (1 - f_j) (matrix order).  One pass forms M tile by tile (a
// rank-2J product in FP64 registers) and reads every per-mode matrix once,
// instead of one pass over each P^nu per stage.

// A, B, C, D [J][S] in matrix order from f, lam [J][S] in state order
__global__ void k_panel_gather(int S, int J, const int32_t* __restrict__ perm, const double* __restrict__ f,
                               const double* __restrict__ lam, double* __restrict__ A, double* __restrict__ B,
                               double* __restrict__ C, double* __restrict__ D) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)J * S) return;
    const long j = t / S;
    const int i = (int)(t % S);
    const long src = j * S + perm[i];
    const double fv = f[src], lv = lam[src];
    A[t] = fv * lv;
    B[t] = 1.0 - fv;
    C[t] = fv;
    D[t] = lv * (1.0 - fv);
}

constexpr int kPT = 128;   // panel tile: kPT x kPT entries per 256-thread workgroup
constexpr int kPJ = 16;    // stages staged in LDS at a time (a multiple of 4)

// One live tile per workgroup, M formed on the FP64 matrix cores: the K
// dimension is the stage index, M = A B^T - C D^T as two 16 x 16 x 4 products
// per block and four stages.  Wave w owns rows 64 (w / 2) + [0, 64) and
// columns 64 (w % 2) + [0, 64) of the tile: 4 x 4 blocks of 16 x 16.  Operand
// layout of v_mfma_f64_16x16x4f64: lane l gives A[l % 16][l / 16] and
// B[l / 16][l % 16]; it holds D[l / 16 + 4 v][l % 16], v = 0..3.
// partial[tile][nu] = sum over the tile of P^nu_rc M_rc.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
__global__ __launch_bounds__(256) void k_mode_panel(int S, long ld, int J, int nm, const T* __restrict__ pm,
                                                    long mat, const double* __restrict__ A,
                                                    const double* __restrict__ B, const double* __restrict__ C,
                                                    const double* __restrict__ D, const int32_t* __restrict__ tiles,
                                                    double* __restrict__ partial) {
    // the staged vectors [a, -c, b, d][stage][entry] while M is formed, then
    // M itself [row][column] (FP64) for the contraction with the per-mode
    // matrices, read in rows of 16-byte loads
    __shared__ __attribute__((aligned(16))) double ms[kPT * kPT];
    __shared__ double red[kMaxModes][256];
    static_assert(4 * kPJ * kPT <= kPT * kPT, "staging space");
    double* stg = ms;
    const int tile = blockIdx.x;
    const int r0 = tiles[2 * tile] * kPT, c0 = tiles[2 * tile + 1] * kPT;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int wr = 64 * (w >> 1), wc = 64 * (w & 1);
    const int li = l & 15, lk = l >> 4;
    f64x4 m[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) m[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    // each chunk of kPJ stages goes global -> registers -> LDS; the next
    // chunk's loads are issued before the current chunk's products
    constexpr int kPer = kPJ * kPT / 256;
    double q[4][kPer];
    auto load = [&](int j0) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int x = tid + 256 * u;
            const int j = j0 + x / kPT, e = x % kPT;
            const bool jr = j < J;
            const int r = r0 + e, c = c0 + e;
            q[0][u] = jr && r < S ? A[(long)j * S + r] : 0.0;
            q[1][u] = jr && r < S ? -C[(long)j * S + r] : 0.0;
            q[2][u] = jr && c < S ? B[(long)j * S + c] : 0.0;
            q[3][u] = jr && c < S ? D[(long)j * S + c] : 0.0;
        }
    };
    auto at = [&](int v, int jj, int e) -> double& { return stg[(v * kPJ + jj) * kPT + e]; };
    load(0);
    for (int j0 = 0; j0 < J; j0 += kPJ) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int x = tid + 256 * u;
#pragma unroll
            for (int v = 0; v < 4; ++v) at(v, x / kPT, x % kPT) = q[v][u];
        }
        __syncthreads();
        if (j0 + kPJ < J) load(j0 + kPJ);
#pragma unroll
        for (int k4 = 0; k4 < kPJ; k4 += 4) {
            double oa[4], oc[4], ob[4], od[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                oa[a] = at(0, k4 + lk, wr + 16 * a + li);
                oc[a] = at(1, k4 + lk, wr + 16 * a + li);
                ob[a] = at(2, k4 + lk, wc + 16 * a + li);
                od[a] = at(3, k4 + lk, wc + 16 * a + li);
            }
            // the two updates of a block are 16 instructions apart
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) m[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(oa[a], ob[b], m[a][b], 0, 0, 0);
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) m[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(oc[a], od[b], m[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    // M into LDS, [row][column]
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int b = 0; b < 4; ++b) ms[(wr + 16 * a + lk + 4 * v) * kPT + wc + 16 * b + li] = m[a][b][v];
    __syncthreads();
    // sum P^nu_rc M_rc: thread t takes 4 consecutive columns 4 (t % 32) of the
    // rows t / 32 + 8 i; a row of the tile is 32 lanes x 16 bytes (FP32)
    double acc[kMaxModes];
#pragma unroll
    for (int nu = 0; nu < kMaxModes; ++nu) acc[nu] = 0.0;
    const int cg = 4 * (tid & 31);
    if (c0 + cg < S) {
#pragma unroll 4
        for (int i = 0; i < kPT / 8; ++i) {
            const int rl = (tid >> 5) + 8 * i;
            const int r = r0 + rl;
            if (r >= S) break;
            const double* mr = ms + rl * kPT + cg;
            const double x0 = mr[0], x1 = mr[1], x2 = mr[2], x3 = mr[3];
            const T* p = pm + (long)r * ld + c0 + cg;
#pragma unroll
            for (int nu = 0; nu < kMaxModes; ++nu)
                if (nu < nm) {
                    const T* pn = p + (long)nu * mat;
                    if constexpr (sizeof(T) == 4) {
                        const float4 v = *reinterpret_cast<const float4*>(pn);
                        acc[nu] = fma((double)v.x, x0, fma((double)v.y, x1, fma((double)v.z, x2, fma((double)v.w, x3, acc[nu]))));
                    } else {
                        const double2 v0 = reinterpret_cast<const double2*>(pn)[0];
                        const double2 v1 = reinterpret_cast<const double2*>(pn)[1];
                        acc[nu] = fma(v0.x, x0, fma(v0.y, x1, fma(v1.x, x2, fma(v1.y, x3, acc[nu]))));
                    }
                }
        }
    }
#pragma unroll
    for (int nu = 0; nu < kMaxModes; ++nu)
        if (nu < nm) red[nu][tid] = acc[nu];
    __syncthreads();
    for (int x = 128; x >= 1; x >>= 1) {
        if (tid < x)
            for (int nu = 0; nu < nm; ++nu) red[nu][tid] += red[nu][tid + x];
        __syncthreads();
    }
    if (tid < nm) partial[(long)tile * nm + tid] = red[tid][0];
}

// s_bar[nu] (=/+=) -c sum over tiles of partial[tile][nu], in tile order
__global__ void k_mode_panel_finish(int n_tiles, int nm, const double* __restrict__ partial, double c,
                                    double* __restrict__ sbar, int accumulate) {
    __shared__ double red[256];
    const int nu = blockIdx.x;
    double a = 0.0;
    for (int t = threadIdx.x; t < n_tiles; t += 256) a += partial[(long)t * nm + nu];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sbar[nu] = (accumulate ? sbar[nu] : 0.0) - c * red[0];
}

}  // namespace

long table_ld(int S) { return ((long)S + 63) / 64 * 64; }

void pair_epilogue(const PairEpilogue& e, int f32, long ld, void* g2out, hipStream_t st) {
    dim3 grid((e.S + 127) / 128, e.ns_chunk);
    if (f32) {
        PairEpilogue ee = e;
        ee.g2raw = (float*)g2out;
        hipLaunchKernelGGL(k_pair_epilogue_f32, grid, dim3(128), 0, st, ee, ld);
    } else {
        hipLaunchKernelGGL(k_pair_epilogue_f64, grid, dim3(128), 0, st, e, ld, (double*)g2out);
    }
    check_launch("pair_epilogue");
}

void table_symmetrise(int nm, int S, long ld, void* g2, int f32, hipStream_t st) {
    const int nb = (S + 31) / 32;
    dim3 grid(nb, nb, nm);
    if (f32)
        hipLaunchKernelGGL(k_symmetrise<float>, grid, dim3(32, 8), 0, st, S, ld, (float*)g2);
    else
        hipLaunchKernelGGL(k_symmetrise<double>, grid, dim3(32, 8), 0, st, S, ld, (double*)g2);
    check_launch("table_symmetrise");
}

void build_matrix(int transport, int S, int nm, long ld, const void* g2, int f32, const int32_t* kc, int n1, int n2,
                  int n3, const double* omega, const double* eps, double temp, double mu, double sigma,
                  double omega_cut, const double* scale, const int32_t* perm, void* out, double dcut,
                  hipStream_t st) {
    if (S <= 0) return;
    dim3 grid((unsigned)((long)(S + 255) / 256 * ((S + 7) / 8 * 8)));
    if (f32) {
        if (transport)
            hipLaunchKernelGGL((k_build_matrix<float, true>), grid, dim3(256), 0, st, S, nm, ld, (const float*)g2, kc,
                               n1, n2, n3, omega, eps, temp, mu, sigma, omega_cut, scale, perm, (float*)out, dcut);
        else
            hipLaunchKernelGGL((k_build_matrix<float, false>), grid, dim3(256), 0, st, S, nm, ld, (const float*)g2, kc,
                               n1, n2, n3, omega, eps, temp, mu, sigma, omega_cut, scale, perm, (float*)out, dcut);
    } else {
        if (transport)
            hipLaunchKernelGGL((k_build_matrix<double, true>), grid, dim3(256), 0, st, S, nm, ld, (const double*)g2,
                               kc, n1, n2, n3, omega, eps, temp, mu, sigma, omega_cut, scale, perm, (double*)out, dcut);
        else
            hipLaunchKernelGGL((k_build_matrix<double, false>), grid, dim3(256), 0, st, S, nm, ld, (const double*)g2,
                               kc, n1, n2, n3, omega, eps, temp, mu, sigma, omega_cut, scale, perm, (double*)out, dcut);
    }
    check_launch("build_matrix");
}

namespace {
// blocks of one stream kernel instance resident on the current device at once
template <typename T, int NA, int NB>
int stream_slots() {
    constexpr int kMaxDev = 64;
    static std::atomic<int> cache[kMaxDev];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) throw Error{-3, "stream_plan: hipGetDevice failed"};
    const int slot = dev >= 0 && dev < kMaxDev ? dev : -1;
    int v = slot >= 0 ? cache[slot].load(std::memory_order_relaxed) : 0;
    if (v == 0) {
        int occ = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_stream<T, NA, NB>, 256, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            throw Error{-3, "stream_plan: occupancy query failed"};
        v = std::max(1, occ) * std::max(1, cus);
        if (slot >= 0) cache[slot].store(v, std::memory_order_relaxed);
    }
    return v;
}
}  // namespace

namespace {
int slot_count(int f32, int na, int nb) {
    int slots = 0;
#define EPHX_SLOTS(T)                                             \
    if (na == 1 && nb == 1) slots = stream_slots<T, 1, 1>();      \
    else if (na == 2 && nb == 2) slots = stream_slots<T, 2, 2>(); \
    else if (na == 1 && nb == 0) slots = stream_slots<T, 1, 0>(); \
    else if (na == 2 && nb == 0) slots = stream_slots<T, 2, 0>(); \
    else if (na == 4 && nb == 0) slots = stream_slots<T, 4, 0>(); \
    else if (na == 3 && nb == 0) slots = stream_slots<T, 3, 0>(); \
    else if (na == 0 && nb == 3) slots = stream_slots<T, 0, 3>(); \
    else throw Error{-1, "stream_plan: unsupported vector counts"};
    if (f32) {
        EPHX_SLOTS(float)
    } else {
        EPHX_SLOTS(double)
    }
#undef EPHX_SLOTS
    return slots;
}
}  // namespace

StreamPlan stream_plan(int S, int f32, int na, int nb) {
    StreamPlan p{};
    p.S = S;
    p.f32 = f32;
    p.na = na;
    p.nb = nb;
    if (S <= 0) return p;
    const int slots = slot_count(f32, na, nb);
    p.n_ct = (S + kTC - 1) / kTC;
    const int n_rt = std::max(1, slots / p.n_ct);
    p.rpb = ((S + n_rt - 1) / n_rt + 3) / 4 * 4;
    p.n_rt = (S + p.rpb - 1) / p.rpb;
    return p;
}

StreamPlan stream_plan_banded(int S, int f32, int na, int nb, const std::vector<double>& esort, double half_width,
                              std::vector<int32_t>& tiles, int& n_live) {
    StreamPlan p = stream_plan(S, f32, na, nb);
    tiles.clear();
    n_live = 0;
    if (S <= 0) return p;
    if ((int)esort.size() != S) throw Error{-1, "stream_plan_banded: energy list size"};
    const int slots = slot_count(f32, na, nb);
    const int n_ct = p.n_ct;
    // a tile is live unless every row energy is further than half_width from every column energy
    auto live = [&](int rpb, int rt, int ct) {
        const int r0 = rt * rpb, r1 = std::min(S, r0 + rpb);
        const int c0 = ct * kTC, c1 = std::min(S, c0 + kTC);
        const double gap = std::max(esort[c0] - esort[r1 - 1], esort[r0] - esort[c1 - 1]);
        return !(gap > half_width);
    };
    auto count = [&](int rpb) {
        const int n_rt = (S + rpb - 1) / rpb;
        int n = 0;
        for (int rt = 0; rt < n_rt; ++rt)
            for (int ct = 0; ct < n_ct; ++ct) n += live(rpb, rt, ct) ? 1 : 0;
        return n;
    };
    // smallest row tiles whose live tiles still fit one resident wave
    int best = p.rpb;
    for (int n_rt = p.n_rt + 1; n_rt <= 8 * p.n_rt; n_rt += std::max(1, p.n_rt / 16)) {
        const int rpb = ((S + n_rt - 1) / n_rt + 3) / 4 * 4;
        if (rpb < 4 || rpb >= best) continue;
        if (count(rpb) > slots) break;
        best = rpb;
    }
    p.rpb = best;
    p.n_rt = (S + best - 1) / best;
    std::vector<int32_t> dead;
    for (int rt = 0; rt < p.n_rt; ++rt)
        for (int ct = 0; ct < n_ct; ++ct) {
            std::vector<int32_t>& dst = live(best, rt, ct) ? tiles : dead;
            dst.push_back(ct);
            dst.push_back(rt);
        }
    n_live = (int)tiles.size() / 2;
    tiles.insert(tiles.end(), dead.begin(), dead.end());
    p.n_live = n_live;
    p.n_tiles = (int)tiles.size() / 2;
    return p;
}

namespace {
// out[k][i] = v_k[perm[i]] for the na + nb vectors of a pass: matrix order
__global__ void k_gather_vectors(int S, int nv, const int32_t* __restrict__ perm, VecPtrs x, VecPtrs y, int na,
                                 double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    const int s = perm[i];
    for (int k = 0; k < nv; ++k) out[(long)k * S + i] = k < na ? x.p[k][s] : y.p[k - na][s];
}

// The collision pass's vectors in matrix order straight from the occupations:
// gbuf[0][i] = 1 - f[perm[i]] (rows), gbuf[1][i] = f[perm[i]] (columns)
__global__ void k_gather_occupations(int S, const int32_t* __restrict__ perm, const double* __restrict__ f,
                                     double* __restrict__ gbuf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    const double fs = f[perm[i]];
    gbuf[i] = 1.0 - fs;
    gbuf[(long)S + i] = fs;
}

// The pass's partials reduced and the collision finished in one kernel: the
// thread of matrix index i sums the row partials (n_ct) and column partials
// (n_rt) of state s = perm[i] in fixed order, then forms
//   I_s = -c [ f_s R_s - (1 - f_s) C_s ]
// and the RK4 / Euler stage update: acc_s (=/+=) w_acc (I_s + drift_s),
// f_next_s = f_base_s + a_next (I_s + drift_s), the drift from the neighbour
// table (cf.rowp, cf.colp hold the unreduced matrix-order partials).
__global__ void k_reduce_finish(CollisionFinish cf, const int32_t* __restrict__ perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cf.S) return;
    const int s = perm[i];
    double r = 0.0, c = 0.0;
    for (int ct = 0; ct < cf.n_ct; ++ct) r += cf.rowp[(long)ct * cf.S + i];
    for (int rt = 0; rt < cf.n_rt; ++rt) c += cf.colp[(long)rt * cf.S + i];
    const double f = cf.f[s];
    const double in = -cf.c * (f * r - (1.0 - f) * c);
    if (cf.i_out) cf.i_out[s] = in;
    if (cf.acc) {
        double rhs = in;
        if (cf.nbr) {
            const int32_t* nb = cf.nbr + 6L * s;
            for (int d = 0; d < 3; ++d) {
                const int p = nb[2 * d], m = nb[2 * d + 1];
                rhs += cf.dc[d] * ((p >= 0 ? cf.f[p] : 0.0) - (m >= 0 ? cf.f[m] : 0.0));
            }
        }
        const double an = (cf.acc_init ? cf.f_base[s] : cf.acc[s]) + cf.w_acc * rhs;
        cf.acc[s] = an;
        const double fn = cf.f_next ? cf.f_base[s] + cf.a_next * rhs : 0.0;
        if (cf.f_next) cf.f_next[s] = fn;
        if (cf.gnext) {
            const double v = cf.gnext_acc ? an : fn;
            cf.gnext[i] = 1.0 - v;
            cf.gnext[(long)cf.S + i] = v;
        }
    }
}

// Reverse-RK4 stage, before the pass: lam = c0 + sum_k c_k v_k (state order,
// into lam_out) and the 2+2 pass's vectors in matrix order.
__global__ void k_adj_prep(int S, const int32_t* __restrict__ perm, Lincomb lc, const double* __restrict__ Y,
                           double* __restrict__ lam_out, double* __restrict__ gbuf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    const int s = perm[i];
    double lam = lc.c0;
    for (int k = 0; k < lc.n; ++k) lam += lc.c[k] * lc.v[k][s];
    lam_out[s] = lam;
    const double f = Y[s];
    gbuf[i] = 1.0 - f;
    gbuf[(long)S + i] = lam * (1.0 - f);
    gbuf[2L * S + i] = f;
    gbuf[3L * S + i] = lam * f;
}

// ... and after it: ybar_s = -c (lam_s (R0 + C0) - C1 - R1) from the unreduced
// partials (rows P(1-f), P(lam(1-f)); columns P^T f, P^T(lam f)); with a_acc,
// a_s += ybar_s + yb1_s + yb2_s + yb3_s.
__global__ void k_adj_finish(int S, const int32_t* __restrict__ perm, int n_ct, int n_rt,
                             const double* __restrict__ rowp, const double* __restrict__ colp,
                             const double* __restrict__ lam, double c, double* __restrict__ ybar,
                             double* __restrict__ a_acc, const double* __restrict__ yb1,
                             const double* __restrict__ yb2, const double* __restrict__ yb3) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    const int s = perm[i];
    double r0 = 0.0, r1 = 0.0, c0 = 0.0, c1 = 0.0;
    for (int ct = 0; ct < n_ct; ++ct) {
        r0 += rowp[(long)ct * S + i];
        r1 += rowp[((long)n_ct + ct) * S + i];
    }
    for (int rt = 0; rt < n_rt; ++rt) {
        c0 += colp[(long)rt * S + i];
        c1 += colp[((long)n_rt + rt) * S + i];
    }
    const double y = -c * (lam[s] * (r0 + c0) - c1 - r1);
    ybar[s] = y;
    if (a_acc) a_acc[s] = a_acc[s] + y + yb1[s] + yb2[s] + yb3[s];
}

// rout[a][perm[i]] = sum_ct rowp[a][ct][i], cout[b][perm[i]] = sum_rt colp[b][rt][i]
// (fixed order: deterministic)
__global__ void k_reduce_partials(int S, int na, int n_ct, const double* __restrict__ rowp, int nb, int n_rt,
                                  const double* __restrict__ colp, const int32_t* __restrict__ perm,
                                  double* __restrict__ rout, double* __restrict__ cout) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S) return;
    const int s = perm[i];
    for (int a = 0; a < na; ++a) {
        double acc = 0.0;
        for (int ct = 0; ct < n_ct; ++ct) acc += rowp[((long)a * n_ct + ct) * S + i];
        rout[(long)a * S + s] = acc;
    }
    for (int b = 0; b < nb; ++b) {
        double acc = 0.0;
        for (int rt = 0; rt < n_rt; ++rt) acc += colp[((long)b * n_rt + rt) * S + i];
        cout[(long)b * S + s] = acc;
    }
}
}  // namespace

void stream_gather(const StreamPlan& pl, VecPtrs x, VecPtrs y, hipStream_t st) {
    if (pl.S <= 0) return;
    if (!pl.tiles || !pl.perm || !pl.gbuf || (pl.na > 0 && !pl.rout) || (pl.nb > 0 && !pl.cout))
        throw Error{-1, "stream_gather: incomplete plan"};
    hipLaunchKernelGGL(k_gather_vectors, dim3((pl.S + 255) / 256), dim3(256), 0, st, pl.S, pl.na + pl.nb, pl.perm, x,
                       y, pl.na, pl.gbuf);
    check_launch("gather_vectors");
}

void stream_run(const StreamPlan& pl, long ld, const void* P, double* rowp, double* colp, hipStream_t st) {
    if (pl.S <= 0) return;
    VecPtrs xg{{nullptr, nullptr, nullptr, nullptr}}, yg{{nullptr, nullptr, nullptr, nullptr}};
    for (int k = 0; k < pl.na; ++k) xg.p[k] = pl.gbuf + (long)k * pl.S;
    for (int k = 0; k < pl.nb; ++k) yg.p[k] = pl.gbuf + (long)(pl.na + k) * pl.S;
    if (pl.n_tiles > 0) {
        dim3 grid(pl.n_tiles);
#define EPHX_STREAM(T, A, B)                                                                                      \
    hipLaunchKernelGGL((k_stream<T, A, B>), grid, dim3(256), 0, st, pl.S, ld, (const T*)P, xg, yg, rowp, colp, \
                       pl.n_ct, pl.n_rt, pl.rpb, pl.tiles, pl.n_live)
        const int na = pl.na, nb = pl.nb;
        if (pl.f32) {
            if (na == 1 && nb == 1) EPHX_STREAM(float, 1, 1);
            else if (na == 2 && nb == 2) EPHX_STREAM(float, 2, 2);
            else if (na == 1 && nb == 0) EPHX_STREAM(float, 1, 0);
            else if (na == 2 && nb == 0) EPHX_STREAM(float, 2, 0);
            else if (na == 4 && nb == 0) EPHX_STREAM(float, 4, 0);
            else if (na == 3 && nb == 0) EPHX_STREAM(float, 3, 0);
            else if (na == 0 && nb == 3) EPHX_STREAM(float, 0, 3);
            else throw Error{-1, "stream_pass: unsupported vector counts"};
        } else {
            if (na == 1 && nb == 1) EPHX_STREAM(double, 1, 1);
            else if (na == 2 && nb == 2) EPHX_STREAM(double, 2, 2);
            else if (na == 1 && nb == 0) EPHX_STREAM(double, 1, 0);
            else if (na == 2 && nb == 0) EPHX_STREAM(double, 2, 0);
            else if (na == 4 && nb == 0) EPHX_STREAM(double, 4, 0);
            else if (na == 3 && nb == 0) EPHX_STREAM(double, 3, 0);
            else if (na == 0 && nb == 3) EPHX_STREAM(double, 0, 3);
            else throw Error{-1, "stream_pass: unsupported vector counts"};
        }
#undef EPHX_STREAM
        check_launch("stream_pass");
    }
}

PassOut stream_reduce(const StreamPlan& pl, const double* rowp, const double* colp, hipStream_t st) {
    PassOut out{pl.rout, 1, pl.cout, 1};
    if (pl.S <= 0) return out;
    hipLaunchKernelGGL(k_reduce_partials, dim3((pl.S + 255) / 256), dim3(256), 0, st, pl.S, pl.na, pl.n_ct, rowp,
                       pl.nb, pl.n_rt, colp, pl.perm, pl.rout, pl.cout);
    check_launch("reduce_partials");
    return out;
}

void gather_occupations(const StreamPlan& pl, const double* f, hipStream_t st) {
    if (pl.S <= 0) return;
    if (pl.na != 1 || pl.nb != 1 || !pl.perm || !pl.gbuf) throw Error{-1, "gather_occupations: needs a 1+1 plan"};
    hipLaunchKernelGGL(k_gather_occupations, dim3((pl.S + 255) / 256), dim3(256), 0, st, pl.S, pl.perm, f, pl.gbuf);
    check_launch("gather_occupations");
}

void reduce_finish(const StreamPlan& pl, const CollisionFinish& cf, hipStream_t st) {
    if (cf.S <= 0) return;
    if (!pl.perm || cf.S != pl.S) throw Error{-1, "reduce_finish: plan and finish disagree"};
    hipLaunchKernelGGL(k_reduce_finish, dim3((cf.S + 255) / 256), dim3(256), 0, st, cf, pl.perm);
    check_launch("reduce_finish");
}

void adjoint_stage(const StreamPlan& pl, long ld, const void* P, const double* Y, const Lincomb& lc, double* lam_out,
                   double c, double* rowp, double* colp, double* ybar, double* a_acc, const double* yb1,
                   const double* yb2, const double* yb3, hipStream_t st) {
    const int S = pl.S;
    if (S <= 0) return;
    if (pl.na != 2 || pl.nb != 2 || !pl.perm || !pl.gbuf) throw Error{-1, "adjoint_stage: needs a 2+2 plan"};
    if (a_acc && !(yb1 && yb2 && yb3)) throw Error{-1, "adjoint_stage: accumulation needs the other stages"};
    hipLaunchKernelGGL(k_adj_prep, dim3((S + 255) / 256), dim3(256), 0, st, S, pl.perm, lc, Y, lam_out, pl.gbuf);
    check_launch("adj_prep");
    stream_run(pl, ld, P, rowp, colp, st);
    hipLaunchKernelGGL(k_adj_finish, dim3((S + 255) / 256), dim3(256), 0, st, S, pl.perm, pl.n_ct, pl.n_rt, rowp, colp,
                       lam_out, c, ybar, a_acc, yb1, yb2, yb3);
    check_launch("adj_finish");
}

void vjp_finish(int S, int n_ct, int n_rt, const double* rowp, const double* colp, const double* lam, double c,
                double* fbar, hipStream_t st) {
    hipLaunchKernelGGL(k_vjp_finish, dim3((S + 255) / 256), dim3(256), 0, st, S, n_ct, n_rt, rowp, colp, lam, c, fbar);
    check_launch("vjp_finish");
}

void mode_finish(int S, int nm, int ns, const double* r, VecPtrs f, VecPtrs lam, double c, double* sbar,
                 int accumulate, hipStream_t st) {
    if (ns < 1 || ns > 4) throw Error{-1, "mode_finish: 1 to 4 pairs"};
    hipLaunchKernelGGL(k_mode_finish, dim3(nm), dim3(256), 0, st, S, ns, r, f, lam, c, sbar, accumulate);
    check_launch("mode_finish");
}

void ita_gamma(int S, int n_ct, const double* rowp, double n_q, const double* vel, double* tau, double* f0, double* f,
               hipStream_t st) {
    hipLaunchKernelGGL(k_ita_gamma, dim3((S + 255) / 256), dim3(256), 0, st, S, n_ct, rowp, n_q, vel, tau, f0, f);
    check_launch("ita_gamma");
}

void ita_update(int S, int n_ct, const double* rowp, double n_q, const double* tau, const double* f0, double* f,
                hipStream_t st, const double* fprev, unsigned long long* chg) {
    hipLaunchKernelGGL(k_ita_update, dim3((S + 255) / 256), dim3(256), 0, st, S, n_ct, rowp, n_q, tau, f0, f, fprev,
                       chg);
    check_launch("ita_update");
}

void mobility_reduce(int S, const double* eps, const double* vel, const double* f, double mu, double temp,
                     double* fout, double* mob, hipStream_t st) {
    hipLaunchKernelGGL(k_mobility, dim3(1), dim3(256), 0, st, S, eps, vel, f, mu, temp, fout, mob);
    check_launch("mobility");
}

void mob_seed(int S, const double* eps, const double* vel, const double* lam, double mu, double temp, double* fbar,
              hipStream_t st) {
    hipLaunchKernelGGL(k_mob_seed, dim3(1), dim3(256), 0, st, S, eps, vel, lam, mu, temp, fbar);
    check_launch("mob_seed");
}

void ita_adj_step(int S, const double* tau, const double* fbar, const double* fnext, double* taubar, double* ubar,
                  int first, hipStream_t st) {
    hipLaunchKernelGGL(k_ita_adj_step, dim3((S + 255) / 256), dim3(256), 0, st, S, tau, fbar, fnext, taubar, ubar,
                       first);
    check_launch("ita_adj_step");
}

void ita_adj_cols(int S, int n_rt, const double* colp, double n_q, double* fbar, hipStream_t st) {
    hipLaunchKernelGGL(k_ita_adj_cols, dim3((S + 255) / 256), dim3(256), 0, st, S, n_rt, colp, n_q, fbar);
    check_launch("ita_adj_cols");
}

void ita_adj_final(int S, const double* tau, const double* fbar0, const double* vel, const double* taubar, int first,
                   double* gbar, hipStream_t st) {
    hipLaunchKernelGGL(k_ita_adj_final, dim3((S + 255) / 256), dim3(256), 0, st, S, tau, fbar0, vel, taubar, first,
                       gbar);
    check_launch("ita_adj_final");
}

void pair_adjoint(const PairAdjoint& e, hipStream_t st) {
    if (e.nm > kMaxModes) throw Error{-6, "pair_adjoint: more modes than supported"};
    dim3 grid((e.S + 127) / 128, e.ns_chunk);
    hipLaunchKernelGGL(k_pair_adjoint, grid, dim3(128), 0, st, e);
    check_launch("pair_adjoint");
}

void apply_u_column_adj(int Z, int nrp, int nm, int nw, int s_off, const double* in, const double* ks,
                        const int32_t* rp, const double* us, const int32_t* band, double* out, hipStream_t st) {
    const long per = (long)nrp * nm * nw * nw;
    hipLaunchKernelGGL(k_apply_u_column_adj, dim3((unsigned)((per + 255) / 256), Z), dim3(256), 0, st, nrp, nm, nw,
                       s_off, in, ks, rp, us, band, out);
    check_launch("apply_u_column_adj");
}

void axpy_copy(int S, const double* x, double a, const double* y, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_axpy_copy, dim3((S + 255) / 256), dim3(256), 0, st, S, x, a, y, out);
    check_launch("axpy_copy");
}

void lincomb(int S, const Lincomb& lc, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_lincomb, dim3((S + 255) / 256), dim3(256), 0, st, S, lc, out);
    check_launch("lincomb");
}

int mode_panel_tile() { return kPT; }

void mode_panel_tiles(const std::vector<double>& esort, double half_width, std::vector<int32_t>& tiles) {
    const int S = (int)esort.size();
    const int nt = (S + kPT - 1) / kPT;
    tiles.clear();
    for (int rt = 0; rt < nt; ++rt)
        for (int ct = 0; ct < nt; ++ct) {
            const int r0 = rt * kPT, r1 = std::min(S, r0 + kPT);
            const int c0 = ct * kPT, c1 = std::min(S, c0 + kPT);
            // every entry of a tile whose energies differ everywhere by more than
            // the band's half-width is zero in every per-mode matrix
            const double gap = std::max(esort[c0] - esort[r1 - 1], esort[r0] - esort[c1 - 1]);
            if (gap > half_width) continue;
            tiles.push_back(rt);
            tiles.push_back(ct);
        }
}

void mode_panel(int S, long ld, int J, int nm, int f32, const void* pm, long mat_elems, const int32_t* perm,
                const double* f, const double* lam, double* work, const int32_t* tiles, int n_tiles,
                double* partial, double c, double* sbar, int accumulate, hipStream_t st) {
    if (S <= 0 || J <= 0 || nm > kMaxModes) throw Error{-1, "mode_panel: bad sizes"};
    double* A = work;
    double* B = A + (long)J * S;
    double* C = B + (long)J * S;
    double* D = C + (long)J * S;
    const long n = (long)J * S;
    hipLaunchKernelGGL(k_panel_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, S, J, perm, f, lam, A, B,
                       C, D);
    check_launch("panel_gather");
    if (n_tiles > 0) {
        if (f32)
            hipLaunchKernelGGL(k_mode_panel<float>, dim3(n_tiles), dim3(256), 0, st, S, ld, J, nm, (const float*)pm,
                               mat_elems, A, B, C, D, tiles, partial);
        else
            hipLaunchKernelGGL(k_mode_panel<double>, dim3(n_tiles), dim3(256), 0, st, S, ld, J, nm, (const double*)pm,
                               mat_elems, A, B, C, D, tiles, partial);
        check_launch("mode_panel");
    }
    hipLaunchKernelGGL(k_mode_panel_finish, dim3(nm), dim3(256), 0, st, n_tiles, nm, partial, c, sbar, accumulate);
    check_launch("mode_panel_finish");
}

void occ_vectors(int S, const double* f, const double* lam, double* o0, double* o1, double* o2, hipStream_t st) {
    hipLaunchKernelGGL(k_occ_vectors, dim3((S + 255) / 256), dim3(256), 0, st, S, f, lam, o0, o1, o2);
    check_launch("occ_vectors");
}

void fill(long n, double v, double* out, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, v, out);
    check_launch("fill");
}

}  // namespace ephx
