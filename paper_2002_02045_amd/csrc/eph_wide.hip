// Per-pair work of the e-ph matrix elements for large models (Nw > 16 or more
// than 12 modes, e.g. a 40-atom cell with 64 Wannier functions), where one
// pair's block Nw x Nw x 3nat no longer fits a workgroup's registers and LDS.
// The rotation and the mode projection (Eq. eph_mat with g^H of Eq.
// eph_mat_wann2) are then batched complex GEMMs on MFMA:
//
//   rotation    g^H[pair][x] = U(k+q)^dag g'^W[pair][x]        (Nw x Nw x Nw per x)
//   long range  g^H[pair][x] += C_x(q) U(k+q)^dag U(k)          (polar models)
//   projection  g[pair]      = P(q) g^H[pair],  P_nu,x = sqrt(hbar/2 w_nu) e_x,nu / sqrt(M_x)
//
// where g'^W already carries U(k) on the right (applied once per k).  The
// rates reduction (Eqs. scatter_rate, BTE_W) and the |g|^2 output then read g.
#include "internal.h"

namespace ephx {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

inline void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{-3, std::string(what) + ": " + hipGetErrorString(e)};
}

__device__ __forceinline__ dbl4 mfma(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ flt4 mfma(float a, float b, flt4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> struct Acc;
template <> struct Acc<double> {
    typedef dbl4 type;
    // accumulator element v of lane l is C[l/16 + 4v][l%16] for the f64 instruction
    static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <> struct Acc<float> {
    typedef flt4 type;
    static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

constexpr int kT = 64;    // output tile (rows and columns)
constexpr int kKs = 16;   // K per staging step

// Batched complex GEMM, C[b] = op(A[b]) B[b], row-major, interleaved complex.
// op(A)(m,k) = A[m*lda + k], or conj(A[k*lda + m]) when CA.  The batch index is
// b = (b0 * n1 + b1), offsets b0*s?0 + b1*s?1 (complex elements).  256 threads
// own a 64 x 16 CB tile: wave w the rows 16w..16w+15, CB 16-column MFMA
// blocks (CB = 8 halves the A reads per product where N allows).
template <typename T, typename TA, typename TB, bool CA, int CB = 4>
__global__ __launch_bounds__(256) void k_cgemm(int M, int N, int K, int mt, int ntl, CBatch bt, const TA* __restrict__ A,
                                               long lda, const TB* __restrict__ B, long ldb, T* __restrict__ C,
                                               long ldc) {
    typedef typename Acc<T>::type acc_t;
    constexpr int kTN = 16 * CB;   // columns of the tile
    __shared__ T as[kKs][kT][2];   // [k][m]
    __shared__ T bs[kKs][kTN][2];  // [k][n]
    long bid = blockIdx.x;
    const int nti = (int)(bid % ntl);
    bid /= ntl;
    const int mti = (int)(bid % mt);
    bid /= mt;
    const long b1 = bid % bt.n1, b0 = bid / bt.n1;
    A += 2 * (b0 * bt.sa0 + b1 * bt.sa1);
    B += 2 * (b0 * bt.sb0 + b1 * bt.sb1);
    C += 2 * (b0 * bt.sc0 + b1 * bt.sc1);
    const int row0 = mti * kT, col0 = nti * kTN;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    acc_t are[CB], aim[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        are[cb] = acc_t{0, 0, 0, 0};
        aim[cb] = acc_t{0, 0, 0, 0};
    }
    typedef TA ta2 __attribute__((ext_vector_type(2)));
    typedef TB tb2 __attribute__((ext_vector_type(2)));
    constexpr int EPA = kKs * kT / 256, EPB = kKs * kTN / 256;   // elements per thread and step
    // load phases per step: all of a step's loads are issued before its LDS
    // writes for FP32 tiles; FP64 takes two phases held apart by a scheduling
    // barrier, whose operands and addresses would otherwise halve the waves a
    // SIMD holds
    constexpr int NPH = sizeof(T) == 4 ? 1 : 2, PA = EPA / NPH, PB = EPB / NPH;
    for (int kc = 0; kc < K; kc += kKs) {
        // indices clamped into the matrices, the values past their edges
        // replaced by zeros: the thread waits on NPH memory latencies per step
        // instead of one per element
#pragma unroll
        for (int ph = 0; ph < NPH; ++ph) {
            ta2 av[PA];
            tb2 bv[PB];
#pragma unroll
            for (int jj = 0; jj < PA; ++jj) {
                const int e = tid + 256 * (ph * PA + jj);
                // A: for CA the stored matrix is read along m (contiguous), else along k
                const int kk = CA ? e / kT : e % kKs, m = CA ? e % kT : e / kKs;
                const long ka = min(kc + kk, K - 1), ma = min(row0 + m, M - 1);
                av[jj] = *reinterpret_cast<const ta2*>(A + 2 * (CA ? ka * lda + ma : ma * lda + ka));
            }
#pragma unroll
            for (int jj = 0; jj < PB; ++jj) {
                const int e = tid + 256 * (ph * PB + jj);
                const int kb = e / kTN, n = e % kTN;
                const long kbb = min(kc + kb, K - 1), nb = min(col0 + n, N - 1);
                bv[jj] = *reinterpret_cast<const tb2*>(B + 2 * (kbb * ldb + nb));
            }
#pragma unroll
            for (int jj = 0; jj < PA; ++jj) {
                const int e = tid + 256 * (ph * PA + jj);
                const int kk = CA ? e / kT : e % kKs, m = CA ? e % kT : e / kKs;
                const bool aok = kc + kk < K && row0 + m < M;
                as[kk][m][0] = aok ? (T)av[jj].x : (T)0;
                as[kk][m][1] = aok ? (CA ? -(T)av[jj].y : (T)av[jj].y) : (T)0;
            }
#pragma unroll
            for (int jj = 0; jj < PB; ++jj) {
                const int e = tid + 256 * (ph * PB + jj);
                const int kb = e / kTN, n = e % kTN;
                const bool bok = kc + kb < K && col0 + n < N;
                bs[kb][n][0] = bok ? (T)bv[jj].x : (T)0;
                bs[kb][n][1] = bok ? (T)bv[jj].y : (T)0;
            }
            // keeps the next phase's loads behind these writes
            if constexpr (NPH > 1) __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kKs / 4; ++s) {
            const int kk = 4 * s + lk;
            const T ar = as[kk][wave * 16 + li][0], ai = as[kk][wave * 16 + li][1];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const T br = bs[kk][cb * 16 + li][0], bi = bs[kk][cb * 16 + li][1];
                are[cb] = mfma(ar, br, are[cb]);
                are[cb] = mfma(-ai, bi, are[cb]);
                aim[cb] = mfma(ar, bi, aim[cb]);
                aim[cb] = mfma(ai, br, aim[cb]);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int col = col0 + cb * 16 + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = row0 + wave * 16 + Acc<T>::row(lk, v);
            if (row < M && col < N) {
                const long o = (long)row * ldc + col;
                C[2 * o] = are[cb][v];
                C[2 * o + 1] = aim[cb][v];
            }
        }
    }
}

template <typename T, typename TA, typename TB, bool CA>
void launch_cgemm(int M, int N, int K, long nbatch, const CBatch& bt, const TA* A, long lda, const TB* B, long ldb,
                  T* C, long ldc, hipStream_t st) {
    // 128-column tiles for FP32 products wide enough to fill them (the mode
    // projection, N = Nw^2): each staged A element then feeds twice the MFMAs
    const bool wide = sizeof(T) == 4 && N >= 128;
    const int tn = wide ? 128 : 64;
    const int mt = (M + kT - 1) / kT, ntl = (N + tn - 1) / tn;
    const long blocks = nbatch * mt * ntl;
    if (blocks <= 0) return;
    if (blocks > 0x7fffffffL) throw Error{-1, "cgemm: grid too large"};
    if constexpr (sizeof(T) == 4) {
        if (wide) {
            hipLaunchKernelGGL((k_cgemm<T, TA, TB, CA, 8>), dim3((unsigned)blocks), dim3(256), 0, st, M, N, K, mt, ntl,
                               bt, A, lda, B, ldb, C, ldc);
            check_launch("cgemm");
            return;
        }
    }
    hipLaunchKernelGGL((k_cgemm<T, TA, TB, CA, 4>), dim3((unsigned)blocks), dim3(256), 0, st, M, N, K, mt, ntl, bt, A,
                       lda, B, ldb, C, ldc);
    check_launch("cgemm");
}

// P[q][nu][x] = sqrt(hbar^2/(2 M_x omega_nu)) e_x,nu(q) (zero for omega <= cut),
// formed in FP64 and stored in the precision of the product that reads it
template <typename TP>
__global__ void k_proj_matrix(int nq, int q_off, int nm, const double* __restrict__ omega, const double* __restrict__ evec,
                              const double* __restrict__ minv, double omega_cut, TP* __restrict__ P) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long per = (long)nm * nm;
    if (t >= nq * per) return;
    const long q = t / per;
    const int nu = (int)((t % per) / nm), x = (int)(t % nm);
    const long qg = q_off + q;
    const double om = omega[qg * nm + nu];
    const double amp = om > omega_cut ? sqrt(kHbar2AmuA2 / (2.0 * om)) * minv[x] : 0.0;
    P[2 * t] = (TP)(amp * evec[2 * ((qg * nm + x) * nm + nu)]);
    P[2 * t + 1] = (TP)(amp * evec[2 * ((qg * nm + x) * nm + nu) + 1]);
}

// gh[pair][x][m][n] += C_x(q) ov[pair][m][n]
template <typename T>
__global__ void k_polar_add(long npair, int nq, int q_off, int nm, int nw2, const double* __restrict__ lr,
                            const double* __restrict__ ov, T* __restrict__ gh) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long per = (long)nm * nw2;
    if (t >= npair * per) return;
    const long pair = t / per;
    const int x = (int)((t % per) / nw2), mn = (int)(t % nw2);
    const long qg = q_off + pair % nq;
    const double cr = lr[2 * (qg * nm + x)], ci = lr[2 * (qg * nm + x) + 1];
    const double orr = ov[2 * (pair * nw2 + mn)], oi = ov[2 * (pair * nw2 + mn) + 1];
    gh[2 * t] += (T)(cr * orr - ci * oi);
    gh[2 * t + 1] += (T)(cr * oi + ci * orr);
}

// |g|^2 into the [nk][nq_total][nm][nw][nw] output
template <typename T>
__global__ void k_wide_g2(WideChunk w) {
    const long per = (long)w.nm * w.nw * w.nw;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)w.nkb * w.nq * per) return;
    const long pair = t / per, el = t % per;
    const int z = (int)(pair / w.nq), q = (int)(pair % w.nq);
    const T* g = reinterpret_cast<const T*>(w.g);
    const T gr = g[2 * t], gi = g[2 * t + 1];
    const long off = ((long)(w.k_off + z) * w.nq_total + w.q_off + q) * per + el;
    reinterpret_cast<T*>(w.g2)[off] = gr * gr + gi * gi;
}

// partial[z][blk][n][nu] = (2 pi/hbar) x sum over the block's q and all m of
//   w_q |g_mn,nu|^2 [delta(e_n - hw - e_m)(1 + N - f_m) + delta(e_n + hw - e_m)(N + f_m)]
// Workgroup (output tile of 256 (nu, n), q block, k): one thread per (nu, n);
// the energies and occupations at k+q of the block's q are staged in LDS.  The
// Gaussians are evaluated in T, as in the register epilogue of small models.
constexpr int kWideQ = 32;    // q per block (the partial layout's block size)

template <typename T>
__global__ __launch_bounds__(256) void k_wide_rates(WideChunk w) {
    __shared__ double s_em[kWideQ][kMaxNwWide], s_fm[kWideQ][kMaxNwWide];
    const int z = blockIdx.z, blk = blockIdx.y;
    const int nw = w.nw, nm = w.nm;
    const int q0 = blk * w.qpb, q1 = min(w.nq, q0 + w.qpb);
    const double kt = kBoltzEv * w.temp;
    for (int e = threadIdx.x; e < (q1 - q0) * nw; e += blockDim.x) {
        const int ql = e / nw, m = e % nw;
        const double em = w.ekq[((long)z * w.nq + q0 + ql) * nw + m];
        s_em[ql][m] = em;
        s_fm[ql][m] = 1.0 / (exp((em - w.mu) / kt) + 1.0);
    }
    __syncthreads();
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= nm * nw) return;
    const int nu = o / nw, n = o % nw;
    const T is = (T)(1.0 / w.sigma), nrm = (T)(1.0 / (sqrt(kPi) * w.sigma));
    const T* g = reinterpret_cast<const T*>(w.g);
    const double en = w.ek[(long)z * nw + n];
    double acc = 0.0;
    for (int q = q0; q < q1; ++q) {
        const long qg = (long)w.q_off + q;
        const double om = w.omega[qg * nm + nu];
        if (!(om > w.omega_cut)) continue;
        const double nb = 1.0 / expm1(om / kt);
        const double wq = w.qw ? w.qw[qg] : w.uniform_w;
        const long pair = (long)z * w.nq + q;
        const T* gp = g + 2 * ((pair * nm + nu) * nw) * nw + 2 * n;
        double s = 0.0;
        for (int m = 0; m < nw; ++m) {
            const double em = s_em[q - q0][m], fm = s_fm[q - q0][m];
            const T gr = gp[2 * m * nw], gi = gp[2 * m * nw + 1];
            const T x1 = (T)(en - om - em) * is, x2 = (T)(en + om - em) * is;
            const T d_em = x1 * x1 > (T)200 ? (T)0 : nrm * exp(-x1 * x1);
            const T d_ab = x2 * x2 > (T)200 ? (T)0 : nrm * exp(-x2 * x2);
            s += (double)(gr * gr + gi * gi) * ((double)d_em * (1.0 + nb - fm) + (double)d_ab * (nb + fm));
        }
        acc += wq * s;
    }
    w.partial[(((long)z * w.nblk + blk) * nw + n) * nm + nu] = acc * (2.0 * kPi / kHbarEvFs);
}

// rotation, long-range term and projection: w.g ends as g_mn,nu; w.gh and
// w.pmat hold g^H and P(q)
template <typename T>
void wide_forward(const WideChunk& w, hipStream_t st) {
    const int nw = w.nw, nm = w.nm, nw2 = nw * nw;
    const long npair = (long)w.nkb * w.nq;
    T* gw = reinterpret_cast<T*>(w.g);
    T* gh = reinterpret_cast<T*>(w.gh);
    // rotation: batch (pair, x), A = U(k+q)^dag
    {
        CBatch b{};
        b.n1 = nm;
        b.sa0 = nw2;
        b.sa1 = 0;
        b.sb0 = (long)nm * nw2;
        b.sb1 = nw2;
        b.sc0 = (long)nm * nw2;
        b.sc1 = nw2;
        launch_cgemm<T, double, T, true>(nw, nw, nw, npair * nm, b, w.ukq, nw, gw, nw, gh, nw, st);
    }
    if (w.lr != nullptr) {
        // ov = U(k+q)^dag U(k): batch (z, q)
        CBatch b{};
        b.n1 = w.nq;
        b.sa0 = (long)w.nq * nw2;
        b.sa1 = nw2;
        b.sb0 = nw2;
        b.sb1 = 0;
        b.sc0 = (long)w.nq * nw2;
        b.sc1 = nw2;
        launch_cgemm<double, double, double, true>(nw, nw, nw, npair, b, w.ukq, nw, w.uk, nw, w.ov, nw, st);
        const long tot = npair * nm * nw2;
        hipLaunchKernelGGL(k_polar_add<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, npair, w.nq, w.q_off,
                           nm, nw2, w.lr, w.ov, gh);
        check_launch("polar_add");
    }
    // projection: batch (z, q), A = P(q), result over g'^W's storage
    {
        const long tot = (long)w.nq * nm * nm;
        // P in T: the FP32 product reads half the bytes of its shared operand,
        // the same values it would have rounded while staging FP64 ones
        T* pm = reinterpret_cast<T*>(w.pmat);
        hipLaunchKernelGGL(k_proj_matrix<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, w.nq, w.q_off, nm,
                           w.omega, w.evec, w.minv, w.omega_cut, pm);
        check_launch("proj_matrix");
        CBatch b{};
        b.n1 = w.nq;
        b.sa0 = 0;
        b.sa1 = (long)nm * nm;
        b.sb0 = (long)w.nq * nm * nw2;
        b.sb1 = (long)nm * nw2;
        b.sc0 = b.sb0;
        b.sc1 = b.sb1;
        launch_cgemm<T, T, T, false>(nm, nw2, nm, npair, b, pm, nm, gh, nw2, gw, nw2, st);
    }
}

template <typename T>
void wide_chunk(const WideChunk& w, int rates, hipStream_t st) {
    const int nw = w.nw, nm = w.nm, nw2 = nw * nw;
    const long npair = (long)w.nkb * w.nq;
    wide_forward<T>(w, st);
    if (rates) {
        if (w.qpb > kWideQ) throw Error{-1, "wide_rates: q block too large"};
        hipLaunchKernelGGL(k_wide_rates<T>, dim3((nm * nw + 255) / 256, w.nblk, w.nkb), dim3(256), 0, st, w);
        check_launch("wide_rates");
    } else {
        const long tot = npair * nm * nw2;
        hipLaunchKernelGGL(k_wide_g2<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, w);
        check_launch("wide_g2");
    }
}

// Adjoint of the rates for L = sum_nk lam_nk Gamma_nk, per element (pair, nu, m, n):
//   gbar_mn,nu = 2 (2 pi/hbar) lam_n w_q D_mn,nu g_mn,nu,
//   D = delta(e_n - hw - e_m)(1 + N - f_m) + delta(e_n + hw - e_m)(N + f_m)
// (FP64, the same Gaussians and cut-offs as the forward).
__global__ void k_wide_rates_bar(WideChunk w, const double* __restrict__ lam, double* __restrict__ gbar) {
    const int nw = w.nw, nm = w.nm;
    const long per = (long)nm * nw * nw;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)w.nkb * w.nq * per) return;
    const long pair = t / per;
    const int nu = (int)((t % per) / (nw * nw)), m = (int)((t / nw) % nw), n = (int)(t % nw);
    const int z = (int)(pair / w.nq);
    const long qg = (long)w.q_off + pair % w.nq;
    const double om = w.omega[qg * nm + nu];
    double f = 0.0;
    if (om > w.omega_cut) {
        const double kt = kBoltzEv * w.temp;
        const double is = 1.0 / w.sigma, nrm = 1.0 / (sqrt(kPi) * w.sigma);
        const double nb = 1.0 / expm1(om / kt);
        const double em = w.ekq[pair * nw + m];
        const double fm = 1.0 / (exp((em - w.mu) / kt) + 1.0);
        const double en = w.ek[(long)z * nw + n];
        const double wq = w.qw ? w.qw[qg] : w.uniform_w;
        const double x1 = (en - om - em) * is, x2 = (en + om - em) * is;
        const double de = x1 * x1 > 200.0 ? 0.0 : nrm * exp(-x1 * x1);
        const double da = x2 * x2 > 200.0 ? 0.0 : nrm * exp(-x2 * x2);
        f = 2.0 * (2.0 * kPi / kHbarEvFs) * lam[(long)(w.k_off + z) * nw + n] * wq *
            (de * (1.0 + nb - fm) + da * (nb + fm));
    }
    const double* g = reinterpret_cast<const double*>(w.g);
    gbar[2 * t] = f * g[2 * t];
    gbar[2 * t + 1] = f * g[2 * t + 1];
}

}  // namespace

// FP64: g'W_bar[pair][x] = U(k+q) sum_nu conj(P_nu,x) gbar_nu, through w.g and
// w.gh as work (the forward is recomputed first).
void eph_wide_rates_vjp(const WideChunk& w, const double* lam, double* gwbar, hipStream_t st) {
    if (w.nkb <= 0 || w.nq <= 0) return;
    const int nw = w.nw, nm = w.nm, nw2 = nw * nw;
    const long npair = (long)w.nkb * w.nq;
    wide_forward<double>(w, st);
    double* g = reinterpret_cast<double*>(w.g);
    double* gb = reinterpret_cast<double*>(w.gh);
    const long tot = npair * nm * nw2;
    hipLaunchKernelGGL(k_wide_rates_bar, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, w, lam, gb);
    check_launch("wide_rates_bar");
    {
        // adjoint of the projection: batch (z, q), A = P(q) read conjugate-transposed
        CBatch b{};
        b.n1 = w.nq;
        b.sa0 = 0;
        b.sa1 = (long)nm * nm;
        b.sb0 = (long)w.nq * nm * nw2;
        b.sb1 = (long)nm * nw2;
        b.sc0 = b.sb0;
        b.sc1 = b.sb1;
        launch_cgemm<double, double, double, true>(nm, nw2, nm, npair, b, w.pmat, nm, gb, nw2, g, nw2, st);
    }
    {
        // adjoint of the rotation: batch (pair, x), A = U(k+q)
        CBatch b{};
        b.n1 = nm;
        b.sa0 = nw2;
        b.sa1 = 0;
        b.sb0 = (long)nm * nw2;
        b.sb1 = nw2;
        b.sc0 = (long)nm * nw2;
        b.sc1 = nw2;
        launch_cgemm<double, double, double, false>(nw, nw, nw, npair * nm, b, w.ukq, nw, g, nw, gwbar, nw, st);
    }
}

void cgemm_f64_batched(int M, int N, int K, long nbatch, const CBatch& b, const double* A, long lda, const double* B,
                       long ldb, double* C, long ldc, hipStream_t st) {
    launch_cgemm<double, double, double, false>(M, N, K, nbatch, b, A, lda, B, ldb, C, ldc, st);
}

void eph_wide_chunk(const WideChunk& w, int f32, int rates, hipStream_t st) {
    if (w.nkb <= 0 || w.nq <= 0) return;
    if (f32)
        wide_chunk<float>(w, rates, st);
    else
        wide_chunk<double>(w, rates, st);
}

}  // namespace ephx
