// Per-(k,q) work after the Fourier contractions: band rotation (Eq.
// eph_mat_wann2), mode projection (Eq. eph_mat), |g|^2, the Gaussian-weighted
// scattering-rate sums (Eqs. scatter_rate, BTE_W), the Froehlich long-range
// term (Eq. e_ph_long with the bra-ket of Eq. smooth_phase) and band velocities
// (Eqs. velocity, wannier_4).
#include "internal.h"

namespace ephx {
namespace {

inline void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{-3, std::string(what) + ": " + hipGetErrorString(e)};
}

typedef float flt4 __attribute__((ext_vector_type(4)));

template <typename T>
struct cx {
    T x, y;
};
template <typename T>
__device__ __forceinline__ cx<T> ld(const T* p, long i) {
    return {p[2 * i], p[2 * i + 1]};
}
template <typename T>
__device__ __forceinline__ cx<T> ldd(const double* p, long i) {
    return {(T)p[2 * i], (T)p[2 * i + 1]};
}
template <typename T>
__device__ __forceinline__ void cfma(cx<T>& acc, cx<T> a, cx<T> b) {  // acc += a*b
    acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
template <typename T>
__device__ __forceinline__ void cjfma(cx<T>& acc, cx<T> a, cx<T> b) {  // acc += conj(a)*b
    acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
    acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
}

__global__ void k_apply_u_right(int nrp, int nm, int nw, const double* __restrict__ g, const double* __restrict__ u,
                                double* __restrict__ out) {
    // out[z][p][x][i][n] = sum_j g[z][p][x][i][j] u[z][j][n]
    const int z = blockIdx.y;
    const long per = (long)nrp * nm * nw * nw;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= per) return;
    const int n = (int)(t % nw);
    const long row = t / nw;  // (p, x, i)
    const double* gz = g + (long)z * per * 2;
    const double* uz = u + (long)z * nw * nw * 2;
    cx<double> acc = {0.0, 0.0};
    for (int j = 0; j < nw; ++j) cfma(acc, ld(gz, row * nw + j), ld(uz, (long)j * nw + n));
    out[((long)z * per + t) * 2] = acc.x;
    out[((long)z * per + t) * 2 + 1] = acc.y;
}

__global__ void k_apply_u_column(int nrp, int nm, int nw, const double* __restrict__ g, const double* __restrict__ us,
                                 const int32_t* __restrict__ band, double* __restrict__ out) {
    // out[z][p][x][i] = sum_j g[z][p][x][i][j] us[z][j][band_z]
    const int z = blockIdx.y;
    const long per = (long)nrp * nm * nw;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= per) return;
    const int bz = band[z];
    const double* gz = g + (long)z * per * nw * 2;
    const double* uz = us + (long)z * nw * nw * 2;
    cx<double> acc = {0.0, 0.0};
    for (int j = 0; j < nw; ++j) cfma(acc, ld(gz, t * nw + j), ld(uz, (long)j * nw + bz));
    out[((long)z * per + t) * 2] = acc.x;
    out[((long)z * per + t) * 2 + 1] = acc.y;
}

constexpr int kQPB = 32;   // (k, q) pairs per epilogue workgroup

__global__ void k_apply_u_right_adj(int nrp, int nm, int nw, const double* __restrict__ g, const double* __restrict__ u,
                                    double* __restrict__ out) {
    // out[z][p][x][i][j] = sum_n g[z][p][x][i][n] conj(u[z][j][n])
    const int z = blockIdx.y;
    const long per = (long)nrp * nm * nw * nw;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= per) return;
    const int j = (int)(t % nw);
    const long row = t / nw;
    const double* gz = g + (long)z * per * 2;
    const double* uz = u + (long)z * nw * nw * 2;
    cx<double> acc = {0.0, 0.0};
    for (int n = 0; n < nw; ++n) {
        const cx<double> a = ld(gz, row * nw + n), b = ld(uz, (long)j * nw + n);
        acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));   // a * conj(b)
        acc.y = fma(a.y, b.x, fma(-a.x, b.y, acc.y));
    }
    out[((long)z * per + t) * 2] = acc.x;
    out[((long)z * per + t) * 2 + 1] = acc.y;
}

// Adjoint of the per-pair epilogue for L = sum_nk lam_nk Gamma_nk (FP64).  With
// D = delta(e_n - hw - e_m)(1 + N - f_m) + delta(e_n + hw - e_m)(N + f_m):
//   gbar_mn,nu   = 2 (2 pi/hbar) lam_n w_q D g_mn,nu          (gradient of lam w c D |g|^2)
//   gHbar[x]_mn  = sum_nu conj(es[x][nu]) gbar_mn,nu          (adjoint of the mode projection)
//   g'Wbar[x]_in = sum_m U_im(k+q) gHbar[x]_mn                 (adjoint of U^dag(k+q) .)
// The long-range term enters through g (it does not depend on g(Re,Rp)).
__global__ __launch_bounds__(64) void k_eph_adjoint(EphEpilogue e, const double* __restrict__ lam,
                                                    double* __restrict__ gwbar) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const int nw = e.nw, nm = e.nm, nw2 = nw * nw, ng = nm * nw2;
    cx<double>* s_gw = reinterpret_cast<cx<double>*>(smem);
    cx<double>* s_gb = s_gw + ng;
    cx<double>* s_u = s_gb + ng;
    cx<double>* s_es = s_u + nw2;
    double* s_nb = reinterpret_cast<double*>(s_es + nm * nm);
    double* s_om = s_nb + nm;
    double* s_em = s_om + nm;
    double* s_fm = s_em + nw;
    const int z = blockIdx.y, blk = blockIdx.x, lane = threadIdx.x;
    const int q0 = blk * kQPB, q1 = min(e.nq, q0 + kQPB);
    const double* gwz = reinterpret_cast<const double*>(e.gw) + (long)z * e.nq * ng * 2;
    const double kt = kBoltzEv * e.temp;
    const double is = 1.0 / e.sigma, nrm = 1.0 / (sqrt(kPi) * e.sigma);
    const double c2 = 2.0 * (2.0 * kPi / kHbarEvFs);
    for (int ql = q0; ql < q1; ++ql) {
        const long qg = (long)e.q_off + ql;
        const long pair = (long)z * e.nq + ql;
        const double* gp = gwz + (long)ql * ng * 2;
        const double* uq = e.ukq + pair * nw2 * 2;
        for (int i = lane; i < ng; i += 64) s_gw[i] = ld(gp, i);
        for (int i = lane; i < nw2; i += 64) s_u[i] = ld(uq, e.u_cm ? (i % nw) * nw + i / nw : i);
        for (int i = lane; i < nm * nm; i += 64) {
            const int x = i / nm, nu = i % nm;
            const double om = e.omega[qg * nm + nu];
            const double amp = om > e.omega_cut ? sqrt(kHbar2AmuA2 / (2.0 * om)) * e.minv[x] : 0.0;
            s_es[i] = {amp * e.evec[2 * ((qg * nm + x) * nm + nu)], amp * e.evec[2 * ((qg * nm + x) * nm + nu) + 1]};
        }
        if (lane < nm) {
            const double om = e.omega[qg * nm + lane];
            s_om[lane] = om;
            s_nb[lane] = om > e.omega_cut ? 1.0 / expm1(om / kt) : 0.0;
        }
        if (lane < nw) {
            const double em = e.ekq[pair * nw + lane];
            s_em[lane] = em;
            s_fm[lane] = 1.0 / (exp((em - e.mu) / kt) + 1.0);
        }
        __syncthreads();
        const double wq = e.qw ? e.qw[qg] : e.uniform_w;
        for (int el = lane; el < nw2; el += 64) {
            const int m = el / nw, n = el % nw;
            cx<double> gh[kMaxModes];
            for (int x = 0; x < nm; ++x) {
                cx<double> a = {0, 0};
                for (int i = 0; i < nw; ++i) cjfma(a, s_u[i * nw + m], s_gw[(x * nw + i) * nw + n]);
                gh[x] = a;
            }
            if (e.lr != nullptr) {
                cx<double> ov = {0, 0};
                const double* ukz = e.uk + (long)z * nw2 * 2;
                for (int i = 0; i < nw; ++i) cjfma(ov, s_u[i * nw + m], ld(ukz, (long)i * nw + n));
                for (int x = 0; x < nm; ++x) cfma(gh[x], ld(e.lr, qg * nm + x), ov);
            }
            const double en = e.ek[(long)z * nw + n], em = s_em[m], fm = s_fm[m];
            const double ln = lam[(long)(e.k_off + z) * nw + n];
            cx<double> ghb[kMaxModes];
            for (int x = 0; x < nm; ++x) ghb[x] = {0.0, 0.0};
            for (int nu = 0; nu < nm; ++nu) {
                const double om = s_om[nu];
                if (!(om > e.omega_cut)) continue;
                cx<double> g = {0, 0};
                for (int x = 0; x < nm; ++x) cfma(g, s_es[x * nm + nu], gh[x]);
                const double nb = s_nb[nu];
                const double x1 = (en - om - em) * is, x2 = (en + om - em) * is;
                const double de = x1 * x1 > 200.0 ? 0.0 : nrm * exp(-x1 * x1);
                const double da = x2 * x2 > 200.0 ? 0.0 : nrm * exp(-x2 * x2);
                const double w = c2 * ln * wq * (de * (1.0 + nb - fm) + da * (nb + fm));
                const cx<double> gb = {w * g.x, w * g.y};
                for (int x = 0; x < nm; ++x) cjfma(ghb[x], s_es[x * nm + nu], gb);
            }
            for (int x = 0; x < nm; ++x) s_gb[(x * nw + m) * nw + n] = ghb[x];
        }
        __syncthreads();
        double* out = gwbar + ((long)z * e.nq + ql) * ng * 2;
        for (int o = lane; o < ng; o += 64) {
            const int x = o / nw2, i = (o / nw) % nw, n = o % nw;
            cx<double> a = {0, 0};
            for (int m = 0; m < nw; ++m) cfma(a, s_u[i * nw + m], s_gb[(x * nw + m) * nw + n]);
            out[2 * o] = a.x;
            out[2 * o + 1] = a.y;
        }
        __syncthreads();
    }
}

__global__ void k_scale_rows(long rows, long cols, const double* __restrict__ w, double* __restrict__ data) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * cols) return;
    const double s = w[t / cols];
    data[2 * t] *= s;
    data[2 * t + 1] *= s;
}

// Bound of the fp16 scale of a device copy of g(Re,Rp), times the weights
// w[Re][Rp] if given: for each (Rp, mode component, row i) the sum over Re and
// j of |w g_ij|, then
// the largest of them, as the bit pattern of a non-negative double in out[0]
// (atomicMax on the pattern orders non-negative doubles); out[1] != 0 if an
// entry is not finite.  One thread per (Rp, component, row).
template <typename TG>
__global__ void k_g_row_bound(int n_re, long rows, int nw, const TG* __restrict__ g,
                              const double* __restrict__ w, long rows_per_rp, int n_rp,
                              unsigned long long* __restrict__ out) {
    const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double t = 0.0;
    bool bad = false;
    if (r < rows) {
        for (int e = 0; e < n_re; ++e) {
            const TG* x = g + ((size_t)e * rows + r) * nw * 2;
            double u = 0.0;
            for (int j = 0; j < nw; ++j) {
                const double a = x[2 * j], b = x[2 * j + 1];
                bad = bad || !isfinite(a) || !isfinite(b);
                u += hypot(a, b);
            }
            t += w ? fabs(w[(long)e * n_rp + r / rows_per_rp]) * u : u;
        }
    }
    __shared__ double red[256];
    __shared__ int badf;
    if (threadIdx.x == 0) badf = 0;
    red[threadIdx.x] = t;
    __syncthreads();
    if (bad) atomicOr(&badf, 1);
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&out[0], (unsigned long long)__double_as_longlong(red[0]));
        if (badf) atomicOr(&out[1], 1ull);
    }
}

// g(Re,Rp) drawn on the device by the counter scheme of the inputs: Philox4x32
// with 10 rounds (Salmon et al., SC11: multipliers 0xD2511F53 and 0xCD9E8D57,
// key increments 0x9E3779B9 and 0xBB67AE85), six blocks per complex entry t
// with the 64-bit counter 6t + b, and an Irwin-Hall sum of twelve words per
// part: x = (sum of the words) 2^-32 - 6, stored as float(env[Re][Rp] x).
__device__ __forceinline__ void philox10(unsigned int& c0, unsigned int& c1, unsigned int& c2, unsigned int& c3,
                                         unsigned int k0, unsigned int k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const unsigned int hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const unsigned int hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const unsigned int n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// A grid-stride loop: the dispatch counts work-items in 32 bits, and the
// large cell's tensor has 2.3e10 entries.
__global__ void k_gen_coupling(long n, long per, int n_rp, unsigned long long seed, const double* __restrict__ env,
                               float* __restrict__ out) {
    const unsigned int k0 = (unsigned int)(seed & 0xFFFFFFFFull), k1 = (unsigned int)(seed >> 32);
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        unsigned long long sum[2] = {0, 0};
#pragma unroll
        for (int b = 0; b < 6; ++b) {
            const unsigned long long ctr = (unsigned long long)t * 6ull + (unsigned long long)b;
            unsigned int c0 = (unsigned int)(ctr & 0xFFFFFFFFull), c1 = (unsigned int)(ctr >> 32), c2 = 0, c3 = 0;
            philox10(c0, c1, c2, c3, k0, k1);
            sum[b / 3] += (unsigned long long)c0 + c1 + (unsigned long long)c2 + c3;
        }
        const double a = env[t / per];
        const double xr = (double)sum[0] * 0x1p-32 - 6.0, xi = (double)sum[1] * 0x1p-32 - 6.0;
        out[2 * t] = (float)(a * xr);
        out[2 * t + 1] = (float)(a * xi);
    }
}

__global__ void k_convert(long count, const double* __restrict__ in, float* __restrict__ out) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) out[t] = (float)in[t];
}

// The factors the epilogue stages per pair that depend on q alone (scaled mode
// eigenvectors e[x][nu] sqrt(hbar^2/(2 M_x omega_nu)) and Bose factors) or on
// the pair's k+q energies alone (Fermi factors), formed once per chunk with
// the same expressions, so the values are those the per-pair path forms.
template <typename T>
__global__ void k_mode_factors(int nq, int q_off, int nm, const double* __restrict__ omega,
                               const double* __restrict__ evec, const double* __restrict__ minv, double omega_cut,
                               double temp, cx<T>* __restrict__ es, double* __restrict__ nb) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;   // (q, x, nu)
    if (t >= (long)nq * nm * nm) return;
    const int i = (int)(t % (nm * nm));
    const long ql = t / (nm * nm), qg = q_off + ql;
    const int x = i / nm, nu = i % nm;
    const double om = omega[qg * nm + nu];
    const double amp = om > omega_cut ? sqrt(kHbar2AmuA2 / (2.0 * om)) * minv[x] : 0.0;
    es[t] = {(T)(amp * evec[2 * ((qg * nm + x) * nm + nu)]), (T)(amp * evec[2 * ((qg * nm + x) * nm + nu) + 1])};
    if (x == 0) nb[ql * nm + nu] = om > omega_cut ? 1.0 / expm1(om / (kBoltzEv * temp)) : 0.0;
}

__global__ void k_fermi_factors(long n, const double* __restrict__ eps, double mu, double temp,
                                double* __restrict__ f) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) f[t] = 1.0 / (exp((eps[t] - mu) / (kBoltzEv * temp)) + 1.0);
}

// One 64-lane workgroup walks QPB consecutive (k, q) pairs of one k.  Per pair
// the wavefront stages g'(k,q), U(k+q), the scaled mode eigenvectors
// e[x][nu] sqrt(hbar^2/(2 M_x omega_nu)), the Bose factors, and the final-band
// energies and Fermi factors in LDS (each computed once per pair); then lane
// <-> element (m, n) (up to 4 elements per lane) forms
//   g^H[x] = sum_i conj(U_im(k+q)) g'[x][i][n],  g_nu = sum_x es[x][nu] g^H[x]
// and either writes |g_nu|^2 or accumulates the delta-weighted rate terms.

// NW, NM > 0 fix the band and mode counts at compile time (fully unrolled,
// register-resident accumulators); NW = NM = 0 is the runtime-sized fallback.
template <typename T, bool RATES, int NW, int NM>
__global__ __launch_bounds__(64) void k_eph_epilogue(EphEpilogue e) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    constexpr int EPT = NW > 0 ? (NW * NW + 63) / 64 : 4;      // elements per lane
    constexpr int MM = NM > 0 ? NM : kMaxModes;
    const int nw = NW > 0 ? NW : e.nw, nm = NM > 0 ? NM : e.nm, nw2 = nw * nw, ng = nm * nw2;
    cx<T>* s_gw = reinterpret_cast<cx<T>*>(smem);           // [nm][nw][nw]
    cx<T>* s_u = s_gw + ng;                                  // [nw][nw]
    cx<T>* s_es = s_u + nw2;                                 // [nm][nm]
    double* s_d = reinterpret_cast<double*>(s_es + nm * nm); // nb[nm], om[nm], em[nw], fm[nw]
    double* s_nb = s_d;
    double* s_om = s_d + nm;
    double* s_em = s_d + 2 * nm;
    double* s_fm = s_d + 2 * nm + nw;
    const int z = blockIdx.y;
    const int blk = blockIdx.x;
    const int lane = threadIdx.x;
    const int q0 = blk * kQPB, q1 = min(e.nq, q0 + kQPB);
    const T* gwz = reinterpret_cast<const T*>(e.gw) + (long)z * e.nq * ng * 2;
    const double kt = kBoltzEv * e.temp;

    double acc[EPT][MM];
#pragma unroll
    for (int a = 0; a < EPT; ++a)
#pragma unroll
        for (int b = 0; b < MM; ++b) acc[a][b] = 0.0;
    double en[EPT];
#pragma unroll
    for (int t = 0; t < EPT; ++t) en[t] = 0.0;
    if (RATES)
#pragma unroll
        for (int t = 0; t < EPT; ++t) {
            const int el = lane + 64 * t;
            if (el < nw2) en[t] = e.ek[(long)z * nw + el % nw];
        }
    const T is = (T)(1.0 / e.sigma), nrm = (T)(1.0 / (sqrt(kPi) * e.sigma));

    // Per-pair inputs: with fixed sizes, the next pair's are loaded into
    // registers while the current pair is computed (one pair of prefetch), so
    // the loads' latency overlaps the arithmetic; the runtime-sized fallback
    // loads them in place.
    constexpr bool kPre = NW > 0 && NM > 0;
    constexpr int GPL = kPre ? (NM * NW * NW + 63) / 64 : 1;   // g' elements per lane
    constexpr int UPL = kPre ? (NW * NW + 63) / 64 : 1;        // U elements per lane
    constexpr int EPL = kPre ? (NM * NM + 63) / 64 : 1;        // e(q) elements per lane
    // (the fixed-size instances read the mode and Fermi factors formed once per
    // chunk; their launcher guarantees them)
    cx<T> rg[GPL], ru[UPL], res[EPL];
    double rom = 0.0, rem = 0.0, rnb = 0.0, rfm = 0.0;
    const cx<T>* esq = reinterpret_cast<const cx<T>*>(e.esq);
    auto fetch = [&](int ql) {
        const long qg = (long)e.q_off + ql;
        const long pair = (long)z * e.nq + ql;
        const T* gp = gwz + (long)ql * ng * 2;
        const double* uq = e.ukq + pair * nw2 * 2;
#pragma unroll
        for (int j = 0; j < GPL; ++j) {
            const int i = lane + 64 * j;
            if (i < ng) rg[j] = ld(gp, i);
        }
#pragma unroll
        for (int j = 0; j < UPL; ++j) {
            const int i = lane + 64 * j;
            if (i < nw2) ru[j] = ldd<T>(uq, e.u_cm ? (i % nw) * nw + i / nw : i);
        }
#pragma unroll
        for (int j = 0; j < EPL; ++j) {
            const int i = lane + 64 * j;
            if (i < nm * nm) res[j] = esq[(long)ql * nm * nm + i];
        }
        if (lane < nm) {
            rom = e.omega[qg * nm + lane];
            rnb = e.nbq[(long)ql * nm + lane];
        }
        if (RATES && lane < nw) {
            rem = e.ekq[pair * nw + lane];
            rfm = e.fkq[pair * nw + lane];
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int j = 0; j < GPL; ++j) {
            const int i = lane + 64 * j;
            if (i < ng) s_gw[i] = rg[j];
        }
#pragma unroll
        for (int j = 0; j < UPL; ++j) {
            const int i = lane + 64 * j;
            if (i < nw2) s_u[i] = ru[j];
        }
#pragma unroll
        for (int j = 0; j < EPL; ++j) {
            const int i = lane + 64 * j;
            if (i < nm * nm) s_es[i] = res[j];
        }
        if (lane < nm) {
            s_om[lane] = rom;
            s_nb[lane] = rnb;
        }
        if (RATES && lane < nw) {
            s_em[lane] = rem;
            s_fm[lane] = rfm;
        }
    };
    if (kPre && q0 < q1) fetch(q0);

    for (int ql = q0; ql < q1; ++ql) {
        const long qg = (long)e.q_off + ql;
        if constexpr (kPre) {
            stage();
            __syncthreads();
            if (ql + 1 < q1) fetch(ql + 1);
        } else {
            const long pair = (long)z * e.nq + ql;
            const T* gp = gwz + (long)ql * ng * 2;
            const double* uq = e.ukq + pair * nw2 * 2;
            for (int i = lane; i < ng; i += 64) s_gw[i] = ld(gp, i);
            for (int i = lane; i < nw2; i += 64) s_u[i] = ldd<T>(uq, e.u_cm ? (i % nw) * nw + i / nw : i);
            for (int i = lane; i < nm * nm; i += 64) {
                const int x = i / nm, nu = i % nm;
                const double om = e.omega[qg * nm + nu];
                const double amp = om > e.omega_cut ? sqrt(kHbar2AmuA2 / (2.0 * om)) * e.minv[x] : 0.0;
                s_es[i] = {(T)(amp * e.evec[2 * ((qg * nm + x) * nm + nu)]),
                           (T)(amp * e.evec[2 * ((qg * nm + x) * nm + nu) + 1])};
            }
            if (lane < nm) {
                const double om = e.omega[qg * nm + lane];
                s_om[lane] = om;
                s_nb[lane] = om > e.omega_cut ? 1.0 / expm1(om / kt) : 0.0;
            }
            if (RATES && lane < nw) {
                const double em = e.ekq[pair * nw + lane];
                s_em[lane] = em;
                s_fm[lane] = 1.0 / (exp((em - e.mu) / kt) + 1.0);
            }
            __syncthreads();
        }
        const double wq = RATES ? (e.qw ? e.qw[qg] : e.uniform_w) : 0.0;
#pragma unroll
        for (int t = 0; t < EPT; ++t) {
            const int el = lane + 64 * t;
            if (el >= nw2) break;
            const int m = el / nw, n = el % nw;
            cx<T> gh[MM];  // register-resident when NM is fixed
#pragma unroll
            for (int x = 0; x < MM; ++x) {
                cx<T> a = {0, 0};
                if (x < nm)
                    for (int i = 0; i < nw; ++i) cjfma(a, s_u[i * nw + m], s_gw[(x * nw + i) * nw + n]);
                gh[x] = a;
            }
            cx<T> ov = {0, 0};
            if (e.lr != nullptr) {
                // Wannier-gauge long-range term C(q) delta_ij, rotated: C(q) [U^dag(k+q) U(k)]_mn
                const double* ukz = e.uk + (long)z * nw2 * 2;
                for (int i = 0; i < nw; ++i) cjfma(ov, s_u[i * nw + m], ldd<T>(ukz, (long)i * nw + n));
#pragma unroll
                for (int x = 0; x < MM; ++x)
                    if (x < nm) cfma(gh[x], ldd<T>(e.lr, qg * nm + x), ov);
            }
            const double em = RATES ? s_em[m] : 0.0, fm = RATES ? s_fm[m] : 0.0;
#pragma unroll
            for (int nu = 0; nu < MM; ++nu) {
                if (nu >= nm) break;
                const double om = s_om[nu];
                cx<T> g = {0, 0};
#pragma unroll
                for (int x = 0; x < MM; ++x)
                    if (x < nm) cfma(g, s_es[x * nm + nu], gh[x]);
                T g2 = g.x * g.x + g.y * g.y;
                if (RATES && e.part != 0) {
                    // long-range coupling alone: g_L = (sum_x es[x][nu] C_x(q)) [U^dag(k+q) U(k)]_mn
                    cx<T> l = {0, 0};
#pragma unroll
                    for (int x = 0; x < MM; ++x)
                        if (x < nm) cfma(l, s_es[x * nm + nu], ldd<T>(e.lr, qg * nm + x));
                    const T gl2 = (l.x * l.x + l.y * l.y) * (ov.x * ov.x + ov.y * ov.y);
                    g2 = e.part == 1 ? gl2 : g2 - gl2;
                }
                if (!RATES) {
                    const long off = ((((long)(e.k_off + z) * e.nq_total + qg) * nm + nu) * nw + m) * nw + n;
                    reinterpret_cast<T*>(e.g2)[off] = om > e.omega_cut ? g2 : (T)0;
                } else if (om > e.omega_cut) {
                    const double nb = s_nb[nu];
                    const T x1 = (T)(en[t] - om - em) * is, x2 = (T)(en[t] + om - em) * is;
                    const T y1 = x1 * x1, y2 = x2 * x2;
                    T d_em, d_ab;
                    if constexpr (sizeof(T) == 4) {
                        // exp(-y) = 2^(-y log2 e) on the hardware exp2 (FP32 paths)
                        d_em = y1 > (T)200 ? (T)0 : nrm * __builtin_amdgcn_exp2f(-y1 * 1.4426950408889634f);
                        d_ab = y2 > (T)200 ? (T)0 : nrm * __builtin_amdgcn_exp2f(-y2 * 1.4426950408889634f);
                    } else {
                        d_em = y1 > (T)200 ? (T)0 : nrm * exp(-y1);
                        d_ab = y2 > (T)200 ? (T)0 : nrm * exp(-y2);
                    }
                    acc[t][nu] += wq * (double)g2 * ((double)d_em * (1.0 + nb - fm) + (double)d_ab * (nb + fm));
                }
            }
        }
        __syncthreads();
    }
    if (!RATES) return;
    // deterministic reduction over m: [element][nu] in LDS -> partial[z][blk][n][nu]
    double* red = reinterpret_cast<double*>(smem);
#pragma unroll
    for (int t = 0; t < EPT; ++t) {
        const int el = lane + 64 * t;
        if (el >= nw2) break;
#pragma unroll
        for (int nu = 0; nu < MM; ++nu)
            if (nu < nm) red[(long)el * nm + nu] = acc[t][nu];
    }
    __syncthreads();
    for (int o = lane; o < nw * nm; o += 64) {
        const int n = o / nm, nu = o % nm;
        double sum = 0.0;
        for (int m = 0; m < nw; ++m) sum += red[((long)m * nw + n) * nm + nu];
        e.partial[(((long)z * e.nblk + blk) * nw + n) * nm + nu] = sum * (2.0 * kPi / kHbarEvFs);
    }
}

// The rates epilogue of the FP32 paths for Nw = 8 bands and 6 modes on the
// matrix cores.  One wavefront walks kQPB pairs of one k; per pair
//   rotation   X[x][m][n] = sum_i conj(U_im(k+q)) g'[x][i][n]
// is a real 16 x 16 by 16 x 48 product (rows (m, re|im), contraction (i, re|im),
// columns (x, n)): 12 v_mfma_f32_16x16x4f32 with both operands loaded in
// operand layout (A from U(k+q), B from g'); X goes through LDS to the layout
//   projection g[nu][m][n] = sum_x es[x][nu] X[x][m][n]
// needs, a 12 x 12 by 12 x 64 real product (rows (nu, re|im), contraction
// (x, re|im), columns (m, n)): 12 more MFMAs (rows 12..15 zero).  Lane l then
// holds g for modes 2(l/16), 2(l/16)+1 at the columns (m, n), n = l%8, of
// its four column blocks, and forms |g|^2 and the Gaussian-weighted terms
// for its k-side band n; the lanes l, l^8 (the two halves of m) are summed in
// fixed order.  Same sums as k_eph_epilogue<float, true, 8, 6> (the products'
// rounding differs); no long-range term, no part selection.
// Each wavefront keeps kEpiDepth pairs' operands in flight in a register
// ring.  A pair's band and mode values (energies, Fermi and Bose factors,
// omega) reach the lanes through LDS: each lane loads one of them, converts
// it and writes it where the lanes that use it read it as one vector, so no
// lane selects among wavefront-uniform values.
constexpr int kEpiDepth = 2;   // with 2, three wavefronts fit a SIMD
static_assert(kQPB % kEpiDepth == 0, "whole ring turns per workgroup");

// LDS staging of a pair's band and mode values, in floats:
//   [0, 64)   eps_n(k) - eps_m(k+q) at ((m % 2) 8 + n) 4 + m / 2, so that lane
//             (m % 2, n) reads its four m = 2 cb + m % 2 as one float4
//   [64, 72)  f_m(k+q) at (m % 2) 4 + m / 2
//   [72, 78)  omega_nu; [78, 84) Bose factor n_nu; [84, 90) 1 if omega_nu is
//             above the cut, else 0 (lane group lg reads nu = 2 lg, 2 lg + 1)
//   95        written by lanes that carry no value
constexpr int kPsD = 0, kPsF = 64, kPsOm = 72, kPsNb = 78, kPsLive = 84, kPsDump = 95, kPsLen = 96;

// read-only, wavefront-uniform values through the constant address space:
// scalar loads, counted apart from the vector loads in flight
template <typename T>
__device__ __forceinline__ T ld_uniform(const T* p, long i) {
    return reinterpret_cast<const __attribute__((address_space(4))) T*>(reinterpret_cast<uintptr_t>(p))[i];
}

struct EpiOperands {
    float2 ga[3], gb[3];   // g'[2 cb + l%16/8][l/16 (+4)][l%8] (re, im)
    double2 ua, ub;        // U[l/16 (+4)][l%8] (re, im)
    float es[3];           // the one component of es[(4 ks + l/16)/2][l%16/2] lane l multiplies
    double em;             // eps_{l/8}(k+q)
    double sv;             // f_l(k+q) (l < 8), omega_{l-16} (16 <= l < 22), n_{l-24} (24 <= l < 30)
};

__global__ __launch_bounds__(64) void k_eph_rates_mfma(EphEpilogue e) {
    constexpr int NW = 8, NM = 6, GSZ = NM * NW * NW * 2;   // floats of one pair's g'
    constexpr int XLD = 65;                                 // LDS row stride of X
    __shared__ float xs[12 * XLD];
    __shared__ __align__(16) float ps[kPsLen];
    const int z = blockIdx.y, blk = blockIdx.x, lane = threadIdx.x;
    const int q0 = blk * kQPB, q1 = min(e.nq, q0 + kQPB);
    const int l16 = lane & 15, lg = lane >> 4;
    const int pm = l16 >> 3, n = l16 & 7;      // column parity bit, k-side band
    const int mr = l16 & 7;                    // rotation row: band m of row l16
    const bool ci_r = l16 >= 8;                // rotation row holds the imaginary part
    const int nup = l16 >> 1, co = l16 & 1;    // projection row: mode, re|im
    const bool rv = l16 < 12;
    const int ci = lg & 1;                     // projection contraction index: re|im of X
    const int nupc = min(nup, NM - 1);
    // projection operand: component co ^ ci of es, negated for (re row, im part)
    const int esc = co ^ ci;
    const float ess = co == 0 && ci == 1 ? -1.f : 1.f;
    const float* gwz = reinterpret_cast<const float*>(e.gw) + (long)z * e.nq * GSZ;
    const float* esq = reinterpret_cast<const float*>(e.esq);
    // staging roles: lane l forms eps_n(k) - eps_m(k+q) for m = l/8, n = l%8,
    // and carries one small value (see EpiOperands::sv)
    const int mst = lane >> 3;
    const int dst_d = kPsD + ((mst & 1) * 8 + n) * 4 + (mst >> 1);
    const double* svb;
    long svs;
    int dst_v;
    if (lane < 8) {
        svb = e.fkq + (long)z * e.nq * NW + lane;
        svs = NW;
        dst_v = kPsF + (lane & 1) * 4 + (lane >> 1);
    } else if (lane >= 16 && lane < 22) {
        svb = e.omega + (long)e.q_off * NM + (lane - 16);
        svs = NM;
        dst_v = kPsOm + lane - 16;
    } else if (lane >= 24 && lane < 30) {
        svb = e.nbq + (lane - 24);
        svs = NM;
        dst_v = kPsNb + lane - 24;
    } else {
        svb = e.fkq + (long)z * e.nq * NW + (lane & 7);
        svs = NW;
        dst_v = kPsDump;
    }
    const int dst_l = lane >= 16 && lane < 22 ? kPsLive + lane - 16 : kPsDump;
    const double en = e.ek[(long)z * NW + n];
    // U(k+q) entries (i, m) = (l/16 (+4), l%8) of lane l, in either stored layout
    const int ua_off = (e.u_cm ? mr * NW + lg : lg * NW + mr) * 2;
    const int ub_off = (e.u_cm ? mr * NW + 4 + lg : (4 + lg) * NW + mr) * 2;
    const float is = (float)(1.0 / e.sigma);
    double acc[2] = {0.0, 0.0};
    EpiOperands ring[kEpiDepth];
    // loads of pair ql (any pair of the block: past the last one they are
    // never used), unconditional so every pair waits only for its own
    auto fetch = [&](int ql, EpiOperands& o) {
        const float* gp = gwz + (long)ql * GSZ;
#pragma unroll
        for (int cb = 0; cb < 3; ++cb) {
            const int x = 2 * cb + pm;
            o.ga[cb] = *reinterpret_cast<const float2*>(gp + ((x * NW + lg) * NW + n) * 2);
            o.gb[cb] = *reinterpret_cast<const float2*>(gp + ((x * NW + 4 + lg) * NW + n) * 2);
        }
        const long pair = (long)z * e.nq + ql;
        const double* uq = e.ukq + pair * NW * NW * 2;
        o.ua = *reinterpret_cast<const double2*>(uq + ua_off);
        o.ub = *reinterpret_cast<const double2*>(uq + ub_off);
#pragma unroll
        for (int ks = 0; ks < 3; ++ks) o.es[ks] = esq[((long)ql * NM * NM + ((4 * ks + lg) >> 1) * NM + nupc) * 2 + esc];
        o.em = e.ekq[pair * NW + mst];
        o.sv = svb[(long)ql * svs];
    };
    auto pair_step = [&](int ql, EpiOperands& o) {
        // rotation from the ring slot, then the slot refilled (its values are
        // consumed by the issued products and the staging below)
        const float uar = (float)o.ua.x, uai = (float)o.ua.y, ubr = (float)o.ub.x, ubi = (float)o.ub.y;
        const float a[4] = {ci_r ? -uai : uar, ci_r ? -ubi : ubr, ci_r ? uar : uai, ci_r ? ubr : ubi};
        flt4 xr[3];
#pragma unroll
        for (int cb = 0; cb < 3; ++cb) {
            xr[cb] = flt4{0.f, 0.f, 0.f, 0.f};
            xr[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], o.ga[cb].x, xr[cb], 0, 0, 0);
            xr[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], o.gb[cb].x, xr[cb], 0, 0, 0);
            xr[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], o.ga[cb].y, xr[cb], 0, 0, 0);
            xr[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], o.gb[cb].y, xr[cb], 0, 0, 0);
        }
        float pa[3];
#pragma unroll
        for (int ks = 0; ks < 3; ++ks) pa[ks] = rv ? ess * o.es[ks] : 0.f;
        const float dv = (float)(en - o.em), sv = (float)o.sv, lv = o.sv > e.omega_cut ? 1.f : 0.f;
        fetch(min(ql + kEpiDepth, q1 - 1), o);
        if (ql >= q1) return;   // uniform: past the block's last pair
        const double wq = e.qw ? ld_uniform(e.qw, (long)e.q_off + ql) : e.uniform_w;
        // X[x][m][n] (re|im) to LDS as row 2x + (re|im), column 8m + n; element v
        // of lane l is row 4(l/16) + v of the rotation, i.e. m = (4 l/16 + v) % 8
        // and re|im = l/32
#pragma unroll
        for (int cb = 0; cb < 3; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 4 * lg + v;
                xs[(2 * (2 * cb + pm) + (r >> 3)) * XLD + 8 * (r & 7) + n] = xr[cb][v];
            }
        ps[dst_d] = dv;
        ps[dst_v] = sv;
        ps[dst_l] = lv;
        // the workgroup is one wavefront: its LDS writes are complete once its
        // LDS counter drains (a __syncthreads() here would also wait for the
        // loads in flight)
        __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        flt4 gr[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            gr[cb] = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 3; ++ks)
                gr[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(pa[ks], xs[(4 * ks + lg) * XLD + 16 * cb + l16], gr[cb], 0,
                                                              0, 0);
        }
        // element v of lane l: mode 2 (l/16) + v/2, re|im = v%2, column (m, n) =
        // (2 cb + l%16 / 8, l%8); lanes with l/16 = 3 hold the zero rows.
        // exp(-x^2) = 2^-(x sqrt(log2 e))^2; below 2^-126 it is zero or
        // subnormal, as the cut at (x/sigma)^2 > 200 of the FP64 path
        if (lg < 3) {
            const flt4 dm = *reinterpret_cast<const flt4*>(ps + kPsD + (pm * 8 + n) * 4);
            const flt4 fm = *reinterpret_cast<const flt4*>(ps + kPsF + pm * 4);
            const float2 om = *reinterpret_cast<const float2*>(ps + kPsOm + 2 * lg);
            const float2 nb = *reinterpret_cast<const float2*>(ps + kPsNb + 2 * lg);
            const float2 live = *reinterpret_cast<const float2*>(ps + kPsLive + 2 * lg);
            const float isl = is * 1.2011224087864498f;   // sqrt(log2 e) / sigma
            // arguments in units of sigma / sqrt(log2 e): x = dm' -+ om'
            float dms[4];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) dms[cb] = dm[cb] * isl;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if ((j ? live.y : live.x) == 0.f) continue;
                const float oms = (j ? om.y : om.x) * isl, nbj = j ? nb.y : nb.x;
                float t = 0.f;
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {
                    const float g2 = gr[cb][2 * j] * gr[cb][2 * j] + gr[cb][2 * j + 1] * gr[cb][2 * j + 1];
                    const float x1 = dms[cb] - oms, x2 = dms[cb] + oms;
                    const float d1 = __builtin_amdgcn_exp2f(-x1 * x1), d2 = __builtin_amdgcn_exp2f(-x2 * x2);
                    t += g2 * (d1 * (1.f + nbj - fm[cb]) + d2 * (nbj + fm[cb]));
                }
                acc[j] += wq * (double)t;
            }
        }
    };
    if (q0 < q1) {
#pragma unroll
        for (int j = 0; j < kEpiDepth; ++j) fetch(min(q0 + j, q1 - 1), ring[j]);
        for (int g0 = q0; g0 < q0 + kQPB; g0 += kEpiDepth) {
#pragma unroll
            for (int j = 0; j < kEpiDepth; ++j) pair_step(g0 + j, ring[j]);
        }
    }
    // the two halves of m (lanes l and l^8), then partial[z][blk][n][nu]
    const double nrm = 1.0 / (sqrt(kPi) * e.sigma);
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[j] += __shfl_xor(acc[j], 8, 64);
    if (pm == 0 && lg < 3)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            e.partial[(((long)z * e.nblk + blk) * NW + n) * NM + 2 * lg + j] = acc[j] * nrm * (2.0 * kPi / kHbarEvFs);
}

template <typename T, bool RATES>
void launch_epilogue(const EphEpilogue& e, dim3 grid, size_t lds, hipStream_t st) {
    // the fixed-size instances read the precomputed factors; without them the
    // runtime-sized instance forms them per pair
    const bool pre = e.esq != nullptr && e.nbq != nullptr && (!RATES || e.fkq != nullptr);
    if (!pre)
        hipLaunchKernelGGL((k_eph_epilogue<T, RATES, 0, 0>), grid, dim3(64), lds, st, e);
    else if (e.nw == 8 && e.nm == 6)
        hipLaunchKernelGGL((k_eph_epilogue<T, RATES, 8, 6>), grid, dim3(64), lds, st, e);
    else if (e.nw == 4 && e.nm == 6)
        hipLaunchKernelGGL((k_eph_epilogue<T, RATES, 4, 6>), grid, dim3(64), lds, st, e);
    else
        hipLaunchKernelGGL((k_eph_epilogue<T, RATES, 0, 0>), grid, dim3(64), lds, st, e);
}

template <typename T>
size_t epilogue_lds(int nw, int nm) {
    const size_t ng = (size_t)nm * nw * nw;
    const size_t stage = (ng + nw * nw + nm * nm) * 2 * sizeof(T) + (2 * nm + 2 * nw) * sizeof(double);
    const size_t red = (size_t)nw * nw * nm * sizeof(double);
    return stage > red ? stage : red;
}

// acc[z][o] += sum_b partial[z][b][o]: one 64-lane workgroup per (z, o), each lane a
// fixed strided subset, then a fixed shuffle tree (deterministic).
__global__ __launch_bounds__(64) void k_rates_reduce(int nblk, int nwm, const double* __restrict__ partial,
                                                     double* __restrict__ acc) {
    const int z = blockIdx.y, o = blockIdx.x, lane = threadIdx.x;
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += partial[((long)z * nblk + b) * nwm + o];
    for (int w = 32; w >= 1; w >>= 1) s += __shfl_xor(s, w, 64);
    if (lane == 0) acc[(long)z * nwm + o] += s;
}

__global__ void k_rates_finish(int nkb, int nw, int nm, const double* __restrict__ acc, double* __restrict__ gamma,
                               double* __restrict__ gmode) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nkb * nw) return;
    double s = 0.0;
    for (int nu = 0; nu < nm; ++nu) {
        const double v = acc[(long)t * nm + nu];
        s += v;
        if (gmode) gmode[(long)t * nm + nu] = v;
    }
    gamma[t] = s;
}

// Froehlich term, one thread per (q, kappa); loops over the G box.
__global__ void k_frohlich(int nq, const double* __restrict__ q, PolarDev p, double* __restrict__ lr) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nq * p.nat) return;
    const int iq = t / p.nat, kap = t % p.nat;
    double qr[3];
    for (int d = 0; d < 3; ++d) qr[d] = q[3 * iq + d] - rint(q[3 * iq + d]);
    double acc_re[3] = {0, 0, 0}, acc_im[3] = {0, 0, 0};
    for (int m0 = -p.mmax[0]; m0 <= p.mmax[0]; ++m0)
        for (int m1 = -p.mmax[1]; m1 <= p.mmax[1]; ++m1)
            for (int m2 = -p.mmax[2]; m2 <= p.mmax[2]; ++m2) {
                double v[3];
                for (int d = 0; d < 3; ++d)
                    v[d] = (qr[0] + m0) * p.bvec[d] + (qr[1] + m1) * p.bvec[3 + d] + (qr[2] + m2) * p.bvec[6 + d];
                const double nrm = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                if (!(nrm < p.gcut) || !(nrm > 1e-12)) continue;
                double qeq = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int b2 = 0; b2 < 3; ++b2) qeq += v[a] * p.eps[3 * a + b2] * v[b2];
                const double damp = exp(-qeq / (4.0 * p.alpha)) / qeq;
                const double arg = -(v[0] * p.tau[3 * kap] + v[1] * p.tau[3 * kap + 1] + v[2] * p.tau[3 * kap + 2]);
                double sn, cs;
                sincos(arg, &sn, &cs);
                for (int a = 0; a < 3; ++a) {
                    double qz = 0.0;
                    for (int b2 = 0; b2 < 3; ++b2) qz += v[b2] * p.zstar[(kap * 3 + b2) * 3 + a];
                    acc_re[a] += damp * cs * qz;
                    acc_im[a] += damp * sn * qz;
                }
            }
    for (int a = 0; a < 3; ++a) {
        // i * pref * (re + i im) = pref * (-im + i re)
        const long o = ((long)iq * 3 * p.nat + 3 * kap + a) * 2;
        lr[o] = -p.pref * acc_im[a];
        lr[o + 1] = p.pref * acc_re[a];
    }
}

// Dipole-dipole (LO-TO) part of D(q), added to the mass-scaled D(q) before the
// eigensolve.  One thread per (q, kappa, kappa') block:
//   D_{ka,k'b} += minv_ka minv_k'b pref [ sum_{G, q+G != 0, |q+G| < gcut}
//        [K.Z_k]_a [K.Z_k']_b e^{-K.eps.K/(4 Lambda)}/(K.eps.K) e^{i K.(tau_k - tau_k')}
//        - delta_kk' corr_k(a,b) ],  K = q + G, q brought to [-1/2,1/2)^3,
// with corr the q = 0 sum over G != 0 and all k'' (acoustic sum rule).
__global__ void k_dipole_add(int nq, const double* __restrict__ q, PolarDev p, const double* __restrict__ corr,
                             const double* __restrict__ minv, double* __restrict__ D) {
    const int nat = p.nat, nm = 3 * nat;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)nq * nat * nat) return;
    const int iq = (int)(t / (nat * nat)), k1 = (int)(t % (nat * nat)) / nat, k2 = (int)(t % nat);
    double qr[3];
    for (int d = 0; d < 3; ++d) qr[d] = q[3 * iq + d] - rint(q[3 * iq + d]);
    const double dt[3] = {p.tau[3 * k1] - p.tau[3 * k2], p.tau[3 * k1 + 1] - p.tau[3 * k2 + 1],
                          p.tau[3 * k1 + 2] - p.tau[3 * k2 + 2]};
    double are[9] = {0}, aim[9] = {0};
    for (int m0 = -p.mmax[0]; m0 <= p.mmax[0]; ++m0)
        for (int m1 = -p.mmax[1]; m1 <= p.mmax[1]; ++m1)
            for (int m2 = -p.mmax[2]; m2 <= p.mmax[2]; ++m2) {
                double v[3];
                for (int d = 0; d < 3; ++d)
                    v[d] = (qr[0] + m0) * p.bvec[d] + (qr[1] + m1) * p.bvec[3 + d] + (qr[2] + m2) * p.bvec[6 + d];
                const double nrm = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                if (!(nrm < p.gcut) || !(nrm > 1e-12)) continue;
                double kek = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int b2 = 0; b2 < 3; ++b2) kek += v[a] * p.eps[3 * a + b2] * v[b2];
                const double damp = exp(-kek / (4.0 * p.alpha)) / kek;
                double sn, cs;
                sincos(v[0] * dt[0] + v[1] * dt[1] + v[2] * dt[2], &sn, &cs);
                double z1[3], z2[3];
                for (int a = 0; a < 3; ++a) {
                    z1[a] = z2[a] = 0.0;
                    for (int b2 = 0; b2 < 3; ++b2) {
                        z1[a] += v[b2] * p.zstar[(k1 * 3 + b2) * 3 + a];
                        z2[a] += v[b2] * p.zstar[(k2 * 3 + b2) * 3 + a];
                    }
                }
                for (int a = 0; a < 3; ++a)
                    for (int b2 = 0; b2 < 3; ++b2) {
                        const double w = damp * z1[a] * z2[b2];
                        are[3 * a + b2] += w * cs;
                        aim[3 * a + b2] += w * sn;
                    }
            }
    double* dq = D + (long)iq * nm * nm * 2;
    for (int a = 0; a < 3; ++a)
        for (int b2 = 0; b2 < 3; ++b2) {
            double re = are[3 * a + b2], im = aim[3 * a + b2];
            if (k1 == k2) {
                re -= corr[2 * ((k1 * 3 + a) * 3 + b2)];
                im -= corr[2 * ((k1 * 3 + a) * 3 + b2) + 1];
            }
            const int r = 3 * k1 + a, c = 3 * k2 + b2;
            const double s = p.pref * minv[r] * minv[c];
            dq[2 * ((long)r * nm + c)] += s * re;
            dq[2 * ((long)r * nm + c) + 1] += s * im;
        }
}

// Velocities: one thread per (k, alpha).  M = U^dag dH_a U restricted to
// degenerate groups; the group block is diagonalised by a serial cyclic
// Jacobi (group blocks are tiny), eigenvalues sorted ascending in the group.
__global__ void k_band_velocity(int nk, int nw, const double* __restrict__ dh, const double* __restrict__ u,
                                const double* __restrict__ eps, double* __restrict__ vel) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nk * 3) return;
    const int ik = t / 3, a = t % 3;
    const int nw2 = nw * nw;
    const double* uk = u + (long)ik * nw2 * 2;
    const double* hk = dh + ((long)ik * 3 + a) * nw2 * 2;
    const double* ek = eps + (long)ik * nw;
    cx<double> mm[kMaxNw * kMaxNw];
    // M_mn = sum_ij conj(U_im) dH_ij U_jn, only inside degenerate groups
    int grp[kMaxNw];
    int g = 0;
    for (int m = 0; m < nw; ++m) {
        if (m > 0 && !(ek[m] - ek[m - 1] < kDegTol)) ++g;
        grp[m] = g;
    }
    for (int m = 0; m < nw; ++m)
        for (int n = 0; n < nw; ++n) {
            cx<double> s = {0.0, 0.0};
            if (grp[m] == grp[n]) {
                for (int i = 0; i < nw; ++i) {
                    cx<double> r = {0.0, 0.0};
                    for (int j = 0; j < nw; ++j) cfma(r, ld(hk, (long)i * nw + j), ld(uk, (long)j * nw + n));
                    cjfma(s, ld(uk, (long)i * nw + m), r);
                }
            }
            mm[m * nw + n] = s;
        }
    // Jacobi sweeps on the block-diagonal matrix (cross-group entries stay zero)
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int m = 0; m < nw; ++m)
            for (int n = 0; n < nw; ++n) {
                const double v2 = mm[m * nw + n].x * mm[m * nw + n].x + mm[m * nw + n].y * mm[m * nw + n].y;
                tot += v2;
                if (m != n) off += v2;
            }
        if (!(off > 1e-30 * tot)) break;
        for (int p = 0; p < nw; ++p)
            for (int q = p + 1; q < nw; ++q) {
                if (grp[p] != grp[q]) continue;
                const cx<double> apq = mm[p * nw + q];
                const double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
                if (!(mag > 0.0)) continue;
                const double th = (mm[q * nw + q].x - mm[p * nw + p].x) / (2.0 * mag);
                const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
                const cx<double> ep = {apq.x / mag, apq.y / mag};
                // columns: A <- A J, J_pq = s e, J_qp = -s conj(e)
                for (int r = 0; r < nw; ++r) {
                    const cx<double> arp = mm[r * nw + p], arq = mm[r * nw + q];
                    // new col p = c*arp + arq*(-s conj(e)); new col q = arp*(s e) + c*arq
                    mm[r * nw + p] = {c * arp.x - s * (arq.x * ep.x + arq.y * ep.y), c * arp.y - s * (arq.y * ep.x - arq.x * ep.y)};
                    mm[r * nw + q] = {c * arq.x + s * (arp.x * ep.x - arp.y * ep.y), c * arq.y + s * (arp.x * ep.y + arp.y * ep.x)};
                }
                // rows: A <- J^dag A
                for (int r = 0; r < nw; ++r) {
                    const cx<double> apr = mm[p * nw + r], aqr = mm[q * nw + r];
                    // new row p = c*apr + conj(-s conj(e)) aqr = c apr - s e aqr
                    // new row q = conj(s e) apr + c aqr
                    mm[p * nw + r] = {c * apr.x - s * (ep.x * aqr.x - ep.y * aqr.y), c * apr.y - s * (ep.x * aqr.y + ep.y * aqr.x)};
                    mm[q * nw + r] = {c * aqr.x + s * (ep.x * apr.x + ep.y * apr.y), c * aqr.y + s * (ep.x * apr.y - ep.y * apr.x)};
                }
            }
    }
    // ascending order inside each group
    double d[kMaxNw];
    for (int m = 0; m < nw; ++m) d[m] = mm[m * nw + m].x;
    for (int m = 0; m < nw; ++m)
        for (int n = m + 1; n < nw && grp[n] == grp[m]; ++n)
            if (d[n] < d[m]) {
                const double tmp = d[m];
                d[m] = d[n];
                d[n] = tmp;
            }
    for (int m = 0; m < nw; ++m) vel[((long)ik * nw + m) * 3 + a] = d[m] / kHbarEvFs;
}

}  // namespace

void apply_u_right(int Z, int nrp, int nm, int nw, const double* g, const double* u, double* out, hipStream_t st) {
    const long per = (long)nrp * nm * nw * nw;
    if (nw > 16) {
        // large models: Z x nrp x nm products of nw x nw blocks with U(k) on
        // the matrix cores (U shared by the blocks of one k)
        CBatch b{};
        b.n1 = (long)nrp * nm;
        b.sa0 = per;
        b.sa1 = (long)nw * nw;
        b.sb0 = (long)nw * nw;
        b.sb1 = 0;
        b.sc0 = per;
        b.sc1 = (long)nw * nw;
        cgemm_f64_batched(nw, nw, nw, (long)Z * nrp * nm, b, g, nw, u, nw, out, nw, st);
        return;
    }
    hipLaunchKernelGGL(k_apply_u_right, dim3((unsigned)((per + 255) / 256), Z), dim3(256), 0, st, nrp, nm, nw, g, u, out);
    check_launch("apply_u_right");
}

void apply_u_column(int Z, int nrp, int nm, int nw, const double* g, const double* us, const int32_t* band,
                    double* out, hipStream_t st) {
    const long per = (long)nrp * nm * nw;
    hipLaunchKernelGGL(k_apply_u_column, dim3((unsigned)((per + 255) / 256), Z), dim3(256), 0, st, nrp, nm, nw, g,
                       us, band, out);
    check_launch("apply_u_column");
}

void apply_u_right_adj(int Z, int nrp, int nm, int nw, const double* g, const double* u, double* out, hipStream_t st) {
    const long per = (long)nrp * nm * nw * nw;
    hipLaunchKernelGGL(k_apply_u_right_adj, dim3((unsigned)((per + 255) / 256), Z), dim3(256), 0, st, nrp, nm, nw, g, u,
                       out);
    check_launch("apply_u_right_adj");
}

void eph_adjoint_epilogue(const EphEpilogue& e, const double* lam, double* gw_bar, hipStream_t st) {
    dim3 grid(eph_epilogue_blocks(e.nq), e.nkb);
    const size_t ng = (size_t)e.nm * e.nw * e.nw;
    const size_t lds = (2 * ng + e.nw * e.nw + e.nm * e.nm) * 16 + (2 * e.nm + 2 * e.nw) * 8;
    if (lds > 65536) throw Error{-6, "rates_vjp: nw^2 * 3nat too large for one workgroup's staging buffer"};
    hipLaunchKernelGGL(k_eph_adjoint, grid, dim3(64), lds, st, e, lam, gw_bar);
    check_launch("eph_adjoint_epilogue");
}

namespace {
__global__ void k_add_into(long n, const double* __restrict__ src, double* __restrict__ dst) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) dst[t] += src[t];
}
}  // namespace

void add_into(long n, const double* src, double* dst, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_add_into, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, src, dst);
    check_launch("add_into");
}

void scale_rows(long rows, long cols, const double* w, double* data, hipStream_t st) {
    const long n = rows * cols;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scale_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rows, cols, w, data);
    check_launch("scale_rows");
}

void g_row_bound(int n_re, long rows, int nw, const double* g, const double* w, long rows_per_rp, int n_rp,
                 unsigned long long* out, hipStream_t st) {
    if (hipMemsetAsync(out, 0, 2 * sizeof(unsigned long long), st) != hipSuccess)
        throw Error{-3, "g_row_bound: hipMemsetAsync failed"};
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_g_row_bound<double>, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, n_re, rows, nw,
                       g, w, rows_per_rp, n_rp, out);
    check_launch("g_row_bound");
}

void g_row_bound_f32(int n_re, long rows, int nw, const float* g, unsigned long long* out, hipStream_t st) {
    if (hipMemsetAsync(out, 0, 2 * sizeof(unsigned long long), st) != hipSuccess)
        throw Error{-3, "g_row_bound: hipMemsetAsync failed"};
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_g_row_bound<float>, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, n_re, rows, nw,
                       g, (const double*)nullptr, 1L, 1, out);
    check_launch("g_row_bound");
}

void gen_coupling(int n_re, int n_rp, long per, unsigned long long seed, const double* env, float* out,
                  hipStream_t st) {
    const long n = (long)n_re * n_rp * per;
    if (n <= 0) return;
    const long blocks = std::min<long>((n + 255) / 256, 1L << 20);
    hipLaunchKernelGGL(k_gen_coupling, dim3((unsigned)blocks), dim3(256), 0, st, n, per, n_rp, seed, env, out);
    check_launch("gen_coupling");
}

void convert_f64_f32(long count, const double* in, float* out, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_convert, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, in, out);
    check_launch("convert");
}

int eph_epilogue_blocks(int nq) { return (nq + kQPB - 1) / kQPB; }

namespace {
__global__ void k_gather_points(int n, const int32_t* __restrict__ idx, const double* __restrict__ src,
                                double* __restrict__ dst) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const long i = idx[j];
    dst[3L * j] = src[3 * i];
    dst[3L * j + 1] = src[3 * i + 1];
    dst[3L * j + 2] = src[3 * i + 2];
}

__global__ void k_scatter_blocks(int n, const int32_t* __restrict__ pos, const uint32_t* __restrict__ src,
                                 uint32_t* __restrict__ dst, long words) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * words) return;
    const long j = e / words, w = e % words;
    dst[(long)pos[j] * words + w] = src[e];
}
}  // namespace

void gather_points(int n, const int32_t* idx, const double* src, double* dst, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_points, dim3((n + 255) / 256), dim3(256), 0, st, n, idx, src, dst);
    check_launch("gather_points");
}

void scatter_blocks(int n, const int32_t* pos, const void* src, void* dst, long words, hipStream_t st) {
    if (n <= 0 || words <= 0) return;
    const long total = (long)n * words;
    if ((total + 255) / 256 > 0x7fffffffL) throw Error{-1, "scatter_blocks: too large"};
    hipLaunchKernelGGL(k_scatter_blocks, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, n, pos,
                       (const uint32_t*)src, (uint32_t*)dst, words);
    check_launch("scatter_blocks");
}

void eph_epilogue_g2(const EphEpilogue& e, int f32, hipStream_t st) {
    dim3 grid(eph_epilogue_blocks(e.nq), e.nkb);
    const size_t lds = f32 ? epilogue_lds<float>(e.nw, e.nm) : epilogue_lds<double>(e.nw, e.nm);
    if (lds > 65536) throw Error{-6, "gkq: nw^2 * 3nat too large for one workgroup's staging buffer"};
    if (f32) launch_epilogue<float, false>(e, grid, lds, st);
    else launch_epilogue<double, false>(e, grid, lds, st);
    check_launch("eph_epilogue_g2");
}

void eph_epilogue_factors(const EphEpilogue& e, int f32, void* esq, double* nbq, double* fkq, hipStream_t st) {
    const long n = (long)e.nq * e.nm * e.nm;
    if (n > 0) {
        const dim3 grid((unsigned)((n + 255) / 256));
        if (f32)
            hipLaunchKernelGGL(k_mode_factors<float>, grid, dim3(256), 0, st, e.nq, e.q_off, e.nm, e.omega, e.evec,
                               e.minv, e.omega_cut, e.temp, (cx<float>*)esq, nbq);
        else
            hipLaunchKernelGGL(k_mode_factors<double>, grid, dim3(256), 0, st, e.nq, e.q_off, e.nm, e.omega, e.evec,
                               e.minv, e.omega_cut, e.temp, (cx<double>*)esq, nbq);
    }
    const long nf = (long)e.nkb * e.nq * e.nw;
    if (fkq != nullptr && nf > 0)
        hipLaunchKernelGGL(k_fermi_factors, dim3((unsigned)((nf + 255) / 256)), dim3(256), 0, st, nf, e.ekq, e.mu,
                           e.temp, fkq);
    check_launch("eph_epilogue_factors");
}

void eph_epilogue_rates(const EphEpilogue& e, int f32, hipStream_t st) {
    dim3 grid(eph_epilogue_blocks(e.nq), e.nkb);
    if (f32 && e.nw == 8 && e.nm == 6 && e.lr == nullptr && e.part == 0 && e.esq != nullptr && e.nbq != nullptr &&
        e.fkq != nullptr) {
        hipLaunchKernelGGL(k_eph_rates_mfma, grid, dim3(64), 0, st, e);
        check_launch("eph_epilogue_rates");
        return;
    }
    const size_t lds = f32 ? epilogue_lds<float>(e.nw, e.nm) : epilogue_lds<double>(e.nw, e.nm);
    if (lds > 65536) throw Error{-6, "rates: nw^2 * 3nat too large for one workgroup's staging buffer"};
    if (f32) launch_epilogue<float, true>(e, grid, lds, st);
    else launch_epilogue<double, true>(e, grid, lds, st);
    check_launch("eph_epilogue_rates");
}

void rates_reduce(int nkb, int nblk, int nw, int nm, const double* partial, double* acc, hipStream_t st) {
    hipLaunchKernelGGL(k_rates_reduce, dim3(nw * nm, nkb), dim3(64), 0, st, nblk, nw * nm, partial, acc);
    check_launch("rates_reduce");
}

void rates_finish(int nkb, int nw, int nm, const double* acc, double* gamma, double* gmode, hipStream_t st) {
    const int n = nkb * nw;
    hipLaunchKernelGGL(k_rates_finish, dim3((n + 127) / 128), dim3(128), 0, st, nkb, nw, nm, acc, gamma, gmode);
    check_launch("rates_finish");
}

void dipole_add(int nq, const double* q, const PolarDev& p, const double* corr, const double* minv, double* D,
                hipStream_t st) {
    const long n = (long)nq * p.nat * p.nat;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_dipole_add, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, nq, q, p, corr, minv, D);
    check_launch("dipole_add");
}

void frohlich(int nq, const double* q, const PolarDev& p, double* lr, hipStream_t st) {
    const int n = nq * p.nat;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_frohlich, dim3((n + 127) / 128), dim3(128), 0, st, nq, q, p, lr);
    check_launch("frohlich");
}

void band_velocity(int nk, int nw, const double* dh, const double* u, const double* eps, double* vel, hipStream_t st) {
    const int n = nk * 3;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_band_velocity, dim3((n + 63) / 64), dim3(64), 0, st, nk, nw, dh, u, eps, vel);
    check_launch("band_velocity");
}

}  // namespace ephx
