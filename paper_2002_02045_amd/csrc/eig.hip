// Batched Hermitian eigensolver in FP64 for the small matrices of the method:
// H(k) and H(k+q) (n = Nw, Eq. wannier_3) and D(q) (n = 3 nat, Eq. IFC2).
//
// Cyclic Jacobi with the round-robin (tournament) ordering, so each round
// applies n/2 disjoint plane rotations at once (Golub & Van Loan, "Matrix
// Computations", Sec. 8.5, in its complex Hermitian form).  For a pair (p, q)
// with a_pq = |a_pq| e^{i phi}:
//   th = (a_qq - a_pp)/(2|a_pq|), t = sgn(th)/(|th| + sqrt(th^2 + 1)),
//   c = 1/sqrt(1 + t^2), s = t c, J_pq = s e^{i phi}, J_qp = -s e^{-i phi},
// and A <- J^dag A J, V <- V J.
//
// Layout: one lane per matrix row, R = 2^ceil(log2 n) lanes per matrix, so a
// 64-lane wavefront works on 64/R matrices at once.  Column rotations (A J,
// V J) act inside a lane's own row; row rotations (J^dag A) take the partner
// row with cross-lane shuffles.  The matrix order n is a template parameter,
// which unrolls every round of the tournament into register code.  Sweeps
// run until the off-diagonal Frobenius norm of every matrix in the wavefront
// is below 1e-15 of its norm; eigenpairs are then sorted ascending.
#include "internal.h"

namespace ephx {
namespace {

template <int NE>
__device__ __forceinline__ int rr_partner(int idx, int r) {
    // circle method: position 0 fixed, the others rotate by r each round
    constexpr int m = NE - 1;
    const int pos = idx == 0 ? 0 : ((idx - 1 - r) % m + m) % m + 1;
    const int pp = NE - 1 - pos;
    return pp == 0 ? 0 : (pp - 1 + r) % m + 1;
}

__device__ __forceinline__ double shfl(double v, int src) { return __shfl(v, src, 64); }

template <typename Tin, int N>
__global__ __launch_bounds__(256) void k_eig_rows(int batch, const Tin* __restrict__ A, long strideA,
                                                  double* __restrict__ evals, double* __restrict__ evecs) {
    constexpr int R = N <= 1 ? 1 : (N <= 2 ? 2 : (N <= 4 ? 4 : 8));
    constexpr int NE = N + (N & 1);
    const int lane = threadIdx.x & 63;
    const long slot = ((long)blockIdx.x * 256 + threadIdx.x) / R;
    const int i = lane % R;
    const int base = lane - i;
    const bool valid = slot < batch;
    const bool act = valid && i < N;
    double ar[N], ai[N], vr[N], vi[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        ar[j] = ai[j] = vi[j] = 0.0;
        vr[j] = (j == i) ? 1.0 : 0.0;
    }
    if (act) {
        const Tin* ab = A + slot * strideA * 2;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            // Hermitian part 0.5 (A + A^dag)
            const double xr = (double)ab[2 * (i * N + j)], xi = (double)ab[2 * (i * N + j) + 1];
            const double yr = (double)ab[2 * (j * N + i)], yi = (double)ab[2 * (j * N + i) + 1];
            ar[j] = 0.5 * (xr + yr);
            ai[j] = 0.5 * (xi - yi);
        }
    }
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, tot = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const double m2 = ar[j] * ar[j] + ai[j] * ai[j];
            tot += m2;
            off += (j != i) ? m2 : 0.0;
        }
#pragma unroll
        for (int w = R / 2; w >= 1; w >>= 1) {
            off += __shfl_xor(off, w, 64);
            tot += __shfl_xor(tot, w, 64);
        }
        const bool done = !(off > 1e-30 * tot);
        if (__all(done)) break;
#pragma unroll
        for (int r = 0; r < NE - 1; ++r) {
            const int p = i < NE ? rr_partner<NE>(i, r) : i;
            // rotation of the pair (i, p), computed by its lower lane
            double dself = 0.0, apr = 0.0, api = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                dself = (j == i) ? ar[j] : dself;
                apr = (j == p) ? ar[j] : apr;
                api = (j == p) ? ai[j] : api;
            }
            const double dpart = shfl(dself, base + (p < R ? p : i));
            double c = 1.0, ser = 0.0, sei = 0.0;   // se = s e^{i phi}
            if (i < p && p < N) {
                const double mag = sqrt(apr * apr + api * api);
                if (mag > 0.0) {
                    const double th = (dpart - dself) / (2.0 * mag);
                    const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                    c = 1.0 / sqrt(t * t + 1.0);
                    const double s = t * c;
                    ser = s * apr / mag;
                    sei = s * api / mag;
                }
            }
            // column rotations A J and V J, every pair of the round (indices are compile-time)
#pragma unroll
            for (int p0 = 0; p0 < N; ++p0) {
                const int q0 = rr_partner<NE>(p0, r);
                if (!(p0 < q0 && q0 < N)) continue;
                const double cc = shfl(c, base + p0), sr = shfl(ser, base + p0), si = shfl(sei, base + p0);
                // (AJ)_{.p} = c A_.p - conj(se) A_.q ; (AJ)_{.q} = se A_.p + c A_.q
                const double xr = ar[p0], xi = ai[p0], yr = ar[q0], yi = ai[q0];
                ar[p0] = cc * xr - (sr * yr + si * yi);
                ai[p0] = cc * xi - (sr * yi - si * yr);
                ar[q0] = (sr * xr - si * xi) + cc * yr;
                ai[q0] = (sr * xi + si * xr) + cc * yi;
                const double ur = vr[p0], ui = vi[p0], wr = vr[q0], wi = vi[q0];
                vr[p0] = cc * ur - (sr * wr + si * wi);
                vi[p0] = cc * ui - (sr * wi - si * wr);
                vr[q0] = (sr * ur - si * ui) + cc * wr;
                vi[q0] = (sr * ui + si * ur) + cc * wi;
            }
            // row rotation J^dag A with the partner row
            const int lo = i < p ? i : p;
            const double co = shfl(c, base + (lo < R ? lo : i));
            const double sro = shfl(ser, base + (lo < R ? lo : i));
            const double sio = shfl(sei, base + (lo < R ? lo : i));
            const int src = base + (p < R ? p : i);
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const double qr = shfl(ar[j], src), qi = shfl(ai[j], src);
                if (p < N && p != i) {
                    if (i < p) {
                        // (J^dag A)_{p.} = c A_p. - se A_q.
                        const double nr = co * ar[j] - (sro * qr - sio * qi);
                        const double ni = co * ai[j] - (sro * qi + sio * qr);
                        ar[j] = nr;
                        ai[j] = ni;
                    } else {
                        // (J^dag A)_{q.} = conj(se) A_p. + c A_q.
                        const double nr = (sro * qr + sio * qi) + co * ar[j];
                        const double ni = (sro * qi - sio * qr) + co * ai[j];
                        ar[j] = nr;
                        ai[j] = ni;
                    }
                }
            }
        }
    }
    // sort ascending, ties by index
    double d = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) d = (j == i) ? ar[j] : d;
    int rk = 0;
#pragma unroll
    for (int m = 0; m < N; ++m) {
        const double dm = shfl(d, base + m);
        rk += (dm < d || (dm == d && m < i)) ? 1 : 0;
    }
    if (act) evals[slot * N + rk] = d;
    if (evecs != nullptr) {
#pragma unroll
        for (int c2 = 0; c2 < N; ++c2) {
            const int rc = __shfl(rk, base + c2, 64);
            if (act) {
                const long off = ((slot * N + i) * N + rc) * 2;
                evecs[off] = vr[c2];
                evecs[off + 1] = vi[c2];
            }
        }
    }
}

__global__ void k_phonon_omega(long count, double* lam) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const double w2 = kHbar2AmuA2 * lam[t];
    lam[t] = (w2 >= 0.0 ? 1.0 : -1.0) * sqrt(fabs(w2));
}

template <typename Tin>
void launch_eig(int batch, int n, const Tin* A, long strideA, double* evals, double* evecs, hipStream_t st) {
    const int R = n <= 1 ? 1 : (n <= 2 ? 2 : (n <= 4 ? 4 : 8));
    const long threads = (long)batch * R;
    dim3 grid((unsigned)((threads + 255) / 256));
    switch (n) {
#define EPHX_EIG_CASE(NN) \
    case NN: hipLaunchKernelGGL((k_eig_rows<Tin, NN>), grid, dim3(256), 0, st, batch, A, strideA, evals, evecs); break;
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

void eig_herm(int batch, int n, const void* A, int a_f32, long strideA, double* evals, double* evecs,
              hipStream_t st) {
    if (batch <= 0) return;
    if (n < 1 || n > kEigMax) throw Error{-6, "eig_herm: matrix order above 8 is not supported in this build"};
    if (a_f32)
        launch_eig(batch, n, (const float*)A, strideA, evals, evecs, st);
    else
        launch_eig(batch, n, (const double*)A, strideA, evals, evecs, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{-3, std::string("eig_herm: ") + hipGetErrorString(e)};
}

void phonon_omega(long count, double* lam, hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_phonon_omega, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, count, lam);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{-3, std::string("phonon_omega: ") + hipGetErrorString(e)};
}

}  // namespace ephx
