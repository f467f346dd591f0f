// Batched Hermitian eigensolver in FP64 for the small matrices of the method:
// H(k) and H(k+q) (n = Nw, Eq. wannier_3) and D(q) (n = 3 nat, Eq. IFC2).
//
// One 64-lane wavefront owns one matrix (n <= 8, lane = matrix element
// (i, j)).  Cyclic Jacobi with the round-robin (tournament) ordering applies
// n/2 disjoint plane rotations at once, so every lane updates its element from
// four entries of the previous iterate:
//   A'_ij = a_i a_j A_ij + a_i b_j A_ij' + conj(b_i) a_j A_i'j + conj(b_i) b_j A_i'j'
//   V'_ij = a_j V_ij + b_j V_ij'
// where j' is the partner of j in the current round and column j of the
// rotation is (a_j at row j, b_j at row j').  A pair (p, q) with a_pq =
// |a_pq| e^{i phi} uses t = sgn(th)/(|th| + sqrt(th^2+1)), th = (a_qq - a_pp)/(2|a_pq|),
// c = 1/sqrt(1+t^2), s = t c, J_pq = s e^{i phi}, J_qp = -s e^{-i phi} (Golub & Van Loan,
// "Matrix Computations", Sec. 8.5, in its complex Hermitian form).  Sweeps run
// until the off-diagonal Frobenius norm is below 1e-15 of the total, then the
// eigenpairs are sorted ascending.
#include "internal.h"

namespace ephx {
namespace {

__device__ __forceinline__ int rr_partner(int idx, int r, int ne) {
    // circle method: position 0 fixed, the others rotate by r each round
    const int m = ne - 1;
    int pos;
    if (idx == 0) pos = 0;
    else pos = ((idx - 1 - r) % m + m) % m + 1;
    const int pp = ne - 1 - pos;
    if (pp == 0) return 0;
    return (pp - 1 + r) % m + 1;
}

struct cplx {
    double x, y;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ cplx cconj(cplx a) { return {a.x, -a.y}; }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cplx cscale(double s, cplx a) { return {s * a.x, s * a.y}; }

template <typename Tin>
__global__ __launch_bounds__(64) void k_eig_herm(int batch, int n, const Tin* __restrict__ A, long strideA,
                                                 double* __restrict__ evals, double* __restrict__ evecs) {
    __shared__ cplx a[64];
    __shared__ cplx v[64];
    __shared__ double ra[kEigMax + 1];
    __shared__ cplx rb[kEigMax + 1];
    __shared__ int rank[kEigMax];
    const int b = blockIdx.x;
    if (b >= batch) return;
    const int l = threadIdx.x;
    const int nn = n * n;
    const bool act = l < nn;
    const int i = act ? l / n : 0, j = act ? l % n : 0;
    const Tin* ab = A + (long)b * strideA * 2;
    if (act) {
        // Hermitian part 0.5 (A + A^dag)
        const double xr = (double)ab[2 * (i * n + j)], xi = (double)ab[2 * (i * n + j) + 1];
        const double yr = (double)ab[2 * (j * n + i)], yi = (double)ab[2 * (j * n + i) + 1];
        a[l] = {0.5 * (xr + yr), 0.5 * (xi - yi)};
        v[l] = {i == j ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
    const int ne = n + (n & 1);
    for (int sweep = 0; sweep < 30; ++sweep) {
        // convergence test on the current iterate
        double off = 0.0, tot = 0.0;
        if (act) {
            const double m2 = a[l].x * a[l].x + a[l].y * a[l].y;
            tot = m2;
            off = (i != j) ? m2 : 0.0;
        }
        for (int w = 32; w >= 1; w >>= 1) {
            off += __shfl_xor(off, w, 64);
            tot += __shfl_xor(tot, w, 64);
        }
        if (!(off > 1e-30 * tot)) break;
        for (int r = 0; r < ne - 1; ++r) {
            if (l < ne) {
                ra[l] = 1.0;
                rb[l] = {0.0, 0.0};
            }
            __syncthreads();
            if (act && i < j && rr_partner(i, r, ne) == j) {
                const cplx apq = a[i * n + j];
                const double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
                if (mag > 0.0) {
                    const double th = (a[j * n + j].x - a[i * n + i].x) / (2.0 * mag);
                    const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                    const double c = 1.0 / sqrt(t * t + 1.0);
                    const double s = t * c;
                    const cplx e = {apq.x / mag, apq.y / mag};
                    ra[i] = c;
                    ra[j] = c;
                    rb[i] = cscale(-s, cconj(e));   // J_{j,i}: row j of column i
                    rb[j] = cscale(s, e);           // J_{i,j}: row i of column j
                }
            }
            __syncthreads();
            cplx na = {0, 0}, nv = {0, 0};
            if (act) {
                const int ip = rr_partner(i, r, ne), jp = rr_partner(j, r, ne);
                const double ai = ra[i], aj = ra[j];
                const cplx bi = rb[i], bj = rb[j];
                na = cscale(ai * aj, a[i * n + j]);
                if (jp < n) na = cadd(na, cscale(ai, cmul(a[i * n + jp], bj)));
                if (ip < n) na = cadd(na, cscale(aj, cmul(cconj(bi), a[ip * n + j])));
                if (ip < n && jp < n) na = cadd(na, cmul(cmul(cconj(bi), a[ip * n + jp]), bj));
                nv = cscale(aj, v[i * n + j]);
                if (jp < n) nv = cadd(nv, cmul(v[i * n + jp], bj));
            }
            __syncthreads();
            if (act) {
                a[l] = na;
                v[l] = nv;
            }
            __syncthreads();
        }
    }
    // sort ascending, ties by index
    if (l < n) {
        const double d = a[l * n + l].x;
        int rk = 0;
        for (int m = 0; m < n; ++m) {
            const double dm = a[m * n + m].x;
            rk += (dm < d || (dm == d && m < l)) ? 1 : 0;
        }
        rank[l] = rk;
        evals[(long)b * n + rk] = d;
    }
    __syncthreads();
    if (evecs != nullptr && act) {
        const long off = ((long)b * nn + i * n + rank[j]) * 2;
        evecs[off] = v[l].x;
        evecs[off + 1] = v[l].y;
    }
}

__global__ void k_phonon_omega(long count, double* lam) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const double w2 = kHbar2AmuA2 * lam[t];
    lam[t] = (w2 >= 0.0 ? 1.0 : -1.0) * sqrt(fabs(w2));
}

}  // namespace

void eig_herm(int batch, int n, const void* A, int a_f32, long strideA, double* evals, double* evecs,
              hipStream_t st) {
    if (batch <= 0) return;
    if (n < 1 || n > kEigMax) throw Error{-6, "eig_herm: matrix order above 8 is not supported in this build"};
    if (a_f32)
        hipLaunchKernelGGL(k_eig_herm<float>, dim3(batch), dim3(64), 0, st, batch, n, (const float*)A, strideA,
                           evals, evecs);
    else
        hipLaunchKernelGGL(k_eig_herm<double>, dim3(batch), dim3(64), 0, st, batch, n, (const double*)A,
                           strideA, evals, evecs);
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
