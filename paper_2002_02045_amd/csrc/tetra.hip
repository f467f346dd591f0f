// Linear tetrahedron integration over the window states of a grid (paper
// Sec. 4.3; Bloechl, PRB 49, 16223 (1994)): the transport distribution
// function of Eq. cond_tdf2, the conductivity and Seebeck coefficient of
// Eqs. cond_tdf and seebeck, and the carrier population of Eq. pop.
//
// With the energy and the integrand X linear inside a tetrahedron,
//   sum_nk X_nk delta(E - eps_nk) -> sum_T (1/6) sum_j c_j(E) X_j,
//   c_j(E) = (1/V_T) int_T delta(E - eps) lambda_j dV.
// The plane eps = E cuts the tetrahedron in a triangle (E below the second or
// above the third corner energy) or a quadrilateral (between them).  With the
// corners sorted by energy and placed at (0,0,0), (1,0,0), (0,1,0), (0,0,1) of
// barycentric space, c_j = 6 A/|grad eps| <lambda_j>, where A is the area of
// the cut and <lambda_j> its area-weighted mean (vertex means of the triangles;
// the quadrilateral is split along the diagonal between its cuts on edges
// (0,2) and (1,3)).
#include "internal.h"

namespace ephx {
namespace {

inline void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{-3, std::string(what) + ": " + hipGetErrorString(e)};
}

struct P3 {
    double x, y, z;
};
__device__ __forceinline__ double tri_area(P3 a, P3 b, P3 c) {
    const double ux = b.x - a.x, uy = b.y - a.y, uz = b.z - a.z;
    const double vx = c.x - a.x, vy = c.y - a.y, vz = c.z - a.z;
    const double cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
    return 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
}

// c[j] for corner energies ein[j] at energy E
__device__ void tet_weights(const double ein[4], double E, double c[4]) {
    int p[4] = {0, 1, 2, 3};
    double e[4] = {ein[0], ein[1], ein[2], ein[3]};
    // sort ascending (sorting network), carrying the corner labels
#define EPHX_CS(a, b)                       \
    if (e[b] < e[a]) {                      \
        const double te = e[a];             \
        e[a] = e[b];                        \
        e[b] = te;                          \
        const int tp = p[a];                \
        p[a] = p[b];                        \
        p[b] = tp;                          \
    }
    EPHX_CS(0, 1)
    EPHX_CS(2, 3)
    EPHX_CS(0, 2)
    EPHX_CS(1, 3)
    EPHX_CS(1, 2)
#undef EPHX_CS
    c[0] = c[1] = c[2] = c[3] = 0.0;
    if (!(E > e[0] && E < e[3])) return;
    const double g1 = e[1] - e[0], g2 = e[2] - e[0], g3 = e[3] - e[0];
    const double gn = sqrt(g1 * g1 + g2 * g2 + g3 * g3);
    double area, l[4];
    if (E <= e[1]) {
        // cuts on edges (0,1), (0,2), (0,3)
        const double t1 = (E - e[0]) / g1, t2 = (E - e[0]) / g2, t3 = (E - e[0]) / g3;
        area = tri_area(P3{t1, 0, 0}, P3{0, t2, 0}, P3{0, 0, t3});
        l[0] = (3.0 - t1 - t2 - t3) / 3.0;
        l[1] = t1 / 3.0;
        l[2] = t2 / 3.0;
        l[3] = t3 / 3.0;
    } else if (E < e[2]) {
        // cuts on edges (0,2), (0,3), (1,3), (1,2), in that cyclic order
        const double a02 = (E - e[0]) / (e[2] - e[0]), a03 = (E - e[0]) / (e[3] - e[0]);
        const double a13 = (E - e[1]) / (e[3] - e[1]), a12 = (E - e[1]) / (e[2] - e[1]);
        const P3 q02{0, a02, 0}, q03{0, 0, a03}, q13{1.0 - a13, 0, a13}, q12{1.0 - a12, a12, 0};
        const double A1 = tri_area(q02, q03, q13), A2 = tri_area(q02, q13, q12);
        area = A1 + A2;
        // lambda at the cuts: q02 (1-a02, 0, a02, 0), q03 (1-a03, 0, 0, a03),
        // q13 (0, 1-a13, 0, a13), q12 (0, 1-a12, a12, 0)
        l[0] = (A1 * ((1.0 - a02) + (1.0 - a03)) + A2 * (1.0 - a02)) / (3.0 * area);
        l[1] = (A1 * (1.0 - a13) + A2 * ((1.0 - a13) + (1.0 - a12))) / (3.0 * area);
        l[2] = (A1 * a02 + A2 * (a02 + a12)) / (3.0 * area);
        l[3] = (A1 * (a03 + a13) + A2 * a13) / (3.0 * area);
    } else {
        // cuts on edges (0,3), (1,3), (2,3)
        const double s0 = (E - e[0]) / (e[3] - e[0]), s1 = (E - e[1]) / (e[3] - e[1]), s2 = (E - e[2]) / (e[3] - e[2]);
        area = tri_area(P3{0, 0, s0}, P3{1.0 - s1, 0, s1}, P3{0, 1.0 - s2, s2});
        l[0] = (1.0 - s0) / 3.0;
        l[1] = (1.0 - s1) / 3.0;
        l[2] = (1.0 - s2) / 3.0;
        l[3] = (s0 + s1 + s2) / 3.0;
    }
    if (!(area > 0.0)) return;
    const double d = 6.0 * area / gn;
#pragma unroll
    for (int k = 0; k < 4; ++k) c[p[k]] = d * l[k];
}

constexpr int kTetChunk = 2048;     // tetrahedra per workgroup
constexpr int kMaxComp = 9;

// partial[chunk][e][comp] = sum over the chunk's tetrahedra of (1/6) sum_j c_j x_j
__global__ __launch_bounds__(256) void k_tetra_sum(int n_tet, const int32_t* __restrict__ tet,
                                                   const double* __restrict__ eps, int nc, const double* __restrict__ x,
                                                   const double* __restrict__ egrid, int n_e,
                                                   double* __restrict__ partial) {
    __shared__ double red[kMaxComp][256];
    const int chunk = blockIdx.x, ie = blockIdx.y;
    const double E = egrid[ie];
    double acc[kMaxComp];
#pragma unroll
    for (int k = 0; k < kMaxComp; ++k) acc[k] = 0.0;
    const int t1 = min(n_tet, (chunk + 1) * kTetChunk);
    for (int t = chunk * kTetChunk + threadIdx.x; t < t1; t += 256) {
        int s[4];
        double e[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            s[j] = tet[4 * t + j];
            e[j] = eps[s[j]];
        }
        if (!(E > fmin(fmin(e[0], e[1]), fmin(e[2], e[3])) && E < fmax(fmax(e[0], e[1]), fmax(e[2], e[3]))))
            continue;
        double c[4];
        tet_weights(e, E, c);
        for (int k = 0; k < nc; ++k) {
            double v = 0.0;
#pragma unroll
            for (int j = 0; j < 4; ++j) v = fma(c[j], x[(long)s[j] * nc + k], v);
            acc[k] += v / 6.0;
        }
    }
    for (int k = 0; k < nc; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < nc; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if ((int)threadIdx.x < nc) partial[((long)chunk * n_e + ie) * nc + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_tetra_reduce(int n_chunk, int n_e, int nc, const double* __restrict__ partial, double scale,
                               double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_e * nc) return;
    double s = 0.0;
    for (int c = 0; c < n_chunk; ++c) s += partial[(long)c * n_e * nc + i];
    out[i] = scale * s;
}

// x[s][3a+b] = v[s][a] F[s][b]
__global__ void k_vf(int S, const double* __restrict__ vel, const double* __restrict__ ff, double* __restrict__ x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 9 * S) return;
    const int s = i / 9, ab = i % 9;
    x[i] = vel[3 * s + ab / 3] * ff[3 * s + ab % 3];
}

// Eq. cond_tdf and Eq. seebeck by the trapezoid rule on the energy grid:
//   V1 = int (-df0/dE) Sigma dE,  V2 = int (-df0/dE)(E - mu) Sigma dE,
//   sigma = e^2 V1 (S/m),  S = V1^{-1} V2 / (q T) with q = -e (V/K)
__global__ void k_tdf_transport(int n_e, const double* __restrict__ egrid, const double* __restrict__ tdf, double mu,
                                double temp, double sigma_unit, double* __restrict__ sigma,
                                double* __restrict__ seebeck) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double kt = kBoltzEv * temp;
    double v1[9] = {0}, v2[9] = {0};
    for (int i = 0; i + 1 < n_e; ++i) {
        const double ea = egrid[i], eb = egrid[i + 1], h = 0.5 * (eb - ea);
        const double fa = 1.0 / (exp((ea - mu) / kt) + 1.0), fb = 1.0 / (exp((eb - mu) / kt) + 1.0);
        const double wa = fa * (1.0 - fa) / kt, wb = fb * (1.0 - fb) / kt;
        for (int k = 0; k < 9; ++k) {
            v1[k] += h * (wa * tdf[9 * i + k] + wb * tdf[9 * (i + 1) + k]);
            v2[k] += h * (wa * (ea - mu) * tdf[9 * i + k] + wb * (eb - mu) * tdf[9 * (i + 1) + k]);
        }
    }
    for (int k = 0; k < 9; ++k) sigma[k] = sigma_unit * v1[k];
    // inverse of V1 by its adjugate
    const double a = v1[0], b = v1[1], c = v1[2], d = v1[3], e = v1[4], f = v1[5], g = v1[6], h = v1[7], i = v1[8];
    const double det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
    double inv[9] = {e * i - f * h, c * h - b * i, b * f - c * e, f * g - d * i, a * i - c * g,
                     c * d - a * f, d * h - e * g, b * g - a * h, a * e - b * d};
    for (int k = 0; k < 9; ++k) inv[k] /= det;
    for (int r = 0; r < 3; ++r)
        for (int col = 0; col < 3; ++col) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += inv[3 * r + k] * v2[3 * k + col];
            seebeck[3 * r + col] = -s / temp;
        }
}

}  // namespace

int tetra_chunks(int n_tet) { return (n_tet + kTetChunk - 1) / kTetChunk; }

void tetra_sum(int n_tet, const int32_t* tet, const double* eps, int nc, const double* x, int n_e, const double* egrid,
               double scale, double* partial, double* out, hipStream_t st) {
    if (nc < 1 || nc > kMaxComp) throw Error{-1, "tetra_sum: 1 to 9 components"};
    if (n_e <= 0) return;
    if (n_e > 65535) throw Error{-1, "tetra_sum: at most 65535 energies"};
    const int nch = tetra_chunks(n_tet);
    if (nch > 0) {
        hipLaunchKernelGGL(k_tetra_sum, dim3(nch, n_e), dim3(256), 0, st, n_tet, tet, eps, nc, x, egrid, n_e, partial);
        check_launch("tetra_sum");
    }
    hipLaunchKernelGGL(k_tetra_reduce, dim3((n_e * nc + 255) / 256), dim3(256), 0, st, nch, n_e, nc, partial, scale,
                       out);
    check_launch("tetra_reduce");
}

void vf_products(int S, const double* vel, const double* ff, double* x, hipStream_t st) {
    hipLaunchKernelGGL(k_vf, dim3((9 * S + 255) / 256), dim3(256), 0, st, S, vel, ff, x);
    check_launch("vf_products");
}

void tdf_transport(int n_e, const double* egrid, const double* tdf, double mu, double temp, double sigma_unit,
                   double* sigma, double* seebeck, hipStream_t st) {
    hipLaunchKernelGGL(k_tdf_transport, dim3(1), dim3(64), 0, st, n_e, egrid, tdf, mu, temp, sigma_unit, sigma,
                       seebeck);
    check_launch("tdf_transport");
}

}  // namespace ephx
