// Phase-factor Fourier contractions on MFMA (gfx950).
//
//   C[z][m][n] = sum_r exp(2 pi i (x_m + x0_z) . n_r) B[z][r][n]        (complex)
//
// This single contraction is every Fourier sum of the method: H(k) (Eq.
// wannier_3), D(q) (Eq. IFC2), the Re sum g(k,Rp) and the Rp sum g^W(k,q)
// of Eq. eph_mat_wann2, and H(k+q) per (k,q) pair.  The phase matrix A is
// generated in registers: the argument t = x.n is formed in FP64 and reduced
// to [-1/2, 1/2) before sin/cos, so A is never read from memory.
//
// Tiling: a 256-thread workgroup owns a 64-row x (16*CB)-column output tile;
// wave w computes rows 16w..16w+15 with 16x16 MFMA blocks.  B is staged
// through LDS one K chunk at a time.  Complex products use four real MFMAs:
//   Cre += Are*Bre - Aim*Bim ,  Cim += Are*Bim + Aim*Bre.
// MFMA 16x16xK operand layout: lane l holds A[l%16][k-group l/16] and
// B[k-group l/16][l%16].  Accumulator element v of lane l is C[r][l%16] with
// r = 4*(l/16) + v for the f32 and bf16 instructions but r = l/16 + 4*v for
// v_mfma_f64_16x16x4f64 (measured on gfx950).
#include <type_traits>

#include "internal.h"

namespace ephx {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

template <typename NT>
__device__ __forceinline__ double reduced_arg(double a, double b, double c, const NT* n) {
    double t = fma(a, (double)n[0], fma(b, (double)n[1], c * (double)n[2]));
    return t - rint(t);
}

__device__ __forceinline__ void phase_of(double r, double& c, double& s) { sincospi(2.0 * r, &s, &c); }
__device__ __forceinline__ void phase_of(double r, float& c, float& s) {
    sincospif((float)(2.0 * r), &s, &c);
}

__device__ __forceinline__ dbl4 mfma(double a, double b, dbl4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ flt4 mfma(float a, float b, flt4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> struct AccOf;
template <> struct AccOf<double> {
    typedef dbl4 type;
    static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};
template <> struct AccOf<float> {
    typedef flt4 type;
    static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};

constexpr int kBM = 64;
constexpr int kKC = 16;

// HERM = true: Hermitian sums H(x) = sum_r [cos(2 pi x.n_r) A_r + sin(2 pi x.n_r) B_r]
// over half of a +/-R symmetric set, with A_r = H(R)+H(R)^dag, B_r = i(H(R)-H(R)^dag)
// (A_0 = H(0), B_0 = 0); B holds [r][2][N] complex.  Real coefficients against
// complex columns need two MFMAs per complex product instead of four, over half
// the vectors.
// KD = true: the contraction-side points are real (double [K][3]) instead of
// integer vectors -- used by the adjoint sums over q and k; ACC = true adds the
// product to C.
// TB: element type of B (float B is widened as it is staged, for FP64 sums
// over a complex-float coupling tensor).  WC = true (few rows, M <= 16): the
// four waves take the same 16 rows and four consecutive column blocks, so a
// workgroup covers 16 rows x 64 CB columns instead of padding M to 64 rows.
// PT = true: the phases come from a table [M][K] of (cos, sin) that x0 points
// to (filled by k_phase_table with the same expression, so the same values),
// each lane loading its four of a chunk one chunk ahead, instead of every
// column block of the launch generating them again.
template <typename T, int CB, bool HERM = false, bool KD = false, bool ACC = false, typename TB = T,
          bool WC = false, bool PT = false>
__global__ __launch_bounds__(256) void k_phase_gemm(int M, int N, int K, const double* __restrict__ x,
                                                    const double* __restrict__ x0,
                                                    const void* __restrict__ nvec_,
                                                    const TB* __restrict__ B, long sB,
                                                    T* __restrict__ C, long sC, int cg) {
    typedef typename AccOf<T>::type acc_t;
    typedef typename std::conditional<KD, double, int32_t>::type NT;
    const NT* nvec = reinterpret_cast<const NT*>(nvec_);
    constexpr int BN = 16 * CB;
    constexpr int NB = HERM ? 2 : 1;
    constexpr int WBN = WC ? 4 * BN : BN;     // columns of the workgroup
    // component-major rows: the 16 lanes of a read phase take 16 consecutive
    // columns of one component, one contiguous run of LDS words (no bank
    // conflicts; a column-major [BN][components] layout had 3.7 per read)
    __shared__ T bs[kKC][2 * NB][WBN];
    __shared__ NT ns[kKC][3];
    const int z = blockIdx.z;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int row0 = WC ? blockIdx.y * 16 : blockIdx.y * kBM;
    const int col0 = blockIdx.x * WBN;
    const int wrow = WC ? 0 : wave * 16;      // the wave's first row in the tile
    const int wcol = WC ? wave * BN : 0;      // ... and first column
    const TB* bz = B + (long)z * sB * 2;
    T* cz = C + (long)z * sC * 2;

    const int arow = row0 + wrow + li;
    const bool rowok = arow < M;
    double xa = 0.0, xb = 0.0, xc = 0.0;
    if (rowok) {
        xa = x[3 * arow];
        xb = x[3 * arow + 1];
        xc = x[3 * arow + 2];
    }
    if (!PT && x0 != nullptr) {
        xa += x0[3 * z];
        xb += x0[3 * z + 1];
        xc += x0[3 * z + 2];
    }
    // PT: this lane's (cos, sin) for the four k-steps of a chunk
    const double2* tab = reinterpret_cast<const double2*>(x0);
    const long trow = (long)min(arow, M - 1) * K;
    double2 tph[kKC / 4];
    auto load_ph = [&](int kc) {
#pragma unroll
        for (int s = 0; s < kKC / 4; ++s) tph[s] = tab[trow + min(kc + 4 * s + lk, K - 1)];
    };
    if (PT && K > 0) load_ph(0);

    acc_t are[CB], aim[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        are[cb] = acc_t{0, 0, 0, 0};
        aim[cb] = acc_t{0, 0, 0, 0};
    }

    typedef TB tb2 __attribute__((ext_vector_type(2)));
    for (int kc = 0; kc < K; kc += kKC) {
        // rows past K and columns past N load the last valid one (a row past K
        // meets a zero phase, a column past N is never stored): no branch, one
        // (re, im) load per element and plane.  Every load of the chunk is
        // issued before the first LDS write, so the thread waits on one
        // memory latency per chunk, not one per element.
        static_assert(kKC * WBN % 256 == 0, "whole elements per thread");
        constexpr int EPT = kKC * WBN / 256;
        tb2 bv[EPT][NB];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = tid + 256 * j;
            const int kk = e / WBN, nn = e % WBN;
            const long r = min(kc + kk, K - 1), col = min(col0 + nn, N - 1);
#pragma unroll
            for (int h = 0; h < NB; ++h) bv[j][h] = *reinterpret_cast<const tb2*>(bz + ((r * NB + h) * N + col) * 2);
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int e = tid + 256 * j;
            const int kk = e / WBN, nn = e % WBN;
#pragma unroll
            for (int h = 0; h < NB; ++h) {
                bs[kk][2 * h][nn] = (T)bv[j][h].x;
                bs[kk][2 * h + 1][nn] = (T)bv[j][h].y;
            }
        }
        if (tid < kKC * 3) {
            const int kk = tid / 3, d = tid % 3;
            ns[kk][d] = (kc + kk < K) ? nvec[3 * (kc + kk) + d] : 0;
        }
        __syncthreads();
        double2 cph[kKC / 4];
        if (PT) {
#pragma unroll
            for (int s = 0; s < kKC / 4; ++s) cph[s] = tph[s];
            if (kc + kKC < K) load_ph(kc + kKC);
        }
#pragma unroll
        for (int s = 0; s < kKC / 4; ++s) {
            // k-steps wholly past K add nothing (zero phases): skipped, a
            // branch on a workgroup-uniform value
            if (kc + 4 * s >= K) break;
            const int kk = 4 * s + lk;
            T pc = 0, ps = 0;
            if (rowok && kc + kk < K) {
                if (PT) {
                    pc = (T)cph[s].x;
                    ps = (T)cph[s].y;
                } else {
                    phase_of(reduced_arg(xa, xb, xc, ns[kk]), pc, ps);
                }
            }
            const T nps = -ps;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const T bre = bs[kk][0][wcol + cb * 16 + li];
                const T bim = bs[kk][1][wcol + cb * 16 + li];
                if (HERM) {
                    const T b2re = bs[kk][2 * NB - 2][wcol + cb * 16 + li];
                    const T b2im = bs[kk][2 * NB - 1][wcol + cb * 16 + li];
                    are[cb] = mfma(pc, bre, are[cb]);
                    are[cb] = mfma(ps, b2re, are[cb]);
                    aim[cb] = mfma(pc, bim, aim[cb]);
                    aim[cb] = mfma(ps, b2im, aim[cb]);
                } else {
                    are[cb] = mfma(pc, bre, are[cb]);
                    are[cb] = mfma(nps, bim, are[cb]);
                    aim[cb] = mfma(pc, bim, aim[cb]);
                    aim[cb] = mfma(ps, bre, aim[cb]);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int col = col0 + wcol + cb * 16 + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = row0 + wrow + AccOf<T>::row(lk, v);
            if (row < M && col < N) {
                // cg > 0: the columns are groups of cg (one matrix each), stored
                // group-major as [N/cg][M][cg]
                const long off = (cg > 0 ? ((long)(col / cg) * M + row) * cg + col % cg : (long)row * N + col) * 2;
                cz[off] = ACC ? cz[off] + are[cb][v] : are[cb][v];
                cz[off + 1] = ACC ? cz[off + 1] + aim[cb][v] : aim[cb][v];
            }
        }
    }
}

// ------------------------------------------- split-precision (bf16 / fp16) variants
__device__ __forceinline__ unsigned short bf16_bits_rn(float f) {
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_float(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

// split x into NS bf16 parts (round to nearest even each time): x ~ p0 + p1 (+ p2)
template <int NS>
__device__ __forceinline__ void split_n(float x, unsigned short* part) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        part[i] = bf16_bits_rn(x);
        x -= bf16_to_float(part[i]);
    }
}

// split x into NS fp16 parts (round to nearest even each time): 11 significant
// bits per part against 8 for bf16, over a narrower exponent range (the
// callers scale the operand into it)
template <int NS>
__device__ __forceinline__ void split_h(float x, unsigned short* part) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const _Float16 h = (_Float16)x;
        part[i] = __builtin_bit_cast(unsigned short, h);
        x -= (float)h;
    }
}
template <int NS, bool F16>
__device__ __forceinline__ void split_p(float x, unsigned short* part) {
    if constexpr (F16)
        split_h<NS>(x, part);
    else
        split_n<NS>(x, part);
}

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <bool F16>
__device__ __forceinline__ flt4 mfma_bf(const u16x8& a, const u16x8& b, flt4 c) {
    if constexpr (F16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                      0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                       __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

constexpr int kBK = 32;     // K per MFMA step
constexpr int kPadK = 8;    // LDS row padding (bf16 elements)

// NS = 2: "BF16x3" (products p_i q_j with i + j <= 1, three per real product);
// NS = 3: "BF16x6" (i + j <= 2, six per real product).  F16: the parts are fp16
// ("FP16x3" with NS = 2), B scaled by a power of two that the output undoes
// (oscale).  Accumulation in FP32; the smallest products are issued first.
template <int CB, int NS, bool F16 = false>
__global__ __launch_bounds__(256) void k_phase_gemm_bf16(int M, int N, int K, int Kp,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ x0,
                                                         const int32_t* __restrict__ nvec,
                                                         const uint16_t* __restrict__ Bs, long sB,
                                                         float* __restrict__ C, long sC, float oscale) {
    constexpr int BN = 16 * CB;
    constexpr int NP = 2 * NS;   // planes: re parts 0..NS-1, im parts NS..2NS-1
    __shared__ __attribute__((aligned(16))) uint16_t bsh[NP][BN][kBK + kPadK];
    __shared__ int32_t ns[kBK][3];
    const int z = blockIdx.z;
    const int row0 = blockIdx.y * kBM;
    const int col0 = blockIdx.x * BN;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const uint16_t* bz = Bs + (long)z * sB;
    float* cz = C + (long)z * sC * 2;

    const int arow = row0 + wave * 16 + li;
    const bool rowok = arow < M;
    double xa = 0.0, xb = 0.0, xc = 0.0;
    if (rowok) {
        xa = x[3 * arow];
        xb = x[3 * arow + 1];
        xc = x[3 * arow + 2];
    }
    if (x0 != nullptr) {
        xa += x0[3 * z];
        xb += x0[3 * z + 1];
        xc += x0[3 * z + 2];
    }
    flt4 are[CB], aim[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        are[cb] = flt4{0, 0, 0, 0};
        aim[cb] = flt4{0, 0, 0, 0};
    }
    for (int kc = 0; kc < Kp; kc += kBK) {
        // stage the planes of a [BN][32] chunk: 16-byte loads along K
        for (int e = tid; e < NP * BN * (kBK / 8); e += 256) {
            const int seg = e % (kBK / 8);
            const int nn = (e / (kBK / 8)) % BN;
            const int pl = e / ((kBK / 8) * BN);
            const int col = col0 + nn;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (col < N) v = *reinterpret_cast<const uint4*>(bz + ((long)pl * N + col) * Kp + kc + seg * 8);
            *reinterpret_cast<uint4*>(&bsh[pl][nn][seg * 8]) = v;
        }
        if (tid < kBK * 3) {
            const int kk = tid / 3, d = tid % 3;
            ns[kk][d] = (kc + kk < K) ? nvec[3 * (kc + kk) + d] : 0;
        }
        __syncthreads();
        u16x8 ar[NS], ai[NS], nai[NS];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int kk = 8 * lk + j;
            float pc = 0.f, ps = 0.f;
            if (rowok && kc + kk < K) phase_of(reduced_arg(xa, xb, xc, ns[kk]), pc, ps);
            unsigned short pr[NS], pi[NS];
            split_p<NS, F16>(pc, pr);
            split_p<NS, F16>(ps, pi);
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                ar[t][j] = pr[t];
                ai[t][j] = pi[t];
                nai[t][j] = pi[t] ^ 0x8000u;   // sign bit of bf16 and fp16 alike
            }
        }
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int nn = cb * 16 + li;
            u16x8 br[NS], bi[NS];
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                br[t] = *reinterpret_cast<const u16x8*>(&bsh[t][nn][8 * lk]);
                bi[t] = *reinterpret_cast<const u16x8*>(&bsh[NS + t][nn][8 * lk]);
            }
#pragma unroll
            for (int ord = NS - 1; ord >= 0; --ord) {
#pragma unroll
                for (int i = 0; i <= ord; ++i) {
                    const int j = ord - i;
                    are[cb] = mfma_bf<F16>(ar[i], br[j], are[cb]);
                    are[cb] = mfma_bf<F16>(nai[i], bi[j], are[cb]);
                    aim[cb] = mfma_bf<F16>(ar[i], bi[j], aim[cb]);
                    aim[cb] = mfma_bf<F16>(ai[i], br[j], aim[cb]);
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        const int col = col0 + cb * 16 + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = row0 + wave * 16 + AccOf<float>::row(lk, v);
            if (row < M && col < N) {
                const long off = ((long)row * N + col) * 2;
                cz[off] = are[cb][v] * oscale;
                cz[off + 1] = aim[cb][v] * oscale;
            }
        }
    }
}

template <int NS, bool F16 = false>
__global__ void k_split_bf16(int K, int N, int Kp, double scale, const double* __restrict__ B,
                             uint16_t* __restrict__ out) {
    // one thread per (z, n, k) output element, k fastest; planes re_0..re_{NS-1}, im_0..
    const int z = blockIdx.z;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)N * Kp) return;
    const int n = (int)(idx / Kp), k = (int)(idx % Kp);
    float re = 0.f, im = 0.f;
    if (k < K) {
        const long off = ((long)z * K * N + (long)k * N + n) * 2;
        re = (float)(scale * B[off]);
        im = (float)(scale * B[off + 1]);
    }
    unsigned short pr[NS], pi[NS];
    split_p<NS, F16>(re, pr);
    split_p<NS, F16>(im, pi);
    uint16_t* oz = out + (long)z * 2 * NS * N * Kp;
    for (int t = 0; t < NS; ++t) {
        oz[((long)t * N + n) * Kp + k] = pr[t];
        oz[((long)(NS + t) * N + n) * Kp + k] = pi[t];
    }
}

// Split phase planes (bf16, or fp16 with F16) of one point set, computed once and read by every
// contraction over the same points (all k of a batch, all column blocks):
//   planes[t][m][r]      = part t of cos(2 pi x_m . n_r)      (t < NS)
//   planes[NS + t][m][r] = part t of sin(2 pi x_m . n_r)
// r padded to Kp with zero parts.  The values equal those the in-register
// path generates (same reduced argument, same FP32 sin/cos, same split).
template <int NS, bool F16 = false>
__global__ void k_phase_planes(int M, int K, int Kp, const double* __restrict__ x, const int32_t* __restrict__ nvec,
                               uint16_t* __restrict__ out) {
    const int kg = Kp / 8;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;   // (m, group of 8 r)
    if (idx >= (long)M * kg) return;
    const int m = (int)(idx / kg), r0 = (int)(idx % kg) * 8;
    const double xa = x[3L * m], xb = x[3L * m + 1], xc = x[3L * m + 2];
    u16x8 pr[NS], pi[NS];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        float pc = 0.f, ps = 0.f;
        if (r0 + j < K) phase_of(reduced_arg(xa, xb, xc, nvec + 3L * (r0 + j)), pc, ps);
        unsigned short hr[NS], hi[NS];
        split_p<NS, F16>(pc, hr);
        split_p<NS, F16>(ps, hi);
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            pr[t][j] = hr[t];
            pi[t][j] = hi[t];
        }
    }
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        *reinterpret_cast<u16x8*>(out + ((long)t * M + m) * Kp + r0) = pr[t];
        *reinterpret_cast<u16x8*>(out + ((long)(NS + t) * M + m) * Kp + r0) = pi[t];
    }
}

// C[z] = A B[z] with A given as phase planes [2NS][M][Kp] (real A: [NS][M][Kp])
// and B[z] as planes [2NS][N][Kp], on the 32x32x16 bf16 (or fp16) MFMA (twice
// the rate of the 16x16x32 shape on gfx950, measured from registers).  Operand
// lane l holds row (A) or column (B) l%32 and the 8 consecutive k of group
// l/32; accumulator element v of lane l is C[8(v/4) + 4(l/32) + v%4][l%32].  A
// workgroup of NWV waves owns 32 RTW NWV rows x 32*CT columns, wave w the rows
// of its RTW 32-row tiles against all CT column tiles.
// Workgroups are numbered so that each of the 8 XCDs (which receive
// consecutive workgroup ids in turn) runs a contiguous range of (column, row, z)
// tiles: the B panel of one z stays in that XCD's L2 while its row tiles
// stream the shared A planes.
//
// Software pipeline, one barrier per K chunk of 32: while the MFMAs of chunk c
// run, the B panel of chunk c+1 streams into the other half of a double LDS
// buffer by direct global->LDS loads (each wave instruction fills 1 KB: 16
// rows x 64 bytes) and the A fragments of chunk c+1 load into registers.  LDS
// rows are 64 bytes with their four 16-byte segments XOR-swizzled by bits 2-3
// of the row, so the 16-lane passes of a ds_read_b128 hit distinct banks.
typedef float flt16 __attribute__((ext_vector_type(16)));

template <bool F16>
__device__ __forceinline__ flt16 mfma_bf32(const u16x8& a, const u16x8& b, flt16 c) {
    if constexpr (F16)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                      0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
}


__device__ __forceinline__ int swz(int row, int seg) { return seg ^ ((row >> 2) & 3); }

// RA = true: A is real, [NS][M][Kp] (the cos and sin parts of a half-set sum
// side by side along k), and C = A B takes two MFMAs per product instead of four.
// F16 = true: fp16 parts (FP16x3), the output multiplied by oscale (the power of
// two that undoes the scaling of B).
// NWV waves per workgroup (4 or 8; with 8, two per SIMD).
template <int CT, int NS, bool RA = false, bool F16 = false, int RTW = 1, int NWV = 4>
__global__ __launch_bounds__(64 * NWV) void k_gemm_bf16_planes(int M, int N, int Kp, int nbx, int nby, int nz,
                                                          const uint16_t* __restrict__ As,
                                                          const uint16_t* __restrict__ Bs, long sB,
                                                          float* __restrict__ C, long sC, float oscale) {
    // RTW row tiles of 32 per wave: each B fragment read from LDS feeds RTW
    // times the MFMAs
    constexpr int BMW = 32 * RTW, BM = NWV * BMW;
    constexpr int BN = 32 * CT;
    constexpr int NP = 2 * NS;
    constexpr int PLANE = BN * kBK;          // bf16 elements of one plane in one buffer
    constexpr int BUF = NP * PLANE;
    constexpr int NBLK = NP * (BN / 16);     // 1 KB blocks per chunk
    __shared__ __attribute__((aligned(16))) uint16_t bsh[2 * BUF];
    // workgroup id -> tile id, contiguous per XCD
    const int nblk = nbx * nby * nz;
    const int b = blockIdx.x;
    const int xcd = b % 8, slot = b / 8;
    const int base = nblk / 8, rem = nblk % 8;
    const int tile = (xcd < rem ? xcd * (base + 1) : rem * (base + 1) + (xcd - rem) * base) + slot;
    const int bx = tile % nbx, by = (tile / nbx) % nby, z = tile / (nbx * nby);
    const int row0 = by * BM, col0 = bx * BN;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int l32 = lane & 31, kg = lane >> 5;
    const uint16_t* bz = Bs + (long)z * sB;
    float* cz = C + (long)z * sC * 2;
    flt16 are[RTW][CT], aim[RTW][CT];
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                are[rt][ct][v] = 0.f;
                aim[rt][ct][v] = 0.f;
            }
    // rows and columns past the edge load the last valid one: their results are
    // never stored, and the loads need no branch
    const uint16_t* arow[RTW];
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt)
        arow[rt] = As + (long)min(row0 + wave * BMW + rt * 32 + l32, M - 1) * Kp + 8 * kg;
    const long plane = (long)M * Kp;
    const u16x8 sign = {0x8000u, 0x8000u, 0x8000u, 0x8000u, 0x8000u, 0x8000u, 0x8000u, 0x8000u};
    // B panel of the chunk at kc into buffer h: wave w fills blocks w, w+NWV,
    // ...; lane l writes row (l/4) of the block, LDS segment l%4
    static_assert(NBLK % NWV == 0, "whole blocks per wave");
    auto issue_b = [&](int kc, int h) {
#pragma unroll
        for (int j = 0; j < NBLK / NWV; ++j) {
            const int i = NWV * j + wave;
            const int pl = i / (BN / 16), rb = i % (BN / 16);
            const int r = rb * 16 + (lane >> 2);
            const int col = min(col0 + r, N - 1);
            uint16_t* dst = bsh + h * BUF + pl * PLANE + rb * 16 * kBK;
            __builtin_amdgcn_global_load_lds((const void*)(bz + ((long)pl * N + col) * Kp + kc + 8 * swz(r, lane & 3)),
                                             (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
        }
    };
    // A fragments of the chunk at kc: k-steps s = 0, 1 of 16
    u16x8 anr[RTW][2][NS], ani[RTW][2][NS];
    auto load_a = [&](int kc) {
#pragma unroll
        for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int t = 0; t < NS; ++t) {
                    anr[rt][s][t] = *reinterpret_cast<const u16x8*>(arow[rt] + t * plane + kc + 16 * s);
                    if (!RA)
                        ani[rt][s][t] = *reinterpret_cast<const u16x8*>(arow[rt] + (NS + t) * plane + kc + 16 * s);
                }
    };
    issue_b(0, 0);
    load_a(0);
    int h = 0;
    for (int kc = 0; kc < Kp; kc += kBK, h ^= 1) {
        // chunk kc's panel and fragments have arrived (this wave's loads), and
        // every wave has finished reading the other buffer
        __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        u16x8 ar[RTW][2][NS], ai[RTW][2][NS], nai[RTW][2][NS];
#pragma unroll
        for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int t = 0; t < NS; ++t) {
                    ar[rt][s][t] = anr[rt][s][t];
                    if (!RA) {
                        ai[rt][s][t] = ani[rt][s][t];
                        nai[rt][s][t] = ani[rt][s][t] ^ sign;
                    }
                }
        if (kc + kBK < Kp) {
            issue_b(kc + kBK, h ^ 1);
            load_a(kc + kBK);
        }
        const uint16_t* bb = bsh + h * BUF;
        // groups g = (column tile, k-step); the B fragments of group g + RD are
        // read from LDS while the MFMAs of group g run, RD = 2 for two-part
        // operands (three register slots, the order held by scheduling
        // barriers: left alone, the compiler moved each read next to its
        // MFMAs and reused one register set, so most MFMAs waited on an LDS
        // read issued just before them; 2-3 % faster at the Si-like shape),
        // RD = 1 for three parts (the barriers cost those forms registers).
        constexpr int RD = NS == 2 ? 2 : 1, NSL = RD + 1;
        u16x8 br[NSL][NS], bi[NSL][NS];
        auto read_b = [&](int g, int slotb) {
            const int nn = (g >> 1) * 32 + l32;
            const int so = nn * kBK + 8 * swz(nn, 2 * (g & 1) + kg);
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                br[slotb][t] = *reinterpret_cast<const u16x8*>(bb + t * PLANE + so);
                bi[slotb][t] = *reinterpret_cast<const u16x8*>(bb + (NS + t) * PLANE + so);
            }
        };
#pragma unroll
        for (int g = 0; g < RD; ++g) read_b(g, g);
#pragma unroll
        for (int g = 0; g < 2 * CT; ++g) {
            if (g + RD < 2 * CT) read_b(g + RD, (g + RD) % NSL);
            if constexpr (RD == 2) __builtin_amdgcn_sched_barrier(0);
            const int ct = g >> 1, s = g & 1, cs = g % NSL;
#pragma unroll
            for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
                for (int ord = NS - 1; ord >= 0; --ord) {
#pragma unroll
                    for (int i = 0; i <= ord; ++i) {
                        const int j = ord - i;
                        are[rt][ct] = mfma_bf32<F16>(ar[rt][s][i], br[cs][j], are[rt][ct]);
                        aim[rt][ct] = mfma_bf32<F16>(ar[rt][s][i], bi[cs][j], aim[rt][ct]);
                        if (!RA) {
                            are[rt][ct] = mfma_bf32<F16>(nai[rt][s][i], bi[cs][j], are[rt][ct]);
                            aim[rt][ct] = mfma_bf32<F16>(ai[rt][s][i], br[cs][j], aim[rt][ct]);
                        }
                    }
                }
            if constexpr (RD == 2) __builtin_amdgcn_sched_barrier(0);
        }
    }
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            const int col = col0 + ct * 32 + l32;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = row0 + wave * BMW + rt * 32 + 8 * (v >> 2) + 4 * kg + (v & 3);
                if (row < M && col < N) {
                    const float2 o = {are[rt][ct][v] * oscale, aim[rt][ct][v] * oscale};
                    *reinterpret_cast<float2*>(cz + ((long)row * N + col) * 2) = o;
                }
            }
        }
}

// Half-set form of a Fourier sum over a vector list that is closed under
// R -> -R apart from some unpaired vectors:
//   sum_p e^{2 pi i x.R_p} G_p = sum_h cos(2 pi x.R_h) Gc_h + sin(2 pi x.R_h) Gs_h
// with Gc_h = G_p + G_n, Gs_h = i (G_p - G_n) for a pair (p, n), R_n = -R_p, and
// Gc_h = G_p, Gs_h = i G_p for an unpaired vector (R = 0 among them).  The
// coefficients are real, so a pair costs half the products of the complex sum.
// pair: [Kh][2] = (p, n), n = -1 when unpaired.  G: [Z][K][N] complex double.
// k_half_combine writes [Z][Kh][2][N] complex (Gc_h, Gs_h) in T.
template <typename T>
__global__ void k_half_combine(int K, int N, int Kh, const int32_t* __restrict__ pair, const double* __restrict__ G,
                               T* __restrict__ out) {
    const int z = blockIdx.z;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;   // (h, n), n fastest
    if (idx >= (long)Kh * N) return;
    const int h = (int)(idx / N), n = (int)(idx % N);
    const double* gz = G + (long)z * K * N * 2;
    const int p = pair[2 * h], q = pair[2 * h + 1];
    const double ar = gz[((long)p * N + n) * 2], ai = gz[((long)p * N + n) * 2 + 1];
    const double br = q >= 0 ? gz[((long)q * N + n) * 2] : 0.0, bi = q >= 0 ? gz[((long)q * N + n) * 2 + 1] : 0.0;
    T* oz = out + (long)z * Kh * 2 * N * 2;
    oz[((long)h * 2 * N + n) * 2] = (T)(ar + br);
    oz[((long)h * 2 * N + n) * 2 + 1] = (T)(ai + bi);
    oz[(((long)h * 2 + 1) * N + n) * 2] = (T)(bi - ai);
    oz[(((long)h * 2 + 1) * N + n) * 2 + 1] = (T)(ar - br);
}

// The same coefficients as split planes (bf16, or fp16 with F16, after the
// scale) for the real-A contraction:
// [Z][2NS][N][2 Kh16] (re parts, then im parts), k = h for Gc_h and Kh16 + h for
// Gs_h, zero parts at h >= Kh (Kh16 = Kh rounded up to 16).
template <int NS, bool F16 = false>
__global__ void k_split_bf16_half(int K, int N, int Kh, int Kh16, double scale, const int32_t* __restrict__ pair,
                                  const double* __restrict__ G, uint16_t* __restrict__ out) {
    const int z = blockIdx.z;
    const int Kp = 2 * Kh16;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;   // (n, k), k fastest
    if (idx >= (long)N * Kp) return;
    const int n = (int)(idx / Kp), k = (int)(idx % Kp);
    const bool sn = k >= Kh16;
    const int h = sn ? k - Kh16 : k;
    float re = 0.f, im = 0.f;
    if (h < Kh) {
        const double* gz = G + (long)z * K * N * 2;
        const int p = pair[2 * h], q = pair[2 * h + 1];
        const double ar = gz[((long)p * N + n) * 2], ai = gz[((long)p * N + n) * 2 + 1];
        const double br = q >= 0 ? gz[((long)q * N + n) * 2] : 0.0;
        const double bi = q >= 0 ? gz[((long)q * N + n) * 2 + 1] : 0.0;
        re = (float)(scale * (sn ? bi - ai : ar + br));
        im = (float)(scale * (sn ? ar - br : ai + bi));
    }
    unsigned short pr[NS], pi[NS];
    split_p<NS, F16>(re, pr);
    split_p<NS, F16>(im, pi);
    uint16_t* oz = out + (long)z * 2 * NS * N * Kp;
    for (int t = 0; t < NS; ++t) {
        oz[((long)t * N + n) * Kp + k] = pr[t];
        oz[((long)(NS + t) * N + n) * Kp + k] = pi[t];
    }
}

// Real phase planes of a half set for the same contraction: [NS][M][2 Kh16],
// part t of cos(2 pi x_m.R_h) at k = h and of sin(2 pi x_m.R_h) at Kh16 + h.
template <int NS, bool F16 = false>
__global__ void k_phase_planes_half(int M, int Kh, int Kh16, const double* __restrict__ x,
                                    const int32_t* __restrict__ nvec, uint16_t* __restrict__ out) {
    const int kg = Kh16 / 8, Kp = 2 * Kh16;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;   // (m, group of 8 h)
    if (idx >= (long)M * kg) return;
    const int m = (int)(idx / kg), h0 = (int)(idx % kg) * 8;
    const double xa = x[3L * m], xb = x[3L * m + 1], xc = x[3L * m + 2];
    u16x8 pr[NS], pi[NS];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        float pc = 0.f, ps = 0.f;
        if (h0 + j < Kh) phase_of(reduced_arg(xa, xb, xc, nvec + 3L * (h0 + j)), pc, ps);
        unsigned short hr[NS], hi[NS];
        split_p<NS, F16>(pc, hr);
        split_p<NS, F16>(ps, hi);
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            pr[t][j] = hr[t];
            pi[t][j] = hi[t];
        }
    }
#pragma unroll
    for (int t = 0; t < NS; ++t) {
        *reinterpret_cast<u16x8*>(out + ((long)t * M + m) * Kp + h0) = pr[t];
        *reinterpret_cast<u16x8*>(out + ((long)t * M + m) * Kp + Kh16 + h0) = pi[t];
    }
}

// Packed Hermitian form of an n x n Hermitian X: n*n reals with
// P[i][j] = Re X_ij for i <= j and P[i][j] = Im X_ji for i > j.  The map is real
// and linear, so real combinations of packed matrices are packed combinations.
// Folding k into the half-set coefficients (angle addition): the sum at k + q,
//   sum_r cos(2 pi (k+q).n_r) A_r + sin(2 pi (k+q).n_r) B_r,
// is the same sum over q with
//   A_r(k) = cos(2 pi k.n_r) A_r + sin(2 pi k.n_r) B_r,
//   B_r(k) = cos(2 pi k.n_r) B_r - sin(2 pi k.n_r) A_r,
// so one phase of q serves every k of a batch.  hpack: [Kh][2][P], out:
// [Kh][2][nk][P]; one thread per output pair (r, k, e).
__global__ void k_fold_herm(int nk, const double* __restrict__ kpts, int Kh, const int32_t* __restrict__ nvec, int P,
                            const double* __restrict__ hpack, double* __restrict__ out) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)Kh * nk * P) return;
    const int e = (int)(t % P);
    const long rk = t / P;
    const int kk = (int)(rk % nk), r = (int)(rk / nk);
    double c, s;
    phase_of(reduced_arg(kpts[3 * kk], kpts[3 * kk + 1], kpts[3 * kk + 2], nvec + 3 * r), c, s);
    const double a = hpack[(long)r * 2 * P + e], b = hpack[((long)r * 2 + 1) * P + e];
    out[((long)r * 2 * nk + kk) * P + e] = fma(c, a, s * b);
    out[(((long)r * 2 + 1) * nk + kk) * P + e] = fma(c, b, -s * a);
}

// C[m] = sum_r e^{2 pi i x_m.n_r} B[r] for a few rows m (M <= MR, a k batch)
// against a complex-float B of very many columns (the drawn g(Re,Rp) of a
// large cell, 10^8 columns): one thread per column streams its B[r][col]
// down r, widens it and accumulates every row in FP64 registers; the phases,
// the same for every thread, come from a table [M][K] by scalar loads.  One
// pass over B at the HBM rate, instead of MFMA tiles whose 16 rows are half
// empty for 8 k and whose B panel is widened through LDS.
template <int MR, int CPT>
__global__ __launch_bounds__(256) void k_re_sum_b32(int M, long N, int K, const double2* __restrict__ tab,
                                                    const float* __restrict__ B, double* __restrict__ C) {
    // CPT adjacent columns per thread (CPT = 2 needs N even: one 16-byte load
    // per vector r); past the end the last columns are loaded, nothing stored
    typedef float fv __attribute__((ext_vector_type(2 * CPT)));
    const long col = CPT * ((long)blockIdx.x * 256 + threadIdx.x);
    const bool ok = col < N;
    const long cc = ok ? col : N - CPT;
    const auto* ut = reinterpret_cast<const __attribute__((address_space(4))) double*>(reinterpret_cast<uintptr_t>(tab));
    double ar[CPT][MR], ai[CPT][MR];
#pragma unroll
    for (int h = 0; h < CPT; ++h)
#pragma unroll
        for (int m = 0; m < MR; ++m) {
            ar[h][m] = 0.0;
            ai[h][m] = 0.0;
        }
#pragma unroll 4
    for (int r = 0; r < K; ++r) {
        const fv b = *reinterpret_cast<const fv*>(B + ((long)r * N + cc) * 2);
#pragma unroll
        for (int m = 0; m < MR; ++m) {
            if (m < M) {
                const double pc = ut[2 * ((long)m * K + r)], ps = ut[2 * ((long)m * K + r) + 1];
#pragma unroll
                for (int h = 0; h < CPT; ++h) {
                    // two FMAs into the accumulator per real part (the
                    // expression acc + (p b - q c) costs a product, an FMA and
                    // an add)
                    const double br = b[2 * h], bi = b[2 * h + 1];
                    ar[h][m] = fma(-ps, bi, fma(pc, br, ar[h][m]));
                    ai[h][m] = fma(ps, br, fma(pc, bi, ai[h][m]));
                }
            }
        }
    }
    if (!ok) return;
#pragma unroll
    for (int h = 0; h < CPT; ++h)
#pragma unroll
        for (int m = 0; m < MR; ++m)
            if (m < M) *reinterpret_cast<double2*>(C + ((long)m * N + col + h) * 2) = double2{ar[h][m], ai[h][m]};
}

// Phase table of one point set against a vector list: tab[m][r] =
// (cos, sin)(2 pi x_m . n_r), the argument reduced in FP64 as in the sums.
__global__ void k_phase_table(int M, int K, const double* __restrict__ x, const int32_t* __restrict__ nvec,
                              double2* __restrict__ tab) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)M * K) return;
    const int m = (int)(t / K), r = (int)(t % K);
    double c, s;
    phase_of(reduced_arg(x[3L * m], x[3L * m + 1], x[3L * m + 2], nvec + 3L * r), c, s);
    tab[t] = double2{c, s};
}

inline void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{-3, std::string(what) + ": " + hipGetErrorString(e)};
}

}  // namespace

// Column blocks per workgroup: as many as the output width uses, up to 8.
static int pick_cb(int N, int cap) {
    if (N <= 48) return 3;
    if (N <= 64 || cap <= 4) return 4;
    return 8;
}

void phase_gemm_f64(int M, int N, int K, int Z, const double* x, const double* x0, const int32_t* nvec,
                    const double* B, long sB, double* C, long sC, hipStream_t st) {
    if (M <= 0 || N <= 0 || Z <= 0) return;
    const int cb = pick_cb(N, 4);
    dim3 grid((N + 16 * cb - 1) / (16 * cb), (M + kBM - 1) / kBM, Z);
    if (cb == 3)
        hipLaunchKernelGGL((k_phase_gemm<double, 3>), grid, dim3(256), 0, st, M, N, K, x, x0, nvec, B, sB, C, sC, 0);
    else
        hipLaunchKernelGGL((k_phase_gemm<double, 4>), grid, dim3(256), 0, st, M, N, K, x, x0, nvec, B, sB, C, sC, 0);
    check_launch("phase_gemm_f64");
}

void phase_gemm_f64_b32(int M, int N, int K, int Z, const double* x, const double* x0, const int32_t* nvec,
                        const float* B, long sB, double* C, long sC, double* tab, hipStream_t st) {
    if (M <= 0 || N <= 0 || Z <= 0) return;
    if (M <= 8 && N % 2 == 0 && tab != nullptr && x0 == nullptr && Z == 1 && K > 0) {
        // a k batch of at most 8 (and an even column count): the rows' phases
        // once into a table, then one streaming pass over B (k_re_sum_b32)
        const long nt = (long)M * K;
        hipLaunchKernelGGL(k_phase_table, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, M, K, x, nvec,
                           reinterpret_cast<double2*>(tab));
        const long nb = ((long)N + 511) / 512;
        if (nb > 0x7fffffffL) throw Error{-1, "phase_gemm_f64_b32: grid too large"};
        hipLaunchKernelGGL((k_re_sum_b32<8, 2>), dim3((unsigned)nb), dim3(256), 0, st, M, (long)N, K,
                           reinterpret_cast<const double2*>(tab), B, C);
    } else if (M <= 16) {
        // a k batch of at most 16: 16-row tiles, the waves along the columns
        dim3 grid((N + 255) / 256, 1, Z);
        hipLaunchKernelGGL((k_phase_gemm<double, 4, false, false, false, float, true>), grid, dim3(256), 0, st, M, N,
                           K, x, x0, (const void*)nvec, B, sB, C, sC, 0);
    } else {
        dim3 grid((N + 63) / 64, (M + kBM - 1) / kBM, Z);
        hipLaunchKernelGGL((k_phase_gemm<double, 4, false, false, false, float>), grid, dim3(256), 0, st, M, N, K, x,
                           x0, (const void*)nvec, B, sB, C, sC, 0);
    }
    check_launch("phase_gemm_f64_b32");
}

void phase_gemm_adj_f64(int M, int N, int K, int Z, const double* x, const double* kpts, const double* B, long sB,
                        double* C, long sC, int accumulate, hipStream_t st) {
    if (M <= 0 || N <= 0 || Z <= 0 || K <= 0) return;
    dim3 grid((N + 63) / 64, (M + kBM - 1) / kBM, Z);
    if (accumulate)
        hipLaunchKernelGGL((k_phase_gemm<double, 4, false, true, true>), grid, dim3(256), 0, st, M, N, K, x,
                           (const double*)nullptr, (const void*)kpts, B, sB, C, sC, 0);
    else
        hipLaunchKernelGGL((k_phase_gemm<double, 4, false, true, false>), grid, dim3(256), 0, st, M, N, K, x,
                           (const double*)nullptr, (const void*)kpts, B, sB, C, sC, 0);
    check_launch("phase_gemm_adj_f64");
}

void phase_gemm_herm_f64(int M, int N, int Kh, int Z, const double* x, const double* x0, const int32_t* nvec,
                         const double* B, double* C, long sC, hipStream_t st) {
    if (M <= 0 || N <= 0 || Z <= 0) return;
    dim3 grid((N + 63) / 64, (M + kBM - 1) / kBM, Z);
    hipLaunchKernelGGL((k_phase_gemm<double, 4, true>), grid, dim3(256), 0, st, M, N, Kh, x, x0, nvec, B, 0L, C, sC, 0);
    check_launch("phase_gemm_herm_f64");
}

void fold_herm_f64(int nk, const double* kpts, int Kh, const int32_t* nvec, int P, const double* hpack, double* out,
                   hipStream_t st) {
    const long total = (long)Kh * nk * P;
    if (total <= 0) return;
    hipLaunchKernelGGL(k_fold_herm, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, nk, kpts, Kh, nvec, P,
                       hpack, out);
    check_launch("fold_herm_f64");
}

void phase_gemm_herm_groups_f64(int M, int nk, int P, int Kh, const double* x, const int32_t* nvec, const double* B,
                                double* C, double* tab, hipStream_t st) {
    if (M <= 0 || nk <= 0 || Kh <= 0) return;
    if (P <= 0 || P % 2 != 0) throw Error{-1, "phase_gemm_herm_groups_f64: P must be even"};
    const int cg = P / 2, N = nk * cg;
    // the rows' phases once (every column block of the launch reads them)
    const long nt = (long)M * Kh;
    hipLaunchKernelGGL(k_phase_table, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, M, Kh, x, nvec,
                       reinterpret_cast<double2*>(tab));
    // column blocks fastest: the 8 XCDs take the blocks in turn, so each XCD
    // reads the coefficients of a fixed subset of the k
    dim3 grid((N + 63) / 64, (M + kBM - 1) / kBM, 1);
    hipLaunchKernelGGL((k_phase_gemm<double, 4, true, false, false, double, false, true>), grid, dim3(256), 0, st, M,
                       N, Kh, x, (const double*)tab, nvec, B, 0L, C, 0L, cg);
    check_launch("phase_gemm_herm_groups_f64");
}

void phase_gemm_f32(int M, int N, int K, int Z, const double* x, const double* x0, const int32_t* nvec,
                    const float* B, long sB, float* C, long sC, hipStream_t st) {
    if (M <= 0 || N <= 0 || Z <= 0) return;
    const int cb = pick_cb(N, 8);
    dim3 grid((N + 16 * cb - 1) / (16 * cb), (M + kBM - 1) / kBM, Z);
    if (cb == 3)
        hipLaunchKernelGGL((k_phase_gemm<float, 3>), grid, dim3(256), 0, st, M, N, K, x, x0, nvec, B, sB, C, sC, 0);
    else if (cb == 4)
        hipLaunchKernelGGL((k_phase_gemm<float, 4>), grid, dim3(256), 0, st, M, N, K, x, x0, nvec, B, sB, C, sC, 0);
    else
        hipLaunchKernelGGL((k_phase_gemm<float, 8>), grid, dim3(256), 0, st, M, N, K, x, x0, nvec, B, sB, C, sC, 0);
    check_launch("phase_gemm_f32");
}

void phase_gemm_bf16(int nsplit, int f16, int M, int N, int K, int Kp, int Z, const double* x, const double* x0,
                     const int32_t* nvec, const uint16_t* Bs, long sB, float* C, long sC, float oscale,
                     hipStream_t st) {
    if (M <= 0 || N <= 0 || Z <= 0) return;
    if (Kp % kBK != 0 || Kp < K) throw Error{-1, "phase_gemm_bf16: bad Kp"};
    if (nsplit != 2 && nsplit != 3) throw Error{-1, "phase_gemm_bf16: nsplit must be 2 or 3"};
    if (f16 && nsplit != 2) throw Error{-1, "phase_gemm_bf16: fp16 parts need nsplit 2"};
    const int cb = pick_cb(N, 8);
    dim3 grid((N + 16 * cb - 1) / (16 * cb), (M + kBM - 1) / kBM, Z);
#define EPHX_BF(CBV, NSV, F16V)                                                                                      \
    hipLaunchKernelGGL((k_phase_gemm_bf16<CBV, NSV, F16V>), grid, dim3(256), 0, st, M, N, K, Kp, x, x0, nvec, Bs, sB, \
                       C, sC, oscale)
    if (f16) {
        if (cb == 3) EPHX_BF(3, 2, true);
        else if (cb == 4) EPHX_BF(4, 2, true);
        else EPHX_BF(8, 2, true);
    } else if (nsplit == 2) {
        if (cb == 3) EPHX_BF(3, 2, false);
        else if (cb == 4) EPHX_BF(4, 2, false);
        else EPHX_BF(8, 2, false);
    } else {
        if (cb == 3) EPHX_BF(3, 3, false);
        else if (cb == 4) EPHX_BF(4, 3, false);
        else EPHX_BF(8, 3, false);
    }
#undef EPHX_BF
    check_launch("phase_gemm_bf16");
}

void phase_planes_bf16(int nsplit, int f16, int M, int K, int Kp, const double* x, const int32_t* nvec,
                       uint16_t* out, hipStream_t st) {
    if (M <= 0) return;
    if (Kp % kBK != 0 || Kp < K) throw Error{-1, "phase_planes_bf16: bad Kp"};
    if (f16 && nsplit != 2) throw Error{-1, "phase_planes_bf16: fp16 parts need nsplit 2"};
    const long total = (long)M * (Kp / 8);
    dim3 grid((unsigned)((total + 255) / 256));
    if (f16)
        hipLaunchKernelGGL((k_phase_planes<2, true>), grid, dim3(256), 0, st, M, K, Kp, x, nvec, out);
    else if (nsplit == 2)
        hipLaunchKernelGGL((k_phase_planes<2, false>), grid, dim3(256), 0, st, M, K, Kp, x, nvec, out);
    else if (nsplit == 3)
        hipLaunchKernelGGL((k_phase_planes<3, false>), grid, dim3(256), 0, st, M, K, Kp, x, nvec, out);
    else
        throw Error{-1, "phase_planes_bf16: nsplit must be 2 or 3"};
    check_launch("phase_planes_bf16");
}

void gemm_bf16_planes(int nsplit, int f16, int M, int N, int Kp, int Z, const uint16_t* A, const uint16_t* Bs,
                      long sB, float* C, long sC, int real_a, float oscale, hipStream_t st) {
    if (M <= 0 || N <= 0 || Z <= 0) return;
    if (Kp <= 0 || Kp % kBK != 0) throw Error{-1, "gemm_bf16_planes: bad Kp"};
    if (nsplit != 2 && nsplit != 3) throw Error{-1, "gemm_bf16_planes: nsplit must be 2 or 3"};
    if (f16 && nsplit != 2) throw Error{-1, "gemm_bf16_planes: fp16 parts need nsplit 2"};
    // three-product real-A forms where 128 divides N and the rows fill a tile:
    // 256 x 128 tiles of eight waves (two per SIMD, one 32-row tile each; with
    // fewer rows the idle waves would share the matrix pipe with the working
    // ones); measured at the Si-like shape
    // 0.35 -> 0.42 of the ceiling against 256 x 96 tiles of four waves with two
    // row tiles each (one wave per SIMD), and 0.40 for 128 x 96 tiles of four
    // waves (two workgroups per CU)
    const bool wide8 = real_a && nsplit == 2 && N > 64 && N % 128 == 0 && M >= 256;
    // real A otherwise: 96-column tiles where they divide N (72 KB of LDS for
    // BF16x6, two workgroups per CU)
    const int ct = wide8 ? 4 : (N <= 64 ? 2 : (real_a && N % 96 == 0 ? 3 : 4));
    // two 32-row tiles per wave for the other three-product real-A forms
    const int rtw = !wide8 && real_a && nsplit == 2 ? 2 : 1;
    const int nwv = wide8 ? 8 : 4;
    const int nbx = (N + 32 * ct - 1) / (32 * ct), nby = (M + 32 * nwv * rtw - 1) / (32 * nwv * rtw);
    const long nblk = (long)nbx * nby * Z;
    if (nblk > 0x7fffffffL) throw Error{-1, "gemm_bf16_planes: grid too large"};
    dim3 grid((unsigned)nblk);
#define EPHX_BFP(CTV, NSV, RAV, F16V, RTV)                                                                           \
    hipLaunchKernelGGL((k_gemm_bf16_planes<CTV, NSV, RAV, F16V, RTV>), grid, dim3(256), 0, st, M, N, Kp, nbx, nby, Z, \
                       A, Bs, sB, C, sC, oscale)
#define EPHX_BFP_CT(NSV, RAV, F16V, RTV)                \
    do {                                                \
        if (ct == 2) EPHX_BFP(2, NSV, RAV, F16V, RTV);       \
        else if (ct == 3) EPHX_BFP(3, NSV, RAV, F16V, RTV);  \
        else EPHX_BFP(4, NSV, RAV, F16V, RTV);               \
    } while (0)
    if (wide8) {
        if (f16)
            hipLaunchKernelGGL((k_gemm_bf16_planes<4, 2, true, true, 1, 8>), grid, dim3(512), 0, st, M, N, Kp, nbx,
                               nby, Z, A, Bs, sB, C, sC, oscale);
        else
            hipLaunchKernelGGL((k_gemm_bf16_planes<4, 2, true, false, 1, 8>), grid, dim3(512), 0, st, M, N, Kp, nbx,
                               nby, Z, A, Bs, sB, C, sC, oscale);
    } else if (f16) {
        if (real_a) EPHX_BFP_CT(2, true, true, 2);
        else EPHX_BFP_CT(2, false, true, 1);
    } else if (real_a) {
        if (nsplit == 2) EPHX_BFP_CT(2, true, false, 2);
        else EPHX_BFP_CT(3, true, false, 1);
    } else {
        if (nsplit == 2) EPHX_BFP_CT(2, false, false, 1);
        else EPHX_BFP_CT(3, false, false, 1);
    }
#undef EPHX_BFP_CT
#undef EPHX_BFP
    check_launch("gemm_bf16_planes");
}

void half_combine_f64(int Z, int K, int N, int Kh, const int32_t* pair, const double* G, double* out, hipStream_t st) {
    const long total = (long)Kh * N;
    if (total <= 0 || Z <= 0) return;
    dim3 grid((unsigned)((total + 255) / 256), 1, Z);
    hipLaunchKernelGGL(k_half_combine<double>, grid, dim3(256), 0, st, K, N, Kh, pair, G, out);
    check_launch("half_combine_f64");
}

void half_combine_f32(int Z, int K, int N, int Kh, const int32_t* pair, const double* G, float* out, hipStream_t st) {
    const long total = (long)Kh * N;
    if (total <= 0 || Z <= 0) return;
    dim3 grid((unsigned)((total + 255) / 256), 1, Z);
    hipLaunchKernelGGL(k_half_combine<float>, grid, dim3(256), 0, st, K, N, Kh, pair, G, out);
    check_launch("half_combine_f32");
}

void split_bf16_half(int nsplit, int f16, double scale, int Z, int K, int N, int Kh, int Kh16, const int32_t* pair,
                     const double* G, uint16_t* out, hipStream_t st) {
    if (Kh16 % 16 != 0 || Kh16 < Kh) throw Error{-1, "split_bf16_half: bad Kh16"};
    if (f16 && nsplit != 2) throw Error{-1, "split_bf16_half: fp16 parts need nsplit 2"};
    const long total = (long)N * 2 * Kh16;
    if (total <= 0 || Z <= 0) return;
    dim3 grid((unsigned)((total + 255) / 256), 1, Z);
    if (f16)
        hipLaunchKernelGGL((k_split_bf16_half<2, true>), grid, dim3(256), 0, st, K, N, Kh, Kh16, scale, pair, G, out);
    else if (nsplit == 2)
        hipLaunchKernelGGL((k_split_bf16_half<2, false>), grid, dim3(256), 0, st, K, N, Kh, Kh16, scale, pair, G, out);
    else if (nsplit == 3)
        hipLaunchKernelGGL((k_split_bf16_half<3, false>), grid, dim3(256), 0, st, K, N, Kh, Kh16, scale, pair, G, out);
    else
        throw Error{-1, "split_bf16_half: nsplit must be 2 or 3"};
    check_launch("split_bf16_half");
}

void phase_planes_half(int nsplit, int f16, int M, int Kh, int Kh16, const double* x, const int32_t* nvec,
                       uint16_t* out, hipStream_t st) {
    if (M <= 0) return;
    if (Kh16 % 16 != 0 || Kh16 < Kh) throw Error{-1, "phase_planes_half: bad Kh16"};
    if (f16 && nsplit != 2) throw Error{-1, "phase_planes_half: fp16 parts need nsplit 2"};
    const long total = (long)M * (Kh16 / 8);
    dim3 grid((unsigned)((total + 255) / 256));
    if (f16)
        hipLaunchKernelGGL((k_phase_planes_half<2, true>), grid, dim3(256), 0, st, M, Kh, Kh16, x, nvec, out);
    else if (nsplit == 2)
        hipLaunchKernelGGL((k_phase_planes_half<2, false>), grid, dim3(256), 0, st, M, Kh, Kh16, x, nvec, out);
    else if (nsplit == 3)
        hipLaunchKernelGGL((k_phase_planes_half<3, false>), grid, dim3(256), 0, st, M, Kh, Kh16, x, nvec, out);
    else
        throw Error{-1, "phase_planes_half: nsplit must be 2 or 3"};
    check_launch("phase_planes_half");
}

void phase_gemm_half_f64(int M, int N, int Kh, int Z, const double* x, const int32_t* nvec, const double* B, long sB,
                         double* C, long sC, hipStream_t st) {
    if (M <= 0 || N <= 0 || Z <= 0) return;
    dim3 grid((N + 63) / 64, (M + kBM - 1) / kBM, Z);
    hipLaunchKernelGGL((k_phase_gemm<double, 4, true>), grid, dim3(256), 0, st, M, N, Kh, x, (const double*)nullptr,
                       nvec, B, sB, C, sC, 0);
    check_launch("phase_gemm_half_f64");
}

void phase_gemm_half_f32(int M, int N, int Kh, int Z, const double* x, const int32_t* nvec, const float* B, long sB,
                         float* C, long sC, hipStream_t st) {
    if (M <= 0 || N <= 0 || Z <= 0) return;
    const int cb = pick_cb(N, 8);
    dim3 grid((N + 16 * cb - 1) / (16 * cb), (M + kBM - 1) / kBM, Z);
    if (cb == 3)
        hipLaunchKernelGGL((k_phase_gemm<float, 3, true>), grid, dim3(256), 0, st, M, N, Kh, x, (const double*)nullptr,
                           nvec, B, sB, C, sC, 0);
    else if (cb == 4)
        hipLaunchKernelGGL((k_phase_gemm<float, 4, true>), grid, dim3(256), 0, st, M, N, Kh, x, (const double*)nullptr,
                           nvec, B, sB, C, sC, 0);
    else
        hipLaunchKernelGGL((k_phase_gemm<float, 8, true>), grid, dim3(256), 0, st, M, N, Kh, x, (const double*)nullptr,
                           nvec, B, sB, C, sC, 0);
    check_launch("phase_gemm_half_f32");
}

void split_bf16_f64(int nsplit, int f16, double scale, int Z, int K, int N, int Kp, const double* B, uint16_t* out,
                    hipStream_t st) {
    if (f16 && nsplit != 2) throw Error{-1, "split_bf16_f64: fp16 parts need nsplit 2"};
    const long total = (long)N * Kp;
    dim3 grid((unsigned)((total + 255) / 256), 1, Z);
    if (f16)
        hipLaunchKernelGGL((k_split_bf16<2, true>), grid, dim3(256), 0, st, K, N, Kp, scale, B, out);
    else if (nsplit == 2)
        hipLaunchKernelGGL((k_split_bf16<2, false>), grid, dim3(256), 0, st, K, N, Kp, scale, B, out);
    else
        hipLaunchKernelGGL((k_split_bf16<3, false>), grid, dim3(256), 0, st, K, N, Kp, scale, B, out);
    check_launch("split_bf16");
}

}  // namespace ephx
