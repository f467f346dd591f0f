// Internal declarations shared by the host API and the kernel files of the
// electron-phonon library.  Not part of the public ABI (see include/ephx.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace ephx {

// Physical constants (CODATA 2018); energies in eV, time in fs.
constexpr double kHbarEvFs = 0.6582119569;              // hbar, eV*fs
constexpr double kBoltzEv = 8.617333262e-5;             // k_B, eV/K
constexpr double kHbar2AmuA2 = 0.004180159280496722;    // hbar^2/(amu*A^2), eV
constexpr double kE2Over4PiEps0 = 14.3996454784;        // e^2/(4 pi eps0), eV*A
constexpr double kPi = 3.14159265358979323846;
// The BTE table matrices take the Gaussian delta as zero beyond 6 sigma
// ((x/sigma)^2 > 36, a factor e^-36 below the peak), so that tiles of state
// pairs further apart in energy than the largest phonon plus 6 sigma are exact
// zeros and need not be stored or read.
constexpr double kDeltaCut2 = 36.0;
constexpr double kDegTol = 1e-4;                        // degenerate-group threshold, eV

constexpr int kMaxNw = 16;      // Wannier functions handled by the per-pair kernels
constexpr int kMaxModes = 12;   // 3*natoms handled by the per-pair kernels
constexpr int kEigMax = 8;      // largest matrix of the one-lane eigensolver (eig_ql.h)
constexpr int kMaxNwWide = 64;  // Wannier functions of the batched-GEMM path
constexpr int kMaxModesWide = 126;   // 3*natoms of the batched-GEMM path (eigensolver n <= 128)

// Thrown inside the host code, converted to an error code at the ABI edge.
struct Error {
    int code;
    std::string msg;
};

// ------------------------------------------------------------------ launchers
// Phase contractions  C[z][m][n] = sum_r exp(2 pi i (x_m + x0_z) . n_r) B[z][r][n]
// (complex interleaved).  x: [M][3] reduced coordinates (device), x0: [Z][3] or
// nullptr, nvec: [K][3] int32 (device), B stride sB and C stride sC in complex
// elements per z.
void phase_gemm_f64(int M, int N, int K, int Z, const double* x, const double* x0,
                    const int32_t* nvec, const double* B, long sB, double* C, long sC,
                    hipStream_t st);
// Adjoint sums C[z][m][n] (+)= sum_k exp(2 pi i x_m . p_k) B[z][k][n] with real
// points on both sides (x: [M][3], p: [K][3]), FP64.
void phase_gemm_adj_f64(int M, int N, int K, int Z, const double* x, const double* kpts, const double* B,
                        long sB, double* C, long sC, int accumulate, hipStream_t st);
// Hermitian Fourier sum over a half set (see phase_gemm.hip): B = [Kh][2][N] complex
// (A_r, B_r), real coefficients cos/sin of 2 pi (x_m + x0_z).n_r; B shared by all z.
void phase_gemm_herm_f64(int M, int N, int Kh, int Z, const double* x, const double* x0,
                         const int32_t* nvec, const double* B, double* C, long sC, hipStream_t st);
// H(k+q) for every (k, q) of a batch in the packed Hermitian form (n*n reals,
// P[i][j] = Re H_ij for i <= j, Im H_ji for i > j), two steps:
//  fold_herm_f64: hpack [Kh][2][P] (packed A_r, B_r; P = n*n rounded up to even)
//    -> out [Kh][2][nk][P], the coefficients of the sum at k + q as a sum over q;
//  phase_gemm_herm_groups_f64: C [nk][M][P] = sum_r cos/sin(2 pi x_m.n_r) out_r,
//    one phase per (m, r) for all nk matrices (B given as [Kh][2][nk*P/2] complex);
//    tab: work buffer of M * Kh * 16 bytes (the phase table).
void fold_herm_f64(int nk, const double* kpts, int Kh, const int32_t* nvec, int P, const double* hpack, double* out,
                   hipStream_t st);
void phase_gemm_herm_groups_f64(int M, int nk, int P, int Kh, const double* x, const int32_t* nvec, const double* B,
                                double* C, double* tab, hipStream_t st);
// phase_gemm_f64 with a complex-float B (FP64 arithmetic; B widened on load).
// tab (M*K complex doubles of work memory, or nullptr): with M <= 16, Z = 1
// and no x0 the rows' phases are formed there once per call.
void phase_gemm_f64_b32(int M, int N, int K, int Z, const double* x, const double* x0, const int32_t* nvec,
                        const float* B, long sB, double* C, long sC, double* tab, hipStream_t st);
void phase_gemm_f32(int M, int N, int K, int Z, const double* x, const double* x0,
                    const int32_t* nvec, const float* B, long sB, float* C, long sC,
                    hipStream_t st);
// Split-bf16 contraction: B given as 2*nsplit bf16 planes [Z][2*nsplit][N][Kp]
// (re parts then im parts), Kp % 32 == 0; nsplit 2 = BF16x3, 3 = BF16x6.
// f16 = 1 (nsplit 2): fp16 parts instead ("FP16x3"), B scaled by a power of two
// when split and the output multiplied by oscale, its inverse (1 for bf16).
void phase_gemm_bf16(int nsplit, int f16, int M, int N, int K, int Kp, int Z, const double* x, const double* x0,
                     const int32_t* nvec, const uint16_t* Bs, long sB, float* C, long sC, float oscale,
                     hipStream_t st);
// Split-bf16 phase planes [2*nsplit][M][Kp] of exp(2 pi i x_m . n_r) (cos parts
// then sin parts), and the contraction C[z] = A B[z] that reads them.
void phase_planes_bf16(int nsplit, int f16, int M, int K, int Kp, const double* x, const int32_t* nvec,
                       uint16_t* out, hipStream_t st);
// real_a = 1: A is real, [nsplit][M][Kp] (half-set cos and sin parts along k).
void gemm_bf16_planes(int nsplit, int f16, int M, int N, int Kp, int Z, const uint16_t* A, const uint16_t* Bs,
                      long sB, float* C, long sC, int real_a, float oscale, hipStream_t st);
// Half-set form of a Fourier sum over a list closed under R -> -R apart from
// unpaired vectors (see phase_gemm.hip): pair [Kh][2] = (index of R_h, index of
// -R_h or -1) into the list, G [Z][K][N] complex double.
//  half_combine_*: [Z][Kh][2][N] complex coefficients (Gc_h, Gs_h);
//  phase_gemm_half_*: C[z] = sum_h cos(2 pi x.R_h) Gc_h + sin(2 pi x.R_h) Gs_h,
//    B = those coefficients (stride sB complex per z), nvec = the R_h;
//  split_bf16_half / phase_planes_half: split-bf16 planes of the coefficients
//    [Z][2 nsplit][N][2 Kh16] and of the real phases [nsplit][M][2 Kh16] for
//    gemm_bf16_planes with real_a = 1 (Kh16 = Kh rounded up to 16).
void half_combine_f64(int Z, int K, int N, int Kh, const int32_t* pair, const double* G, double* out, hipStream_t st);
void half_combine_f32(int Z, int K, int N, int Kh, const int32_t* pair, const double* G, float* out, hipStream_t st);
void phase_gemm_half_f64(int M, int N, int Kh, int Z, const double* x, const int32_t* nvec, const double* B, long sB,
                         double* C, long sC, hipStream_t st);
void phase_gemm_half_f32(int M, int N, int Kh, int Z, const double* x, const int32_t* nvec, const float* B, long sB,
                         float* C, long sC, hipStream_t st);
void split_bf16_half(int nsplit, int f16, double scale, int Z, int K, int N, int Kh, int Kh16, const int32_t* pair,
                     const double* G, uint16_t* out, hipStream_t st);
void phase_planes_half(int nsplit, int f16, int M, int Kh, int Kh16, const double* x, const int32_t* nvec,
                       uint16_t* out, hipStream_t st);
// Split complex double B[Z][K][N], times scale, into those planes.
void split_bf16_f64(int nsplit, int f16, double scale, int Z, int K, int N, int Kp, const double* B, uint16_t* out,
                    hipStream_t st);

// Hermitian eigensolver in FP64: n <= kEigMax by wavefronts (64/n-ish matrices
// each), 8 < n <= 128 by one workgroup per matrix.  A: [batch] matrices of n*n
// complex (stride strideA complex elements), float (a_f32 = 1, n <= 8 only) or
// double; for n > 8 A is overwritten.  evals [batch][n] ascending; evecs
// [batch][n][n] complex double (column j = eigenvector j) or nullptr.
void eig_herm(int batch, int n, void* A, int a_f32, long strideA, double* evals, double* evecs, hipStream_t st);
// The same for n <= 8 from the packed Hermitian form: n*n reals per matrix
// (stride strideP reals), P[i][j] = Re X_ij for i <= j, Im X_ji for i > j;
// evecs_cm = 1 stores each matrix's eigenvectors column-major (eigenvector j
// at [j][0..n), contiguous).
void eig_herm_packed(int batch, int n, const double* P, long strideP, double* evals, double* evecs, int evecs_cm,
                     hipStream_t st);

// omega_nu = sign(lam) sqrt(|hbar^2/amu/A^2 * lam|) in place.
void phonon_omega(long count, double* lam, hipStream_t st);

// g'(z)[p][x][i][n] = sum_j g(z)[p][x][i][j] U(z)[j][n]; complex double in and out.
void apply_u_right(int Z, int nrp, int nm, int nw, const double* g, const double* u,
                   double* out, hipStream_t st);
void convert_f64_f32(long count, const double* in, float* out, hipStream_t st);
// out[0] = bit pattern of max over the rows r of sum_{e,j} |w[e][r / rows_per_rp] g[e][r][j]|
// for complex g [n_re][rows][nw] (w [n_re][n_rp], or nullptr for 1); out[1] != 0 if
// an entry is not finite (out cleared first)
void g_row_bound(int n_re, long rows, int nw, const double* g, const double* w, long rows_per_rp, int n_rp,
                 unsigned long long* out, hipStream_t st);
// the same bound for complex float g [n_re][rows][nw] with unit weights
void g_row_bound_f32(int n_re, long rows, int nw, const float* g, unsigned long long* out, hipStream_t st);
// g(Re,Rp) [n_re][n_rp][per] complex float drawn by the counter scheme
// (Philox4x32-10, Irwin-Hall twelve-word variates) with amplitudes env [n_re][n_rp]
void gen_coupling(int n_re, int n_rp, long per, unsigned long long seed, const double* env, float* out,
                  hipStream_t st);
// dst[i] += src[i], i < n
void add_into(long n, const double* src, double* dst, hipStream_t st);
// data[r][c] *= w[r] for complex data [rows][cols]
void scale_rows(long rows, long cols, const double* w, double* data, hipStream_t st);
// out(z)[p][x][i][j] = sum_n g'(z)[p][x][i][n] conj(U(z)[j][n])   (adjoint of apply_u_right)
void apply_u_right_adj(int Z, int nrp, int nm, int nw, const double* g, const double* u, double* out,
                       hipStream_t st);


struct EphEpilogue {
    int nkb;            // k points in the batch (grid.y)
    int nq;             // q points in the chunk
    int q_off;          // global index of the first q of the chunk
    int nw, nm;
    const void* gw;     // [nkb][nq][nm][nw][nw] complex (float or double)
    const double* ukq;  // [nkb][nq][nw][nw] complex
    int u_cm;           // 1: each U(k+q) stored column-major ([m][i], eigenvector m contiguous)
    const double* ekq;  // [nkb][nq][nw]
    const double* ek;   // [nkb][nw]
    const double* uk;   // [nkb][nw][nw] complex (polar term)
    const double* omega;  // [nq_total][nm]
    const double* evec;   // [nq_total][nm][nm] complex
    const double* lr;     // [nq_total][nm] complex long-range term, or nullptr
    const double* minv;   // [nm] 1/sqrt(M_kappa)
    double omega_cut;
    // per-q and per-pair factors formed once by eph_epilogue_factors (nullptr:
    // the epilogue forms them per pair)
    const void* esq;      // [nq][nm][nm] complex (float or double): e[x][nu] sqrt(hbar^2/(2 M_x omega_nu))
    const double* nbq;    // [nq][nm] Bose factors
    const double* fkq;    // [nkb][nq][nw] Fermi factors of the k+q states (rates mode)
    // |g|^2 output mode
    void* g2;            // [nk_total][nq_total][nm][nw][nw]
    long nq_total;
    int k_off;
    // rates mode
    double temp, mu, sigma;
    const double* qw;    // [nq_total] or nullptr (then uniform_w)
    double uniform_w;
    double* partial;     // [nkb][nblk][nw][nm]
    int nblk;
    // rates of a part of |g|^2 (polar models): 0 all of it, 1 the long-range
    // coupling alone |g_L|^2, 2 the rest |g|^2 - |g_L|^2
    int part;
};
void eph_epilogue_g2(const EphEpilogue& e, int f32, hipStream_t st);
// The per-q mode factors (esq, nbq) of the chunk, and with fkq != nullptr the
// Fermi factors of its pairs, into the buffers e points at.
void eph_epilogue_factors(const EphEpilogue& e, int f32, void* esq, double* nbq, double* fkq, hipStream_t st);
// per pair: gw_bar[x][i][n] = sum_m U(k+q)_im sum_nu conj(es[x][nu]) 2 c lam_n w_q D_mnu g_mnu (FP64)
void eph_adjoint_epilogue(const EphEpilogue& e, const double* lam, double* gw_bar, hipStream_t st);
void eph_epilogue_rates(const EphEpilogue& e, int f32, hipStream_t st);
int eph_epilogue_blocks(int nq);
// dst[j][0..2] = src[idx[j]][0..2] (double points)
void gather_points(int n, const int32_t* idx, const double* src, double* dst, hipStream_t st);
// block pos[j] of dst = block j of src, blocks of `words` 32-bit words
void scatter_blocks(int n, const int32_t* pos, const void* src, void* dst, long words, hipStream_t st);
// acc[z][n][nu] += sum_b partial[z][b][n][nu]
void rates_reduce(int nkb, int nblk, int nw, int nm, const double* partial, double* acc,
                  hipStream_t st);
void rates_finish(int nkb, int nw, int nm, const double* acc, double* gamma, double* gamma_mode,
                  hipStream_t st);

// Large models (nw > kMaxNw or 3nat > kMaxModes): per-pair rotation and mode
// projection as batched complex GEMMs on MFMA (eph_wide.hip).
struct CBatch {                 // batch index b = b0 * n1 + b1; offsets in complex elements
    long n1;
    long sa0, sa1, sb0, sb1, sc0, sc1;
};
struct WideChunk {
    int nkb, nq, q_off, nw, nm;
    void* g;              // [nkb][nq][nm][nw][nw] Rp contraction (U(k) applied), overwritten by g_mn,nu
    void* gh;             // same size, work
    double* pmat;         // [nq][nm][nm] complex, work
    double* ov;           // [nkb][nq][nw][nw] complex, work (polar) or nullptr
    const double* ukq;    // [nkb][nq][nw][nw]
    const double* ekq;    // [nkb][nq][nw]
    const double* ek;     // [nkb][nw]
    const double* uk;     // [nkb][nw][nw]
    const double* omega;  // [nq_total][nm]
    const double* evec;   // [nq_total][nm][nm]
    const double* lr;     // [nq_total][nm] or nullptr
    const double* minv;
    double omega_cut;
    void* g2;             // |g|^2 output [nk_total][nq_total][nm][nw][nw]
    long nq_total;
    int k_off;
    double temp, mu, sigma;
    const double* qw;
    double uniform_w;
    double* partial;      // [nkb][nblk][nw][nm]
    int nblk, qpb;
};
void eph_wide_chunk(const WideChunk& w, int f32, int rates, hipStream_t st);
// C[b] = A[b] B[b] for a batch of complex FP64 matrices (row-major, strides of
// CBatch) on the FP64 matrix cores, 64 x 64 tiles
void cgemm_f64_batched(int M, int N, int K, long nbatch, const CBatch& b, const double* A, long lda, const double* B,
                       long ldb, double* C, long ldc, hipStream_t st);
// Adjoint of the rates of a chunk (FP64; w.g holds g'^W on entry and is work):
// gwbar [nkb][nq][nm][nw][nw] = dL/dg'^W for L = sum_nk lam_nk Gamma_nk.
void eph_wide_rates_vjp(const WideChunk& w, const double* lam, double* gwbar, hipStream_t st);

// Froehlich term: lr[q][3*kappa+a] (complex double) for q in [nq][3].
struct PolarDev {
    const double* bvec;   // [3][3] rows b_i
    const double* tau;    // [nat][3]
    const double* zstar;  // [nat][3][3]
    const double* eps;    // [3][3]
    double pref, alpha, gcut;
    int nat, mmax[3];
};
void frohlich(int nq, const double* q, const PolarDev& p, double* lr, hipStream_t st);
// D[q] += dipole-dipole part of the mass-scaled dynamical matrix (LO-TO);
// corr: [nat][3][3] complex q = 0 sum-rule term; D [nq][3nat][3nat] complex.
void dipole_add(int nq, const double* q, const PolarDev& p, const double* corr, const double* minv, double* D,
                hipStream_t st);

// Band velocities from H(k) derivatives: dh [nk][3][nw][nw] complex, u, eps -> vel [nk][nw][3]
void band_velocity(int nk, int nw, const double* dh, const double* u, const double* eps,
                   double* vel, hipStream_t st);

// ---------------------------------------------------------------- BTE side
struct PairEpilogue {
    int ns_chunk;         // sources in this chunk (grid.y)
    int s_off;            // global index of first source
    int S;                // states (targets)
    int nw, nm;
    const void* gw;       // [ns_chunk][S][nm][nw] complex (float or double)
    const double* ut;     // [S][nw][nw] complex, U(k_t)
    const int32_t* band;  // [S]
    const int32_t* kc;    // [S][3] grid coordinates
    int n1, n2, n3;
    const double* omega;  // [Ngrid][nm]
    const double* evec;   // [Ngrid][nm][nm] complex
    const double* lr;     // [Ngrid][nm] complex or nullptr
    const double* us;     // [S][nw][nw] complex, U(k_s) (polar term)
    const double* minv;
    double omega_cut;
    float* g2raw;         // set by the launcher for FP32 tables
};
// Adjoint of the table epilogue for the mobility gradient (see bte_kernels.hip).
struct PairAdjoint {
    int ns_chunk, s_off, S, nw, nm;
    const double* gw;         // [ns_chunk][S][nm][nw] complex, FP64 Rp contraction
    const double* ut;         // [S][nw][nw] complex, U(k) of the states
    const double* us;         // same array (polar overlap)
    const int32_t* band;
    const int32_t* kc;
    int n1, n2, n3;
    const double* omega;      // [Ngrid][nm]
    const double* evec;       // [Ngrid][nm][nm] complex
    const double* lr;         // [Ngrid][nm] complex or nullptr
    const double* minv;
    double omega_cut_table;   // cut of the table's |g|^2
    int n_hist;               // W_bar_st = (1/N_q)(sum_h ubar[h][s] fhist[h][t] + gamma_bar[s])
    const double* ubar;
    const double* fhist;
    const double* gamma_bar;
    double n_q;
    const double* eps;        // transport weights (as in the transport matrix)
    double temp, mu, sigma, omega_cut;
    double* gw_bar;           // [ns_chunk][S][nm][nw] complex
};
void pair_adjoint(const PairAdjoint& e, hipStream_t st);
// out[z][p][x][i][j] = exp(2 pi i k_s.Rp_p) in[z][p][x][i] conj(U(k_s)[j][band_s]), s = s_off + z
void apply_u_column_adj(int Z, int nrp, int nm, int nw, int s_off, const double* in, const double* ks,
                        const int32_t* rp, const double* us, const int32_t* band, double* out, hipStream_t st);
// reverse of the ITA (layouts [3][S])
void mob_seed(int S, const double* eps, const double* vel, const double* lam, double mu, double temp, double* fbar,
              hipStream_t st);
void ita_adj_step(int S, const double* tau, const double* fbar, const double* fnext, double* taubar, double* ubar,
                  int first, hipStream_t st);
void ita_adj_cols(int S, int n_rt, const double* colp, double n_q, double* fbar, hipStream_t st);
void ita_adj_final(int S, const double* tau, const double* fbar0, const double* vel, const double* taubar, int first,
                   double* gbar, hipStream_t st);
// Linear tetrahedron integration (tetra.hip): out[e][comp] = scale * sum_T (1/6)
// sum_j c_j(E_e) x[T_j][comp], nc <= 9 components; partial holds
// tetra_chunks(n_tet) * n_e * nc doubles.
int tetra_chunks(int n_tet);
void tetra_sum(int n_tet, const int32_t* tet, const double* eps, int nc, const double* x, int n_e, const double* egrid,
               double scale, double* partial, double* out, hipStream_t st);
void vf_products(int S, const double* vel, const double* ff, double* x, hipStream_t st);
// sigma (S/m) and Seebeck (V/K) from the TDF [n_e][3][3] by the trapezoid rule
void tdf_transport(int n_e, const double* egrid, const double* tdf, double mu, double temp, double sigma_unit,
                   double* sigma, double* seebeck, hipStream_t st);
// Leading dimension (elements) of S x S tables: rows start 256-byte aligned.
long table_ld(int S);
void pair_epilogue(const PairEpilogue& e, int f32, long ld, void* g2out, hipStream_t st);
// g'(s)[p][x][i] = sum_j g(s)[p][x][i][j] U(k_s)[j][band_s]
void apply_u_column(int Z, int nrp, int nm, int nw, const double* g, const double* us,
                    const int32_t* band, double* out, hipStream_t st);
void table_symmetrise(int nm, int S, long ld, void* g2, int f32, hipStream_t st);
// transport = 0: collision matrix P (mode scales applied);
// transport = 1: scattering probabilities W (Eq. BTE_W, 1/fs, scale ignored but required).
// Row/column i of out is state perm[i] (perm nullptr: identity).  Entries whose
// energy difference exceeds dcut > 0 (at least the largest phonon energy +
// 6 sigma) are written as zero without evaluating the sum; dcut <= 0: none.
void build_matrix(int transport, int S, int nm, long ld, const void* g2, int f32, const int32_t* kc,
                  int n1, int n2, int n3, const double* omega, const double* eps, double temp,
                  double mu, double sigma, double omega_cut, const double* scale, const int32_t* perm,
                  void* out, double dcut, hipStream_t st);

// Streaming pass over a dense S x S matrix P (row stride ld):
//   rowp[a][ct][s] = sum_{t in col tile ct} P[s][t] x_a[t]      (a < na)
//   colp[b][rt][t] = sum_{s in row tile rt} P[s][t] y_b[s]      (b < nb)
struct VecPtrs {
    const double* p[4];
};
// The plan fixes the kernel instance and its tiling; the finish kernels sum
// the n_ct row partials and n_rt column partials it produces.
// The matrix is stored in the state order `perm` (row/column i is state
// perm[i]) and only the listed tiles are launched: entries [0, n_live) are
// (column tile, row tile) pairs that are read, the rest are tiles known to
// hold only zeros, whose partials are written as 0 without reading the
// matrix.  A pass gathers the vectors into matrix order (gbuf), streams, and
// reduces the partials back into state order (rout [na][S], cout [nb][S]).
struct StreamPlan {
    int S;
    int f32, na, nb;      // matrix precision and vector counts
    int n_rt, n_ct;       // row and column tiles
    int rpb;              // rows per row tile
    const int32_t* tiles; // device [n_tiles][2]
    int n_live, n_tiles;
    const int32_t* perm;  // device [S]
    double* gbuf;         // device [na + nb][S]
    double* rout;         // device [na][S]
    double* cout;         // device [nb][S]
};
// Where the finishing kernels read a pass's results: n_ct row partials per
// row sum and n_rt column partials per column sum, in state order.
struct PassOut {
    const double* rowp;
    int n_ct;
    const double* colp;
    int n_rt;
};
constexpr int kStreamTileCols = 1024;   // columns per tile of the streaming pass
StreamPlan stream_plan(int S, int f32, int na, int nb);
// Tiling of a matrix stored in ascending-energy order (esort[i] = energy of
// row/column i) whose entries vanish where the two energies differ by more
// than half_width: row tiles are made as small as keeps the live tiles within
// one resident wave of blocks.  tiles receives the host tile list, live first.
StreamPlan stream_plan_banded(int S, int f32, int na, int nb, const std::vector<double>& esort, double half_width,
                              std::vector<int32_t>& tiles, int& n_live);
// One pass = gather the vectors into matrix order, stream the live tiles into
// partials (matrix order), reduce the partials into state order.
void stream_gather(const StreamPlan& pl, VecPtrs x, VecPtrs y, hipStream_t st);
void stream_run(const StreamPlan& pl, long ld, const void* P, double* rowp, double* colp, hipStream_t st);
PassOut stream_reduce(const StreamPlan& pl, const double* rowp, const double* colp, hipStream_t st);
// I_s = -c [ f_s R_s - (1-f_s) C_s ] with R, C the reduced partials; optional
// RK4 stage update: acc = (acc_init ? f_base : acc) + w_acc * I ; f_next = f_base + a_next * I.
struct CollisionFinish {
    int S;
    int n_rt, n_ct;
    const double* rowp;   // [n_ct][S]
    const double* colp;   // [n_rt][S]
    const double* f;      // occupations the integral is evaluated at
    double c;             // (2 pi/hbar)/N_q
    double* i_out;        // I (may be nullptr)
    double* acc;          // stage accumulator (nullptr: no update)
    int acc_init;
    double w_acc;
    const double* f_base;
    double a_next;
    double* f_next;       // may be nullptr
    // field drift added to I in the stage update (not in i_out): nbr [S][6]
    // holds the +/- neighbour along each reduced direction (-1 = empty state),
    // dc[i] = (|e|/hbar)(E . a_i)/(2 pi) (N_i/2); nbr nullptr = no field
    const int32_t* nbr;
    double dc[3];
    // with gnext: the next pass's occupations gathered to matrix order
    // ([2][S]: 1 - v, v), v = the updated acc (gnext_acc) or f_next
    double* gnext;
    int gnext_acc;
};
// The collision pass of a 1+1 plan without the separate occupation, gather and
// reduction kernels: gather_occupations fills the plan's gather buffer with
// 1 - f and f in matrix order; reduce_finish takes the stream's unreduced
// matrix-order partials (cf.rowp [n_ct][S], cf.colp [n_rt][S]) to I and the
// stage update in state order.
void gather_occupations(const StreamPlan& pl, const double* f, hipStream_t st);
void reduce_finish(const StreamPlan& pl, const CollisionFinish& cf, hipStream_t st);
void vjp_finish(int S, int n_ct, int n_rt, const double* rowp, const double* colp, const double* lam, double c,
                double* fbar, hipStream_t st);
// sbar[nu] (= or +=) -c sum_j sum_s f_js (lam_js r1_s - r2_s) over ns pairs (f_j, lam_j),
// r1 = r[2 (nu ns + j)] = P^nu (1-f_j), r2 = the next row = P^nu (lam_j (1-f_j))
// ([2 nm ns][S]): the mode-scale derivative -c sum_st P^nu_st f_s (1-f_t) (lam_s - lam_t)
void mode_finish(int S, int nm, int ns, const double* r, VecPtrs f, VecPtrs lam, double c, double* sbar,
                 int accumulate, hipStream_t st);
void ita_gamma(int S, int n_ct, const double* rowp, double n_q, const double* vel, double* tau, double* f0,
               double* f, hipStream_t st);
// F = F0 + tau/N_q * (row sums); with chg, max|F - fprev| and max|F| into chg[0..1]
// (bit patterns, cleared by the caller)
void ita_update(int S, int n_ct, const double* rowp, double n_q, const double* tau, const double* f0, double* f,
                hipStream_t st, const double* fprev = nullptr, unsigned long long* chg = nullptr);
void mobility_reduce(int S, const double* eps, const double* vel, const double* f, double mu, double temp,
                     double* fout, double* mob, hipStream_t st);
struct Lincomb {
    int n;
    double c0;
    double c[5];
    const double* v[5];
};
void lincomb(int S, const Lincomb& lc, double* out, hipStream_t st);
// One stage of the reverse RK4 as three launches: prep forms lam = lincomb(lc)
// (state order, into lam_out) and the 2+2 pass's vectors of Y in matrix order
// (pl.gbuf: 1 - f, lam (1 - f), f, lam f); the stream; finish reduces the
// partials and writes ybar = lam^T dI/dY (state order) and, with a_acc,
// a += ybar + yb1 + yb2 + yb3.
void adjoint_stage(const StreamPlan& pl, long ld, const void* P, const double* Y, const Lincomb& lc, double* lam_out,
                   double c, double* rowp, double* colp, double* ybar, double* a_acc, const double* yb1,
                   const double* yb2, const double* yb3, hipStream_t st);
void occ_vectors(int S, const double* f, const double* lam, double* o0, double* o1, double* o2, hipStream_t st);
// Mode-scale gradient of the collision integral summed over J stages (f_j,
// lam_j), f and lam [J][S] in state order:
//   sbar[nu] (=/+=) -c sum_j sum_st P^nu_st f_js (1 - f_jt)(lam_js - lam_jt)
// over the live kPT x kPT tiles (tiles [n_tiles][2] = (row tile, column tile)
// of the matrices in energy order, perm as for the stream); pm holds the nm
// per-mode matrices [S][ld] of element type float (f32) or double, mat_elems
// apart.  work: 4 J S doubles; partial: n_tiles * nm doubles.
int mode_panel_tile();
void mode_panel_tiles(const std::vector<double>& esort, double half_width, std::vector<int32_t>& tiles);
void mode_panel(int S, long ld, int J, int nm, int f32, const void* pm, long mat_elems, const int32_t* perm,
                const double* f, const double* lam, double* work, const int32_t* tiles, int n_tiles,
                double* partial, double c, double* sbar, int accumulate, hipStream_t st);
void axpy_copy(int S, const double* x, double a, const double* y, double* out, hipStream_t st);
void fill(long n, double v, double* out, hipStream_t st);

}  // namespace ephx
