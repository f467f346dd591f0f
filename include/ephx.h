/*
 * ephx.h -- C ABI of the MI355X (gfx950) electron-phonon hot path.
 *
 * The library computes, for a Wannier model {H(Re), force constants C(Rp),
 * g(Re,Rp)}, the interpolated bands, phonons and e-ph matrix elements
 * g_mn,nu(k,q), the Gaussian-smeared scattering rates, and the BTE work built
 * on stored |g|^2 pair tables (collision integral, RK4 carrier dynamics,
 * iterative linearised BTE), following Zhou et al., "PERTURBO"
 * (arXiv:2002.02045), Sec. 2.1-2.3 and 4.3.
 *
 * Conventions (every entry point)
 * -------------------------------
 *  - Every call returns int: EPHX_OK (0) or a negative error code below;
 *    ephx_last_error() then returns a thread-local message.  No C++ exception
 *    crosses this boundary.  Arguments are validated before any launch: on an
 *    error return nothing has been enqueued.
 *  - Units: energies eV (phonons as hbar*omega in eV), lengths Angstrom,
 *    masses amu, temperature K, time fs, rates 1/fs.
 *  - k and q points are reduced (crystal) coordinates, double[n][3].
 *  - Complex arrays are interleaved (re, im) doubles or floats, row-major.
 *  - "device" arrays are owned by the caller, allocated on the current HIP
 *    device, contiguous, row-major and 16-byte aligned (as hipMalloc and
 *    torch allocate them: kernels move complex doubles as 16-byte vectors);
 *    "host" arrays are ordinary host memory.
 *  - The library owns the opaque handles (ephx_model, ephx_table), their
 *    device copies and their work buffers; release them with *_destroy.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  Every
 *    compute call is asynchronous on it, except where a host output is
 *    documented (those calls synchronise the stream before returning).
 *  - Calls on one handle must not overlap in time (they share work buffers);
 *    calls on distinct handles are independent.  A handle's work buffers grow
 *    on demand: a call that needs more than the handle holds frees and
 *    allocates device memory, which synchronises the device (size them ahead
 *    with ephx_workspace_query and a first call).
 *  - Precision: EPHX_FP64 (all steps FP64), EPHX_FP32 (Rp contraction of g,
 *    band rotation and mode projection in FP32; phases reduced in FP64; the Re
 *    contraction, H(k+q), eigensolves, eps, omega and rate sums in FP64), or
 *    EPHX_BF16X3 (as FP32, but the Rp contraction of g runs on bf16 MFMA with
 *    each FP32 operand split into two bf16 parts and three products kept), or
 *    EPHX_BF16X6 (three bf16 parts per operand, six products kept), or
 *    EPHX_FP16X3 (two fp16 parts per operand, three products kept: 11
 *    significant bits per part against bf16's 8; the g(k,Rp) operand is scaled
 *    into fp16's range by a power of two fixed per model from a bound on its
 *    entries, and the product scaled back).
 */
#ifndef EPHX_H
#define EPHX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EPHX_OK 0
#define EPHX_EINVAL (-1)       /* bad argument: null pointer, size, shape or range */
#define EPHX_ENOMEM (-2)       /* device allocation failed */
#define EPHX_EHIP (-3)         /* a HIP runtime call or kernel launch failed */
#define EPHX_ENOTHERM (-4)     /* model tensors violate H(-R) = H(R)^dag or C_kk'(-R) = C_k'k(R)^T */
#define EPHX_ENAN (-5)         /* non-finite value detected in an input or result */
#define EPHX_EUNSUPPORTED (-6) /* valid request outside what this build implements */

#define EPHX_FP64 0
#define EPHX_FP32 1
#define EPHX_BF16X3 2
#define EPHX_BF16X6 3
#define EPHX_FP16X3 4

/* Time steppers of ephx_dynamics_field (Sec. 2.1, carrier dynamics) */
#define EPHX_RK4 0
#define EPHX_EULER 1

typedef struct ephx_model ephx_model;
typedef struct ephx_table ephx_table;

/* Wannier model, all pointers host memory, read only during ephx_model_create.
 * Real-space vectors are integer triples n (R = n1 a1 + n2 a2 + n3 a3), each
 * with a weight w (multiplied into the tensor at load).
 *   h   [n_re][nw][nw] complex           H_ij(Re)              (paper Eq. wannier_2)
 *   ifc [n_rp_ph][3nat][3nat] real       C_{k a, k' b}(Rp)     (Eq. IFC1, no mass factor)
 *   g   [n_re_g][n_rp_g][3nat][nw][nw] complex  g^{k a}_ij(Re,Rp) (Eq. eph_mat_wann), eV/Angstrom
 * Polar models (polar != 0) carry Born charges zstar[nat][3][3] (index
 * [kappa][beta][alpha]), the dielectric tensor eps_inf[3][3], an Ewald parameter
 * alpha_ewald (1/Angstrom^2) and a cutoff gcut on |q+G| (1/Angstrom).  Bit 0 of
 * polar adds the Froehlich term of Eq. e_ph_long to g; bit 1 adds the
 * dipole-dipole (LO-TO) part of the force constants to D(q) (Sec. 2.3, the
 * reciprocal-space sum over K = q+G with the q = 0 sum subtracted on the
 * diagonal blocks, so the acoustic sum rule holds; ifc is then the short-range
 * part). */
typedef struct {
    double lattice[3][3];      /* rows a_1, a_2, a_3 in Angstrom */
    int natoms;
    const double* tau;         /* [natoms][3] Cartesian, Angstrom */
    const double* mass;        /* [natoms] amu */
    int nw;
    int n_re;
    const int32_t* re;
    const double* w_re;        /* may be NULL (all 1) */
    const double* h;
    int n_rp_ph;
    const int32_t* rp_ph;
    const double* w_rp_ph;     /* may be NULL */
    const double* ifc;
    int n_re_g;
    const int32_t* re_g;
    const double* w_re_g;      /* may be NULL */
    int n_rp_g;
    const int32_t* rp_g;
    const double* w_rp_g;      /* may be NULL */
    const double* g;
    int polar;
    const double* zstar;
    const double* eps_inf;
    double alpha_ewald;
    double gcut;
    /* g_gen = 1: g is not given (g may be NULL) but drawn on the device and
     * stored as complex float, for tensors too large to pass from the host
     * (216 x 216 vectors, 120 modes and 64 functions: 1.1e10 entries, 183 GB
     * of complex float).  Entry t of the flat
     * [n_re_g][n_rp_g][3nat][nw][nw] index is drawn by Philox4x32-10 (Salmon
     * et al., SC11) under the key (g_seed mod 2^32, g_seed div 2^32): the six
     * blocks with 64-bit counter 6t + b (b = 0..5; counter words 2, 3 zero),
     * the twelve words of blocks 0-2 summed exactly for the real part and of
     * blocks 3-5 for the imaginary part, x = sum * 2^-32 - 6, and the stored
     * value float(g_env[Re][Rp] * x).  g_env: host double [n_re_g][n_rp_g];
     * the weights w_re_g, w_rp_g must be NULL or 1.  Such a model supports
     * bands, phonons, gkq, gkq_pairs and rates (the Re contraction reads the
     * complex float tensor in FP64 arithmetic); pair tables, ephx_model_set_g
     * and the adjoints w.r.t. g return EPHX_EUNSUPPORTED. */
    int g_gen;
    uint64_t g_seed;
    const double* g_env;
} ephx_model_desc;

/* Physical parameters of rates, tables and transport.
 * sigma: Gaussian width, delta(x) = exp(-(x/sigma)^2)/(sqrt(pi) sigma).
 * omega_cut: modes with hbar*omega <= omega_cut contribute nothing.
 * n_q: the normalisation N_q of the q sums (Eq. e_ph_scattering); ignored by
 *      ephx_rates, which uses the q weights. */
typedef struct {
    double temp;
    double mu;
    double sigma;
    double omega_cut;
    double n_q;
} ephx_params;

const char* ephx_last_error(void);
const char* ephx_version(void);

/* Copy a model to the current device.  Checks sizes (1 <= nw <= 64 and
 * 1 <= natoms <= 42, i.e. at most 126 modes, in this build; above nw = 16 or
 * 12 modes the per-pair work runs as batched GEMMs and the calls marked so
 * below return EPHX_EUNSUPPORTED), finiteness and the Hermiticity relations
 * above (relative tolerance 1e-12) -> EPHX_EINVAL / EPHX_ENAN / EPHX_ENOTHERM.
 * *out receives a handle that the caller releases with ephx_model_destroy. */
int ephx_model_create(const ephx_model_desc* d, ephx_model** out);
int ephx_model_destroy(ephx_model* m);

/* Diagnostic read-back of the model's device copy of g(Re,Rp) (Eq.
 * eph_mat_wann, weights folded in; the complex-float values of a drawn g
 * widened to double): out[2i], out[2i+1] = entry idx[i] of the flat
 * [n_re_g][n_rp_g][3nat][nw][nw] index.  idx and out are host arrays of n
 * entries; an index out of range returns EPHX_EINVAL.  Synchronous. */
int ephx_model_g_entries(ephx_model* m, int n, const int64_t* idx, double* out);

/* Replace the model's coupling tensor g(Re,Rp) of Eq. eph_mat_wann (the
 * quantity the adjoints ephx_rates_vjp / ephx_mobility_vjp differentiate
 * against) by new values on the device, keeping every other part of the model.
 * g: device complex128 [n_re_g][n_rp_g][3nat][nw][nw], the layout and units of
 * ephx_model_desc.g (weights not folded in: the model's weights are applied
 * again), owned by the caller and only read.  The fp16 scale of the FP16x3
 * contraction is recomputed from the new values.  Checks finiteness
 * (EPHX_ENAN, the model then keeps its previous g).  Synchronises `stream`
 * (the scale is read back); later calls on the model use the new g.  Pair
 * tables created before keep the |g|^2 they were built from. */
int ephx_model_set_g(ephx_model* m, const double* g, void* stream);

/* Band interpolation, Eqs. wannier_3, velocity, wannier_4.
 * k_red device [nk][3]; eps device [nk][nw] (ascending);
 * u device [nk][nw][nw] complex128 or NULL, column n is the eigenvector of band n
 * (H^(W)(k) = U diag(eps) U^dag); vel device [nk][nw][3] (Angstrom/fs) or NULL.
 * In degenerate groups (gaps < 1e-4 eV) velocities are the eigenvalues of the
 * group block of U^dag dH/dk U, ascending within the group. */
int ephx_bands(ephx_model* m, int nk, const double* k_red, double* eps, double* u,
               double* vel, void* stream);

/* Phonon interpolation, Eq. IFC2: omega device [nq][3nat] (hbar*omega in eV,
 * ascending in omega^2, negative for omega^2 < 0); evec device
 * [nq][3nat][3nat] complex128 (column nu = e_nu) or NULL. */
int ephx_phonons(ephx_model* m, int nq, const double* q_red, double* omega, double* evec,
                 void* stream);

/* |g_mn,nu(k,q)|^2 for the outer product of a k list and a q list, Eqs.
 * eph_mat_wann2, eph_mat (+ e_ph_long for polar models).  g2 device
 * [nk][nq][3nat][nw][nw] indexed [k][q][nu][m][n] (m final band at k+q, n
 * initial band at k), double for EPHX_FP64, float otherwise.  Modes with
 * omega <= omega_cut are zero. */
int ephx_gkq(ephx_model* m, int nk, const double* k_red, int nq, const double* q_red,
             int precision, double omega_cut, void* g2, void* stream);

/* |g_mn,nu(k,q)|^2 for a list of (k, q) pairs instead of the outer product:
 * pair j is (k_red[ik[j]], q_red[iq[j]]).  ik, iq: host int32 [npairs], each
 * index in range (else EPHX_EINVAL); k_red device [nk][3], q_red device
 * [nq][3].  g2 device [npairs][3nat][nw][nw] (double for EPHX_FP64, float
 * otherwise), the values of ephx_gkq for those pairs.  Pairs are processed
 * grouped by k (each group one k against its q list), so the call is efficient
 * when many pairs share a k.  Synchronises `stream` before returning. */
int ephx_gkq_pairs(ephx_model* m, int nk, const double* k_red, int nq, const double* q_red, int npairs,
                   const int32_t* ik, const int32_t* iq, int precision, double omega_cut, void* g2,
                   void* stream);

/* Device bytes of the work buffers that one ephx_gkq (call = EPHX_CALL_GKQ)
 * or ephx_rates (EPHX_CALL_RATES) call of nk k points and nq q points at the
 * given precision takes from the model's workspace (kept by the model for
 * later calls, released by ephx_model_destroy); inputs and outputs are the
 * caller's and not counted.  For ephx_gkq_pairs, query EPHX_CALL_GKQ with
 * nk = 1 and nq = the largest number of pairs sharing one k. */
#define EPHX_CALL_GKQ 0
#define EPHX_CALL_RATES 1
int ephx_workspace_query(ephx_model* m, int call, int nk, int nq, int precision, size_t* bytes);

/* Scattering rates, Eqs. scatter_rate and BTE_W, summed over the q list with
 * weights q_w (device [nq], or NULL for 1/nq each):
 *   Gamma_nk = sum_q w_q sum_{m,nu} (2 pi/hbar)|g_mn,nu|^2 [delta(e_nk - hw - e_mk+q)(1 + N - f_m)
 *                                                         + delta(e_nk + hw - e_mk+q)(N + f_m)]
 * f = Fermi-Dirac(mu, temp), N = Bose-Einstein(temp).  gamma device [nk][nw],
 * gamma_mode device [nk][nw][3nat] or NULL; 1/fs, accumulated in FP64. */
int ephx_rates(ephx_model* m, const ephx_params* p, int nk, const double* k_red, int nq,
               const double* q_red, const double* q_w, int precision, double* gamma,
               double* gamma_mode, void* stream);

/* Parts of |g|^2 for the rates of polar models (Eq. e_ph_long): the
 * long-range coupling alone, g_L = sqrt(hbar/2 omega) sum_{kappa a} e/sqrt(M)
 * C^{kappa a}(q) [U^dag(k+q) U(k)]_mn, or what remains of |g|^2 without it. */
#define EPHX_PART_FULL 0
#define EPHX_PART_POLAR 1   /* |g_L|^2 */
#define EPHX_PART_RMPOL 2   /* |g|^2 - |g_L|^2 */

/* ephx_rates with |g|^2 replaced by one of the parts above (EPHX_PART_FULL
 * is ephx_rates).  The rates are linear in |g|^2, so the two parts add up to
 * the full rates on any q set.  EPHX_EINVAL for a part other than FULL on a
 * model without the Froehlich term; EPHX_EUNSUPPORTED above nw = 16 or 12
 * modes. */
int ephx_rates_part(ephx_model* m, const ephx_params* p, int part, int nk, const double* k_red, int nq,
                    const double* q_red, const double* q_w, int precision, double* gamma, double* gamma_mode,
                    void* stream);

/* Polar split of the q sum (Sec. 4.3 and 5.2: small-q polar scattering is
 * sampled best from a distribution peaked at Gamma, the rest uniformly):
 *   Gamma = sum_{q in set u} w_u(q) Gamma_rmpol(q) + sum_{q in set c} w_c(q) Gamma_polar(q),
 * each part estimated with its own q set and weights (device arrays as for
 * ephx_rates: q [n][3], w [n] or NULL for 1/n), e.g. uniform points for the
 * first and Cauchy points with weights 1/(n p(q)) for the second.  gamma,
 * gamma_mode as for ephx_rates.  Needs a polar model (else EPHX_EINVAL). */
int ephx_rates_polar_split(ephx_model* m, const ephx_params* p, int nk, const double* k_red, int nq_u,
                           const double* q_u, const double* w_u, int nq_c, const double* q_c,
                           const double* w_c, int precision, double* gamma, double* gamma_mode, void* stream);

/* Adjoint of ephx_rates with respect to the coupling tensor (FP64): for
 * L = sum_nk gamma_bar[n][k] Gamma_nk (gamma_bar device [nk][nw]), writes
 * g_bar = dL/dRe g(Re,Rp) + i dL/dIm g(Re,Rp), device complex128 with the
 * layout of the model's g, [n_re_g][n_rp_g][3nat][nw][nw] (overwritten).  The
 * eigenvectors of H and D do not depend on g, so the chain is the adjoint of
 * Eqs. eph_mat, eph_mat_wann2 and scatter_rate: per pair
 * g_bar = 2 (2 pi/hbar) gamma_bar w_q D g, back through the mode projection and
 * rotation, then the conjugate-phase sums over q and k.  Above Nw = 16 or 12
 * modes the per-pair adjoint runs as batched GEMMs, like the forward. */
int ephx_rates_vjp(ephx_model* m, const ephx_params* p, int nk, const double* k_red, int nq,
                   const double* q_red, const double* q_w, const double* gamma_bar, double* g_bar,
                   void* stream);

/* Window states on a Gamma-centred n_grid[0] x n_grid[1] x n_grid[2] grid
 * (Sec. 4.3): grid point (i1,i2,i3) has index (i1*N2 + i2)*N3 + i3 and reduced
 * coordinates i/N.  mode 0: every (k, band) with band_lo <= band < band_hi and
 * e_lo < eps < e_hi, the edges first moved to the midpoint between the two
 * sorted energies straddling them.  mode 1: the `count` lowest states of band
 * band_lo ordered by (eps, k index), grown while the next energy is within
 * 1e-9 eV of the last kept.  Results are sorted by (k index, band).
 * k_idx, band, eps: host arrays of capacity `capacity`; *n_states receives the
 * number found (EPHX_EINVAL with *n_states set if it exceeds capacity).
 * Synchronises `stream`. */
int ephx_grid_states(ephx_model* m, const int n_grid[3], int mode, int band_lo, int band_hi,
                     double e_lo, double e_hi, int count, int capacity, int* n_states,
                     int32_t* k_idx, int32_t* band, double* eps, void* stream);

/* Pair table of S grid states (host arrays k_idx[S], band[S] as returned above),
 * the (k, q) pairs of Sec. 4.3 with commensurate k and q grids and both ends in
 * the energy window: for every ordered pair (s,t), q = k_t - k_s on the grid and
 *   G[nu][s][t] = 1/2 (|g_{n_t n_s nu}(k_s, q)|^2 + |g_{n_s n_t nu}(k_t, -q)|^2)   (FP32)
 * together with omega_nu(q).  The symmetrisation gives |g(s->t)|^2 = |g(t->s)|^2,
 * which exact carrier conservation needs.  precision selects the arithmetic of
 * the g contractions.  The table keeps O(3nat * S^2) floats on the device. */
int ephx_table_create(ephx_model* m, const int n_grid[3], int n_states, const int32_t* k_idx,
                      const int32_t* band, int precision, double omega_cut, ephx_table** out,
                      void* stream);
int ephx_table_destroy(ephx_table* t);
/* Copies G (device [3nat][S][S]: double for an EPHX_FP64 table, float
 * otherwise; or NULL) and the state energies (device double [S], or NULL). */
int ephx_table_g2(ephx_table* t, void* g2, double* eps, void* stream);

/* Collision integral of Eq. e_ph_scattering on the table's states:
 *   I_s = -(2 pi/hbar)(1/N_q) sum_{t,nu} s_nu G[nu][s][t] [delta(e_s - hw - e_t) F_em + delta(e_s + hw - e_t) F_abs]
 * with F_abs, F_em of Sec. 2.1, N = Bose-Einstein(temp) fixed.  The call
 * ephx_collision_setup(t, p, mode_scale) (host mode_scale[3nat] or NULL = 1)
 * must precede the calls below and again after any parameter change.
 * f and I: device double [S]. */
int ephx_collision_setup(ephx_table* t, const ephx_params* p, const double* mode_scale,
                         void* stream);
int ephx_collision(ephx_table* t, const double* f, double* i_out, void* stream);

/* ephx_collision for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same result, computed by the same kernels, but the call allocates
 * nothing.  Its work memory (the occupations gathered into matrix order and
 * the row and column partials of the pass, (2 + column tiles + row tiles) * S
 * doubles) lives in one static 64 MiB device array per GPU, held by the
 * library until the process ends; a table that needs more returns
 * EPHX_EINVAL with the size in ephx_last_error().  ephx_collision_setup must
 * have been called on the table (it builds the pass's tile list), on the
 * table's device, which must be current (else EPHX_EINVAL).  All calls on one
 * GPU share that array: calls that overlap in time on one GPU (two streams,
 * two tables, two threads) race and must be serialised by the caller.  Every
 * entry of the work memory is written before it is read, so nothing is
 * cleared between calls.  f, i_out: device double [S], as for ephx_collision. */
int ephx_collision_noalloc(ephx_table* t, const double* f, double* i_out, void* stream);

/* Storage of the collision matrix (matrix 0, after ephx_collision_setup) or
 * the transport matrix (matrix 1, after ephx_mobility): both are kept with
 * rows and columns in ascending state energy, and the Gaussian delta of
 * Eq. BTE_W is taken as zero beyond 6 sigma, so every block of state pairs
 * whose energies differ by more than the largest phonon energy + 6 sigma is
 * zero and is not read.  live_entries: matrix entries one pass reads (the
 * collision pass, or one iteration of the iterative BTE); n_live_tiles of
 * n_tiles tiles of up to 1024 columns are read.  A compaction of storage
 * order only: results agree with the dense matrix up to summation order. */
int ephx_table_stream_info(ephx_table* t, int matrix, long long* live_entries, int* n_live_tiles,
                           int* n_tiles, void* stream);

/* RK4 carrier dynamics df/dt = I[f] (Eq. BTE_E with E = 0, classic four-stage
 * Runge-Kutta): n_steps steps of dt fs from f0 (device [S]) into f_out (device
 * [S]).  If ckpts is not NULL it receives f after every ckpt_every steps,
 * device [n_steps/ckpt_every + 1][S] (row 0 = f0). */
int ephx_dynamics(ephx_table* t, const double* f0, double dt, int n_steps, int ckpt_every,
                  double* f_out, double* ckpts, void* stream);

/* Carrier dynamics with an external field and a choice of stepper, Eq. BTE_E:
 *   df_s/dt = I[f]_s + (|e|/hbar) E . grad_k f_s
 * (the electron's charge is -|e|, so a distribution drifts in k at -|e|E/hbar).
 * grad_k f is the central difference along the grid's reduced directions,
 * band by band: with a_i the lattice rows and N_i the grid,
 *   E . grad_k f_s = sum_i (E . a_i / 2 pi) (N_i/2) (f[s + e_i] - f[s - e_i]),
 * where a neighbour that is not a state of the table counts as empty (f = 0).
 * efield: host [3] in V/Angstrom, or NULL for E = 0.  method: EPHX_RK4 (the
 * classic four stages) or EPHX_EULER (first order, one collision pass per
 * step).  f0, f_out, ckpts as for ephx_dynamics; with EPHX_RK4 and E = 0 the
 * result equals ephx_dynamics'.  The neighbour table (24 bytes per state) is
 * built on the first call with a field.  ephx_dynamics_vjp differentiates the
 * RK4, E = 0 dynamics only. */
int ephx_dynamics_field(ephx_table* t, const double* f0, double dt, int n_steps, int method,
                        const double* efield, int ckpt_every, double* f_out, double* ckpts,
                        void* stream);

/* Vector-Jacobian product of the collision integral: given f and lambda
 * (device [S]), f_bar = lambda^T dI/df (device [S]) and, if s_bar is not
 * NULL, s_bar[nu] = lambda^T dI/ds_nu (device [3nat]).  The first s_bar after
 * each ephx_collision_setup builds the collision matrix of every mode alone
 * (3nat more matrices the size of the collision matrix, kept by the table);
 * s_bar then costs one banded pass over each of them. */
int ephx_collision_vjp(ephx_table* t, const double* f, const double* lam, double* f_bar,
                       double* s_bar, void* stream);

/* Backward through ephx_dynamics for a loss L(f_final): given checkpoints
 * (as written by ephx_dynamics with the same dt, n_steps, ckpt_every) and
 * f_bar_final = dL/df(t_end) (device [S]), returns dL/df0 (device [S]) and
 * dL/ds_nu at the current mode scales (device [3nat], or NULL).  Each
 * checkpoint segment is replayed forward, then differentiated in reverse. */
int ephx_dynamics_vjp(ephx_table* t, const double* ckpts, double dt, int n_steps,
                      int ckpt_every, const double* f_bar_final, double* f0_bar,
                      double* s_bar, void* stream);

/* Iterative linearised BTE (Eqs. BTE_lin, BTE_iter, BTE_W) on the table's
 * states with equilibrium occupations f0 = Fermi-Dirac(p->mu, p->temp):
 *   Gamma_s = (1/N_q) sum_t W_st, tau = 1/Gamma, F^0 = tau v,
 *   F^{i+1} = F^0 + (tau/N_q) sum_t W_st F^i.
 * Stopping rule (Eq. BTE_iter iterates until F changes by less than a
 * threshold): with tol > 0 the iteration stops after the first update i + 1
 * with max_{s,a} |F^{i+1} - F^i| < tol * max_{s,a} |F^{i+1}|, or after
 * n_iter_max updates; with tol <= 0 exactly n_iter_max updates are made.
 * n_iter_max = 0 gives the RTA.  With tol > 0 every iteration reads two
 * doubles back, so the call then synchronises `stream` once per iteration.
 * vel device [S][3] (Angstrom/fs).  F_out device [S][3] (Angstrom), tau_out
 * device [S] (fs) or NULL.  The mobility of Eq. cond divided by e n_c,
 * mu_ab = e sum v^a F^b (-df0/de) / sum f0, goes to mob_out (device double
 * [3][3], cm^2/(V s)) unless NULL.  Host outputs (each may be NULL): *n_iter
 * the number of updates made; *last_change the relative change of the last
 * update (-1 when tol <= 0, where it is not measured).  A result with
 * *n_iter == n_iter_max and *last_change >= tol did not converge.  When Gamma
 * is the row sum of the same W, (tau/N_q) W has the constant vector as a unit
 * eigenvector, so the iteration converges only for F^0 orthogonal to it (for
 * example an inversion- or time-reversal-symmetric set of states, where F^0 is
 * odd).  A non-finite iterate returns EPHX_ENAN. */
int ephx_mobility(ephx_table* t, const ephx_params* p, const double* vel, int n_iter_max, double tol,
                  double* f_out, double* tau_out, double* mob_out, int* n_iter, double* last_change,
                  void* stream);

/* Adjoint of ephx_mobility with respect to the coupling tensor (FP64): for
 * L = sum_ab mob_bar[a][b] mu_ab (mob_bar device double [3][3]) and the same
 * table, p and vel as the forward call, with n_iter the number of updates the
 * forward made (its *n_iter: the gradient is that of the iterate returned,
 * not an implicit derivative of the fixed point), writes g_bar = dL/dRe g(Re,Rp)
 * + i dL/dIm g(Re,Rp) (device complex128, layout of the model's g, overwritten).
 * The chain is the reverse of Eqs. BTE_iter and cond (the iteration is rerun
 * and kept, then reversed with one pass of W^T per iteration), W_bar through
 * Eq. BTE_W and the symmetrisation of the table, and the adjoint of Eqs.
 * eph_mat and eph_mat_wann2 for every ordered pair of states: conjugate-phase
 * sums over the targets (q = k_t - k_s) and the sources.  The forward g is
 * recomputed in FP64 whatever the table's precision.  Synchronises the stream
 * before returning (the workspace is reused by the next call). */
int ephx_mobility_vjp(ephx_table* t, const ephx_params* p, const double* vel, int n_iter,
                      const double* mob_bar, double* g_bar, void* stream);

/* Transport distribution function, Eq. cond_tdf2, by linear tetrahedron
 * integration (Sec. 4.3) over the table's states: the grid's cubes are cut
 * into 6 tetrahedra along their (0,0,0)-(1,1,1) diagonal and a tetrahedron
 * enters for each band whose four corners are all table states.
 *   Sigma_ab(E) = (2/(N_k Omega)) sum_nk v^a F^b delta(E - eps_nk)
 * with spin degeneracy 2, N_k the grid size and Omega the cell volume.
 * vel and f_ita: device [S][3] (Angstrom/fs; F as returned by ephx_mobility,
 * Angstrom); e_grid: device [n_e] ascending energies (eV), 2 <= n_e <= 65535.
 * Outputs (device, each may be NULL): tdf [n_e][3][3] in 1/(fs Angstrom eV);
 * sigma [3][3], Eq. cond_tdf, in S/m; seebeck [3][3], Eq. seebeck with the
 * electron charge -e, in V/K (both by the trapezoid rule on e_grid, f0 at
 * p->mu and p->temp).  Synchronises the stream before returning. */
int ephx_tdf(ephx_table* t, const ephx_params* p, const double* vel, const double* f_ita, int n_e,
             const double* e_grid, double* tdf, double* sigma, double* seebeck, void* stream);

/* Carrier population, Eq. pop: pop[e] = sum_nk f_nk delta(eps_nk - E_e) (1/eV)
 * by the same tetrahedra; f device [S], e_grid device [n_e], pop device [n_e].
 * Synchronises the stream before returning. */
int ephx_population(ephx_table* t, const double* f, int n_e, const double* e_grid, double* pop,
                    void* stream);

/* Stage timers (instrumentation, not part of the method).  While enabled,
 * the library brackets each launch of its main kernels with HIP events on the
 * launch stream, keyed by stage name: "re_contraction", "hkq_fourier",
 * "eig_hkq", "rp_contraction", "epilogue", "phonons", "bands",
 * "table_pairs", "collision_stream", "collision_finish".
 * ephx_timer_get synchronises the recorded events and returns the number of
 * launches and their summed duration in ms (zeros for an unknown stage). */
int ephx_timer_enable(int on);
int ephx_timer_reset(void);
int ephx_timer_get(const char* stage, int* launches, double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* EPHX_H */
