// Host-side state shared by the API translation units.
#pragma once

#include <functional>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/ephx.h"
#include "internal.h"

namespace ephx {

extern thread_local std::string g_last_error;

// Growable named device buffers owned by a handle.
struct Workspace {
    struct Buf {
        void* ptr = nullptr;
        size_t size = 0;
    };
    std::map<std::string, Buf> bufs;
    void* get(const std::string& name, size_t bytes);
    void release();
};

void hip_check(hipError_t e, const char* what);
void* dev_upload(const void* host, size_t bytes);
void require(bool ok, const std::string& msg);

// Stage timers: HIP events around launches while enabled.
struct StageTimer {
    const char* name;
    hipStream_t st;
    hipEvent_t e0 = nullptr;
    StageTimer(const char* n, hipStream_t s);
    void stop();   // records the end event (idempotent)
    ~StageTimer() { stop(); }
};

template <class F>
int guarded(F&& f) {
    try {
        f();
        g_last_error.clear();
        return EPHX_OK;
    } catch (const Error& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return EPHX_ENOMEM;
    } catch (...) {
        g_last_error = "unexpected internal error";
        return EPHX_EHIP;
    }
}

}  // namespace ephx

struct ephx_model {
    int device = 0;
    int nw = 0, nat = 0, nm = 0;
    double lattice[9] = {0};
    double bvec[9] = {0};
    double volume = 0.0;
    std::vector<double> mass, tau;
    int n_re = 0, n_rp_ph = 0, n_re_g = 0, n_rp_g = 0;
    int32_t *d_re = nullptr, *d_rp_ph = nullptr, *d_re_g = nullptr, *d_rp_g = nullptr;
    double* d_h = nullptr;       // [n_re][nw*nw] complex, weights folded
    double* d_hvel = nullptr;    // [n_re][3][nw*nw] complex, H(R) * (i R_a)
    int n_re_half = 0;           // Hermitian half set: R = 0 and one of each +/-R pair
    int32_t* d_re_half = nullptr;
    double* d_h_half = nullptr;  // [n_re_half][2][nw*nw] complex: H+H^dag, i(H-H^dag)
    int h_pack = 0;              // reals per packed Hermitian matrix: nw*nw rounded up to even
    double* d_h_pack = nullptr;  // [n_re_half][2][h_pack]: the same, packed (nw <= 8 only)
    int n_rp_half = 0;           // half set of the Rp vectors of g: one of each +/-Rp pair, unpaired once
    int32_t* d_rp_half = nullptr;  // [n_rp_half][3] its vectors
    int32_t* d_rp_pair = nullptr;  // [n_rp_half][2] index of R and of -R (-1: absent) in the Rp list
    double* d_cm = nullptr;      // [n_rp_ph][nm*nm] complex, C / sqrt(M M')
    double g_scale = 1.0;        // power of two taking the Rp-contraction operand of g into fp16 range
    double* d_g = nullptr;       // [n_re_g][n_rp_g][nm][nw][nw] complex
    float* d_g32 = nullptr;      // the same as complex float when counter-drawn (g_c64)
    bool g_c64 = false;
    double* d_minv = nullptr;    // [nm]
    double* d_wg = nullptr;      // [n_re_g][n_rp_g] weight products, only if not all 1
    double* d_nrp_g = nullptr;   // -Rp then -Re as doubles (adjoint sums), created on first use
    double* d_nre_g = nullptr;
    bool polar = false;          // Froehlich term in g
    bool dipole = false;         // dipole-dipole (LO-TO) part of D(q)
    double* d_dipcorr = nullptr; // [nat][3][3] complex sum-rule term
    double *d_bvec = nullptr, *d_tau = nullptr, *d_zstar = nullptr, *d_eps = nullptr;
    ephx::PolarDev pd{};
    std::vector<void*> owned;
    ephx::Workspace ws;
    ~ephx_model();
};

namespace ephx {
void bands_impl(ephx_model* m, int nk, const double* k, double* eps, double* u, double* vel, hipStream_t st,
                const std::string& tag);
void phonons_impl(ephx_model* m, int nq, const double* q, double* omega, double* evec, hipStream_t st,
                  const std::string& tag);
void negated_vectors(ephx_model* m);
// models beyond the per-pair register kernels (batched-GEMM path only)
inline bool is_wide(const ephx_model* m) { return m->nw > kMaxNw || m->nm > kMaxModes; }
}  // namespace ephx
