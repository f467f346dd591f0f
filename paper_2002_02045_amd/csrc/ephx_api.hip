// Host side of the C ABI declared in include/ephx.h: argument checks, model
// upload, work buffers and the orchestration of the kernels for bands,
// phonons, g(k,q) and scattering rates.  BTE entry points live in bte_api.hip.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/ephx.h"
#include "api_common.h"

namespace ephx {

thread_local std::string g_last_error;

void Workspace::release() {
    for (auto& kv : bufs)
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    bufs.clear();
}

void* Workspace::get(const std::string& name, size_t bytes) {
    Buf& b = bufs[name];
    if (b.size >= bytes && b.ptr) return b.ptr;
    if (b.ptr) {
        (void)hipDeviceSynchronize();
        (void)hipFree(b.ptr);
        b.ptr = nullptr;
        b.size = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) {
        (void)hipGetLastError();
        throw Error{EPHX_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes for " + name + " failed"};
    }
    b.ptr = p;
    b.size = bytes;
    return p;
}

// ---------------------------------------------------------------- stage timers
namespace {
struct TimerState {
    bool on = false;
    std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> ev;
} g_timer;
}  // namespace

StageTimer::StageTimer(const char* n, hipStream_t s) : name(n), st(s) {
    if (!g_timer.on) return;
    if (hipEventCreate(&e0) != hipSuccess) {
        e0 = nullptr;
        return;
    }
    (void)hipEventRecord(e0, st);
}

void StageTimer::stop() {
    if (!e0) return;
    hipEvent_t e1 = nullptr;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        e0 = nullptr;
        return;
    }
    (void)hipEventRecord(e1, st);
    g_timer.ev[name].push_back({e0, e1});
    e0 = nullptr;
}

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) throw Error{EPHX_EHIP, std::string(what) + ": " + hipGetErrorString(e)};
}

void* dev_upload(const void* host, size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) {
        (void)hipGetLastError();
        throw Error{EPHX_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    }
    if (host) hip_check(hipMemcpy(p, host, bytes, hipMemcpyHostToDevice), "hipMemcpy");
    return p;
}

void require(bool ok, const std::string& msg) {
    if (!ok) throw Error{EPHX_EINVAL, msg};
}

// The largest power of two that keeps a bound on the half-set coefficients of
// the Rp contraction's g operand under 2^14 (fp16 ends at 65504).
static double fp16_scale(double bound) {
    return bound > 0.0 ? std::ldexp(1.0, std::max(-60, std::min(60, (int)std::floor(std::log2(16384.0 / bound)))))
                       : 1.0;
}

static bool finite_all(const double* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

static std::map<std::vector<int>, int> index_of(const int32_t* v, int n) {
    std::map<std::vector<int>, int> m;
    for (int i = 0; i < n; ++i) m[{v[3 * i], v[3 * i + 1], v[3 * i + 2]}] = i;
    return m;
}

}  // namespace ephx

using namespace ephx;

ephx_model::~ephx_model() {
    ws.release();
    for (void* p : owned)
        if (p) (void)hipFree(p);
}

extern "C" const char* ephx_last_error(void) { return g_last_error.c_str(); }

extern "C" int ephx_timer_reset(void) {
    return guarded([&] {
        for (auto& kv : g_timer.ev)
            for (auto& pr : kv.second) {
                (void)hipEventSynchronize(pr.second);
                (void)hipEventDestroy(pr.first);
                (void)hipEventDestroy(pr.second);
            }
        g_timer.ev.clear();
    });
}

extern "C" int ephx_timer_enable(int on) {
    return guarded([&] { g_timer.on = on != 0; });
}

extern "C" int ephx_timer_get(const char* stage, int* launches, double* total_ms) {
    return guarded([&] {
        require(stage && launches && total_ms, "timer_get: null argument");
        *launches = 0;
        *total_ms = 0.0;
        auto it = g_timer.ev.find(stage);
        if (it == g_timer.ev.end()) return;
        for (auto& pr : it->second) {
            hip_check(hipEventSynchronize(pr.second), "hipEventSynchronize");
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, pr.first, pr.second), "hipEventElapsedTime");
            *total_ms += ms;
            *launches += 1;
        }
    });
}
extern "C" const char* ephx_version(void) { return "ephx 0.1 gfx950"; }

extern "C" int ephx_model_create(const ephx_model_desc* d, ephx_model** out) {
    return guarded([&] {
        require(d != nullptr && out != nullptr, "model_create: null argument");
        *out = nullptr;
        require(d->natoms >= 1 && 3 * d->natoms <= kMaxModesWide, "model_create: need 1 <= natoms <= 42");
        require(d->nw >= 1 && d->nw <= kMaxNwWide, "model_create: need 1 <= nw <= 64");
        require(d->n_re >= 1 && d->n_rp_ph >= 1 && d->n_re_g >= 1 && d->n_rp_g >= 1, "model_create: empty vector set");
        require(d->g_gen == 0 || d->g_gen == 1, "model_create: g_gen must be 0 (g given) or 1 (counter-drawn)");
        const bool gen = d->g_gen == 1;
        require(d->tau && d->mass && d->re && d->h && d->rp_ph && d->ifc && d->re_g && d->rp_g && (gen || d->g),
                "model_create: null array");
        require(!gen || d->g_env, "model_create: a counter-drawn g needs g_env");
        const int nw = d->nw, nat = d->natoms, nm = 3 * nat, nw2 = nw * nw;
        const size_t nh = (size_t)d->n_re * nw2 * 2, nc = (size_t)d->n_rp_ph * nm * nm;
        const size_t ng = (size_t)d->n_re_g * d->n_rp_g * nm * nw2 * 2;
        if (gen) {
            bool unit = true;
            for (int e = 0; e < d->n_re_g && d->w_re_g; ++e) unit = unit && d->w_re_g[e] == 1.0;
            for (int p = 0; p < d->n_rp_g && d->w_rp_g; ++p) unit = unit && d->w_rp_g[p] == 1.0;
            require(unit, "model_create: a counter-drawn g takes unit weights on Re and Rp");
            if (!finite_all(d->g_env, (size_t)d->n_re_g * d->n_rp_g))
                throw Error{EPHX_ENAN, "model_create: non-finite g_env"};
        }
        if (!finite_all(d->h, nh) || !finite_all(d->ifc, nc) || (!gen && !finite_all(d->g, ng)) ||
            !finite_all(d->tau, 3 * nat) || !finite_all(d->mass, nat) || !finite_all(&d->lattice[0][0], 9))
            throw Error{EPHX_ENAN, "model_create: non-finite value in the model"};
        for (int a = 0; a < nat; ++a) require(d->mass[a] > 0.0, "model_create: masses must be positive");
        double det = d->lattice[0][0] * (d->lattice[1][1] * d->lattice[2][2] - d->lattice[1][2] * d->lattice[2][1]) -
                     d->lattice[0][1] * (d->lattice[1][0] * d->lattice[2][2] - d->lattice[1][2] * d->lattice[2][0]) +
                     d->lattice[0][2] * (d->lattice[1][0] * d->lattice[2][1] - d->lattice[1][1] * d->lattice[2][0]);
        require(std::fabs(det) > 1e-12, "model_create: singular lattice");
        // Hermiticity: H(-R) = H(R)^dag and C_kk'(-R) = C_k'k(R)^T where -R is in the set
        {
            auto idx = index_of(d->re, d->n_re);
            double hmax = 0.0;
            for (size_t i = 0; i < nh; ++i) hmax = std::fmax(hmax, std::fabs(d->h[i]));
            for (int r = 0; r < d->n_re; ++r) {
                auto it = idx.find({-d->re[3 * r], -d->re[3 * r + 1], -d->re[3 * r + 2]});
                if (it == idx.end()) continue;
                const int s = it->second;
                const double wr = d->w_re ? d->w_re[r] : 1.0, ws_ = d->w_re ? d->w_re[s] : 1.0;
                for (int i = 0; i < nw; ++i)
                    for (int j = 0; j < nw; ++j) {
                        const double* a = d->h + ((size_t)r * nw2 + i * nw + j) * 2;
                        const double* b = d->h + ((size_t)s * nw2 + j * nw + i) * 2;
                        if (std::fabs(wr * a[0] - ws_ * b[0]) > 1e-12 * hmax ||
                            std::fabs(wr * a[1] + ws_ * b[1]) > 1e-12 * hmax)
                            throw Error{EPHX_ENOTHERM, "model_create: H(-R) != H(R)^dagger"};
                    }
            }
            auto idc = index_of(d->rp_ph, d->n_rp_ph);
            double cmax = 0.0;
            for (size_t i = 0; i < nc; ++i) cmax = std::fmax(cmax, std::fabs(d->ifc[i]));
            for (int r = 0; r < d->n_rp_ph; ++r) {
                auto it = idc.find({-d->rp_ph[3 * r], -d->rp_ph[3 * r + 1], -d->rp_ph[3 * r + 2]});
                if (it == idc.end()) continue;
                const int s = it->second;
                const double wr = d->w_rp_ph ? d->w_rp_ph[r] : 1.0, ws_ = d->w_rp_ph ? d->w_rp_ph[s] : 1.0;
                for (int a = 0; a < nm; ++a)
                    for (int b = 0; b < nm; ++b)
                        if (std::fabs(wr * d->ifc[(size_t)r * nm * nm + a * nm + b] -
                                      ws_ * d->ifc[(size_t)s * nm * nm + b * nm + a]) > 1e-12 * cmax)
                            throw Error{EPHX_ENOTHERM, "model_create: C(-R) != C(R)^T"};
            }
        }
        if (d->polar) {
            require(d->zstar && d->eps_inf, "model_create: polar model needs zstar and eps_inf");
            require(d->alpha_ewald > 0 && d->gcut > 0, "model_create: polar model needs alpha_ewald, gcut > 0");
        }
        int dev = 0;
        hip_check(hipGetDevice(&dev), "hipGetDevice");
        ephx_model* m = new ephx_model();
        try {
            m->device = dev;
            m->nw = nw;
            m->nat = nat;
            m->nm = nm;
            std::memcpy(m->lattice, &d->lattice[0][0], sizeof(m->lattice));
            m->mass.assign(d->mass, d->mass + nat);
            m->tau.assign(d->tau, d->tau + 3 * nat);
            m->n_re = d->n_re;
            m->n_rp_ph = d->n_rp_ph;
            m->n_re_g = d->n_re_g;
            m->n_rp_g = d->n_rp_g;
            m->volume = std::fabs(det);
            // inverse-transpose times 2 pi: reciprocal vectors b_i as rows
            {
                const double* L = m->lattice;
                double inv[9];
                inv[0] = (L[4] * L[8] - L[5] * L[7]) / det;
                inv[1] = (L[2] * L[7] - L[1] * L[8]) / det;
                inv[2] = (L[1] * L[5] - L[2] * L[4]) / det;
                inv[3] = (L[5] * L[6] - L[3] * L[8]) / det;
                inv[4] = (L[0] * L[8] - L[2] * L[6]) / det;
                inv[5] = (L[2] * L[3] - L[0] * L[5]) / det;
                inv[6] = (L[3] * L[7] - L[4] * L[6]) / det;
                inv[7] = (L[1] * L[6] - L[0] * L[7]) / det;
                inv[8] = (L[0] * L[4] - L[1] * L[3]) / det;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) m->bvec[3 * i + j] = 2.0 * kPi * inv[3 * j + i];
            }
            auto up = [&](const void* h, size_t bytes) {
                void* p = dev_upload(h, bytes);
                m->owned.push_back(p);
                return p;
            };
            m->d_re = (int32_t*)up(d->re, sizeof(int32_t) * 3 * d->n_re);
            m->d_rp_ph = (int32_t*)up(d->rp_ph, sizeof(int32_t) * 3 * d->n_rp_ph);
            m->d_re_g = (int32_t*)up(d->re_g, sizeof(int32_t) * 3 * d->n_re_g);
            m->d_rp_g = (int32_t*)up(d->rp_g, sizeof(int32_t) * 3 * d->n_rp_g);
            {
                // half set of the Rp list for the Rp sum with real coefficients: each
                // +/-R pair once (at its first member), every unpaired vector once;
                // left empty if the list repeats a vector
                auto idp = index_of(d->rp_g, d->n_rp_g);
                if ((int)idp.size() == d->n_rp_g) {
                    std::vector<int32_t> rv, pr;
                    for (int p = 0; p < d->n_rp_g; ++p) {
                        const int a = d->rp_g[3 * p], b = d->rp_g[3 * p + 1], c = d->rp_g[3 * p + 2];
                        auto it = idp.find({-a, -b, -c});
                        const int n = (it != idp.end() && it->second != p) ? it->second : -1;
                        if (n >= 0 && n < p) continue;
                        rv.insert(rv.end(), {a, b, c});
                        pr.insert(pr.end(), {p, n});
                    }
                    m->n_rp_half = (int)(pr.size() / 2);
                    m->d_rp_half = (int32_t*)up(rv.data(), rv.size() * sizeof(int32_t));
                    m->d_rp_pair = (int32_t*)up(pr.data(), pr.size() * sizeof(int32_t));
                }
            }
            // H(R) with weights folded in, and H(R) * (i R_a) for velocities
            std::vector<double> h(nh), hv((size_t)d->n_re * 3 * nw2 * 2);
            for (int r = 0; r < d->n_re; ++r) {
                const double w = d->w_re ? d->w_re[r] : 1.0;
                double rc[3];
                for (int a = 0; a < 3; ++a)
                    rc[a] = d->re[3 * r] * m->lattice[a] + d->re[3 * r + 1] * m->lattice[3 + a] + d->re[3 * r + 2] * m->lattice[6 + a];
                for (int e = 0; e < nw2; ++e) {
                    const double re_ = w * d->h[((size_t)r * nw2 + e) * 2], im_ = w * d->h[((size_t)r * nw2 + e) * 2 + 1];
                    h[((size_t)r * nw2 + e) * 2] = re_;
                    h[((size_t)r * nw2 + e) * 2 + 1] = im_;
                    for (int a = 0; a < 3; ++a) {
                        // (re + i im) * (i R_a) = -im R_a + i re R_a
                        hv[(((size_t)r * 3 + a) * nw2 + e) * 2] = -im_ * rc[a];
                        hv[(((size_t)r * 3 + a) * nw2 + e) * 2 + 1] = re_ * rc[a];
                    }
                }
            }
            m->d_h = (double*)up(h.data(), h.size() * sizeof(double));
            {
                // Hermitian half set.  The Hermitian part of sum_R e^{ik.R} H(R) equals
                //   sum_half [cos(k.R)(M + M^dag) + sin(k.R) i(M - M^dag)],
                // M = (H(R) + H(-R)^dag)/2 for a +/-R pair (taken once), M = H(R)/2 for a
                // vector whose -R is absent, and the R = 0 term (H(0) + H(0)^dag)/2.
                auto idx = index_of(d->re, d->n_re);
                std::vector<int32_t> rh;
                std::vector<double> hh;
                std::vector<double> mre(nw2), mim(nw2);
                for (int r = 0; r < d->n_re; ++r) {
                    const int a = d->re[3 * r], b = d->re[3 * r + 1], c = d->re[3 * r + 2];
                    const bool zero = a == 0 && b == 0 && c == 0;
                    auto it = idx.find({-a, -b, -c});
                    const bool paired = it != idx.end();
                    if (paired && !zero && std::vector<int>{a, b, c} < std::vector<int>{-a, -b, -c}) continue;
                    const int s2 = paired ? it->second : -1;
                    for (int e = 0; e < nw2; ++e) {
                        const int i = e / nw, j = e % nw;
                        const double* x = &h[((size_t)r * nw2 + e) * 2];
                        double yr = 0.0, yi = 0.0;  // (H(-R)^dag)_ij = conj(H(-R)_ji)
                        if (paired) {
                            const double* y = &h[((size_t)s2 * nw2 + j * nw + i) * 2];
                            yr = y[0];
                            yi = -y[1];
                        }
                        mre[e] = 0.5 * (x[0] + yr);
                        mim[e] = 0.5 * (x[1] + yi);
                    }
                    rh.insert(rh.end(), {a, b, c});
                    for (int part = 0; part < 2; ++part)
                        for (int e = 0; e < nw2; ++e) {
                            const int i = e / nw, j = e % nw;
                            const double pr = mre[e], pi = mim[e];               // M_ij
                            const double qr = mre[j * nw + i], qi = -mim[j * nw + i];  // (M^dag)_ij
                            double re_, im_;
                            if (zero) {
                                // R = 0 (M already Hermitian part of H(0)): cos = 1, sin = 0
                                re_ = part == 0 ? pr : 0.0;
                                im_ = part == 0 ? pi : 0.0;
                            } else if (part == 0) {  // M + M^dag
                                re_ = pr + qr;
                                im_ = pi + qi;
                            } else {  // i (M - M^dag)
                                re_ = -(pi - qi);
                                im_ = pr - qr;
                            }
                            hh.push_back(re_);
                            hh.push_back(im_);
                        }
                }
                m->n_re_half = (int)(rh.size() / 3);
                m->d_re_half = (int32_t*)up(rh.data(), rh.size() * sizeof(int32_t));
                m->d_h_half = (double*)up(hh.data(), hh.size() * sizeof(double));
                if (nw <= kEigMax) {
                    // packed form of each Hermitian A_r, B_r: Re of the upper triangle
                    // (diagonal included) in place, Im of the upper triangle mirrored
                    // into the lower one, padded to an even count
                    const int pk = nw2 + (nw2 & 1);
                    std::vector<double> hp((size_t)m->n_re_half * 2 * pk, 0.0);
                    for (size_t rp = 0; rp < (size_t)m->n_re_half * 2; ++rp)
                        for (int i = 0; i < nw; ++i)
                            for (int j = 0; j < nw; ++j) {
                                const int lo = i < j ? i : j, hi = i < j ? j : i;
                                const double* x = &hh[(rp * nw2 + lo * nw + hi) * 2];
                                hp[rp * pk + i * nw + j] = i <= j ? x[0] : x[1];
                            }
                    m->h_pack = pk;
                    m->d_h_pack = (double*)up(hp.data(), hp.size() * sizeof(double));
                }
            }
            m->d_hvel = (double*)up(hv.data(), hv.size() * sizeof(double));
            // C(R) / sqrt(M_k M_k') as complex, weights folded
            std::vector<double> cm((size_t)d->n_rp_ph * nm * nm * 2, 0.0);
            for (int r = 0; r < d->n_rp_ph; ++r) {
                const double w = d->w_rp_ph ? d->w_rp_ph[r] : 1.0;
                for (int a = 0; a < nm; ++a)
                    for (int b = 0; b < nm; ++b)
                        cm[(((size_t)r * nm + a) * nm + b) * 2] =
                            w * d->ifc[((size_t)r * nm + a) * nm + b] / std::sqrt(d->mass[a / 3] * d->mass[b / 3]);
            }
            m->d_cm = (double*)up(cm.data(), cm.size() * sizeof(double));
            if (gen) {
                // g(Re,Rp) drawn on the device by the counter scheme, stored as
                // complex float; the fp16 scale from its entries as below
                const long per = (long)nm * nw2;
                double* denv = (double*)dev_upload(d->g_env, (size_t)d->n_re_g * d->n_rp_g * 8);
                m->d_g32 = (float*)up(nullptr, (size_t)d->n_re_g * d->n_rp_g * per * 8);
                m->g_c64 = true;
                gen_coupling(d->n_re_g, d->n_rp_g, per, (unsigned long long)d->g_seed, denv, m->d_g32, nullptr);
                unsigned long long* red = (unsigned long long*)m->ws.get("create.red", 16);
                g_row_bound_f32(d->n_re_g, (long)d->n_rp_g * nm * nw, nw, m->d_g32, red, nullptr);
                unsigned long long h2[2] = {0, 0};
                hip_check(hipMemcpy(h2, red, sizeof(h2), hipMemcpyDeviceToHost), "hipMemcpy");
                (void)hipFree(denv);
                if (h2[1]) throw Error{EPHX_ENAN, "model_create: non-finite drawn g"};
                double rowmax;
                std::memcpy(&rowmax, &h2[0], 8);
                m->g_scale = fp16_scale(2.0 * rowmax);
            } else {
                const size_t per = (size_t)nm * nw2 * 2;
                std::vector<double> g(ng);
                for (int e = 0; e < d->n_re_g; ++e)
                    for (int p = 0; p < d->n_rp_g; ++p) {
                        const double w = (d->w_re_g ? d->w_re_g[e] : 1.0) * (d->w_rp_g ? d->w_rp_g[p] : 1.0);
                        const size_t o = ((size_t)e * d->n_rp_g + p) * per;
                        for (size_t i = 0; i < per; ++i) g[o + i] = w * d->g[o + i];
                    }
                m->d_g = (double*)up(g.data(), ng * sizeof(double));
                // fp16 scale of the Rp-contraction operand: an entry of g(k,Rp) V
                // (V unitary, or one of its columns) is at most sum_Re sum_j
                // |g(Re,Rp)_ij| for its row i, and a half-set coefficient at most twice
                // that; the largest power of two keeping it under 2^14 (fp16 ends at
                // 65504) is the model's scale
                std::vector<double> rs((size_t)d->n_rp_g * nm * nw, 0.0);
                for (int e = 0; e < d->n_re_g; ++e)
                    for (int p = 0; p < d->n_rp_g; ++p)
                        for (int a = 0; a < nm; ++a)
                            for (int i = 0; i < nw; ++i) {
                                double t = 0.0;
                                for (int j = 0; j < nw; ++j) {
                                    const size_t o = (((((size_t)e * d->n_rp_g + p) * nm + a) * nw + i) * nw + j) * 2;
                                    t += std::hypot(g[o], g[o + 1]);
                                }
                                rs[((size_t)p * nm + a) * nw + i] += t;
                            }
                double bound = 0.0;
                for (double v : rs) bound = std::max(bound, 2.0 * v);
                m->g_scale = fp16_scale(bound);
            }
            if (!gen) {
                bool unit = true;
                std::vector<double> wg((size_t)d->n_re_g * d->n_rp_g);
                for (int e = 0; e < d->n_re_g; ++e)
                    for (int p = 0; p < d->n_rp_g; ++p) {
                        const double w = (d->w_re_g ? d->w_re_g[e] : 1.0) * (d->w_rp_g ? d->w_rp_g[p] : 1.0);
                        wg[(size_t)e * d->n_rp_g + p] = w;
                        unit = unit && w == 1.0;
                    }
                if (!unit) m->d_wg = (double*)up(wg.data(), wg.size() * sizeof(double));
            }
            std::vector<double> minv(nm);
            for (int a = 0; a < nm; ++a) minv[a] = 1.0 / std::sqrt(d->mass[a / 3]);
            m->d_minv = (double*)up(minv.data(), nm * sizeof(double));
            m->polar = (d->polar & 1) != 0;
            m->dipole = (d->polar & 2) != 0;
            if (d->polar != 0) {
                m->d_bvec = (double*)up(m->bvec, 9 * sizeof(double));
                m->d_tau = (double*)up(d->tau, 3 * nat * sizeof(double));
                m->d_zstar = (double*)up(d->zstar, 9 * nat * sizeof(double));
                m->d_eps = (double*)up(d->eps_inf, 9 * sizeof(double));
                PolarDev& p = m->pd;
                p.bvec = m->d_bvec;
                p.tau = m->d_tau;
                p.zstar = m->d_zstar;
                p.eps = m->d_eps;
                p.pref = 4.0 * kPi * kE2Over4PiEps0 / m->volume;
                p.alpha = d->alpha_ewald;
                p.gcut = d->gcut;
                p.nat = nat;
                // |m_i| <= (gcut + |q|) |a_i| / (2 pi), |q| <= half the sum of |b_i|
                double bsum = 0.0;
                for (int i = 0; i < 3; ++i)
                    bsum += std::sqrt(m->bvec[3 * i] * m->bvec[3 * i] + m->bvec[3 * i + 1] * m->bvec[3 * i + 1] +
                                      m->bvec[3 * i + 2] * m->bvec[3 * i + 2]);
                for (int i = 0; i < 3; ++i) {
                    const double al = std::sqrt(m->lattice[3 * i] * m->lattice[3 * i] + m->lattice[3 * i + 1] * m->lattice[3 * i + 1] +
                                                m->lattice[3 * i + 2] * m->lattice[3 * i + 2]);
                    p.mmax[i] = (int)std::ceil((d->gcut + 0.5 * bsum) * al / (2.0 * kPi)) + 1;
                }
                if (m->dipole) {
                    // q = 0 sum over G != 0 and all k'' of the dipole-dipole blocks
                    std::vector<double> corr(2 * 9 * nat, 0.0);
                    for (int m0 = -p.mmax[0]; m0 <= p.mmax[0]; ++m0)
                        for (int m1 = -p.mmax[1]; m1 <= p.mmax[1]; ++m1)
                            for (int m2 = -p.mmax[2]; m2 <= p.mmax[2]; ++m2) {
                                double v[3];
                                for (int c = 0; c < 3; ++c)
                                    v[c] = m0 * m->bvec[c] + m1 * m->bvec[3 + c] + m2 * m->bvec[6 + c];
                                const double nrm = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                                if (!(nrm < d->gcut) || !(nrm > 1e-12)) continue;
                                double kek = 0.0;
                                for (int a = 0; a < 3; ++a)
                                    for (int b2 = 0; b2 < 3; ++b2) kek += v[a] * d->eps_inf[3 * a + b2] * v[b2];
                                const double damp = std::exp(-kek / (4.0 * d->alpha_ewald)) / kek;
                                for (int k1 = 0; k1 < nat; ++k1) {
                                    double z1[3];
                                    for (int a = 0; a < 3; ++a) {
                                        z1[a] = 0.0;
                                        for (int b2 = 0; b2 < 3; ++b2) z1[a] += v[b2] * d->zstar[(k1 * 3 + b2) * 3 + a];
                                    }
                                    for (int k2 = 0; k2 < nat; ++k2) {
                                        double z2[3], arg = 0.0;
                                        for (int a = 0; a < 3; ++a) {
                                            z2[a] = 0.0;
                                            for (int b2 = 0; b2 < 3; ++b2) z2[a] += v[b2] * d->zstar[(k2 * 3 + b2) * 3 + a];
                                            arg += v[a] * (d->tau[3 * k1 + a] - d->tau[3 * k2 + a]);
                                        }
                                        for (int a = 0; a < 3; ++a)
                                            for (int b2 = 0; b2 < 3; ++b2) {
                                                corr[2 * ((k1 * 3 + a) * 3 + b2)] += damp * z1[a] * z2[b2] * std::cos(arg);
                                                corr[2 * ((k1 * 3 + a) * 3 + b2) + 1] += damp * z1[a] * z2[b2] * std::sin(arg);
                                            }
                                    }
                                }
                            }
                    m->d_dipcorr = (double*)up(corr.data(), corr.size() * sizeof(double));
                }
            }
        } catch (...) {
            delete m;
            throw;
        }
        *out = m;
    });
}

extern "C" int ephx_model_set_g(ephx_model* m, const double* g, void* stream) {
    return guarded([&] {
        require(m != nullptr && g != nullptr, "model_set_g: null argument");
        if (m->g_c64) throw Error{EPHX_EUNSUPPORTED, "model_set_g: the model's g is counter-drawn (complex float)"};
        hipStream_t st = (hipStream_t)stream;
        const long rows = (long)m->n_rp_g * m->nm * m->nw;
        const size_t bytes = (size_t)m->n_re_g * rows * m->nw * 16;
        // check the new values (and bound them for the fp16 scale) before they
        // replace the model's copy
        unsigned long long* red = (unsigned long long*)m->ws.get("setg.red", 2 * sizeof(unsigned long long));
        g_row_bound(m->n_re_g, rows, m->nw, g, m->d_wg, (long)m->nm * m->nw, m->n_rp_g, red, st);
        unsigned long long h[2] = {0, 0};
        hip_check(hipMemcpyAsync(h, red, sizeof(h), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        if (h[1]) throw Error{EPHX_ENAN, "model_set_g: non-finite entry in g"};
        double rowmax;
        std::memcpy(&rowmax, &h[0], sizeof(rowmax));
        hip_check(hipMemcpyAsync(m->d_g, g, bytes, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
        if (m->d_wg) scale_rows((long)m->n_re_g * m->n_rp_g, (long)m->nm * m->nw * m->nw, m->d_wg, m->d_g, st);
        m->g_scale = fp16_scale(2.0 * rowmax);
    });
}

extern "C" int ephx_model_g_entries(ephx_model* m, int n, const int64_t* idx, double* out) {
    return guarded([&] {
        require(m != nullptr && (n == 0 || (idx && out)), "model_g_entries: null argument");
        require(n >= 0, "model_g_entries: n < 0");
        const int64_t total = (int64_t)m->n_re_g * m->n_rp_g * m->nm * m->nw * m->nw;
        for (int i = 0; i < n; ++i) require(idx[i] >= 0 && idx[i] < total, "model_g_entries: index out of range");
        for (int i = 0; i < n; ++i) {
            if (m->g_c64) {
                float v[2];
                hip_check(hipMemcpy(v, m->d_g32 + 2 * idx[i], 8, hipMemcpyDeviceToHost), "hipMemcpy");
                out[2 * i] = v[0];
                out[2 * i + 1] = v[1];
            } else {
                hip_check(hipMemcpy(out + 2 * i, m->d_g + 2 * idx[i], 16, hipMemcpyDeviceToHost), "hipMemcpy");
            }
        }
    });
}

extern "C" int ephx_model_destroy(ephx_model* m) {
    return guarded([&] {
        if (!m) return;
        (void)hipDeviceSynchronize();
        delete m;
    });
}

namespace ephx {

// eps/U (and optionally velocities) for nk points; chunked.
void bands_impl(ephx_model* m, int nk, const double* k, double* eps, double* u, double* vel, hipStream_t st,
                const std::string& tag) {
    const int nw = m->nw, nw2 = nw * nw;
    const int chunk = 1 << 16;
    for (int k0 = 0; k0 < nk; k0 += chunk) {
        const int n = std::min(chunk, nk - k0);
        double* hk = (double*)m->ws.get(tag + ".hk", (size_t)n * nw2 * 16);
        phase_gemm_herm_f64(n, nw2, m->n_re_half, 1, k + 3L * k0, nullptr, m->d_re_half, m->d_h_half, hk, 0, st);
        double* uu = u ? u + (size_t)k0 * nw2 * 2 : (vel ? (double*)m->ws.get(tag + ".u", (size_t)n * nw2 * 16) : nullptr);
        eig_herm(n, nw, hk, 0, nw2, eps + (size_t)k0 * nw, uu, st);
        if (vel) {
            double* dh = (double*)m->ws.get(tag + ".dh", (size_t)n * 3 * nw2 * 16);
            phase_gemm_f64(n, 3 * nw2, m->n_re, 1, k + 3L * k0, nullptr, m->d_re, m->d_hvel, 0, dh, 0, st);
            band_velocity(n, nw, dh, uu, eps + (size_t)k0 * nw, vel + (size_t)k0 * nw * 3, st);
        }
    }
}

void phonons_impl(ephx_model* m, int nq, const double* q, double* omega, double* evec, hipStream_t st,
                  const std::string& tag) {
    const int nm = m->nm, nm2 = nm * nm;
    const int chunk = 1 << 17;
    for (int q0 = 0; q0 < nq; q0 += chunk) {
        const int n = std::min(chunk, nq - q0);
        double* dq = (double*)m->ws.get(tag + ".dq", (size_t)n * nm2 * 16);
        phase_gemm_f64(n, nm2, m->n_rp_ph, 1, q + 3L * q0, nullptr, m->d_rp_ph, m->d_cm, 0, dq, 0, st);
        if (m->dipole) dipole_add(n, q + 3L * q0, m->pd, m->d_dipcorr, m->d_minv, dq, st);
        eig_herm(n, nm, dq, 0, nm2, omega + (size_t)q0 * nm, evec ? evec + (size_t)q0 * nm2 * 2 : nullptr, st);
    }
    phonon_omega((long)nq * nm, omega, st);
}

// Shared driver of ephx_gkq (rates == false) and ephx_rates (rates == true).
// Batch shape of the rates / |g|^2 driver: bk_eff k points x qc q points per
// inner step, and the sizes of its work buffers.
struct DriverPlan {
    int nw, nm, nw2, bk_eff, qc, kp, nsplit;
    long ngcol, nre_cols;
    bool f32, wide;
    size_t npair;
    bool f16;      // split parts in fp16 (FP16x3)
    bool half;     // Rp sum over the half set with real coefficients
    int kh, kh16;  // half-set size, and rounded up to 16
};

size_t driver_workspace_bytes(const ephx_model* m, const DriverPlan& d, int nq, bool rates);

// The plan; wide_gib sets the per-pair buffers of large models (GiB).
static DriverPlan driver_plan_mem(const ephx_model* m, int nk, int nq, int precision, long wide_gib) {
    DriverPlan d{};
    d.nw = m->nw;
    d.nm = m->nm;
    d.nw2 = d.nw * d.nw;
    d.ngcol = (long)d.nm * d.nw2;                    // columns of the Rp contraction
    d.nre_cols = (long)m->n_rp_g * d.ngcol;          // columns of the Re contraction
    d.f32 = precision != EPHX_FP64;
    // k per Re contraction pass: g(k,Rp) and g(k,Rp)U(k) in FP64 take 32 bytes
    // per column and k; 3 GiB of them, or, for a counter-drawn complex-float
    // g (whose every pass reads the whole tensor), up to 8 k within 32 GiB
    const size_t kbudget = m->g_c64 ? ((size_t)32 << 30) : ((size_t)3 << 30);
    int bk = std::max(1, std::min(nk, std::max(1, (int)(kbudget / (d.nre_cols * 16 * 2)))));
    if (m->g_c64) bk = std::min(bk, 8);
    // large models: the per-pair blocks (nm nw^2 complex, twice) set the chunk size
    d.wide = d.nw > kMaxNw || d.nm > kMaxModes;
    const long pair_bytes = d.ngcol * (d.f32 ? 8 : 16) * 2 + (long)d.nw2 * 48;
    const long wide_pairs = std::max(16L, (wide_gib << 30) / pair_bytes);
    // up to 32 k per batch (16 for large models): the q-only work of a chunk
    // (phase planes and table, mode factors) is done once per batch
    d.bk_eff = std::min(bk, 32);
    if (d.wide) d.bk_eff = std::max(1, std::min<int>(std::min(d.bk_eff, 16), (int)(wide_pairs / 16)));
    const long pairs_target = d.wide ? wide_pairs : 1L << 19;
    long qc = std::max(d.wide ? 1L : 64L, std::min((long)std::max(nq, 1), pairs_target / d.bk_eff));
    // whole 256-row tiles of the split contraction where the chunk allows
    if (d.wide && qc > 256) qc -= qc % 256;
    d.qc = (int)qc;
    // the half set pays whenever the Rp list holds a +/-R pair (R != 0)
    d.half = m->n_rp_half > 0 && m->n_rp_half < m->n_rp_g;
    d.kh = m->n_rp_half;
    d.kh16 = ((d.kh + 15) / 16) * 16;
    d.kp = d.half ? 2 * d.kh16 : ((m->n_rp_g + 31) / 32) * 32;
    d.nsplit = (precision == EPHX_BF16X3 || precision == EPHX_FP16X3) ? 2 : (precision == EPHX_BF16X6 ? 3 : 0);
    d.f16 = precision == EPHX_FP16X3;
    d.npair = (size_t)d.bk_eff * d.qc;
    return d;
}

// Large models take 6 GiB of per-pair buffers, or 16 GiB when the device holds
// them beside the call's other buffers and 8 GiB of headroom (free memory plus
// the buffers the model already holds): the q chunk, the row count of the Rp
// contraction, then fills its 256-row tiles (the large cell: 96 -> 256 q per
// chunk at 8 k).
DriverPlan driver_plan(const ephx_model* m, int nk, int nq, int precision) {
    const DriverPlan d6 = driver_plan_mem(m, nk, nq, precision, 6);
    if (!d6.wide) return d6;
    const DriverPlan d16 = driver_plan_mem(m, nk, nq, precision, 16);
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        fr = 0;
    }
    size_t held = 0;
    for (const auto& kv : m->ws.bufs) held += kv.second.size;
    return fr + held >= driver_workspace_bytes(m, d16, nq, true) + ((size_t)8 << 30) ? d16 : d6;
}

// H(k+q) of every pair of a (k batch) x (q chunk) block, pair index k * nq + q,
// and its eigenpairs, in FP64.  With the packed half set (nw <= 8) the phases of
// the k batch are folded into the coefficients once per batch (hfold) and each
// H(k+q) is formed as nw*nw packed reals: one cos/sin(2 pi q.R) serves every k
// and the Hermitian output needs half the products of the complex one.
static void hkq_fold(ephx_model* m, int nb, const double* kb, double* hfold, hipStream_t st) {
    if (m->d_h_pack) fold_herm_f64(nb, kb, m->n_re_half, m->d_re_half, m->h_pack, m->d_h_pack, hfold, st);
}
static void hkq_fourier(ephx_model* m, int nb, const double* kb, const double* hfold, int nq, const double* qb,
                        double* hkq, hipStream_t st) {
    const int nw2 = m->nw * m->nw;
    if (m->d_h_pack)
        phase_gemm_herm_groups_f64(nq, nb, m->h_pack, m->n_re_half, qb, m->d_re_half, hfold, hkq,
                                   (double*)m->ws.get("hkq.ptab", (size_t)nq * m->n_re_half * 16), st);
    else
        phase_gemm_herm_f64(nq, nw2, m->n_re_half, nb, qb, kb, m->d_re_half, m->d_h_half, hkq, (long)nq * nw2, st);
}
// H(k+q) eigenpairs; U(k+q) column-major per matrix when want_cm and the
// one-lane solver runs (the epilogues read either layout, the batched-GEMM
// path of large models only row-major).  Returns the layout written.
static int hkq_eig(ephx_model* m, long npair, double* hkq, double* ekq, double* ukq, bool want_cm, hipStream_t st) {
    if (m->d_h_pack) {
        eig_herm_packed((int)npair, m->nw, hkq, m->h_pack, ekq, ukq, want_cm ? 1 : 0, st);
        return want_cm ? 1 : 0;
    }
    eig_herm((int)npair, m->nw, hkq, 0, m->nw * m->nw, ekq, ukq, st);
    return 0;
}
static size_t hfold_bytes(const ephx_model* m, int nb) {
    return m->d_h_pack ? (size_t)m->n_re_half * 2 * nb * m->h_pack * 8 : 0;
}

// Bytes of the driver's work buffers for one call of this shape (the buffers
// eph_driver, and the band and phonon interpolation it calls, take from the
// model's workspace).
size_t driver_workspace_bytes(const ephx_model* m, const DriverPlan& d, int nq, bool rates) {
    const size_t nm = d.nm, nw = d.nw, nw2 = d.nw2;
    size_t b = (size_t)nq * nm * 8 + (size_t)nq * nm * nm * 16;          // omega, e
    if (m->polar) b += (size_t)nq * nm * 16;                              // long-range term
    b += (size_t)std::min(nq, 1 << 17) * nm * nm * 16;                    // D(q) chunk
    b += (size_t)d.bk_eff * (nw * 8 + nw2 * 16 + nw2 * 16);               // eps(k), U(k), H(k)
    b += (size_t)d.bk_eff * d.nre_cols * 16 * 2;                          // g(k,Rp), g(k,Rp) U(k)
    if (!d.nsplit && d.half) b += (size_t)d.bk_eff * d.kh * 2 * d.ngcol * (d.f32 ? 8 : 16);   // half-set coefficients
    else if (!d.nsplit && d.f32) b += (size_t)d.bk_eff * d.nre_cols * 8;
    if (d.nsplit) {
        b += (size_t)d.bk_eff * 2 * d.nsplit * d.ngcol * d.kp * 2;        // B planes
        b += (size_t)2 * d.nsplit * d.qc * d.kp * 2;                      // phase planes
    }
    b += d.npair * (nw2 * 16 + nw * 8 + nw2 * 16);                        // H(k+q), eps, U
    b += hfold_bytes(m, d.bk_eff);                                        // k-folded half set
    if (m->d_h_pack) b += (size_t)d.qc * m->n_re_half * 16;                  // phase table of H(k+q)
    if (m->g_c64) b += (size_t)d.bk_eff * m->n_re_g * 16;                    // phase table of the Re sum
    b += d.npair * d.ngcol * (d.f32 ? 8 : 16) * (d.wide ? 2 : 1);         // g^W (and g^H)
    if (d.wide) b += (size_t)d.qc * nm * nm * 16 + (m->polar ? d.npair * nw2 * 16 : 0);
    if (rates) b += (size_t)d.bk_eff * eph_epilogue_blocks(d.qc) * nw * nm * 8 + (size_t)d.bk_eff * nw * nm * 8;
    if (!d.wide) b += (size_t)d.qc * nm * nm * (d.f32 ? 8 : 16) + (size_t)d.qc * nm * 8 + (rates ? d.npair * nw * 8 : 0);
    return b;
}

void eph_driver(ephx_model* m, int nk, const double* k, int nq, const double* q, int precision,
                double omega_cut, void* g2, const ephx_params* p, const double* qw, double* gamma,
                double* gmode, hipStream_t st, int part = 0) {
    const DriverPlan dp = driver_plan(m, nk, nq, precision);
    const int nw = dp.nw, nm = dp.nm, nw2 = dp.nw2;
    const long ngcol = dp.ngcol;
    const long nre_cols = dp.nre_cols;
    const bool f32 = dp.f32;
    // phonons (and the long-range term) at every q of the call
    double* om = (double*)m->ws.get("drv.omega", (size_t)nq * nm * 8);
    double* ev = (double*)m->ws.get("drv.evec", (size_t)nq * nm * nm * 16);
    {
        StageTimer t("phonons", st);
        phonons_impl(m, nq, q, om, ev, st, "drv");
    }
    double* lr = nullptr;
    if (m->polar) {
        lr = (double*)m->ws.get("drv.lr", (size_t)nq * nm * 16);
        frohlich(nq, q, m->pd, lr, st);
    }
    // batch sizes: bk_eff k points x qc q points per inner step
    const bool wide = dp.wide;
    const int bk_eff = dp.bk_eff;
    const int qc = dp.qc;
    const int kp = dp.kp;

    double* ek = (double*)m->ws.get("drv.ek", (size_t)bk_eff * nw * 8);
    double* uk = (double*)m->ws.get("drv.uk", (size_t)bk_eff * nw2 * 16);
    double* gk = (double*)m->ws.get("drv.gk", (size_t)bk_eff * nre_cols * 16);
    double* gp = (double*)m->ws.get("drv.gp", (size_t)bk_eff * nre_cols * 16);
    float* gp32 = nullptr;
    uint16_t* gpbf = nullptr;
    void* gph = nullptr;   // half-set coefficients [k][Kh][2][ngcol] complex (FP64, FP32)
    const bool half = dp.half;
    // fp16 parts: g(k,Rp) U(k) scaled into fp16 range (bf16 keeps FP32's range)
    const int f16s = dp.f16 ? 1 : 0;
    const double gsc = dp.f16 ? m->g_scale : 1.0;
    if (half && !dp.nsplit) gph = m->ws.get("drv.gph", (size_t)bk_eff * dp.kh * 2 * ngcol * (f32 ? 8 : 16));
    if (precision == EPHX_FP32 && !half) gp32 = (float*)m->ws.get("drv.gp32", (size_t)bk_eff * nre_cols * 8);
    const int nsplit = dp.nsplit;
    uint16_t* qpl = nullptr;
    if (nsplit) {
        gpbf = (uint16_t*)m->ws.get("drv.gpbf", (size_t)bk_eff * 2 * nsplit * ngcol * kp * 2);
        qpl = (uint16_t*)m->ws.get("drv.qpl", (size_t)2 * nsplit * qc * kp * 2);
    }
    const size_t npair = dp.npair;
    void* hkq = m->ws.get("drv.hkq", npair * nw2 * 16);
    double* hfold = (double*)m->ws.get("drv.hfold", hfold_bytes(m, bk_eff));
    double* ekq = (double*)m->ws.get("drv.ekq", npair * nw * 8);
    double* ukq = (double*)m->ws.get("drv.ukq", npair * nw2 * 16);
    void* gw = m->ws.get("drv.gw", npair * ngcol * (f32 ? 8 : 16));
    void* gh = wide ? m->ws.get("drv.gh", npair * ngcol * (f32 ? 8 : 16)) : nullptr;
    double* pmat = wide ? (double*)m->ws.get("drv.pmat", (size_t)qc * nm * nm * 16) : nullptr;
    double* ovb = wide && m->polar ? (double*)m->ws.get("drv.ov", npair * nw2 * 16) : nullptr;
    const int nblk = eph_epilogue_blocks(qc);
    void* esq = nullptr;
    double *nbq = nullptr, *fkq = nullptr;
    if (!wide) {
        esq = m->ws.get("drv.esq", (size_t)qc * nm * nm * (f32 ? 8 : 16));
        nbq = (double*)m->ws.get("drv.nbq", (size_t)qc * nm * 8);
        if (gamma) fkq = (double*)m->ws.get("drv.fkq", npair * nw * 8);
    }
    double* partial = nullptr;
    double* acc = nullptr;
    if (gamma) {
        partial = (double*)m->ws.get("drv.partial", (size_t)bk_eff * nblk * nw * nm * 8);
        acc = (double*)m->ws.get("drv.acc", (size_t)bk_eff * nw * nm * 8);
    }
    int u_cm = 0;   // layout of U(k+q) the eigensolver wrote (column-major: 1)
    for (int k0 = 0; k0 < nk; k0 += bk_eff) {
        const int nb = std::min(bk_eff, nk - k0);
        const double* kb = k + 3L * k0;
        bands_impl(m, nb, kb, ek, uk, nullptr, st, "drv.bk");
        {
            StageTimer t("hkq_fourier", st);
            hkq_fold(m, nb, kb, hfold, st);
        }
        // Re contraction (FP64, amortised over all q), then U(k) on the right
        {
            StageTimer t("re_contraction", st);
            if (m->g_c64)
                phase_gemm_f64_b32(nb, (int)nre_cols, m->n_re_g, 1, kb, nullptr, m->d_re_g, m->d_g32, 0, gk, 0,
                                   (double*)m->ws.get("drv.retab", (size_t)bk_eff * m->n_re_g * 16), st);
            else
                phase_gemm_f64(nb, (int)nre_cols, m->n_re_g, 1, kb, nullptr, m->d_re_g, m->d_g, 0, gk, 0, st);
        }
        apply_u_right(nb, m->n_rp_g, nm, nw, gk, uk, gp, st);
        if (half) {
            if (nsplit)
                split_bf16_half(nsplit, f16s, gsc, nb, m->n_rp_g, (int)ngcol, dp.kh, dp.kh16, m->d_rp_pair, gp, gpbf,
                                st);
            else if (precision == EPHX_FP32)
                half_combine_f32(nb, m->n_rp_g, (int)ngcol, dp.kh, m->d_rp_pair, gp, (float*)gph, st);
            else
                half_combine_f64(nb, m->n_rp_g, (int)ngcol, dp.kh, m->d_rp_pair, gp, (double*)gph, st);
        } else {
            if (precision == EPHX_FP32) convert_f64_f32((long)nb * nre_cols * 2, gp, gp32, st);
            if (nsplit) split_bf16_f64(nsplit, f16s, gsc, nb, m->n_rp_g, (int)ngcol, kp, gp, gpbf, st);
        }
        if (acc) hip_check(hipMemsetAsync(acc, 0, (size_t)nb * nw * nm * 8, st), "hipMemsetAsync");
        for (int q0 = 0; q0 < nq; q0 += qc) {
            const int nqc = std::min(qc, nq - q0);
            const double* qb = q + 3L * q0;
            // H(k+q) for every pair and its eigenpairs, in FP64 for every precision:
            // an FP32 sum perturbs H by ~1e-7 |H| and mixes bands closer than
            // ~1e-2 eV at the 1e-5 level of |g|^2.
            {
                StageTimer t("hkq_fourier", st);
                hkq_fourier(m, nb, kb, hfold, nqc, qb, (double*)hkq, st);
            }
            {
                StageTimer t("eig_hkq", st);
                u_cm = hkq_eig(m, (long)nb * nqc, (double*)hkq, ekq, ukq, !wide, st);
            }
            // phases of the q chunk for the split-bf16 paths, shared by every k of the batch
            if (nsplit) {
                StageTimer tph("rp_phases", st);
                if (half)
                    phase_planes_half(nsplit, f16s, nqc, dp.kh, dp.kh16, qb, m->d_rp_half, qpl, st);
                else
                    phase_planes_bf16(nsplit, f16s, nqc, m->n_rp_g, kp, qb, m->d_rp_g, qpl, st);
            }
            // Rp contraction per k
            StageTimer trp("rp_contraction", st);
            const long sh = (long)dp.kh * 2 * ngcol;
            if (nsplit)
                gemm_bf16_planes(nsplit, f16s, nqc, (int)ngcol, kp, nb, qpl, gpbf, 2L * nsplit * ngcol * kp,
                                 (float*)gw, (long)nqc * ngcol, half ? 1 : 0, (float)(1.0 / gsc), st);
            else if (half && precision == EPHX_FP64)
                phase_gemm_half_f64(nqc, (int)ngcol, dp.kh, nb, qb, m->d_rp_half, (const double*)gph, sh,
                                    (double*)gw, (long)nqc * ngcol, st);
            else if (half)
                phase_gemm_half_f32(nqc, (int)ngcol, dp.kh, nb, qb, m->d_rp_half, (const float*)gph, sh, (float*)gw,
                                    (long)nqc * ngcol, st);
            else if (precision == EPHX_FP64)
                phase_gemm_f64(nqc, (int)ngcol, m->n_rp_g, nb, qb, nullptr, m->d_rp_g, gp, nre_cols, (double*)gw,
                               (long)nqc * ngcol, st);
            else
                phase_gemm_f32(nqc, (int)ngcol, m->n_rp_g, nb, qb, nullptr, m->d_rp_g, gp32, nre_cols, (float*)gw,
                               (long)nqc * ngcol, st);
            trp.stop();
            StageTimer tep("epilogue", st);
            if (wide) {
                WideChunk w{};
                w.nkb = nb;
                w.nq = nqc;
                w.q_off = q0;
                w.nw = nw;
                w.nm = nm;
                w.g = gw;
                w.gh = gh;
                w.pmat = pmat;
                w.ov = ovb;
                w.ukq = ukq;
                w.ekq = ekq;
                w.ek = ek;
                w.uk = uk;
                w.omega = om;
                w.evec = ev;
                w.lr = lr;
                w.minv = m->d_minv;
                w.omega_cut = omega_cut;
                w.g2 = g2;
                w.nq_total = nq;
                w.k_off = k0;
                if (gamma) {
                    w.temp = p->temp;
                    w.mu = p->mu;
                    w.sigma = p->sigma;
                    w.qw = qw;
                    w.uniform_w = 1.0 / nq;
                    w.partial = partial;
                    w.nblk = eph_epilogue_blocks(nqc);
                    w.qpb = (nqc + w.nblk - 1) / w.nblk;
                }
                eph_wide_chunk(w, f32 ? 1 : 0, gamma ? 1 : 0, st);
                if (gamma) rates_reduce(nb, w.nblk, nw, nm, partial, acc, st);
                continue;
            }
            EphEpilogue e{};
            e.nkb = nb;
            e.nq = nqc;
            e.q_off = q0;
            e.nw = nw;
            e.nm = nm;
            e.gw = gw;
            e.ukq = ukq;
            e.u_cm = u_cm;
            e.ekq = ekq;
            e.ek = ek;
            e.uk = uk;
            e.omega = om;
            e.evec = ev;
            e.lr = lr;
            e.minv = m->d_minv;
            e.omega_cut = omega_cut;
            if (gamma) {
                e.temp = p->temp;
                e.mu = p->mu;
                e.sigma = p->sigma;
            }
            // mode factors of the chunk's q, Fermi factors of its pairs: once per chunk
            e.esq = esq;
            e.nbq = nbq;
            e.fkq = gamma ? fkq : nullptr;
            eph_epilogue_factors(e, f32 ? 1 : 0, esq, nbq, gamma ? fkq : nullptr, st);
            if (!gamma) {
                e.g2 = g2;
                e.nq_total = nq;
                e.k_off = k0;
                eph_epilogue_g2(e, f32 ? 1 : 0, st);
            } else {
                e.qw = qw;
                e.uniform_w = 1.0 / nq;
                e.partial = partial;
                e.nblk = eph_epilogue_blocks(nqc);
                e.part = part;
                eph_epilogue_rates(e, f32 ? 1 : 0, st);
                rates_reduce(nb, e.nblk, nw, nm, partial, acc, st);
            }
        }
        if (gamma)
            rates_finish(nb, nw, nm, acc, gamma + (size_t)k0 * nw, gmode ? gmode + (size_t)k0 * nw * nm : nullptr, st);
    }
}

}  // namespace ephx

namespace ephx {

// Negated real-space vectors -Rp, -Re of g(Re,Rp) as doubles: the row points of
// the adjoint Fourier sums.  Created on first use and kept with the model.
void negated_vectors(ephx_model* m) {
    if (m->d_nrp_g) return;
    std::vector<int32_t> hv(3 * (m->n_rp_g + m->n_re_g));
    hip_check(hipMemcpy(hv.data(), m->d_rp_g, 3 * m->n_rp_g * 4, hipMemcpyDeviceToHost), "hipMemcpy");
    hip_check(hipMemcpy(hv.data() + 3 * m->n_rp_g, m->d_re_g, 3 * m->n_re_g * 4, hipMemcpyDeviceToHost), "hipMemcpy");
    std::vector<double> dv(hv.size());
    for (size_t i = 0; i < hv.size(); ++i) dv[i] = -(double)hv[i];
    m->d_nrp_g = (double*)dev_upload(dv.data(), dv.size() * 8);
    m->owned.push_back(m->d_nrp_g);
    m->d_nre_g = m->d_nrp_g + 3 * m->n_rp_g;
}

// dL/dg(Re,Rp) for L = sum_nk lam_nk Gamma_nk, FP64.  Recomputes the forward
// quantities per k batch and q chunk, then
//   per pair:  g'W_bar = U(k+q) sum_nu conj(e amp) 2c lam w D g        (adjoint epilogue)
//   g'(k,Rp)_bar += sum_q e^{-iq.Rp} g'W_bar(k,q)                      (adjoint Rp sum)
//   g(k,Rp)_bar   = g'(k,Rp)_bar U(k)^dag
//   g(Re,Rp)_bar += sum_k e^{-ik.Re} g(k,Rp)_bar                       (adjoint Re sum)
void rates_vjp_impl(ephx_model* m, const ephx_params* p, int nk, const double* k, int nq, const double* q,
                    const double* qw, const double* lam, double* gbar, hipStream_t st) {
    const int nw = m->nw, nm = m->nm, nw2 = nw * nw;
    const long ngcol = (long)nm * nw2;
    const long nre_cols = (long)m->n_rp_g * ngcol;
    double* om = (double*)m->ws.get("adj.omega", (size_t)nq * nm * 8);
    double* ev = (double*)m->ws.get("adj.evec", (size_t)nq * nm * nm * 16);
    phonons_impl(m, nq, q, om, ev, st, "adj");
    double* lr = nullptr;
    if (m->polar) {
        lr = (double*)m->ws.get("adj.lr", (size_t)nq * nm * 16);
        frohlich(nq, q, m->pd, lr, st);
    }
    negated_vectors(m);
    const bool wide = is_wide(m);
    const int bk = std::min(nk, 16);
    int qc = (int)std::max(64L, std::min((long)nq, (1L << 17) / bk));
    if (wide) {
        // large models: the per-pair blocks (g'^W, its adjoint and the GEMM work,
        // nm nw^2 complex each) set the chunk, about 6 GB of them
        const long per_pair = ngcol * 16 * 3 + (long)nw2 * 48 + (m->polar ? (long)nw2 * 16 : 0);
        qc = (int)std::max(1L, std::min((long)nq, std::max(16L, (6L << 30) / per_pair) / bk));
    }
    double* ek = (double*)m->ws.get("adj.ek", (size_t)bk * nw * 8);
    double* uk = (double*)m->ws.get("adj.uk", (size_t)bk * nw2 * 16);
    double* gk = (double*)m->ws.get("adj.gk", (size_t)bk * nre_cols * 16);
    double* gp = (double*)m->ws.get("adj.gp", (size_t)bk * nre_cols * 16);
    double* gpb = (double*)m->ws.get("adj.gpb", (size_t)bk * nre_cols * 16);
    const size_t npair = (size_t)bk * qc;
    double* hkq = (double*)m->ws.get("adj.hkq", npair * nw2 * 16);
    double* hfold = (double*)m->ws.get("adj.hfold", hfold_bytes(m, bk));
    double* ekq = (double*)m->ws.get("adj.ekq", npair * nw * 8);
    double* ukq = (double*)m->ws.get("adj.ukq", npair * nw2 * 16);
    double* gw = (double*)m->ws.get("adj.gw", npair * ngcol * 16);
    double* gwb = (double*)m->ws.get("adj.gwb", npair * ngcol * 16);
    double* gh = wide ? (double*)m->ws.get("adj.gh", npair * ngcol * 16) : nullptr;
    double* pmat = wide ? (double*)m->ws.get("adj.pmat", (size_t)qc * nm * nm * 16) : nullptr;
    double* ovb = wide && m->polar ? (double*)m->ws.get("adj.ov", npair * nw2 * 16) : nullptr;
    hip_check(hipMemsetAsync(gbar, 0, (size_t)m->n_re_g * nre_cols * 16, st), "hipMemsetAsync");
    int u_cm = 0;   // layout of U(k+q) the eigensolver wrote (column-major: 1)
    for (int k0 = 0; k0 < nk; k0 += bk) {
        const int nb = std::min(bk, nk - k0);
        const double* kb = k + 3L * k0;
        bands_impl(m, nb, kb, ek, uk, nullptr, st, "adj.bk");
        phase_gemm_f64(nb, (int)nre_cols, m->n_re_g, 1, kb, nullptr, m->d_re_g, m->d_g, 0, gk, 0, st);
        apply_u_right(nb, m->n_rp_g, nm, nw, gk, uk, gp, st);
        hkq_fold(m, nb, kb, hfold, st);
        for (int q0 = 0; q0 < nq; q0 += qc) {
            const int nqc = std::min(qc, nq - q0);
            const double* qb = q + 3L * q0;
            hkq_fourier(m, nb, kb, hfold, nqc, qb, hkq, st);
            u_cm = hkq_eig(m, (long)nb * nqc, hkq, ekq, ukq, !wide, st);
            phase_gemm_f64(nqc, (int)ngcol, m->n_rp_g, nb, qb, nullptr, m->d_rp_g, gp, nre_cols, gw,
                           (long)nqc * ngcol, st);
            if (wide) {
                WideChunk w{};
                w.nkb = nb;
                w.nq = nqc;
                w.q_off = q0;
                w.nw = nw;
                w.nm = nm;
                w.g = gw;
                w.gh = gh;
                w.pmat = pmat;
                w.ov = ovb;
                w.ukq = ukq;
                w.ekq = ekq;
                w.ek = ek;
                w.uk = uk;
                w.omega = om;
                w.evec = ev;
                w.lr = lr;
                w.minv = m->d_minv;
                w.omega_cut = p->omega_cut;
                w.temp = p->temp;
                w.mu = p->mu;
                w.sigma = p->sigma;
                w.qw = qw;
                w.uniform_w = 1.0 / nq;
                w.k_off = k0;
                eph_wide_rates_vjp(w, lam, gwb, st);
                phase_gemm_adj_f64(m->n_rp_g, (int)ngcol, nqc, nb, m->d_nrp_g, qb, gwb, (long)nqc * ngcol, gpb,
                                   nre_cols, q0 > 0 ? 1 : 0, st);
                continue;
            }
            EphEpilogue e{};
            e.nkb = nb;
            e.nq = nqc;
            e.q_off = q0;
            e.nw = nw;
            e.nm = nm;
            e.gw = gw;
            e.ukq = ukq;
            e.u_cm = u_cm;
            e.ekq = ekq;
            e.ek = ek;
            e.uk = uk;
            e.omega = om;
            e.evec = ev;
            e.lr = lr;
            e.minv = m->d_minv;
            e.omega_cut = p->omega_cut;
            e.temp = p->temp;
            e.mu = p->mu;
            e.sigma = p->sigma;
            e.qw = qw;
            e.uniform_w = 1.0 / nq;
            e.k_off = k0;
            eph_adjoint_epilogue(e, lam, gwb, st);
            // g'(k,Rp)_bar (+)= sum_q e^{-i q.Rp} g'W_bar(k,q): rows Rp, contraction over the q chunk
            phase_gemm_adj_f64(m->n_rp_g, (int)ngcol, nqc, nb, m->d_nrp_g, qb, gwb, (long)nqc * ngcol, gpb,
                               nre_cols, q0 > 0 ? 1 : 0, st);
        }
        apply_u_right_adj(nb, m->n_rp_g, nm, nw, gpb, uk, gk, st);
        // g(Re,Rp)_bar += sum_k e^{-i k.Re} g(k,Rp)_bar
        phase_gemm_adj_f64(m->n_re_g, (int)nre_cols, nb, 1, m->d_nre_g, kb, gk, 0, gbar, 0, 1, st);
    }
    if (m->d_wg) scale_rows((long)m->n_re_g * m->n_rp_g, ngcol, m->d_wg, gbar, st);
}

}  // namespace ephx

extern "C" int ephx_rates_vjp(ephx_model* m, const ephx_params* p, int nk, const double* k_red, int nq,
                              const double* q_red, const double* q_w, const double* gamma_bar, double* g_bar,
                              void* stream) {
    return guarded([&] {
        require(m != nullptr && p != nullptr, "rates_vjp: null argument");
        require(nk >= 0 && nq >= 0, "rates_vjp: negative size");
        require(p->temp > 0 && p->sigma > 0 && std::isfinite(p->mu) && std::isfinite(p->omega_cut),
                "rates_vjp: need temp > 0, sigma > 0, finite mu and omega_cut");
        require(g_bar != nullptr, "rates_vjp: null output");
        if (m->g_c64)
            throw Error{EPHX_EUNSUPPORTED, "rates_vjp: not built for a counter-drawn (complex float) g"};
        hipStream_t st = (hipStream_t)stream;
        if (nk == 0 || nq == 0) {
            hip_check(hipMemsetAsync(g_bar, 0, (size_t)m->n_re_g * m->n_rp_g * m->nm * m->nw * m->nw * 16, st),
                      "hipMemsetAsync");
            return;
        }
        require(k_red && q_red && gamma_bar, "rates_vjp: null array");
        rates_vjp_impl(m, p, nk, k_red, nq, q_red, q_w, gamma_bar, g_bar, st);
    });
}

extern "C" int ephx_bands(ephx_model* m, int nk, const double* k_red, double* eps, double* u, double* vel,
                          void* stream) {
    return guarded([&] {
        require(m != nullptr, "bands: null model");
        require(nk >= 0, "bands: nk < 0");
        if (nk == 0) return;
        require(k_red && eps, "bands: null array");
        if (vel && m->nw > kMaxNw) throw Error{EPHX_EUNSUPPORTED, "bands: velocities not built for nw > 16"};
        bands_impl(m, nk, k_red, eps, u, vel, (hipStream_t)stream, "bands");
    });
}

extern "C" int ephx_phonons(ephx_model* m, int nq, const double* q_red, double* omega, double* evec, void* stream) {
    return guarded([&] {
        require(m != nullptr, "phonons: null model");
        require(nq >= 0, "phonons: nq < 0");
        if (nq == 0) return;
        require(q_red && omega, "phonons: null array");
        phonons_impl(m, nq, q_red, omega, evec, (hipStream_t)stream, "phonons");
    });
}

static void check_precision(int precision) {
    require(precision == EPHX_FP64 || precision == EPHX_FP32 || precision == EPHX_BF16X3 ||
                precision == EPHX_BF16X6 || precision == EPHX_FP16X3,
            "unknown precision");
}

extern "C" int ephx_gkq(ephx_model* m, int nk, const double* k_red, int nq, const double* q_red, int precision,
                        double omega_cut, void* g2, void* stream) {
    return guarded([&] {
        require(m != nullptr, "gkq: null model");
        require(nk >= 0 && nq >= 0, "gkq: negative size");
        if (nk == 0 || nq == 0) return;
        require(k_red && q_red && g2, "gkq: null array");
        require(std::isfinite(omega_cut), "gkq: omega_cut not finite");
        check_precision(precision);
        eph_driver(m, nk, k_red, nq, q_red, precision, omega_cut, g2, nullptr, nullptr, nullptr, nullptr,
                   (hipStream_t)stream);
    });
}

extern "C" int ephx_gkq_pairs(ephx_model* m, int nk, const double* k_red, int nq, const double* q_red, int npairs,
                              const int32_t* ik, const int32_t* iq, int precision, double omega_cut, void* g2,
                              void* stream) {
    return guarded([&] {
        require(m != nullptr, "gkq_pairs: null model");
        require(nk >= 0 && nq >= 0 && npairs >= 0, "gkq_pairs: negative size");
        if (npairs == 0) return;
        require(k_red && q_red && ik && iq && g2, "gkq_pairs: null array");
        require(std::isfinite(omega_cut), "gkq_pairs: omega_cut not finite");
        check_precision(precision);
        for (int j = 0; j < npairs; ++j)
            require(0 <= ik[j] && ik[j] < nk && 0 <= iq[j] && iq[j] < nq, "gkq_pairs: pair index out of range");
        hipStream_t st = (hipStream_t)stream;
        // pairs grouped by k (stable): each group is one k against its q list
        std::vector<int32_t> order(npairs);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return ik[a] < ik[b]; });
        std::vector<int32_t> qsel(npairs);
        for (int j = 0; j < npairs; ++j) qsel[j] = iq[order[j]];
        int32_t* d_qsel = (int32_t*)m->ws.get("gp.qsel", (size_t)npairs * 4);
        int32_t* d_pos = (int32_t*)m->ws.get("gp.pos", (size_t)npairs * 4);
        double* d_q = (double*)m->ws.get("gp.q", (size_t)npairs * 3 * 8);
        hip_check(hipMemcpyAsync(d_qsel, qsel.data(), (size_t)npairs * 4, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
        hip_check(hipMemcpyAsync(d_pos, order.data(), (size_t)npairs * 4, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
        gather_points(npairs, d_qsel, q_red, d_q, st);
        const long words = (long)m->nm * m->nw * m->nw * (precision == EPHX_FP64 ? 2 : 1);
        int gmax = 0;
        for (int a = 0; a < npairs;) {
            int b = a;
            while (b < npairs && ik[order[b]] == ik[order[a]]) ++b;
            gmax = std::max(gmax, b - a);
            a = b;
        }
        void* tmp = m->ws.get("gp.out", (size_t)gmax * words * 4);
        for (int a = 0; a < npairs;) {
            int b = a;
            while (b < npairs && ik[order[b]] == ik[order[a]]) ++b;
            eph_driver(m, 1, k_red + 3L * ik[order[a]], b - a, d_q + 3L * a, precision, omega_cut, tmp, nullptr,
                       nullptr, nullptr, nullptr, st);
            scatter_blocks(b - a, d_pos + a, tmp, g2, words, st);
            a = b;
        }
        // the host index arrays above are read by the copies queued on st
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    });
}

extern "C" int ephx_workspace_query(ephx_model* m, int call, int nk, int nq, int precision, size_t* bytes) {
    return guarded([&] {
        require(m != nullptr && bytes != nullptr, "workspace_query: null argument");
        require(call == EPHX_CALL_GKQ || call == EPHX_CALL_RATES, "workspace_query: unknown call");
        require(nk >= 0 && nq >= 0, "workspace_query: negative size");
        check_precision(precision);
        *bytes = 0;
        if (nk == 0 || nq == 0) return;
        const DriverPlan d = driver_plan(m, nk, nq, precision);
        *bytes = driver_workspace_bytes(m, d, nq, call == EPHX_CALL_RATES);
    });
}

extern "C" int ephx_rates(ephx_model* m, const ephx_params* p, int nk, const double* k_red, int nq,
                          const double* q_red, const double* q_w, int precision, double* gamma, double* gamma_mode,
                          void* stream) {
    return ephx_rates_part(m, p, EPHX_PART_FULL, nk, k_red, nq, q_red, q_w, precision, gamma, gamma_mode, stream);
}

extern "C" int ephx_rates_part(ephx_model* m, const ephx_params* p, int part, int nk, const double* k_red, int nq,
                               const double* q_red, const double* q_w, int precision, double* gamma,
                               double* gamma_mode, void* stream) {
    return guarded([&] {
        require(m != nullptr && p != nullptr, "rates: null argument");
        require(part == EPHX_PART_FULL || part == EPHX_PART_POLAR || part == EPHX_PART_RMPOL,
                "rates: part must be EPHX_PART_FULL, EPHX_PART_POLAR or EPHX_PART_RMPOL");
        require(part == EPHX_PART_FULL || m->polar, "rates: the polar and rmpol parts need a polar model");
        if (part != EPHX_PART_FULL && is_wide(m))
            throw Error{EPHX_EUNSUPPORTED, "rates: the polar and rmpol parts are not built for nw > 16 or more than "
                                           "12 modes"};
        require(nk >= 0 && nq >= 0, "rates: negative size");
        require(p->temp > 0 && p->sigma > 0 && std::isfinite(p->mu) && std::isfinite(p->omega_cut),
                "rates: need temp > 0, sigma > 0, finite mu and omega_cut");
        if (nk == 0) return;
        require(k_red && gamma, "rates: null array");
        check_precision(precision);
        if (nq == 0) {
            hip_check(hipMemsetAsync(gamma, 0, (size_t)nk * m->nw * 8, (hipStream_t)stream), "hipMemsetAsync");
            if (gamma_mode)
                hip_check(hipMemsetAsync(gamma_mode, 0, (size_t)nk * m->nw * m->nm * 8, (hipStream_t)stream),
                          "hipMemsetAsync");
            return;
        }
        require(q_red != nullptr, "rates: null q array");
        eph_driver(m, nk, k_red, nq, q_red, precision, p->omega_cut, nullptr, p, q_w, gamma, gamma_mode,
                   (hipStream_t)stream, part);
    });
}

extern "C" int ephx_rates_polar_split(ephx_model* m, const ephx_params* p, int nk, const double* k_red, int nq_u,
                                      const double* q_u, const double* w_u, int nq_c, const double* q_c,
                                      const double* w_c, int precision, double* gamma, double* gamma_mode,
                                      void* stream) {
    return guarded([&] {
        require(m != nullptr && p != nullptr, "rates_polar_split: null argument");
        require(m->polar, "rates_polar_split: needs a polar model");
        require(nk >= 0 && nq_u >= 0 && nq_c >= 0, "rates_polar_split: negative size");
        if (nk == 0) return;
        require(k_red && gamma, "rates_polar_split: null array");
        hipStream_t st = (hipStream_t)stream;
        // the long-range part on the second q set into work buffers, then the rest
        // on the first set into the outputs, then the sum
        double* g2 = (double*)m->ws.get("split.g", (size_t)nk * m->nw * 8);
        double* gm2 = gamma_mode ? (double*)m->ws.get("split.gm", (size_t)nk * m->nw * m->nm * 8) : nullptr;
        auto check = [](int rc) {
            if (rc != EPHX_OK) throw Error{rc, std::string("rates_polar_split: ") + g_last_error};
        };
        check(ephx_rates_part(m, p, EPHX_PART_POLAR, nk, k_red, nq_c, q_c, w_c, precision, g2, gm2, stream));
        check(ephx_rates_part(m, p, EPHX_PART_RMPOL, nk, k_red, nq_u, q_u, w_u, precision, gamma, gamma_mode,
                              stream));
        add_into((long)nk * m->nw, g2, gamma, st);
        if (gamma_mode) add_into((long)nk * m->nw * m->nm, gm2, gamma_mode, st);
    });
}
