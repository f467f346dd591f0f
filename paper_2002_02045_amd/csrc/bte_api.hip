// BTE entry points of the C ABI: grid states, pair tables, the collision
// integral, RK4 dynamics and their adjoints, and the iterative linearised BTE.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <unordered_map>
#include <vector>

#include "../../include/ephx.h"
#include "api_common.h"

using namespace ephx;

struct ephx_table {
    ephx_model* m = nullptr;
    int S = 0;
    int n1 = 0, n2 = 0, n3 = 0;
    int nm = 0, nw = 0;
    bool f32 = true;
    long ld = 0;
    int32_t* d_kc = nullptr;      // [S][3]
    int32_t* d_band = nullptr;    // [S]
    double* d_eps = nullptr;      // [S]
    double* d_omega = nullptr;    // [Ngrid][nm]
    void* d_g2 = nullptr;         // [nm][S][ld]
    void* d_p = nullptr;          // [S][ld] collision matrix
    void* d_w = nullptr;          // [S][ld] transport matrix
    void* d_pmode = nullptr;      // [nm][S][ld] collision matrix of each mode alone at unit scale
    double* d_eunit = nullptr;    // [nm][nm] unit scale vectors
    int pmode_gen = -1;           // gen[0] the per-mode matrices were built for
    const int32_t* panel_tiles = nullptr;   // live tiles of the per-mode matrices for the stage-panel gradient
    int n_panel_tiles = 0;
    int panel_gen = -1;
    double* d_scale = nullptr;    // [nm] collision mode scales
    double* d_unit = nullptr;     // [nm] ones (transport matrix)
    double* d_ones = nullptr;     // [S]
    ephx_params par{};
    double build_cut = 0.0;       // omega cut of the table's |g|^2
    bool ready = false;
    double c = 0.0;               // (2 pi/hbar)/N_q
    std::vector<void*> owned;
    Workspace ws;
    std::vector<int32_t> h_kc, h_band;   // host copies of the states
    int32_t* d_tet = nullptr;            // [n_tet][4] tetrahedra of window states, built on first use
    int n_tet = -1;
    int32_t* d_nbr = nullptr;            // [S][6] grid neighbours of each state (field drift), built on first use
    // P and W are stored with rows and columns in ascending state energy; tiles
    // of state pairs further apart than the band half-width are exact zeros
    int32_t* d_perm = nullptr;           // [S] state of each matrix row/column
    std::vector<double> h_esort;         // energies in that order
    double omega_max = -1.0;             // largest phonon energy on the grid
    double band[2] = {0.0, 0.0};         // half-widths of the stored P (0) and W (1)
    int gen[2] = {0, 0};                 // rebuild counters of P and W
    struct CachedPlan {
        StreamPlan pl;
        int gen;
    };
    std::map<int, CachedPlan> plans;     // key: matrix * 64 + na * 8 + nb
    ~ephx_table() {
        ws.release();
        for (void* p : owned)
            if (p) (void)hipFree(p);
    }
    void* alloc(size_t bytes) {
        void* p = dev_upload(nullptr, bytes);
        owned.push_back(p);
        return p;
    }
};

namespace {

void grid_dims(const int* n_grid, int& n1, int& n2, int& n3) {
    require(n_grid != nullptr, "null grid");
    n1 = n_grid[0];
    n2 = n_grid[1];
    n3 = n_grid[2];
    require(n1 >= 1 && n2 >= 1 && n3 >= 1, "grid dimensions must be >= 1");
    require((long)n1 * n2 * n3 <= (1L << 28), "grid too large");
}

std::vector<double> grid_points(int n1, int n2, int n3) {
    const long ng = (long)n1 * n2 * n3;
    std::vector<double> k(ng * 3);
    for (long i = 0; i < ng; ++i) {
        const long a = i / ((long)n2 * n3), b = (i / n3) % n2, c = i % n3;
        k[3 * i] = (double)a / n1;
        k[3 * i + 1] = (double)b / n2;
        k[3 * i + 2] = (double)c / n3;
    }
    return k;
}

// edge moved to the midpoint between the sorted energies straddling it
double snap_edge(const std::vector<double>& e, double edge) {
    auto it = std::lower_bound(e.begin(), e.end(), edge);
    if (e.empty()) return edge;
    if (it == e.begin()) return e.front() - 1.0;
    if (it == e.end()) return e.back() + 1.0;
    return 0.5 * (*(it - 1) + *it);
}

// Energy order of the states and the largest phonon energy, once per table.
void ensure_order(ephx_table* t, hipStream_t st) {
    if (t->d_perm) return;
    const int S = t->S;
    std::vector<double> e(S);
    const long nom = (long)t->n1 * t->n2 * t->n3 * t->nm;
    std::vector<double> om(nom);
    hip_check(hipMemcpyAsync(e.data(), t->d_eps, (size_t)S * 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hip_check(hipMemcpyAsync(om.data(), t->d_omega, (size_t)nom * 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    std::vector<int32_t> perm(S);
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return e[a] < e[b]; });
    t->h_esort.resize(S);
    for (int i = 0; i < S; ++i) t->h_esort[i] = e[perm[i]];
    double wmax = 0.0;
    for (double w : om)
        if (std::isfinite(w)) wmax = std::max(wmax, std::fabs(w));   // |omega|: a mode below a negative cut counts too
    t->omega_max = wmax;
    t->d_perm = (int32_t*)t->alloc((size_t)std::max(1, S) * 4);
    hip_check(hipMemcpy(t->d_perm, perm.data(), (size_t)S * 4, hipMemcpyHostToDevice), "hipMemcpy");
}

// Build P (matrix 0) or W (matrix 1) in energy order and record its band.
void build_banded(ephx_table* t, int matrix, const ephx_params* p, const double* scale, void* out, hipStream_t st) {
    ensure_order(t, st);
    StageTimer tm("matrix_build", st);
    // |e_s - e_t| > omega + 6 sigma (with a margin for rounding) puts both
    // delta arguments beyond the cut for every mode
    const double hw = t->omega_max + 6.0 * p->sigma * (1.0 + 1e-9) + 1e-12;
    build_matrix(matrix, t->S, t->nm, t->ld, t->d_g2, t->f32 ? 1 : 0, t->d_kc, t->n1, t->n2, t->n3, t->d_omega,
                 t->d_eps, p->temp, p->mu, p->sigma, p->omega_cut, scale, t->d_perm, out, hw, st);
    t->band[matrix] = hw;
    ++t->gen[matrix];
}

StreamPlan plan_for(ephx_table* t, int matrix, int na, int nb, hipStream_t st) {
    const int key = matrix * 64 + na * 8 + nb;
    auto it = t->plans.find(key);
    if (it != t->plans.end() && it->second.gen == t->gen[matrix]) return it->second.pl;
    std::vector<int32_t> tiles;
    int n_live = 0;
    StreamPlan pl = stream_plan_banded(t->S, t->f32 ? 1 : 0, na, nb, t->h_esort, t->band[matrix], tiles, n_live);
    // earlier passes on this stream may still read the old list
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    int32_t* d = (int32_t*)t->ws.get("tiles." + std::to_string(key), std::max<size_t>(8, tiles.size() * 4));
    if (!tiles.empty()) hip_check(hipMemcpy(d, tiles.data(), tiles.size() * 4, hipMemcpyHostToDevice), "hipMemcpy");
    pl.tiles = d;
    pl.perm = t->d_perm;
    const size_t S1 = (size_t)std::max(1, t->S);
    pl.gbuf = (double*)t->ws.get("gbuf." + std::to_string(key), (size_t)std::max(1, na + nb) * S1 * 8);
    pl.rout = na > 0 ? (double*)t->ws.get("rout." + std::to_string(key), (size_t)na * S1 * 8) : nullptr;
    pl.cout = nb > 0 ? (double*)t->ws.get("cout." + std::to_string(key), (size_t)nb * S1 * 8) : nullptr;
    t->plans[key] = {pl, t->gen[matrix]};
    return pl;
}

// The stage timer `tag` covers the streaming kernel alone; the gather and the
// reduction are timed as "stream_permute".
PassOut one_pass(ephx_table* t, const StreamPlan& pl, const void* mat, VecPtrs x, VecPtrs y, double* rowp,
                 double* colp, hipStream_t st, const char* tag) {
    {
        StageTimer tm("stream_permute", st);
        stream_gather(pl, x, y, st);
    }
    {
        StageTimer tm(tag, st);
        stream_run(pl, t->ld, mat, rowp, colp, st);
    }
    StageTimer tm("stream_permute", st);
    return stream_reduce(pl, rowp, colp, st);
}

// I at occupations y; optional RK4 stage update
// Field drift of the stage update: neighbour table and coefficients
struct Field {
    const int32_t* nbr = nullptr;
    double dc[3] = {0.0, 0.0, 0.0};
};

// gathered: the plan's gather buffer already holds y (written by the previous
// evaluation's finish); gather_next: this evaluation's finish writes the next
// one's occupations there (f_next, or acc when next_from_acc).
void collision_eval(ephx_table* t, const double* y, double* i_out, double* acc, int acc_init, double w_acc,
                    const double* f_base, double a_next, double* f_next, hipStream_t st,
                    const Field* fld = nullptr, bool gathered = false, bool gather_next = false,
                    bool next_from_acc = false) {
    const int S = t->S;
    const StreamPlan pl = plan_for(t, 0, 1, 1, st);
    double* rowp = (double*)t->ws.get("c.rowp", (size_t)pl.n_ct * S * 8);
    double* colp = (double*)t->ws.get("c.colp", (size_t)pl.n_rt * S * 8);
    // kernels per evaluation: 1 - f and f gathered to matrix order (unless the
    // previous finish did it), the stream over P, and the partials reduced and
    // finished in state order
    if (!gathered) {
        StageTimer tm("stream_permute", st);
        gather_occupations(pl, y, st);
    }
    {
        StageTimer tm("collision_stream", st);
        stream_run(pl, t->ld, t->d_p, rowp, colp, st);
    }
    CollisionFinish cf{};
    cf.S = S;
    cf.n_rt = pl.n_rt;
    cf.n_ct = pl.n_ct;
    cf.rowp = rowp;
    cf.colp = colp;
    cf.f = y;
    cf.c = t->c;
    cf.i_out = i_out;
    cf.acc = acc;
    cf.acc_init = acc_init;
    cf.w_acc = w_acc;
    cf.f_base = f_base;
    cf.a_next = a_next;
    cf.f_next = f_next;
    cf.nbr = fld ? fld->nbr : nullptr;
    for (int d = 0; d < 3; ++d) cf.dc[d] = fld ? fld->dc[d] : 0.0;
    if (gather_next && acc && (next_from_acc || f_next)) {
        cf.gnext = pl.gbuf;
        cf.gnext_acc = next_from_acc ? 1 : 0;
    }
    StageTimer tm("stream_permute", st);
    reduce_finish(pl, cf, st);
}

// The per-mode matrices P^nu = dP/ds_nu, in the layout and band of P, built
// when a mode-scale gradient is first asked for after each collision setup.
void ensure_pmode(ephx_table* t, hipStream_t st) {
    if (t->pmode_gen == t->gen[0]) return;
    const size_t esz = t->f32 ? 4 : 8, mat = (size_t)t->S * t->ld * esz;
    if (!t->d_pmode) {
        t->d_pmode = t->alloc(t->nm * mat);
        hip_check(hipMemsetAsync(t->d_pmode, 0, t->nm * mat, st), "hipMemsetAsync");
        std::vector<double> eu((size_t)t->nm * t->nm, 0.0);
        for (int nu = 0; nu < t->nm; ++nu) eu[(size_t)nu * t->nm + nu] = 1.0;
        t->d_eunit = (double*)t->alloc(eu.size() * 8);
        hip_check(hipMemcpyAsync(t->d_eunit, eu.data(), eu.size() * 8, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    }
    StageTimer tm("matrix_build", st);
    for (int nu = 0; nu < t->nm; ++nu)
        build_matrix(0, t->S, t->nm, t->ld, t->d_g2, t->f32 ? 1 : 0, t->d_kc, t->n1, t->n2, t->n3, t->d_omega,
                     t->d_eps, t->par.temp, t->par.mu, t->par.sigma, t->par.omega_cut, t->d_eunit + nu * t->nm,
                     t->d_perm, (char*)t->d_pmode + nu * mat, t->band[0], st);
    t->pmode_gen = t->gen[0];
}

// Live kPT x kPT tiles of the per-mode matrices (energy order, band of P),
// built once per collision setup.
void panel_tiles(ephx_table* t, hipStream_t st, const int32_t*& tiles, int& n) {
    if (t->panel_gen != t->gen[0]) {
        std::vector<int32_t> h;
        mode_panel_tiles(t->h_esort, t->band[0], h);
        // earlier launches on this stream may still read the old list
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        int32_t* d = (int32_t*)t->ws.get("panel.tiles", std::max<size_t>(8, h.size() * 4));
        if (!h.empty()) hip_check(hipMemcpy(d, h.data(), h.size() * 4, hipMemcpyHostToDevice), "hipMemcpy");
        t->panel_tiles = d;
        t->n_panel_tiles = (int)(h.size() / 2);
        t->panel_gen = t->gen[0];
    }
    tiles = t->panel_tiles;
    n = t->n_panel_tiles;
}

// s_bar (=/+=) sum_j lam_j^T dI/ds at f_j for ns pairs (f_j, lam_j): per mode,
// banded passes over P^nu with the rows (1-f_j) and lam_j (1-f_j), two pairs
// (four row vectors) per pass; the vectors of a pass are gathered once, and
// the partials of all modes are reduced together and finished in one launch.
void mode_grad(ephx_table* t, int ns, const double* const* f, const double* const* lam, double* sbar,
               int accumulate, hipStream_t st) {
    const int S = t->S;
    ensure_pmode(t, st);
    const size_t mat = (size_t)S * t->ld * (t->f32 ? 4 : 8);
    double* o[4];
    for (int q = 0; q < 4; ++q) o[q] = (double*)t->ws.get("v.om" + std::to_string(q), (size_t)S * 8);
    double* o2 = (double*)t->ws.get("v.omx", (size_t)S * 8);   // lam f, not used here
    for (int j0 = 0; j0 < ns; j0 += 2) {
        const int m = std::min(2, ns - j0);
        for (int jj = 0; jj < m; ++jj) occ_vectors(S, f[j0 + jj], lam[j0 + jj], o[2 * jj], o[2 * jj + 1], o2, st);
        const StreamPlan pm = plan_for(t, 0, 2 * m, 0, st);
        const size_t part = (size_t)2 * m * pm.n_ct * S;
        double* rowm = (double*)t->ws.get("v.rowm", (size_t)t->nm * 4 * pm.n_ct * S * 8);
        VecPtrs xm{{o[0], o[1], m > 1 ? o[2] : nullptr, m > 1 ? o[3] : nullptr}};
        VecPtrs ym{{nullptr, nullptr, nullptr, nullptr}};
        {
            StageTimer tm("stream_permute", st);
            stream_gather(pm, xm, ym, st);
        }
        {
            StageTimer tm("mode_stream", st);
            for (int nu = 0; nu < t->nm; ++nu)
                stream_run(pm, t->ld, (const char*)t->d_pmode + nu * mat, rowm + nu * part, nullptr, st);
        }
        StreamPlan pr = pm;
        pr.na = 2 * m * t->nm;
        pr.nb = 0;
        pr.rout = (double*)t->ws.get("v.routm", (size_t)4 * t->nm * S * 8);
        StageTimer tm("stream_permute", st);
        const PassOut po = stream_reduce(pr, rowm, nullptr, st);
        VecPtrs fv{{f[j0], m > 1 ? f[j0 + 1] : nullptr, nullptr, nullptr}};
        VecPtrs lv{{lam[j0], m > 1 ? lam[j0 + 1] : nullptr, nullptr, nullptr}};
        mode_finish(S, t->nm, m, po.rowp, fv, lv, t->c, sbar, accumulate || j0 > 0, st);
    }
}

// f_bar = lam^T dI/df at f; s_bar (=/+=) lam^T dI/ds
void collision_vjp_impl(ephx_table* t, const double* f, const double* lam, double* fbar, double* sbar,
                        int s_accumulate, hipStream_t st) {
    const int S = t->S;
    double* o0 = (double*)t->ws.get("v.o0", S * 8);
    double* o1 = (double*)t->ws.get("v.o1", S * 8);
    double* o2 = (double*)t->ws.get("v.o2", S * 8);
    const StreamPlan pl = plan_for(t, 0, 2, 2, st);
    double* rowp = (double*)t->ws.get("v.rowp", (size_t)2 * pl.n_ct * S * 8);
    double* colp = (double*)t->ws.get("v.colp", (size_t)2 * pl.n_rt * S * 8);
    occ_vectors(S, f, lam, o0, o1, o2, st);
    // rows: P(1-f), P(lam(1-f)); columns: P^T f, P^T (lam f)
    VecPtrs x{{o0, o1, nullptr, nullptr}}, y{{f, o2, nullptr, nullptr}};
    const PassOut po = one_pass(t, pl, t->d_p, x, y, rowp, colp, st, "collision_stream");
    vjp_finish(S, po.n_ct, po.n_rt, po.rowp, po.colp, lam, t->c, fbar, st);
    if (sbar) {
        mode_grad(t, 1, &f, &lam, sbar, s_accumulate, st);
    }
}

// One RK4 step f -> f_new; stage inputs optionally saved (Y1..Y4).  gathered:
// the collision plan's gather buffer holds f on entry; it holds f_new on exit
// (each stage's finish gathers the next stage's input).
// With stage4 = false the step stops once y4 is formed (f_new is then
// incomplete): a replay that needs the stage inputs but not the result.
void rk4_step(ephx_table* t, const double* f, double dt, double* f_new, double* y2, double* y3, double* y4,
              hipStream_t st, const Field* fld, bool& gathered, bool stage4 = true) {
    // stage 1 at f: acc = f + dt/6 k1 ; y2 = f + dt/2 k1
    collision_eval(t, f, nullptr, f_new, 1, dt / 6.0, f, dt / 2.0, y2, st, fld, gathered, true);
    collision_eval(t, y2, nullptr, f_new, 0, dt / 3.0, f, dt / 2.0, y3, st, fld, true, true);
    collision_eval(t, y3, nullptr, f_new, 0, dt / 3.0, f, dt, y4, st, fld, true, true);
    if (stage4) collision_eval(t, y4, nullptr, f_new, 0, dt / 6.0, f, 0.0, nullptr, st, fld, true, true, true);
    gathered = stage4;
}

// One explicit Euler step f -> f_new = f + dt (I[f] + drift)
void euler_step(ephx_table* t, const double* f, double dt, double* f_new, hipStream_t st, const Field* fld,
                bool& gathered) {
    collision_eval(t, f, nullptr, f_new, 1, dt, f, 0.0, nullptr, st, fld, gathered, true, true);
    gathered = true;
}

// Neighbours of each state along +/- each reduced direction, same band, on
// the periodic grid; -1 where that state is not in the table.
void ensure_neighbours(ephx_table* t) {
    if (t->d_nbr) return;
    const int S = t->S;
    const long n[3] = {t->n1, t->n2, t->n3};
    auto lin = [&](const long* c) {
        long r = 0;
        for (int d = 0; d < 3; ++d) r = r * n[d] + ((c[d] % n[d]) + n[d]) % n[d];
        return r;
    };
    std::unordered_map<long, int> state;
    for (int s = 0; s < S; ++s) {
        const long c[3] = {t->h_kc[3 * s], t->h_kc[3 * s + 1], t->h_kc[3 * s + 2]};
        state[lin(c) * t->nw + t->h_band[s]] = s;
    }
    std::vector<int32_t> nbr((size_t)S * 6, -1);
    for (int s = 0; s < S; ++s)
        for (int d = 0; d < 3; ++d)
            for (int j = 0; j < 2; ++j) {
                long c[3] = {t->h_kc[3 * s], t->h_kc[3 * s + 1], t->h_kc[3 * s + 2]};
                c[d] += j == 0 ? 1 : -1;
                auto it = state.find(lin(c) * t->nw + t->h_band[s]);
                if (it != state.end()) nbr[(size_t)s * 6 + 2 * d + j] = it->second;
            }
    t->d_nbr = (int32_t*)t->alloc(nbr.size() * 4);
    hip_check(hipMemcpy(t->d_nbr, nbr.data(), nbr.size() * 4, hipMemcpyHostToDevice), "hipMemcpy");
}

void require_ready(ephx_table* t) {
    require(t != nullptr, "null table");
    require(t->ready, "ephx_collision_setup must be called first");
}

}  // namespace

extern "C" int ephx_grid_states(ephx_model* m, const int n_grid[3], int mode, int band_lo, int band_hi, double e_lo,
                                double e_hi, int count, int capacity, int* n_states, int32_t* k_idx, int32_t* band,
                                double* eps, void* stream) {
    return guarded([&] {
        require(m != nullptr && n_states != nullptr, "grid_states: null argument");
        *n_states = 0;
        int n1, n2, n3;
        grid_dims(n_grid, n1, n2, n3);
        require(mode == 0 || mode == 1, "grid_states: mode must be 0 (window) or 1 (lowest)");
        require(0 <= band_lo && band_lo < m->nw, "grid_states: band_lo out of range");
        if (mode == 0) require(band_lo < band_hi && band_hi <= m->nw, "grid_states: bad band range");
        if (mode == 1) require(count >= 1, "grid_states: count must be >= 1");
        require(capacity >= 0 && (capacity == 0 || (k_idx && band && eps)), "grid_states: null output");
        hipStream_t st = (hipStream_t)stream;
        const long ng = (long)n1 * n2 * n3;
        const int nw = m->nw;
        std::vector<double> kp = grid_points(n1, n2, n3);
        double* dk = (double*)m->ws.get("gs.k", ng * 3 * 8);
        double* de = (double*)m->ws.get("gs.e", ng * nw * 8);
        hip_check(hipMemcpyAsync(dk, kp.data(), ng * 3 * 8, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
        bands_impl(m, (int)ng, dk, de, nullptr, nullptr, st, "gs");
        std::vector<double> e(ng * nw);
        hip_check(hipMemcpyAsync(e.data(), de, ng * nw * 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        std::vector<std::pair<long, int>> sel;
        if (mode == 0) {
            std::vector<double> all;
            all.reserve(ng * (band_hi - band_lo));
            for (long k = 0; k < ng; ++k)
                for (int b = band_lo; b < band_hi; ++b) all.push_back(e[k * nw + b]);
            std::sort(all.begin(), all.end());
            const double lo = snap_edge(all, e_lo), hi = snap_edge(all, e_hi);
            for (long k = 0; k < ng; ++k)
                for (int b = band_lo; b < band_hi; ++b) {
                    const double v = e[k * nw + b];
                    if (v > lo && v < hi) sel.push_back({k, b});
                }
        } else {
            std::vector<long> order(ng);
            std::iota(order.begin(), order.end(), 0L);
            std::stable_sort(order.begin(), order.end(), [&](long a, long b) {
                const double ea = e[a * nw + band_lo], eb = e[b * nw + band_lo];
                return ea < eb || (ea == eb && a < b);
            });
            long n = std::min<long>(count, ng);
            while (n < ng && std::fabs(e[order[n] * nw + band_lo] - e[order[n - 1] * nw + band_lo]) <= 1e-9) ++n;
            std::vector<long> ks(order.begin(), order.begin() + n);
            std::sort(ks.begin(), ks.end());
            for (long k : ks) sel.push_back({k, band_lo});
        }
        *n_states = (int)sel.size();
        if ((long)sel.size() > capacity) throw Error{EPHX_EINVAL, "grid_states: more states than capacity"};
        for (size_t i = 0; i < sel.size(); ++i) {
            k_idx[i] = (int32_t)sel[i].first;
            band[i] = sel[i].second;
            eps[i] = e[sel[i].first * nw + sel[i].second];
        }
    });
}

extern "C" int ephx_table_create(ephx_model* m, const int n_grid[3], int n_states, const int32_t* k_idx,
                                 const int32_t* band, int precision, double omega_cut, ephx_table** out,
                                 void* stream) {
    return guarded([&] {
        require(m != nullptr && out != nullptr, "table_create: null argument");
        *out = nullptr;
        if (is_wide(m))
            throw Error{EPHX_EUNSUPPORTED, "table_create: not built for models with nw > 16 or more than 12 modes"};
        if (m->g_c64) throw Error{EPHX_EUNSUPPORTED, "table_create: not built for a counter-drawn (complex float) g"};
        int n1, n2, n3;
        grid_dims(n_grid, n1, n2, n3);
        require(n_states >= 1 && n_states <= 60000, "table_create: need 1 <= n_states <= 60000");
        require(k_idx && band, "table_create: null state arrays");
        require(precision == EPHX_FP64 || precision == EPHX_FP32 || precision == EPHX_BF16X3 ||
                    precision == EPHX_BF16X6 || precision == EPHX_FP16X3,
                "table_create: unknown precision");
        require(std::isfinite(omega_cut), "table_create: omega_cut not finite");
        const long ng = (long)n1 * n2 * n3;
        for (int s = 0; s < n_states; ++s) {
            require(k_idx[s] >= 0 && k_idx[s] < ng, "table_create: k index out of range");
            require(band[s] >= 0 && band[s] < m->nw, "table_create: band out of range");
        }
        hipStream_t st = (hipStream_t)stream;
        const int S = n_states, nw = m->nw, nm = m->nm, nw2 = nw * nw;
        ephx_table* t = new ephx_table();
        try {
            t->m = m;
            t->S = S;
            t->n1 = n1;
            t->n2 = n2;
            t->n3 = n3;
            t->nm = nm;
            t->nw = nw;
            t->f32 = precision != EPHX_FP64;
            t->ld = table_ld(S);
            const size_t esz = t->f32 ? 4 : 8;
            // states: grid coordinates, reduced points, negated points
            std::vector<int32_t> kc(3 * S);
            std::vector<double> ks(3 * S), nks(3 * S);
            for (int s = 0; s < S; ++s) {
                const long i = k_idx[s];
                kc[3 * s] = (int32_t)(i / ((long)n2 * n3));
                kc[3 * s + 1] = (int32_t)((i / n3) % n2);
                kc[3 * s + 2] = (int32_t)(i % n3);
                ks[3 * s] = (double)kc[3 * s] / n1;
                ks[3 * s + 1] = (double)kc[3 * s + 1] / n2;
                ks[3 * s + 2] = (double)kc[3 * s + 2] / n3;
                for (int d = 0; d < 3; ++d) nks[3 * s + d] = -ks[3 * s + d];
            }
            t->d_kc = (int32_t*)t->alloc(3 * S * 4);
            t->d_band = (int32_t*)t->alloc(S * 4);
            hip_check(hipMemcpy(t->d_kc, kc.data(), 3 * S * 4, hipMemcpyHostToDevice), "hipMemcpy");
            hip_check(hipMemcpy(t->d_band, band, S * 4, hipMemcpyHostToDevice), "hipMemcpy");
            t->h_kc = kc;
            t->h_band.assign(band, band + S);
            double* dks = (double*)t->ws.get("t.ks", 3 * S * 8);
            double* dnks = (double*)t->ws.get("t.nks", 3 * S * 8);
            hip_check(hipMemcpy(dks, ks.data(), 3 * S * 8, hipMemcpyHostToDevice), "hipMemcpy");
            hip_check(hipMemcpy(dnks, nks.data(), 3 * S * 8, hipMemcpyHostToDevice), "hipMemcpy");
            // bands at the states
            double* eall = (double*)t->ws.get("t.eall", (size_t)S * nw * 8);
            double* us = (double*)t->ws.get("t.u", (size_t)S * nw2 * 16);
            bands_impl(m, S, dks, eall, us, nullptr, st, "tab");
            {
                std::vector<double> e((size_t)S * nw), es(S);
                hip_check(hipMemcpyAsync(e.data(), eall, (size_t)S * nw * 8, hipMemcpyDeviceToHost, st), "copy");
                hip_check(hipStreamSynchronize(st), "sync");
                for (int s = 0; s < S; ++s) es[s] = e[(size_t)s * nw + band[s]];
                t->d_eps = (double*)t->alloc(S * 8);
                hip_check(hipMemcpy(t->d_eps, es.data(), S * 8, hipMemcpyHostToDevice), "hipMemcpy");
            }
            // phonons on the whole grid (every q = k_t - k_s is a grid point)
            std::vector<double> qp = grid_points(n1, n2, n3);
            double* dq = (double*)t->ws.get("t.q", ng * 3 * 8);
            hip_check(hipMemcpy(dq, qp.data(), ng * 3 * 8, hipMemcpyHostToDevice), "hipMemcpy");
            t->d_omega = (double*)t->alloc(ng * nm * 8);
            double* evec = (double*)t->ws.get("t.evec", (size_t)ng * nm * nm * 16);
            phonons_impl(m, (int)ng, dq, t->d_omega, evec, st, "tab");
            double* lr = nullptr;
            if (m->polar) {
                lr = (double*)t->ws.get("t.lr", (size_t)ng * nm * 16);
                frohlich((int)ng, dq, m->pd, lr, st);
            }
            // the table
            t->d_g2 = t->alloc((size_t)nm * S * t->ld * esz);
            hip_check(hipMemsetAsync(t->d_g2, 0, (size_t)nm * S * t->ld * esz, st), "hipMemsetAsync");
            const long nre_cols = (long)m->n_rp_g * nm * nw2;
            const long ncol = (long)nm * nw;       // Rp-contraction columns per source
            const int kp = ((m->n_rp_g + 31) / 32) * 32;
            const int nsplit = (precision == EPHX_BF16X3 || precision == EPHX_FP16X3) ? 2
                               : (precision == EPHX_BF16X6 ? 3 : 0);
            const int f16s = precision == EPHX_FP16X3 ? 1 : 0;
            const double gsc = f16s ? m->g_scale : 1.0;
            int sc = (int)std::max(1L, std::min<long>(64, (1L << 29) / std::max(1L, (long)S * ncol * 16)));
            sc = std::min(sc, S);
            double* gk = (double*)t->ws.get("t.gk", (size_t)sc * nre_cols * 16);
            double* gcol = (double*)t->ws.get("t.gcol", (size_t)sc * m->n_rp_g * ncol * 16);
            float* gcol32 = t->f32 && !nsplit ? (float*)t->ws.get("t.gcol32", (size_t)sc * m->n_rp_g * ncol * 8) : nullptr;
            uint16_t* gbf = nsplit ? (uint16_t*)t->ws.get("t.gbf", (size_t)sc * 2 * nsplit * ncol * kp * 2) : nullptr;
            void* gwt = t->ws.get("t.gwt", (size_t)sc * S * ncol * (t->f32 ? 8 : 16));
            for (int s0 = 0; s0 < S; s0 += sc) {
                const int nb = std::min(sc, S - s0);
                StageTimer tm("table_pairs", st);
                phase_gemm_f64(nb, (int)nre_cols, m->n_re_g, 1, dks + 3L * s0, nullptr, m->d_re_g, m->d_g, 0, gk, 0,
                               st);
                apply_u_column(nb, m->n_rp_g, nm, nw, gk, us + (size_t)s0 * nw2 * 2, t->d_band + s0, gcol, st);
                const long sB = (long)m->n_rp_g * ncol;
                if (precision == EPHX_FP64) {
                    phase_gemm_f64(S, (int)ncol, m->n_rp_g, nb, dks, dnks + 3L * s0, m->d_rp_g, gcol, sB,
                                   (double*)gwt, (long)S * ncol, st);
                } else if (!nsplit) {
                    convert_f64_f32((long)nb * sB * 2, gcol, gcol32, st);
                    phase_gemm_f32(S, (int)ncol, m->n_rp_g, nb, dks, dnks + 3L * s0, m->d_rp_g, gcol32, sB,
                                   (float*)gwt, (long)S * ncol, st);
                } else {
                    split_bf16_f64(nsplit, f16s, gsc, nb, m->n_rp_g, (int)ncol, kp, gcol, gbf, st);
                    phase_gemm_bf16(nsplit, f16s, S, (int)ncol, m->n_rp_g, kp, nb, dks, dnks + 3L * s0, m->d_rp_g,
                                    gbf, 2L * nsplit * ncol * kp, (float*)gwt, (long)S * ncol, (float)(1.0 / gsc),
                                    st);
                }
                PairEpilogue e{};
                e.ns_chunk = nb;
                e.s_off = s0;
                e.S = S;
                e.nw = nw;
                e.nm = nm;
                e.gw = gwt;
                e.ut = us;
                e.band = t->d_band;
                e.kc = t->d_kc;
                e.n1 = n1;
                e.n2 = n2;
                e.n3 = n3;
                e.omega = t->d_omega;
                e.evec = evec;
                e.lr = lr;
                e.us = us;
                e.minv = m->d_minv;
                e.omega_cut = omega_cut;
                pair_epilogue(e, t->f32 ? 1 : 0, t->ld, t->d_g2, st);
            }
            table_symmetrise(nm, S, t->ld, t->d_g2, t->f32 ? 1 : 0, st);
            t->d_ones = (double*)t->alloc(S * 8);
            fill(S, 1.0, t->d_ones, st);
            t->d_scale = (double*)t->alloc(nm * 8);
            t->d_unit = (double*)t->alloc(nm * 8);
            fill(nm, 1.0, t->d_unit, st);
            t->par.omega_cut = omega_cut;
            t->build_cut = omega_cut;
            hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
            // release the build buffers
            t->ws.release();
        } catch (...) {
            delete t;
            throw;
        }
        *out = t;
    });
}

extern "C" int ephx_table_destroy(ephx_table* t) {
    return guarded([&] {
        if (!t) return;
        (void)hipDeviceSynchronize();
        delete t;
    });
}

extern "C" int ephx_table_g2(ephx_table* t, void* g2, double* eps, void* stream) {
    return guarded([&] {
        require(t != nullptr, "table_g2: null table");
        hipStream_t st = (hipStream_t)stream;
        const size_t esz = t->f32 ? 4 : 8;
        if (g2)
            hip_check(hipMemcpy2DAsync(g2, t->S * esz, t->d_g2, t->ld * esz, t->S * esz, (size_t)t->nm * t->S,
                                       hipMemcpyDeviceToDevice, st),
                      "hipMemcpy2DAsync");
        if (eps) hip_check(hipMemcpyAsync(eps, t->d_eps, t->S * 8, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
    });
}

extern "C" int ephx_collision_setup(ephx_table* t, const ephx_params* p, const double* mode_scale, void* stream) {
    return guarded([&] {
        require(t != nullptr && p != nullptr, "collision_setup: null argument");
        require(p->temp > 0 && p->sigma > 0 && p->n_q > 0 && std::isfinite(p->omega_cut),
                "collision_setup: need temp > 0, sigma > 0, n_q > 0");
        hipStream_t st = (hipStream_t)stream;
        std::vector<double> sc(t->nm, 1.0);
        if (mode_scale)
            for (int i = 0; i < t->nm; ++i) {
                require(std::isfinite(mode_scale[i]), "collision_setup: non-finite mode scale");
                sc[i] = mode_scale[i];
            }
        hip_check(hipMemcpyAsync(t->d_scale, sc.data(), t->nm * 8, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
        const size_t esz = t->f32 ? 4 : 8;
        if (!t->d_p) {
            t->d_p = t->alloc((size_t)t->S * t->ld * esz);
            hip_check(hipMemsetAsync(t->d_p, 0, (size_t)t->S * t->ld * esz, st), "hipMemsetAsync");
        }
        build_banded(t, 0, p, t->d_scale, t->d_p, st);
        t->par = *p;
        t->c = 2.0 * kPi / kHbarEvFs / p->n_q;
        // the tile list of the collision pass, so that ephx_collision_noalloc
        // finds it ready
        (void)plan_for(t, 0, 1, 1, st);
        t->ready = true;
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    });
}

extern "C" int ephx_table_stream_info(ephx_table* t, int matrix, long long* live_entries, int* n_live_tiles,
                                      int* n_tiles, void* stream) {
    return guarded([&] {
        require(t != nullptr && live_entries && n_live_tiles && n_tiles, "stream_info: null argument");
        require(matrix == 0 || matrix == 1, "stream_info: matrix must be 0 (collision) or 1 (transport)");
        require(t->gen[matrix] > 0, "stream_info: that matrix has not been built");
        const StreamPlan pl = matrix == 0 ? plan_for(t, 0, 1, 1, (hipStream_t)stream)
                                          : plan_for(t, 1, 3, 0, (hipStream_t)stream);
        std::vector<int32_t> tiles((size_t)2 * pl.n_tiles);
        if (pl.n_tiles > 0)
            hip_check(hipMemcpy(tiles.data(), pl.tiles, tiles.size() * 4, hipMemcpyDeviceToHost), "hipMemcpy");
        long long n = 0;
        for (int i = 0; i < pl.n_live; ++i) {
            const int ct = tiles[2 * i], rt = tiles[2 * i + 1];
            const long long rows = std::min(t->S, (rt + 1) * pl.rpb) - (long long)rt * pl.rpb;
            const long long c0 = (long long)ct * kStreamTileCols;
            const long long cols = std::min<long long>(t->S, c0 + kStreamTileCols) - c0;
            n += rows * cols;
        }
        *live_entries = n;
        *n_live_tiles = pl.n_live;
        *n_tiles = pl.n_tiles;
    });
}

extern "C" int ephx_collision(ephx_table* t, const double* f, double* i_out, void* stream) {
    return guarded([&] {
        require_ready(t);
        require(f && i_out, "collision: null array");
        collision_eval(t, f, i_out, nullptr, 0, 0.0, nullptr, 0.0, nullptr, (hipStream_t)stream);
    });
}

namespace {

// Work memory of ephx_collision_noalloc: one array per device for the whole
// process (each GPU the library runs on holds its own copy at its own
// address).  Host code must use the address from hipGetSymbolAddress, never
// the array's name, which on the host is only a stand-in for the symbol.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device -> address of its scratch

// Address of the current device's scratch, looked up once per device.
void* scratch_on(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) return it->second;
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) throw Error{EPHX_EHIP, "hipGetSymbolAddress(scratch) returned no address"};
    g_scratch_ptr[dev] = p;
    return p;
}

}  // namespace

// ephx_collision with every work buffer (the occupations gathered into matrix
// order and the row and column partials of the pass) in the static scratch
// array: the call allocates nothing.  The collision plan it needs (the live
// tile list) is built by ephx_collision_setup.
extern "C" int ephx_collision_noalloc(ephx_table* t, const double* f, double* i_out, void* stream) {
    return guarded([&] {
        require_ready(t);
        require(f && i_out, "collision_noalloc: null array");
        int dev = -1;
        hip_check(hipGetDevice(&dev), "hipGetDevice");
        require(dev == t->m->device, "collision_noalloc: the table lives on device " + std::to_string(t->m->device) +
                                         ", the current device is " + std::to_string(dev));
        auto it = t->plans.find(0 * 64 + 1 * 8 + 1);
        require(it != t->plans.end() && it->second.gen == t->gen[0],
                "collision_noalloc: no collision plan for the current setup (call ephx_collision_setup)");
        StreamPlan pl = it->second.pl;
        const int S = t->S;
        // gathered 1 - f and f [2][S], row partials [n_ct][S], column partials [n_rt][S]
        const size_t vec = (size_t)S * 8;
        const size_t need = (2 + (size_t)pl.n_ct + (size_t)pl.n_rt) * vec;
        if (need > kNoAllocScratchBytes)
            throw Error{EPHX_EINVAL, "collision_noalloc: this table needs " + std::to_string(need) +
                                         " bytes of work memory, more than the " +
                                         std::to_string(kNoAllocScratchBytes) + " the library holds"};
        if (S == 0) return;
        char* base = (char*)scratch_on(dev);
        hipStream_t st = (hipStream_t)stream;
        pl.gbuf = (double*)base;
        pl.rout = nullptr;
        pl.cout = nullptr;
        double* rowp = (double*)(base + 2 * vec);
        double* colp = rowp + (size_t)pl.n_ct * S;
        // every entry of the buffers is written before it is read (dead tiles
        // write zero partials), so nothing is cleared
        gather_occupations(pl, f, st);
        stream_run(pl, t->ld, t->d_p, rowp, colp, st);
        CollisionFinish cf{};
        cf.S = S;
        cf.n_rt = pl.n_rt;
        cf.n_ct = pl.n_ct;
        cf.rowp = rowp;
        cf.colp = colp;
        cf.f = f;
        cf.c = t->c;
        cf.i_out = i_out;
        reduce_finish(pl, cf, st);
    });
}

extern "C" int ephx_dynamics(ephx_table* t, const double* f0, double dt, int n_steps, int ckpt_every, double* f_out,
                             double* ckpts, void* stream) {
    return ephx_dynamics_field(t, f0, dt, n_steps, EPHX_RK4, nullptr, ckpt_every, f_out, ckpts, stream);
}

extern "C" int ephx_dynamics_field(ephx_table* t, const double* f0, double dt, int n_steps, int method,
                                   const double* efield, int ckpt_every, double* f_out, double* ckpts, void* stream) {
    return guarded([&] {
        require_ready(t);
        require(f0 && f_out, "dynamics: null array");
        require(n_steps >= 0 && std::isfinite(dt), "dynamics: bad step count or dt");
        require(!ckpts || ckpt_every >= 1, "dynamics: ckpt_every must be >= 1 with checkpoints");
        require(method == EPHX_RK4 || method == EPHX_EULER, "dynamics: method must be EPHX_RK4 or EPHX_EULER");
        hipStream_t st = (hipStream_t)stream;
        const int S = t->S;
        Field fld;
        const bool field = efield && (efield[0] != 0.0 || efield[1] != 0.0 || efield[2] != 0.0);
        if (field) {
            require(std::isfinite(efield[0]) && std::isfinite(efield[1]) && std::isfinite(efield[2]),
                    "dynamics: non-finite field");
            ensure_neighbours(t);
            fld.nbr = t->d_nbr;
            const int nd[3] = {t->n1, t->n2, t->n3};
            for (int d = 0; d < 3; ++d) {
                const double* a = t->m->lattice + 3 * d;
                const double ea = efield[0] * a[0] + efield[1] * a[1] + efield[2] * a[2];
                fld.dc[d] = ea / (2.0 * kPi * kHbarEvFs) * (0.5 * nd[d]);
            }
        }
        const Field* fp = field ? &fld : nullptr;
        double* fa = (double*)t->ws.get("d.fa", S * 8);
        double* fb = (double*)t->ws.get("d.fb", S * 8);
        double* y2 = (double*)t->ws.get("d.y2", S * 8);
        double* y3 = (double*)t->ws.get("d.y3", S * 8);
        double* y4 = (double*)t->ws.get("d.y4", S * 8);
        hip_check(hipMemcpyAsync(fa, f0, S * 8, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
        if (ckpts) hip_check(hipMemcpyAsync(ckpts, f0, S * 8, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
        bool gathered = false;
        for (int n = 0; n < n_steps; ++n) {
            if (method == EPHX_RK4) rk4_step(t, fa, dt, fb, y2, y3, y4, st, fp, gathered);
            else euler_step(t, fa, dt, fb, st, fp, gathered);
            std::swap(fa, fb);
            if (ckpts && (n + 1) % ckpt_every == 0)
                hip_check(hipMemcpyAsync(ckpts + (size_t)((n + 1) / ckpt_every) * S, fa, S * 8,
                                         hipMemcpyDeviceToDevice, st),
                          "hipMemcpyAsync");
        }
        hip_check(hipMemcpyAsync(f_out, fa, S * 8, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
    });
}

extern "C" int ephx_collision_vjp(ephx_table* t, const double* f, const double* lam, double* f_bar, double* s_bar,
                                  void* stream) {
    return guarded([&] {
        require_ready(t);
        require(f && lam && f_bar, "collision_vjp: null array");
        collision_vjp_impl(t, f, lam, f_bar, s_bar, 0, (hipStream_t)stream);
    });
}

extern "C" int ephx_dynamics_vjp(ephx_table* t, const double* ckpts, double dt, int n_steps, int ckpt_every,
                                 const double* f_bar_final, double* f0_bar, double* s_bar, void* stream) {
    return guarded([&] {
        require_ready(t);
        require(ckpts && f_bar_final && f0_bar, "dynamics_vjp: null array");
        require(n_steps >= 0 && ckpt_every >= 1 && n_steps % ckpt_every == 0,
                "dynamics_vjp: n_steps must be a multiple of ckpt_every >= 1");
        hipStream_t st = (hipStream_t)stream;
        const int S = t->S;
        const int L = ckpt_every;
        double* a = (double*)t->ws.get("b.a", S * 8);
        double* yb[4];
        for (int i = 0; i < 4; ++i) yb[i] = (double*)t->ws.get("b.yb" + std::to_string(i), S * 8);
        double* ys = (double*)t->ws.get("b.ys", (size_t)L * 4 * S * 8);   // stage inputs of the segment
        // the stage adjoints k_i_bar of the segment, [step][stage][S] like ys,
        // kept for the segment's mode-scale gradient
        double* kbp = (double*)t->ws.get("b.kbp", (size_t)L * 4 * S * 8);
        double* fn = (double*)t->ws.get("b.fn", S * 8);
        hip_check(hipMemcpyAsync(a, f_bar_final, S * 8, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
        const int32_t* ptiles = nullptr;
        int n_ptiles = 0;
        double *pwork = nullptr, *ppart = nullptr;
        if (s_bar) {
            hip_check(hipMemsetAsync(s_bar, 0, t->nm * 8, st), "hipMemsetAsync");
            ensure_pmode(t, st);
            panel_tiles(t, st, ptiles, n_ptiles);
            pwork = (double*)t->ws.get("b.pwork", (size_t)4 * 4 * L * S * 8);
            ppart = (double*)t->ws.get("b.ppart", (size_t)std::max(1, n_ptiles) * t->nm * 8);
        }
        const StreamPlan pl2 = plan_for(t, 0, 2, 2, st);
        double* rowp2 = (double*)t->ws.get("b.rowp", (size_t)2 * pl2.n_ct * S * 8);
        double* colp2 = (double*)t->ws.get("b.colp", (size_t)2 * pl2.n_rt * S * 8);
        const int nseg = n_steps / L;
        for (int seg = nseg - 1; seg >= 0; --seg) {
            // replay the segment, keeping the four stage inputs of each step:
            // step j starts from its slot (j, 0) and writes its result into
            // slot (j + 1, 0); the last step's result (the next checkpoint)
            // is not needed, and neither is its fourth stage
            hip_check(hipMemcpyAsync(ys, ckpts + (size_t)seg * S, S * 8, hipMemcpyDeviceToDevice, st),
                      "hipMemcpyAsync");
            bool gathered = false;
            for (int j = 0; j < L; ++j) {
                double* y1 = ys + ((size_t)j * 4) * S;
                const bool last = j + 1 == L;
                rk4_step(t, y1, dt, last ? fn : y1 + 4 * S, y1 + S, y1 + 2 * S, y1 + 3 * S, st, nullptr, gathered,
                         !last);
            }
            for (int j = L - 1; j >= 0; --j) {
                const double* Y[4];
                double* kbs[4];
                for (int i = 0; i < 4; ++i) {
                    Y[i] = ys + ((size_t)j * 4 + i) * S;
                    kbs[i] = kbp + ((size_t)j * 4 + i) * S;
                }
                // k4b = dt/6 a ; Y4b = J4^T k4b
                adjoint_stage(pl2, t->ld, t->d_p, Y[3], Lincomb{1, 0.0, {dt / 6.0}, {a}}, kbs[3], t->c, rowp2,
                              colp2, yb[3], nullptr, nullptr, nullptr, nullptr, st);
                // k3b = dt/3 a + dt Y4b
                adjoint_stage(pl2, t->ld, t->d_p, Y[2], Lincomb{2, 0.0, {dt / 3.0, dt}, {a, yb[3]}}, kbs[2], t->c,
                              rowp2, colp2, yb[2], nullptr, nullptr, nullptr, nullptr, st);
                // k2b = dt/3 a + dt/2 Y3b
                adjoint_stage(pl2, t->ld, t->d_p, Y[1], Lincomb{2, 0.0, {dt / 3.0, dt / 2.0}, {a, yb[2]}}, kbs[1],
                              t->c, rowp2, colp2, yb[1], nullptr, nullptr, nullptr, nullptr, st);
                // k1b = dt/6 a + dt/2 Y2b; then a <- a + Y1b + Y2b + Y3b + Y4b
                adjoint_stage(pl2, t->ld, t->d_p, Y[0], Lincomb{2, 0.0, {dt / 6.0, dt / 2.0}, {a, yb[1]}}, kbs[0],
                              t->c, rowp2, colp2, yb[0], a, yb[1], yb[2], yb[3], st);
            }
            // s_bar += sum over the segment's 4L stages of k_i_bar^T dI/ds at Y_i:
            // one pass over each per-mode matrix for the whole segment
            if (s_bar) {
                StageTimer tm("mode_panel", st);
                mode_panel(S, t->ld, 4 * L, t->nm, t->f32 ? 1 : 0, t->d_pmode, (long)S * t->ld,
                           t->d_perm, ys, kbp, pwork, ptiles, n_ptiles, ppart, t->c, s_bar, 1, st);
            }
        }
        hip_check(hipMemcpyAsync(f0_bar, a, S * 8, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
    });
}

extern "C" int ephx_mobility(ephx_table* t, const ephx_params* p, const double* vel, int n_iter_max, double tol,
                             double* f_out, double* tau_out, double* mob_out, int* n_iter, double* last_change,
                             void* stream) {
    return guarded([&] {
        require(t != nullptr && p != nullptr, "mobility: null argument");
        require(vel != nullptr, "mobility: null velocities");
        require(n_iter_max >= 0, "mobility: n_iter_max < 0");
        require(std::isfinite(tol), "mobility: tol is not finite");
        require(p->temp > 0 && p->sigma > 0 && p->n_q > 0 && std::isfinite(p->mu), "mobility: bad parameters");
        hipStream_t st = (hipStream_t)stream;
        const int S = t->S;
        const size_t esz = t->f32 ? 4 : 8;
        if (!t->d_w) {
            t->d_w = t->alloc((size_t)S * t->ld * esz);
            hip_check(hipMemsetAsync(t->d_w, 0, (size_t)S * t->ld * esz, st), "hipMemsetAsync");
        }
        build_banded(t, 1, p, t->d_unit, t->d_w, st);
        double* tau = (double*)t->ws.get("m.tau", S * 8);
        double* f0 = (double*)t->ws.get("m.f0", 3 * S * 8);
        double* f = (double*)t->ws.get("m.f", 3 * S * 8);
        double* fn = (double*)t->ws.get("m.fn", 3 * S * 8);
        const StreamPlan pl1 = plan_for(t, 1, 1, 0, st), pl3 = plan_for(t, 1, 3, 0, st);
        double* rowp = (double*)t->ws.get("m.rowp", (size_t)3 * pl3.n_ct * S * 8);
        VecPtrs one{{t->d_ones, nullptr, nullptr, nullptr}}, none{{nullptr, nullptr, nullptr, nullptr}};
        PassOut po = one_pass(t, pl1, t->d_w, one, none, rowp, nullptr, st, "transport_stream");
        ita_gamma(S, po.n_ct, po.rowp, p->n_q, vel, tau, f0, f, st);
        // with tol > 0: stop after the first iteration whose largest change of any
        // component is below tol times the largest component (one 16-byte read
        // back per iteration); with tol <= 0: exactly n_iter_max iterations
        unsigned long long* chg = tol > 0 ? (unsigned long long*)t->ws.get("m.chg", 2 * 8) : nullptr;
        int done = 0;
        double change = -1.0;
        for (int it = 0; it < n_iter_max; ++it) {
            VecPtrs x{{f, f + S, f + 2 * S, nullptr}};
            po = one_pass(t, pl3, t->d_w, x, none, rowp, nullptr, st, "transport_stream");
            if (chg) hip_check(hipMemsetAsync(chg, 0, 2 * 8, st), "hipMemsetAsync");
            ita_update(S, po.n_ct, po.rowp, p->n_q, tau, f0, fn, st, f, chg);
            std::swap(f, fn);
            done = it + 1;
            if (chg) {
                unsigned long long h[2] = {0, 0};
                hip_check(hipMemcpyAsync(h, chg, sizeof(h), hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
                hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
                double dmax, amax;
                std::memcpy(&dmax, &h[0], 8);
                std::memcpy(&amax, &h[1], 8);
                if (!std::isfinite(dmax) || !std::isfinite(amax)) throw Error{EPHX_ENAN, "mobility: non-finite iterate"};
                change = amax > 0 ? dmax / amax : 0.0;
                if (change < tol) break;
            }
        }
        if (n_iter) *n_iter = done;
        if (last_change) *last_change = change;
        mobility_reduce(S, t->d_eps, vel, f, p->mu, p->temp, f_out, mob_out, st);
        if (tau_out) hip_check(hipMemcpyAsync(tau_out, tau, S * 8, hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
    });
}

// dL/dg(Re,Rp) for L = sum_ab lam_ab mu_ab, mu from ephx_mobility with the same
// arguments.  The iteration is rerun keeping F^0..F^n, reversed with one
// column pass over W per step, and the resulting W_bar (never stored) is taken
// back through the transport weights, the symmetrisation, the table epilogue,
// the Rp sum over the targets of each source, U(k_s) and the Re sum, per
// chunk of source states, all in FP64.
extern "C" int ephx_mobility_vjp(ephx_table* t, const ephx_params* p, const double* vel, int n_iter,
                                 const double* mob_bar, double* g_bar, void* stream) {
    return guarded([&] {
        require(t != nullptr && p != nullptr, "mobility_vjp: null argument");
        require(vel != nullptr && mob_bar != nullptr && g_bar != nullptr, "mobility_vjp: null array");
        require(n_iter >= 0, "mobility_vjp: n_iter < 0");
        require(p->temp > 0 && p->sigma > 0 && p->n_q > 0 && std::isfinite(p->mu), "mobility_vjp: bad parameters");
        ephx_model* m = t->m;
        hipStream_t st = (hipStream_t)stream;
        const int S = t->S, nm = t->nm, nw = t->nw, nw2 = nw * nw;
        const size_t esz = t->f32 ? 4 : 8;
        // forward iteration with its history
        if (!t->d_w) {
            t->d_w = t->alloc((size_t)S * t->ld * esz);
            hip_check(hipMemsetAsync(t->d_w, 0, (size_t)S * t->ld * esz, st), "hipMemsetAsync");
        }
        build_banded(t, 1, p, t->d_unit, t->d_w, st);
        const long s3 = 3L * S;
        double* tau = (double*)t->ws.get("mv.tau", S * 8);
        double* fh = (double*)t->ws.get("mv.fh", (size_t)(n_iter + 1) * s3 * 8);
        double* fscr = (double*)t->ws.get("mv.f", s3 * 8);
        const StreamPlan pl1 = plan_for(t, 1, 1, 0, st), pl3 = plan_for(t, 1, 3, 0, st),
                         plc = plan_for(t, 1, 0, 3, st);
        double* rowp = (double*)t->ws.get("mv.rowp", (size_t)3 * pl3.n_ct * S * 8);
        double* colp = (double*)t->ws.get("mv.colp", (size_t)3 * plc.n_rt * S * 8);
        VecPtrs one{{t->d_ones, nullptr, nullptr, nullptr}}, none{{nullptr, nullptr, nullptr, nullptr}};
        PassOut po = one_pass(t, pl1, t->d_w, one, none, rowp, nullptr, st, "transport_stream");
        ita_gamma(S, po.n_ct, po.rowp, p->n_q, vel, tau, fh, fscr, st);
        for (int it = 0; it < n_iter; ++it) {
            const double* fi = fh + it * s3;
            VecPtrs x{{fi, fi + S, fi + 2 * S, nullptr}};
            po = one_pass(t, pl3, t->d_w, x, none, rowp, nullptr, st, "transport_stream");
            ita_update(S, po.n_ct, po.rowp, p->n_q, tau, fh, fh + (it + 1) * s3, st);
        }
        // reverse
        double* fbar = (double*)t->ws.get("mv.fbar", s3 * 8);
        double* taubar = (double*)t->ws.get("mv.taubar", S * 8);
        double* ubar = (double*)t->ws.get("mv.ubar", (size_t)std::max(1, n_iter) * s3 * 8);
        double* gambar = (double*)t->ws.get("mv.gambar", S * 8);
        mob_seed(S, t->d_eps, vel, mob_bar, p->mu, p->temp, fbar, st);
        for (int it = n_iter - 1; it >= 0; --it) {
            double* ui = ubar + it * s3;
            ita_adj_step(S, tau, fbar, fh + (it + 1) * s3, taubar, ui, it == n_iter - 1 ? 1 : 0, st);
            VecPtrs y{{ui, ui + S, ui + 2 * S, nullptr}};
            const PassOut pc = one_pass(t, plc, t->d_w, none, y, nullptr, colp, st, "transport_stream");
            ita_adj_cols(S, pc.n_rt, pc.colp, p->n_q, fbar, st);
        }
        ita_adj_final(S, tau, fbar, vel, taubar, n_iter == 0 ? 1 : 0, gambar, st);

        // states, their U(k), phonon eigenvectors on the grid, long-range term
        std::vector<int32_t> kc(3 * S);
        hip_check(hipMemcpyAsync(kc.data(), t->d_kc, 3 * S * 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        std::vector<double> ks(3 * S), nks(3 * S);
        const int nn[3] = {t->n1, t->n2, t->n3};
        for (int i = 0; i < 3 * S; ++i) {
            ks[i] = (double)kc[i] / nn[i % 3];
            nks[i] = -ks[i];
        }
        double* dks = (double*)t->ws.get("mv.ks", 3 * S * 8);
        double* dnks = (double*)t->ws.get("mv.nks", 3 * S * 8);
        hip_check(hipMemcpyAsync(dks, ks.data(), 3 * S * 8, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
        hip_check(hipMemcpyAsync(dnks, nks.data(), 3 * S * 8, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
        double* eall = (double*)t->ws.get("mv.eall", (size_t)S * nw * 8);
        double* us = (double*)t->ws.get("mv.u", (size_t)S * nw2 * 16);
        bands_impl(m, S, dks, eall, us, nullptr, st, "mv");
        const long ng = (long)t->n1 * t->n2 * t->n3;
        std::vector<double> qp = grid_points(t->n1, t->n2, t->n3);
        double* dq = (double*)t->ws.get("mv.q", ng * 3 * 8);
        hip_check(hipMemcpyAsync(dq, qp.data(), ng * 3 * 8, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
        double* omg = (double*)t->ws.get("mv.om", ng * nm * 8);
        double* evec = (double*)t->ws.get("mv.evec", (size_t)ng * nm * nm * 16);
        phonons_impl(m, (int)ng, dq, omg, evec, st, "mv");
        double* lr = nullptr;
        if (m->polar) {
            lr = (double*)t->ws.get("mv.lr", (size_t)ng * nm * 16);
            frohlich((int)ng, dq, m->pd, lr, st);
        }
        negated_vectors(m);
        const long ncol = (long)nm * nw;
        const long nre_cols = (long)m->n_rp_g * nm * nw2;
        hip_check(hipMemsetAsync(g_bar, 0, (size_t)m->n_re_g * nre_cols * 16, st), "hipMemsetAsync");
        int sc = (int)std::max(1L, std::min<long>(64, (1L << 28) / std::max(1L, (long)S * ncol * 16)));
        sc = std::min(sc, S);
        double* gk = (double*)t->ws.get("mv.gk", (size_t)sc * nre_cols * 16);
        double* gcol = (double*)t->ws.get("mv.gcol", (size_t)sc * m->n_rp_g * ncol * 16);
        double* gwt = (double*)t->ws.get("mv.gw", (size_t)sc * S * ncol * 16);
        double* gwb = (double*)t->ws.get("mv.gwb", (size_t)sc * S * ncol * 16);
        const long sB = (long)m->n_rp_g * ncol;
        for (int s0 = 0; s0 < S; s0 += sc) {
            const int nb = std::min(sc, S - s0);
            StageTimer tm("mobility_adjoint_pairs", st);
            phase_gemm_f64(nb, (int)nre_cols, m->n_re_g, 1, dks + 3L * s0, nullptr, m->d_re_g, m->d_g, 0, gk, 0, st);
            apply_u_column(nb, m->n_rp_g, nm, nw, gk, us + (size_t)s0 * nw2 * 2, t->d_band + s0, gcol, st);
            phase_gemm_f64(S, (int)ncol, m->n_rp_g, nb, dks, dnks + 3L * s0, m->d_rp_g, gcol, sB, gwt, (long)S * ncol,
                           st);
            PairAdjoint pa{};
            pa.ns_chunk = nb;
            pa.s_off = s0;
            pa.S = S;
            pa.nw = nw;
            pa.nm = nm;
            pa.gw = gwt;
            pa.ut = us;
            pa.us = us;
            pa.band = t->d_band;
            pa.kc = t->d_kc;
            pa.n1 = t->n1;
            pa.n2 = t->n2;
            pa.n3 = t->n3;
            pa.omega = omg;
            pa.evec = evec;
            pa.lr = lr;
            pa.minv = m->d_minv;
            pa.omega_cut_table = t->build_cut;
            pa.n_hist = 3 * n_iter;
            pa.ubar = ubar;
            pa.fhist = fh;
            pa.gamma_bar = gambar;
            pa.n_q = p->n_q;
            pa.eps = t->d_eps;
            pa.temp = p->temp;
            pa.mu = p->mu;
            pa.sigma = p->sigma;
            pa.omega_cut = p->omega_cut;
            pa.gw_bar = gwb;
            pair_adjoint(pa, st);
            // g'(k_s,Rp)_bar = sum_t exp(-2 pi i (k_t - k_s).Rp) g'W_bar(s,t): the sum over
            // exp(-2 pi i k_t.Rp) here, the exp(2 pi i k_s.Rp) factor with U(k_s)^dag
            phase_gemm_adj_f64(m->n_rp_g, (int)ncol, S, nb, m->d_nrp_g, dks, gwb, (long)S * ncol, gcol, sB, 0, st);
            apply_u_column_adj(nb, m->n_rp_g, nm, nw, s0, gcol, dks, m->d_rp_g, us, t->d_band, gk, st);
            // g(Re,Rp)_bar += sum_s exp(-2 pi i k_s.Re) g(k_s,Rp)_bar
            phase_gemm_adj_f64(m->n_re_g, (int)nre_cols, nb, 1, m->d_nre_g, dks + 3L * s0, gk, 0, g_bar, 0, 1, st);
        }
        if (m->d_wg) scale_rows((long)m->n_re_g * m->n_rp_g, nm * nw2, m->d_wg, g_bar, st);
        // keep the workspace alive until the stream has used it
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    });
}

namespace ephx {
namespace {

// Tetrahedra of the window states: every grid cube is cut into 6 tetrahedra
// along its (0,0,0)-(1,1,1) diagonal; one enters per band whose four corners
// are all states.  Ordered by (cube origin index, path, band).
void ensure_tetrahedra(ephx_table* t) {
    if (t->n_tet >= 0) return;
    const int S = t->S;
    const long n1 = t->n1, n2 = t->n2, n3 = t->n3;
    auto lin = [&](long a, long b, long c) { return ((a % n1 + n1) % n1 * n2 + (b % n2 + n2) % n2) * n3 + (c % n3 + n3) % n3; };
    std::unordered_map<long, int> state;
    std::vector<int> bands;
    for (int s = 0; s < S; ++s) {
        const long k = lin(t->h_kc[3 * s], t->h_kc[3 * s + 1], t->h_kc[3 * s + 2]);
        state[k * t->nw + t->h_band[s]] = s;
        bands.push_back(t->h_band[s]);
    }
    std::sort(bands.begin(), bands.end());
    bands.erase(std::unique(bands.begin(), bands.end()), bands.end());
    std::vector<long> origins;
    for (int s = 0; s < S; ++s)
        for (int d = 0; d < 8; ++d)
            origins.push_back(lin(t->h_kc[3 * s] - (d & 1), t->h_kc[3 * s + 1] - ((d >> 1) & 1), t->h_kc[3 * s + 2] - ((d >> 2) & 1)));
    std::sort(origins.begin(), origins.end());
    origins.erase(std::unique(origins.begin(), origins.end()), origins.end());
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    std::vector<int32_t> tets;
    for (long o : origins) {
        const long c0[3] = {o / (n2 * n3), (o / n3) % n2, o % n3};
        for (int pth = 0; pth < 6; ++pth) {
            long cr[4][3];
            for (int d = 0; d < 3; ++d) {
                cr[0][d] = c0[d];
                cr[1][d] = c0[d] + (perm[pth][0] == d ? 1 : 0);
                cr[2][d] = cr[1][d] + (perm[pth][1] == d ? 1 : 0);
                cr[3][d] = c0[d] + 1;
            }
            long kc4[4];
            for (int j = 0; j < 4; ++j) kc4[j] = lin(cr[j][0], cr[j][1], cr[j][2]);
            for (int b : bands) {
                int st4[4];
                bool all = true;
                for (int j = 0; j < 4 && all; ++j) {
                    auto it = state.find(kc4[j] * t->nw + b);
                    if (it == state.end()) all = false;
                    else st4[j] = it->second;
                }
                if (all) tets.insert(tets.end(), st4, st4 + 4);
            }
        }
    }
    t->n_tet = (int)(tets.size() / 4);
    if (t->n_tet > 0) {
        t->d_tet = (int32_t*)t->alloc(tets.size() * 4);
        hip_check(hipMemcpy(t->d_tet, tets.data(), tets.size() * 4, hipMemcpyHostToDevice), "hipMemcpy");
    }
}

constexpr double kSigmaUnit = 1.602176634e6;   // e^2/(fs Angstrom eV) in S/m
constexpr double kSpin = 2.0;                  // spin degeneracy of Eq. cond_tdf2

}  // namespace
}  // namespace ephx

extern "C" int ephx_tdf(ephx_table* t, const ephx_params* p, const double* vel, const double* f_ita, int n_e,
                        const double* e_grid, double* tdf, double* sigma, double* seebeck, void* stream) {
    return guarded([&] {
        require(t != nullptr && p != nullptr, "tdf: null argument");
        require(vel != nullptr && f_ita != nullptr && e_grid != nullptr, "tdf: null array");
        require(n_e >= 2 && n_e <= 65535, "tdf: need 2 <= n_e <= 65535");
        require(p->temp > 0 && std::isfinite(p->mu), "tdf: bad parameters");
        hipStream_t st = (hipStream_t)stream;
        ensure_tetrahedra(t);
        const int S = t->S;
        double* x = (double*)t->ws.get("td.x", (size_t)9 * S * 8);
        double* part = (double*)t->ws.get("td.part", (size_t)std::max(1, tetra_chunks(t->n_tet)) * n_e * 9 * 8);
        double* out = tdf ? tdf : (double*)t->ws.get("td.out", (size_t)n_e * 9 * 8);
        vf_products(S, vel, f_ita, x, st);
        const double nk = (double)t->n1 * t->n2 * t->n3;
        StageTimer tm("tdf_tetra", st);
        tetra_sum(t->n_tet, t->d_tet, t->d_eps, 9, x, n_e, e_grid, kSpin / (nk * t->m->volume), part, out, st);
        tm.stop();
        if (sigma && seebeck) {
            tdf_transport(n_e, e_grid, out, p->mu, p->temp, kSigmaUnit, sigma, seebeck, st);
        } else if (sigma || seebeck) {
            double* tmp = (double*)t->ws.get("td.tmp", 18 * 8);
            tdf_transport(n_e, e_grid, out, p->mu, p->temp, kSigmaUnit, sigma ? sigma : tmp, seebeck ? seebeck : tmp + 9,
                          st);
        }
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    });
}

extern "C" int ephx_population(ephx_table* t, const double* f, int n_e, const double* e_grid, double* pop,
                               void* stream) {
    return guarded([&] {
        require(t != nullptr && f != nullptr && e_grid != nullptr && pop != nullptr, "population: null argument");
        require(n_e >= 1 && n_e <= 65535, "population: need 1 <= n_e <= 65535");
        hipStream_t st = (hipStream_t)stream;
        ensure_tetrahedra(t);
        double* part = (double*)t->ws.get("pp.part", (size_t)std::max(1, tetra_chunks(t->n_tet)) * n_e * 8);
        StageTimer tm("population_tetra", st);
        tetra_sum(t->n_tet, t->d_tet, t->d_eps, 1, f, n_e, e_grid, 1.0, part, pop, st);
        tm.stop();
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    });
}
