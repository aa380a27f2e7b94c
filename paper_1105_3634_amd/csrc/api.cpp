// C ABI of the mlb library (declared in include/mlb.h).
//
// A mixture is a batch of one system in the batched kernel layout: the
// system descriptor, the block->system map, the stencil tables and all
// fields live in the caller's workspace; this file validates parameters,
// builds the tables on the host, lays out the workspace and sequences the
// passes of each step on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mlb.h"
#include "mlb_internal.h"
#include "spectral.h"

namespace {

thread_local std::string g_err;

mlb_status fail(mlb_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

#define HIP_TRY(call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(MLB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kSeriesCap = 8192;
constexpr int kRedParts = 512;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Host view of the tables of one system.
struct HostTables {
    std::vector<int32_t> sh_e, tl_e, bl_e;
    std::vector<double> sh_u, tl_w;
    int sh_start[mlb::kMaxS][mlb::kMaxS] = {}, sh_cnt[mlb::kMaxS][mlb::kMaxS] = {};
    int sh_full[mlb::kMaxS][mlb::kMaxS] = {};
    int tl_start[mlb::kMaxS][mlb::kMaxS] = {}, tl_cnt[mlb::kMaxS][mlb::kMaxS] = {};
    int bl_start[mlb::kMaxS] = {}, bl_cnt[mlb::kMaxS] = {}, bl_full[mlb::kMaxS] = {};
    int reach[3] = {0, 0, 0};
};

bool validate(const mlb_params *p, std::string &why)
{
    if (!p) { why = "params is NULL"; return false; }
    const int M = p->nspecies;
    if (M < 1 || M > MLB_MAX_SPECIES) { why = "nspecies must be 1..4"; return false; }
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) { why = "lattice sizes must be positive"; return false; }
    if (p->precision != 32 && p->precision != 64) { why = "precision must be 32 or 64"; return false; }
    if (p->scheme != MLB_SCHEME_CN_J1 && p->scheme != MLB_SCHEME_FE) { why = "unknown scheme"; return false; }
    if (p->tail_mode < MLB_TAIL_AUTO || p->tail_mode > MLB_TAIL_SPECTRAL) { why = "unknown tail mode"; return false; }
    if (!(p->tau > 0.5)) { why = "tau must exceed 1/2"; return false; }
    if (std::fabs(p->kT - 1.0 / 3.0) > 1e-12) { why = "kT must be 1/3 (unit masses on D3Q19)"; return false; }
    if (p->walls_y && p->ny < 3) { why = "walls need ny >= 3"; return false; }
    for (int a = 0; a < M; ++a) {
        if (p->mass[a] != 1.0) { why = "only unit masses are supported"; return false; }
        if (!(p->sigma[a] > 0.0) || p->sigma[a] > 40.0) { why = "sigma must be in (0, 40]"; return false; }
        for (int b = 0; b < M; ++b) {
            const double e = p->eps[a * MLB_MAX_SPECIES + b];
            if (!(e >= 0.0) || e != p->eps[b * MLB_MAX_SPECIES + a]) { why = "eps must be symmetric and >= 0"; return false; }
            if (e > 0.0 && !(p->rc_factor > 1.0)) { why = "rc_factor must exceed 1 when a tail is on"; return false; }
        }
    }
    return true;
}

bool build_tables(const mlb_params *p, HostTables &t, std::string &why)
{
    const int M = p->nspecies;
    auto reach = [&](const mlb::HostStencil &s) {
        for (int d = 0; d < 3; ++d) t.reach[d] = std::max(t.reach[d], s.max_abs[d]);
    };
    for (int c = 0; c < M; ++c) {
        mlb::HostStencil b = mlb::build_stencil(mlb::kBall, p->sigma[c], 0.0);
        t.bl_start[c] = (int)t.bl_e.size();
        t.bl_cnt[c] = (int)b.e.size();
        t.bl_full[c] = b.full;
        t.bl_e.insert(t.bl_e.end(), b.e.begin(), b.e.end());
        reach(b);
    }
    for (int a = 0; a < M; ++a)
        for (int b = 0; b < M; ++b) {
            const double sab = 0.5 * (p->sigma[a] + p->sigma[b]);
            mlb::HostStencil sh = mlb::build_stencil(mlb::kShell, sab, 0.0);
            if (sh.e.empty()) { why = "empty lattice shell (sigma too small)"; return false; }
            t.sh_start[a][b] = (int)t.sh_e.size();
            t.sh_cnt[a][b] = (int)sh.e.size();
            t.sh_full[a][b] = sh.full;
            t.sh_e.insert(t.sh_e.end(), sh.e.begin(), sh.e.end());
            t.sh_u.insert(t.sh_u.end(), sh.v.begin(), sh.v.end());
            reach(sh);
            const double eps = p->eps[a * MLB_MAX_SPECIES + b];
            if (eps > 0.0) {
                mlb::HostStencil tl = mlb::build_stencil(mlb::kTail, sab, p->rc_factor);
                t.tl_start[a][b] = (int)t.tl_e.size();
                t.tl_cnt[a][b] = (int)tl.e.size();
                const double s6 = ((sab * sab) * (sab * sab)) * (sab * sab);
                for (size_t k = 0; k < tl.e.size(); ++k) {
                    int ex, ey, ez;
                    mlb::unpack_offset(tl.e[k], ex, ey, ez);
                    const double r2 = (double)(ex * ex + ey * ey + ez * ez);
                    const double len = std::sqrt(r2);
                    const double r7 = ((r2 * r2) * r2) * len;
                    // -dU/dr of U = -eps (sigma/r)^6: 6 eps sigma^6 / r^7
                    const double coef = ((6.0 * eps) * s6) / r7;
                    t.tl_w.push_back(coef * tl.v[3 * k + 0]);
                    t.tl_w.push_back(coef * tl.v[3 * k + 1]);
                    t.tl_w.push_back(coef * tl.v[3 * k + 2]);
                }
                t.tl_e.insert(t.tl_e.end(), tl.e.begin(), tl.e.end());
                reach(tl);
            }
        }
    if (t.reach[0] >= p->nx || t.reach[2] >= p->nz || (!p->walls_y && t.reach[1] >= p->ny)) {
        why = "a stencil reaches as far as the box edge (reach " + std::to_string(t.reach[0]) + "," +
              std::to_string(t.reach[1]) + "," + std::to_string(t.reach[2]) + "); enlarge the box";
        return false;
    }
    if (t.reach[0] > 127 || t.reach[1] > 127 || t.reach[2] > 127) { why = "stencil too wide"; return false; }
    return true;
}

struct Layout {
    size_t sys, blk, sh_e, sh_u, tl_e, tl_w, bl_e;
    size_t f0, f1, n, j, u, g, vh, H, Nf;
    size_t red, red_out, series, series_cnt, fit_out;
    // spectral tail (float32 only)
    size_t wxf, wxi, wyf, wyi, wzf, wzi, S, s1, s2, tail;
    size_t total;
};

// Spectral mode: float32, a tail on some pair, y periodic.
bool wants_spectral(const mlb_params *p, const HostTables &t)
{
    if (t.tl_e.empty() || p->walls_y || p->precision != 32) return false;
    return p->tail_mode == MLB_TAIL_AUTO || p->tail_mode == MLB_TAIL_SPECTRAL;
}

Layout make_layout(const mlb_params *p, const HostTables &t, size_t tsize, size_t sys_size, int nblk)
{
    const size_t M = (size_t)p->nspecies, N = (size_t)p->nx * p->ny * p->nz;
    const size_t P = M * (M + 1) / 2;
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + std::max<size_t>(bytes, 1)); return o; };
    L.sys = take(2 * sys_size);
    L.blk = take(sizeof(int) * (size_t)nblk);
    L.sh_e = take(sizeof(int32_t) * t.sh_e.size());
    L.sh_u = take(tsize * t.sh_u.size());
    L.tl_e = take(sizeof(int32_t) * t.tl_e.size());
    L.tl_w = take(tsize * t.tl_w.size());
    L.bl_e = take(sizeof(int32_t) * t.bl_e.size());
    L.f0 = take(tsize * M * mlb::kQ * N);
    L.f1 = take(tsize * M * mlb::kQ * N);
    L.n = take(tsize * M * N);
    L.j = take(tsize * 3 * M * N);
    L.u = take(tsize * 3 * N);
    L.g = take(tsize * P * N);
    L.vh = take(tsize * 3 * M * N);
    L.H = take(tsize * 3 * M * N);
    L.Nf = take(tsize * 3 * M * N);
    L.red = take(sizeof(double) * kRedParts * 16);
    L.red_out = take(sizeof(double) * 16);
    L.series = take(sizeof(double) * 2 * kSeriesCap);
    L.series_cnt = take(sizeof(int));
    L.fit_out = take(sizeof(double) * 4);
    if (wants_spectral(p, t)) {
        const size_t nkx = (size_t)p->nx / 2 + 1, Sp = nkx * p->ny * p->nz;
        const size_t fields = std::max(3 * M, 3 * P);
        L.wxf = take(sizeof(float) * p->nx * 2 * nkx);
        L.wxi = take(sizeof(float) * 2 * nkx * p->nx);
        L.wyf = take(sizeof(float) * 4 * p->ny * p->ny);
        L.wyi = take(sizeof(float) * 4 * p->ny * p->ny);
        L.wzf = take(sizeof(float) * 4 * p->nz * p->nz);
        L.wzi = take(sizeof(float) * 4 * p->nz * p->nz);
        L.S = take(sizeof(float) * 3 * P * Sp);
        L.s1 = take(sizeof(float) * 2 * fields * Sp);
        L.s2 = take(sizeof(float) * 2 * fields * Sp);
        L.tail = take(sizeof(float) * 3 * M * N);
    }
    L.total = off;
    return L;
}

}  // namespace

// --------------------------------------------------------------- the handle
struct mlb_mixture_s {
    mlb_params p;
    int M = 0, P = 0;
    long long N = 0;
    int nblk = 0;
    char *ws = nullptr;
    Layout L{};
    HostTables tabs;
    int parity = 0;
    int64_t steps = 0;
    std::vector<unsigned char> sys_host;   // two descriptors: [0] stepping, [1] query
    size_t sys_size = 0;
    int tail_direct = 1;
    bool spectral = false;
    mlb::SpectralPlan plan;
    // per-pass event timing
    bool profiling = false;
    std::vector<hipEvent_t> events;          // pool, reused
    std::vector<std::pair<int, int>> marks;  // (pass, index of the start event)
    size_t next_event = 0;
    ~mlb_mixture_s()
    {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
    }

    template <typename T> mlb::SysDesc<T> *host_desc(int k) { return reinterpret_cast<mlb::SysDesc<T> *>(sys_host.data() + k * sys_size); }
    template <typename T> const mlb::SysDesc<T> *dev_desc(int k) const { return reinterpret_cast<const mlb::SysDesc<T> *>(ws + L.sys + k * sys_size); }
    const int *blk() const { return reinterpret_cast<const int *>(ws + L.blk); }
    template <typename T> mlb::Tables<T> tables() const
    {
        mlb::Tables<T> tb;
        tb.sh_e = reinterpret_cast<const int32_t *>(ws + L.sh_e);
        tb.sh_u = reinterpret_cast<const T *>(ws + L.sh_u);
        tb.tl_e = reinterpret_cast<const int32_t *>(ws + L.tl_e);
        tb.tl_w = reinterpret_cast<const T *>(ws + L.tl_w);
        tb.bl_e = reinterpret_cast<const int32_t *>(ws + L.bl_e);
        return tb;
    }
};

namespace {

template <typename T>
void fill_desc(mlb_mixture_s *h, mlb::SysDesc<T> &S)
{
    const mlb_params *p = &h->p;
    std::memset(&S, 0, sizeof(S));
    S.nx = p->nx; S.ny = p->ny; S.nz = p->nz; S.M = h->M; S.P = h->P; S.walls = p->walls_y ? 1 : 0;
    S.N = h->N;
    S.block_start = 0;
    S.nblocks = h->nblk;
    char *ws = h->ws;
    S.f[0] = reinterpret_cast<T *>(ws + h->L.f0);
    S.f[1] = reinterpret_cast<T *>(ws + h->L.f1);
    S.n = reinterpret_cast<T *>(ws + h->L.n);
    S.j = reinterpret_cast<T *>(ws + h->L.j);
    S.u = reinterpret_cast<T *>(ws + h->L.u);
    S.g = reinterpret_cast<T *>(ws + h->L.g);
    S.vh = reinterpret_cast<T *>(ws + h->L.vh);
    S.H = reinterpret_cast<T *>(ws + h->L.H);
    S.Nf = reinterpret_cast<T *>(ws + h->L.Nf);
    S.tail = h->spectral ? reinterpret_cast<T *>(ws + h->L.tail) : nullptr;
    S.parts = nullptr;
    S.parts_mask = 0;
    S.tail_direct = h->tail_direct;
    S.scheme = p->scheme;
    S.omega_is_one = (1.0 / p->tau == 1.0) ? 1 : 0;
    const HostTables &t = h->tabs;
    for (int a = 0; a < h->M; ++a) {
        S.bl_start[a] = t.bl_start[a]; S.bl_cnt[a] = t.bl_cnt[a]; S.bl_full[a] = t.bl_full[a];
        const double sg = p->sigma[a];
        S.s2[a] = (T)((M_PI / 6.0) * (sg * sg));
        S.s3[a] = (T)((M_PI / 6.0) * ((sg * sg) * sg));
        for (int d = 0; d < 3; ++d) S.fext[a][d] = (T)p->ext_force[a * 3 + d];
        for (int b = 0; b < h->M; ++b) {
            S.sh_start[a][b] = t.sh_start[a][b]; S.sh_cnt[a][b] = t.sh_cnt[a][b];
            S.tl_start[a][b] = t.tl_start[a][b]; S.tl_cnt[a][b] = t.tl_cnt[a][b];
            const mlb::PairConst c = mlb::pair_constants(p->sigma[a], p->sigma[b], p->kT, t.sh_full[a][b]);
            S.cm[a][b] = (T)c.cm; S.cg[a][b] = (T)c.cg; S.ck[a][b] = (T)c.ck; S.dd[a][b] = (T)c.dd;
        }
    }
    const double omega = 1.0 / p->tau;
    S.omega = (T)omega;
    S.om1 = (T)(1.0 - omega);
    S.wall_ux[0] = (T)p->wall_ux[0];
    S.wall_ux[1] = (T)p->wall_ux[1];
}

template <typename T>
mlb_status upload_tables(mlb_mixture_s *h, hipStream_t st)
{
    const HostTables &t = h->tabs;
    std::vector<T> su(t.sh_u.begin(), t.sh_u.end()), tw(t.tl_w.begin(), t.tl_w.end());
    char *ws = h->ws;
    if (!t.sh_e.empty()) HIP_TRY(hipMemcpyAsync(ws + h->L.sh_e, t.sh_e.data(), 4 * t.sh_e.size(), hipMemcpyHostToDevice, st));
    if (!su.empty()) HIP_TRY(hipMemcpyAsync(ws + h->L.sh_u, su.data(), sizeof(T) * su.size(), hipMemcpyHostToDevice, st));
    if (!t.tl_e.empty()) HIP_TRY(hipMemcpyAsync(ws + h->L.tl_e, t.tl_e.data(), 4 * t.tl_e.size(), hipMemcpyHostToDevice, st));
    if (!tw.empty()) HIP_TRY(hipMemcpyAsync(ws + h->L.tl_w, tw.data(), sizeof(T) * tw.size(), hipMemcpyHostToDevice, st));
    if (!t.bl_e.empty()) HIP_TRY(hipMemcpyAsync(ws + h->L.bl_e, t.bl_e.data(), 4 * t.bl_e.size(), hipMemcpyHostToDevice, st));
    std::vector<int> blk((size_t)h->nblk, 0);
    HIP_TRY(hipMemcpyAsync(ws + h->L.blk, blk.data(), sizeof(int) * blk.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));   // host staging vectors die here
    return MLB_OK;
}

template <typename T>
mlb_status upload_desc(mlb_mixture_s *h, int k, hipStream_t st)
{
    HIP_TRY(hipMemcpyAsync(h->ws + h->L.sys + k * h->sys_size, h->sys_host.data() + k * h->sys_size, h->sys_size,
                           hipMemcpyHostToDevice, st));
    return MLB_OK;
}

enum { kPassMoments = 0, kPassContact = 1, kPassTail = 2, kPassGather1 = 3, kPassStep2 = 4 };
const char *kPassNames[MLB_NPASS] = {"moments", "contact", "tail", "gather1", "step2"};

hipEvent_t take_event(mlb_mixture_s *h)
{
    if (h->next_event == h->events.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->events.push_back(e);
    }
    return h->events[h->next_event++];
}

// Run one pass; when profiling, bracket it with an event pair on `st`.
template <typename F>
void pass(mlb_mixture_s *h, int id, hipStream_t st, F &&launch)
{
    if (!h->profiling) {
        launch();
        return;
    }
    const size_t k = h->next_event;
    hipEvent_t a = take_event(h), b = take_event(h);
    if (!a || !b) {
        launch();
        return;
    }
    (void)hipEventRecord(a, st);
    launch();
    (void)hipEventRecord(b, st);
    h->marks.emplace_back(id, (int)k);
}

void run_tail(mlb_mixture_s *h, hipStream_t st)
{
    char *ws = h->ws;
    h->plan.apply(reinterpret_cast<const float *>(ws + h->L.n), reinterpret_cast<float *>(ws + h->L.s1),
                  reinterpret_cast<float *>(ws + h->L.s2), reinterpret_cast<float *>(ws + h->L.tail), st);
}

template <typename T>
void run_step(mlb_mixture_s *h, hipStream_t st)
{
    const mlb::SysDesc<T> *sys = h->dev_desc<T>(0);
    const mlb::Tables<T> tb = h->tables<T>();
    const int *blk = h->blk();
    const int nblk = h->nblk, M = h->M, par = h->parity;
    pass(h, kPassMoments, st, [&] { mlb::Launch<T>::moments(sys, blk, nblk, par, st); });
    pass(h, kPassContact, st, [&] { mlb::Launch<T>::contact(sys, blk, nblk, tb, st); });
    if (h->spectral) pass(h, kPassTail, st, [&] { run_tail(h, st); });
    pass(h, kPassGather1, st, [&] { mlb::Launch<T>::gather1(sys, blk, nblk, M, tb, st); });
    pass(h, kPassStep2, st, [&] { mlb::Launch<T>::step2(sys, blk, nblk, M, tb, par, 0, st); });
    h->parity ^= 1;
    h->steps += 1;
}

// Evaluate the passes up to the force on the current populations with the
// query descriptor (parts accumulator optionally set).
template <typename T>
mlb_status run_query(mlb_mixture_s *h, T *parts, unsigned mask, hipStream_t st)
{
    mlb::SysDesc<T> *q = h->host_desc<T>(1);
    *q = *h->host_desc<T>(0);
    q->parts = parts;
    q->parts_mask = mask;
    mlb_status s = upload_desc<T>(h, 1, st);
    if (s != MLB_OK) return s;
    const mlb::SysDesc<T> *sys = h->dev_desc<T>(1);
    const mlb::Tables<T> tb = h->tables<T>();
    mlb::Launch<T>::moments(sys, h->blk(), h->nblk, h->parity, st);
    mlb::Launch<T>::contact(sys, h->blk(), h->nblk, tb, st);
    if (h->spectral) run_tail(h, st);
    mlb::Launch<T>::gather1(sys, h->blk(), h->nblk, h->M, tb, st);
    mlb::Launch<T>::step2(sys, h->blk(), h->nblk, h->M, tb, h->parity, 1, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return MLB_OK;
}

size_t tsize_of(const mlb_params *p) { return p->precision == 64 ? sizeof(double) : sizeof(float); }

// Upload the DFT matrices, place the tail kernels w_ab on the periodic grid
// (the population buffer f1 serves as scratch; it is overwritten by the
// first step) and transform them into the sine spectra S_ab.
mlb_status setup_spectral(mlb_mixture_s *h, hipStream_t st)
{
    const mlb_params *p = &h->p;
    mlb::SpectralPlan &pl = h->plan;
    char *ws = h->ws;
    pl.nx = p->nx; pl.ny = p->ny; pl.nz = p->nz; pl.nkx = p->nx / 2 + 1;
    pl.M = h->M; pl.P = h->P;
    pl.Sz = (long long)pl.ny * pl.nkx;
    pl.Sp = pl.Sz * pl.nz;
    pl.wxf = reinterpret_cast<const float *>(ws + h->L.wxf);
    pl.wxi = reinterpret_cast<const float *>(ws + h->L.wxi);
    pl.wyf = reinterpret_cast<const float *>(ws + h->L.wyf);
    pl.wyi = reinterpret_cast<const float *>(ws + h->L.wyi);
    pl.wzf = reinterpret_cast<const float *>(ws + h->L.wzf);
    pl.wzi = reinterpret_cast<const float *>(ws + h->L.wzi);
    pl.S = reinterpret_cast<float *>(ws + h->L.S);
    std::vector<float> m[6] = {mlb::SpectralPlan::dft_x_forward(p->nx), mlb::SpectralPlan::dft_x_inverse(p->nx),
                               mlb::SpectralPlan::dft_block(p->ny, false), mlb::SpectralPlan::dft_block(p->ny, true),
                               mlb::SpectralPlan::dft_block(p->nz, false), mlb::SpectralPlan::dft_block(p->nz, true)};
    const size_t offs[6] = {h->L.wxf, h->L.wxi, h->L.wyf, h->L.wyi, h->L.wzf, h->L.wzi};
    for (int k = 0; k < 6; ++k)
        HIP_TRY(hipMemcpyAsync(ws + offs[k], m[k].data(), sizeof(float) * m[k].size(), hipMemcpyHostToDevice, st));
    // kernels on the grid: field (p, d) = sum over the full tail set of w_d(e) at e mod L
    const long long N = h->N;
    std::vector<float> placed((size_t)3 * h->P * N, 0.0f);
    std::vector<double> acc((size_t)3 * N);
    const HostTables &t = h->tabs;
    for (int a = 0; a < h->M; ++a)
        for (int b = a; b < h->M; ++b) {
            const int pi = a * h->M - (a * (a - 1)) / 2 + (b - a);
            std::fill(acc.begin(), acc.end(), 0.0);
            for (int k = 0; k < t.tl_cnt[a][b]; ++k) {
                int ex, ey, ez;
                mlb::unpack_offset(t.tl_e[t.tl_start[a][b] + k], ex, ey, ez);
                for (int sgn = -1; sgn <= 1; sgn += 2) {
                    const int x = ((sgn * ex) % p->nx + p->nx) % p->nx;
                    const int y = ((sgn * ey) % p->ny + p->ny) % p->ny;
                    const int z = ((sgn * ez) % p->nz + p->nz) % p->nz;
                    const long long site = ((long long)z * p->ny + y) * p->nx + x;
                    for (int d = 0; d < 3; ++d) acc[(size_t)d * N + site] += sgn * t.tl_w[3 * (t.tl_start[a][b] + k) + d];
                }
            }
            for (int d = 0; d < 3; ++d)
                for (long long i = 0; i < N; ++i) placed[((size_t)pi * 3 + d) * N + i] = (float)acc[(size_t)d * N + i];
        }
    float *scratch = reinterpret_cast<float *>(ws + h->L.f1);
    HIP_TRY(hipMemcpyAsync(scratch, placed.data(), sizeof(float) * placed.size(), hipMemcpyHostToDevice, st));
    pl.build_spectrum(scratch, reinterpret_cast<float *>(ws + h->L.s1), reinterpret_cast<float *>(ws + h->L.s2), st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));   // host staging vectors die here
    return MLB_OK;
}

}  // namespace

// ===================================================================== ABI
extern "C" {

size_t mlb_workspace_bytes(const mlb_params *p)
{
    std::string why;
    if (!validate(p, why)) { g_err = why; return 0; }
    HostTables t;
    if (!build_tables(p, t, why)) { g_err = why; return 0; }
    const long long N = (long long)p->nx * p->ny * p->nz;
    const int nblk = (int)((N + mlb::kBlock - 1) / mlb::kBlock);
    const size_t sys_size = p->precision == 64 ? sizeof(mlb::SysDesc<double>) : sizeof(mlb::SysDesc<float>);
    return make_layout(p, t, tsize_of(p), align_up(sys_size), nblk).total;
}

mlb_status mlb_init_mixture(const mlb_params *p, void *workspace, size_t workspace_bytes, const double *n0,
                            const double *u0, void *stream, mlb_mixture *out)
{
    if (!out) return fail(MLB_EINVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    if (!validate(p, why)) return fail(MLB_EINVAL, why);
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return fail(MLB_EINVAL, "workspace must be a 256-byte aligned device pointer");
    if (!n0 || !u0) return fail(MLB_EINVAL, "n0 and u0 are required");
    std::unique_ptr<mlb_mixture_s> h(new mlb_mixture_s());
    h->p = *p;
    if (!build_tables(p, h->tabs, why)) return fail(MLB_EINVAL, why);
    h->M = p->nspecies;
    h->P = h->M * (h->M + 1) / 2;
    h->N = (long long)p->nx * p->ny * p->nz;
    h->nblk = (int)((h->N + mlb::kBlock - 1) / mlb::kBlock);
    const bool f64 = p->precision == 64;
    h->sys_size = align_up(f64 ? sizeof(mlb::SysDesc<double>) : sizeof(mlb::SysDesc<float>));
    h->L = make_layout(p, h->tabs, tsize_of(p), h->sys_size, h->nblk);
    if (workspace_bytes < h->L.total)
        return fail(MLB_ENOMEM, "workspace too small: need " + std::to_string(h->L.total) + " bytes");
    const bool any_tail = !h->tabs.tl_e.empty();
    if (p->tail_mode == MLB_TAIL_SPECTRAL && any_tail && (p->precision != 32 || p->walls_y))
        return fail(MLB_EUNSUPPORTED, "the spectral tail needs float32 and a periodic box");
    h->spectral = wants_spectral(p, h->tabs);
    h->tail_direct = h->spectral ? 0 : 1;
    h->ws = static_cast<char *>(workspace);
    h->sys_host.assign(2 * h->sys_size, 0);
    hipStream_t st = static_cast<hipStream_t>(stream);
    mlb_status s;
    if (f64) {
        fill_desc<double>(h.get(), *h->host_desc<double>(0));
        *h->host_desc<double>(1) = *h->host_desc<double>(0);
        if ((s = upload_tables<double>(h.get(), st)) != MLB_OK) return s;
        if ((s = upload_desc<double>(h.get(), 0, st)) != MLB_OK) return s;
        mlb::Launch<double>::init_pop(h->dev_desc<double>(0), h->blk(), h->nblk, n0, u0, st);
    } else {
        fill_desc<float>(h.get(), *h->host_desc<float>(0));
        *h->host_desc<float>(1) = *h->host_desc<float>(0);
        if ((s = upload_tables<float>(h.get(), st)) != MLB_OK) return s;
        if ((s = upload_desc<float>(h.get(), 0, st)) != MLB_OK) return s;
        if (h->spectral && (s = setup_spectral(h.get(), st)) != MLB_OK) return s;
        mlb::Launch<float>::init_pop(h->dev_desc<float>(0), h->blk(), h->nblk, n0, u0, st);
    }
    mlb::launch_zero_i32(reinterpret_cast<int *>(h->ws + h->L.series_cnt), 1, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    *out = h.release();
    return MLB_OK;
}

mlb_status mlb_step(mlb_mixture h, int32_t nsteps, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    if (nsteps < 0) return fail(MLB_EINVAL, "nsteps must be >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int t = 0; t < nsteps; ++t) {
        if (h->p.precision == 64) run_step<double>(h, st);
        else run_step<float>(h, st);
    }
    HIP_TRY(hipGetLastError());
    return MLB_OK;
}

mlb_status mlb_moments(mlb_mixture h, void *n_out, void *j_out, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t ts = tsize_of(&h->p);
    if (h->p.precision == 64) mlb::Launch<double>::moments(h->dev_desc<double>(0), h->blk(), h->nblk, h->parity, st);
    else mlb::Launch<float>::moments(h->dev_desc<float>(0), h->blk(), h->nblk, h->parity, st);
    if (n_out) HIP_TRY(hipMemcpyAsync(n_out, h->ws + h->L.n, ts * h->M * h->N, hipMemcpyDeviceToDevice, st));
    if (j_out) HIP_TRY(hipMemcpyAsync(j_out, h->ws + h->L.j, ts * 3 * h->M * h->N, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipGetLastError());
    return MLB_OK;
}

mlb_status mlb_forces(mlb_mixture h, void *nphi_out, uint32_t parts, void *stream)
{
    if (!h || !nphi_out) return fail(MLB_EINVAL, "handle and output are required");
    if (parts == 0 || parts > MLB_PART_ALL) return fail(MLB_EINVAL, "parts mask must be a non-empty subset of MLB_PART_ALL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (h->p.precision == 64) return run_query<double>(h, static_cast<double *>(nphi_out), parts, st);
    return run_query<float>(h, static_cast<float *>(nphi_out), parts, st);
}

mlb_status mlb_fields(mlb_mixture h, void *n, void *j, void *u, void *g, void *vhat, void *H, void *nphi, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    mlb_status s = h->p.precision == 64 ? run_query<double>(h, nullptr, 0, st) : run_query<float>(h, nullptr, 0, st);
    if (s != MLB_OK) return s;
    const size_t ts = tsize_of(&h->p), M = h->M, N = (size_t)h->N;
    struct { void *dst; size_t off, bytes; } cp[] = {
        {n, h->L.n, ts * M * N}, {j, h->L.j, ts * 3 * M * N}, {u, h->L.u, ts * 3 * N},
        {g, h->L.g, ts * (size_t)h->P * N}, {vhat, h->L.vh, ts * 3 * M * N}, {H, h->L.H, ts * 3 * M * N},
        {nphi, h->L.Nf, ts * 3 * M * N}};
    for (auto &c : cp)
        if (c.dst) HIP_TRY(hipMemcpyAsync(c.dst, h->ws + c.off, c.bytes, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return MLB_OK;
}

mlb_status mlb_get_populations(mlb_mixture h, void *f_out, void *stream)
{
    if (!h || !f_out) return fail(MLB_EINVAL, "handle and output are required");
    const size_t bytes = tsize_of(&h->p) * h->M * mlb::kQ * h->N;
    HIP_TRY(hipMemcpyAsync(f_out, h->ws + (h->parity ? h->L.f1 : h->L.f0), bytes, hipMemcpyDeviceToDevice,
                           static_cast<hipStream_t>(stream)));
    return MLB_OK;
}

mlb_status mlb_set_populations(mlb_mixture h, const void *f_in, void *stream)
{
    if (!h || !f_in) return fail(MLB_EINVAL, "handle and input are required");
    const size_t bytes = tsize_of(&h->p) * h->M * mlb::kQ * h->N;
    HIP_TRY(hipMemcpyAsync(h->ws + (h->parity ? h->L.f1 : h->L.f0), f_in, bytes, hipMemcpyDeviceToDevice,
                           static_cast<hipStream_t>(stream)));
    return MLB_OK;
}

mlb_status mlb_conserved(mlb_mixture h, double *mass, double *mom, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    hipStream_t st = static_cast<hipStream_t>(stream);
    mlb_status s = mlb_moments(h, nullptr, nullptr, stream);
    if (s != MLB_OK) return s;
    double *out = reinterpret_cast<double *>(h->ws + h->L.red_out);
    mlb::launch_conserved(h->ws + h->L.n, h->ws + h->L.j, h->p.precision, h->M, h->N,
                          reinterpret_cast<double *>(h->ws + h->L.red), kRedParts, out, st);
    double host[16];
    HIP_TRY(hipMemcpyAsync(host, out, sizeof(double) * 4 * h->M, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    bool finite = true;
    for (int k = 0; k < 4 * h->M; ++k) finite = finite && std::isfinite(host[k]);
    if (mass) for (int a = 0; a < h->M; ++a) mass[a] = host[a];
    if (mom) for (int k = 0; k < 3 * h->M; ++k) mom[k] = host[h->M + k];
    if (!finite) return fail(MLB_ENONFINITE, "a conserved sum is not finite");
    return MLB_OK;
}

mlb_status mlb_record_mode(mlb_mixture h, int32_t a, int32_t b, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    if (a < 0 || b < 0 || a >= h->M || b >= h->M || a == b) return fail(MLB_EINVAL, "bad species pair");
    hipStream_t st = static_cast<hipStream_t>(stream);
    mlb_status s = mlb_moments(h, nullptr, nullptr, stream);
    if (s != MLB_OK) return s;
    mlb::launch_mode(h->ws + h->L.n, h->p.precision, a, b, h->p.nx, h->N, reinterpret_cast<double *>(h->ws + h->L.red),
                     kRedParts, reinterpret_cast<double *>(h->ws + h->L.series),
                     reinterpret_cast<int *>(h->ws + h->L.series_cnt), kSeriesCap, (double)h->steps, st);
    HIP_TRY(hipGetLastError());
    return MLB_OK;
}

mlb_status mlb_record_spread(mlb_mixture h, int32_t a, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    if (a < 0 || a >= h->M) return fail(MLB_EINVAL, "bad species");
    hipStream_t st = static_cast<hipStream_t>(stream);
    mlb_status s = mlb_moments(h, nullptr, nullptr, stream);
    if (s != MLB_OK) return s;
    mlb::launch_spread(h->ws + h->L.n, h->p.precision, a, h->p.nx, h->N, reinterpret_cast<double *>(h->ws + h->L.red),
                       kRedParts, reinterpret_cast<double *>(h->ws + h->L.series),
                       reinterpret_cast<int *>(h->ws + h->L.series_cnt), kSeriesCap, (double)h->steps, st);
    HIP_TRY(hipGetLastError());
    return MLB_OK;
}

int32_t mlb_series_capacity(void) { return kSeriesCap; }

mlb_status mlb_series_reset(mlb_mixture h, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    mlb::launch_zero_i32(reinterpret_cast<int *>(h->ws + h->L.series_cnt), 1, static_cast<hipStream_t>(stream));
    HIP_TRY(hipGetLastError());
    return MLB_OK;
}

mlb_status mlb_fit_series(mlb_mixture h, int32_t kind, double t_min, double *D_out, void *stream)
{
    if (!h || !D_out) return fail(MLB_EINVAL, "handle and output are required");
    if (kind != 0 && kind != 1) return fail(MLB_EINVAL, "kind must be 0 (mode) or 1 (spread)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double k = 2.0 * M_PI / (double)h->p.nx;
    double *out = reinterpret_cast<double *>(h->ws + h->L.fit_out);
    mlb::launch_fit(reinterpret_cast<const double *>(h->ws + h->L.series),
                    reinterpret_cast<const int *>(h->ws + h->L.series_cnt), kSeriesCap, kind, t_min, k * k, out, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(D_out, out, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return MLB_OK;
}

mlb_status mlb_get_series(mlb_mixture h, double *t, double *v, int32_t capacity, int32_t *count, void *stream)
{
    if (!h || !count) return fail(MLB_EINVAL, "handle and count are required");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int c = 0;
    HIP_TRY(hipMemcpyAsync(&c, h->ws + h->L.series_cnt, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    c = std::min(c, kSeriesCap);
    *count = c;
    const int n = std::min(c, capacity);
    if (n > 0 && (t || v)) {
        std::vector<double> buf(2 * (size_t)n);
        HIP_TRY(hipMemcpyAsync(buf.data(), h->ws + h->L.series, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int i = 0; i < n; ++i) {
            if (t) t[i] = buf[2 * i];
            if (v) v[i] = buf[2 * i + 1];
        }
    }
    return MLB_OK;
}

int64_t mlb_step_count(mlb_mixture h) { return h ? h->steps : -1; }

mlb_status mlb_profile_begin(mlb_mixture h)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    h->profiling = true;
    h->marks.clear();
    h->next_event = 0;
    return MLB_OK;
}

mlb_status mlb_profile_end(mlb_mixture h, double *ms, int32_t *launches, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    if (!h->profiling) return fail(MLB_ESTATE, "profiling was not started");
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    double acc[MLB_NPASS] = {0, 0, 0, 0, 0};
    int cnt[MLB_NPASS] = {0, 0, 0, 0, 0};
    for (auto &m : h->marks) {
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, h->events[m.second], h->events[m.second + 1]));
        acc[m.first] += t;
        cnt[m.first] += 1;
    }
    for (int k = 0; k < MLB_NPASS; ++k) {
        if (ms) ms[k] = acc[k];
        if (launches) launches[k] = cnt[k];
    }
    h->profiling = false;
    h->marks.clear();
    h->next_event = 0;
    return MLB_OK;
}

const char *mlb_pass_name(int32_t k) { return (k >= 0 && k < MLB_NPASS) ? kPassNames[k] : ""; }

mlb_status mlb_destroy(mlb_mixture h)
{
    delete h;
    return MLB_OK;
}

const char *mlb_last_error(void) { return g_err.c_str(); }

}  // extern "C"
