// C ABI of the mlb library (declared in include/mlb.h).
//
// The core object is a batch of lattice systems.  A mixture is a batch of
// one.  All device memory is the caller's workspace; this file validates
// parameters, builds the stencil tables on the host, lays out the
// workspace, builds the block->system maps, sequences the passes of a step
// on the caller's stream (optionally replaying a captured hipGraph) and
// runs the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/mlb.h"
#include "cnn.h"
#include "collide_f32.h"
#include "mlb_internal.h"
#include "net_internal.h"
#include "spectral.h"

// Workspace of mlb_init_mixture_static (one copy per GPU).
static __device__ __align__(256) char scratch[MLB_STATIC_WORKSPACE_BYTES];

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

#define TRY(expr)                    \
    do {                             \
        mlb_status s_ = (expr);      \
        if (s_ != MLB_OK) return s_; \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kSeriesCap = 8192;
constexpr int kRedParts = 512;
constexpr int kFitOut = 8;   // doubles per fit result: D, slope, samples, R^2, well-conditioned flag
constexpr int kXcds = 8;   // MI355X: workgroups are dealt round-robin over 8 XCDs
constexpr double kMassMin = 0.625, kMassMax = 2.5;   // species masses the lattice equilibrium represents

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// ----------------------------------------------------------- host tables
struct HostTables {
    std::vector<int32_t> sh_e, tl_e, bl_e;
    std::vector<double> sh_u, tl_w;
    std::vector<float> sg;   // sign groups, 4 floats per float4
    int sg_start[mlb::kMaxS][mlb::kMaxS][mlb::kGroupKinds] = {}, sg_cnt[mlb::kMaxS][mlb::kMaxS][mlb::kGroupKinds] = {};
    int sh_start[mlb::kMaxS][mlb::kMaxS] = {}, sh_cnt[mlb::kMaxS][mlb::kMaxS] = {};
    int sh_full[mlb::kMaxS][mlb::kMaxS] = {};
    int tl_start[mlb::kMaxS][mlb::kMaxS] = {}, tl_cnt[mlb::kMaxS][mlb::kMaxS] = {};
    int bl_start[mlb::kMaxS] = {}, bl_cnt[mlb::kMaxS] = {}, bl_full[mlb::kMaxS] = {};
    int reach[3] = {0, 0, 0};
    int shell_reach = 0, ball_reach = 0;
    int tail_reach_y = 0;   // largest |e_y| of any tail offset
};

bool validate(const mlb_params *p, std::string &why)
{
    if (!p) { why = "params is NULL"; return false; }
    const int M = p->nspecies;
    if (M < 1 || M > MLB_MAX_SPECIES) { why = "nspecies must be 1..4"; return false; }
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) { why = "lattice sizes must be positive"; return false; }
    if ((long long)p->nx * p->ny * p->nz > (1LL << 31) / 4) { why = "lattice too large"; return false; }
    if (p->precision != 32 && p->precision != 64) { why = "precision must be 32 or 64"; return false; }
    if (p->scheme != MLB_SCHEME_CN_J1 && p->scheme != MLB_SCHEME_FE) { why = "unknown scheme"; return false; }
    if (p->tail_mode < MLB_TAIL_AUTO || p->tail_mode > MLB_TAIL_SPECTRAL) { why = "unknown tail mode"; return false; }
    if (!(p->tau > 0.5)) { why = "tau must exceed 1/2"; return false; }
    if (std::fabs(p->kT - 1.0 / 3.0) > 1e-12) { why = "kT must be 1/3 (the D3Q19 lattice's c_s^2)"; return false; }
    if (p->walls_y && p->ny < 3) { why = "walls need ny >= 3"; return false; }
    for (int a = 0; a < M; ++a) {
        // theta_a = kT/m_a in [2/15, 8/15]: the lattice equilibrium at rest
        // keeps at least a tenth of its weight on every velocity
        if (!(p->mass[a] >= kMassMin && p->mass[a] <= kMassMax)) {
            why = "masses must lie in [0.625, 2.5]";
            return false;
        }
        if (!(p->sigma[a] > 0.0) || p->sigma[a] > 40.0) { why = "sigma must be in (0, 40]"; return false; }
        for (int b = 0; b < M; ++b) {
            const double e = p->eps[a * MLB_MAX_SPECIES + b];
            if (!(e >= 0.0) || e != p->eps[b * MLB_MAX_SPECIES + a]) { why = "eps must be symmetric and >= 0"; return false; }
            if (e > 0.0 && !(p->rc_factor > 1.0)) { why = "rc_factor must exceed 1 when a tail is on"; return false; }
        }
    }
    return true;
}

// Sign groups of the (a, b) shell half-list for the float32 first gather:
// points that differ only in the signs of their y and z components share
// |e_hat| and are summed together.  The representative of a group has
// e_y, e_z >= 0; members follow in the order (+y, +z), (-y, +z), (+y, -z),
// (-y, -z).  Returns false if the half-list is not closed under these sign
// changes (it always is: they keep |e|^2 and the first component).
bool build_groups(const mlb::HostStencil &sh, HostTables &t, int a, int b)
{
    std::map<int32_t, size_t> at;
    for (size_t k = 0; k < sh.e.size(); ++k) at[sh.e[k]] = k;
    auto bits = [](int32_t v) { float f; std::memcpy(&f, &v, 4); return f; };
    std::vector<float> kind[mlb::kGroupKinds];
    int cnt[mlb::kGroupKinds] = {}, covered = 0;
    for (size_t k = 0; k < sh.e.size(); ++k) {
        int ex, ey, ez;
        mlb::unpack_offset(sh.e[k], ex, ey, ez);
        const double ux = sh.v[3 * k], uy = sh.v[3 * k + 1], uz = sh.v[3 * k + 2];
        auto member = [&](int x, int y, int z) { return at.count(mlb::pack_offset(x, y, z)) == 1; };
        const int nz = (ex != 0) + (ey != 0) + (ez != 0);
        if (nz == 3 && ey > 0 && ez > 0) {
            if (!member(ex, -ey, ez) || !member(ex, ey, -ez) || !member(ex, -ey, -ez)) return false;
            const float f[16] = {bits(mlb::pack_offset(ex, ey, ez)), bits(mlb::pack_offset(ex, -ey, ez)),
                                 bits(mlb::pack_offset(ex, ey, -ez)), bits(mlb::pack_offset(ex, -ey, -ez)),
                                 (float)ux, (float)uy, (float)uz, 0.f,
                                 (float)(ux * ux), (float)(uy * uy), (float)(uz * uz), 0.f,
                                 (float)(ux * uy), (float)(ux * uz), (float)(uy * uz), 0.f};
            kind[0].insert(kind[0].end(), f, f + 16);
            ++cnt[0]; covered += 4;
        } else if (nz == 2 && ((ez == 0 && ey > 0) || (ey == 0 && ez > 0) || (ex == 0 && ez > 0))) {
            // shared axis A (e_x, or e_y when e_x = 0), flipped axis B
            const int kd = ez == 0 ? 1 : ey == 0 ? 2 : 3;
            const double A = kd == 3 ? uy : ux, B = kd == 1 ? uy : uz;
            const int32_t o2 = kd == 1 ? mlb::pack_offset(ex, -ey, ez) : mlb::pack_offset(ex, ey, -ez);
            if (at.count(o2) != 1) return false;
            const float f[8] = {bits(sh.e[k]), bits(o2), (float)A, (float)B,
                                (float)(A * A), (float)(B * B), (float)(A * B), 0.f};
            kind[kd].insert(kind[kd].end(), f, f + 8);
            ++cnt[kd]; covered += 2;
        } else if (nz == 1) {
            const float f[4] = {bits(sh.e[k]), (float)ux, (float)uy, (float)uz};
            kind[4].insert(kind[4].end(), f, f + 4);
            ++cnt[4]; covered += 1;
        }
    }
    if (covered != (int)sh.e.size()) return false;
    for (int kd = 0; kd < mlb::kGroupKinds; ++kd) {
        t.sg_start[a][b][kd] = (int)(t.sg.size() / 4);
        t.sg_cnt[a][b][kd] = cnt[kd];
        t.sg.insert(t.sg.end(), kind[kd].begin(), kind[kd].end());
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
        for (int d = 0; d < 3; ++d) t.ball_reach = std::max(t.ball_reach, b.max_abs[d]);
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
            if (!build_groups(sh, t, a, b)) { why = "shell half-list not closed under sign changes"; return false; }
            for (int d = 0; d < 3; ++d) t.shell_reach = std::max(t.shell_reach, sh.max_abs[d]);
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
                t.tail_reach_y = std::max(t.tail_reach_y, tl.max_abs[1]);
                reach(tl);
            }
        }
    if (t.reach[0] >= p->nx || t.reach[2] >= p->nz || (!p->walls_y && t.reach[1] >= p->ny)) {
        why = "a stencil reaches as far as the box edge (reach " + std::to_string(t.reach[0]) + "," +
              std::to_string(t.reach[1]) + "," + std::to_string(t.reach[2]) + "); enlarge the box";
        return false;
    }
    // with walls the hard-core stencils read mirror images of the fluid
    // beyond a wall: one reflection must land inside the ny - 2 fluid rows
    if (p->walls_y && std::max(t.shell_reach, t.ball_reach) > p->ny - 2) {
        why = "walls need at least " + std::to_string(std::max(t.shell_reach, t.ball_reach)) +
              " fluid rows (the shell reach) between them; enlarge ny";
        return false;
    }
    if (t.reach[0] > 127 || t.reach[1] > 127 || t.reach[2] > 127) { why = "stencil too wide"; return false; }
    return true;
}

bool has_tail(const HostTables &t) { return !t.tl_e.empty(); }

// Transform length along y of the spectral field: ny for a periodic box;
// with walls, y is zero-padded past the tail's reach (rounded up to a
// multiple of 8), so the circular convolution on the padded line equals the
// linear one, in which points beyond the walls contribute nothing.
int spectral_ny(const mlb_params *p, const HostTables &t)
{
    if (!p->walls_y) return p->ny;
    return (p->ny + t.tail_reach_y + 7) / 8 * 8;
}

// Spectral attractive field: float32, a tail on some pair, single system,
// the (y, z) plane of the transform within the LDS budget.
bool spectral_possible(const mlb_params *p, const HostTables &t, int count)
{
    if (!has_tail(t) || p->precision != 32 || count != 1) return false;
    return mlb::SpectralPlan::fused_fits(spectral_ny(p, t), p->nz, p->nspecies);
}

bool wants_spectral(const mlb_params *p, const HostTables &t, int count)
{
    if (!spectral_possible(p, t, count)) return false;
    return p->tail_mode == MLB_TAIL_AUTO || p->tail_mode == MLB_TAIL_SPECTRAL;
}

// ----------------------------------------------------------- per system
struct SysHost {
    mlb_params p{};
    int M = 0, P = 0;
    long long N = 0;
    HostTables tabs;
    int sh_base = 0, tl_base = 0, bl_base = 0;   // offsets into the batch tables
    int sg_base = 0;                             // float4 offset of the sign groups
    bool spectral = false;
    mlb::SpectralPlan plan;
    int nblocks = 0;
    size_t f0 = 0, f1 = 0, n = 0, j = 0, u = 0, g = 0, vh = 0, H = 0, Nf = 0, Tloc = 0, gfac = 0;
    size_t wxf = 0, wxi = 0, wyf = 0, wyi = 0, wzf = 0, wzi = 0, S = 0, s1 = 0, s2 = 0, tail = 0;
    size_t series = 0, series_cnt = 0;
    size_t fprof = 0;            // body force per lattice row [M][3][ny]
    bool has_profile = false;
};

// Float32 tiling: tile shape, block order, the first gather's thread
// groups per site (2 or 3), its shell loop (plain or sign-grouped) and its
// own tile shape (the common one, or 4x8x8); trial_ms[(split - 2) 2 V +
// 2 shape + order] with the plain loop, groups_ms the chosen tiling with the
// sign-grouped loop.
constexpr int kSplitChoices = 2, kTrials = 2 * mlb::kTileVariants * kSplitChoices;
constexpr int kG1Own = 3;   // the first gather's own shape variant (4x8x8)
struct Tuning {
    int shape = 0, order = 1, g1split = 3, g1shape = 0;
    bool groups = false;
    double trial_ms[kTrials] = {};
    double groups_ms = 0.0;
};

// Static device workspace of mlb_init_mixture_static.  In host code the
// name stands for a host-side shadow, not a device address: the device
// address comes from hipGetSymbolAddress, once per device (each GPU holds
// its own copy), and is kept in g_static_ptr.  At most one live mixture per
// device uses it.
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};
bool g_static_busy[kMaxDevices] = {};

void release_static(int dev)
{
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (dev >= 0 && dev < kMaxDevices) g_static_busy[dev] = false;
}

// Autotuner results keyed by a signature of the batch (process-wide).
std::mutex g_tune_mu;
std::map<std::string, Tuning> g_tune_cache;

enum { kPassMoments = 0, kPassContact = 1, kPassTail = 2, kPassGather1 = 3, kPassStep2 = 4, kPassClosure = 5 };
const char *kPassNames[MLB_NPASS] = {"moments", "contact", "tail", "gather1", "step2", "closure"};

}  // namespace

namespace mlb {
mlb_status set_error(mlb_status st, const std::string &msg) { return fail(st, msg); }
}  // namespace mlb

// ---------------------------------------------------------------- the core
struct mlb_batch_s {
    int count = 0, prec = 32, maxM = 1, reach_max = 0, ball_reach_max = 0, ball_total_max = 1;
    bool tiled = false;
    std::vector<SysHost> sys;
    char *ws = nullptr;
    size_t total = 0;
    // shared regions
    size_t desc = 0, map_site = 0, map_tile = 0, map_g1 = 0, map_ident = 0;
    size_t t_sh_e = 0, t_sh_u = 0, t_tl_e = 0, t_tl_w = 0, t_bl_e = 0, t_sh_q = 0, t_sg_q = 0;
    size_t red = 0, red_out = 0, fit_out = 0;
    size_t desc_size = 0;
    int nblk_site = 0, nblk_tile = 0, nblk_g1 = 0, ident_len = 0;
    int map_tile_cap = 0, map_g1_cap = 0;
    Tuning tune;
    std::vector<unsigned char> desc_host;   // count stepping descriptors + 1 query descriptor
    int parity = 0;
    int64_t steps = 0;
    // per-pass timing
    bool profiling = false;
    std::vector<hipEvent_t> events;
    std::vector<std::pair<int, int>> marks;
    size_t next_event = 0;
    // graph of two steps (starting at parity 0)
    bool use_graph = true;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    // learned closure (single float32 binary system)
    mlb_net_s *net = nullptr;
    bool closure_active = false;   // the last check passed: steps until the next one take the network's force
    int check_every = 50;
    double closure_tol = 1e-2;
    int64_t closure_checks = 0, fallback_step = -1, failed_checks = 0, net_steps = 0;
    double last_err = -1.0;
    hipGraphExec_t graph_closure = nullptr;
    unsigned long long graph_closure_version = 0;   // net version the closure graph was captured with
    // second stream for the contact pass while the spectral field runs
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // device whose static workspace this handle holds (-1: caller's workspace)
    int static_dev = -1;

    virtual ~mlb_batch_s()
    {
        if (static_dev >= 0) release_static(static_dev);
        if (graph) (void)hipGraphExecDestroy(graph);
        if (graph_closure) (void)hipGraphExecDestroy(graph_closure);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (side) (void)hipStreamDestroy(side);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
    }
    template <typename T> mlb::SysDesc<T> *hdesc(int k) { return reinterpret_cast<mlb::SysDesc<T> *>(desc_host.data() + k * desc_size); }
    template <typename T> const mlb::SysDesc<T> *ddesc(int k) const { return reinterpret_cast<const mlb::SysDesc<T> *>(ws + desc + k * desc_size); }
    const int2 *map_of(size_t off) const { return reinterpret_cast<const int2 *>(ws + off); }
    template <typename T> mlb::Tables<T> tables() const
    {
        mlb::Tables<T> tb;
        tb.sh_e = reinterpret_cast<const int32_t *>(ws + t_sh_e);
        tb.sh_u = reinterpret_cast<const T *>(ws + t_sh_u);
        tb.tl_e = reinterpret_cast<const int32_t *>(ws + t_tl_e);
        tb.tl_w = reinterpret_cast<const T *>(ws + t_tl_w);
        tb.bl_e = reinterpret_cast<const int32_t *>(ws + t_bl_e);
        tb.sh_q = reinterpret_cast<const float4 *>(ws + t_sh_q);
        tb.sg_q = reinterpret_cast<const float4 *>(ws + t_sg_q);
        return tb;
    }
};

struct mlb_mixture_s : mlb_batch_s {};

namespace {

using Batch = mlb_batch_s;

size_t tsize_of(int prec) { return prec == 64 ? sizeof(double) : sizeof(float); }

// ---------------------------------------------------------------- layout
// Prepare every SysHost (tables, flags) and lay out the workspace.
bool plan_batch(Batch &B, const mlb_params *params, int count, std::string &why)
{
    if (count < 1) { why = "count must be >= 1"; return false; }
    B.count = count;
    B.prec = params[0].precision;
    B.sys.resize(count);
    B.maxM = 1;
    B.reach_max = 0;
    bool any_direct_tail = false;
    for (int k = 0; k < count; ++k) {
        if (!validate(&params[k], why)) { why = "system " + std::to_string(k) + ": " + why; return false; }
        if (params[k].precision != B.prec) { why = "all systems must share the precision"; return false; }
        SysHost &S = B.sys[k];
        S.p = params[k];
        if (!build_tables(&S.p, S.tabs, why)) { why = "system " + std::to_string(k) + ": " + why; return false; }
        S.M = S.p.nspecies;
        S.P = S.M * (S.M + 1) / 2;
        S.N = (long long)S.p.nx * S.p.ny * S.p.nz;
        S.nblocks = (int)((S.N + mlb::kBlock - 1) / mlb::kBlock);
        if (S.p.tail_mode == MLB_TAIL_SPECTRAL && has_tail(S.tabs) && !spectral_possible(&S.p, S.tabs, count)) {
            why = "the spectral tail needs float32, a single system and a (y, z) transform plane that fits LDS";
            return false;
        }
        S.spectral = wants_spectral(&S.p, S.tabs, count);
        any_direct_tail = any_direct_tail || (has_tail(S.tabs) && !S.spectral);
        B.maxM = std::max(B.maxM, S.M);
        B.reach_max = std::max(B.reach_max, S.tabs.shell_reach);
        B.ball_reach_max = std::max(B.ball_reach_max, S.tabs.ball_reach);
        B.ball_total_max = std::max(B.ball_total_max, (int)S.tabs.bl_e.size());
    }
    bool fits = true;
    for (int v = 0; v < mlb::kTileVariants; ++v)
        fits = fits && mlb::tile_lds_bytes_of(v, B.reach_max) <= 160 * 1024 &&
               mlb::contact_lds_bytes_of(v, B.ball_reach_max, B.ball_total_max, B.maxM) <= 160 * 1024;
    B.tiled = B.prec == 32 && !any_direct_tail && fits;
    const size_t ts = tsize_of(B.prec);
    // kernels index the descriptor array with the struct's own stride
    B.desc_size = B.prec == 64 ? sizeof(mlb::SysDesc<double>) : sizeof(mlb::SysDesc<float>);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + std::max<size_t>(bytes, 1)); return o; };
    B.desc = take((size_t)(count + 1) * B.desc_size);
    // maps
    B.nblk_site = 0;
    int max_tiles_any = 0, ident = 0, tiles_total_max = 0;
    for (auto &S : B.sys) {
        B.nblk_site += S.nblocks;
        ident = std::max(ident, S.nblocks);
    }
    int g1_tiles_total = 0;
    for (int v = 0; v < mlb::kG1Variants; ++v) {
        int tot = 0;
        for (auto &S : B.sys) {
            const int nt = mlb::tile_count(v, S.p.nx, S.p.ny, S.p.nz);
            tot += nt;
            max_tiles_any = std::max(max_tiles_any, nt);
        }
        if (v < mlb::kTileVariants) tiles_total_max = std::max(tiles_total_max, tot);
        else g1_tiles_total = tot;
    }
    B.ident_len = std::max(ident, max_tiles_any);
    B.map_tile_cap = (tiles_total_max + kXcds - 1) / kXcds * kXcds;
    B.map_g1_cap = (g1_tiles_total + kXcds - 1) / kXcds * kXcds;
    B.map_site = take(sizeof(int2) * (size_t)B.nblk_site);
    B.map_tile = take(sizeof(int2) * (size_t)B.map_tile_cap);
    B.map_g1 = take(sizeof(int2) * (size_t)B.map_g1_cap);
    B.map_ident = take(sizeof(int2) * (size_t)B.ident_len);
    // tables (concatenated)
    size_t nsh = 0, ntl = 0, nbl = 0, nsg = 0;
    for (auto &S : B.sys) {
        S.sh_base = (int)nsh; S.tl_base = (int)ntl; S.bl_base = (int)nbl; S.sg_base = (int)nsg;
        nsh += S.tabs.sh_e.size(); ntl += S.tabs.tl_e.size(); nbl += S.tabs.bl_e.size(); nsg += S.tabs.sg.size() / 4;
    }
    B.t_sh_e = take(4 * nsh);
    B.t_sh_u = take(ts * 3 * nsh);
    B.t_tl_e = take(4 * ntl);
    B.t_tl_w = take(ts * 3 * ntl);
    B.t_bl_e = take(4 * nbl);
    B.t_sh_q = take(16 * (nsh + mlb::kShellPad));
    B.t_sg_q = take(16 * (nsg + mlb::kShellPad));
    B.red = take(sizeof(double) * kRedParts * 16);
    B.red_out = take(sizeof(double) * 16);
    B.fit_out = take(sizeof(double) * kFitOut * (size_t)count);
    for (auto &S : B.sys) {
        const size_t M = (size_t)S.M, N = (size_t)S.N, P = (size_t)S.P;
        S.f0 = take(ts * M * mlb::kQ * N);
        S.f1 = take(ts * M * mlb::kQ * N);
        S.n = take(ts * M * N);
        S.j = take(ts * 3 * M * N);
        S.u = take(ts * 3 * N);
        S.g = take(ts * P * N);
        S.vh = take(ts * 3 * M * N);
        S.H = take(ts * 3 * M * N);
        S.Nf = take(ts * 3 * M * N);
        S.Tloc = B.tiled ? take(ts * 6 * M * N) : 0;
        if (S.spectral) {
            const size_t nyt = (size_t)spectral_ny(&S.p, S.tabs);
            const size_t nkx = (size_t)S.p.nx / 2 + 1, Sp = nkx * nyt * S.p.nz;
            const size_t fields = std::max(3 * M, 3 * P);
            S.wxf = take(sizeof(float) * S.p.nx * 2 * nkx);
            S.wxi = take(sizeof(float) * 2 * nkx * S.p.nx);
            S.wyf = take(sizeof(float) * 4 * nyt * nyt);
            S.wyi = take(sizeof(float) * 4 * nyt * nyt);
            S.wzf = take(sizeof(float) * 4 * S.p.nz * S.p.nz);
            S.wzi = take(sizeof(float) * 4 * S.p.nz * S.p.nz);
            S.S = take(sizeof(float) * 3 * P * Sp);
            S.s1 = take(sizeof(float) * 2 * fields * Sp);
            S.s2 = take(sizeof(float) * 2 * fields * Sp);
            S.tail = take(sizeof(float) * 3 * M * N);
            S.gfac = take(sizeof(float) * M * N);
        }
        S.series = take(sizeof(double) * 2 * kSeriesCap);
        S.series_cnt = take(sizeof(int));
        S.fprof = take(ts * 3 * M * (size_t)S.p.ny);
    }
    B.total = off;
    return true;
}

template <typename T>
void fill_desc(Batch &B, int k, mlb::SysDesc<T> &D)
{
    SysHost &S = B.sys[k];
    const mlb_params *p = &S.p;
    std::memset(&D, 0, sizeof(D));
    D.nx = p->nx; D.ny = p->ny; D.nz = p->nz; D.M = S.M; D.P = S.P; D.walls = p->walls_y ? 1 : 0;
    D.N = S.N;
    D.nblocks = S.nblocks;
    D.reach = S.tabs.shell_reach;
    D.ball_reach = S.tabs.ball_reach;
    D.ball_total = (int)S.tabs.bl_e.size();
    char *ws = B.ws;
    D.f[0] = reinterpret_cast<T *>(ws + S.f0);
    D.f[1] = reinterpret_cast<T *>(ws + S.f1);
    D.n = reinterpret_cast<T *>(ws + S.n);
    D.j = reinterpret_cast<T *>(ws + S.j);
    D.u = reinterpret_cast<T *>(ws + S.u);
    D.g = reinterpret_cast<T *>(ws + S.g);
    D.vh = reinterpret_cast<T *>(ws + S.vh);
    D.H = reinterpret_cast<T *>(ws + S.H);
    D.Nf = reinterpret_cast<T *>(ws + S.Nf);
    D.Tloc = B.tiled ? reinterpret_cast<T *>(ws + S.Tloc) : nullptr;
    D.tail = S.spectral ? reinterpret_cast<T *>(ws + S.tail) : nullptr;
    // tiled float32: the spectral field runs beside contact values and the first gather
    D.tail_deferred = (S.spectral && B.tiled) ? 1 : 0;
    D.gfac = D.tail_deferred ? reinterpret_cast<T *>(ws + S.gfac) : nullptr;
    D.parts = nullptr;
    D.parts_mask = 0;
    D.fprof = S.has_profile ? reinterpret_cast<const T *>(ws + S.fprof) : nullptr;
    D.tail_direct = S.spectral ? 0 : 1;
    D.scheme = p->scheme;
    D.omega_is_one = (1.0 / p->tau == 1.0) ? 1 : 0;
    const HostTables &t = S.tabs;
    D.unit_mass = 1;
    for (int a = 0; a < S.M; ++a) {
        const double ma = p->mass[a];
        D.unit_mass = D.unit_mass && ma == 1.0;
        D.mass[a] = (T)ma;
        D.im[a] = (T)(1.0 / ma);
        D.ith[a] = (T)(ma / p->kT);
        D.dth[a] = (T)(4.5 * (p->kT / ma - 1.0 / 3.0));
    }
    for (int a = 0; a < S.M; ++a) {
        D.bl_start[a] = S.bl_base + t.bl_start[a]; D.bl_cnt[a] = t.bl_cnt[a]; D.bl_full[a] = t.bl_full[a];
        const double sg = p->sigma[a];
        D.s2[a] = (T)((M_PI / 6.0) * (sg * sg));
        D.s3[a] = (T)((M_PI / 6.0) * ((sg * sg) * sg));
        for (int d = 0; d < 3; ++d) D.fext[a][d] = (T)p->ext_force[a * 3 + d];
        for (int b = 0; b < S.M; ++b) {
            D.sh_start[a][b] = S.sh_base + t.sh_start[a][b]; D.sh_cnt[a][b] = t.sh_cnt[a][b];
            for (int kd = 0; kd < mlb::kGroupKinds; ++kd) {
                D.sg_start[a][b][kd] = S.sg_base + t.sg_start[a][b][kd];
                D.sg_cnt[a][b][kd] = t.sg_cnt[a][b][kd];
            }
            D.tl_start[a][b] = S.tl_base + t.tl_start[a][b]; D.tl_cnt[a][b] = t.tl_cnt[a][b];
            const mlb::PairConst c =
                mlb::pair_constants(p->sigma[a], p->sigma[b], p->kT, t.sh_full[a][b], p->mass[a], p->mass[b]);
            D.cm[a][b] = (T)c.cm; D.cg[a][b] = (T)c.cg; D.ck[a][b] = (T)c.ck; D.dd[a][b] = (T)c.dd;
        }
    }
    const double omega = 1.0 / p->tau;
    D.omega = (T)omega;
    D.om1 = (T)(1.0 - omega);
    D.wall_ux[0] = (T)p->wall_ux[0];
    D.wall_ux[1] = (T)p->wall_ux[1];
}

// Tile map for tile shape v: logical tiles (system-major, z-slab order)
// dealt to physical blocks.  order 1 gives XCD x the contiguous chunk
// [x C, (x+1) C) of logical tiles (block b runs on XCD b mod 8), so tiles
// that share halos share an L2; padding blocks idle.
std::vector<int2> tile_map(const Batch &B, int v, int order, int &nblk)
{
    std::vector<int2> logical;
    for (int k = 0; k < B.count; ++k) {
        const SysHost &S = B.sys[k];
        const int nt = mlb::tile_count(v, S.p.nx, S.p.ny, S.p.nz);
        for (int i = 0; i < nt; ++i) logical.push_back(make_int2(k, i));
    }
    const int T = (int)logical.size();
    if (order == 0) {
        nblk = T;
        return logical;
    }
    const int chunk = (T + kXcds - 1) / kXcds;
    nblk = chunk * kXcds;
    std::vector<int2> phys((size_t)nblk, make_int2(-1, 0));
    for (int b = 0; b < nblk; ++b) {
        const int L = (b % kXcds) * chunk + b / kXcds;
        if (L < T) phys[(size_t)b] = logical[(size_t)L];
    }
    return phys;
}

template <typename T>
mlb_status upload_static(Batch &B, hipStream_t st)
{
    // concatenated tables
    std::vector<int32_t> sh_e, tl_e, bl_e;
    std::vector<T> sh_u, tl_w;
    for (auto &S : B.sys) {
        sh_e.insert(sh_e.end(), S.tabs.sh_e.begin(), S.tabs.sh_e.end());
        tl_e.insert(tl_e.end(), S.tabs.tl_e.begin(), S.tabs.tl_e.end());
        bl_e.insert(bl_e.end(), S.tabs.bl_e.begin(), S.tabs.bl_e.end());
        for (double v : S.tabs.sh_u) sh_u.push_back((T)v);
        for (double v : S.tabs.tl_w) tl_w.push_back((T)v);
    }
    char *ws = B.ws;
    auto up = [&](size_t off, const void *src, size_t bytes) -> mlb_status {
        if (bytes) HIP_TRY(hipMemcpyAsync(ws + off, src, bytes, hipMemcpyHostToDevice, st));
        return MLB_OK;
    };
    TRY(up(B.t_sh_e, sh_e.data(), 4 * sh_e.size()));
    TRY(up(B.t_sh_u, sh_u.data(), sizeof(T) * sh_u.size()));
    TRY(up(B.t_tl_e, tl_e.data(), 4 * tl_e.size()));
    TRY(up(B.t_tl_w, tl_w.data(), sizeof(T) * tl_w.size()));
    TRY(up(B.t_bl_e, bl_e.data(), 4 * bl_e.size()));
    std::vector<float4> sh_q(sh_e.size() + mlb::kShellPad, make_float4(0.f, 0.f, 0.f, 0.f));
    for (size_t k = 0; k < sh_e.size(); ++k) {
        float bits;
        std::memcpy(&bits, &sh_e[k], 4);
        sh_q[k] = make_float4(bits, (float)sh_u[3 * k], (float)sh_u[3 * k + 1], (float)sh_u[3 * k + 2]);
    }
    TRY(up(B.t_sh_q, sh_q.data(), sizeof(float4) * sh_q.size()));
    std::vector<float> sg;
    for (auto &S : B.sys) sg.insert(sg.end(), S.tabs.sg.begin(), S.tabs.sg.end());
    sg.resize(sg.size() + 4 * mlb::kShellPad, 0.f);
    TRY(up(B.t_sg_q, sg.data(), sizeof(float) * sg.size()));
    // per-site block map and the identity map used by single-system launches
    std::vector<int2> site, ident((size_t)B.ident_len);
    for (int k = 0; k < B.count; ++k)
        for (int i = 0; i < B.sys[k].nblocks; ++i) site.push_back(make_int2(k, i));
    for (int i = 0; i < B.ident_len; ++i) ident[(size_t)i] = make_int2(0, i);
    TRY(up(B.map_site, site.data(), sizeof(int2) * site.size()));
    TRY(up(B.map_ident, ident.data(), sizeof(int2) * ident.size()));
    // descriptors
    B.desc_host.assign((size_t)(B.count + 1) * B.desc_size, 0);
    for (int k = 0; k < B.count; ++k) fill_desc<T>(B, k, *B.hdesc<T>(k));
    TRY(up(B.desc, B.desc_host.data(), (size_t)B.count * B.desc_size));
    HIP_TRY(hipStreamSynchronize(st));   // host staging vectors die here
    return MLB_OK;
}

// g1shape: the first gather's tile shape (`shape`, or kG1Own with its own
// block map in the same order)
mlb_status set_tiling(Batch &B, int shape, int order, int g1split, bool groups, int g1shape, hipStream_t st)
{
    int nblk = 0, ng1 = 0;
    std::vector<int2> m = tile_map(B, shape, order, nblk);
    if (nblk > B.map_tile_cap) return fail(MLB_EINVAL, "tile map overflow");
    HIP_TRY(hipMemcpyAsync(B.ws + B.map_tile, m.data(), sizeof(int2) * m.size(), hipMemcpyHostToDevice, st));
    std::vector<int2> m1;
    if (g1shape != shape) {
        m1 = tile_map(B, g1shape, order, ng1);
        if (ng1 > B.map_g1_cap) return fail(MLB_EINVAL, "tile map overflow");
        HIP_TRY(hipMemcpyAsync(B.ws + B.map_g1, m1.data(), sizeof(int2) * m1.size(), hipMemcpyHostToDevice, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    B.nblk_tile = nblk;
    B.nblk_g1 = g1shape != shape ? ng1 : nblk;
    B.tune.shape = shape;
    B.tune.order = order;
    B.tune.g1split = g1split;
    B.tune.groups = groups;
    B.tune.g1shape = g1shape;
    if (B.graph) {
        (void)hipGraphExecDestroy(B.graph);
        B.graph = nullptr;
    }
    return MLB_OK;
}

// Upload the DFT matrices, place the tail kernels on the periodic grid
// (population buffer f1 is scratch; the first step overwrites it) and
// transform them into the sine spectra.
mlb_status setup_spectral(Batch &B, SysHost &S, hipStream_t st)
{
    const mlb_params *p = &S.p;
    mlb::SpectralPlan &pl = S.plan;
    char *ws = B.ws;
    const int nyt = spectral_ny(p, S.tabs);
    pl.nx = p->nx; pl.ny = nyt; pl.nyr = p->ny; pl.nz = p->nz; pl.nkx = p->nx / 2 + 1;
    pl.M = S.M; pl.P = S.P;
    pl.Sz = (long long)pl.ny * pl.nkx;
    pl.Sp = pl.Sz * pl.nz;
    pl.wxf = reinterpret_cast<const float *>(ws + S.wxf);
    pl.wxi = reinterpret_cast<const float *>(ws + S.wxi);
    pl.wyf = reinterpret_cast<const float *>(ws + S.wyf);
    pl.wyi = reinterpret_cast<const float *>(ws + S.wyi);
    pl.wzf = reinterpret_cast<const float *>(ws + S.wzf);
    pl.wzi = reinterpret_cast<const float *>(ws + S.wzi);
    pl.S = reinterpret_cast<float *>(ws + S.S);
    std::vector<float> m[6] = {mlb::SpectralPlan::dft_x_forward(p->nx), mlb::SpectralPlan::dft_x_inverse(p->nx),
                               mlb::SpectralPlan::dft_block(nyt, false), mlb::SpectralPlan::dft_block(nyt, true),
                               mlb::SpectralPlan::dft_block(p->nz, false), mlb::SpectralPlan::dft_block(p->nz, true)};
    if (!mlb::SpectralPlan::prepare(nyt, p->nz, S.M)) return fail(MLB_EHIP, "cannot raise the LDS limit of the tail kernel");
    const size_t offs[6] = {S.wxf, S.wxi, S.wyf, S.wyi, S.wzf, S.wzi};
    for (int k = 0; k < 6; ++k)
        HIP_TRY(hipMemcpyAsync(ws + offs[k], m[k].data(), sizeof(float) * m[k].size(), hipMemcpyHostToDevice, st));
    // the kernels w_ab placed on the transform grid (nx x nyt x nz), offsets
    // wrapped on it; the placed fields are staged in the second population
    // buffer, not yet in use
    const long long N = (long long)p->nx * nyt * p->nz;
    if ((size_t)3 * S.P * N > (size_t)mlb::kQ * S.M * S.N) return fail(MLB_EINVAL, "padded tail transform too large");
    std::vector<float> placed((size_t)3 * S.P * N, 0.0f);
    std::vector<double> acc((size_t)3 * N);
    const HostTables &t = S.tabs;
    for (int a = 0; a < S.M; ++a)
        for (int b = a; b < S.M; ++b) {
            const int pi = a * S.M - (a * (a - 1)) / 2 + (b - a);
            std::fill(acc.begin(), acc.end(), 0.0);
            for (int k = 0; k < t.tl_cnt[a][b]; ++k) {
                int ex, ey, ez;
                mlb::unpack_offset(t.tl_e[t.tl_start[a][b] + k], ex, ey, ez);
                for (int sgn = -1; sgn <= 1; sgn += 2) {
                    const int x = ((sgn * ex) % p->nx + p->nx) % p->nx;
                    const int y = ((sgn * ey) % nyt + nyt) % nyt;
                    const int z = ((sgn * ez) % p->nz + p->nz) % p->nz;
                    const long long site = ((long long)z * nyt + y) * p->nx + x;
                    for (int d = 0; d < 3; ++d) acc[(size_t)d * N + site] += sgn * t.tl_w[3 * (t.tl_start[a][b] + k) + d];
                }
            }
            for (int d = 0; d < 3; ++d)
                for (long long i = 0; i < N; ++i) placed[((size_t)pi * 3 + d) * N + i] = (float)acc[(size_t)d * N + i];
        }
    float *scratch = reinterpret_cast<float *>(ws + S.f1);
    HIP_TRY(hipMemcpyAsync(scratch, placed.data(), sizeof(float) * placed.size(), hipMemcpyHostToDevice, st));
    pl.build_spectrum(scratch, reinterpret_cast<float *>(ws + S.s1), reinterpret_cast<float *>(ws + S.s2), st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return MLB_OK;
}

// ------------------------------------------------------------------ passes
hipEvent_t take_event(Batch &B)
{
    if (B.next_event == B.events.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        B.events.push_back(e);
    }
    return B.events[B.next_event++];
}

template <typename F>
void pass(Batch &B, int id, hipStream_t st, F &&launch)
{
    if (!B.profiling) {
        launch();
        return;
    }
    const size_t k = B.next_event;
    hipEvent_t a = take_event(B), b = take_event(B);
    if (!a || !b) {
        launch();
        return;
    }
    (void)hipEventRecord(a, st);
    launch();
    (void)hipEventRecord(b, st);
    B.marks.emplace_back(id, (int)k);
}

void run_tail(Batch &B, SysHost &S, hipStream_t st)
{
    char *ws = B.ws;
    S.plan.apply(reinterpret_cast<const float *>(ws + S.n), reinterpret_cast<float *>(ws + S.s1),
                 reinterpret_cast<float *>(ws + S.s2), reinterpret_cast<float *>(ws + S.tail), st);
}

// One step over all systems (query == false) or the force evaluation of
// system `qk` through the query descriptor (query == true).
template <typename T>
void run_passes(Batch &B, hipStream_t st, bool query, int qk, int force_only)
{
    const mlb::SysDesc<T> *sys = query ? B.ddesc<T>(B.count) : B.ddesc<T>(0);
    const mlb::Tables<T> tb = B.tables<T>();
    const int par = B.parity;
    const int2 *smap = query ? B.map_of(B.map_ident) : B.map_of(B.map_site);
    const int nsite = query ? B.sys[qk].nblocks : B.nblk_site;
    const int M = query ? B.sys[qk].M : B.maxM;
    // float32 LDS tiles: contact values and both gathers share the tile map
    bool tiled = false;
    int shape = 0, ntl = 0, g1shape = 0, ng1 = 0;
    const int2 *tmap = nullptr, *g1map = nullptr;
    if constexpr (std::is_same<T, float>::value) {
        if (B.tiled) {
            tiled = true;
            shape = B.tune.shape;
            g1shape = B.tune.g1shape;
            tmap = query ? B.map_of(B.map_ident) : B.map_of(B.map_tile);
            ntl = query ? mlb::tile_count(shape, B.sys[qk].p.nx, B.sys[qk].p.ny, B.sys[qk].p.nz) : B.nblk_tile;
            g1map = query ? tmap : B.map_of(g1shape != shape ? B.map_g1 : B.map_tile);
            ng1 = query ? mlb::tile_count(g1shape, B.sys[qk].p.nx, B.sys[qk].p.ny, B.sys[qk].p.nz) : B.nblk_g1;
        }
    }
    auto contact = [&](hipStream_t s) {
        if constexpr (std::is_same<T, float>::value) {
            if (tiled) {
                pass(B, kPassContact, s, [&] {
                    mlb::launch_contact_tile(shape, sys, tmap, ntl, tb, B.ball_reach_max, B.ball_total_max, B.maxM, s);
                });
                return;
            }
        }
        pass(B, kPassContact, s, [&] { mlb::Launch<T>::contact(sys, smap, nsite, tb, s); });
    };
    auto gathers = [&] {
        if constexpr (std::is_same<T, float>::value) {
            if (tiled) {
                pass(B, kPassGather1, st,
                     [&] {
                         mlb::launch_gather1_tile(g1shape, B.tune.g1split, B.tune.groups, sys, g1map, ng1, M, tb,
                                                  B.reach_max, st);
                     });
                return;
            }
        }
        pass(B, kPassGather1, st, [&] { mlb::Launch<T>::gather1(sys, smap, nsite, M, tb, st); });
    };
    auto second = [&] {
        if constexpr (std::is_same<T, float>::value) {
            if (tiled) {
                pass(B, kPassStep2, st, [&] {
                    mlb::launch_step2_tile(shape, sys, tmap, ntl, M, tb, B.reach_max, par, force_only, st);
                });
                return;
            }
        }
        pass(B, kPassStep2, st, [&] { mlb::Launch<T>::step2(sys, smap, nsite, M, tb, par, force_only, st); });
    };
    auto tails = [&](hipStream_t s) {
        for (int k = 0; k < B.count; ++k)
            if ((!query || k == qk) && B.sys[k].spectral) pass(B, kPassTail, s, [&] { run_tail(B, B.sys[k], s); });
    };

    pass(B, kPassMoments, st, [&] { mlb::Launch<T>::moments(sys, smap, nsite, par, st); });
    bool spectral = false;
    for (int k = 0; k < B.count; ++k) spectral = spectral || ((!query || k == qk) && B.sys[k].spectral);
    // per-pass timing wants each pass alone on the GPU: no side stream then
    const bool overlap = B.side && !B.profiling;
    if (spectral && tiled && !overlap) {
        tails(st);
        contact(st);
        gathers();
        pass(B, kPassTail, st, [&] { mlb::Launch<T>::add_tail(sys, smap, nsite, M, st); });
        second();
        return;
    }
    if (spectral && tiled) {
        // the spectral field needs only the densities and enters through H and
        // V-hat: it runs on the side stream beside contact values and the first
        // gather, and k_add_tail folds it in before the second gather
        (void)hipEventRecord(B.ev_fork, st);
        (void)hipStreamWaitEvent(B.side, B.ev_fork, 0);
        tails(B.side);
        (void)hipEventRecord(B.ev_join, B.side);
        contact(st);
        gathers();
        (void)hipStreamWaitEvent(st, B.ev_join, 0);
        pass(B, kPassTail, st, [&] { mlb::Launch<T>::add_tail(sys, smap, nsite, M, st); });
        second();
        return;
    }
    if (spectral && overlap) {
        // contact values and the spectral field both need only the moments
        (void)hipEventRecord(B.ev_fork, st);
        (void)hipStreamWaitEvent(B.side, B.ev_fork, 0);
        contact(B.side);
        (void)hipEventRecord(B.ev_join, B.side);
        tails(st);
        (void)hipStreamWaitEvent(st, B.ev_join, 0);
    } else {
        contact(st);
        tails(st);
    }
    gathers();
    second();
}

void step_once(Batch &B, hipStream_t st)
{
    if (B.prec == 64) run_passes<double>(B, st, false, 0, 0);
    else run_passes<float>(B, st, false, 0, 0);
    B.parity ^= 1;
    B.steps += 1;
}

// A step with the closure's force: moments, network, collision + streaming.
// With `check` the exact force is evaluated as well and used instead, and
// the squared-error partials of the network's force land in the net.
void closure_step(Batch &B, hipStream_t st, bool check)
{
    using T = float;
    const mlb::SysDesc<T> *sys = B.ddesc<T>(0);
    const int2 *smap = B.map_of(B.map_site);
    SysHost &S = B.sys[0];
    const int par = B.parity;
    T *n = reinterpret_cast<T *>(B.ws + S.n), *j = reinterpret_cast<T *>(B.ws + S.j);
    T *Nf = reinterpret_cast<T *>(B.ws + S.Nf);
    if (!check) {
        pass(B, kPassMoments, st, [&] { mlb::Launch<T>::moments(sys, smap, B.nblk_site, par, st); });
        pass(B, kPassClosure, st, [&] { mlb::net_infer_fields(B.net, n, j, Nf, st); });
    } else {
        run_passes<T>(B, st, false, 0, 1);   // exact force into Nf, populations untouched
        T *Nc = mlb::net_check_buffer(B.net);
        pass(B, kPassClosure, st, [&] { mlb::net_infer_fields(B.net, n, j, Nc, st); });
        int nparts = 0;
        double *part = mlb::net_err_buffer(B.net, &nparts);
        mlb::cnn_err_partial(3 * S.M * S.N, Nc, Nf, part, nparts, st);
    }
    pass(B, kPassStep2, st, [&] { mlb::launch_collide_f32(sys, smap, B.nblk_site, B.maxM, par, st); });
    B.parity ^= 1;
    B.steps += 1;
}

mlb_status capture_pair(Batch &B, hipGraphExec_t *out, void (*one)(Batch &, hipStream_t))
{
    if (!B.cap_stream) HIP_TRY(hipStreamCreateWithFlags(&B.cap_stream, hipStreamNonBlocking));
    const int par0 = B.parity;
    const int64_t steps0 = B.steps;
    B.parity = 0;
    HIP_TRY(hipStreamBeginCapture(B.cap_stream, hipStreamCaptureModeRelaxed));
    one(B, B.cap_stream);
    one(B, B.cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(B.cap_stream, &g);
    B.parity = par0;
    B.steps = steps0;
    if (e != hipSuccess) return fail(MLB_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        *out = nullptr;
        return fail(MLB_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    return MLB_OK;
}

void plain_step(Batch &B, hipStream_t st) { step_once(B, st); }
void net_step(Batch &B, hipStream_t st) { closure_step(B, st, false); }

// `nsteps` steps of one kind: pairs replay the captured graph of that kind
// (which starts at parity 0), the rest launch eagerly.
mlb_status run_steps(Batch &B, int nsteps, hipStream_t st, bool with_net)
{
    hipGraphExec_t &graph = with_net ? B.graph_closure : B.graph;
    void (*one)(Batch &, hipStream_t) = with_net ? net_step : plain_step;
    // the network's scales are kernel arguments of the captured inference:
    // a graph captured before they changed would replay the old ones
    if (with_net && graph && B.graph_closure_version != mlb::net_version(B.net)) {
        (void)hipGraphExecDestroy(graph);
        graph = nullptr;
    }
    int left = nsteps;
    if (B.use_graph && !B.profiling && left >= 2) {
        if (B.parity == 1) {
            one(B, st);
            --left;
        }
        if (left >= 2) {
            if (!graph) {
                TRY(capture_pair(B, &graph, one));
                if (with_net) B.graph_closure_version = mlb::net_version(B.net);
            }
            while (left >= 2) {
                HIP_TRY(hipGraphLaunch(graph, st));
                B.steps += 2;
                left -= 2;
            }
        }
    }
    while (left-- > 0) one(B, st);
    HIP_TRY(hipGetLastError());
    return MLB_OK;
}

// exact-force check step; switches the closure off when the error is above tolerance
mlb_status check_closure(Batch &B, hipStream_t st)
{
    const int64_t at_step = B.steps;
    closure_step(B, st, true);
    HIP_TRY(hipGetLastError());
    int nparts = 0;
    const double *part = mlb::net_err_buffer(B.net, &nparts);
    std::vector<double> h(2 * (size_t)nparts);
    HIP_TRY(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double e = 0.0, w = 0.0;
    for (int k = 0; k < nparts; ++k) {
        e += h[2 * k];
        w += h[2 * k + 1];
    }
    // a non-finite sum (diverged state or network output) counts as a failed check
    double err = NAN;
    if (std::isfinite(e) && std::isfinite(w)) err = w > 0.0 ? std::sqrt(e / w) : (e > 0.0 ? INFINITY : 0.0);
    B.last_err = err;
    B.closure_checks += 1;
    B.closure_active = err <= B.closure_tol;
    if (!B.closure_active) {
        B.failed_checks += 1;
        if (B.fallback_step < 0) B.fallback_step = at_step;
    }
    return MLB_OK;
}

mlb_status do_steps(Batch &B, int nsteps, hipStream_t st)
{
    if (nsteps < 0) return fail(MLB_EINVAL, "nsteps must be >= 0");
    int left = nsteps;
    // with a network attached: every step whose index is a multiple of
    // check_every is a check; the steps up to the next check take the
    // network's force if that check passed, the exact force if it failed
    while (left > 0 && B.net) {
        const int64_t phase = B.steps % B.check_every;
        if (phase == 0) {
            TRY(check_closure(B, st));
            --left;
            continue;
        }
        const int run = (int)std::min<int64_t>(left, B.check_every - phase);
        TRY(run_steps(B, run, st, B.closure_active));
        if (B.closure_active) B.net_steps += run;
        left -= run;
    }
    return run_steps(B, left, st, false);
}

template <typename T>
mlb_status run_query(Batch &B, int k, T *parts, unsigned mask, hipStream_t st)
{
    mlb::SysDesc<T> *q = B.hdesc<T>(B.count);
    *q = *B.hdesc<T>(k);
    q->parts = parts;
    q->parts_mask = mask;
    HIP_TRY(hipMemcpyAsync(B.ws + B.desc + (size_t)B.count * B.desc_size, q, B.desc_size, hipMemcpyHostToDevice, st));
    run_passes<T>(B, st, true, k, 1);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    return MLB_OK;
}

template <typename T>
mlb_status init_populations(Batch &B, const double *const *n0, const double *const *u0, hipStream_t st)
{
    for (int k = 0; k < B.count; ++k) {
        // query descriptor slot + identity map: one system per launch
        mlb::SysDesc<T> *q = B.hdesc<T>(B.count);
        *q = *B.hdesc<T>(k);
        HIP_TRY(hipMemcpyAsync(B.ws + B.desc + (size_t)B.count * B.desc_size, q, B.desc_size, hipMemcpyHostToDevice,
                               st));
        mlb::Launch<T>::init_pop(B.ddesc<T>(B.count), B.map_of(B.map_ident), B.sys[k].nblocks, n0[k], u0[k], st);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(st));
    }
    B.parity = 0;
    B.steps = 0;
    return MLB_OK;
}

std::string tune_key(const Batch &B)
{
    std::string k = std::to_string(B.prec) + ":" + std::to_string(B.count);
    for (const auto &S : B.sys) {
        k += "|" + std::to_string(S.p.nx) + "x" + std::to_string(S.p.ny) + "x" + std::to_string(S.p.nz) + ":" +
             std::to_string(S.M) + ":" + std::to_string(S.tabs.shell_reach) + ":" + std::to_string(S.tabs.sh_e.size());
    }
    return k;
}

// Time every tile shape and block order over full steps, run the way
// mlb_step runs them (graph-replayed pairs unless graphs are off: the
// spectral field's overlap with the first gather differs between the two);
// keep the fastest.
template <typename T>
mlb_status autotune(Batch &B, const double *const *n0, const double *const *u0, hipStream_t st)
{
    const std::string key = tune_key(B);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            const Tuning cached = it->second;
            TRY(set_tiling(B, cached.shape, cached.order, cached.g1split, cached.groups, cached.g1shape, st));
            B.tune = cached;
            return MLB_OK;
        }
    }
    Tuning best;
    double best_ms = 1e300;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    mlb_status status = MLB_OK;
    // ms per step of `steps` graph-replayed steps (< 0 on failure)
    auto timed = [&](int steps) -> double {
        float ms = 0.f;
        if (hipEventRecord(e0, st) != hipSuccess) { status = fail(MLB_EHIP, "event record"); return -1.0; }
        status = run_steps(B, steps, st, false);
        if (status != MLB_OK) return -1.0;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            status = fail(MLB_EHIP, "event timing");
            return -1.0;
        }
        return ms / steps;
    };
    // one tiling: two warm-up steps (they capture its graph), then at least
    // six timed steps and at least min_ms of GPU time in one timed run
    auto trial = [&](int v, int order, int split, bool groups, int g1v, double min_ms) -> double {
        status = set_tiling(B, v, order, split, groups, g1v, st);
        if (status != MLB_OK) return -1.0;
        status = run_steps(B, 2, st, false);
        if (status != MLB_OK) return -1.0;
        const double per = timed(6);
        if (status != MLB_OK || 6 * per >= min_ms) return per;
        const int reps = 2 * std::min(200, (int)std::ceil(min_ms / per / 2.0));
        return timed(reps);
    };
    // the clocks settle on the first tiling before anything is timed
    (void)trial(0, 0, 2, false, 0, 10.0);
    for (int split = 2; split < 2 + kSplitChoices && status == MLB_OK; ++split)
    for (int v = 0; v < mlb::kTileVariants && status == MLB_OK; ++v)
        for (int order = 0; order < 2 && status == MLB_OK; ++order) {
            const double per = trial(v, order, split, false, v, 5.0);
            if (status != MLB_OK) break;
            best.trial_ms[(split - 2) * 2 * mlb::kTileVariants + 2 * v + order] = per;
        }
    // final round, timed longer: the two fastest tilings with the plain and
    // the sign-grouped shell loop, each with the first gather on the
    // tiling's shape and on its own 4x8x8 tiles
    const bool own_fits = mlb::gather1_lds_bytes_of(kG1Own, B.reach_max) <= 160 * 1024;
    if (status == MLB_OK) {
        int idx[kTrials];
        for (int k = 0; k < kTrials; ++k) idx[k] = k;
        std::sort(idx, idx + kTrials, [&](int x, int y) { return best.trial_ms[x] < best.trial_ms[y]; });
        for (int c = 0; c < 2 && status == MLB_OK; ++c) {
            const int k = idx[c];
            const int split = 2 + k / (2 * mlb::kTileVariants), v = (k / 2) % mlb::kTileVariants, order = k % 2;
            double grouped_ms = 0.0;
            bool chosen = false;
            for (int g1 = 0; g1 < (own_fits ? 2 : 1) && status == MLB_OK; ++g1)
                for (int groups = 0; groups < 2 && status == MLB_OK; ++groups) {
                    const int g1v = g1 ? kG1Own : v;
                    const double per = trial(v, order, split, groups != 0, g1v, 30.0);
                    if (status != MLB_OK) break;
                    if (groups && g1 == 0) grouped_ms = per;
                    if (per < best_ms) {
                        best_ms = per;
                        best.shape = v;
                        best.order = order;
                        best.g1split = split;
                        best.groups = groups != 0;
                        best.g1shape = g1v;
                        chosen = true;
                    }
                }
            // the sign-grouped time reported is that of the chosen tiling
            if (chosen) best.groups_ms = grouped_ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (status != MLB_OK) return status;
    TRY(set_tiling(B, best.shape, best.order, best.g1split, best.groups, best.g1shape, st));
    B.tune = best;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
    }
    return init_populations<T>(B, n0, u0, st);   // the trial steps changed the state
}

mlb_status moments_of(Batch &B, int k, void *n_out, void *j_out, hipStream_t st);

// Spectral radii already evaluated, keyed by the parameter block and the
// densities (tests and ensembles create the same states many times).
std::mutex g_stab_mu;
std::map<std::string, double> g_stab_cache;

double cached_radius(const mlb_params *p, const double *n)
{
    std::string key(reinterpret_cast<const char *>(p), sizeof(mlb_params));
    key.append(reinterpret_cast<const char *>(n), sizeof(double) * (size_t)p->nspecies);
    {
        std::lock_guard<std::mutex> lk(g_stab_mu);
        auto it = g_stab_cache.find(key);
        if (it != g_stab_cache.end()) return it->second;
    }
    const double rho = mlb::stability_radius(p, n, 8);
    std::lock_guard<std::mutex> lk(g_stab_mu);
    g_stab_cache[key] = rho;
    return rho;
}

// The linear-stability guard at every system's box-mean densities (species
// masses from the float64 sums over the fluid sites).
mlb_status check_mean_states(Batch &B, hipStream_t st)
{
    for (int k = 0; k < B.count; ++k) {
        SysHost &S = B.sys[k];
        TRY(moments_of(B, k, nullptr, nullptr, st));
        double *out = reinterpret_cast<double *>(B.ws + B.red_out);
        mlb::launch_conserved(B.ws + S.n, B.ws + S.j, B.prec, S.M, S.N, reinterpret_cast<double *>(B.ws + B.red),
                              kRedParts, out, st);
        double host[16];
        HIP_TRY(hipMemcpyAsync(host, out, sizeof(double) * 4 * S.M, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        const double fluid = (double)S.p.nx * S.p.nz * (S.p.walls_y ? S.p.ny - 2 : S.p.ny);
        double nb[MLB_MAX_SPECIES];
        for (int a = 0; a < S.M; ++a) nb[a] = host[a] / fluid;
        const double rho = cached_radius(&S.p, nb);
        if (!(rho <= 1.0 + 1e-6))
            return fail(MLB_EUNSTABLE, "system " + std::to_string(k) + ": the scheme is linearly unstable at the box-mean " +
                                           "densities (spectral radius " + std::to_string(rho) + "); use the " +
                                           "Crank-Nicolson scheme, or MLB_OPT_NO_STABILITY_CHECK to run anyway");
    }
    return MLB_OK;
}

// no_alloc: no graph replay and no second stream (both allocate), no autotuning.
template <typename T>
mlb_status create(Batch &B, const mlb_params *params, int count, void *workspace, size_t bytes,
                  const double *const *n0, const double *const *u0, uint32_t options, hipStream_t st,
                  bool no_alloc = false)
{
    std::string why;
    // the fixed-tiling option fields, checked before any device work
    const int fixed_shape = (int)((options >> 4) & 15u) - 1, fixed_order = (int)((options >> 8) & 1u);
    const int fixed_split = (int)((options >> 10) & 3u);
    const int fixed_groups = (int)((options >> 12) & 3u);
    const int fixed_g1 = (int)((options >> 14) & 3u);
    if (fixed_shape >= mlb::kTileVariants) return fail(MLB_EINVAL, "MLB_OPT_TILING: no such tile shape");
    if (fixed_split == 1) return fail(MLB_EINVAL, "MLB_OPT_GATHER1_SPLIT: 2 or 3 thread groups per site");
    if (fixed_groups == 3) return fail(MLB_EINVAL, "MLB_OPT_GATHER1_SIGN_GROUPS: 0 or 1");
    if (fixed_g1 == 3) return fail(MLB_EINVAL, "MLB_OPT_GATHER1_OWN_TILES: 0 or 1");
    if (!plan_batch(B, params, count, why)) return fail(MLB_EINVAL, why);
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0)
        return fail(MLB_EINVAL, "workspace must be a 256-byte aligned device pointer");
    if (bytes < B.total) return fail(MLB_ENOMEM, "workspace too small: need " + std::to_string(B.total) + " bytes");
    if (!n0 || !u0) return fail(MLB_EINVAL, "n0 and u0 are required");
    for (int k = 0; k < count; ++k)
        if (!n0[k] || !u0[k]) return fail(MLB_EINVAL, "n0 and u0 are required for every system");
    B.ws = static_cast<char *>(workspace);
    B.use_graph = !no_alloc && (options & MLB_OPT_NO_GRAPH) == 0;
    if (B.tiled && !mlb::tile_prepare(B.reach_max, B.ball_reach_max, B.ball_total_max, B.maxM))
        B.tiled = false;
    TRY(upload_static<T>(B, st));
    if (B.tiled) TRY(set_tiling(B, 0, 1, 3, false, 0, st));
    for (auto &S : B.sys)
        if (S.spectral) TRY(setup_spectral(B, S, st));
    bool any_spectral = false;
    for (auto &S : B.sys) any_spectral = any_spectral || S.spectral;
    if (any_spectral && !no_alloc) {
        // default priority, like every stream of the library
        HIP_TRY(hipStreamCreateWithFlags(&B.side, hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&B.ev_fork, hipEventDisableTiming));
        HIP_TRY(hipEventCreateWithFlags(&B.ev_join, hipEventDisableTiming));
    }
    TRY(init_populations<T>(B, n0, u0, st));
    for (auto &S : B.sys) mlb::launch_zero_i32(reinterpret_cast<int *>(B.ws + S.series_cnt), 1, st);
    HIP_TRY(hipStreamSynchronize(st));
    if (!(options & MLB_OPT_NO_STABILITY_CHECK)) TRY(check_mean_states(B, st));
    if (B.tiled && fixed_shape >= 0) {
        TRY(set_tiling(B, fixed_shape, fixed_order, fixed_split ? fixed_split : 3, fixed_groups == 2,
                       fixed_g1 == 2 ? kG1Own : fixed_shape, st));
    } else if (B.tiled && (options & MLB_OPT_TUNE)) {
        TRY(autotune<T>(B, n0, u0, st));
    }
    HIP_TRY(hipGetLastError());
    return MLB_OK;
}

size_t workspace_for(const mlb_params *params, int count)
{
    Batch B;
    std::string why;
    if (!plan_batch(B, params, count, why)) {
        g_err = why;
        return 0;
    }
    return B.total;
}

hipStream_t S_(void *stream) { return static_cast<hipStream_t>(stream); }

// ---------------------------------------------------- per-system helpers
mlb_status moments_of(Batch &B, int k, void *n_out, void *j_out, hipStream_t st)
{
    if (k < 0 || k >= B.count) return fail(MLB_EINVAL, "bad system index");
    SysHost &S = B.sys[k];
    // moments of every system in one launch (cheap), then copy system k
    if (B.prec == 64) mlb::Launch<double>::moments(B.ddesc<double>(0), B.map_of(B.map_site), B.nblk_site, B.parity, st);
    else mlb::Launch<float>::moments(B.ddesc<float>(0), B.map_of(B.map_site), B.nblk_site, B.parity, st);
    const size_t ts = tsize_of(B.prec);
    if (n_out) HIP_TRY(hipMemcpyAsync(n_out, B.ws + S.n, ts * S.M * S.N, hipMemcpyDeviceToDevice, st));
    if (j_out) HIP_TRY(hipMemcpyAsync(j_out, B.ws + S.j, ts * 3 * S.M * S.N, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipGetLastError());
    return MLB_OK;
}

mlb_status populations_of(Batch &B, int k, void *f_out, hipStream_t st)
{
    if (k < 0 || k >= B.count) return fail(MLB_EINVAL, "bad system index");
    SysHost &S = B.sys[k];
    HIP_TRY(hipMemcpyAsync(f_out, B.ws + (B.parity ? S.f1 : S.f0), tsize_of(B.prec) * S.M * mlb::kQ * S.N,
                           hipMemcpyDeviceToDevice, st));
    return MLB_OK;
}

mlb_status set_populations_of(Batch &B, int k, const void *f_in, hipStream_t st)
{
    if (k < 0 || k >= B.count) return fail(MLB_EINVAL, "bad system index");
    const SysHost &S = B.sys[k];
    HIP_TRY(hipMemcpyAsync(B.ws + (B.parity ? S.f1 : S.f0), f_in, tsize_of(B.prec) * S.M * mlb::kQ * S.N,
                           hipMemcpyDeviceToDevice, st));
    return MLB_OK;
}

mlb_status record_mode_of(Batch &B, int k, int a, int b, hipStream_t st)
{
    SysHost &S = B.sys[k];
    mlb::launch_mode(B.ws + S.n, B.prec, a, b, S.p.nx, S.N, reinterpret_cast<double *>(B.ws + B.red), kRedParts,
                     reinterpret_cast<double *>(B.ws + S.series), reinterpret_cast<int *>(B.ws + S.series_cnt),
                     kSeriesCap, (double)B.steps, st);
    HIP_TRY(hipGetLastError());
    return MLB_OK;
}

mlb_status profile_end(Batch &B, double *ms, int32_t *launches, hipStream_t st)
{
    if (!B.profiling) return fail(MLB_ESTATE, "profiling was not started");
    HIP_TRY(hipStreamSynchronize(st));
    double acc[MLB_NPASS] = {};
    int cnt[MLB_NPASS] = {};
    for (auto &m : B.marks) {
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, B.events[m.second], B.events[m.second + 1]));
        acc[m.first] += t;
        cnt[m.first] += 1;
    }
    for (int k = 0; k < MLB_NPASS; ++k) {
        if (ms) ms[k] = acc[k];
        if (launches) launches[k] = cnt[k];
    }
    B.profiling = false;
    B.marks.clear();
    B.next_event = 0;
    return MLB_OK;
}

}  // namespace

namespace {
template <typename T>
mlb_status set_profile(Batch &B, const double *prof, hipStream_t st)
{
    SysHost &S = B.sys[0];
    const int M = S.M, ny = S.p.ny;
    if (prof) {
        // F^a(y) = ext_force[a] + profile[a][y], added in float64 on the host
        std::vector<T> tab((size_t)3 * M * ny);
        for (int a = 0; a < M; ++a)
            for (int d = 0; d < 3; ++d)
                for (int y = 0; y < ny; ++y) {
                    const size_t i = ((size_t)a * 3 + d) * ny + y;
                    if (!std::isfinite(prof[i])) return fail(MLB_EINVAL, "force profile values must be finite");
                    tab[i] = (T)(S.p.ext_force[a * 3 + d] + prof[i]);
                }
        HIP_TRY(hipMemcpyAsync(B.ws + S.fprof, tab.data(), sizeof(T) * tab.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));   // the host table dies here
    }
    S.has_profile = prof != nullptr;
    fill_desc<T>(B, 0, *B.hdesc<T>(0));
    HIP_TRY(hipMemcpyAsync(B.ws + B.desc, B.hdesc<T>(0), B.desc_size, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return MLB_OK;
}
}  // namespace

// ===================================================================== ABI
extern "C" {

size_t mlb_workspace_bytes(const mlb_params *p) { return workspace_for(p, 1); }

mlb_status mlb_check_stability(const mlb_params *p, const double *n_bulk, double *radius)
{
    std::string why;
    if (!validate(p, why)) return fail(MLB_EINVAL, why);
    if (!n_bulk) return fail(MLB_EINVAL, "n_bulk is NULL");
    for (int a = 0; a < p->nspecies; ++a)
        if (!(n_bulk[a] >= 0.0) || !std::isfinite(n_bulk[a])) return fail(MLB_EINVAL, "densities must be >= 0");
    const double rho = cached_radius(p, n_bulk);
    if (radius) *radius = rho;
    if (!(rho <= 1.0 + 1e-6)) return fail(MLB_EUNSTABLE, "spectral radius " + std::to_string(rho) + " > 1");
    return MLB_OK;
}

mlb_status mlb_init_mixture_ex(const mlb_params *p, void *workspace, size_t workspace_bytes, const double *n0,
                               const double *u0, uint32_t options, void *stream, mlb_mixture *out)
{
    if (!out) return fail(MLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return fail(MLB_EINVAL, "params is NULL");
    std::unique_ptr<mlb_mixture_s> h(new mlb_mixture_s());
    const double *n0v[1] = {n0}, *u0v[1] = {u0};
    mlb_status s = p->precision == 64
                       ? create<double>(*h, p, 1, workspace, workspace_bytes, n0v, u0v, options, S_(stream))
                       : create<float>(*h, p, 1, workspace, workspace_bytes, n0v, u0v, options, S_(stream));
    if (s != MLB_OK) return s;
    *out = h.release();
    return MLB_OK;
}

mlb_status mlb_init_mixture(const mlb_params *p, void *workspace, size_t workspace_bytes, const double *n0,
                            const double *u0, void *stream, mlb_mixture *out)
{
    return mlb_init_mixture_ex(p, workspace, workspace_bytes, n0, u0, 0, stream, out);
}

mlb_status mlb_init_mixture_static(const mlb_params *p, const double *n0, const double *u0, void *stream,
                                   mlb_mixture *out)
{
    if (!out) return fail(MLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return fail(MLB_EINVAL, "params is NULL");
    const size_t need = workspace_for(p, 1);
    if (need == 0) return MLB_EINVAL;   // workspace_for left the reason
    if (need > MLB_STATIC_WORKSPACE_BYTES)
        return fail(MLB_ENOMEM, "the mixture needs " + std::to_string(need) + " bytes of workspace; the static " +
                                    "workspace holds " + std::to_string((size_t)MLB_STATIC_WORKSPACE_BYTES));
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MLB_EUNSUPPORTED, "device index beyond the static workspace table");
    void *ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_busy[dev])
            return fail(MLB_ESTATE, "the static workspace of this device is held by another mixture; destroy it first");
        if (!g_static_ptr[dev]) {
            void *ptr = nullptr;
            HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
            if (!ptr) return fail(MLB_EHIP, "hipGetSymbolAddress returned no address for the static workspace");
            g_static_ptr[dev] = ptr;
        }
        ws = g_static_ptr[dev];
        g_static_busy[dev] = true;
    }
    std::unique_ptr<mlb_mixture_s> h(new mlb_mixture_s());
    h->static_dev = dev;   // the destructor releases the array, also on failure below
    const double *n0v[1] = {n0}, *u0v[1] = {u0};
    mlb_status s = p->precision == 64
                       ? create<double>(*h, p, 1, ws, MLB_STATIC_WORKSPACE_BYTES, n0v, u0v, 0, S_(stream), true)
                       : create<float>(*h, p, 1, ws, MLB_STATIC_WORKSPACE_BYTES, n0v, u0v, 0, S_(stream), true);
    if (s != MLB_OK) return s;
    *out = h.release();
    return MLB_OK;
}

mlb_status mlb_step(mlb_mixture h, int32_t nsteps, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    return do_steps(*h, nsteps, S_(stream));
}

mlb_status mlb_set_graph(mlb_mixture h, int32_t enable)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    h->use_graph = enable != 0;
    return MLB_OK;
}

mlb_status mlb_moments(mlb_mixture h, void *n_out, void *j_out, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    return moments_of(*h, 0, n_out, j_out, S_(stream));
}

mlb_status mlb_forces(mlb_mixture h, void *nphi_out, uint32_t parts, void *stream)
{
    if (!h || !nphi_out) return fail(MLB_EINVAL, "handle and output are required");
    if (parts == 0 || parts > MLB_PART_ALL) return fail(MLB_EINVAL, "parts mask must be a non-empty subset of MLB_PART_ALL");
    if (h->prec == 64) return run_query<double>(*h, 0, static_cast<double *>(nphi_out), parts, S_(stream));
    return run_query<float>(*h, 0, static_cast<float *>(nphi_out), parts, S_(stream));
}

mlb_status mlb_fields(mlb_mixture h, void *n, void *j, void *u, void *g, void *vhat, void *H, void *nphi, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    hipStream_t st = S_(stream);
    TRY(h->prec == 64 ? run_query<double>(*h, 0, nullptr, 0, st) : run_query<float>(*h, 0, nullptr, 0, st));
    const SysHost &S = h->sys[0];
    const size_t ts = tsize_of(h->prec), M = S.M, N = (size_t)S.N;
    struct { void *dst; size_t off, bytes; } cp[] = {
        {n, S.n, ts * M * N}, {j, S.j, ts * 3 * M * N}, {u, S.u, ts * 3 * N}, {g, S.g, ts * (size_t)S.P * N},
        {vhat, S.vh, ts * 3 * M * N}, {H, S.H, ts * 3 * M * N}, {nphi, S.Nf, ts * 3 * M * N}};
    for (auto &c : cp)
        if (c.dst) HIP_TRY(hipMemcpyAsync(c.dst, h->ws + c.off, c.bytes, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return MLB_OK;
}

mlb_status mlb_get_populations(mlb_mixture h, void *f_out, void *stream)
{
    if (!h || !f_out) return fail(MLB_EINVAL, "handle and output are required");
    return populations_of(*h, 0, f_out, S_(stream));
}

mlb_status mlb_set_populations(mlb_mixture h, const void *f_in, void *stream)
{
    if (!h || !f_in) return fail(MLB_EINVAL, "handle and input are required");
    return set_populations_of(*h, 0, f_in, S_(stream));
}

mlb_status mlb_set_step_count(mlb_mixture h, int64_t steps)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    if (steps < 0) return fail(MLB_EINVAL, "step count must be >= 0");
    h->steps = steps;
    return MLB_OK;
}


mlb_status mlb_set_force_profile(mlb_mixture h, const double *profile, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    if (h->count != 1) return fail(MLB_EUNSUPPORTED, "force profiles are per mixture");
    return h->prec == 64 ? set_profile<double>(*h, profile, S_(stream)) : set_profile<float>(*h, profile, S_(stream));
}

mlb_status mlb_conserved(mlb_mixture h, double *mass, double *mom, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    hipStream_t st = S_(stream);
    TRY(moments_of(*h, 0, nullptr, nullptr, st));
    const SysHost &S = h->sys[0];
    double *out = reinterpret_cast<double *>(h->ws + h->red_out);
    mlb::launch_conserved(h->ws + S.n, h->ws + S.j, h->prec, S.M, S.N, reinterpret_cast<double *>(h->ws + h->red),
                          kRedParts, out, st);
    double host[16];
    HIP_TRY(hipMemcpyAsync(host, out, sizeof(double) * 4 * S.M, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    bool finite = true;
    for (int k = 0; k < 4 * S.M; ++k) finite = finite && std::isfinite(host[k]);
    if (mass) for (int a = 0; a < S.M; ++a) mass[a] = host[a];
    if (mom) for (int k = 0; k < 3 * S.M; ++k) mom[k] = host[S.M + k];
    if (!finite) return fail(MLB_ENONFINITE, "a conserved sum is not finite");
    return MLB_OK;
}

mlb_status mlb_record_mode(mlb_mixture h, int32_t a, int32_t b, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    const SysHost &S = h->sys[0];
    if (a < 0 || b < -1 || a >= S.M || b >= S.M || a == b) return fail(MLB_EINVAL, "bad species pair");
    TRY(moments_of(*h, 0, nullptr, nullptr, S_(stream)));
    return record_mode_of(*h, 0, a, b, S_(stream));
}

mlb_status mlb_record_spread(mlb_mixture h, int32_t a, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    const SysHost &S = h->sys[0];
    if (a < 0 || a >= S.M) return fail(MLB_EINVAL, "bad species");
    hipStream_t st = S_(stream);
    TRY(moments_of(*h, 0, nullptr, nullptr, st));
    mlb::launch_spread(h->ws + S.n, h->prec, a, S.p.nx, S.N, reinterpret_cast<double *>(h->ws + h->red), kRedParts,
                       reinterpret_cast<double *>(h->ws + S.series), reinterpret_cast<int *>(h->ws + S.series_cnt),
                       kSeriesCap, (double)h->steps, st);
    HIP_TRY(hipGetLastError());
    return MLB_OK;
}

int32_t mlb_series_capacity(void) { return kSeriesCap; }

mlb_status mlb_series_reset(mlb_mixture h, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    mlb::launch_zero_i32(reinterpret_cast<int *>(h->ws + h->sys[0].series_cnt), 1, S_(stream));
    HIP_TRY(hipGetLastError());
    return MLB_OK;
}

mlb_status mlb_fit_series_ex(mlb_mixture h, int32_t kind, double t_min, double *out5, void *stream)
{
    if (!h || !out5) return fail(MLB_EINVAL, "handle and output are required");
    if (kind != 0 && kind != 1) return fail(MLB_EINVAL, "kind must be 0 (mode) or 1 (spread)");
    hipStream_t st = S_(stream);
    const SysHost &S = h->sys[0];
    const double k = 2.0 * M_PI / (double)S.p.nx;
    double *out = reinterpret_cast<double *>(h->ws + h->fit_out);
    mlb::launch_fit(reinterpret_cast<const double *>(h->ws + S.series),
                    reinterpret_cast<const int *>(h->ws + S.series_cnt), kSeriesCap, kind, t_min, k * k, out, st);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out5, out, sizeof(double) * 5, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return MLB_OK;
}

mlb_status mlb_fit_series(mlb_mixture h, int32_t kind, double t_min, double *D_out, void *stream)
{
    if (!h || !D_out) return fail(MLB_EINVAL, "handle and output are required");
    double out[5];
    TRY(mlb_fit_series_ex(h, kind, t_min, out, stream));
    *D_out = out[0];
    return MLB_OK;
}

namespace {
mlb_status copy_series(Batch &B, int k, double *t, double *v, int32_t capacity, int32_t *count, void *stream)
{
    Batch *h = &B;
    hipStream_t st = S_(stream);
    const SysHost &S = h->sys[(size_t)k];
    int c = 0;
    HIP_TRY(hipMemcpyAsync(&c, h->ws + S.series_cnt, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    c = std::min(c, kSeriesCap);
    *count = c;
    const int n = std::min(c, capacity);
    if (n > 0 && (t || v)) {
        std::vector<double> buf(2 * (size_t)n);
        HIP_TRY(hipMemcpyAsync(buf.data(), h->ws + S.series, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int i = 0; i < n; ++i) {
            if (t) t[i] = buf[2 * i];
            if (v) v[i] = buf[2 * i + 1];
        }
    }
    return MLB_OK;
}
}  // namespace

mlb_status mlb_get_series(mlb_mixture h, double *t, double *v, int32_t capacity, int32_t *count, void *stream)
{
    if (!h || !count) return fail(MLB_EINVAL, "handle and count are required");
    return copy_series(*h, 0, t, v, capacity, count, stream);
}

mlb_status mlb_batch_get_series(mlb_batch h, int32_t system, double *t, double *v, int32_t capacity,
                                int32_t *count, void *stream)
{
    if (!h || !count) return fail(MLB_EINVAL, "handle and count are required");
    if (system < 0 || system >= h->count) return fail(MLB_EINVAL, "system index out of range");
    return copy_series(*h, system, t, v, capacity, count, stream);
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
    return profile_end(*h, ms, launches, S_(stream));
}

const char *mlb_pass_name(int32_t k) { return (k >= 0 && k < MLB_NPASS) ? kPassNames[k] : ""; }

mlb_status mlb_destroy(mlb_mixture h)
{
    delete h;
    return MLB_OK;
}

const char *mlb_last_error(void) { return g_err.c_str(); }

mlb_status mlb_set_closure(mlb_mixture h, mlb_net net, int32_t check_every, double tol)
{
    if (!h) return fail(MLB_EINVAL, "null handle");
    Batch &B = *h;
    if (B.graph_closure) {
        (void)hipGraphExecDestroy(B.graph_closure);
        B.graph_closure = nullptr;
    }
    if (!net) {
        B.net = nullptr;
        B.closure_active = false;
        return MLB_OK;
    }
    const SysHost &S = B.sys[0];
    if (B.count != 1 || B.prec != 32 || S.M != 2 || S.p.walls_y)
        return fail(MLB_EUNSUPPORTED, "the closure needs a float32 binary periodic mixture");
    int nx = 0, ny = 0, nz = 0;
    mlb::net_grid(net, &nx, &ny, &nz);
    if (nx != S.p.nx || ny != S.p.ny || nz != S.p.nz) return fail(MLB_EINVAL, "network grid differs from the mixture's");
    if (check_every < 1) return fail(MLB_EINVAL, "check_every must be >= 1");
    if (!(tol >= 0.0)) return fail(MLB_EINVAL, "tol must be >= 0");
    B.net = net;
    B.check_every = check_every;
    B.closure_tol = tol;
    B.closure_active = true;
    B.closure_checks = 0;
    B.fallback_step = -1;
    B.failed_checks = 0;
    B.net_steps = 0;
    B.last_err = -1.0;
    return MLB_OK;
}

mlb_status mlb_closure_stats(mlb_mixture h, int64_t *checks, int64_t *fallback_step, double *last_err,
                             int32_t *active)
{
    if (!h) return fail(MLB_EINVAL, "null handle");
    if (checks) *checks = h->closure_checks;
    if (fallback_step) *fallback_step = h->fallback_step;
    if (last_err) *last_err = h->last_err;
    if (active) *active = (h->net && h->closure_active) ? 1 : 0;
    return MLB_OK;
}

mlb_status mlb_closure_usage(mlb_mixture h, int64_t *net_steps, int64_t *failed_checks)
{
    if (!h) return fail(MLB_EINVAL, "null handle");
    if (net_steps) *net_steps = h->net_steps;
    if (failed_checks) *failed_checks = h->failed_checks;
    return MLB_OK;
}

mlb_status mlb_closure_sample(mlb_mixture h, mlb_net net, float *x_out, float *target_out, void *stream)
{
    if (!h || !net) return fail(MLB_EINVAL, "null handle");
    if (!x_out || !target_out) return fail(MLB_EINVAL, "x_out and target_out must be device pointers");
    Batch &B = *h;
    const SysHost &S = B.sys[0];
    if (B.count != 1 || B.prec != 32 || S.M != 2) return fail(MLB_EUNSUPPORTED, "needs a float32 binary mixture");
    int nx = 0, ny = 0, nz = 0;
    mlb::net_grid(net, &nx, &ny, &nz);
    if (nx != S.p.nx || ny != S.p.ny || nz != S.p.nz) return fail(MLB_EINVAL, "network grid differs from the mixture's");
    hipStream_t st = S_(stream);
    run_passes<float>(B, st, false, 0, 1);
    mlb::net_sample(net, reinterpret_cast<const float *>(B.ws + S.n), reinterpret_cast<const float *>(B.ws + S.j),
                    reinterpret_cast<const float *>(B.ws + S.Nf), x_out, target_out, st);
    HIP_TRY(hipGetLastError());
    return MLB_OK;
}

// ------------------------------------------------------------------ batch
size_t mlb_batch_workspace_bytes(const mlb_params *systems, int32_t count)
{
    if (!systems || count < 1) {
        g_err = "systems and count >= 1 are required";
        return 0;
    }
    return workspace_for(systems, count);
}

mlb_status mlb_init_batch(const mlb_params *systems, int32_t count, void *workspace, size_t workspace_bytes,
                          const double *const *n0, const double *const *u0, uint32_t options, void *stream,
                          mlb_batch *out)
{
    if (!out) return fail(MLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (!systems || count < 1) return fail(MLB_EINVAL, "systems and count >= 1 are required");
    std::unique_ptr<mlb_batch_s> h(new mlb_batch_s());
    mlb_status s = systems[0].precision == 64
                       ? create<double>(*h, systems, count, workspace, workspace_bytes, n0, u0, options, S_(stream))
                       : create<float>(*h, systems, count, workspace, workspace_bytes, n0, u0, options, S_(stream));
    if (s != MLB_OK) return s;
    *out = h.release();
    return MLB_OK;
}

mlb_status mlb_batch_step(mlb_batch h, int32_t nsteps, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    return do_steps(*h, nsteps, S_(stream));
}

mlb_status mlb_batch_moments(mlb_batch h, int32_t system, void *n_out, void *j_out, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    return moments_of(*h, system, n_out, j_out, S_(stream));
}

mlb_status mlb_batch_get_populations(mlb_batch h, int32_t system, void *f_out, void *stream)
{
    if (!h || !f_out) return fail(MLB_EINVAL, "handle and output are required");
    return populations_of(*h, system, f_out, S_(stream));
}

mlb_status mlb_batch_record_modes(mlb_batch h, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    hipStream_t st = S_(stream);
    TRY(moments_of(*h, 0, nullptr, nullptr, st));
    for (int k = 0; k < h->count; ++k)
        if (h->sys[k].M >= 2) TRY(record_mode_of(*h, k, 0, 1, st));
    return MLB_OK;
}

mlb_status mlb_batch_fit_ex(mlb_batch h, double t_min, double *out5, void *stream)
{
    if (!h || !out5) return fail(MLB_EINVAL, "handle and output are required");
    hipStream_t st = S_(stream);
    double *out = reinterpret_cast<double *>(h->ws + h->fit_out);
    for (int k = 0; k < h->count; ++k) {
        const SysHost &S = h->sys[k];
        const double kk = 2.0 * M_PI / (double)S.p.nx;
        mlb::launch_fit(reinterpret_cast<const double *>(h->ws + S.series),
                        reinterpret_cast<const int *>(h->ws + S.series_cnt), kSeriesCap, 0, t_min, kk * kk,
                        out + kFitOut * k, st);
    }
    HIP_TRY(hipGetLastError());
    std::vector<double> host(kFitOut * (size_t)h->count);
    HIP_TRY(hipMemcpyAsync(host.data(), out, sizeof(double) * host.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int k = 0; k < h->count; ++k)
        for (int i = 0; i < 5; ++i) out5[5 * (size_t)k + i] = host[kFitOut * (size_t)k + i];
    return MLB_OK;
}

mlb_status mlb_batch_fit(mlb_batch h, double t_min, double *D_out, void *stream)
{
    if (!h || !D_out) return fail(MLB_EINVAL, "handle and output are required");
    std::vector<double> all(5 * (size_t)h->count);
    TRY(mlb_batch_fit_ex(h, t_min, all.data(), stream));
    for (int k = 0; k < h->count; ++k) D_out[k] = all[5 * (size_t)k];
    return MLB_OK;
}

mlb_status mlb_tuning(mlb_mixture h, int32_t *shape, int32_t *order, double *trial_ms)
{
    return mlb_batch_tuning(h, shape, order, trial_ms);
}

mlb_status mlb_batch_tuning(mlb_batch h, int32_t *shape, int32_t *order, double *trial_ms)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    if (shape) *shape = h->tiled ? h->tune.shape : -1;
    if (order) *order = h->tiled ? h->tune.order : -1;
    if (trial_ms)
        // per tile shape and order, the faster of the first gather's splits
        for (int i = 0; i < 2 * mlb::kTileVariants; ++i) {
            double best = 0.0;
            for (int c = 0; c < kSplitChoices; ++c) {
                const double v = h->tune.trial_ms[c * 2 * mlb::kTileVariants + i];
                if (v > 0.0 && (best == 0.0 || v < best)) best = v;
            }
            trial_ms[i] = best;
        }
    return MLB_OK;
}

mlb_status mlb_batch_tuning_ex(mlb_batch h, int32_t *shape, int32_t *order, int32_t *gather1_split,
                               double *trial_ms)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    if (shape) *shape = h->tiled ? h->tune.shape : -1;
    if (order) *order = h->tiled ? h->tune.order : -1;
    if (gather1_split) *gather1_split = h->tiled ? h->tune.g1split : -1;
    if (trial_ms)
        for (int i = 0; i < kTrials; ++i) trial_ms[i] = h->tune.trial_ms[i];
    return MLB_OK;
}

mlb_status mlb_tuning_ex(mlb_mixture h, int32_t *shape, int32_t *order, int32_t *gather1_split, double *trial_ms)
{
    return mlb_batch_tuning_ex(h, shape, order, gather1_split, trial_ms);
}

mlb_status mlb_batch_tuning_groups(mlb_batch h, int32_t *sign_groups, double *groups_ms)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    if (sign_groups) *sign_groups = h->tiled ? (h->tune.groups ? 1 : 0) : -1;
    if (groups_ms) *groups_ms = h->tune.groups_ms;
    return MLB_OK;
}

mlb_status mlb_tuning_groups(mlb_mixture h, int32_t *sign_groups, double *groups_ms)
{
    return mlb_batch_tuning_groups(h, sign_groups, groups_ms);
}

mlb_status mlb_batch_tuning_gather1_shape(mlb_batch h, int32_t *shape)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    if (shape) *shape = h->tiled ? h->tune.g1shape : -1;
    return MLB_OK;
}

mlb_status mlb_tuning_gather1_shape(mlb_mixture h, int32_t *shape)
{
    return mlb_batch_tuning_gather1_shape(h, shape);
}

mlb_status mlb_batch_profile_begin(mlb_batch h)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    h->profiling = true;
    h->marks.clear();
    h->next_event = 0;
    return MLB_OK;
}

mlb_status mlb_batch_profile_end(mlb_batch h, double *ms, int32_t *launches, void *stream)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    return profile_end(*h, ms, launches, S_(stream));
}

int64_t mlb_batch_step_count(mlb_batch h) { return h ? h->steps : -1; }

mlb_status mlb_batch_set_populations(mlb_batch h, int32_t system, const void *f_in, void *stream)
{
    if (!h || !f_in) return fail(MLB_EINVAL, "handle and input are required");
    return set_populations_of(*h, system, f_in, S_(stream));
}

mlb_status mlb_batch_set_step_count(mlb_batch h, int64_t steps)
{
    if (!h) return fail(MLB_EINVAL, "handle is NULL");
    if (steps < 0) return fail(MLB_EINVAL, "step count must be >= 0");
    h->steps = steps;
    return MLB_OK;
}

mlb_status mlb_batch_destroy(mlb_batch h)
{
    delete h;
    return MLB_OK;
}

}  // extern "C"
