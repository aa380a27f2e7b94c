// Internal declarations of the mlb GPU library: the per-system descriptor the
// kernels read, the stencil tables built on the host, and the launch entry
// points of each pass.  Not part of the public ABI (include/mlb.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mlb.h"

namespace mlb {

constexpr int kMaxS = 4;
constexpr int kQ = 19;
// Sign groups of a shell half-list (float32 first gather): 0 = four points
// (+-e_y, +-e_z), 1 = two points (+-e_y, e_z = 0), 2 = two points (e_y = 0,
// +-e_z), 3 = two points (e_x = 0, +-e_z), 4 = single points on an axis.
constexpr int kGroupKinds = 5;
constexpr int kBlock = 256;          // threads per block of the per-site passes

// Stencil offsets travel packed: three signed bytes (ex, ey, ez).
__host__ __device__ inline int32_t pack_offset(int ex, int ey, int ez)
{
    return (ex & 0xff) | ((ey & 0xff) << 8) | ((ez & 0xff) << 16);
}
__host__ __device__ inline void unpack_offset(int32_t p, int &ex, int &ey, int &ez)
{
    ex = (int)(int8_t)(p & 0xff);
    ey = (int)(int8_t)((p >> 8) & 0xff);
    ez = (int)(int8_t)((p >> 16) & 0xff);
}

// One lattice system as the kernels see it.  Lives in device memory; every
// block belongs to one system, so all loads from it are wave-uniform.
template <typename T>
struct SysDesc {
    int nx, ny, nz, M, P, walls;
    long long N;
    int nblocks;                     // per-site blocks of this system (ceil(N / kBlock))
    int reach;                       // largest |component| of any shell offset
    int ball_reach;                  // largest |component| of any smoothing-ball offset
    int ball_total;                  // entries of this system's ball half-lists (all species)
    T *f[2];                         // population double buffer [M][19][N]
    T *n, *j, *u, *g, *vh, *H, *Nf;  // fields (see mlb.h for layouts)
    T *tail;                         // attractive field sum_b K_ab * n_b [M][3][N] (spectral mode)
    T *parts;                        // optional force-part accumulator [M][3][N] (forces query)
    T *Tloc;                         // local friction tensor sum_b ck Ts_b [M][6][N] (tiled path)
    T *gfac;                         // (1/m_a) / (1 + Gamma_a / (2 m_a)) per species-site when the tail is deferred [M][N]
    unsigned parts_mask;
    int tail_direct;                 // 1: direct tail sum in the first gather
    int tail_deferred;               // 1: the first gather leaves the spectral tail out; k_add_tail adds it
    int scheme;
    int omega_is_one;
    // stencils: indices into the batch-wide tables
    int sh_start[kMaxS][kMaxS], sh_cnt[kMaxS][kMaxS];
    int sg_start[kMaxS][kMaxS][kGroupKinds], sg_cnt[kMaxS][kMaxS][kGroupKinds];   // sign groups (float4 index, groups)
    int tl_start[kMaxS][kMaxS], tl_cnt[kMaxS][kMaxS];
    int bl_start[kMaxS], bl_cnt[kMaxS], bl_full[kMaxS];
    // constants (computed in float64 on the host, rounded to T)
    T cm[kMaxS][kMaxS];              // -kT sigma_ab^2 w_hat / 2
    T cg[kMaxS][kMaxS];              // kappa_ab / 6
    T ck[kMaxS][kMaxS];              // kappa_ab / 2
    T dd[kMaxS][kMaxS];              // sigma_a sigma_b / (sigma_a + sigma_b)
    T s2[kMaxS], s3[kMaxS];          // (pi/6) sigma^2, (pi/6) sigma^3
    T fext[kMaxS][3];
    // species masses (Sec. 2): m_a, 1/m_a, m_a/kT = 1/theta_a and the weight
    // (9/2)(theta_a - 1/3) of the lattice equilibrium's temperature term;
    // unit_mass = 1 when every m_a is 1 (the term then vanishes everywhere)
    T mass[kMaxS], im[kMaxS], ith[kMaxS], dth[kMaxS];
    int unit_mass;
    const T *fprof;                  // body force per lattice row [M][3][ny] (replaces fext when set)
    T omega, om1;
    T wall_ux[2];
};

// Batch-wide stencil tables (device).
template <typename T>
struct Tables {
    const int32_t *sh_e;  const T *sh_u;     // shell half-lists: packed offset, unit vector [3]
    const int32_t *tl_e;  const T *tl_w;     // tail half-lists: packed offset, vector weight [3]
    const int32_t *bl_e;                     // ball half-lists: packed offset
    // float32 tiled gathers: the shell half-lists as float4 (packed offset
    // bits, unit vector), followed by kShellPad zero entries
    const float4 *sh_q;
    // the same half-lists in sign groups (see kGroupKinds): a four-point
    // group is four float4 (the members' packed offsets; |e_hat|; the
    // squares; the products xy, xz, yz), a two-point group two float4 ((the
    // members' offsets, |e_hat| on the shared and the flipped axis); the
    // squares and their product), a single point the sh_q entry
    const float4 *sg_q;
};
constexpr int kShellPad = 8;

// ---------------------------------------------------------------- host side
struct HostStencil {
    std::vector<int32_t> e;      // packed offsets
    std::vector<double> v;       // 3 per entry: unit vector (shell) or weight (tail)
    int full = 0;                // size of the symmetric set
    int max_abs[3] = {0, 0, 0};  // largest |component| per axis
};

enum { kShell = 0, kBall = 1, kTail = 2 };
HostStencil build_stencil(int kind, double s, double rc);

// Spectral radius of the linearised step at uniform densities n0 (host
// float64) over the wavevectors pi (i, j, l) / kgrid, k = 0 excluded.
double stability_radius(const mlb_params *p, const double *n0, int kgrid);

struct PairConst {
    double cm, cg, ck, dd;
};
PairConst pair_constants(double sa, double sb, double kT, int shell_full, double ma, double mb);

// A launch covers the blocks of many systems: block b works on system
// map[b].x (a negative value idles the block), local block map[b].y.
// Launch entry points (one per precision), all on `st`; `maxM` is the
// largest species count (grid y of the per-species passes).
template <typename T>
struct Launch {
    static void moments(const SysDesc<T> *sys, const int2 *map, int nblk, int parity, hipStream_t st);
    static void contact(const SysDesc<T> *sys, const int2 *map, int nblk, Tables<T> tb, hipStream_t st);
    static void gather1(const SysDesc<T> *sys, const int2 *map, int nblk, int maxM, Tables<T> tb,
                        hipStream_t st);
    static void step2(const SysDesc<T> *sys, const int2 *map, int nblk, int maxM, Tables<T> tb,
                      int parity, int write_force_only, hipStream_t st);
    // the deferred spectral tail: H += n_a C_a, V-hat += (C_a / m_a) / (1 + Gamma_a / (2 m_a))
    static void add_tail(const SysDesc<T> *sys, const int2 *map, int nblk, int maxM, hipStream_t st);
    static void init_pop(const SysDesc<T> *sys, const int2 *map, int nblk, const double *n0,
                         const double *u0, hipStream_t st);
};

// Float32 tiled gathers (gather_tile.h, built in step_f32.hip); tile shape
// variant v: 0 = 16x4x4, 1 = 8x8x4, 2 = 32x4x2 sites for all tiled passes;
// the first gather also runs on 3 = 4x8x8 (rows of 4 + 2R halo sites: at
// reach 4 its 16-byte LDS reads fall on distinct banks, at the LDS
// footprint of 8x8x4).
constexpr int kTileVariants = 3;
constexpr int kG1Variants = 4;
void tile_dims(int v, int &tx, int &ty, int &tz);
// (groups: the sign-grouped shell loop, see gather_tile.h)
void launch_gather1_tile(int v, int split, bool groups, const SysDesc<float> *sys, const int2 *map, int nblk,
                         int maxM, Tables<float> tb, int reach_max, hipStream_t st);
// dynamic LDS of the first gather on shape v (SIZE_MAX if it cannot stage)
size_t gather1_lds_bytes_of(int v, int reach);
void launch_step2_tile(int v, const SysDesc<float> *sys, const int2 *map, int nblk, int maxM, Tables<float> tb,
                       int reach_max, int parity, int write_force_only, hipStream_t st);
// contact values on the same tiles (halo = ball reach), one thread per site
void launch_contact_tile(int v, const SysDesc<float> *sys, const int2 *map, int nblk, Tables<float> tb,
                         int ball_reach_max, int ball_total_max, int maxM, hipStream_t st);
int tile_count(int v, int nx, int ny, int nz);
// raise the dynamic-LDS limits; false if a kernel cannot fit
bool tile_prepare(int reach_max, int ball_reach_max, int ball_total_max, int maxM);
size_t tile_lds_bytes_of(int v, int reach);
size_t contact_lds_bytes_of(int v, int ball_reach, int ball_total, int maxM);

// float64 reductions (reduce.hip)
void launch_conserved(const void *n, const void *j, int prec, int M, long long N, double *partials,
                      int nparts, double *out, hipStream_t st);
void launch_mode(const void *n, int prec, int a, int b, int nx, long long N, double *partials,
                 int nparts, double *series, int *count, int cap, double t, hipStream_t st);
void launch_spread(const void *n, int prec, int a, int nx, long long N, double *partials, int nparts,
                   double *series, int *count, int cap, double t, hipStream_t st);
void launch_fit(const double *series, const int *count, int cap, int kind, double t_min, double k2,
                double *out, hipStream_t st);
void launch_zero_i32(int *p, int n, hipStream_t st);

}  // namespace mlb
