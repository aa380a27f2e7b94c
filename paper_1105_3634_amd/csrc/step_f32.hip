// Float32 instantiation of the per-site passes (contraction allowed) and
// the tiled float32 gathers in three tile shapes (four for the first gather).
#include <cstdint>
#include <initializer_list>

#include "gather_tile.h"

namespace mlb {
template struct Launch<float>;

void tile_dims(int v, int &tx, int &ty, int &tz)
{
    static const int D[kG1Variants][3] = {{16, 4, 4}, {8, 8, 4}, {32, 4, 2}, {4, 8, 8}};
    tx = D[v][0]; ty = D[v][1]; tz = D[v][2];
}

int tile_count(int v, int nx, int ny, int nz)
{
    int tx, ty, tz;
    tile_dims(v, tx, ty, tz);
    return ((nx + tx - 1) / tx) * ((ny + ty - 1) / ty) * ((nz + tz - 1) / tz);
}

namespace {
size_t gather_lds_bytes_of(int v, int reach, int layouts, bool second)
{
    int tx, ty, tz;
    tile_dims(v, tx, ty, tz);
    if (tx + 2 * reach > kBlock) return SIZE_MAX;   // not stageable: one halo column per thread
    return tile_lds_bytes(tx, ty, tz, reach, layouts, second);
}
}  // namespace

size_t gather1_lds_bytes_of(int v, int reach) { return gather_lds_bytes_of(v, reach, MLB_G1_LAYOUTS, false); }

size_t tile_lds_bytes_of(int v, int reach)
{
    return std::max(gather_lds_bytes_of(v, reach, MLB_G1_LAYOUTS, false), gather_lds_bytes_of(v, reach, MLB_S2_LAYOUTS, true));
}

size_t contact_lds_bytes_of(int v, int ball_reach, int ball_total, int maxM)
{
    int tx, ty, tz;
    tile_dims(v, tx, ty, tz);
    if (tx + 2 * ball_reach > kBlock) return SIZE_MAX;
    return contact_lds_bytes(tx, ty, tz, ball_reach, ball_total, maxM);
}

namespace {
constexpr size_t kLdsMax = 160 * 1024;   // LDS of one CU

// The limits are set to the whole LDS of a CU, not to this handle's need:
// handles with a smaller reach created later must not lower them under the
// launches of a live handle with a larger one.
bool raise_lds_limit(std::initializer_list<const void *> fns)
{
    for (const void *fn : fns)
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax) != hipSuccess)
            return false;
    return true;
}

template <int TX, int TY, int TZ>
bool prepare_gather1(int reach)
{
    if (tile_lds_bytes(TX, TY, TZ, reach, MLB_G1_LAYOUTS, false) > kLdsMax) return false;
    if (TX + 2 * reach > kBlock) return false;   // staging gives each thread one halo column
    return raise_lds_limit({(const void *)k_gather1_tile<TX, TY, TZ, 2, false>, (const void *)k_gather1_tile<TX, TY, TZ, 3, false>,
                            (const void *)k_gather1_tile<TX, TY, TZ, 2, true>, (const void *)k_gather1_tile<TX, TY, TZ, 3, true>});
}

template <int TX, int TY, int TZ>
bool prepare_one(int reach, int ball_reach, int ball_total, int maxM)
{
    const size_t bytes = tile_lds_bytes(TX, TY, TZ, reach, MLB_S2_LAYOUTS, true);
    const size_t cbytes = contact_lds_bytes(TX, TY, TZ, ball_reach, ball_total, maxM);
    if (bytes > kLdsMax || cbytes > kLdsMax) return false;
    if (TX + 2 * reach > kBlock || TX + 2 * ball_reach > kBlock) return false;
    return prepare_gather1<TX, TY, TZ>(reach) &&
           raise_lds_limit({(const void *)k_contact_tile<TX, TY, TZ>, (const void *)k_step2_tile<TX, TY, TZ>});
}
}  // namespace

bool tile_prepare(int reach_max, int ball_reach_max, int ball_total_max, int maxM)
{
    return prepare_one<16, 4, 4>(reach_max, ball_reach_max, ball_total_max, maxM) &&
           prepare_one<8, 8, 4>(reach_max, ball_reach_max, ball_total_max, maxM) &&
           prepare_one<32, 4, 2>(reach_max, ball_reach_max, ball_total_max, maxM) && prepare_gather1<4, 8, 8>(reach_max);
}

void launch_contact_tile(int v, const SysDesc<float> *sys, const int2 *map, int nblk, Tables<float> tb,
                         int ball_reach_max, int ball_total_max, int maxM, hipStream_t st)
{
    const size_t lds = contact_lds_bytes_of(v, ball_reach_max, ball_total_max, maxM);
    if (v == 0) hipLaunchKernelGGL((k_contact_tile<16, 4, 4>), dim3(nblk), dim3(kBlock), lds, st, sys, map, tb);
    else if (v == 1) hipLaunchKernelGGL((k_contact_tile<8, 8, 4>), dim3(nblk), dim3(kBlock), lds, st, sys, map, tb);
    else hipLaunchKernelGGL((k_contact_tile<32, 4, 2>), dim3(nblk), dim3(kBlock), lds, st, sys, map, tb);
}

namespace {
template <int SPLIT, bool GROUPED>
void gather1_split(int v, const SysDesc<float> *sys, const int2 *map, dim3 grid, size_t lds, Tables<float> tb,
                   hipStream_t st)
{
    const dim3 block(SPLIT * kBlock);
    if (v == 0) hipLaunchKernelGGL((k_gather1_tile<16, 4, 4, SPLIT, GROUPED>), grid, block, lds, st, sys, map, tb);
    else if (v == 1) hipLaunchKernelGGL((k_gather1_tile<8, 8, 4, SPLIT, GROUPED>), grid, block, lds, st, sys, map, tb);
    else if (v == 2) hipLaunchKernelGGL((k_gather1_tile<32, 4, 2, SPLIT, GROUPED>), grid, block, lds, st, sys, map, tb);
    else hipLaunchKernelGGL((k_gather1_tile<4, 8, 8, SPLIT, GROUPED>), grid, block, lds, st, sys, map, tb);
}
}  // namespace

void launch_gather1_tile(int v, int split, bool groups, const SysDesc<float> *sys, const int2 *map, int nblk,
                         int maxM, Tables<float> tb, int reach_max, hipStream_t st)
{
    const size_t lds = gather_lds_bytes_of(v, reach_max, MLB_G1_LAYOUTS, false);
    const dim3 grid(nblk, maxM);
    if (split == 2) {
        if (groups) gather1_split<2, true>(v, sys, map, grid, lds, tb, st);
        else gather1_split<2, false>(v, sys, map, grid, lds, tb, st);
    } else {
        if (groups) gather1_split<3, true>(v, sys, map, grid, lds, tb, st);
        else gather1_split<3, false>(v, sys, map, grid, lds, tb, st);
    }
}

void launch_step2_tile(int v, const SysDesc<float> *sys, const int2 *map, int nblk, int maxM, Tables<float> tb,
                       int reach_max, int parity, int write_force_only, hipStream_t st)
{
    const size_t lds = gather_lds_bytes_of(v, reach_max, MLB_S2_LAYOUTS, true);
    const dim3 grid(nblk, maxM);
    if (v == 0)
        hipLaunchKernelGGL((k_step2_tile<16, 4, 4>), grid, dim3(kStep2Threads), lds, st, sys, map, tb, parity, write_force_only);
    else if (v == 1)
        hipLaunchKernelGGL((k_step2_tile<8, 8, 4>), grid, dim3(kStep2Threads), lds, st, sys, map, tb, parity, write_force_only);
    else
        hipLaunchKernelGGL((k_step2_tile<32, 4, 2>), grid, dim3(kStep2Threads), lds, st, sys, map, tb, parity, write_force_only);
}
}  // namespace mlb
