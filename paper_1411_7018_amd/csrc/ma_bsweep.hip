// Launchers of the block sweep (ma_fsweep.h) and of the z-stream sweep
// (ma_zsweep.h): the shapes they are built for and the automatic choice
// between them.
#include "ma_fsweep.h"
#include "ma_zsweep.h"

#include <algorithm>

namespace mafas {

namespace {

struct BCfg {
    int tx, ty, tz, nt;
    // z-stream sweeps: -1 chunks chosen by the model below, > 0 about zwg
    // workgroups in all; 0: a block sweep
    int zwg;
};
// Shapes (index = tile_config - 1).  Block sweeps: small blocks keep the
// recomputation cheap in absolute terms and give many workgroups; more
// threads per block cut the rounds of updates per phase, which is what a
// sweep of a small grid waits on.  Z-stream sweeps (tz unused): TX x TY
// columns whose update items (TX TY + 3 (TX + TY) + 14 per step) nearly
// fill the workgroup once or twice; 32 x 24 fills 1024 items with one
// colour per wavefront, which makes the colour's plane and ring slots
// scalars (a step about 2% faster than 32 x 26 with its two mixed
// wavefronts).  The planes are cut into chunks, by the model of zs_chunks
// or into about zwg workgroups (one per compute unit at a time, the ring
// filling most of the LDS).
constexpr BCfg kCfg[] = {{8, 8, 8, 256, 0},   {8, 8, 8, 512, 0},  {8, 8, 8, 1024, 0},
                         {16, 8, 4, 256, 0},  {16, 16, 8, 512, 0}, {8, 8, 4, 512, 0},
                         {8, 8, 4, 256, 0},   {32, 26, 0, 1024, -1}, {32, 26, 0, 512, -1},
                         {32, 26, 0, 1024, 1536}, {40, 20, 0, 1024, -1},
                         {32, 24, 0, 1024, -1}};
constexpr int kZsPureConfig = 11;

// Compute units of the current device (one z-stream workgroup each at a time).
int device_cus()
{
    static int cus = 0;
    if (cus <= 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            v > 0)
            cus = v;
        else
            cus = 256;
    }
    return cus;
}

// Chunks of a z-stream sweep over `cols` columns of an n grid: a chunk of zc
// planes takes zc + 10 steps (the phases are skewed over 7 planes, plus the
// pipeline's prefetch), and the workgroups run in rounds of one per compute
// unit, so the sweep takes about ceil(cols * chunks / CUs) * (zc + 10) step
// times; the chunk count minimising that (at least 16 planes a chunk).
int zs_chunks(int n, int cols)
{
    const int cus = device_cus();
    int best = 1;
    long best_cost = -1;
    for (int c = 1; c <= std::max(1, (n - 1) / 16); ++c) {
        const int zc = zs_chunk(n, c);
        const int t = (n - 1 + zc - 1) / zc;
        const long rounds = (long(cols) * t + cus - 1) / cus;
        const long cost = rounds * (zc + 10);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = t;
        }
    }
    return best;
}
constexpr int kNumCfg = int(sizeof(kCfg) / sizeof(kCfg[0]));

// Automatic z-stream shape of an n grid: 32 x 26 or the one-colour-per-
// wavefront 32 x 24, whichever the chunk model (rounds x (planes + 10) step
// times, the 32 x 24 step counted 2% shorter) gives the shorter sweep.  At
// n = 256 the 88 columns of 32 x 24 make three chunks one workgroup too
// many per compute unit, where the 80 of 32 x 26 fit.
int zs_model_cost100(int n, int cfg)
{
    const BCfg &b = kCfg[cfg];
    const int cols = ((n - 1 + b.tx - 1) / b.tx) * ((n - 1 + b.ty - 1) / b.ty);
    const int zc = zs_chunk(n, zs_chunks(n, cols));
    const long t = (n - 1 + zc - 1) / zc;
    const long rounds = (long(cols) * t + device_cus() - 1) / device_cus();
    return int(rounds * (zc + 10) * (cfg == kZsPureConfig ? 98 : 100));
}

template <int OP, int TX, int TY, int NT>
hipError_t zgo_list(hipStream_t st, const FsList *L, int blocks, unsigned long long *nc, bool pro)
{
    if (pro)
        hipLaunchKernelGGL((k_zsweep<OP, TX, TY, NT, true>), dim3(blocks), dim3(NT), 0, st, L, nc);
    else
        hipLaunchKernelGGL((k_zsweep<OP, TX, TY, NT, false>), dim3(blocks), dim3(NT), 0, st, L, nc);
    return hipGetLastError();
}

template <int OP, int TX, int TY, int NT>
hipError_t zgo_one(hipStream_t st, const FsGrid &G, unsigned long long *nc)
{
    const int blocks = G.tiles_x * G.tiles_y * G.tiles_z;
    hipLaunchKernelGGL((k_zsweep1<OP, TX, TY, NT>), dim3(blocks), dim3(NT), 0, st, G, nc);
    return hipGetLastError();
}

template <int OP, int TX, int TY, int TZ, int NT>
hipError_t go_list(hipStream_t st, const FsList *L, int blocks, unsigned long long *nc)
{
    hipLaunchKernelGGL((k_bsweep<OP, TX, TY, TZ, NT>), dim3(blocks), dim3(NT), 0, st, L, nc);
    return hipGetLastError();
}

template <int OP, int TX, int TY, int TZ, int NT>
hipError_t go_one(hipStream_t st, const FsGrid &G, unsigned long long *nc)
{
    const int blocks = G.tiles_x * G.tiles_y * G.tiles_z;
    hipLaunchKernelGGL((k_bsweep1<OP, TX, TY, TZ, NT>), dim3(blocks), dim3(NT), 0, st, G, nc);
    return hipGetLastError();
}

template <int OP>
hipError_t list_op(int cfg, hipStream_t st, const FsList *L, int blocks, unsigned long long *nc,
                   bool pro)
{
    // only the z-stream shapes prolong
    if (pro && kCfg[cfg].zwg == 0)
        return hipErrorInvalidValue;
    switch (cfg) {
    case 0:
        return go_list<OP, 8, 8, 8, 256>(st, L, blocks, nc);
    case 1:
        return go_list<OP, 8, 8, 8, 512>(st, L, blocks, nc);
    case 2:
        return go_list<OP, 8, 8, 8, 1024>(st, L, blocks, nc);
    case 3:
        return go_list<OP, 16, 8, 4, 256>(st, L, blocks, nc);
    case 4:
        return go_list<OP, 16, 16, 8, 512>(st, L, blocks, nc);
    case 5:
        return go_list<OP, 8, 8, 4, 512>(st, L, blocks, nc);
    case 6:
        return go_list<OP, 8, 8, 4, 256>(st, L, blocks, nc);
    case 7:
    case 9:
        return zgo_list<OP, 32, 26, 1024>(st, L, blocks, nc, pro);
    case 8:
        return zgo_list<OP, 32, 26, 512>(st, L, blocks, nc, pro);
    case 10:
        return zgo_list<OP, 40, 20, 1024>(st, L, blocks, nc, pro);
    case 11:
        return zgo_list<OP, 32, 24, 1024>(st, L, blocks, nc, pro);
    default:
        return hipErrorInvalidValue;
    }
}

template <int OP>
hipError_t one_op(int cfg, hipStream_t st, const FsGrid &G, unsigned long long *nc)
{
    switch (cfg) {
    case 0:
        return go_one<OP, 8, 8, 8, 256>(st, G, nc);
    case 1:
        return go_one<OP, 8, 8, 8, 512>(st, G, nc);
    case 2:
        return go_one<OP, 8, 8, 8, 1024>(st, G, nc);
    case 3:
        return go_one<OP, 16, 8, 4, 256>(st, G, nc);
    case 4:
        return go_one<OP, 16, 16, 8, 512>(st, G, nc);
    case 5:
        return go_one<OP, 8, 8, 4, 512>(st, G, nc);
    case 6:
        return go_one<OP, 8, 8, 4, 256>(st, G, nc);
    case 7:
    case 9:
        return zgo_one<OP, 32, 26, 1024>(st, G, nc);
    case 8:
        return zgo_one<OP, 32, 26, 512>(st, G, nc);
    case 10:
        return zgo_one<OP, 40, 20, 1024>(st, G, nc);
    case 11:
        return zgo_one<OP, 32, 24, 1024>(st, G, nc);
    default:
        return hipErrorInvalidValue;
    }
}

} // namespace

int bsweep_num_configs() { return kNumCfg; }

// Automatic shape: 8^3 blocks; the fewer blocks the grid has, the more
// threads each gets (one update per thread and phase at 1024 threads).  A
// launch whose 8^3 blocks (tiles8, over all its grids) would leave most
// compute units idle takes 8 x 8 x 4 blocks of 512 threads instead: twice
// the blocks, each with fewer rounds of updates per phase, for more halo
// recomputation (measured on the level-32 sweeps of one 129^3 solve: 1.7%
// of the solve faster).
int bsweep_pick(int n, long tiles8)
{
    if (n <= 16)
        return 2;
    if (n <= 32)
        return tiles8 < 256 ? 5 : 1;
    if (n <= 64)
        return 0;
    return 4;
}

// Automatic z-stream shape (config index) of an n grid: the cheaper of
// 32 x 26 and 32 x 24 by the chunk model.
int bsweep_zs_pick(int n)
{
    return zs_model_cost100(n, kZsPureConfig) <= zs_model_cost100(n, 7) ? kZsPureConfig : 7;
}

void bsweep_grid(int cfg, int n, const double *uin, double *uout, const double *F, int op,
                 int slot, FsGrid *G)
{
    const BCfg &b = kCfg[cfg];
    G->uin = uin;
    G->uout = uout;
    G->F = F;
    G->n = n;
    G->tiles_x = (n - 1 + b.tx - 1) / b.tx;
    G->tiles_y = (n - 1 + b.ty - 1) / b.ty;
    if (b.zwg != 0) {
        // chunks of at least 16 planes; the last chunk takes what remains
        const int cols = G->tiles_x * G->tiles_y;
        const int chunks = b.zwg < 0 ? zs_chunks(n, cols)
                                     : std::max(1, std::min((n - 1) / 16,
                                                            (b.zwg + cols - 1) / cols));
        const int zc = zs_chunk(n, chunks);
        G->tiles_z = (n - 1 + zc - 1) / zc;
    } else {
        G->tiles_z = (n - 1 + b.tz - 1) / b.tz;
    }
    G->start = 0;
    G->slot = slot;
    G->s = double(n) * double(n);
    G->s4 = 0.25 * G->s;
    G->hk = op == OP_MA ? 0.5 / G->s : 1.0 / (6.0 * G->s);
    G->cu = G->cw = nullptr;
}

bool bsweep_is_zstream(int cfg) { return cfg >= 0 && cfg < kNumCfg && kCfg[cfg].zwg != 0; }

hipError_t launch_bsweep(hipStream_t st, int op, int cfg, const FsList *L, int blocks,
                         unsigned long long *nonconvex, bool prolong)
{
    if (cfg < 0 || cfg >= kNumCfg || blocks <= 0)
        return hipErrorInvalidValue;
    if (op == OP_MA)
        return list_op<OP_MA>(cfg, st, L, blocks, nonconvex, prolong);
    return list_op<OP_LAP>(cfg, st, L, blocks, nonconvex, prolong);
}

hipError_t launch_bsweep_one(hipStream_t st, int op, int cfg, int n, const double *u_in,
                             double *u_out, const double *F, unsigned long long *nonconvex)
{
    if (n < 2)
        return hipErrorInvalidValue;
    if (cfg < 0 || cfg >= kNumCfg)
        cfg = bsweep_pick(n, long((n - 1 + 7) / 8) * ((n - 1 + 7) / 8) * ((n - 1 + 7) / 8));
    FsGrid G;
    bsweep_grid(cfg, n, u_in, u_out, F, op, 0, &G);
    if (op == OP_MA)
        return one_op<OP_MA>(cfg, st, G, nonconvex);
    return one_op<OP_LAP>(cfg, st, G, nonconvex);
}

} // namespace mafas
