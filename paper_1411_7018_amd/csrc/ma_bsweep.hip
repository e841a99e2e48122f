// Launchers of the block sweep (ma_fsweep.h): the block shapes it is built
// for and the automatic choice between them.
#include "ma_fsweep.h"

namespace mafas {

namespace {

struct BCfg {
    int tx, ty, tz, nt;
};
// Block shapes (index = tile_config - 1).  Small blocks keep the
// recomputation cheap in absolute terms and give many workgroups; more
// threads per block cut the rounds of updates per phase, which is what a
// sweep of a small grid waits on.
constexpr BCfg kCfg[] = {{8, 8, 8, 256}, {8, 8, 8, 512},  {8, 8, 8, 1024}, {16, 8, 4, 256},
                         {16, 16, 8, 512}, {8, 8, 4, 512}, {8, 8, 4, 256}};
constexpr int kNumCfg = int(sizeof(kCfg) / sizeof(kCfg[0]));

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
hipError_t list_op(int cfg, hipStream_t st, const FsList *L, int blocks, unsigned long long *nc)
{
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
    G->tiles_z = (n - 1 + b.tz - 1) / b.tz;
    G->start = 0;
    G->slot = slot;
    G->s = double(n) * double(n);
    G->s4 = 0.25 * G->s;
    G->hk = op == OP_MA ? 0.5 / G->s : 1.0 / (6.0 * G->s);
}

hipError_t launch_bsweep(hipStream_t st, int op, int cfg, const FsList *L, int blocks,
                         unsigned long long *nonconvex)
{
    if (cfg < 0 || cfg >= kNumCfg || blocks <= 0)
        return hipErrorInvalidValue;
    if (op == OP_MA)
        return list_op<OP_MA>(cfg, st, L, blocks, nonconvex);
    return list_op<OP_LAP>(cfg, st, L, blocks, nonconvex);
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
