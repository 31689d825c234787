// Internal interface between the host runtime (runtime.hip) and the device
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hydro {

constexpr int kMaxComp = 5;

// Device control block, one per mesh, in the caller's workspace.
struct Ctrl {
    double dt_raw;                  // cfl / (max CFL rate) of the current state
    double t;                       // simulation time
    unsigned long long rate_bits;   // max accumulator: non-negative doubles order as integers
    unsigned int flags;             // sticky error flags
    unsigned int dt_valid;          // dt_raw belongs to the current state
    unsigned long long steps;       // completed steps
    double sums[2 * kMaxComp];      // totals: (sum, compensation) per component
    double t_end;                   // run limit in time (0: none)
    unsigned long long max_steps;   // run limit in steps (0: none)
    unsigned int done;              // a limit is reached: device-dt stages skip this mesh
    unsigned int pad0;
    double pad[6];
};
static_assert(sizeof(Ctrl) == 192, "control block layout");

enum : unsigned int { FLAG_NONPHYSICAL = 1u };

enum CtrlOp : int {
    CTRL_INIT = 0,           // t = a0, steps = 0, flags = 0, dt invalid, no limits
    CTRL_RESET_MIN = 1,      // rate accumulator = 0
    CTRL_FINALIZE_DT = 2,    // dt_raw = cfl / rate, dt valid
    CTRL_FINALIZE_STEP = 3,  // t += clamped dt, steps += 1, dt_raw = cfl / rate, reset, done
    CTRL_ADVANCE_T = 4,      // t += a0 (host dt), dt invalid
    CTRL_SET_LIMITS = 5,     // t_end = a0, max_steps = a1 (relative to the steps done), done
};

// Geometry in kernel axes.  Kernel axis 0 is x.  For 3-D, kernel axes
// (0, 1, 2) are (x, y, z); for 2-D, kernel axis 2 (the marching axis)
// is the physical y axis and kernel axis 1 has extent 1; for 1-D only
// kernel axis 0 is active.  The cell index (k * n1 + j) * n0 + i is the
// physical storage index in every case.
//
// A mesh may be split into blocks[0] x blocks[1] x blocks[2] blocks of equal
// extents (kernel axes); n and ncells are those of one block.  Fields are
// stored block after block, [block][comp][cell of the block], with block
// index b0 + blocks[0] (b1 + blocks[1] b2).  The boundary codes are those of
// the whole mesh: a side of a block inside the mesh, or on a periodic axis,
// reads its ghosts from the neighbouring block (a c-boundary); one block on a
// periodic axis is its own neighbour.
struct Geo {
    int ndim;
    int n[3];
    int blocks[3];
    double dx[3];
    double inv_dx[3];
    int bc[3][2];
    double gamma;
    double cfl;
    long long ncells;
};

struct Tile {
    int tx, ty, kz;
};

struct StageArgs {
    const double* in;    // stencil source: U^n (stage 1 / rhs) or U1 (stage 2)
    const double* base;  // U^n for the stage-2 combine (may alias out)
    double* out;         // U1, U^{n+1} (in place over base) or the increment
    Ctrl* ctrl;
    Geo geo;
    double dt_host;      // dt when use_device_dt == 0
    int use_device_dt;   // dt from ctrl (clamped to its t_end); skip the mesh when done
    int want_dt;         // stage 2: accumulate the next CFL candidate
    int tiles_x, tiles_y, chunks_z, kz;  // per block
    int blk0, nblk;      // the launch covers blocks blk0 .. blk0 + nblk - 1
    int conc;            // blocks whose stage work runs at once (automatic chunk length)
    // static refinement: per block 6 side codes (else null: the uniform
    // block grid of geo), and the ghost slots of the sides at level jumps
    const int* side;
    const double* gbuf;
    long long gcs;       // component stride within a ghost slot (slot = ncomp * gcs)
};

// Side codes of a refined mesh's blocks, [block][kernel axis][low, high]:
// >= 0 the block of the same level across the side; kSidePhys a face of the
// mesh (its boundary rule); kSideSlot0 - q the ghost slot q, which holds the
// two ghost layers of the side, [comp][layer][t_hi][t_lo] over the side's two
// transverse kernel axes (t_lo the lower), layer 0 next to the face.
constexpr int kSidePhys = -1;
constexpr int kSideSlot0 = -2;

// One ghost slot: the side (ax, s) of block `leaf` at a level jump.
// kind 0 (restriction; leaf is coarse): src[o] is the fine block on the face
// at transverse child offsets o (bit 0: t_lo, bit 1: t_hi).  kind 1
// (prolongation; leaf is fine): src[0] is the coarse block, child[] the
// leaf's offsets (0/1) per kernel axis within its parent.  lev: the leaf's
// refinement level (its cell widths are level 0's times 2^-lev).
struct GhostTask {
    int leaf, ax, s, kind;
    int src[4];
    int child[3];
    int slot;
    int lev;
};

// Refinement levels 0 .. kMaxLevels - 1; a refined block is named by the code
// level * 2^kLevelShift + its index on that level's block grid.
constexpr int kMaxLevels = 4;
constexpr int kLevelShift = 26;

// First block of each level 1 .. kMaxLevels - 1 in a refined mesh's leaf
// order (a level with no leaves starts where the next one does; unrefined
// meshes: every entry at the block count).
struct LevelStarts {
    int s[kMaxLevels - 1];
};

// One member of a batch: the stage kernels build StageArgs from it.
struct MeshDesc {
    double* U;
    double* U1;
    Ctrl* ctrl;
    Geo geo;
    int tiles_x, tiles_y, chunks_z, kz;
};

// Stage kernels: the Heun stages (and the stage right-hand side), and the
// van Leer predictor and corrector (Sec. 3.3).  The _C forms keep the
// predicted state conserved in FP64 (a refined mesh, whose level-jump passes
// read conserved stage inputs): the predictor writes U* = U^n + (dt/2) L_1(U^n)
// and the corrector reads U* as its stencil input.
enum StageMode : int {
    MODE_RHS = 0,
    MODE_STAGE1 = 1,
    MODE_STAGE2 = 2,
    MODE_VL2_PRED = 3,
    MODE_VL2_CORR = 4,
    MODE_VL2_PRED_C = 5,
    MODE_VL2_CORR_C = 6
};

hipError_t launch_stage(int precision, int mode, const Tile& tile, StageArgs a, hipStream_t s);
// The same launch described (kernel, grid, block, arguments) instead of
// enqueued, for a caller that adds it to a graph as a kernel node.
struct StageLaunch {
    const void* func;
    dim3 grid, block;
    StageArgs args;
};
hipError_t plan_stage_launch(int precision, int mode, const Tile& tile, StageArgs a, StageLaunch* out);
// Fill the tiling fields of a descriptor for a tile.
void plan_tiles(const Geo& g, const Tile& t, int& tiles_x, int& tiles_y, int& chunks_z, int& kz);
// One stage over every mesh of a group sharing ndim, precision and tile:
// blk[i] = (member, work-group within the member), nblk entries.
hipError_t launch_stage_batch(int ndim, int precision, int mode, const Tile& tile, const MeshDesc* d,
                              const int2* blk, int nblk, hipStream_t s);
// (done, flags, steps) of members [0, n) of a descriptor table into out[3 i ..].
hipError_t launch_status_gather(const MeshDesc* d, int n, unsigned long long* out, hipStream_t s);
// CTRL_FINALIZE_STEP for members [0, n) of a descriptor table.
hipError_t launch_ctrl_batch(const MeshDesc* d, int n, hipStream_t s);
hipError_t launch_dt(const Geo& g, const double* U, Ctrl* ctrl, hipStream_t s);
hipError_t launch_ctrl(Ctrl* c, int op, double a0, double a1, double cfl, hipStream_t s);
hipError_t launch_totals(const Geo& g, const double* U, double* partials, int nparts, Ctrl* ctrl,
                         hipStream_t s);
// The same reduction, written as out[c] = dV (sum + compensation) on the
// device (partials: 2 ncomp nparts doubles of scratch).
hipError_t launch_totals_out(const Geo& g, const double* U, double* partials, int nparts, double* out, double dV,
                             hipStream_t s);
// W and U in the block layout; in place when W == U.
hipError_t launch_prim_to_cons(const Geo& g, const double* W, double* U, hipStream_t s);
// Copy a field between the mesh layout [comp][k][j][i] (mesh) and the block
// layout (blk): to_blocks != 0 reads mesh and writes blk, else the reverse.
hipError_t launch_relayout(const Geo& g, double* mesh, double* blk, int to_blocks, hipStream_t s);
hipError_t launch_padded_prim(const Geo& g, int precision, const double* U, double* Wpad, Ctrl* ctrl,
                              hipStream_t s);
hipError_t launch_riemann(int precision, int ntan, double gamma, long long n, const double* WL,
                          const double* WR, double* F, hipStream_t s);

// Static refinement passes over the ghost slots tasks[0, n) (all of one
// kind): restriction or prolongation of the stage input U into gbuf
// (conserved FP64 values); the fine-flux corrections of the coarse cells next
// to every level jump, from the stage input in, into dbuf (factor * lam *
// (coarse flux - mean of the fine fluxes), [slot][comp][face]; first: fluxes
// of piecewise-constant states, as in the van Leer predictor); and their
// addition to out for the restriction slots idx0 .. idx0 + n - 1 of one
// kernel axis.  g0 and g1 are the coarse and fine levels' geometries.
hipError_t launch_smr_restrict(const Geo& g, const double* U, const int* side, double* gbuf, long long gcs,
                               const GhostTask* tasks, int n, Ctrl* ctrl, hipStream_t s);
hipError_t launch_smr_prolong(const Geo& g, const double* U, const int* side, double* gbuf, long long gcs,
                              const GhostTask* tasks, int n, Ctrl* ctrl, hipStream_t s);
hipError_t launch_smr_reflux(int precision, int first, const Geo& g0, const Geo& g1, const double* in,
                             double* dbuf, double factor, int use_device_dt, double dt_host, const int* side,
                             const double* gbuf, long long gcs, const GhostTask* tasks, int n, Ctrl* ctrl,
                             hipStream_t s);
hipError_t launch_smr_apply(const Geo& g0, double* out, const double* dbuf, long long gcs, const GhostTask* tasks,
                            int idx0, int n, int use_device_dt, Ctrl* ctrl, hipStream_t s);
// dt reduction over the nblk blocks of U, a block of level L (from the level
// starts) with g0's cell widths times 2^-L; with skip_done, nothing once the
// run limit is reached.
hipError_t launch_dt_levels(const Geo& g0, const LevelStarts& starts, int nblk, const double* U, Ctrl* ctrl,
                            int skip_done, hipStream_t s);

// Default tile for a mesh (kernel axes) and precision.
Tile default_tile(const Geo& g, int precision, int mode);
// Whether the stage kernel is compiled for this tile shape.
// Bounds of the automatic chunk length (Tile::kz == 0).
constexpr int kMinAutoKz = 16;
constexpr int kMaxAutoKz = 128;

bool tile_supported(int ndim, const Tile& t);
// Tiles the autotuner tries for a mesh (at most max written); returns how
// many there are.
int tile_candidates(const Geo& g, Tile* out, int max);
// Number of totals partials the runtime reserves.
constexpr int kTotalsParts = 1024;
// Blocks of one mesh: each needs one totals partial at least.
constexpr int kMaxBlocks = kTotalsParts;

__host__ __device__ inline int geo_nblk(const Geo& g) { return g.blocks[0] * g.blocks[1] * g.blocks[2]; }

}  // namespace hydro
