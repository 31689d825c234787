// Host runtime behind include/hydro.h: configuration checks, workspace
// carving, stream-ordered launches and the device-resident time step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "hydro.h"
#include "hydro_internal.h"

using namespace hydro;

// Streams the blocks of a split mesh are spread over when launched one by
// one (the hardware offers four queues per process by default).
constexpr int kBlockStreams = 4;

struct hydro_ctx {
    hydro_config cfg;
    Geo geo;
    int nblk;         // blocks of the mesh (geo holds one block's extents)
    // per-block launches on their own streams (Sec. 3: one stream per block)
    bool block_streams;
    int nbs;                       // streams created (0: none yet)
    hipStream_t bs[kBlockStreams];
    hipEvent_t ev_fork;
    hipEvent_t ev_join[kBlockStreams];
    hipEvent_t* ev_s1;             // per stream's block group: its stage 1 has finished
    int* nbr;                      // per block: up to 6 distinct face neighbours, -1 padded
    // block group g = blocks [g nblk / nbs, (g + 1) nblk / nbs) runs on stream g;
    // gadj[g][o]: a block of group o is a face neighbour of a block of group g
    bool gadj[kBlockStreams][kBlockStreams];
    // static refinement (leaves ordered by level)
    bool smr;
    int nlev;                      // levels present
    int lev_start[kMaxLevels], lev_count[kMaxLevels];
    Geo lgeo[kMaxLevels];          // per level: one block's extents and the level's cell widths
    int* d_side;                   // 6 side codes per leaf
    GhostTask* d_tasks;            // restriction slots by kernel axis, then prolongation slots
    int nres, npro, res_off[4];
    int pro_off[kMaxLevels + 1];   // prolongation slots of level L: tasks [pro_off[L], pro_off[L + 1])
    double* gbuf;
    double* dbuf;                  // flux corrections per restriction slot
    hipStream_t smr_aux;           // second stream of the level-jump passes (null: none)
    hipEvent_t ev_smr[3];          // restriction done, prolongation done, recomputation done
    long long gcs;
    int32_t* leaves;               // host: (level, c0, c1, c2) per leaf
    Tile tile[2];  // stage 1 (and the rhs), stage 2
    hipStream_t stream;
    int ncomp;
    double dV;
    double* U;      // current state U^n
    double* U1;     // predictor U1 / scratch
    double* parts;  // totals partials
    Ctrl* ctrl;
    Ctrl* host_ctrl;  // host mirror for reads (pageable: no pinning or unpinning per handle)
    bool broken;
    bool dt_valid;    // ctrl->dt_raw belongs to the current state (host-side knowledge)
    // optional event timing of the stage launches
    int prof_cap;
    int prof_n[2];
    hipEvent_t* prof_ev[2];  // [stage][2 * launch + {0: start, 1: stop}]
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int blocks_of(const hydro_config* c, int d) { return c->blocks[d] == 0 ? 1 : c->blocks[d]; }

bool config_ok(const hydro_config* c) {
    if (!c) return false;
    if (c->ndim < 1 || c->ndim > 3) return false;
    if (!(c->gamma > 1.0) || !std::isfinite(c->gamma)) return false;
    if (!(c->cfl > 0.0) || !(c->cfl <= 1.0)) return false;
    if (c->precision != HYDRO_FP64 && c->precision != HYDRO_MIXED) return false;
    if (c->integrator != HYDRO_HEUN && c->integrator != HYDRO_VL2) return false;
    long long cells = 1;
    for (int d = 0; d < 3; ++d) {
        if (d < c->ndim) {
            if (c->n[d] < 1) return false;
            if (!(c->hi[d] > c->lo[d]) || !std::isfinite(c->hi[d] - c->lo[d])) return false;
            for (int s = 0; s < 2; ++s)
                if (c->bc[d][s] < HYDRO_BC_PERIODIC || c->bc[d][s] > HYDRO_BC_REFLECT) return false;
            const bool p0 = c->bc[d][0] == HYDRO_BC_PERIODIC, p1 = c->bc[d][1] == HYDRO_BC_PERIODIC;
            if (p0 != p1) return false;
            // periodic and reflecting ghosts read two distinct interior cells
            if ((p0 || c->bc[d][0] == HYDRO_BC_REFLECT || c->bc[d][1] == HYDRO_BC_REFLECT) &&
                c->n[d] < 2)
                return false;
        } else if (c->n[d] != 1) {
            return false;
        }
        // blocks of equal extents; a neighbour supplies both ghost layers of
        // a shared face, so a split axis gives every block two cells at least
        const int B = blocks_of(c, d);
        if (B < 1 || (d >= c->ndim && B != 1) || c->n[d] % B != 0 || (B > 1 && c->n[d] / B < 2)) return false;
        cells *= c->n[d];
        if (cells > (1ll << 40)) return false;
    }
    if ((long long)blocks_of(c, 0) * blocks_of(c, 1) * blocks_of(c, 2) > kMaxBlocks) return false;
    // the stage kernels address one plane of the marching axis (x-y in 3-D,
    // a row in 1-D and 2-D) of a block with 32-bit byte offsets
    const long long plane = (long long)(c->n[0] / blocks_of(c, 0)) * (c->ndim == 3 ? c->n[1] / blocks_of(c, 1) : 1);
    if (plane * 8 >= (1ll << 32)) return false;
    return true;
}

long long ncells_of(const hydro_config* c) { return (long long)c->n[0] * c->n[1] * c->n[2]; }

size_t state_bytes(const hydro_config* c) {
    return align_up((size_t)(c->ndim + 2) * (size_t)ncells_of(c) * sizeof(double));
}

// The second field: the Heun predictor U1 (FP64), or the van Leer predicted
// primitive state in the compute precision.
size_t second_bytes(const hydro_config* c) {
    if (c->integrator == HYDRO_HEUN) return state_bytes(c);
    const size_t r = c->precision == HYDRO_FP64 ? sizeof(double) : sizeof(float);
    return align_up((size_t)(c->ndim + 2) * (size_t)ncells_of(c) * r);
}

int stage1_mode(const hydro_config* c) { return c->integrator == HYDRO_VL2 ? MODE_VL2_PRED : MODE_STAGE1; }
int stage2_mode(const hydro_config* c) { return c->integrator == HYDRO_VL2 ? MODE_VL2_CORR : MODE_STAGE2; }
// Stage st of a refined mesh: the van Leer predictor stays conserved FP64,
// since the level-jump passes read conserved stage inputs.
int smr_mode(const hydro_config* c, int st) {
    if (c->integrator == HYDRO_VL2) return st == 0 ? MODE_VL2_PRED_C : MODE_VL2_CORR_C;
    return st == 0 ? MODE_STAGE1 : MODE_STAGE2;
}

// Kernel-axis geometry of one block (see hydro_internal.h).
Geo make_geo(const hydro_config* c) {
    Geo g;
    std::memset(&g, 0, sizeof(g));
    g.ndim = c->ndim;
    g.gamma = c->gamma;
    g.cfl = c->cfl;
    g.ncells = ncells_of(c) / ((long long)blocks_of(c, 0) * blocks_of(c, 1) * blocks_of(c, 2));
    double dx[3];
    for (int d = 0; d < 3; ++d) dx[d] = d < c->ndim ? (c->hi[d] - c->lo[d]) / c->n[d] : 1.0;
    int map[3];  // kernel axis -> physical axis (-1: inactive)
    if (c->ndim == 3) {
        map[0] = 0; map[1] = 1; map[2] = 2;
    } else if (c->ndim == 2) {
        map[0] = 0; map[1] = -1; map[2] = 1;
    } else {
        map[0] = 0; map[1] = -1; map[2] = -1;
    }
    for (int k = 0; k < 3; ++k) {
        if (map[k] >= 0) {
            g.blocks[k] = blocks_of(c, map[k]);
            g.n[k] = c->n[map[k]] / g.blocks[k];
            g.dx[k] = dx[map[k]];
            g.inv_dx[k] = 1.0 / dx[map[k]];
            g.bc[k][0] = c->bc[map[k]][0];
            g.bc[k][1] = c->bc[map[k]][1];
        } else {
            g.n[k] = 1;
            g.blocks[k] = 1;
            g.dx[k] = 1.0;
            g.inv_dx[k] = 1.0;
            g.bc[k][0] = g.bc[k][1] = HYDRO_BC_PERIODIC;
        }
    }
    return g;
}

int fail(hydro_t h, hipError_t e) {
    if (e == hipSuccess) return HYDRO_OK;
    if (h) h->broken = true;
    return HYDRO_E_DEVICE;
}

int read_ctrl(hydro_t h) {
    hipError_t e = hipMemcpyAsync(h->host_ctrl, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(h, e);
    if (h->host_ctrl->flags & FLAG_NONPHYSICAL) return HYDRO_E_NONPHYSICAL;
    return HYDRO_OK;
}

int usable(hydro_t h) {
    if (!h) return HYDRO_E_INVAL;
    if (h->broken) return HYDRO_E_STATE;
    return HYDRO_OK;
}

// Arguments of a launch over every block of the mesh.
StageArgs stage_args(hydro_t h) {
    StageArgs a;
    std::memset(&a, 0, sizeof(a));
    a.ctrl = h->ctrl;
    a.geo = h->geo;
    a.blk0 = 0;
    a.nblk = h->nblk;
    a.conc = h->nblk;
    a.side = h->smr ? h->d_side : nullptr;
    a.gbuf = h->gbuf;
    a.gcs = h->gcs;
    return a;
}

// Distinct face neighbours of every block (the blocks whose stage-1 output
// a block's stage 2 reads, and which read the state its stage 2 overwrites).
void block_neighbours(hydro_t h) {
    const Geo& g = h->geo;
    for (int b = 0; b < h->nblk; ++b) {
        int* out = h->nbr + 6 * b;
        int k = 0;
        for (int q = 0; q < 6; ++q) out[q] = -1;
        const int c[3] = {b % g.blocks[0], (b / g.blocks[0]) % g.blocks[1], b / (g.blocks[0] * g.blocks[1])};
        for (int ax = 0; ax < 3; ++ax)
            for (int side = 0; side < 2; ++side) {
                int cc[3] = {c[0], c[1], c[2]};
                int q = cc[ax] + (side ? 1 : -1);
                if (q < 0 || q >= g.blocks[ax]) {
                    if (g.bc[ax][side] != HYDRO_BC_PERIODIC) continue;
                    q = (q + g.blocks[ax]) % g.blocks[ax];
                }
                cc[ax] = q;
                const int nb = cc[0] + g.blocks[0] * (cc[1] + g.blocks[1] * cc[2]);
                bool seen = nb == b;
                for (int i = 0; i < k; ++i) seen = seen || out[i] == nb;
                if (!seen) out[k++] = nb;
            }
    }
}

void block_streams_free(hydro_t h) {
    for (int i = 0; i < h->nbs; ++i) {
        (void)hipStreamDestroy(h->bs[i]);
        (void)hipEventDestroy(h->ev_join[i]);
    }
    if (h->nbs > 0) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_s1)
        for (int b = 0; b < h->nblk; ++b) (void)hipEventDestroy(h->ev_s1[b]);
    delete[] h->ev_s1;
    delete[] h->nbr;
    h->ev_s1 = nullptr;
    h->nbr = nullptr;
    h->nbs = 0;
}

// The stream group of block b (contiguous ranges, nbs of them).
int block_group(hydro_t h, int b) {
    int g = (int)(((long long)b * h->nbs) / h->nblk);
    while (g > 0 && b < (int)(((long long)g * h->nblk) / h->nbs)) --g;
    while (g + 1 < h->nbs && b >= (int)(((long long)(g + 1) * h->nblk) / h->nbs)) ++g;
    return g;
}

// Streams and events of the per-group launches, made on first use.
hipError_t block_streams_make(hydro_t h) {
    if (h->nbs > 0) return hipSuccess;
    h->nbr = new (std::nothrow) int[6 * (size_t)h->nblk];
    h->ev_s1 = new (std::nothrow) hipEvent_t[h->nblk];
    if (!h->nbr || !h->ev_s1) {
        delete[] h->nbr;
        delete[] h->ev_s1;
        h->nbr = nullptr;
        h->ev_s1 = nullptr;
        return hipErrorOutOfMemory;
    }
    block_neighbours(h);
    int made = 0;
    hipError_t e = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming);
    for (; made < h->nblk && e == hipSuccess; ++made) e = hipEventCreateWithFlags(&h->ev_s1[made], hipEventDisableTiming);
    if (e != hipSuccess) --made;
    const int ns = std::min(h->nblk, kBlockStreams);
    int nstreams = 0;
    for (; nstreams < ns && e == hipSuccess; ++nstreams) {
        // default priority, not synchronising with the legacy default stream
        e = hipStreamCreateWithFlags(&h->bs[nstreams], hipStreamNonBlocking);
        if (e == hipSuccess) {
            e = hipEventCreateWithFlags(&h->ev_join[nstreams], hipEventDisableTiming);
            if (e != hipSuccess) (void)hipStreamDestroy(h->bs[nstreams]);
        }
    }
    if (e != hipSuccess) {
        --nstreams;
        for (int i = 0; i < nstreams; ++i) {
            (void)hipStreamDestroy(h->bs[i]);
            (void)hipEventDestroy(h->ev_join[i]);
        }
        for (int b = 0; b < made; ++b) (void)hipEventDestroy(h->ev_s1[b]);
        if (made >= 0) (void)hipEventDestroy(h->ev_fork);
        delete[] h->ev_s1;
        delete[] h->nbr;
        h->ev_s1 = nullptr;
        h->nbr = nullptr;
        return e;
    }
    h->nbs = ns;
    for (int g = 0; g < ns; ++g)
        for (int o = 0; o < ns; ++o) h->gadj[g][o] = false;
    for (int b = 0; b < h->nblk; ++b)
        for (int q = 0; q < 6; ++q) {
            const int nb = h->nbr[6 * b + q];
            if (nb >= 0) h->gadj[block_group(h, b)][block_group(h, nb)] = true;
        }
    return hipSuccess;
}

// One step with the blocks' stages launched by group, each group of
// contiguous blocks on a stream of its own: stage 1 of every group, then
// stage 2 of a group once the groups holding its blocks' face neighbours have
// finished stage 1 (no wait on the others), then the step's finalisation on
// the handle's stream after every group.
hipError_t enqueue_step_streams(hydro_t h, bool device_dt, double dt) {
    StageArgs a = stage_args(h);
    a.use_device_dt = device_dt ? 1 : 0;
    a.dt_host = dt;
    a.conc = h->nblk;  // the groups run at once
    hipError_t e = hipEventRecord(h->ev_fork, h->stream);
    for (int i = 0; i < h->nbs && e == hipSuccess; ++i) e = hipStreamWaitEvent(h->bs[i], h->ev_fork, 0);
    auto range = [&](int g) {
        a.blk0 = (int)(((long long)g * h->nblk) / h->nbs);
        a.nblk = (int)(((long long)(g + 1) * h->nblk) / h->nbs) - a.blk0;
    };
    for (int g = 0; g < h->nbs && e == hipSuccess; ++g) {
        range(g);
        a.in = h->U;
        a.base = h->U;
        a.out = h->U1;
        a.want_dt = 0;
        e = launch_stage(h->cfg.precision, stage1_mode(&h->cfg), h->tile[0], a, h->bs[g]);
        if (e == hipSuccess) e = hipEventRecord(h->ev_s1[g], h->bs[g]);
    }
    for (int g = 0; g < h->nbs && e == hipSuccess; ++g) {
        // it reads their stage-1 output, and they read the state it overwrites
        for (int o = 0; o < h->nbs && e == hipSuccess; ++o)
            if (o != g && h->gadj[g][o]) e = hipStreamWaitEvent(h->bs[g], h->ev_s1[o], 0);
        range(g);
        a.in = h->U1;
        a.base = h->U;
        a.out = h->U;
        a.want_dt = device_dt ? 1 : 0;
        if (e == hipSuccess) e = launch_stage(h->cfg.precision, stage2_mode(&h->cfg), h->tile[1], a, h->bs[g]);
    }
    for (int i = 0; i < h->nbs && e == hipSuccess; ++i) {
        e = hipEventRecord(h->ev_join[i], h->bs[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(h->stream, h->ev_join[i], 0);
    }
    if (e != hipSuccess) return e;
    if (device_dt) return launch_ctrl(h->ctrl, CTRL_FINALIZE_STEP, 0.0, 0.0, h->cfg.cfl, h->stream);
    return launch_ctrl(h->ctrl, CTRL_ADVANCE_T, dt, 0.0, h->cfg.cfl, h->stream);
}

// The same step while the handle's stream is captured into a graph: the
// per-group stage launches become kernel nodes of the capture's graph with
// the same dependencies (stage 1 of every group after what the stream had
// captured; stage 2 of a group after stage 1 of its own group and of the
// groups holding its blocks' face neighbours), the stream's capture then
// continues from the stage-2 nodes.  No other stream and no event joins the
// capture.
hipError_t enqueue_step_streams_graph(hydro_t h, bool device_dt, double dt) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    unsigned long long id = 0;
    hipGraph_t graph = nullptr;
    const hipGraphNode_t* deps = nullptr;
    size_t nd = 0;
    hipError_t e = hipStreamGetCaptureInfo_v2(h->stream, &st, &id, &graph, &deps, &nd);
    if (e != hipSuccess) return e;
    if (st != hipStreamCaptureStatusActive || !graph) return hipErrorIllegalState;
    const std::vector<hipGraphNode_t> d0(deps, deps + nd);  // valid until the next capture call
    StageArgs a = stage_args(h);
    a.use_device_dt = device_dt ? 1 : 0;
    a.dt_host = dt;
    a.conc = h->nblk;  // the groups run at once
    auto range = [&](int g) {
        a.blk0 = (int)(((long long)g * h->nblk) / h->nbs);
        a.nblk = (int)(((long long)(g + 1) * h->nblk) / h->nbs) - a.blk0;
    };
    auto add = [&](int mode, const Tile& t, const std::vector<hipGraphNode_t>& dep, hipGraphNode_t* node) {
        StageLaunch L;
        hipError_t r = plan_stage_launch(h->cfg.precision, mode, t, a, &L);
        if (r != hipSuccess) return r;
        void* args[] = {&L.args};
        hipKernelNodeParams p;
        std::memset(&p, 0, sizeof(p));
        p.func = const_cast<void*>(L.func);
        p.gridDim = L.grid;
        p.blockDim = L.block;
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        return hipGraphAddKernelNode(node, graph, dep.empty() ? nullptr : dep.data(), dep.size(), &p);
    };
    std::vector<hipGraphNode_t> s1(h->nbs, nullptr), s2(h->nbs, nullptr);
    for (int g = 0; g < h->nbs && e == hipSuccess; ++g) {
        range(g);
        a.in = h->U;
        a.base = h->U;
        a.out = h->U1;
        a.want_dt = 0;
        e = add(stage1_mode(&h->cfg), h->tile[0], d0, &s1[g]);
    }
    for (int g = 0; g < h->nbs && e == hipSuccess; ++g) {
        // it reads their stage-1 output, and they read the state it overwrites
        std::vector<hipGraphNode_t> dep{s1[g]};
        for (int o = 0; o < h->nbs; ++o)
            if (o != g && h->gadj[g][o]) dep.push_back(s1[o]);
        range(g);
        a.in = h->U1;
        a.base = h->U;
        a.out = h->U;
        a.want_dt = device_dt ? 1 : 0;
        e = add(stage2_mode(&h->cfg), h->tile[1], dep, &s2[g]);
    }
    if (e == hipSuccess)
        e = hipStreamUpdateCaptureDependencies(h->stream, s2.data(), s2.size(), hipStreamSetCaptureDependencies);
    if (e != hipSuccess) return e;
    if (device_dt) return launch_ctrl(h->ctrl, CTRL_FINALIZE_STEP, 0.0, 0.0, h->cfg.cfl, h->stream);
    return launch_ctrl(h->ctrl, CTRL_ADVANCE_T, dt, 0.0, h->cfg.cfl, h->stream);
}

// Whether host transfers convert between the mesh layout and the block
// layout: a split mesh; a refined mesh's transfers use the block layout.
bool mesh_relayout(hydro_t h) { return h->nblk > 1 && !h->smr; }

// Mesh-layout buffer on the handle's stream for a split mesh's transfers.
hipError_t mesh_tmp(hydro_t h, double** d) {
    return hipMallocAsync((void**)d, (size_t)h->ncomp * h->geo.ncells * h->nblk * sizeof(double), h->stream);
}

hipError_t free_tmp(hydro_t h, double* d, hipError_t e) {
    if (!d) return e;
    const hipError_t e2 = hipFreeAsync(d, h->stream);
    return e == hipSuccess ? e2 : e;
}

// Launch one stage, bracketed by events when profiling is on.
hipError_t timed_stage(hydro_t h, int mode, const StageArgs& a) {
    const int st = (mode == MODE_STAGE2 || mode == MODE_VL2_CORR || mode == MODE_VL2_CORR_C) ? 1 : 0;
    const bool rec = h->prof_cap > 0 && h->prof_n[st] < h->prof_cap;
    hipError_t e = hipSuccess;
    if (rec) e = hipEventRecord(h->prof_ev[st][2 * h->prof_n[st]], h->stream);
    if (e == hipSuccess) e = launch_stage(h->cfg.precision, mode, h->tile[st], a, h->stream);
    if (rec && e == hipSuccess) {
        e = hipEventRecord(h->prof_ev[st][2 * h->prof_n[st] + 1], h->stream);
        h->prof_n[st] += 1;
    }
    return e;
}

// One step: stage 1 (Heun: U1 = U^n + dt L(U^n); van Leer: the predicted
// primitive state) then stage 2 in place over U^n, dt either from the host or
// from the device control block (clamped to the run limit kept there).
// Whether the handle's stream is being captured into a graph.  The forms
// that fork work onto other streams and join it back by events are then not
// captured as such: capturing that form (group streams waiting on each
// other's events) crashed the host process in the HIP runtime at the end of
// the capture.  The block-stream step is captured as explicit graph nodes
// with the same dependencies instead (enqueue_step_streams_graph), and a
// refined mesh's second stream runs on the handle's stream.  The results do
// not depend on the form.
bool capturing(hydro_t h) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(h->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// The first leaf of each level 1 .. kMaxLevels - 1 of a refined mesh.
LevelStarts level_starts(hydro_t h) {
    LevelStarts ls;
    for (int L = 1; L < kMaxLevels; ++L) ls.s[L - 1] = L < h->nlev ? h->lev_start[L] : h->nblk;
    return ls;
}

// One step of a refined mesh (Heun, or van Leer with its predicted state
// conserved in U1).  Each stage: the ghost slots of the level jumps from the
// stage input (restriction, then prolongation level by level from the
// coarsest, since a coarse block's stencil may include its own prolonged
// slots), the stage kernel per level, then the flux correction of the coarse
// cells at the level jumps (computed for every jump in one launch, added axis
// by axis: a cell next to two jumps is corrected once per axis, in order).
// The correction's weight: Heun 1 after stage 1 and 1/2 after stage 2 (the
// stage-2 update averages with U^n); van Leer 1/2 after the predictor (half
// a step, fluxes of piecewise-constant states) and 1 after the corrector.
// The CFL rate of the corrected state is a reduction of its own.
hipError_t enqueue_step_smr(hydro_t h, bool device_dt, double dt) {
    hipError_t e = hipSuccess;
    // With a second stream (smr_aux), the passes that the level-0 stage does
    // not need overlap it: the prolongations (read only by the finer levels)
    // and the flux recomputation (reads the stage input and the slots, not
    // the stage's output); the finer levels wait for the prolongations, the
    // additions for the recomputation.
    const bool fork = h->smr_aux && !capturing(h);
    hipStream_t aux = fork ? h->smr_aux : h->stream;
    const bool vl2 = h->cfg.integrator == HYDRO_VL2;
    for (int st = 0; st < 2 && e == hipSuccess; ++st) {
        const int first = vl2 && st == 0 ? 1 : 0;
        const double factor = vl2 ? (st == 0 ? 0.5 : 1.0) : (st == 0 ? 1.0 : 0.5);
        const double* in = st == 0 ? h->U : h->U1;
        double* out = st == 0 ? h->U1 : h->U;
        e = launch_smr_restrict(h->lgeo[0], in, h->d_side, h->gbuf, h->gcs, h->d_tasks, h->nres, h->ctrl, h->stream);
        if (e == hipSuccess && fork) e = hipEventRecord(h->ev_smr[0], h->stream);
        if (e == hipSuccess && fork) e = hipStreamWaitEvent(aux, h->ev_smr[0], 0);
        for (int L = 1; L < h->nlev && e == hipSuccess; ++L)
            e = launch_smr_prolong(h->lgeo[0], in, h->d_side, h->gbuf, h->gcs, h->d_tasks + h->pro_off[L],
                                   h->pro_off[L + 1] - h->pro_off[L], h->ctrl, aux);
        if (e == hipSuccess && fork) e = hipEventRecord(h->ev_smr[1], aux);
        if (e == hipSuccess)
            e = launch_smr_reflux(h->cfg.precision, first, h->lgeo[0], h->lgeo[0], in, h->dbuf, factor,
                                  device_dt ? 1 : 0, dt, h->d_side, h->gbuf, h->gcs, h->d_tasks, h->nres, h->ctrl,
                                  aux);
        if (e == hipSuccess && fork) e = hipEventRecord(h->ev_smr[2], aux);
        for (int lev = 0; lev < h->nlev && e == hipSuccess; ++lev) {
            if (lev == 1 && fork) e = hipStreamWaitEvent(h->stream, h->ev_smr[1], 0);
            if (e != hipSuccess || h->lev_count[lev] == 0) continue;
            StageArgs a = stage_args(h);
            a.geo = h->lgeo[lev];
            a.blk0 = h->lev_start[lev];
            a.nblk = a.conc = h->lev_count[lev];
            a.use_device_dt = device_dt ? 1 : 0;
            a.dt_host = dt;
            a.in = in;
            a.base = h->U;
            a.out = out;
            a.want_dt = 0;
            e = timed_stage(h, smr_mode(&h->cfg, st), a);
        }
        if (e == hipSuccess && fork) e = hipStreamWaitEvent(h->stream, h->ev_smr[2], 0);
        for (int ax = 0; ax < 3 && e == hipSuccess; ++ax)
            e = launch_smr_apply(h->lgeo[0], out, h->dbuf, h->gcs, h->d_tasks + h->res_off[ax], h->res_off[ax],
                                 h->res_off[ax + 1] - h->res_off[ax], device_dt ? 1 : 0, h->ctrl, h->stream);
    }
    if (e != hipSuccess) return e;
    if (!device_dt) return launch_ctrl(h->ctrl, CTRL_ADVANCE_T, dt, 0.0, h->cfg.cfl, h->stream);
    e = launch_dt_levels(h->lgeo[0], level_starts(h), h->nblk, h->U, h->ctrl, 1, h->stream);
    if (e != hipSuccess) return e;
    return launch_ctrl(h->ctrl, CTRL_FINALIZE_STEP, 0.0, 0.0, h->cfg.cfl, h->stream);
}

hipError_t enqueue_step(hydro_t h, bool device_dt, double dt) {
    if (h->smr) return enqueue_step_smr(h, device_dt, dt);
    if (h->block_streams && h->nblk > 1 && h->nbs > 0)
        return capturing(h) ? enqueue_step_streams_graph(h, device_dt, dt) : enqueue_step_streams(h, device_dt, dt);
    StageArgs a = stage_args(h);
    a.use_device_dt = device_dt ? 1 : 0;
    a.dt_host = dt;
    a.in = h->U;
    a.base = h->U;
    a.out = h->U1;
    hipError_t e = timed_stage(h, stage1_mode(&h->cfg), a);
    if (e != hipSuccess) return e;
    a.in = h->U1;
    a.base = h->U;
    a.out = h->U;
    a.want_dt = device_dt ? 1 : 0;
    e = timed_stage(h, stage2_mode(&h->cfg), a);
    if (e != hipSuccess) return e;
    if (device_dt) return launch_ctrl(h->ctrl, CTRL_FINALIZE_STEP, 0.0, 0.0, h->cfg.cfl, h->stream);
    return launch_ctrl(h->ctrl, CTRL_ADVANCE_T, dt, 0.0, h->cfg.cfl, h->stream);
}

hipError_t enqueue_dt(hydro_t h) {
    hipError_t e = launch_ctrl(h->ctrl, CTRL_RESET_MIN, 0.0, 0.0, h->cfg.cfl, h->stream);
    if (h->smr) {
        if (e == hipSuccess)
            e = launch_dt_levels(h->lgeo[0], level_starts(h), h->nblk, h->U, h->ctrl, 0, h->stream);
    } else if (e == hipSuccess) {
        e = launch_dt(h->geo, h->U, h->ctrl, h->stream);
    }
    if (e == hipSuccess) e = launch_ctrl(h->ctrl, CTRL_FINALIZE_DT, 0.0, 0.0, h->cfg.cfl, h->stream);
    if (e == hipSuccess) h->dt_valid = true;
    return e;
}

// ------------------------------------------------------- static refinement

// Leaves, side codes and ghost slots of a refinement of the block grid of
// cfg (Sec. 2.3): each listed block (code level * 2^kLevelShift + its index
// on that level's block grid, x fastest; a block of level >= 1 after its
// parent) is replaced by 2^ndim blocks of half its size and the same extents
// in cells; then, as in the paper, refinement is added on the coarser side
// until face-neighbouring leaves differ by at most one level.  Leaves are
// ordered by level, and within a level by their index on its grid.
struct SmrPlan {
    int nleaf = 0, nlev = 1;
    std::vector<int32_t> leaves;  // (level, c0, c1, c2), physical axes
    std::vector<int> side;        // 6 per leaf, kernel axes
    std::vector<GhostTask> tasks;
    int nres = 0, npro = 0, res_off[4] = {0, 0, 0, 0};
    int pro_off[kMaxLevels + 1] = {0, 0, 0, 0, 0};
    int lev_start[kMaxLevels] = {0, 0, 0, 0}, lev_count[kMaxLevels] = {0, 0, 0, 0};
    long long gcs = 0;
};

bool smr_plan(const hydro_config* c, int nref, const int32_t* refined, SmrPlan& P) {
    if (!config_ok(c) || nref < 0 || (nref > 0 && !refined)) return false;
    const int nd = c->ndim;
    int B[3], nb[3];
    for (int d = 0; d < 3; ++d) {
        B[d] = blocks_of(c, d);
        nb[d] = c->n[d] / B[d];
        // a refined block's children align with its cells, and the two
        // restricted ghost layers of a coarse side cover four fine layers
        if (nref > 0 && d < nd && (nb[d] % 2 != 0 || nb[d] < 4)) return false;
    }
    auto ext = [&](int L, int d) { return d < nd ? B[d] << L : 1; };
    auto count = [&](int L) { return (long long)ext(L, 0) * ext(L, 1) * ext(L, 2); };
    auto key = [&](int L, const int* c3) { return ((long long)c3[2] * ext(L, 1) + c3[1]) * ext(L, 0) + c3[0]; };
    auto coords = [&](int L, long long f, int* c3) {
        c3[0] = (int)(f % ext(L, 0));
        c3[1] = (int)((f / ext(L, 0)) % ext(L, 1));
        c3[2] = (int)(f / ((long long)ext(L, 0) * ext(L, 1)));
    };
    auto parent = [&](int L, const int* c3) {
        int p3[3];
        for (int e = 0; e < 3; ++e) p3[e] = e < nd ? c3[e] / 2 : 0;
        return key(L - 1, p3);
    };
    std::vector<char> ref[kMaxLevels];
    for (int L = 0; L < kMaxLevels; ++L) ref[L].assign((size_t)count(L), 0);
    // a block exists in the tree: a root, or a child of a refined block
    auto exists = [&](int L, const int* c3) { return L == 0 || ref[L - 1][parent(L, c3)] != 0; };
    const int32_t mask = (1 << kLevelShift) - 1;
    for (int r = 0; r < nref; ++r) {
        if (refined[r] < 0) return false;
        const int L = refined[r] >> kLevelShift;
        const long long f = refined[r] & mask;
        if (L > kMaxLevels - 2 || f >= count(L) || ref[L][f]) return false;
        ref[L][f] = 1;
    }
    for (int L = 1; L < kMaxLevels - 1; ++L)
        for (long long f = 0; f < count(L); ++f) {
            int c3[3];
            coords(L, f, c3);
            if (ref[L][f] && !exists(L, c3)) return false;  // listed before its parent was refined
        }
    // 2:1 balance across faces: while a leaf of level L >= 2 faces a region
    // whose level L - 2 ancestor is a leaf (or coarser), refine that ancestor
    for (bool changed = true; changed;) {
        changed = false;
        for (int L = 2; L < kMaxLevels; ++L)
            for (long long f = 0; f < count(L); ++f) {
                int c3[3];
                coords(L, f, c3);
                if (!exists(L, c3) || ref[L][f]) continue;
                for (int d = 0; d < nd; ++d)
                    for (int sd = 0; sd < 2; ++sd) {
                        int q3[3] = {c3[0], c3[1], c3[2]};
                        const int E = ext(L, d);
                        q3[d] += sd ? 1 : -1;
                        if (q3[d] < 0 || q3[d] >= E) {
                            if (c->bc[d][sd] != HYDRO_BC_PERIODIC) continue;
                            q3[d] = (q3[d] + E) % E;
                        }
                        int p2[3];
                        for (int e = 0; e < 3; ++e) p2[e] = e < nd ? q3[e] / 4 : 0;
                        const long long k2 = key(L - 2, p2);
                        if (!ref[L - 2][k2]) {
                            ref[L - 2][k2] = 1;
                            changed = true;
                        }
                    }
            }
        // a block refined for balance may need its own parent refined
        for (int L = kMaxLevels - 2; L >= 1; --L)
            for (long long f = 0; f < count(L); ++f) {
                int c3[3];
                coords(L, f, c3);
                if (ref[L][f] && !exists(L, c3)) {
                    ref[L - 1][parent(L, c3)] = 1;
                    changed = true;
                }
            }
    }
    std::vector<int> look[kMaxLevels];
    for (int L = 0; L < kMaxLevels; ++L) {
        look[L].assign((size_t)count(L), -1);
        P.lev_start[L] = (int)(P.leaves.size() / 4);
        for (long long f = 0; f < count(L); ++f) {
            int c3[3];
            coords(L, f, c3);
            if (!exists(L, c3) || ref[L][f]) continue;
            look[L][f] = (int)(P.leaves.size() / 4);
            P.leaves.insert(P.leaves.end(), {L, c3[0], c3[1], c3[2]});
        }
        P.lev_count[L] = (int)(P.leaves.size() / 4) - P.lev_start[L];
        if (P.lev_count[L] > 0) P.nlev = L + 1;
    }
    P.nleaf = (int)(P.leaves.size() / 4);
    if (P.nleaf > kMaxBlocks) return false;
    const int kmap[3] = {0, nd == 3 ? 1 : -1, nd == 3 ? 2 : (nd == 2 ? 1 : -1)};  // kernel -> physical axis
    auto leaf_at = [&](int L, const int* c3) -> int { return look[L][key(L, c3)]; };
    // sides: what lies across (physical axis d, side s) of leaf b; for FINE,
    // root receives the level-L coordinates of the refined neighbour block
    enum { PHYS, SAME, COARSE, FINE };
    auto across = [&](int b, int d, int s, int& idx, int* root) -> int {
        const int L = P.leaves[4 * b];
        int c3[3] = {P.leaves[4 * b + 1], P.leaves[4 * b + 2], P.leaves[4 * b + 3]};
        const int E = ext(L, d);
        int q = c3[d] + (s ? 1 : -1);
        if (q < 0 || q >= E) {
            if (c->bc[d][s] != HYDRO_BC_PERIODIC) return PHYS;
            q = (q + E) % E;
        }
        c3[d] = q;
        idx = leaf_at(L, c3);
        if (idx >= 0) return SAME;
        if (L > 0) {
            idx = look[L - 1][parent(L, c3)];
            if (idx >= 0) return COARSE;
        }
        for (int e = 0; e < 3; ++e) root[e] = c3[e];
        return FINE;
    };
    P.side.assign(6 * (size_t)P.nleaf, 0);
    std::vector<GhostTask> res[3], pro[kMaxLevels];
    std::vector<std::pair<int, int>> res_at[3], pro_at[kMaxLevels];  // (leaf, side index) owning each task
    for (int b = 0; b < P.nleaf; ++b) {
        for (int k = 0; k < 3; ++k) {
            for (int s = 0; s < 2; ++s) {
                int& code = P.side[6 * b + 2 * k + s];
                const int d = kmap[k];
                if (d < 0) {
                    code = b;  // inactive axis: never read
                    continue;
                }
                int idx = -1, root[3] = {0, 0, 0};
                const int kind = across(b, d, s, idx, root);
                if (kind == PHYS) {
                    code = kSidePhys;
                } else if (kind == SAME) {
                    code = idx;
                } else {
                    GhostTask t;
                    std::memset(&t, 0, sizeof(t));
                    t.leaf = b;
                    t.ax = k;
                    t.s = s;
                    t.lev = P.leaves[4 * b];
                    const int lo = k == 0 ? 1 : 0, hi = k == 2 ? 1 : 2;
                    if (kind == FINE) {
                        t.kind = 0;
                        for (int o = 0; o < 4; ++o) {
                            int f3[3];
                            for (int e = 0; e < 3; ++e) f3[e] = 0;
                            f3[d] = s ? 2 * root[d] : 2 * root[d] + 1;
                            const int bits[2] = {o & 1, (o >> 1) & 1};
                            const int tax[2] = {lo, hi};
                            for (int q = 0; q < 2; ++q) {
                                const int e = kmap[tax[q]];
                                if (e >= 0) f3[e] = 2 * root[e] + bits[q];
                            }
                            t.src[o] = t.lev + 1 < kMaxLevels ? leaf_at(t.lev + 1, f3) : -1;
                            if (t.src[o] < 0) return false;
                        }
                        res[k].push_back(t);
                        res_at[k].push_back({b, 2 * k + s});
                    } else {
                        t.kind = 1;
                        t.src[0] = idx;
                        for (int q = 0; q < 3; ++q) t.child[q] = kmap[q] >= 0 ? P.leaves[4 * b + 1 + kmap[q]] % 2 : 0;
                        if (idx < 0) return false;
                        pro[t.lev].push_back(t);
                        pro_at[t.lev].push_back({b, 2 * k + s});
                    }
                }
            }
        }
    }
    for (int k = 0; k < 3; ++k) {
        P.res_off[k] = (int)P.tasks.size();
        for (size_t i = 0; i < res[k].size(); ++i) {
            res[k][i].slot = (int)P.tasks.size();
            P.side[6 * res_at[k][i].first + res_at[k][i].second] = kSideSlot0 - res[k][i].slot;
            P.tasks.push_back(res[k][i]);
        }
    }
    P.res_off[3] = P.nres = (int)P.tasks.size();
    // prolongation slots by the fine block's level: each level's launch
    // follows the coarser one's, whose slots its coarse stencils may read
    for (int L = 0; L < kMaxLevels; ++L) {
        P.pro_off[L] = (int)P.tasks.size();
        for (size_t i = 0; i < pro[L].size(); ++i) {
            pro[L][i].slot = (int)P.tasks.size();
            P.side[6 * pro_at[L][i].first + pro_at[L][i].second] = kSideSlot0 - pro[L][i].slot;
            P.tasks.push_back(pro[L][i]);
        }
    }
    P.pro_off[kMaxLevels] = (int)P.tasks.size();
    P.npro = (int)P.tasks.size() - P.nres;
    // slot component stride: both layers of the largest side
    long long face = 1;
    const int nk[3] = {nb[kmap[0]], kmap[1] >= 0 ? nb[kmap[1]] : 1, kmap[2] >= 0 ? nb[kmap[2]] : 1};
    for (int k = 0; k < 3; ++k)
        if (kmap[k] >= 0) {
            const int lo = k == 0 ? 1 : 0, hi = k == 2 ? 1 : 2;
            face = std::max(face, (long long)nk[lo] * nk[hi]);
        }
    P.gcs = 2 * face;
    return true;
}

size_t smr_bytes(const hydro_config* c, const SmrPlan& P) {
    const size_t nc = (size_t)c->ndim + 2;
    const size_t cells = (size_t)ncells_of(c) / ((size_t)blocks_of(c, 0) * blocks_of(c, 1) * blocks_of(c, 2));
    const size_t field = align_up(nc * cells * (size_t)P.nleaf * sizeof(double));
    return 2 * field + align_up(sizeof(Ctrl)) + align_up((size_t)kTotalsParts * kMaxComp * 2 * sizeof(double)) +
           align_up(P.side.size() * sizeof(int)) + align_up(P.tasks.size() * sizeof(GhostTask)) +
           align_up(P.tasks.size() * nc * (size_t)P.gcs * sizeof(double)) +
           align_up((size_t)P.nres * nc * (size_t)(P.gcs / 2) * sizeof(double));
}

}  // namespace

extern "C" {

size_t hydro_workspace_bytes(const hydro_config* cfg) {
    if (!config_ok(cfg)) return 0;
    return state_bytes(cfg) + second_bytes(cfg) + align_up(sizeof(Ctrl)) +
           align_up((size_t)kTotalsParts * kMaxComp * 2 * sizeof(double));
}

int hydro_create(const hydro_config* cfg, void* d_workspace, size_t nbytes, void* hip_stream,
                 hydro_t* out) {
    if (!out || !config_ok(cfg) || !d_workspace) return HYDRO_E_INVAL;
    if (((uintptr_t)d_workspace) % kAlign != 0) return HYDRO_E_INVAL;
    if (nbytes < hydro_workspace_bytes(cfg)) return HYDRO_E_INVAL;
    hydro_ctx* h = new (std::nothrow) hydro_ctx;
    if (!h) return HYDRO_E_NOMEM;
    std::memset(h, 0, sizeof(*h));
    h->cfg = *cfg;
    h->geo = make_geo(cfg);
    h->nblk = geo_nblk(h->geo);
    h->tile[0] = default_tile(h->geo, cfg->precision, stage1_mode(cfg));
    h->tile[1] = default_tile(h->geo, cfg->precision, stage2_mode(cfg));
    h->stream = (hipStream_t)hip_stream;
    h->ncomp = cfg->ndim + 2;
    h->dV = 1.0;
    for (int d = 0; d < cfg->ndim; ++d) h->dV *= (cfg->hi[d] - cfg->lo[d]) / cfg->n[d];
    char* p = (char*)d_workspace;
    const size_t sb = state_bytes(cfg), sb2 = second_bytes(cfg);
    h->U = (double*)p;
    p += sb;
    h->U1 = (double*)p;  // van Leer: holds values of the compute type
    p += sb2;
    h->ctrl = (Ctrl*)p;
    p += align_up(sizeof(Ctrl));
    h->parts = (double*)p;
    h->host_ctrl = new (std::nothrow) Ctrl;
    if (!h->host_ctrl) {
        delete h;
        return HYDRO_E_NOMEM;
    }
    // stream-ordered set-up, no host synchronisation: a handle made while
    // other work is in flight on the stream (a serving loop admitting a
    // request behind running steps) does not wait for that work
    hipError_t e = hipMemsetAsync(h->U, 0, sb + sb2, h->stream);
    if (e == hipSuccess) e = launch_ctrl(h->ctrl, CTRL_INIT, 0.0, 0.0, cfg->cfl, h->stream);
    if (e != hipSuccess) {
        delete h->host_ctrl;
        delete h;
        return HYDRO_E_DEVICE;
    }
    *out = h;
    return HYDRO_OK;
}

size_t hydro_smr_workspace_bytes(const hydro_config* cfg, int nref, const int32_t* refined) {
    SmrPlan P;
    if (!smr_plan(cfg, nref, refined, P)) return 0;
    return smr_bytes(cfg, P);
}

int hydro_smr_create(const hydro_config* cfg, int nref, const int32_t* refined, void* d_workspace, size_t nbytes,
                     void* hip_stream, hydro_t* out) {
    SmrPlan P;
    if (!out || !d_workspace || !smr_plan(cfg, nref, refined, P)) return HYDRO_E_INVAL;
    if (((uintptr_t)d_workspace) % kAlign != 0 || nbytes < smr_bytes(cfg, P)) return HYDRO_E_INVAL;
    hydro_ctx* h = new (std::nothrow) hydro_ctx;
    if (!h) return HYDRO_E_NOMEM;
    std::memset(h, 0, sizeof(*h));
    h->leaves = new (std::nothrow) int32_t[P.leaves.size()];
    if (!h->leaves) {
        delete h;
        return HYDRO_E_NOMEM;
    }
    std::memcpy(h->leaves, P.leaves.data(), P.leaves.size() * sizeof(int32_t));
    h->cfg = *cfg;
    h->smr = true;
    h->geo = make_geo(cfg);
    h->nblk = P.nleaf;
    h->geo.blocks[0] = P.nleaf;  // the leaves as a row of blocks (per-cell passes)
    h->geo.blocks[1] = h->geo.blocks[2] = 1;
    h->nlev = P.nlev;
    for (int lev = 0; lev < kMaxLevels; ++lev) {
        Geo g = h->geo;
        for (int k = 0; k < 3; ++k) {
            const bool active = k == 0 || (k == 1 && cfg->ndim == 3) || (k == 2 && cfg->ndim >= 2);
            if (!active) continue;
            g.dx[k] = std::ldexp(h->geo.dx[k], -lev);  // exact: level 0's width times 2^-lev
            g.inv_dx[k] = 1.0 / g.dx[k];
        }
        g.blocks[0] = P.lev_count[lev];
        h->lgeo[lev] = g;
        h->lev_start[lev] = P.lev_start[lev];
        h->lev_count[lev] = P.lev_count[lev];
    }
    for (int L = 0; L <= kMaxLevels; ++L) h->pro_off[L] = P.pro_off[L];
    h->tile[0] = default_tile(h->geo, cfg->precision, smr_mode(cfg, 0));
    h->tile[1] = default_tile(h->geo, cfg->precision, smr_mode(cfg, 1));
    h->stream = (hipStream_t)hip_stream;
    h->ncomp = cfg->ndim + 2;
    h->dV = 1.0;
    for (int d = 0; d < cfg->ndim; ++d) h->dV *= (cfg->hi[d] - cfg->lo[d]) / cfg->n[d];
    h->nres = P.nres;
    h->npro = P.npro;
    for (int k = 0; k < 4; ++k) h->res_off[k] = P.res_off[k];
    h->gcs = P.gcs;
    const size_t nc = (size_t)h->ncomp;
    const size_t field = align_up(nc * (size_t)h->geo.ncells * P.nleaf * sizeof(double));
    char* p = (char*)d_workspace;
    h->U = (double*)p;
    p += field;
    h->U1 = (double*)p;
    p += field;
    h->ctrl = (Ctrl*)p;
    p += align_up(sizeof(Ctrl));
    h->parts = (double*)p;
    p += align_up((size_t)kTotalsParts * kMaxComp * 2 * sizeof(double));
    h->d_side = (int*)p;
    p += align_up(P.side.size() * sizeof(int));
    h->d_tasks = (GhostTask*)p;
    p += align_up(P.tasks.size() * sizeof(GhostTask));
    h->gbuf = (double*)p;
    p += align_up(P.tasks.size() * nc * (size_t)P.gcs * sizeof(double));
    h->dbuf = (double*)p;
    h->host_ctrl = new (std::nothrow) Ctrl;
    if (!h->host_ctrl) {
        delete[] h->leaves;
        delete h;
        return HYDRO_E_NOMEM;
    }
    hipError_t e = hipMemsetAsync(h->U, 0, 2 * field, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->d_side, P.side.data(), P.side.size() * sizeof(int), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && !P.tasks.empty())
        e = hipMemcpyAsync(h->d_tasks, P.tasks.data(), P.tasks.size() * sizeof(GhostTask), hipMemcpyHostToDevice,
                           h->stream);
    if (e == hipSuccess) e = launch_ctrl(h->ctrl, CTRL_INIT, 0.0, 0.0, cfg->cfl, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);  // the plan's host vectors end here
    if (e == hipSuccess && P.tasks.size() > 0) {
        // default priority, not synchronising with the legacy default stream
        hipStream_t aux = nullptr;
        e = hipStreamCreateWithFlags(&aux, hipStreamNonBlocking);
        if (e == hipSuccess) {
            int made = 0;
            for (; made < 3; ++made) {
                e = hipEventCreateWithFlags(&h->ev_smr[made], hipEventDisableTiming);
                if (e != hipSuccess) break;
            }
            if (e == hipSuccess) {
                h->smr_aux = aux;
            } else {
                for (int i = 0; i < made; ++i) (void)hipEventDestroy(h->ev_smr[i]);
                (void)hipStreamDestroy(aux);
            }
        }
    }
    if (e != hipSuccess) {
        delete h->host_ctrl;
        delete[] h->leaves;
        delete h;
        return HYDRO_E_DEVICE;
    }
    *out = h;
    return HYDRO_OK;
}

int hydro_smr_leaves(const hydro_config* cfg, int nref, const int32_t* refined, int32_t* leaves, int max) {
    SmrPlan P;
    if (max < 0 || (max > 0 && !leaves) || !smr_plan(cfg, nref, refined, P)) return HYDRO_E_INVAL;
    for (int b = 0; b < P.nleaf && b < max; ++b)
        for (int q = 0; q < 4; ++q) leaves[4 * b + q] = P.leaves[4 * b + q];
    return P.nleaf;
}

int hydro_set_state(hydro_t h, const double* U_host) {
    int rc = usable(h);
    if (rc) return rc;
    if (!U_host) return HYDRO_E_INVAL;
    const size_t bytes = (size_t)h->ncomp * h->geo.ncells * h->nblk * sizeof(double);
    hipError_t e = hipSuccess;
    if (!mesh_relayout(h)) {
        e = hipMemcpyAsync(h->U, U_host, bytes, hipMemcpyHostToDevice, h->stream);
    } else {
        double* tmp = nullptr;
        e = mesh_tmp(h, &tmp);
        if (e == hipSuccess) e = hipMemcpyAsync(tmp, U_host, bytes, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = launch_relayout(h->geo, tmp, h->U, 1, h->stream);
        e = free_tmp(h, tmp, e);
    }
    if (e == hipSuccess) e = launch_ctrl(h->ctrl, CTRL_INIT, 0.0, 0.0, h->cfg.cfl, h->stream);
    h->dt_valid = false;
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return fail(h, e);
}

int hydro_set_primitive(hydro_t h, const double* W_host) {
    int rc = usable(h);
    if (rc) return rc;
    if (!W_host) return HYDRO_E_INVAL;
    const size_t bytes = (size_t)h->ncomp * h->geo.ncells * h->nblk * sizeof(double);
    // staged in U itself (through a mesh-layout buffer for a split mesh) and
    // converted in place
    hipError_t e = hipSuccess;
    if (!mesh_relayout(h)) {
        e = hipMemcpyAsync(h->U, W_host, bytes, hipMemcpyHostToDevice, h->stream);
    } else {
        double* tmp = nullptr;
        e = mesh_tmp(h, &tmp);
        if (e == hipSuccess) e = hipMemcpyAsync(tmp, W_host, bytes, hipMemcpyHostToDevice, h->stream);
        if (e == hipSuccess) e = launch_relayout(h->geo, tmp, h->U, 1, h->stream);
        e = free_tmp(h, tmp, e);
    }
    if (e == hipSuccess) e = launch_prim_to_cons(h->geo, h->U, h->U, h->stream);
    if (e == hipSuccess) e = launch_ctrl(h->ctrl, CTRL_INIT, 0.0, 0.0, h->cfg.cfl, h->stream);
    h->dt_valid = false;
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return fail(h, e);
}

int hydro_set_primitive_device(hydro_t h, const double* d_W) {
    int rc = usable(h);
    if (rc) return rc;
    if (!d_W) return HYDRO_E_INVAL;
    hipError_t e = hipSuccess;
    if (!mesh_relayout(h)) {
        e = launch_prim_to_cons(h->geo, d_W, h->U, h->stream);
    } else {
        // only read: the relayout writes the block layout into U
        e = launch_relayout(h->geo, const_cast<double*>(d_W), h->U, 1, h->stream);
        if (e == hipSuccess) e = launch_prim_to_cons(h->geo, h->U, h->U, h->stream);
    }
    if (e == hipSuccess) e = launch_ctrl(h->ctrl, CTRL_INIT, 0.0, 0.0, h->cfg.cfl, h->stream);
    h->dt_valid = false;
    return fail(h, e);
}

int hydro_get_state_device(hydro_t h, double* d_U) {
    int rc = usable(h);
    if (rc) return rc;
    if (!d_U) return HYDRO_E_INVAL;
    const size_t bytes = (size_t)h->ncomp * h->geo.ncells * h->nblk * sizeof(double);
    if (mesh_relayout(h)) return fail(h, launch_relayout(h->geo, d_U, h->U, 0, h->stream));
    return fail(h, hipMemcpyAsync(d_U, h->U, bytes, hipMemcpyDeviceToDevice, h->stream));
}

int hydro_get_state(hydro_t h, double* U_host) {
    int rc = usable(h);
    if (rc) return rc;
    if (!U_host) return HYDRO_E_INVAL;
    const size_t bytes = (size_t)h->ncomp * h->geo.ncells * h->nblk * sizeof(double);
    hipError_t e = hipSuccess;
    if (!mesh_relayout(h)) {
        e = hipMemcpyAsync(U_host, h->U, bytes, hipMemcpyDeviceToHost, h->stream);
    } else {
        double* tmp = nullptr;
        e = mesh_tmp(h, &tmp);
        if (e == hipSuccess) e = launch_relayout(h->geo, tmp, h->U, 0, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(U_host, tmp, bytes, hipMemcpyDeviceToHost, h->stream);
        e = free_tmp(h, tmp, e);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    return fail(h, e);
}

int hydro_state_device(hydro_t h, const double** d_U) {
    int rc = usable(h);
    if (rc) return rc;
    if (!d_U) return HYDRO_E_INVAL;
    *d_U = h->U;
    return HYDRO_OK;
}

int hydro_cfl_dt(hydro_t h, double* dt) {
    int rc = usable(h);
    if (rc) return rc;
    if (!dt) return HYDRO_E_INVAL;
    hipError_t e = h->dt_valid ? hipSuccess : enqueue_dt(h);
    if (e != hipSuccess) return fail(h, e);
    rc = read_ctrl(h);
    if (rc) return rc;
    *dt = h->host_ctrl->dt_raw;
    return HYDRO_OK;
}

int hydro_step(hydro_t h, double dt) {
    int rc = usable(h);
    if (rc) return rc;
    if (!(dt > 0.0) || !std::isfinite(dt)) return HYDRO_E_INVAL;
    h->dt_valid = false;
    return fail(h, enqueue_step(h, false, dt));
}

int hydro_step_auto(hydro_t h, int nsteps, double t_end) {
    int rc = usable(h);
    if (rc) return rc;
    if (nsteps < 0 || !(t_end >= 0.0) || !std::isfinite(t_end)) return HYDRO_E_INVAL;
    if (nsteps == 0) return HYDRO_OK;
    // The dt of the first step comes from a standalone reduction when the
    // state changed since the last device-dt step; every later dt from the
    // previous step's epilogue.
    hipError_t e = launch_ctrl(h->ctrl, CTRL_SET_LIMITS, t_end, 0.0, h->cfg.cfl, h->stream);
    if (e == hipSuccess && !h->dt_valid) e = enqueue_dt(h);
    for (int s = 0; s < nsteps && e == hipSuccess; ++s) e = enqueue_step(h, true, 0.0);
    return fail(h, e);
}

int hydro_set_run_limit(hydro_t h, int64_t max_steps, double t_end) {
    int rc = usable(h);
    if (rc) return rc;
    if (max_steps < 0 || !(t_end >= 0.0) || !std::isfinite(t_end)) return HYDRO_E_INVAL;
    return fail(h, launch_ctrl(h->ctrl, CTRL_SET_LIMITS, t_end, (double)max_steps, h->cfg.cfl, h->stream));
}

int hydro_run_done(hydro_t h, int* done) {
    int rc = usable(h);
    if (rc) return rc;
    if (!done) return HYDRO_E_INVAL;
    rc = read_ctrl(h);
    if (rc && rc != HYDRO_E_NONPHYSICAL) return rc;
    *done = h->host_ctrl->done ? 1 : 0;
    return rc;
}

int hydro_conserved_totals(hydro_t h, double* totals) {
    int rc = usable(h);
    if (rc) return rc;
    if (!totals) return HYDRO_E_INVAL;
    if (h->smr) {
        // per level (its own cell volume), then summed
        const long long BS = (long long)h->ncomp * h->geo.ncells;
        for (int c = 0; c < h->ncomp; ++c) totals[c] = 0.0;
        double dV = h->dV;
        for (int lev = 0; lev < h->nlev; ++lev, dV *= 1.0 / (1 << h->cfg.ndim)) {
            if (h->lev_count[lev] == 0) continue;
            hipError_t e = launch_totals(h->lgeo[lev], h->U + h->lev_start[lev] * BS, h->parts, kTotalsParts,
                                         h->ctrl, h->stream);
            if (e != hipSuccess) return fail(h, e);
            rc = read_ctrl(h);
            if (rc && rc != HYDRO_E_NONPHYSICAL) return rc;
            for (int c = 0; c < h->ncomp; ++c)
                totals[c] += dV * (h->host_ctrl->sums[2 * c] + h->host_ctrl->sums[2 * c + 1]);
        }
        return rc;
    }
    hipError_t e = launch_totals(h->geo, h->U, h->parts, kTotalsParts, h->ctrl, h->stream);
    if (e != hipSuccess) return fail(h, e);
    rc = read_ctrl(h);
    if (rc && rc != HYDRO_E_NONPHYSICAL) return rc;
    for (int c = 0; c < h->ncomp; ++c)
        totals[c] = h->dV * (h->host_ctrl->sums[2 * c] + h->host_ctrl->sums[2 * c + 1]);
    return rc;
}

// Scratch of hydro_conserved_totals_noalloc: the per-work-group partials,
// (sum, compensation) per component, of at most kTotalsParts work-groups.
// Every call on a device shares that device's copy; pass 1 writes every
// partial that pass 2 reads, so nothing needs clearing between calls.
constexpr int kScratchParts = kTotalsParts;
static __device__ __align__(256) double scratch[2 * kMaxComp * kScratchParts];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices];  // per device: the device address of its scratch copy

// The current device's scratch address, looked up once per device (the
// symbol's host name is no device address).
hipError_t scratch_address(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = (double*)p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}
}  // namespace

int hydro_conserved_totals_noalloc(const hydro_config* cfg, const double* d_U, double* d_totals,
                                   void* hip_stream) {
    if (!config_ok(cfg) || !d_U || !d_totals) return HYDRO_E_INVAL;
    const Geo g = make_geo(cfg);
    const int nblk = geo_nblk(g);
    // every block takes one partial at least (config_ok caps the blocks at
    // kMaxBlocks == kScratchParts)
    if (nblk > kScratchParts) return HYDRO_E_INVAL;
    double dV = 1.0;
    for (int d = 0; d < cfg->ndim; ++d) dV *= (cfg->hi[d] - cfg->lo[d]) / cfg->n[d];
    double* parts = nullptr;
    hipError_t e = scratch_address(&parts);
    if (e == hipSuccess) e = launch_totals_out(g, d_U, parts, kScratchParts, d_totals, dV, (hipStream_t)hip_stream);
    return e == hipSuccess ? HYDRO_OK : HYDRO_E_DEVICE;
}

int hydro_time(hydro_t h, double* t) {
    int rc = usable(h);
    if (rc) return rc;
    if (!t) return HYDRO_E_INVAL;
    rc = read_ctrl(h);
    if (rc && rc != HYDRO_E_NONPHYSICAL) return rc;
    *t = h->host_ctrl->t;
    return rc;
}

int hydro_steps_done(hydro_t h, int64_t* steps) {
    int rc = usable(h);
    if (rc) return rc;
    if (!steps) return HYDRO_E_INVAL;
    rc = read_ctrl(h);
    if (rc && rc != HYDRO_E_NONPHYSICAL) return rc;
    *steps = (int64_t)h->host_ctrl->steps;
    return rc;
}

int hydro_stage_rhs(hydro_t h, double dt, double* dU_host) {
    int rc = usable(h);
    if (rc) return rc;
    if (h->smr) return HYDRO_E_INVAL;
    if (!dU_host || !(dt > 0.0) || !std::isfinite(dt)) return HYDRO_E_INVAL;
    StageArgs a = stage_args(h);
    a.dt_host = dt;
    a.in = h->U;
    const size_t bytes = (size_t)h->ncomp * h->geo.ncells * h->nblk * sizeof(double);
    // the Heun predictor buffer holds FP64 values of this size; the van Leer
    // one may not, so a temporary buffer takes the result then; a split
    // mesh's result is copied out through a mesh-layout buffer
    double* d_buf = nullptr;
    double* d_mesh = nullptr;
    hipError_t e = hipSuccess;
    if (h->cfg.integrator != HYDRO_HEUN) e = hipMallocAsync((void**)&d_buf, bytes, h->stream);
    double* out = h->cfg.integrator != HYDRO_HEUN ? d_buf : h->U1;
    a.out = out;
    if (e == hipSuccess) e = launch_stage(h->cfg.precision, MODE_RHS, h->tile[0], a, h->stream);
    if (e == hipSuccess && h->nblk > 1) {
        e = mesh_tmp(h, &d_mesh);
        if (e == hipSuccess) e = launch_relayout(h->geo, d_mesh, out, 0, h->stream);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(dU_host, d_mesh ? d_mesh : out, bytes, hipMemcpyDeviceToHost, h->stream);
    e = free_tmp(h, d_mesh, e);
    e = free_tmp(h, d_buf, e);
    if (e != hipSuccess) return fail(h, e);
    return read_ctrl(h);
}

int hydro_padded_primitive(hydro_t h, double* Wpad_host) {
    int rc = usable(h);
    if (rc) return rc;
    if (h->smr) return HYDRO_E_INVAL;
    if (!Wpad_host) return HYDRO_E_INVAL;
    size_t total = (size_t)h->ncomp;
    for (int d = 0; d < 3; ++d) total *= (size_t)(h->cfg.n[d] + (d < h->cfg.ndim ? 4 : 0));
    double* d_buf = nullptr;
    hipError_t e = hipMallocAsync((void**)&d_buf, total * sizeof(double), h->stream);
    if (e == hipSuccess) e = launch_padded_prim(h->geo, h->cfg.precision, h->U, d_buf, h->ctrl, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(Wpad_host, d_buf, total * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (d_buf) {
        hipError_t e2 = hipFreeAsync(d_buf, h->stream);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return fail(h, e);
    return read_ctrl(h);
}

int hydro_set_stage_tile(hydro_t h, int stage, int tx, int ty, int kz) {
    int rc = usable(h);
    if (rc) return rc;
    if (stage < 0 || stage > 2) return HYDRO_E_INVAL;
    Tile t;
    t.tx = tx;
    t.ty = ty;
    t.kz = kz;
    if (!tile_supported(h->cfg.ndim, t)) return HYDRO_E_INVAL;
    if (stage != 2) h->tile[0] = t;
    if (stage != 1) h->tile[1] = t;
    return HYDRO_OK;
}

int hydro_set_tile(hydro_t h, int tx, int ty, int kz) { return hydro_set_stage_tile(h, 0, tx, ty, kz); }

int hydro_get_stage_tile(hydro_t h, int stage, int* tx, int* ty, int* kz) {
    int rc = usable(h);
    if (rc) return rc;
    if (!tx || !ty || !kz || (stage != 1 && stage != 2)) return HYDRO_E_INVAL;
    const Tile& t = h->tile[stage - 1];
    *tx = t.tx;
    *ty = t.ty;
    *kz = t.kz;
    return HYDRO_OK;
}

int hydro_autotune(hydro_t h, int steps_per_tile, double t_end, int* tiles, double* ms_per_step) {
    int rc = usable(h);
    if (rc) return rc;
    if (h->smr) return HYDRO_E_INVAL;
    if (steps_per_tile < 1 || steps_per_tile > 64 || !(t_end >= 0.0) || !std::isfinite(t_end) || !tiles ||
        !ms_per_step)
        return HYDRO_E_INVAL;
    constexpr int kMaxCand = 32;
    Tile cand[kMaxCand];
    const int nc = std::min(tile_candidates(h->geo, cand, kMaxCand), kMaxCand);
    // per candidate and step: before stage 1, between the stages, after stage 2
    std::vector<hipEvent_t> ev((size_t)nc * steps_per_tile * 3);
    size_t made = 0;
    hipError_t e = hipSuccess;
    for (; made < ev.size() && e == hipSuccess; ++made) e = hipEventCreate(&ev[made]);
    if (e != hipSuccess) --made;
    const Tile keep[2] = {h->tile[0], h->tile[1]};
    // The tuning steps are real steps of the run (the results do not depend
    // on the tile): enqueue_step's launches with events between the stages.
    // One untimed step first, then the candidates in turn, round after round,
    // so clock ramp-up or drift does not favour the candidates timed last.
    if (e == hipSuccess) e = launch_ctrl(h->ctrl, CTRL_SET_LIMITS, t_end, 0.0, h->cfg.cfl, h->stream);
    if (e == hipSuccess && !h->dt_valid) e = enqueue_dt(h);
    if (e == hipSuccess) e = enqueue_step(h, true, 0.0);
    for (int s = 0; s < steps_per_tile && e == hipSuccess; ++s) {
        for (int c = 0; c < nc && e == hipSuccess; ++c) {
            hipEvent_t* q = &ev[((size_t)c * steps_per_tile + s) * 3];
            StageArgs a = stage_args(h);
            a.use_device_dt = 1;
            a.in = h->U;
            a.out = h->U1;
            e = hipEventRecord(q[0], h->stream);
            if (e == hipSuccess) e = launch_stage(h->cfg.precision, stage1_mode(&h->cfg), cand[c], a, h->stream);
            if (e == hipSuccess) e = hipEventRecord(q[1], h->stream);
            a.in = h->U1;
            a.base = h->U;
            a.out = h->U;
            a.want_dt = 1;
            if (e == hipSuccess) e = launch_stage(h->cfg.precision, stage2_mode(&h->cfg), cand[c], a, h->stream);
            if (e == hipSuccess) e = hipEventRecord(q[2], h->stream);
            if (e == hipSuccess) e = launch_ctrl(h->ctrl, CTRL_FINALIZE_STEP, 0.0, 0.0, h->cfg.cfl, h->stream);
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    std::vector<double> ms((size_t)nc * 2, 0.0);
    for (int c = 0; c < nc && e == hipSuccess; ++c)
        for (int s = 0; s < steps_per_tile && e == hipSuccess; ++s)
            for (int st = 0; st < 2 && e == hipSuccess; ++st) {
                const hipEvent_t* q = &ev[((size_t)c * steps_per_tile + s) * 3];
                float t = 0.0f;
                e = hipEventElapsedTime(&t, q[st], q[st + 1]);
                ms[2 * c + st] += t;
            }
    for (size_t i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    if (e != hipSuccess) return fail(h, e);
    rc = read_ctrl(h);
    if (rc) return rc;
    // a run that reached its limit while tuning skipped steps: no valid timing
    if (h->host_ctrl->done || nc < 1) return HYDRO_E_STATE;
    for (int st = 0; st < 2; ++st) {
        // the tile in use stays unless a candidate is faster by more than 5 %
        // (about the run-to-run spread of a few steps' timing), so close
        // timings do not flip the choice from run to run
        int keep_c = -1, best = -1;
        for (int c = 0; c < nc; ++c)
            if (cand[c].tx == keep[st].tx && cand[c].ty == keep[st].ty && cand[c].kz == keep[st].kz) keep_c = c;
        for (int c = 0; c < nc; ++c)
            if (best < 0 || ms[2 * c + st] < ms[2 * best + st]) best = c;
        if (keep_c >= 0 && !(ms[2 * best + st] < 0.95 * ms[2 * keep_c + st])) best = keep_c;
        h->tile[st] = cand[best];
        tiles[3 * st] = cand[best].tx;
        tiles[3 * st + 1] = cand[best].ty;
        tiles[3 * st + 2] = cand[best].kz;
        ms_per_step[st] = ms[2 * best + st] / steps_per_tile;
    }
    return HYDRO_OK;
}

int hydro_tile_candidates(const hydro_config* cfg, int* tiles, int max) {
    if (!config_ok(cfg) || max < 0 || (max > 0 && !tiles)) return HYDRO_E_INVAL;
    const Geo g = make_geo(cfg);
    constexpr int kMaxCand = 32;
    Tile cand[kMaxCand];
    const int nc = std::min(tile_candidates(g, cand, kMaxCand), kMaxCand);
    for (int c = 0; c < nc && c < max; ++c) {
        tiles[3 * c] = cand[c].tx;
        tiles[3 * c + 1] = cand[c].ty;
        tiles[3 * c + 2] = cand[c].kz;
    }
    return nc;
}

namespace {
void profile_free(hydro_t h) {
    for (int st = 0; st < 2; ++st) {
        if (!h->prof_ev[st]) continue;
        for (int i = 0; i < 2 * h->prof_cap; ++i) (void)hipEventDestroy(h->prof_ev[st][i]);
        delete[] h->prof_ev[st];
        h->prof_ev[st] = nullptr;
    }
    h->prof_cap = 0;
    h->prof_n[0] = h->prof_n[1] = 0;
}
}  // namespace

int hydro_profile(hydro_t h, int max_launches) {
    int rc = usable(h);
    if (rc) return rc;
    if (max_launches < 0 || max_launches > (1 << 20)) return HYDRO_E_INVAL;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(h, e);
    profile_free(h);
    if (max_launches == 0) return HYDRO_OK;
    for (int st = 0; st < 2; ++st) {
        h->prof_ev[st] = new (std::nothrow) hipEvent_t[2 * max_launches];
        if (!h->prof_ev[st]) {
            profile_free(h);
            return HYDRO_E_NOMEM;
        }
        for (int i = 0; i < 2 * max_launches; ++i) {
            e = hipEventCreate(&h->prof_ev[st][i]);
            if (e != hipSuccess) {
                for (int j = 0; j < i; ++j) (void)hipEventDestroy(h->prof_ev[st][j]);
                delete[] h->prof_ev[st];
                h->prof_ev[st] = nullptr;
                profile_free(h);
                return fail(h, e);
            }
        }
    }
    h->prof_cap = max_launches;
    return HYDRO_OK;
}

int hydro_profile_read(hydro_t h, double* ms_stage1, double* ms_stage2, int64_t* launches) {
    int rc = usable(h);
    if (rc) return rc;
    if (!ms_stage1 || !ms_stage2 || !launches) return HYDRO_E_INVAL;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(h, e);
    double tot[2] = {0.0, 0.0};
    for (int st = 0; st < 2; ++st)
        for (int i = 0; i < h->prof_n[st]; ++i) {
            float ms = 0.0f;
            e = hipEventElapsedTime(&ms, h->prof_ev[st][2 * i], h->prof_ev[st][2 * i + 1]);
            if (e != hipSuccess) return fail(h, e);
            tot[st] += ms;
        }
    *ms_stage1 = tot[0];
    *ms_stage2 = tot[1];
    launches[0] = h->prof_n[0];
    launches[1] = h->prof_n[1];
    h->prof_n[0] = h->prof_n[1] = 0;
    return HYDRO_OK;
}

int hydro_set_block_streams(hydro_t h, int on) {
    int rc = usable(h);
    if (rc) return rc;
    if ((on != 0 && on != 1) || (on && h->smr)) return HYDRO_E_INVAL;
    if (on && h->nblk > 1) {
        // streams made while no work of this handle is in flight
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e == hipSuccess) e = block_streams_make(h);
        if (e == hipErrorOutOfMemory) return HYDRO_E_NOMEM;
        if (e != hipSuccess) return fail(h, e);
    }
    h->block_streams = on != 0;
    return HYDRO_OK;
}

int hydro_destroy(hydro_t h) {
    if (!h) return HYDRO_E_INVAL;
    if (!h->broken) (void)hipStreamSynchronize(h->stream);
    block_streams_free(h);
    profile_free(h);
    if (h->smr_aux) {
        for (int i = 0; i < 3; ++i) (void)hipEventDestroy(h->ev_smr[i]);
        (void)hipStreamDestroy(h->smr_aux);
    }
    delete[] h->leaves;
    delete h->host_ctrl;
    delete h;
    return HYDRO_OK;
}

const char* hydro_strerror(int status) {
    switch (status) {
        case HYDRO_OK: return "ok";
        case HYDRO_E_INVAL: return "invalid argument";
        case HYDRO_E_NOMEM: return "out of host memory";
        case HYDRO_E_DEVICE: return "HIP runtime error";
        case HYDRO_E_NONPHYSICAL: return "non-physical state (rho <= 0, p <= 0 or non-finite)";
        case HYDRO_E_STATE: return "handle unusable after an earlier device error";
        default: return "unknown status";
    }
}

int hydro_riemann_fluxes(int precision, int ntan, double gamma, int64_t nfaces, const double* d_WL,
                         const double* d_WR, double* d_F, void* hip_stream) {
    if (precision != HYDRO_FP64 && precision != HYDRO_MIXED) return HYDRO_E_INVAL;
    if (ntan < 0 || ntan > 2 || nfaces < 0 || !(gamma > 1.0)) return HYDRO_E_INVAL;
    if (nfaces == 0) return HYDRO_OK;
    if (!d_WL || !d_WR || !d_F) return HYDRO_E_INVAL;
    hipError_t e = launch_riemann(precision, ntan, gamma, (long long)nfaces, d_WL, d_WR, d_F,
                                  (hipStream_t)hip_stream);
    return e == hipSuccess ? HYDRO_OK : HYDRO_E_DEVICE;
}

}  // extern "C"

// ------------------------------------------------------------------ batches

struct hydro_batch_ctx {
    std::vector<hydro_t> members;
    hipStream_t stream;
    MeshDesc* d_desc;  // descriptor table in the caller's workspace, in group order
    int2* d_blk;       // work-group table, grouped
    struct Group {
        int ndim, precision, integrator;
        Tile tile;
        int blk_off, nblk;
        int mem_off, nmem;  // the group's descriptors: d_desc[mem_off .. mem_off + nmem)
        double cells;       // cells of its members
    };
    std::vector<Group> groups;
    std::vector<int> order;  // order[k]: the member (caller's index) of descriptor k
    // Direct launches spread the groups over the batch's stream and up to
    // kBatchSideStreams more (group_stream[g]: 0 the batch's stream, i > 0
    // side[i - 1]), forked from and joined back to the batch's stream by events.
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev_join;
    hipEvent_t ev_fork;
    std::vector<int> group_stream;
    hipGraph_t graph;
    hipGraphExec_t exec;
    int graph_steps;
    bool use_graph;
    bool broken;
    unsigned long long* d_status;  // per member (done, flags, steps), gathered on the device
    std::vector<unsigned long long> h_status;
};

namespace {

struct BatchPlan {
    std::vector<MeshDesc> desc;
    std::vector<int> order;
    std::vector<int2> blk;
    std::vector<hydro_batch_ctx::Group> groups;
};

// Two more streams: with the batch's own, three of the four hardware queues
// a process has at HIP's default, leaving one for other work (a server's
// set-up stream).  Streams beyond the queue count share queues, and two
// streams on one queue run in turn; with three more, the saturated serving
// rate varied 1.32-1.40e10 from one server to the next, with two more it
// held at 1.37-1.42e10.
constexpr int kBatchSideStreams = 2;

// Tile rules of the batch autotuner for members of one or two dimensions:
// a row width for every such member (0: the member's own) and a chunk length
// (-1: the member's own, 0: about 2048 work-groups per member).  Rule 0
// keeps every member's tile.  3-D members keep their tiles.
struct BatchRule {
    int tx, kz;
};
constexpr BatchRule kBatchRules[] = {{0, -1}, {64, -1}, {128, -1}, {256, -1}, {0, 16},   {64, 16},
                                     {128, 16}, {0, 32}, {64, 32},   {128, 32},  {0, 64},  {64, 64}};
constexpr int kNumBatchRules = (int)(sizeof(kBatchRules) / sizeof(kBatchRules[0]));

Tile rule_tile(const hydro_t h, int rule) {
    Tile t = h->tile[0];
    if (h->cfg.ndim == 3 || rule <= 0 || rule >= kNumBatchRules) return t;
    if (kBatchRules[rule].tx > 0) t.tx = kBatchRules[rule].tx;
    if (kBatchRules[rule].kz >= 0) t.kz = kBatchRules[rule].kz;
    return t;
}

// Members grouped by (ndim, precision, tile): each group's descriptors and
// work-groups are contiguous in their tables, members in the caller's order
// within a group (P.order maps a descriptor to its member).  Member i runs
// tile rule_tile(members[i], rule).
bool plan_batch(int n, const hydro_t* members, BatchPlan& P, int rule = 0) {
    std::vector<MeshDesc> desc(n);
    std::vector<int> order(n);
    std::vector<Tile> tiles(n);
    for (int i = 0; i < n; ++i) {
        const hydro_t h = members[i];
        tiles[i] = rule_tile(h, rule);
        MeshDesc& d = desc[i];
        d.U = h->U;
        d.U1 = h->U1;
        d.ctrl = h->ctrl;
        d.geo = h->geo;
        plan_tiles(h->geo, tiles[i], d.tiles_x, d.tiles_y, d.chunks_z, d.kz);
        order[i] = i;
    }
    auto key = [&](int i) {
        const hydro_t h = members[i];
        return std::make_tuple(h->cfg.ndim, h->cfg.precision, h->cfg.integrator, tiles[i].tx, tiles[i].ty);
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
    for (int idx = 0; idx < n; ++idx) {
        const int i = order[idx];
        const hydro_t h = members[i];
        if (P.groups.empty() || key(order[idx - 1]) != key(i)) {
            hydro_batch_ctx::Group g;
            g.ndim = h->cfg.ndim;
            g.precision = h->cfg.precision;
            g.integrator = h->cfg.integrator;
            g.tile = tiles[i];
            g.blk_off = (int)P.blk.size();
            g.nblk = 0;
            g.mem_off = idx;
            g.nmem = 0;
            g.cells = 0.0;
            P.groups.push_back(g);
        }
        const MeshDesc& d = desc[i];
        P.desc.push_back(d);
        P.order.push_back(i);
        P.groups.back().nmem += 1;
        P.groups.back().cells += (double)d.geo.ncells;
        const long long nb = (long long)d.tiles_x * d.tiles_y * d.chunks_z;
        if (nb > (1ll << 28) || (long long)P.blk.size() + nb > (1ll << 30)) return false;
        for (int b = 0; b < (int)nb; ++b) P.blk.push_back(make_int2(idx, b));
        P.groups.back().nblk += (int)nb;
    }
    return true;
}

size_t batch_bytes(const BatchPlan& P) {
    return align_up(P.desc.size() * sizeof(MeshDesc)) + align_up(P.blk.size() * sizeof(int2)) +
           align_up(P.desc.size() * 3 * sizeof(unsigned long long));
}

// Groups onto streams, largest first onto the least loaded (by cells), over
// as many streams as there are groups, at most 1 + kBatchSideStreams.
void assign_group_streams(hydro_batch_t b) {
    const int ng = (int)b->groups.size();
    const int ns = std::min(ng, 1 + kBatchSideStreams);
    std::vector<int> by(ng);
    for (int g = 0; g < ng; ++g) by[g] = g;
    std::stable_sort(by.begin(), by.end(), [&](int x, int y) { return b->groups[x].cells > b->groups[y].cells; });
    std::vector<double> load(ns > 0 ? ns : 1, 0.0);
    b->group_stream.assign(ng, 0);
    for (int g : by) {
        int best = 0;
        for (int k = 1; k < ns; ++k)
            if (load[k] < load[best]) best = k;
        b->group_stream[g] = best;
        load[best] += b->groups[g].cells;
    }
}

void side_streams_free(hydro_batch_t b) {
    for (hipEvent_t ev : b->ev_join) (void)hipEventDestroy(ev);
    for (hipStream_t st : b->side) (void)hipStreamDestroy(st);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    b->ev_join.clear();
    b->side.clear();
    b->ev_fork = nullptr;
}

// The side streams and events, made on first use (default priority, not
// synchronising with the legacy default stream).  On failure none are kept
// and the batch launches on its own stream.
bool side_streams_ready(hydro_batch_t b) {
    if (!b->side.empty()) return true;
    hipError_t e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
    if (e != hipSuccess) b->ev_fork = nullptr;
    for (int i = 0; i < kBatchSideStreams && e == hipSuccess; ++i) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) break;
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(st);
            break;
        }
        b->side.push_back(st);
        b->ev_join.push_back(ev);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        side_streams_free(b);
        return false;
    }
    return true;
}

bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

bool members_ok(int n, const hydro_t* members) {
    if (n < 1 || !members) return false;
    for (int i = 0; i < n; ++i) {
        // a batch member is one block (the batch is the level that splits work)
        if (!members[i] || members[i]->broken || members[i]->nblk != 1) return false;
        if (members[i]->stream != members[0]->stream) return false;
        for (int j = 0; j < i; ++j)
            if (members[j] == members[i]) return false;
    }
    return true;
}

// One batched Heun step: every group's stage 1, every group's stage 2, then
// each member's time / dt update.
hipError_t enqueue_batch_step(hydro_batch_t b) {
    hipError_t e = hipSuccess;
    for (const auto& g : b->groups)
        if (e == hipSuccess)
            e = launch_stage_batch(g.ndim, g.precision, g.integrator == HYDRO_VL2 ? MODE_VL2_PRED : MODE_STAGE1,
                                   g.tile, b->d_desc, b->d_blk + g.blk_off, g.nblk, b->stream);
    for (const auto& g : b->groups)
        if (e == hipSuccess)
            e = launch_stage_batch(g.ndim, g.precision, g.integrator == HYDRO_VL2 ? MODE_VL2_CORR : MODE_STAGE2,
                                   g.tile, b->d_desc, b->d_blk + g.blk_off, g.nblk, b->stream);
    if (e == hipSuccess) e = launch_ctrl_batch(b->d_desc, (int)b->members.size(), b->stream);
    return e;
}

// nsteps batched steps with the groups spread over streams: each group's
// stage 1, stage 2 and members' time / dt update on its stream, step after
// step (a member's steps depend on no other group), forked from the batch's
// stream and joined back to it at the end.  The same results as
// enqueue_batch_step nsteps times.
hipError_t enqueue_batch_steps_streams(hydro_batch_t b, int nsteps) {
    hipError_t e = hipEventRecord(b->ev_fork, b->stream);
    const int nside = (int)b->side.size();
    for (int i = 0; i < nside && e == hipSuccess; ++i) e = hipStreamWaitEvent(b->side[i], b->ev_fork, 0);
    for (int s = 0; s < nsteps && e == hipSuccess; ++s)
        for (size_t gi = 0; gi < b->groups.size() && e == hipSuccess; ++gi) {
            const auto& g = b->groups[gi];
            const int k = b->group_stream[gi];
            hipStream_t st = k > 0 && k <= nside ? b->side[k - 1] : b->stream;
            const bool vl2 = g.integrator == HYDRO_VL2;
            e = launch_stage_batch(g.ndim, g.precision, vl2 ? MODE_VL2_PRED : MODE_STAGE1, g.tile, b->d_desc,
                                   b->d_blk + g.blk_off, g.nblk, st);
            if (e == hipSuccess)
                e = launch_stage_batch(g.ndim, g.precision, vl2 ? MODE_VL2_CORR : MODE_STAGE2, g.tile, b->d_desc,
                                       b->d_blk + g.blk_off, g.nblk, st);
            if (e == hipSuccess) e = launch_ctrl_batch(b->d_desc + g.mem_off, g.nmem, st);
        }
    // joined whatever happened above, so no side-stream work outlives a call
    for (int i = 0; i < nside; ++i) {
        hipError_t x = hipEventRecord(b->ev_join[i], b->side[i]);
        if (x == hipSuccess) x = hipStreamWaitEvent(b->stream, b->ev_join[i], 0);
        if (e == hipSuccess) e = x;
    }
    return e;
}

void drop_graph(hydro_batch_t b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_steps = 0;
}

}  // namespace

extern "C" {

size_t hydro_batch_workspace_bytes(int n, const hydro_t* members) {
    if (!members_ok(n, members)) return 0;
    // large enough for the work-group table of any tile rule the autotuner tries
    size_t most = 0;
    for (int r = 0; r < kNumBatchRules; ++r) {
        BatchPlan P;
        if (!plan_batch(n, members, P, r)) return 0;
        most = std::max(most, batch_bytes(P));
    }
    return most;
}

int hydro_batch_create(int n, const hydro_t* members, void* d_workspace, size_t nbytes, int use_graph,
                       hydro_batch_t* out) {
    if (!out || !members_ok(n, members) || !d_workspace) return HYDRO_E_INVAL;
    if (((uintptr_t)d_workspace) % kAlign != 0) return HYDRO_E_INVAL;
    BatchPlan P;
    if (!plan_batch(n, members, P)) return HYDRO_E_INVAL;
    if (nbytes < hydro_batch_workspace_bytes(n, members)) return HYDRO_E_INVAL;
    hydro_batch_ctx* b = new (std::nothrow) hydro_batch_ctx;
    if (!b) return HYDRO_E_NOMEM;
    b->members.assign(members, members + n);
    b->stream = members[0]->stream;
    b->d_desc = (MeshDesc*)d_workspace;
    b->d_blk = (int2*)((char*)d_workspace + align_up(P.desc.size() * sizeof(MeshDesc)));
    b->groups = P.groups;
    b->order = P.order;
    b->ev_fork = nullptr;
    assign_group_streams(b);
    b->graph = nullptr;
    b->exec = nullptr;
    b->graph_steps = 0;
    // stream capture needs a stream other than the legacy default stream
    b->use_graph = use_graph != 0 && b->stream != nullptr;
    b->broken = false;
    // the status table after the two plan tables, whose sizes differ between
    // tile rules: at the end of the workspace the largest plan needs
    b->d_status = (unsigned long long*)((char*)d_workspace + hydro_batch_workspace_bytes(n, members) -
                                        align_up((size_t)n * 3 * sizeof(unsigned long long)));
    b->h_status.assign((size_t)n * 3, 0ull);
    hipError_t e = hipMemcpyAsync(b->d_desc, P.desc.data(), P.desc.size() * sizeof(MeshDesc),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_blk, P.blk.data(), P.blk.size() * sizeof(int2), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        delete b;
        return HYDRO_E_DEVICE;
    }
    *out = b;
    return HYDRO_OK;
}

int hydro_batch_step(hydro_batch_t b, int nsteps) {
    if (!b) return HYDRO_E_INVAL;
    if (b->broken) return HYDRO_E_STATE;
    if (nsteps < 0) return HYDRO_E_INVAL;
    if (nsteps == 0) return HYDRO_OK;
    hipError_t e = hipSuccess;
    for (hydro_t h : b->members) {
        if (h->broken) return HYDRO_E_STATE;
        if (!h->dt_valid && e == hipSuccess) e = enqueue_dt(h);
    }
    if (e == hipSuccess && b->use_graph) {
        if (b->graph_steps != nsteps) {
            drop_graph(b);
            e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
            for (int s = 0; s < nsteps && e == hipSuccess; ++s) e = enqueue_batch_step(b);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(b->stream, &g);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
            if (e == hipSuccess) {
                b->graph = g;
                b->graph_steps = nsteps;
            } else if (g) {
                (void)hipGraphDestroy(g);
            }
        }
        if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->stream);
    } else if (e == hipSuccess && b->groups.size() > 1 && !stream_capturing(b->stream) &&
               side_streams_ready(b)) {
        // (a caller's capture of the forked form is not attempted: the
        // refined-mesh step avoids it for the same reason)
        e = enqueue_batch_steps_streams(b, nsteps);
    } else {
        for (int s = 0; s < nsteps && e == hipSuccess; ++s) e = enqueue_batch_step(b);
    }
    if (e != hipSuccess) {
        b->broken = true;
        return HYDRO_E_DEVICE;
    }
    for (hydro_t h : b->members) h->dt_valid = true;
    return HYDRO_OK;
}

int hydro_batch_autotune(hydro_batch_t b, int steps_per_rule, int* rule_out, double* ms_per_step) {
    if (!b || !rule_out || !ms_per_step || steps_per_rule < 1 || steps_per_rule > 64) return HYDRO_E_INVAL;
    if (b->broken) return HYDRO_E_STATE;
    const int n = (int)b->members.size();
    for (hydro_t h : b->members)
        if (h->broken) return HYDRO_E_STATE;
    std::vector<BatchPlan> plans(kNumBatchRules);
    for (int r = 0; r < kNumBatchRules; ++r)
        if (!plan_batch(n, b->members.data(), plans[r], r)) return HYDRO_E_INVAL;
    drop_graph(b);
    std::vector<hipEvent_t> ev((size_t)kNumBatchRules * steps_per_rule * 2);
    size_t made = 0;
    hipError_t e = hipSuccess;
    for (; made < ev.size() && e == hipSuccess; ++made) e = hipEventCreate(&ev[made]);
    if (e != hipSuccess) --made;
    auto upload = [&](const BatchPlan& P) {
        hipError_t x = hipMemcpyAsync(b->d_desc, P.desc.data(), P.desc.size() * sizeof(MeshDesc),
                                      hipMemcpyHostToDevice, b->stream);
        if (x == hipSuccess)
            x = hipMemcpyAsync(b->d_blk, P.blk.data(), P.blk.size() * sizeof(int2), hipMemcpyHostToDevice,
                               b->stream);
        if (x == hipSuccess) x = hipStreamSynchronize(b->stream);  // P's host data in use until here
        b->groups = P.groups;
        b->order = P.order;
        assign_group_streams(b);
        return x;
    };
    for (hydro_t h : b->members)
        if (!h->dt_valid && e == hipSuccess) e = enqueue_dt(h);
    // one untimed step, then the rules in turn, round after round (real steps
    // of every member; the results do not depend on the tiles)
    if (e == hipSuccess) e = enqueue_batch_step(b);
    for (int s = 0; s < steps_per_rule && e == hipSuccess; ++s)
        for (int r = 0; r < kNumBatchRules && e == hipSuccess; ++r) {
            hipEvent_t* q = &ev[((size_t)s * kNumBatchRules + r) * 2];
            e = upload(plans[r]);
            if (e == hipSuccess) e = hipEventRecord(q[0], b->stream);
            if (e == hipSuccess) e = enqueue_batch_step(b);
            if (e == hipSuccess) e = hipEventRecord(q[1], b->stream);
        }
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    std::vector<double> ms(kNumBatchRules, 0.0);
    for (int s = 0; s < steps_per_rule && e == hipSuccess; ++s)
        for (int r = 0; r < kNumBatchRules && e == hipSuccess; ++r) {
            const hipEvent_t* q = &ev[((size_t)s * kNumBatchRules + r) * 2];
            float t = 0.0f;
            e = hipEventElapsedTime(&t, q[0], q[1]);
            ms[r] += t;
        }
    for (size_t i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    int best = 0;
    if (e == hipSuccess) {
        // rule 0 (the members' own tiles) stays unless beaten by more than 5 %
        for (int r = 1; r < kNumBatchRules; ++r)
            if (ms[r] < ms[best]) best = r;
        if (!(ms[best] < 0.95 * ms[0])) best = 0;
        for (hydro_t h : b->members)
            if (h->cfg.ndim < 3) h->tile[0] = h->tile[1] = rule_tile(h, best);
        BatchPlan P;
        if (!plan_batch(n, b->members.data(), P, 0)) e = hipErrorInvalidValue;
        if (e == hipSuccess) e = upload(P);
    }
    if (e != hipSuccess) {
        b->broken = true;
        return HYDRO_E_DEVICE;
    }
    for (hydro_t h : b->members) h->dt_valid = true;
    *rule_out = best;
    *ms_per_step = ms[best] / steps_per_rule;
    return HYDRO_OK;
}

int hydro_batch_status(hydro_batch_t b, int* done, int64_t* steps, int* flags) {
    if (!b || !done) return HYDRO_E_INVAL;
    if (b->broken) return HYDRO_E_STATE;
    const int n = (int)b->members.size();
    // every member's (done, flags, steps) gathered into one table on the
    // device, one copy, one sync
    hipError_t e = launch_status_gather(b->d_desc, n, b->d_status, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->h_status.data(), b->d_status, (size_t)n * 3 * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        b->broken = true;
        return HYDRO_E_DEVICE;
    }
    // the table is in descriptor order
    for (int k = 0; k < n; ++k) {
        const int i = b->order[k];
        done[i] = b->h_status[3 * k] ? 1 : 0;
        if (flags) flags[i] = (int)b->h_status[3 * k + 1];
        if (steps) steps[i] = (int64_t)b->h_status[3 * k + 2];
    }
    return HYDRO_OK;
}

int hydro_batch_info(hydro_batch_t b, int* groups, int64_t* workgroups, int* graph) {
    if (!b || !groups || !workgroups || !graph) return HYDRO_E_INVAL;
    *groups = (int)b->groups.size();
    int64_t nb = 0;
    for (const auto& g : b->groups) nb += g.nblk;
    *workgroups = nb;
    *graph = b->use_graph ? 1 : 0;
    return HYDRO_OK;
}

int hydro_batch_destroy(hydro_batch_t b) {
    if (!b) return HYDRO_E_INVAL;
    if (!b->broken) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    side_streams_free(b);
    delete b;
    return HYDRO_OK;
}

}  // extern "C"
