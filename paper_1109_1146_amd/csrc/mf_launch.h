// Kernel argument blocks and launch wrappers (host side of mf_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "mf_device.h"

namespace mfd {

struct DischargeArgs {
    Geo G;
    int *res, *rt, *ex;
    const int *labOld;
    int *labNew;
    int *pushb;
    int *ractive;
    const int *order;   // queue of regions in processing order
    int nwork;
    unsigned int *qhead;
    const unsigned long long *actIn;  // active-vertex count at sweep start (0 => no-op)
    int dinf;
    int *scratch;       // 4*V ints per workgroup when the search arrays do not fit in LDS
    const int *ringL;   // local indices of the tile's border vertices
    const unsigned char *ringM;  // per border vertex: bit k set if direction k leaves the tile
    int nring;
    unsigned long long *stats;   // [0] regions discharged, [1] real vertices discharged
    const int *rvcount;          // real (non-padding) vertices per region
    int *err;
    int useLDS;
    int maxIter;
    int *trace;          // optional per-discharge records (MF_TRACE_FIELDS int32 each)
    long long traceCap;
    int sweep;           // sweep index of this launch
    const int *defer;    // optional: 1 = an active region is deferred this sweep (keeps its flag)
    int *regionTicks;    // optional: duration of each region's last discharge (100 MHz ticks)
    int deferRelabel;    // a deferred region runs its region relabel only (Alg. 3, no pushes)
    // Partial discharges (Sec. 6.2): sweep s runs only the stages k <= s, s read
    // from sweepCount (the completed sweeps, so a captured graph replays it
    // right); the region relabel stays complete.  Excess may then stay inside a
    // region: such a region keeps its flag and counts itself in actCarry, which
    // the sweep's gap kernel moves into the next sweep's active count.
    int partial;
    const unsigned long long *sweepCount;
    int capShift;        // log2 of the steps per sweep (colour phases of Alg. 1: 2 or 4 steps)
    unsigned long long *actCarry;  // null unless partial or roundCap
    int roundCap;        // > 0: at most this many push rounds per discharge and sweep
    // Push-relabel region discharge (Sec. 3, Proc. PRD; HBM kernel only): labels
    // are the distance labels of Sec. 2 (d(t) = 0, every arc of length 1, dinf =
    // n) instead of region distances
    int prd;
};

// stage cap of a discharge launch (no cap: INT_MAX)
__device__ __forceinline__ int stage_cap(const DischargeArgs &A) {
    if (!A.partial) return 0x7fffffff;
    const unsigned long long s = *A.sweepCount >> A.capShift;
    return s < 0x7fffffffull ? (int)s : 0x7fffffff;
}

constexpr int kFeat = 6;  // floats per region in the scheduler features

struct FeatArgs {
    Geo G;
    const int *ex, *lab, *res;
    const int *lab2;  // the other label buffer (labels are the larger entry), or null
    const int *ringL;
    const unsigned char *ringM;
    int nring;
    int dinf;
    float *out;  // [nreg][kFeat]
    int ringOnly;  // read only border vertices (after the first sweep)
    const unsigned char *ringX;  // [nring][K] region offset of each leaving arc, 2 bits per axis (x, y, z)
};

struct SchedArgs {
    int nreg;
    const float *feat;    // [nreg][kFeat]
    const float *score;   // [nreg] logits
    float threshold;      // defer an active region when sigmoid(score) < threshold
    int maxDefer;         // ... unless it was deferred this many sweeps in a row
    int *defer, *deferCount, *order;
    const int *regionTicks;  // duration of each region's last discharge: longest first
};

constexpr int kMaxColours = 4;  // colour classes of the region grid (Alg. 1 as phases)

struct PhaseArgs {
    int ncol;
    int cstart[kMaxColours + 1];  // colour c holds corder[cstart[c] .. cstart[c + 1])
    int maxC;                     // the longest colour: entries per phase list
    const int *corder;
    const int *ractive;
    const float *score;           // [nreg] logits of the learned schedule
    int *out;                     // [ncol][maxC] region lists by phase
};

struct FuseArgs {
    Geo G;
    const int *bidx;
    int nB;
    int *res, *ex, *pushb;
    const int *lab;
    int dinf;
    unsigned int *hist;
    int *maxlab;
    const unsigned long long *actIn;
    int histOn;  // 0: the boundary relabel builds the label histogram instead
};

// Boundary relabel heuristic (Sec. 6.1): level-synchronous search over the
// boundary vertices, one workgroup per region and level.
struct BrlArgs {
    Geo G;
    const int *bidx;
    const int *bstart;   // [nreg + 1]: region r holds bidx[bstart[r] .. bstart[r+1])
    int nB;
    const int *res;
    int *lab;            // labels of the sweep (raised in place by the apply step)
    int *dist;           // [N]: d' of the boundary vertices (kInf: not reached yet)
    unsigned int *ctl;   // [4]: level counters (rotating, 3) and the ended flag
    int dinf;
    int levels;          // level launches of this run
    const unsigned long long *actIn;  // null: always run
    unsigned int *hist;  // null: no histogram
    int *maxlab;
};

struct GapArgs {
    unsigned int *hist;
    int *maxlab;
    int *gap;
    int gapOn;
    const unsigned long long *actIn;
    unsigned long long *actOut;
    unsigned int *qheadNext;
    unsigned long long *counters;  // [0] sweeps
    unsigned long long *actCarry;  // partial discharges: regions left active, or null
};

struct GapApplyArgs {
    Geo G;
    const int *bidx;
    int nB;
    int *lab;
    const int *ex;
    int *ractive;
    const int *gap;
    int dinf;
    const unsigned long long *actIn;
    unsigned long long *actOut;
};

struct FloodArgs {
    Geo G;
    int dir;     // 0: forward from excess vertices, 1: backward from t
    int round;
    int *mark;
    int *dirtyIn, *dirtyOut;
    unsigned int *changed;
    const int *res, *ex, *rt;
    int *scratch;  // V ints per workgroup
    const int *ringL;            // tile border list (row-bitmask flood)
    const unsigned char *ringM;
    int nring;
    int noCross;  // generic flood only: search inside each region, mark nothing across its border
};

struct GRelabelArgs {
    Geo G;
    int level;
    const int *res, *rt;
    int *lab;             // output labels (dinf = not reached yet)
    unsigned char *candIn, *candOut;  // seeds of this level / marks for the next
    int *flagIn, *flagOut;            // regions with seeds of this / the next level
    unsigned int *flagged;            // regions flagged for the next level
    const int *ringL;
    const unsigned char *ringM;
    int nring;
    int dinf;
    int *scratch;         // V ints per workgroup
    void *cache;          // per-region residual-arc and unlabelled masks, built at level 0
    unsigned *candBitsIn, *candBitsOut;  // seeds / marks as one bit per vertex (rows kernel)
};

hipError_t launch_grelabel(const GRelabelArgs &A, int blocks, hipStream_t s);
// Relabel level for the tiles of the rows discharge; cache: 7 * ty * tz words per region.
hipError_t launch_grelabel_rows(const GRelabelArgs &A, int blocks, hipStream_t s);
size_t grelabel_rows_lds(int ty, int tz);
hipError_t launch_grelabel_wave(const GRelabelArgs &A, int blocks, hipStream_t s);
// Relabel level for the 64^3 tiles of the 64-vertex-row discharge; cache:
// grelabel_rows64_cache_bytes(nreg) bytes.
hipError_t launch_grelabel_rows64(const GRelabelArgs &A, int blocks, hipStream_t s);
size_t grelabel_rows64_cache_bytes(int nreg);
// Cut flood round for the 64^3 tiles of the 64-vertex-row discharge.
hipError_t launch_flood_rows64(const FloodArgs &A, int blocks, hipStream_t s);
hipError_t launch_activity(const Geo &G, const int *ex, const int *lab, int dinf, int *ractive,
                           unsigned long long *act, hipStream_t s);

// Let every discharge kernel use the full LDS of a compute unit (done once,
// before any launch or stream capture).
void set_wave_attributes();
void set_rows_attributes();
void set_lds_attributes();
void set_hbm_attributes();
void set_sched_attributes();

hipError_t launch_region_features(const FeatArgs &A, hipStream_t s);
hipError_t launch_conv3_fwd(const float *x, int xs, int cin, const float *w, const float *b, int cout,
                            float *y, int D, int H, int W, int relu, int bf16, int roundIn, hipStream_t s);
hipError_t launch_conv3_bwd(const float *x, int xs, int cin, const float *w, const float *gy, int cout,
                            float *gx, float *gw, float *gb, int D, int H, int W, hipStream_t s);
hipError_t launch_relu_bwd(float *g, const float *y, int n, hipStream_t s);
hipError_t launch_bce(const float *z, const float *t, const float *m, int n, float *gz, float *loss,
                      hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);
hipError_t launch_sched_queue(const SchedArgs &A, hipStream_t s);
hipError_t launch_phase_lists(const PhaseArgs &A, hipStream_t s);

hipError_t launch_validate(const Geo &G, const int *cs, const int *ct, const int *nbr, int n,
                           int *err, hipStream_t s);
hipError_t launch_sum_links(const int *cs, const int *ct, int n, unsigned long long *out2,
                            hipStream_t s);
hipError_t launch_init(const Geo &G, const int *cs, const int *ct, const int *nbr, int n, int *res,
                       int *rt, int *ex, int *lab0, int *lab1, int *pushb, int *ractive,
                       unsigned long long *act0, hipStream_t s);
hipError_t launch_discharge(const DischargeArgs &A, int blocks, int threads, size_t lds,
                            hipStream_t s);
hipError_t launch_discharge_lds(const DischargeArgs &A, int blocks, size_t lds, int narrow,
                                hipStream_t s);
size_t discharge_lds_bytes(int V, int K, int nring, int narrow);
// mode 2: 8-bit residuals and t-links, 16-bit excess; 1: 16-bit residuals; 0: 32-bit
hipError_t launch_discharge_wave(const DischargeArgs &A, int blocks, size_t lds, int mode,
                                 hipStream_t s);
size_t discharge_wave_bytes(int V, int K, int nring, int mode);
// Row-bitmask workgroup discharge: 3D 6-connected regions with tx == 32,
// ty, tz >= 2, ty * tz a multiple of 64 and at most 1024, and at most 21 * 1024
// border vertices (rows_slots() == 0: not applicable).
hipError_t launch_discharge_rows(const DischargeArgs &A, int blocks, size_t lds, hipStream_t s);
size_t discharge_rows_bytes(int ty, int tz, int nring);
int rows_slots(int nring);
// Row-bitmask workgroup discharge for 3D 6-connected regions with tx == 64,
// ty, tz >= 2, ty * tz a multiple of 64 and at most 4096 (64^3 regions): one
// 512-thread workgroup, rows in registers, rows64_scratch_bytes() of scratch
// per workgroup at A.scratch + blockIdx.x * 16 * V bytes.
bool rows64_applicable(int K, int tx, int ty, int tz);
size_t discharge_rows64_bytes(int ty, int tz);
size_t rows64_scratch_bytes(int ty, int tz, int nring);
hipError_t launch_discharge_rows64(const DischargeArgs &A, int blocks, size_t lds, hipStream_t s);
void set_rows64_attributes();
hipError_t launch_fuse(const FuseArgs &A, hipStream_t s);
hipError_t launch_boundary_relabel(const BrlArgs &A, int stage, int first, int count, hipStream_t s);
hipError_t launch_label_hist(const int *lab, int N, int dinf, unsigned int *hist, int *maxlab,
                             const unsigned long long *actIn, hipStream_t s);
hipError_t launch_gap_raise_all(int *lab, int N, const int *gap, int dinf,
                                const unsigned long long *actIn, hipStream_t s);
hipError_t launch_gap_find(const GapArgs &A, hipStream_t s);
hipError_t launch_gap_apply(const GapApplyArgs &A, hipStream_t s);
hipError_t launch_sum_i32(const int *a, int n, unsigned long long *out, hipStream_t s);
hipError_t launch_gather_plane(const Geo &G, const int *src, int *dst, int n, hipStream_t s);
hipError_t launch_trace_labels(const Geo &G, const int *lab0, const int *lab1,
                               const unsigned long long *count, int *dst, int n, hipStream_t s);
hipError_t launch_flood(const FloodArgs &A, int blocks, hipStream_t s);
hipError_t launch_flood_wave(const FloodArgs &A, int blocks, hipStream_t s);
hipError_t launch_flood_rows(const FloodArgs &A, int blocks, hipStream_t s);
hipError_t launch_saturate_inflow(const Geo &G, const int *nbr, int n, int *res, int *ex, hipStream_t s);
hipError_t launch_label_max(int *dst, const int *other, int N, hipStream_t s);
hipError_t launch_reduce_classes(const Geo &G, const int *lab, const int *mark, unsigned char *cls,
                                 int dinf, int sinkSide, hipStream_t s);
hipError_t launch_gather_bytes(const Geo &G, const unsigned char *src, unsigned char *out, int n,
                               hipStream_t s);
hipError_t launch_cut_out(const Geo &G, const int *mark, unsigned char *out, int n, int invert,
                          hipStream_t s);
hipError_t launch_fill_i32(int *p, int n, int val, hipStream_t s);
hipError_t launch_scatter_instance(const int *cs, const int *ct, const int *nbr, int h, int w, int Ki,
                                   int *ccs, int *cct, int *cnbr, int Wc, long long nc, int y0,
                                   int x0, hipStream_t s);
hipError_t launch_instance_rt(const Geo &G, const int *rt, const int *reginst,
                              unsigned long long *instRt, hipStream_t s);
hipError_t launch_cut_rect(const Geo &G, const int *mark, unsigned char *out, int h, int w, int y0,
                           int x0, int invert, hipStream_t s);

}  // namespace mfd
