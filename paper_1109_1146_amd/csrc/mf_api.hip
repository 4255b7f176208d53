// C ABI of the region-discharge max-flow solver (see include/mf.h): handle,
// validation, region partition and boundary builder, sweep driver, results.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <mutex>
#include <vector>

#include "mf.h"
#include "mf_launch.h"

using mfd::Geo;
typedef unsigned long long u64;

struct mf_grid {
    Geo G;
    int ndim = 0, conn = 0, K = 0;
    long long n = 0;
    long long nB = 0;
    int dinf = 1;
    int nring = 0;
    int device = 0;
    int numCU = 0;
    // device state
    int *res = nullptr, *rt = nullptr, *ex = nullptr, *lab[2] = {nullptr, nullptr};
    int *pushb = nullptr, *ractive = nullptr, *order = nullptr, *bidx = nullptr;
    int *bstart = nullptr;        // [nreg + 1]: the boundary vertices of region r are bidx[bstart[r]..bstart[r+1])
    int *corder = nullptr;        // regions grouped by colour (MF_SCHED_COLORED), built on first use
    int corder_ncol = 0;
    int *plists = nullptr;        // learned colour phases: [ncol][phase_maxc] region lists by phase
    int phase_maxc = 0;
    std::vector<int> cstart;      // colour c holds corder[cstart[c] .. cstart[c+1])
    std::vector<int> corder_host;
    unsigned int *brlctl = nullptr;  // boundary relabel control words
    int *ringL = nullptr, *rvcount = nullptr, *mark = nullptr, *dirty = nullptr;
    unsigned char *ringM = nullptr, *cutbuf = nullptr, *cand = nullptr;  // cand: 2 x N
    unsigned char *ringX = nullptr;  // per border vertex and leaving direction: region offset (2 bits per axis)
    int *in_cs = nullptr, *in_ct = nullptr, *in_nbr = nullptr;
    int *scratch = nullptr;
    int nslots = 0;
    bool useLDS = false;
    size_t ldsMax = 0;            // LDS bytes a workgroup may use
    int maxPair = 0, maxCt = 0;   // largest c(u,v)+c(v,u) and c(v,t) of the loaded instance
    int maxIn = 0;                // largest c(s,v) + sum_u c(u,v): bounds every excess
    int threads = 256;
    // device control block
    u64 *act = nullptr;           // [2]
    unsigned int *qhead = nullptr;  // [2]
    unsigned int *hist = nullptr;
    int *maxlab = nullptr, *gap = nullptr, *err = nullptr;
    u64 *counters = nullptr;      // [0] sweeps
    u64 *stats = nullptr;         // [0] discharges [1] vertices
    u64 *sums = nullptr;          // [0] sum cs [1] sum ct [2] sum rt
    unsigned int *changed = nullptr;
    void *gcache = nullptr;        // global relabel: per-region masks (allocated on first use)
    size_t gcache_bytes = 0;
    int *tmp_plane = nullptr;
    u64 *pinned = nullptr;        // host pinned mailbox
    // instance state
    bool has_caps = false, solved = false;
    bool has_state = false;       // a solve left a state (completed, or stopped by max_sweeps)
    bool state_prd = false;       // that state carries distance labels (MF_METHOD_PRD)
    long long sum_cs = 0, sum_ct = 0, flow = 0;
    int final_parity = 0;
    int cut_kind_cached = -1;     // kind whose reachability marks g->mark holds
    // batch handles: independent 2D instances packed on one canvas
    int batch = 0;                // number of instances; 0 for a single grid
    std::vector<int> iy0, ix0, ih, iw, iconn;
    std::vector<long long> isum_cs, isum_ct, iflow;
    std::vector<int> imaxpair, imaxct, imaxin;
    std::vector<char> iloaded;
    int *reginst = nullptr;       // instance of each region (-1: canvas padding)
    int *stage = nullptr;         // one instance's caps on their way to the canvas
    u64 *instRt = nullptr;        // per-instance sum of residual t-links
    // learned schedule
    float *feat = nullptr, *score = nullptr;
    int *defer = nullptr, *deferCount = nullptr, *lorder = nullptr, *rticks = nullptr;
    // captured sweep batches
    hipStream_t own_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    long long graph_key = -1;
};

static bool ok(hipError_t e) { return e == hipSuccess; }
#define HIP_TRY(x)                         \
    do {                                   \
        if (!ok(x)) return MF_E_DEVICE;    \
    } while (0)

template <typename T>
static hipError_t dalloc(T **p, size_t count) {
    if (count == 0) count = 1;
    return hipMalloc((void **)p, count * sizeof(T));
}

static void free_all(mf_grid *g) {
    void *ptrs[] = {g->res, g->rt, g->ex, g->lab[0], g->lab[1], g->pushb, g->ractive, g->order,
                    g->bidx, g->ringL, g->rvcount, g->mark, g->dirty, g->ringM, g->ringX, g->cutbuf,
                    g->in_cs, g->in_ct, g->in_nbr, g->scratch, g->act, g->qhead, g->hist,
                    g->maxlab, g->gap, g->err, g->counters, g->stats, g->sums, g->changed,
                    g->tmp_plane, g->cand, g->bstart, g->brlctl, g->corder, g->plists};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (g->reginst) (void)hipFree(g->reginst);
    {
        void *q[] = {g->feat, g->score, g->defer, g->deferCount, g->lorder, g->rticks};
        for (void *x : q)
            if (x) (void)hipFree(x);
    }
    if (g->stage) (void)hipFree(g->stage);
    if (g->instRt) (void)hipFree(g->instRt);
    if (g->gcache) (void)hipFree(g->gcache);
    if (g->graph_exec) (void)hipGraphExecDestroy(g->graph_exec);
    if (g->own_stream) (void)hipStreamDestroy(g->own_stream);
    if (g->pinned) (void)hipHostFree(g->pinned);
}

static constexpr int8_t OFF2D[8][2] = {{0, 1}, {0, -1}, {1, 0}, {-1, 0}, {1, 1}, {-1, -1}, {-1, 1}, {1, -1}};
// the 2D kernels use the same order as compile-time constants
static constexpr bool off2d_matches() {
    for (int k = 0; k < 8; k++)
        if (OFF2D[k][0] != mfd::off2d_dy(k) || OFF2D[k][1] != mfd::off2d_dx(k)) return false;
    return true;
}
static_assert(off2d_matches(), "2D direction table and the kernels' constants differ");
static const int8_t OFF3D[6][3] = {{0, 0, 1}, {0, 0, -1}, {0, 1, 0}, {0, -1, 0}, {1, 0, 0}, {-1, 0, 0}};

extern "C" const char *mf_status_str(mf_status s) {
    switch (s) {
        case MF_OK: return "ok";
        case MF_E_INVAL: return "invalid argument";
        case MF_E_NOMEM: return "out of memory";
        case MF_E_DEVICE: return "device error";
        case MF_E_STATE: return "call order violated";
        case MF_E_OVERFLOW: return "capacities could overflow int32";
        case MF_E_SWEEPS: return "sweep limit reached";
    }
    return "unknown status";
}

extern "C" int64_t mf_discharge_bytes_per_vertex(int32_t connectivity) {
    // read K residuals + t-link + excess, write them back, write the label
    return (int64_t)(2 * connectivity + 5) * 4;
}

static mf_status create_impl(int32_t ndim, const int64_t *dims, int32_t connectivity,
                             const int32_t *region_shape, mf_grid **out);

extern "C" mf_status mf_create_grid(int32_t ndim, const int64_t *dims, int32_t connectivity,
                                    const int32_t *region_shape, mf_grid **out) {
    return create_impl(ndim, dims, connectivity, region_shape, out);
}

static mf_status create_impl(int32_t ndim, const int64_t *dims, int32_t connectivity,
                             const int32_t *region_shape, mf_grid **out) {
    if (!out || !dims || (ndim != 2 && ndim != 3)) return MF_E_INVAL;
    if (ndim == 2 && connectivity != 4 && connectivity != 8) return MF_E_INVAL;
    if (ndim == 3 && connectivity != 6) return MF_E_INVAL;
    long long d[3] = {1, 1, 1};
    for (int i = 0; i < ndim; i++) {
        if (dims[i] < 1) return MF_E_INVAL;
        d[3 - ndim + i] = dims[i];
    }
    long long n = d[0] * d[1] * d[2];
    if (n >= (1LL << 31)) return MF_E_INVAL;
    int t[3] = {1, 1, 1};
    bool given = region_shape != nullptr;
    if (given) {
        bool allzero = true;
        for (int i = 0; i < ndim; i++) allzero = allzero && region_shape[i] == 0;
        if (allzero) given = false;
    }
    for (int i = 0; i < ndim; i++) {
        int ax = 3 - ndim + i;
        if (given) {
            if (region_shape[i] < 1) return MF_E_INVAL;
            t[ax] = (int)std::min<long long>(region_shape[i], d[ax]);
        } else {
            t[ax] = (int)std::min<long long>(ndim == 2 ? 64 : 32, d[ax]);
        }
    }
    mf_grid *g = new (std::nothrow) mf_grid();
    if (!g) return MF_E_NOMEM;
    Geo &G = g->G;
    memset(&G, 0, sizeof(G));
    G.K = connectivity;
    G.dz = (int)d[0]; G.dy = (int)d[1]; G.dx = (int)d[2];
    G.tz = t[0]; G.ty = t[1]; G.tx = t[2];
    G.rz = (int)((d[0] + t[0] - 1) / t[0]);
    G.ry = (int)((d[1] + t[1] - 1) / t[1]);
    G.rx = (int)((d[2] + t[2] - 1) / t[2]);
    long long V = (long long)t[0] * t[1] * t[2];
    long long nreg = (long long)G.rz * G.ry * G.rx;
    if (V * nreg * std::max(connectivity, 1) >= (1LL << 31) * 4LL || V * nreg >= (1LL << 31) || V > (1 << 20)) {
        delete g;
        return MF_E_INVAL;
    }
    G.V = (int)V;
    G.nreg = (int)nreg;
    G.N = (int)(V * nreg);
    for (int k = 0; k < connectivity; k++) {
        if (ndim == 2) {
            G.oz[k] = 0; G.oy[k] = OFF2D[k][0]; G.ox[k] = OFF2D[k][1];
        } else {
            G.oz[k] = OFF3D[k][0]; G.oy[k] = OFF3D[k][1]; G.ox[k] = OFF3D[k][2];
        }
    }
    g->ndim = ndim;
    g->conn = connectivity;
    g->K = connectivity;
    g->n = n;

    // tile border ("ring"): local vertices with a direction leaving the tile
    std::vector<int> ringL;
    std::vector<unsigned char> ringM, ringX;
    for (int l = 0; l < G.V; l++) {
        int lx = l % G.tx, tt = l / G.tx, ly = tt % G.ty, lz = tt / G.ty;
        unsigned m = 0;
        unsigned char xo[mfd::kMaxK] = {0};
        for (int k = 0; k < G.K; k++) {
            int z = lz + G.oz[k], y = ly + G.oy[k], x = lx + G.ox[k];
            if (x < 0 || x >= G.tx || y < 0 || y >= G.ty || z < 0 || z >= G.tz) {
                m |= 1u << k;
                auto code = [](int c, int t) { return c < 0 ? 2 : (c >= t ? 1 : 0); };
                xo[k] = (unsigned char)(code(x, G.tx) | code(y, G.ty) << 2 | code(z, G.tz) << 4);
            }
        }
        if (m) {
            ringL.push_back(l);
            ringM.push_back((unsigned char)m);
            for (int k = 0; k < G.K; k++) ringX.push_back(xo[k]);
        }
    }
    g->nring = (int)ringL.size();
    // boundary set B (Sec. 4.1): real vertices with a real grid neighbour in another region
    std::vector<int> bidx;
    std::vector<int> rvcount(G.nreg);
    std::vector<int> bstart(G.nreg + 1, 0);
    for (int r = 0; r < G.nreg; r++) {
        bstart[r] = (int)bidx.size();
        int rx = r % G.rx, tt = r / G.rx, ry = tt % G.ry, rz = tt / G.ry;
        int oz = rz * G.tz, oy = ry * G.ty, ox = rx * G.tx;
        rvcount[r] = std::min(G.tz, G.dz - oz) * std::min(G.ty, G.dy - oy) * std::min(G.tx, G.dx - ox);
        for (size_t i = 0; i < ringL.size(); i++) {
            int l = ringL[i];
            int lx = l % G.tx, t2 = l / G.tx, ly = t2 % G.ty, lz = t2 / G.ty;
            int z = oz + lz, y = oy + ly, x = ox + lx;
            if (z >= G.dz || y >= G.dy || x >= G.dx) continue;
            bool inB = false;
            for (int k = 0; k < G.K && !inB; k++) {
                if (!((ringM[i] >> k) & 1u)) continue;
                int zz = z + G.oz[k], yy = y + G.oy[k], xx = x + G.ox[k];
                if (zz >= 0 && zz < G.dz && yy >= 0 && yy < G.dy && xx >= 0 && xx < G.dx) inB = true;
            }
            if (inB) bidx.push_back(r * G.V + l);
        }
    }
    bstart[G.nreg] = (int)bidx.size();
    g->nB = (long long)bidx.size();
    g->dinf = g->nB > 0 ? (int)g->nB : 1;

    static bool attributes_set = false;
    if (!attributes_set) {
        mfd::set_wave_attributes();
        mfd::set_rows_attributes();
        mfd::set_rows64_attributes();
        mfd::set_lds_attributes();
        mfd::set_hbm_attributes();
        mfd::set_sched_attributes();
        attributes_set = true;
    }
    hipDeviceProp_t prop;
    if (!ok(hipGetDevice(&g->device)) || !ok(hipGetDeviceProperties(&prop, g->device))) {
        delete g;
        return MF_E_DEVICE;
    }
    g->numCU = prop.multiProcessorCount;
    g->ldsMax = (size_t)prop.sharedMemPerBlock;
    // regions of 8K vertices and more on the HBM kernel are bound by memory
    // latency: a 1024-thread workgroup keeps more loads in flight
    g->threads = G.V >= 8192 ? 1024 : 256;
    // the four search arrays (16 B per vertex) live in LDS when they fit beside
    // the kernel's static shared words; otherwise in per-workgroup HBM scratch
    g->useLDS = (size_t)16 * G.V + 1024 <= (size_t)prop.sharedMemPerBlock;
    g->nslots = std::max(1, std::min(G.nreg, 2 * g->numCU));

    size_t N = (size_t)G.N, K = (size_t)G.K;
    bool good = ok(dalloc(&g->res, K * N)) && ok(dalloc(&g->pushb, K * N)) &&
                ok(dalloc(&g->rt, N)) && ok(dalloc(&g->ex, N)) && ok(dalloc(&g->lab[0], N)) &&
                ok(dalloc(&g->lab[1], N)) && ok(dalloc(&g->mark, N)) &&
                ok(dalloc(&g->ractive, (size_t)G.nreg)) && ok(dalloc(&g->order, (size_t)G.nreg)) &&
                ok(dalloc(&g->rvcount, (size_t)G.nreg)) && ok(dalloc(&g->dirty, 2 * (size_t)G.nreg)) &&
                ok(dalloc(&g->bidx, (size_t)g->nB)) && ok(dalloc(&g->ringL, (size_t)g->nring)) &&
                ok(dalloc(&g->ringM, (size_t)g->nring)) && ok(dalloc(&g->ringX, (size_t)g->nring * G.K)) &&
                ok(dalloc(&g->cutbuf, (size_t)n)) &&
                ok(dalloc(&g->cand, 2 * N)) &&
                ok(dalloc(&g->in_cs, (size_t)n)) && ok(dalloc(&g->in_ct, (size_t)n)) &&
                ok(dalloc(&g->in_nbr, K * (size_t)n)) && ok(dalloc(&g->tmp_plane, (size_t)n)) &&
                ok(dalloc(&g->scratch, (size_t)g->nslots * 4 * G.V)) && ok(dalloc(&g->act, 4)) &&
                ok(dalloc(&g->qhead, 4)) && ok(dalloc(&g->hist, (size_t)mfd::kHistBins)) &&
                ok(dalloc(&g->maxlab, 1)) && ok(dalloc(&g->gap, 1)) && ok(dalloc(&g->err, 4)) &&
                ok(dalloc(&g->counters, 4)) && ok(dalloc(&g->stats, 16)) && ok(dalloc(&g->sums, 4)) &&
                ok(dalloc(&g->changed, 8)) && ok(dalloc(&g->bstart, (size_t)G.nreg + 1)) &&
                ok(dalloc(&g->brlctl, 8)) &&
                ok(hipHostMalloc((void **)&g->pinned, 32 * sizeof(u64), hipHostMallocDefault));
    if (!good) {
        (void)hipGetLastError();
        free_all(g);
        delete g;
        return MF_E_NOMEM;
    }
    std::vector<int> order(G.nreg);
    for (int r = 0; r < G.nreg; r++) order[r] = r;
    good = ok(hipMemcpy(g->order, order.data(), sizeof(int) * G.nreg, hipMemcpyHostToDevice)) &&
           ok(hipMemcpy(g->rvcount, rvcount.data(), sizeof(int) * G.nreg, hipMemcpyHostToDevice)) &&
           ok(hipMemcpy(g->bstart, bstart.data(), sizeof(int) * (G.nreg + 1), hipMemcpyHostToDevice)) &&
           (bidx.empty() || ok(hipMemcpy(g->bidx, bidx.data(), sizeof(int) * bidx.size(), hipMemcpyHostToDevice))) &&
           (ringL.empty() || ok(hipMemcpy(g->ringL, ringL.data(), sizeof(int) * ringL.size(), hipMemcpyHostToDevice))) &&
           (ringM.empty() || ok(hipMemcpy(g->ringM, ringM.data(), ringM.size(), hipMemcpyHostToDevice))) &&
           (ringX.empty() || ok(hipMemcpy(g->ringX, ringX.data(), ringX.size(), hipMemcpyHostToDevice)));
    if (!good) {
        free_all(g);
        delete g;
        return MF_E_DEVICE;
    }
    *out = g;
    return MF_OK;
}

extern "C" void mf_destroy(mf_grid *g) {
    if (!g) return;
    (void)hipDeviceSynchronize();
    free_all(g);
    delete g;
}

extern "C" mf_status mf_get_info(const mf_grid *g, int64_t *n, int32_t *K, int64_t *regions,
                                 int64_t *boundary_size, int32_t *region_shape3) {
    if (!g) return MF_E_INVAL;
    if (n) *n = g->n;
    if (K) *K = g->K;
    if (regions) *regions = g->G.nreg;
    if (boundary_size) *boundary_size = g->nB;
    if (region_shape3) {
        region_shape3[0] = g->G.tz;
        region_shape3[1] = g->G.ty;
        region_shape3[2] = g->G.tx;
    }
    return MF_OK;
}

extern "C" mf_status mf_set_caps(mf_grid *g, const int32_t *src_cap, const int32_t *sink_cap,
                                 const int32_t *nbr_cap, int32_t on_device, void *stream) {
    if (!g || !src_cap || !sink_cap || !nbr_cap || g->batch) return MF_E_INVAL;
    g->cut_kind_cached = -1;
    hipStream_t s = (hipStream_t)stream;
    g->has_caps = false;
    g->solved = false;
    size_t n = (size_t)g->n, K = (size_t)g->K;
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIP_TRY(hipMemcpyAsync(g->in_cs, src_cap, n * sizeof(int), kind, s));
    HIP_TRY(hipMemcpyAsync(g->in_ct, sink_cap, n * sizeof(int), kind, s));
    HIP_TRY(hipMemcpyAsync(g->in_nbr, nbr_cap, K * n * sizeof(int), kind, s));
    HIP_TRY(hipMemsetAsync(g->err, 0, 4 * sizeof(int), s));
    HIP_TRY(hipMemsetAsync(g->sums, 0, 4 * sizeof(u64), s));
    HIP_TRY(mfd::launch_validate(g->G, g->in_cs, g->in_ct, g->in_nbr, (int)n, g->err, s));
    HIP_TRY(mfd::launch_sum_links(g->in_cs, g->in_ct, (int)n, g->sums, s));
    HIP_TRY(hipMemcpyAsync(g->pinned, g->sums, 2 * sizeof(u64), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(g->pinned + 2, g->err, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int err = ((int *)(g->pinned + 2))[0];
    g->maxPair = ((int *)(g->pinned + 2))[1];
    g->maxCt = ((int *)(g->pinned + 2))[2];
    g->maxIn = ((int *)(g->pinned + 2))[3];
    if (err & 1) return MF_E_INVAL;
    if (err & 2) return MF_E_OVERFLOW;
    g->sum_cs = (long long)g->pinned[0];
    g->sum_ct = (long long)g->pinned[1];
    g->has_caps = true;
    return MF_OK;
}

// ---------------------------------------------------------------------------
// Learned region scheduler model: 3 -> C -> C -> 1 channel 3x3x3 CNN over the
// region grid (parameter layout in mf_sched.hip), FP32 master parameters,
// Adam state, and a workspace sized for the largest region grid seen.
// ---------------------------------------------------------------------------
struct mf_model {
    int C = 16;
    int P = 0;  // number of parameters
    float *params = nullptr, *grads = nullptr, *am = nullptr, *av = nullptr;
    int step = 0;
    int cap = 0;  // voxels the workspace holds
    float *h1 = nullptr, *h2 = nullptr, *z = nullptr, *gz = nullptr, *gh2 = nullptr, *gh1 = nullptr;
    float *loss = nullptr;
    float *hloss = nullptr;  // pinned
    size_t off_w1 = 0, off_b1 = 0, off_w2 = 0, off_b2 = 0, off_w3 = 0, off_b3 = 0;
};

static void model_free_ws(mf_model *m) {
    float *p[] = {m->h1, m->h2, m->z, m->gz, m->gh2, m->gh1};
    for (float *q : p)
        if (q) (void)hipFree(q);
    m->h1 = m->h2 = m->z = m->gz = m->gh2 = m->gh1 = nullptr;
    m->cap = 0;
}

static bool model_ws(mf_model *m, int nv) {
    if (nv <= m->cap) return true;
    model_free_ws(m);
    const size_t C = (size_t)m->C;
    if (!ok(dalloc(&m->h1, C * nv)) || !ok(dalloc(&m->h2, C * nv)) || !ok(dalloc(&m->z, (size_t)nv)) ||
        !ok(dalloc(&m->gz, (size_t)nv)) || !ok(dalloc(&m->gh2, C * nv)) || !ok(dalloc(&m->gh1, C * nv)))
        return false;
    m->cap = nv;
    return true;
}

static uint64_t splitmix64(uint64_t &x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

extern "C" mf_status mf_model_create(int32_t channels, uint64_t seed, mf_model **out) {
    if (!out || channels < 1 || channels > 64) return MF_E_INVAL;
    mf_model *m = new (std::nothrow) mf_model();
    if (!m) return MF_E_NOMEM;
    const int C = channels;
    m->C = C;
    m->off_w1 = 0;
    m->off_b1 = m->off_w1 + (size_t)C * 3 * 27;
    m->off_w2 = m->off_b1 + C;
    m->off_b2 = m->off_w2 + (size_t)C * C * 27;
    m->off_w3 = m->off_b2 + C;
    m->off_b3 = m->off_w3 + (size_t)C * 27;
    m->P = (int)(m->off_b3 + 1);
    std::vector<float> h(m->P, 0.f);
    uint64_t st = seed;
    auto fill = [&](size_t off, size_t n, int fan_in) {
        const double a = std::sqrt(6.0 / fan_in);  // He-uniform
        for (size_t i = 0; i < n; i++) {
            const double u = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
            h[off + i] = (float)((2.0 * u - 1.0) * a);
        }
    };
    fill(m->off_w1, (size_t)C * 3 * 27, 3 * 27);
    fill(m->off_w2, (size_t)C * C * 27, C * 27);
    fill(m->off_w3, (size_t)C * 27, C * 27);
    bool good = ok(dalloc(&m->params, (size_t)m->P)) && ok(dalloc(&m->grads, (size_t)m->P)) &&
                ok(dalloc(&m->am, (size_t)m->P)) && ok(dalloc(&m->av, (size_t)m->P)) &&
                ok(dalloc(&m->loss, 1)) &&
                ok(hipHostMalloc((void **)&m->hloss, sizeof(float), hipHostMallocDefault)) &&
                ok(hipMemcpy(m->params, h.data(), sizeof(float) * m->P, hipMemcpyHostToDevice)) &&
                ok(hipMemset(m->grads, 0, sizeof(float) * m->P)) && ok(hipMemset(m->am, 0, sizeof(float) * m->P)) &&
                ok(hipMemset(m->av, 0, sizeof(float) * m->P));
    if (!good) {
        mf_model_destroy(m);
        return MF_E_NOMEM;
    }
    *out = m;
    return MF_OK;
}

extern "C" void mf_model_destroy(mf_model *m) {
    if (!m) return;
    (void)hipDeviceSynchronize();
    model_free_ws(m);
    float *p[] = {m->params, m->grads, m->am, m->av, m->loss};
    for (float *q : p)
        if (q) (void)hipFree(q);
    if (m->hloss) (void)hipHostFree(m->hloss);
    delete m;
}

extern "C" int64_t mf_model_num_params(const mf_model *m) { return m ? m->P : 0; }

extern "C" mf_status mf_model_get_params(const mf_model *m, float *host_out) {
    if (!m || !host_out) return MF_E_INVAL;
    HIP_TRY(hipMemcpy(host_out, m->params, sizeof(float) * m->P, hipMemcpyDeviceToHost));
    return MF_OK;
}

extern "C" mf_status mf_model_set_params(mf_model *m, const float *host_in) {
    if (!m || !host_in) return MF_E_INVAL;
    HIP_TRY(hipMemcpy(m->params, host_in, sizeof(float) * m->P, hipMemcpyHostToDevice));
    return MF_OK;
}

// The three convolutions, with the hidden activations in h1 and h2 (C floats per voxel each).
static hipError_t model_forward_in(const mf_model *m, const float *x, int xs, int D, int H, int W, float *z,
                                   int bf16, float *h1, float *h2, hipStream_t s) {
    const int C = m->C;
    const float *p = m->params;
    hipError_t e = mfd::launch_conv3_fwd(x, xs, 3, p + m->off_w1, p + m->off_b1, C, h1, D, H, W, 1, bf16, 1, s);
    if (e != hipSuccess) return e;
    e = mfd::launch_conv3_fwd(h1, C, C, p + m->off_w2, p + m->off_b2, C, h2, D, H, W, 1, bf16, 0, s);
    if (e != hipSuccess) return e;
    return mfd::launch_conv3_fwd(h2, C, C, p + m->off_w3, p + m->off_b3, 1, z, D, H, W, 0, bf16, 0, s);
}

static hipError_t model_forward(mf_model *m, const float *x, int xs, int D, int H, int W, float *z,
                                int bf16, hipStream_t s) {
    return model_forward_in(m, x, xs, D, H, W, z, bf16, m->h1, m->h2, s);
}

extern "C" mf_status mf_model_forward(mf_model *m, const float *x, int32_t xs, int32_t D, int32_t H,
                                      int32_t W, float *logits, int32_t bf16, void *stream) {
    if (!m || !x || !logits || xs < 3 || D < 1 || H < 1 || W < 1) return MF_E_INVAL;
    if (!model_ws(m, D * H * W)) return MF_E_NOMEM;
    HIP_TRY(model_forward(m, x, xs, D, H, W, logits, bf16 ? 1 : 0, (hipStream_t)stream));
    return MF_OK;
}

// ---- Scheduler inference without allocation ----
// The hidden activations of mf_model_forward_noalloc live in a fixed device
// array (4 MiB), one copy per GPU, held until the process ends and shared by
// every call on that GPU.  Host code uses the array only through the address
// hipGetSymbolAddress returns for the current device (taken once per device).
constexpr size_t kNoAllocFloats = (size_t)1 << 20;
static __device__ __align__(256) float scratch[kNoAllocFloats];
constexpr int kNoAllocDevices = 64;
static std::mutex g_noalloc_mu;
static float *g_noalloc_ptr[kNoAllocDevices] = {};

static mf_status noalloc_scratch(float **out) {
    int dev = 0;
    if (!ok(hipGetDevice(&dev)) || dev < 0 || dev >= kNoAllocDevices) return MF_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        if (!ok(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) || !p) return MF_E_DEVICE;
        g_noalloc_ptr[dev] = (float *)p;
    }
    *out = g_noalloc_ptr[dev];
    return MF_OK;
}

extern "C" mf_status mf_model_forward_noalloc(const mf_model *m, const float *x, int32_t xs, int32_t D,
                                              int32_t H, int32_t W, float *logits, int32_t bf16,
                                              void *stream) {
    if (!m || !x || !logits || xs < 3 || D < 1 || H < 1 || W < 1) return MF_E_INVAL;
    const long long nv = (long long)D * H * W;
    if (nv > (long long)(kNoAllocFloats / 2) / m->C) return MF_E_INVAL;  // two hidden layers must fit
    float *ws = nullptr;
    const mf_status st = noalloc_scratch(&ws);
    if (st != MF_OK) return st;
    // every activation is written before it is read: nothing to clear
    HIP_TRY(model_forward_in(m, x, xs, D, H, W, logits, bf16 ? 1 : 0, ws, ws + (size_t)m->C * nv,
                             (hipStream_t)stream));
    return MF_OK;
}

extern "C" mf_status mf_model_loss_grad(mf_model *m, const float *x, int32_t xs, const float *target,
                                        const float *mask, int32_t D, int32_t H, int32_t W,
                                        float *loss, float *grads_out, void *stream) {
    if (!m || !x || !target || !mask || xs < 3 || D < 1 || H < 1 || W < 1) return MF_E_INVAL;
    const int nv = D * H * W, C = m->C;
    if (!model_ws(m, nv)) return MF_E_NOMEM;
    hipStream_t s = (hipStream_t)stream;
    float *g = m->grads;
    const float *p = m->params;
    HIP_TRY(model_forward(m, x, xs, D, H, W, m->z, 0, s));
    HIP_TRY(mfd::launch_bce(m->z, target, mask, nv, m->gz, m->loss, s));
    HIP_TRY(mfd::launch_conv3_bwd(m->h2, C, C, p + m->off_w3, m->gz, 1, m->gh2, g + m->off_w3, g + m->off_b3,
                                  D, H, W, s));
    HIP_TRY(mfd::launch_relu_bwd(m->gh2, m->h2, nv * C, s));
    HIP_TRY(mfd::launch_conv3_bwd(m->h1, C, C, p + m->off_w2, m->gh2, C, m->gh1, g + m->off_w2, g + m->off_b2,
                                  D, H, W, s));
    HIP_TRY(mfd::launch_relu_bwd(m->gh1, m->h1, nv * C, s));
    HIP_TRY(mfd::launch_conv3_bwd(x, xs, 3, p + m->off_w1, m->gh1, C, nullptr, g + m->off_w1, g + m->off_b1,
                                  D, H, W, s));
    HIP_TRY(hipMemcpyAsync(m->hloss, m->loss, sizeof(float), hipMemcpyDeviceToHost, s));
    if (grads_out) HIP_TRY(hipMemcpyAsync(grads_out, g, sizeof(float) * m->P, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (loss) *loss = *m->hloss;
    return MF_OK;
}

extern "C" mf_status mf_model_adam_step(mf_model *m, float lr, void *stream) {
    if (!m || !(lr > 0.f)) return MF_E_INVAL;
    m->step++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
    HIP_TRY(mfd::launch_adam(m->params, m->grads, m->am, m->av, m->P, lr, b1, b2, 1e-8f, c1, c2,
                             (hipStream_t)stream));
    return MF_OK;
}

// Exact region-distance labels into lab (see k_grelabel), then the active
// regions and the active-vertex count *act for the next sweep.  Returns the
// number of distance levels, or -1 on a HIP error.
static int global_relabel(mf_grid *g, int *lab, u64 *act, hipStream_t s) {
    const Geo &G = g->G;
    if (!ok(mfd::launch_fill_i32(lab, G.N, g->dinf, s))) return -1;
    if (!ok(hipMemsetAsync(g->cand, 0, 2 * (size_t)G.N, s))) return -1;
    if (!ok(hipMemsetAsync(g->dirty, 0, sizeof(int) * 2 * (size_t)G.nreg, s))) return -1;
    mfd::GRelabelArgs A;
    memset(&A, 0, sizeof(A));
    A.G = G;
    A.res = g->res; A.rt = g->rt; A.lab = lab;
    A.ringL = g->ringL; A.ringM = g->ringM; A.nring = g->nring; A.dinf = g->dinf;
    A.scratch = g->scratch;
    // 2D regions of at most 64 x 64: one wavefront per region, row-bitmask flood;
    // 3D regions with 32-vertex rows: one workgroup per region, row-bitmask flood;
    // both keep the region's masks in a cache built at level 0
    const int R = G.ty * G.tz;
    const bool wave = g->ndim == 2 && G.tx <= 64 && G.ty <= 64;
    const bool rows = g->ndim == 3 && G.K == 6 && G.tx == 32 && G.ty >= 2 && G.tz >= 2 &&
                      R % 64 == 0 && R <= 1024;
    // 3D 64^3 regions: one workgroup per region, 64-bit rows in registers
    const bool rows64 = g->ndim == 3 && mfd::rows64_applicable(G.K, G.tx, G.ty, G.tz);
    if (wave || rows || rows64) {
        const size_t need = wave ? (size_t)G.nreg * (G.K + 1) * 64 * sizeof(u64)
                                 : (rows ? (size_t)G.nreg * 7 * R * sizeof(unsigned)
                                         : mfd::grelabel_rows64_cache_bytes(G.nreg));
        if (g->gcache_bytes < need) {
            if (g->gcache) (void)hipFree(g->gcache);
            g->gcache = nullptr;
            g->gcache_bytes = 0;
            if (!ok(hipMalloc(&g->gcache, need))) return -1;
            g->gcache_bytes = need;
        }
        A.cache = g->gcache;
    }
    const int blocks = wave ? std::min(G.nreg, g->numCU * 8)
                            : ((rows || rows64) ? std::min(G.nreg, g->numCU * 2) : std::min(G.nreg, g->nslots * 4));
    // levels are launched in batches; a level with no flagged region is a cheap no-op
    const int batch = 4;
    int D = 0;
    for (;;) {
        for (int j = 0; j < batch; j++) {
            const int lv = D + j;
            A.level = lv;
            A.candIn = g->cand + (size_t)(lv & 1) * G.N;
            A.candOut = g->cand + (size_t)((lv + 1) & 1) * G.N;
            A.flagIn = g->dirty + (size_t)(lv & 1) * G.nreg;
            A.flagOut = g->dirty + (size_t)((lv + 1) & 1) * G.nreg;
            A.flagged = g->changed + j;
            A.candBitsIn = (unsigned *)g->cand + (size_t)(lv & 1) * (G.N / 32);
            A.candBitsOut = (unsigned *)g->cand + (size_t)((lv + 1) & 1) * (G.N / 32);
            if (!ok(hipMemsetAsync(g->changed + j, 0, sizeof(unsigned), s))) return -1;
            hipError_t e = wave ? mfd::launch_grelabel_wave(A, blocks, s)
                                : (rows ? mfd::launch_grelabel_rows(A, blocks, s)
                                        : (rows64 ? mfd::launch_grelabel_rows64(A, blocks, s)
                                                  : mfd::launch_grelabel(A, blocks, s)));
            if (!ok(e)) return -1;
        }
        if (!ok(hipMemcpyAsync(g->pinned + 14, g->changed + batch - 1, sizeof(unsigned), hipMemcpyDeviceToHost, s)))
            return -1;
        if (!ok(hipStreamSynchronize(s))) return -1;
        D += batch;
        if (*(unsigned *)(g->pinned + 14) == 0u) break;
        if (D > g->dinf + batch + 1) return -1;
    }
    if (!ok(hipMemsetAsync(g->ractive, 0, sizeof(int) * G.nreg, s))) return -1;
    if (!ok(hipMemsetAsync(act, 0, sizeof(u64), s))) return -1;
    if (!ok(mfd::launch_activity(G, g->ex, lab, g->dinf, g->ractive, act, s))) return -1;
    return D;
}

// Which region kernel runs the discharges (MF_KERNEL_* request, AUTO = the
// first that applies), its dynamic LDS, storage width and grid size.
struct RegionPick {
    int mode;  // 0: HBM, 1: LDS workgroup, 2: wavefront, 3: row-bitmask workgroup, 4: 64-bit rows
    size_t lds;
    int narrow;
    int blocks;
};

static mf_status pick_region(const mf_grid *g, int region_kernel, bool prd, RegionPick &P) {
    const Geo &G = g->G;
    // Region kernels: a single wavefront with row bitmasks for 2D regions of
    // at most 64 x 64 (WAVE), one workgroup with the whole region in LDS
    // (LDS), or the region left in HBM (HBM).  LDS-resident residuals are int16
    // when every residual (bounded by its pair sum) and t-link fits, else int32.
    const size_t ldsBudget = g->ldsMax > 512 ? g->ldsMax - 512 : 0;
    const bool narrowOk = g->maxPair <= 32767 && g->maxCt <= 32767;
    size_t waveLds = 0, groupLds = 0;
    int waveNarrow = 0, groupNarrow = 0;
    if (g->ndim == 2 && G.tz == 1 && G.tx <= 64 && G.ty <= 64 && g->nring <= 256) {
        // 8-bit residuals and t-links with 16-bit excess, else 16-bit residuals, else 32-bit
        const bool narrow8 = g->maxPair <= 255 && g->maxCt <= 255 && g->maxIn <= 32767;
        size_t b8 = mfd::discharge_wave_bytes(G.V, G.K, g->nring, 2);
        size_t b16 = mfd::discharge_wave_bytes(G.V, G.K, g->nring, 1);
        size_t b32 = mfd::discharge_wave_bytes(G.V, G.K, g->nring, 0);
        if (narrow8 && b8 <= ldsBudget) { waveLds = b8; waveNarrow = 2; }
        else if (narrowOk && b16 <= ldsBudget) { waveLds = b16; waveNarrow = 1; }
        else if (b32 <= ldsBudget) { waveLds = b32; }
    }
    if (G.V <= 32767) {
        size_t b16 = mfd::discharge_lds_bytes(G.V, G.K, g->nring, 1);
        size_t b32 = mfd::discharge_lds_bytes(G.V, G.K, g->nring, 0);
        if (narrowOk && b16 <= ldsBudget) { groupLds = b16; groupNarrow = 1; }
        else if (b32 <= ldsBudget) { groupLds = b32; }
    }
    // 3D 6-connected regions with 32-vertex rows: one workgroup, row bitmasks
    // in registers and LDS, integer state in HBM (ROWS)
    size_t rowsLds = 0;
    {
        const int R = G.ty * G.tz;
        if (g->ndim == 3 && G.K == 6 && G.tx == 32 && G.ty >= 2 && G.tz >= 2 && R % 64 == 0 &&
            R <= 1024 && mfd::rows_slots(g->nring) > 0 && mfd::discharge_rows_bytes(G.ty, G.tz, g->nring) <= ldsBudget) {
            rowsLds = mfd::discharge_rows_bytes(G.ty, G.tz, g->nring);
        }
    }
    // 3D 6-connected regions with 64-vertex rows (64^3): one workgroup, rows in
    // registers, masks and admissible arcs in per-workgroup scratch (ROWS64)
    size_t rows64Lds = 0;
    if (g->ndim == 3 && mfd::rows64_applicable(G.K, G.tx, G.ty, G.tz) &&
        mfd::discharge_rows64_bytes(G.ty, G.tz) <= ldsBudget &&
        mfd::rows64_scratch_bytes(G.ty, G.tz, g->nring) <= (size_t)16 * G.V)
        rows64Lds = mfd::discharge_rows64_bytes(G.ty, G.tz);
    int regionMode = 0;  // 0: HBM, 1: LDS workgroup, 2: wavefront, 3: row-bitmask workgroup, 4: 64-bit rows
    switch (region_kernel) {
        case MF_KERNEL_AUTO:
            regionMode = prd ? 0 : (waveLds ? 2 : (rowsLds ? 3 : (rows64Lds ? 4 : (groupLds ? 1 : 0))));
            break;
        case MF_KERNEL_HBM: regionMode = 0; break;
        case MF_KERNEL_LDS: if (!groupLds) return MF_E_INVAL; regionMode = 1; break;
        case MF_KERNEL_WAVE: if (!waveLds) return MF_E_INVAL; regionMode = 2; break;
        case MF_KERNEL_ROWS: if (!rowsLds) return MF_E_INVAL; regionMode = 3; break;
        case MF_KERNEL_ROWS64: if (!rows64Lds) return MF_E_INVAL; regionMode = 4; break;
        default: return MF_E_INVAL;
    }
    const size_t regionLds = regionMode == 4 ? rows64Lds
                             : (regionMode == 3 ? rowsLds : (regionMode == 2 ? waveLds : groupLds));
    const int regionNarrow = regionMode == 2 ? waveNarrow : groupNarrow;
    int regionBlocks = g->nslots;
    if (regionMode == 4) {
        // one workgroup per compute unit, each with its own scratch slot
        regionBlocks = std::max(1, std::min(std::min(G.nreg, g->numCU), g->nslots));
    } else if (regionMode == 3) {
        // at most two 1024-thread workgroups fit the wave slots of a compute unit
        int occ = (int)std::max<size_t>(1, std::min<size_t>(2, g->ldsMax / (regionLds + 256)));
        regionBlocks = std::max(1, std::min(G.nreg, g->numCU * occ));
    } else if (regionMode) {
        int occ = (int)std::max<size_t>(1, std::min<size_t>(8, g->ldsMax / (regionLds + 256)));
        regionBlocks = std::max(1, std::min(G.nreg, g->numCU * occ));
    }
    P.mode = regionMode;
    P.lds = regionLds;
    P.narrow = regionNarrow;
    P.blocks = regionBlocks;
    return MF_OK;
}

// One discharge launch of the picked region kernel (lds: the HBM kernel's search arrays).
static hipError_t launch_region(const mf_grid *g, const RegionPick &P, const mfd::DischargeArgs &D,
                                size_t lds, hipStream_t s) {
    if (P.mode == 4) return mfd::launch_discharge_rows64(D, P.blocks, P.lds, s);
    if (P.mode == 3) return mfd::launch_discharge_rows(D, P.blocks, P.lds, s);
    if (P.mode == 2) return mfd::launch_discharge_wave(D, P.blocks, P.lds, P.narrow, s);
    if (P.mode == 1) return mfd::launch_discharge_lds(D, P.blocks, P.lds, P.narrow, s);
    return mfd::launch_discharge(D, g->nslots, g->threads, lds, s);
}

extern "C" mf_status mf_solve(mf_grid *g, const mf_solve_opts *opts, mf_solve_stats *st) {
    if (!g) return MF_E_INVAL;
    if (!g->has_caps) return MF_E_STATE;
    mf_solve_opts o;
    memset(&o, 0, sizeof(o));
    o.gap = 1;
    if (opts) o = *opts;
    if (o.schedule < 0 || o.schedule > MF_SCHED_LEARNED_COLORED) return MF_E_INVAL;
    if (o.method != MF_METHOD_ARD && o.method != MF_METHOD_PRD) return MF_E_INVAL;
    const bool prd = o.method == MF_METHOD_PRD;
    const bool learned = o.schedule == MF_SCHED_LEARNED || o.schedule == MF_SCHED_LEARNED_COLORED;
    // Alg. 1 as phases of non-interacting regions: one colour class per phase,
    // each phase's flow applied before the next (the boundary relabel is built
    // for Alg. 2)
    const bool colored = o.schedule == MF_SCHED_COLORED || o.schedule == MF_SCHED_LEARNED_COLORED;
    if (colored && (o.boundary_relabel || (o.features && o.features_cap > 0))) return MF_E_INVAL;
    // push-relabel region discharge: distance labels over every arc; the
    // heuristics and the exact relabel here are those of region distances
    if (o.round_cap < 0) return MF_E_INVAL;
    if (prd && (learned || o.partial || o.boundary_relabel || o.round_cap ||
                o.global_relabel_every || (o.features && o.features_cap > 0) ||
                (o.region_kernel != MF_KERNEL_AUTO && o.region_kernel != MF_KERNEL_HBM)))
        return MF_E_INVAL;
    mf_model *model = (mf_model *)o.model;
    // the scheduler's queue kernel keeps one class byte per region in LDS
    if (learned && (!model || g->G.nreg > 65536)) return MF_E_INVAL;
    const bool feats = learned || (o.features && o.features_cap > 0);
    if (feats) {
        const size_t R = (size_t)g->G.nreg;
        if (!g->feat && !(ok(dalloc(&g->feat, R * mfd::kFeat)) && ok(dalloc(&g->score, R)) &&
                          ok(dalloc(&g->defer, R)) && ok(dalloc(&g->deferCount, R)) &&
                          ok(dalloc(&g->lorder, R)) && ok(dalloc(&g->rticks, R))))
            return MF_E_NOMEM;
        if (learned && !model_ws(model, g->G.nreg)) return MF_E_NOMEM;
    }
    if (learned) o.graph = 0;
    if (feats) o.graph = 0;
    int check_every = o.check_every > 0 ? o.check_every : 8;
    if (o.global_relabel_every < 0) return MF_E_INVAL;
    if (o.partial != 0 && o.partial != 1) return MF_E_INVAL;
    // the level budget is also the number of level launches per sweep
    if (o.boundary_relabel < 0 || o.boundary_relabel > 4096) return MF_E_INVAL;
    const int brl = o.boundary_relabel;
    if (o.global_relabel_every > 0) check_every = o.global_relabel_every;
    // colour classes: regions that share no arc.  Checkerboard for 4- and
    // 6-connected grids; 2D 8-connected grids need four (diagonal neighbours)
    const int ncol = colored ? ((g->ndim == 2 && g->G.K == 8) ? 4 : 2) : 1;
    if (colored && g->corder_ncol != ncol) {
        const Geo &Gc = g->G;
        std::vector<int> ord;
        std::vector<int> cs(ncol + 1, 0);
        for (int c = 0; c < ncol; c++) {
            cs[c] = (int)ord.size();
            for (int r = 0; r < Gc.nreg; r++) {
                const int rx = r % Gc.rx, t = r / Gc.rx, ry = t % Gc.ry, rz = t / Gc.ry;
                const int cr = ncol == 4 ? ((rx & 1) | ((ry & 1) << 1)) : ((rx + ry + rz) & 1);
                if (cr == c) ord.push_back(r);
            }
        }
        cs[ncol] = (int)ord.size();
        if (!g->corder && !ok(dalloc(&g->corder, (size_t)Gc.nreg))) return MF_E_NOMEM;
        if (!ok(hipMemcpy(g->corder, ord.data(), sizeof(int) * ord.size(), hipMemcpyHostToDevice)))
            return MF_E_DEVICE;
        g->cstart = cs;
        g->corder_host = ord;
        g->corder_ncol = ncol;
    }
    if (colored && learned) {
        // phase lists of the learned colour phases: every colour padded to the longest
        int maxc = 0;
        for (int c = 0; c < ncol; c++) maxc = std::max(maxc, g->cstart[c + 1] - g->cstart[c]);
        if (!g->plists && !ok(dalloc(&g->plists, (size_t)mfd::kMaxColours * g->G.nreg))) return MF_E_NOMEM;
        g->phase_maxc = maxc;
    }
    // a check interval counts sweeps; a sweep of the colour schedule is ncol phases
    check_every *= ncol;
    // labels: region distances below dinf = |B| (ARD), or distances below dinf = n (PRD)
    const int dinf = prd ? (int)std::max<long long>(g->n, 1) : g->dinf;
    long long B = prd ? (long long)dinf : (g->nB > 0 ? g->nB : 1);
    long long bound = (B > 2000000000LL) ? (1LL << 62) : 2 * B * B + 1;
    // capped rounds spread one discharge over several sweeps, so the bound of
    // full discharges does not hold: the default guard is then at least 2^20
    if (o.round_cap > 0) bound = std::max(bound, 1LL << 20);
    long long max_sweeps = o.max_sweeps > 0 ? o.max_sweeps : bound;
    // the device counts steps: sweeps (Alg. 2) or colour phases (Alg. 1)
    const long long max_steps = max_sweeps > (1LL << 60) / ncol ? max_sweeps : max_sweeps * ncol;
    hipStream_t s = (hipStream_t)o.stream;
    const bool use_graph = o.graph && !o.profile && !o.trace && !o.label_trace;
    if (o.label_trace_cap < 0) return MF_E_INVAL;
    if (use_graph) {
        // capture needs a stream of our own; it orders with the null stream
        if (!s) {
            if (!g->own_stream && !ok(hipStreamCreate(&g->own_stream))) return MF_E_DEVICE;
            s = g->own_stream;
        }
        check_every += check_every & 1;  // whole even/odd sweep pairs
    }
    g->solved = false;
    g->has_state = false;
    g->state_prd = prd;
    g->cut_kind_cached = -1;
    const Geo &G = g->G;
    auto t0 = std::chrono::high_resolution_clock::now();

    // control block reset + Init
    HIP_TRY(hipMemsetAsync(g->act, 0, 4 * sizeof(u64), s));
    HIP_TRY(hipMemsetAsync(g->qhead, 0, 4 * sizeof(unsigned), s));
    HIP_TRY(hipMemsetAsync(g->hist, 0, sizeof(unsigned) * mfd::kHistBins, s));
    HIP_TRY(hipMemsetAsync(g->maxlab, 0xff, sizeof(int), s));
    HIP_TRY(hipMemsetAsync(g->gap, 0xff, sizeof(int), s));
    HIP_TRY(hipMemsetAsync(g->err, 0, sizeof(int), s));
    HIP_TRY(hipMemsetAsync(g->counters, 0, 4 * sizeof(u64), s));
    HIP_TRY(hipMemsetAsync(g->stats, 0, 16 * sizeof(u64), s));
    HIP_TRY(hipMemsetAsync(g->ractive, 0, sizeof(int) * G.nreg, s));
    if (learned) HIP_TRY(hipMemsetAsync(g->deferCount, 0, sizeof(int) * G.nreg, s));
    if (learned) HIP_TRY(hipMemsetAsync(g->rticks, 0, sizeof(int) * G.nreg, s));
    HIP_TRY(mfd::launch_init(G, g->in_cs, g->in_ct, g->in_nbr, (int)g->n, g->res, g->rt, g->ex,
                             g->lab[0], g->lab[1], g->pushb, g->ractive, g->act, s));

    mfd::DischargeArgs D;
    memset(&D, 0, sizeof(D));
    D.G = G;
    D.res = g->res; D.rt = g->rt; D.ex = g->ex; D.pushb = g->pushb;
    D.ractive = g->ractive; D.order = g->order; D.nwork = G.nreg;
    D.dinf = dinf; D.scratch = g->scratch; D.ringL = g->ringL; D.ringM = g->ringM;
    D.prd = prd ? 1 : 0;
    // partial discharges count sweeps, which are ncol steps in colour phases
    D.capShift = ncol == 4 ? 2 : (ncol == 2 ? 1 : 0);
    D.nring = g->nring; D.stats = g->stats; D.rvcount = g->rvcount; D.err = g->err;
    D.useLDS = g->useLDS ? 1 : 0;
    D.maxIter = 1 << 18;
    D.trace = o.trace;
    D.traceCap = o.trace ? o.trace_cap : 0;
    D.partial = o.partial;
    D.sweepCount = g->counters;
    D.actCarry = (o.partial || o.round_cap > 0) ? g->counters + 1 : nullptr;
    D.roundCap = o.round_cap;
    size_t lds = g->useLDS ? (size_t)16 * G.V : 0;
    RegionPick RP;
    {
        const mf_status ps = pick_region(g, o.region_kernel, prd, RP);
        if (ps != MF_OK) return ps;
    }
    const int regionMode = RP.mode;
    const int regionNarrow = RP.narrow;
    mfd::FuseArgs F;
    memset(&F, 0, sizeof(F));
    F.G = G; F.bidx = g->bidx; F.nB = (int)g->nB; F.res = g->res; F.ex = g->ex; F.pushb = g->pushb;
    F.dinf = dinf; F.hist = g->hist; F.maxlab = g->maxlab;
    // with the boundary relabel the histogram is built from its lifted labels;
    // with push-relabel region discharge over all labels
    F.histOn = (brl > 0 || prd) ? 0 : 1;
    // boundary relabel after the fusion; its distances use the cut marks' buffer
    // (free during a solve)
    mfd::BrlArgs BA;
    memset(&BA, 0, sizeof(BA));
    BA.G = G; BA.bidx = g->bidx; BA.bstart = g->bstart; BA.nB = (int)g->nB; BA.res = g->res;
    BA.dist = g->mark; BA.ctl = g->brlctl; BA.dinf = g->dinf; BA.levels = brl;
    BA.hist = g->hist; BA.maxlab = g->maxlab;

    mfd::GapArgs P;
    P.hist = g->hist; P.maxlab = g->maxlab; P.gap = g->gap; P.gapOn = o.gap ? 1 : 0;
    P.counters = g->counters;
    P.actCarry = D.actCarry;

    mfd::GapApplyArgs Q;
    memset(&Q, 0, sizeof(Q));
    Q.G = G; Q.bidx = g->bidx; Q.nB = (int)g->nB; Q.ex = g->ex; Q.ractive = g->ractive;
    Q.gap = g->gap; Q.dinf = dinf;

    std::vector<hipEvent_t> ev;
    if (o.profile) {
        ev.resize(2 * check_every);
        for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
    }
    double discharge_ms = 0.0;
    long long timed = 0;
    long long sweep = 0;
    long long relabels = 0, relabel_levels = 0;
    long long stepsDone = 0;  // device step counter at the last check
    mf_status status = MF_OK;
    for (;;) {
        if (o.global_relabel_every > 0) {
            const int p = (int)(sweep & 1);
            int lv = global_relabel(g, g->lab[colored ? 0 : p], g->act + p, s);
            if (lv < 0) return MF_E_DEVICE;
            relabels++;
            relabel_levels += lv;
        }
        // one batch of check_every sweeps; sweep parity selects the buffers
        // colour phase order of the current sweep (colour mode): fixed, or by
        // the learned scores when the learned schedule drives the phases (then
        // the phase lists are built on the device)
        std::vector<int> cperm(ncol);
        for (int c = 0; c < ncol; c++) cperm[c] = c;
        auto enqueue_batch = [&](long long first, int count) -> bool {
            for (int j = 0; j < count; j++) {
                const int phase = (int)((first + j) % ncol);
                // features and scores once per sweep: every step of Alg. 2, the
                // first phase of a sweep in colour mode
                const bool sweepStart = phase == 0;
                const int p = (int)((first + j) & 1);
                // one label buffer in colour phases: a phase writes its own
                // regions and reads the labels of other colours
                int *labIn = g->lab[colored ? 0 : p], *labOut = g->lab[colored ? 0 : p ^ 1];
                D.labOld = labIn; D.labNew = labOut;
                D.actIn = g->act + p; D.qhead = g->qhead + p;
                D.sweep = (int)((first + j) / ncol);  // trace records: the sweep, also in colour phases
                if (feats && sweepStart) {
                    // region features at the start of the sweep; the learned
                    // schedule scores them (BF16) and builds the queue
                    mfd::FeatArgs FA;
                    FA.G = G; FA.ex = g->ex; FA.lab = g->lab[p]; FA.res = g->res;
                    FA.lab2 = colored ? nullptr : g->lab[p ^ 1];
                    FA.ringL = g->ringL; FA.ringM = g->ringM; FA.nring = g->nring; FA.dinf = g->dinf;
                    // with partial discharges excess can stay inside a region, and
                    // so it can during the first sweep of colour phases
                    FA.ringOnly = (first + j >= ncol && !o.partial && o.round_cap <= 0) ? 1 : 0;
                    FA.ringX = g->ringX;
                    FA.out = (o.features && first + j < o.features_cap)
                                 ? o.features + (size_t)(first + j) * G.nreg * mfd::kFeat
                                 : g->feat;
                    if (!ok(mfd::launch_region_features(FA, s))) return false;
                    if (learned) {
                        if (!ok(model_forward(model, FA.out, mfd::kFeat, G.rz, G.ry, G.rx, g->score, 1, s)))
                            return false;
                        mfd::SchedArgs SA;
                        SA.nreg = G.nreg; SA.feat = FA.out; SA.score = g->score;
                        // no deferral in the first sweep: every initially active
                        // region is discharged once, so afterwards only boundary
                        // vertices can be active and the active count sees them all
                        SA.threshold = (first + j < ncol) ? -1.f : (o.defer_threshold > 0.f ? o.defer_threshold : 0.5f);
                        SA.maxDefer = o.max_defer > 0 ? o.max_defer : 2;
                        SA.defer = g->defer; SA.deferCount = g->deferCount; SA.order = g->lorder;
                        SA.regionTicks = g->rticks;
                        D.regionTicks = g->rticks;
                        D.deferRelabel = o.defer_mode == 1 ? 1 : 0;
                        if (!ok(mfd::launch_sched_queue(SA, s))) return false;
                        D.defer = g->defer;
                        if (!colored) {
                            D.order = g->lorder;
                        } else {
                            // Alg. 1 lets the order matter: the colours run in
                            // descending predicted progress of their active regions,
                            // ordered on the device (no host round trip per sweep)
                            mfd::PhaseArgs PA;
                            memset(&PA, 0, sizeof(PA));
                            PA.ncol = ncol;
                            for (int c = 0; c <= ncol; c++) PA.cstart[c] = g->cstart[c];
                            PA.maxC = g->phase_maxc;
                            PA.corder = g->corder;
                            PA.ractive = g->ractive;
                            PA.score = g->score;
                            PA.out = g->plists;
                            if (!ok(mfd::launch_phase_lists(PA, s))) return false;
                        }
                    }
                }
                if (colored && learned) {
                    D.order = g->plists + (size_t)phase * g->phase_maxc;
                    D.nwork = g->phase_maxc;
                } else if (colored) {
                    const int c = cperm[phase];
                    D.order = g->corder + g->cstart[c];
                    D.nwork = g->cstart[c + 1] - g->cstart[c];
                }
                if (o.profile && !ok(hipEventRecord(ev[2 * j], s))) return false;
                const hipError_t e = launch_region(g, RP, D, lds, s);
                if (!ok(e)) return false;
                if (o.profile && !ok(hipEventRecord(ev[2 * j + 1], s))) return false;
                F.lab = labOut; F.actIn = g->act + p;
                if (!ok(mfd::launch_fuse(F, s))) return false;
                if (prd && !ok(mfd::launch_label_hist(labOut, G.N, dinf, g->hist, g->maxlab,
                                                      g->act + p, s)))
                    return false;
                if (brl > 0) {
                    BA.lab = labOut; BA.actIn = g->act + p;
                    if (!ok(mfd::launch_boundary_relabel(BA, 0, 0, 0, s)) ||
                        !ok(mfd::launch_boundary_relabel(BA, 1, 0, brl, s)) ||
                        !ok(mfd::launch_boundary_relabel(BA, 2, 0, 0, s)))
                        return false;
                }
                P.actIn = g->act + p; P.actOut = g->act + (p ^ 1); P.qheadNext = g->qhead + (p ^ 1);
                if (!ok(mfd::launch_gap_find(P, s))) return false;
                if (prd && !ok(mfd::launch_gap_raise_all(labOut, G.N, g->gap, dinf, g->act + p, s)))
                    return false;
                Q.lab = labOut; Q.actIn = g->act + p; Q.actOut = g->act + (p ^ 1);
                if (!ok(mfd::launch_gap_apply(Q, s))) return false;
                // regions of colours not yet discharged may still hold excess
                // inside (from Init): count every active vertex, not only B
                if (colored && !ok(mfd::launch_activity(G, g->ex, labOut, dinf, g->ractive,
                                                        g->act + (p ^ 1), s)))
                    return false;
                // the labels after this step, row-major
                if (o.label_trace && first + j < o.label_trace_cap &&
                    !ok(mfd::launch_trace_labels(G, g->lab[0], g->lab[colored ? 0 : 1], g->counters,
                                                 o.label_trace + (size_t)(first + j) * g->n, (int)g->n, s)))
                    return false;
            }
            return true;
        };
        // never enqueue more steps than max_steps allows: each step raises the
        // device counter at most once, so a solve stops at max_steps exactly
        const long long room = max_steps - stepsDone;
        const int count = (int)std::min<long long>(check_every, std::max<long long>(room, 1));
        if (use_graph && count == check_every) {
            // a captured batch replays on any even first sweep: the buffers it
            // uses depend only on parity (labels may be swapped by relabels, so
            // the graph is rebuilt when their order changed)
            const long long key = ((long long)check_every << 8) | (o.gap ? 1 : 0) << 1 |
                                  (long long)(regionMode << 2) | (long long)(regionNarrow << 4) |
                                  (long long)((g->lab[0] < g->lab[1]) ? 1 : 0) << 6 |
                                  (long long)(o.partial ? 1 : 0) << 7 | (long long)brl << 40 |
                                  (long long)std::min(o.round_cap, 0xffff) << 24 |
                                  (long long)(prd ? 1 : 0) << 56 | (long long)(colored ? 1 : 0) << 57;
            if (!g->graph_exec || g->graph_key != key) {
                if (g->graph_exec) { (void)hipGraphExecDestroy(g->graph_exec); g->graph_exec = nullptr; }
                hipGraph_t graph = nullptr;
                HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
                const bool enq = enqueue_batch(0, check_every);
                hipError_t ec = hipStreamEndCapture(s, &graph);
                if (!enq || !ok(ec)) return MF_E_DEVICE;
                hipError_t ei = hipGraphInstantiate(&g->graph_exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (!ok(ei)) return MF_E_DEVICE;
                g->graph_key = key;
            }
            HIP_TRY(hipGraphLaunch(g->graph_exec, s));
            sweep += check_every;
        } else {
            if (!enqueue_batch(sweep, count)) return MF_E_DEVICE;
            sweep += count;
        }
        const int p = (int)(sweep & 1);
        HIP_TRY(hipMemcpyAsync(g->pinned, g->act + p, sizeof(u64), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(g->pinned + 1, g->counters, sizeof(u64), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(g->pinned + 2, g->err, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (o.profile) {
            // every discharge launch is timed, including those of the sweeps
            // enqueued after convergence (they exit at once)
            for (int j = 0; j < count; j++) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, ev[2 * j], ev[2 * j + 1]));
                discharge_ms += ms;
                timed++;
            }
        }
        stepsDone = (long long)g->pinned[1];
        if (*(int *)(g->pinned + 2) & 4) { status = MF_E_DEVICE; break; }
        if (g->pinned[0] == 0ull) break;
        if ((long long)g->pinned[1] >= max_steps) { status = MF_E_SWEEPS; break; }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    // the statistics of the sweeps run (also when the sweep limit ends the solve)
    auto fill_stats = [&](long long sweeps) {
        if (!st) return;
        auto t1 = std::chrono::high_resolution_clock::now();
        memset(st, 0, sizeof(*st));
        st->sweeps = sweeps;
        st->region_discharges = (int64_t)g->pinned[16];
        st->discharged_vertices = (int64_t)g->pinned[17];
        st->discharge_iterations = (int64_t)g->pinned[18];
        st->search_levels = (int64_t)g->pinned[19];
        st->search_stages = (int64_t)g->pinned[20];
        st->trace_records = (int64_t)g->pinned[21];
        st->search_ticks = (int64_t)g->pinned[22];
        st->push_ticks = (int64_t)g->pinned[23];
        st->setup_ticks = (int64_t)g->pinned[24];
        st->flood_ticks = (int64_t)g->pinned[25];
        st->push_iterations = (int64_t)g->pinned[26];
        st->relabel_only = (int64_t)g->pinned[27];
        st->region_kernel = regionMode == 4 ? MF_KERNEL_ROWS64 : regionMode == 3 ? MF_KERNEL_ROWS
                            : (regionMode == 2 ? MF_KERNEL_WAVE : (regionMode == 1 ? MF_KERNEL_LDS : MF_KERNEL_HBM));
        st->global_relabels = relabels;
        st->global_relabel_levels = relabel_levels;
        st->boundary_size = g->nB;
        st->d_inf = dinf;
        st->solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        st->discharge_ms = discharge_ms;
        st->discharge_launches = timed;
        st->discharge_bytes = (double)st->discharged_vertices * (double)mf_discharge_bytes_per_vertex(g->K);
    };
    if (status == MF_E_SWEEPS) {
        // the state after the sweeps run so far stays readable
        g->final_parity = colored ? 0 : (int)(g->pinned[1] & 1ull);
        g->has_state = true;
        // skipped regions refreshed only their border labels: the current labels
        // are the larger entry of the two buffers
        if (!colored) HIP_TRY(mfd::launch_label_max(g->lab[g->final_parity], g->lab[g->final_parity ^ 1], G.N, s));
        HIP_TRY(hipMemcpyAsync(g->pinned + 16, g->stats, 16 * sizeof(u64), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        fill_stats(((long long)g->pinned[1] + ncol - 1) / ncol);
    }
    if (status != MF_OK) return status;
    const long long steps = (long long)g->pinned[1];
    g->final_parity = colored ? 0 : (int)(steps & 1);
    if (!colored) HIP_TRY(mfd::launch_label_max(g->lab[g->final_parity], g->lab[g->final_parity ^ 1], G.N, s));
    const long long sweeps = (steps + ncol - 1) / ncol;
    // flow value |f| = sum (c_t - c_f(., t))
    HIP_TRY(hipMemsetAsync(g->sums + 2, 0, sizeof(u64), s));
    HIP_TRY(mfd::launch_sum_i32(g->rt, G.N, g->sums + 2, s));
    HIP_TRY(hipMemcpyAsync(g->pinned + 3, g->sums + 2, sizeof(u64), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(g->pinned + 16, g->stats, 16 * sizeof(u64), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    g->flow = g->sum_ct - (long long)g->pinned[3];
    if (g->batch) {
        HIP_TRY(hipMemsetAsync(g->instRt, 0, sizeof(u64) * g->batch, s));
        HIP_TRY(mfd::launch_instance_rt(G, g->rt, g->reginst, g->instRt, s));
        std::vector<u64> rts(g->batch);
        HIP_TRY(hipMemcpyAsync(rts.data(), g->instRt, sizeof(u64) * g->batch, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int i = 0; i < g->batch; i++) g->iflow[i] = g->isum_ct[i] - (long long)rts[i];
    }
    g->solved = true;
    g->has_state = true;
    fill_stats(sweeps);
    return MF_OK;
}

extern "C" mf_status mf_flow_value(const mf_grid *g, int64_t *out) {
    if (!g || !out) return MF_E_INVAL;
    if (!g->solved) return MF_E_STATE;
    *out = g->flow;
    return MF_OK;
}

// Residual reachability marks for a cut kind into g->mark (cached until the
// next solve): forward from the excess vertices, or backward from t.
static mf_status compute_marks(mf_grid *g, int32_t kind) {
    if (g->cut_kind_cached == kind) return MF_OK;
    const Geo &G = g->G;
    hipStream_t s = nullptr;
    g->cut_kind_cached = -1;
    HIP_TRY(hipMemsetAsync(g->mark, 0, sizeof(int) * (size_t)G.N, s));
    HIP_TRY(hipMemsetAsync(g->dirty, 0, sizeof(int) * 2 * (size_t)G.nreg, s));
    mfd::FloodArgs A;
    memset(&A, 0, sizeof(A));
    A.G = G;
    A.dir = kind == MF_CUT_MIN_SOURCE ? 0 : 1;
    A.mark = g->mark;
    A.res = g->res; A.ex = g->ex; A.rt = g->rt;
    A.scratch = g->scratch;
    A.changed = g->changed;
    A.ringL = g->ringL; A.ringM = g->ringM; A.nring = g->nring;
    // 2D tiles of at most 64 x 64: one wavefront per region with row bitmasks
    const bool wave = g->ndim == 2 && G.tz == 1 && G.tx <= 64 && G.ty <= 64 && g->nring <= 256;
    // 3D 6-connected tiles with 32-vertex rows: one workgroup per region, row bitmasks
    const int Rr = G.ty * G.tz;
    const bool rows = g->ndim == 3 && G.K == 6 && G.tx == 32 && G.ty >= 2 && G.tz >= 2 &&
                      Rr % 64 == 0 && Rr <= 1024;
    // 3D 64^3 tiles: one workgroup per region, 64-bit rows in registers
    const bool rows64 = g->ndim == 3 && mfd::rows64_applicable(G.K, G.tx, G.ty, G.tz);
    int blocks = wave ? std::min(G.nreg, g->numCU * 16)
                      : ((rows || rows64) ? std::min(G.nreg, g->numCU * 2)
                                          : std::min(G.nreg, g->nslots * 4));  // scratch holds 4V ints per slot
    for (int round = 0;; round++) {
        A.round = round;
        A.dirtyIn = g->dirty + (size_t)(round & 1) * G.nreg;
        A.dirtyOut = g->dirty + (size_t)((round + 1) & 1) * G.nreg;
        HIP_TRY(hipMemsetAsync(g->changed, 0, sizeof(unsigned), s));
        HIP_TRY(wave ? mfd::launch_flood_wave(A, blocks, s)
                     : (rows ? mfd::launch_flood_rows(A, blocks, s)
                             : (rows64 ? mfd::launch_flood_rows64(A, blocks, s) : mfd::launch_flood(A, blocks, s))));
        HIP_TRY(hipMemcpyAsync(g->pinned, g->changed, sizeof(unsigned), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (*(unsigned *)g->pinned == 0u) break;
        if (round > G.N + 8) return MF_E_DEVICE;
    }
    g->cut_kind_cached = kind;
    return MF_OK;
}

extern "C" mf_status mf_min_cut(const mf_grid *gc, int32_t kind, uint8_t *out_source_side) {
    mf_grid *g = const_cast<mf_grid *>(gc);
    if (!g || !out_source_side) return MF_E_INVAL;
    if (kind != MF_CUT_MIN_SOURCE && kind != MF_CUT_MAX_SOURCE) return MF_E_INVAL;
    if (!g->solved) return MF_E_STATE;
    mf_status st = compute_marks(g, kind);
    if (st != MF_OK) return st;
    const Geo &G = g->G;
    hipStream_t s = nullptr;
    HIP_TRY(mfd::launch_cut_out(G, g->mark, g->cutbuf, (int)g->n, kind == MF_CUT_MAX_SOURCE ? 1 : 0, s));
    HIP_TRY(hipMemcpyAsync(out_source_side, g->cutbuf, (size_t)g->n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MF_OK;
}

// ---------------------------------------------------------------------------
// Batches of independent 2D instances
// ---------------------------------------------------------------------------
extern "C" mf_status mf_create_batch(int32_t count, const int64_t *dims, const int32_t *connectivity,
                                     const int32_t *region_shape, mf_grid **out) {
    if (!out || !dims || !connectivity || count < 1) return MF_E_INVAL;
    int th = 32, tw = 32;
    if (region_shape && (region_shape[0] || region_shape[1])) {
        if (region_shape[0] < 1 || region_shape[1] < 1) return MF_E_INVAL;
        th = region_shape[0];
        tw = region_shape[1];
    }
    int K = 4;
    long long area = 0, maxw = 0, maxn = 0;
    std::vector<long long> H(count), W(count);
    for (int i = 0; i < count; i++) {
        const long long h = dims[2 * i], w = dims[2 * i + 1];
        if (h < 1 || w < 1 || h * w >= (1LL << 30)) return MF_E_INVAL;
        if (connectivity[i] != 4 && connectivity[i] != 8) return MF_E_INVAL;
        if (connectivity[i] == 8) K = 8;
        H[i] = (h + th - 1) / th * th;
        W[i] = (w + tw - 1) / tw * tw;
        area += H[i] * W[i];
        maxw = std::max(maxw, W[i]);
        maxn = std::max(maxn, h * w);
    }
    // shelf packing, tallest first, on a canvas about as wide as it is high
    long long Wc = (long long)std::ceil(std::sqrt((double)area) / tw) * tw;
    Wc = std::max(Wc, maxw);
    std::vector<int> order(count);
    for (int i = 0; i < count; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return H[a] > H[b]; });
    std::vector<int> y0(count), x0(count);
    long long shelfY = 0, shelfH = 0, curX = 0;
    for (int i : order) {
        if (curX + W[i] > Wc) {
            shelfY += shelfH;
            shelfH = 0;
            curX = 0;
        }
        y0[i] = (int)shelfY;
        x0[i] = (int)curX;
        curX += W[i];
        shelfH = std::max(shelfH, H[i]);
    }
    const long long Hc = shelfY + shelfH;
    if (Hc * Wc >= (1LL << 31)) return MF_E_INVAL;
    const int64_t cdims[2] = {Hc, Wc};
    const int32_t tile[2] = {th, tw};
    mf_grid *g = nullptr;
    mf_status st = create_impl(2, cdims, K, tile, &g);
    if (st != MF_OK) return st;
    g->batch = count;
    g->iy0 = y0;
    g->ix0 = x0;
    g->ih.resize(count);
    g->iw.resize(count);
    g->iconn.resize(count);
    for (int i = 0; i < count; i++) {
        g->ih[i] = (int)dims[2 * i];
        g->iw[i] = (int)dims[2 * i + 1];
        g->iconn[i] = connectivity[i];
    }
    g->isum_cs.assign(count, 0);
    g->isum_ct.assign(count, 0);
    g->iflow.assign(count, 0);
    g->imaxpair.assign(count, 0);
    g->imaxct.assign(count, 0);
    g->imaxin.assign(count, 0);
    g->iloaded.assign(count, 0);
    const Geo &G = g->G;
    std::vector<int> reginst(G.nreg, -1);
    for (int i = 0; i < count; i++)
        for (int ry = y0[i] / th; ry < (y0[i] + g->ih[i] + th - 1) / th; ry++)
            for (int rx = x0[i] / tw; rx < (x0[i] + g->iw[i] + tw - 1) / tw; rx++) reginst[ry * G.rx + rx] = i;
    const size_t n = (size_t)g->n;
    bool good = ok(dalloc(&g->reginst, (size_t)G.nreg)) && ok(dalloc(&g->stage, (size_t)(K + 2) * maxn)) &&
                ok(dalloc(&g->instRt, (size_t)count)) &&
                ok(hipMemcpy(g->reginst, reginst.data(), sizeof(int) * G.nreg, hipMemcpyHostToDevice)) &&
                ok(hipMemset(g->in_cs, 0, n * sizeof(int))) && ok(hipMemset(g->in_ct, 0, n * sizeof(int))) &&
                ok(hipMemset(g->in_nbr, 0, (size_t)K * n * sizeof(int))) && ok(hipDeviceSynchronize());
    if (!good) {
        mf_destroy(g);
        return MF_E_NOMEM;
    }
    *out = g;
    return MF_OK;
}

extern "C" mf_status mf_batch_info(const mf_grid *g, int32_t index, int64_t *canvas_offset2,
                                   int64_t *canvas_dims2) {
    if (!g || !g->batch || index < -1 || index >= g->batch) return MF_E_INVAL;
    if (index < 0) {
        if (canvas_dims2) { canvas_dims2[0] = g->G.dy; canvas_dims2[1] = g->G.dx; }
        if (canvas_offset2) { canvas_offset2[0] = 0; canvas_offset2[1] = 0; }
        return MF_OK;
    }
    if (canvas_offset2) { canvas_offset2[0] = g->iy0[index]; canvas_offset2[1] = g->ix0[index]; }
    if (canvas_dims2) { canvas_dims2[0] = g->ih[index]; canvas_dims2[1] = g->iw[index]; }
    return MF_OK;
}

extern "C" mf_status mf_batch_set_caps(mf_grid *g, int32_t index, const int32_t *src_cap,
                                       const int32_t *sink_cap, const int32_t *nbr_cap,
                                       int32_t on_device, void *stream) {
    if (!g || !g->batch || index < 0 || index >= g->batch || !src_cap || !sink_cap || !nbr_cap)
        return MF_E_INVAL;
    hipStream_t s = (hipStream_t)stream;
    const int h = g->ih[index], w = g->iw[index], Ki = g->iconn[index];
    const size_t n = (size_t)h * w;
    g->solved = false;
    g->cut_kind_cached = -1;
    g->has_caps = false;
    g->iloaded[index] = 0;
    hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    int *cs = g->stage, *ct = g->stage + n, *nb = g->stage + 2 * n;
    HIP_TRY(hipMemcpyAsync(cs, src_cap, n * sizeof(int), kind, s));
    HIP_TRY(hipMemcpyAsync(ct, sink_cap, n * sizeof(int), kind, s));
    HIP_TRY(hipMemcpyAsync(nb, nbr_cap, (size_t)Ki * n * sizeof(int), kind, s));
    Geo I;
    memset(&I, 0, sizeof(I));
    I.K = Ki;
    I.dz = 1; I.dy = h; I.dx = w;
    for (int k = 0; k < Ki; k++) { I.oz[k] = 0; I.oy[k] = OFF2D[k][0]; I.ox[k] = OFF2D[k][1]; }
    HIP_TRY(hipMemsetAsync(g->err, 0, 4 * sizeof(int), s));
    HIP_TRY(hipMemsetAsync(g->sums, 0, 4 * sizeof(u64), s));
    HIP_TRY(mfd::launch_validate(I, cs, ct, nb, (int)n, g->err, s));
    HIP_TRY(mfd::launch_sum_links(cs, ct, (int)n, g->sums, s));
    HIP_TRY(hipMemcpyAsync(g->pinned, g->sums, 2 * sizeof(u64), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(g->pinned + 2, g->err, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int err = ((int *)(g->pinned + 2))[0];
    if (err & 1) return MF_E_INVAL;
    if (err & 2) return MF_E_OVERFLOW;
    g->isum_cs[index] = (long long)g->pinned[0];
    g->isum_ct[index] = (long long)g->pinned[1];
    g->imaxpair[index] = ((int *)(g->pinned + 2))[1];
    g->imaxct[index] = ((int *)(g->pinned + 2))[2];
    g->imaxin[index] = ((int *)(g->pinned + 2))[3];
    HIP_TRY(mfd::launch_scatter_instance(cs, ct, nb, h, w, Ki, g->in_cs, g->in_ct, g->in_nbr, g->G.dx,
                                         g->n, g->iy0[index], g->ix0[index], s));
    HIP_TRY(hipStreamSynchronize(s));
    g->iloaded[index] = 1;
    bool all = true;
    long long scs = 0, sct = 0;
    int mp = 0, mc = 0, mi = 0;
    for (int i = 0; i < g->batch; i++) {
        all = all && g->iloaded[i];
        scs += g->isum_cs[i];
        sct += g->isum_ct[i];
        mp = std::max(mp, g->imaxpair[i]);
        mc = std::max(mc, g->imaxct[i]);
        mi = std::max(mi, g->imaxin[i]);
    }
    g->sum_cs = scs;
    g->sum_ct = sct;
    g->maxPair = mp;
    g->maxCt = mc;
    g->maxIn = mi;
    g->has_caps = all;
    return MF_OK;
}

extern "C" mf_status mf_batch_flow_values(const mf_grid *g, int64_t *out) {
    if (!g || !g->batch || !out) return MF_E_INVAL;
    if (!g->solved) return MF_E_STATE;
    for (int i = 0; i < g->batch; i++) out[i] = g->iflow[i];
    return MF_OK;
}

extern "C" mf_status mf_batch_min_cut(const mf_grid *gc, int32_t index, int32_t kind,
                                      uint8_t *out_source_side) {
    mf_grid *g = const_cast<mf_grid *>(gc);
    if (!g || !g->batch || index < 0 || index >= g->batch || !out_source_side) return MF_E_INVAL;
    if (kind != MF_CUT_MIN_SOURCE && kind != MF_CUT_MAX_SOURCE) return MF_E_INVAL;
    if (!g->solved) return MF_E_STATE;
    mf_status st = compute_marks(g, kind);
    if (st != MF_OK) return st;
    hipStream_t s = nullptr;
    const int h = g->ih[index], w = g->iw[index];
    HIP_TRY(mfd::launch_cut_rect(g->G, g->mark, g->cutbuf, h, w, g->iy0[index], g->ix0[index],
                                 kind == MF_CUT_MAX_SOURCE ? 1 : 0, s));
    HIP_TRY(hipMemcpyAsync(out_source_side, g->cutbuf, (size_t)h * w, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return MF_OK;
}

extern "C" mf_status mf_get_state(const mf_grid *gc, int32_t *res, int32_t *rt, int32_t *ex,
                                  int32_t *labels) {
    mf_grid *g = const_cast<mf_grid *>(gc);
    if (!g) return MF_E_INVAL;
    if (!g->has_state) return MF_E_STATE;
    const Geo &G = g->G;
    size_t n = (size_t)g->n;
    hipStream_t s = nullptr;
    auto one = [&](const int *src, int32_t *dst) -> bool {
        if (!dst) return true;
        if (!ok(mfd::launch_gather_plane(G, src, g->tmp_plane, (int)n, s))) return false;
        if (!ok(hipMemcpyAsync(dst, g->tmp_plane, n * sizeof(int), hipMemcpyDeviceToHost, s))) return false;
        return ok(hipStreamSynchronize(s));
    };
    if (res)
        for (int k = 0; k < g->K; k++)
            if (!one(g->res + (size_t)k * G.N, res + (size_t)k * n)) return MF_E_DEVICE;
    if (!one(g->rt, rt) || !one(g->ex, ex) || !one(g->lab[g->final_parity], labels)) return MF_E_DEVICE;
    return MF_OK;
}

extern "C" mf_status mf_region_relabel(mf_grid *g, int32_t region_kernel, int64_t *regions_out) {
    if (!g) return MF_E_INVAL;
    if (!g->has_state || g->state_prd) return MF_E_STATE;
    RegionPick RP;
    {
        const mf_status ps = pick_region(g, region_kernel, false, RP);
        if (ps != MF_OK) return ps;
    }
    const Geo &G = g->G;
    hipStream_t s = nullptr;
    if (!g->defer && !ok(dalloc(&g->defer, (size_t)G.nreg))) return MF_E_NOMEM;
    // every region is deferred with a relabel-only discharge: one complete
    // search over the current state, labels written, no pushes
    HIP_TRY(mfd::launch_fill_i32(g->defer, G.nreg, 1, s));
    HIP_TRY(mfd::launch_fill_i32(g->ractive, G.nreg, 1, s));
    HIP_TRY(hipMemsetAsync(g->qhead + 2, 0, sizeof(unsigned), s));
    HIP_TRY(mfd::launch_fill_i32((int *)(g->act + 2), 2, 1, s));  // a non-zero count: the launch runs
    HIP_TRY(hipMemsetAsync(g->stats, 0, 16 * sizeof(u64), s));
    HIP_TRY(hipMemsetAsync(g->err, 0, sizeof(int), s));
    mfd::DischargeArgs D;
    memset(&D, 0, sizeof(D));
    D.G = G;
    D.res = g->res; D.rt = g->rt; D.ex = g->ex; D.pushb = g->pushb;
    D.labOld = g->lab[g->final_parity];
    D.labNew = g->lab[g->final_parity ^ 1];
    D.ractive = g->ractive; D.order = g->order; D.nwork = G.nreg; D.qhead = g->qhead + 2;
    D.actIn = g->act + 2; D.dinf = g->dinf; D.scratch = g->scratch;
    D.ringL = g->ringL; D.ringM = g->ringM; D.nring = g->nring;
    D.stats = g->stats; D.rvcount = g->rvcount; D.err = g->err;
    D.useLDS = g->useLDS ? 1 : 0;
    D.maxIter = 1 << 18;
    D.defer = g->defer;
    D.deferRelabel = 1;
    D.sweepCount = g->counters;
    const size_t lds = g->useLDS ? (size_t)16 * G.V : 0;
    HIP_TRY(launch_region(g, RP, D, lds, s));
    const int *lab = g->lab[g->final_parity ^ 1];
    // the regions' activity flags from the new labels
    HIP_TRY(hipMemsetAsync(g->ractive, 0, sizeof(int) * G.nreg, s));
    HIP_TRY(hipMemsetAsync(g->act + 2, 0, sizeof(u64), s));
    HIP_TRY(mfd::launch_activity(G, g->ex, lab, g->dinf, g->ractive, g->act + 2, s));
    u64 st[16];
    int err = 0;
    HIP_TRY(hipMemcpy(st, g->stats, sizeof(st), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&err, g->err, sizeof(int), hipMemcpyDeviceToHost));
    if (err & 4) return MF_E_DEVICE;
    g->final_parity ^= 1;
    if (regions_out) *regions_out = (int64_t)st[11];
    return MF_OK;
}

// One auxiliary problem of region reduction for every region at once: Init,
// optionally every boundary vertex a source without bound (inflow), the halo
// labels set to `halo` (0: every residual boundary arc is a target, so every
// boundary vertex is a sink without bound; dinf: only t is a target), one full
// discharge of every region, then the in-region forward search from the
// remaining excess.  Adds the problem's class bits to g->cand.
static mf_status reduction_pass(mf_grid *g, const RegionPick &RP, bool inflow, int halo) {
    const Geo &G = g->G;
    hipStream_t s = nullptr;
    HIP_TRY(hipMemsetAsync(g->act, 0, 4 * sizeof(u64), s));
    HIP_TRY(hipMemsetAsync(g->qhead, 0, 4 * sizeof(unsigned), s));
    HIP_TRY(hipMemsetAsync(g->counters, 0, 4 * sizeof(u64), s));
    HIP_TRY(hipMemsetAsync(g->stats, 0, 16 * sizeof(u64), s));
    HIP_TRY(mfd::launch_init(G, g->in_cs, g->in_ct, g->in_nbr, (int)g->n, g->res, g->rt, g->ex, g->lab[0],
                             g->lab[1], g->pushb, g->ractive, g->act, s));
    if (inflow) HIP_TRY(mfd::launch_saturate_inflow(G, g->in_nbr, (int)g->n, g->res, g->ex, s));
    HIP_TRY(mfd::launch_fill_i32(g->lab[0], G.N, halo, s));
    HIP_TRY(mfd::launch_fill_i32(g->ractive, G.nreg, 1, s));
    HIP_TRY(mfd::launch_fill_i32((int *)(g->act + 2), 2, 1, s));  // a non-zero count: the launch runs
    mfd::DischargeArgs D;
    memset(&D, 0, sizeof(D));
    D.G = G;
    D.res = g->res; D.rt = g->rt; D.ex = g->ex; D.pushb = g->pushb;
    D.labOld = g->lab[0]; D.labNew = g->lab[1];
    D.ractive = g->ractive; D.order = g->order; D.nwork = G.nreg; D.qhead = g->qhead + 2;
    D.actIn = g->act + 2; D.dinf = g->dinf; D.scratch = g->scratch;
    D.ringL = g->ringL; D.ringM = g->ringM; D.nring = g->nring;
    D.stats = g->stats; D.rvcount = g->rvcount; D.err = g->err;
    D.useLDS = g->useLDS ? 1 : 0;
    D.maxIter = 1 << 18;
    D.sweepCount = g->counters;
    const size_t lds = g->useLDS ? (size_t)16 * G.V : 0;
    HIP_TRY(launch_region(g, RP, D, lds, s));
    // minimal source side of the auxiliary problem: forward from the excess,
    // inside each region (the boundary vertices are terminals there)
    HIP_TRY(hipMemsetAsync(g->mark, 0, sizeof(int) * (size_t)G.N, s));
    mfd::FloodArgs A;
    memset(&A, 0, sizeof(A));
    A.G = G;
    A.dir = 0;
    A.round = 0;
    A.noCross = 1;
    A.mark = g->mark;
    A.res = g->res; A.ex = g->ex; A.rt = g->rt;
    A.scratch = g->scratch;
    A.changed = g->changed;
    A.dirtyIn = g->dirty;
    A.dirtyOut = g->dirty + G.nreg;
    A.ringL = g->ringL; A.ringM = g->ringM; A.nring = g->nring;
    HIP_TRY(mfd::launch_flood(A, std::min(G.nreg, g->nslots * 4), s));  // scratch holds 4V ints per slot
    HIP_TRY(mfd::launch_reduce_classes(G, g->lab[1], g->mark, g->cand, g->dinf, inflow ? 1 : 0, s));
    return MF_OK;
}

extern "C" mf_status mf_region_reduction(mf_grid *g, int32_t region_kernel, uint8_t *out_class) {
    if (!g || !out_class) return MF_E_INVAL;
    if (g->batch) return MF_E_INVAL;
    if (!g->has_caps) return MF_E_STATE;
    RegionPick RP;
    {
        const mf_status ps = pick_region(g, region_kernel, false, RP);
        if (ps != MF_OK) return ps;
    }
    // the passes overwrite the solver state
    g->solved = false;
    g->has_state = false;
    g->cut_kind_cached = -1;
    hipStream_t s = nullptr;
    HIP_TRY(hipMemsetAsync(g->err, 0, sizeof(int), s));
    mf_status st = reduction_pass(g, RP, false, 0);  // every boundary vertex a sink
    if (st != MF_OK) return st;
    st = reduction_pass(g, RP, true, g->dinf);  // every boundary vertex a source
    if (st != MF_OK) return st;
    HIP_TRY(mfd::launch_gather_bytes(g->G, g->cand, g->cutbuf, (int)g->n, s));
    HIP_TRY(hipMemcpyAsync(out_class, g->cutbuf, (size_t)g->n, hipMemcpyDeviceToHost, s));
    int err = 0;
    HIP_TRY(hipMemcpyAsync(&err, g->err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (err & 4) return MF_E_DEVICE;
    return MF_OK;
}

extern "C" mf_status mf_global_relabel(mf_grid *g, int64_t *levels_out) {
    if (!g) return MF_E_INVAL;
    if (!g->has_state || g->state_prd) return MF_E_STATE;
    const int lv = global_relabel(g, g->lab[g->final_parity], g->act + 2, nullptr);
    if (lv < 0) return MF_E_DEVICE;
    HIP_TRY(hipStreamSynchronize(nullptr));
    if (levels_out) *levels_out = lv;
    return MF_OK;
}

extern "C" mf_status mf_boundary_relabel(mf_grid *g, int32_t max_levels, int64_t *levels_out) {
    if (!g || max_levels <= 0) return MF_E_INVAL;
    if (!g->has_state || g->state_prd) return MF_E_STATE;
    hipStream_t s = nullptr;
    mfd::BrlArgs BA;
    memset(&BA, 0, sizeof(BA));
    BA.G = g->G; BA.bidx = g->bidx; BA.bstart = g->bstart; BA.nB = (int)g->nB; BA.res = g->res;
    BA.lab = g->lab[g->final_parity]; BA.dist = g->mark; BA.ctl = g->brlctl; BA.dinf = g->dinf;
    g->cut_kind_cached = -1;  // the distances overwrite the cut marks
    unsigned int ctl[8] = {0};
    if (g->nB > 0) {
        // levels in batches of eight until the search ends or the budget is spent
        HIP_TRY(mfd::launch_boundary_relabel(BA, 0, 0, 0, s));
        int run = 0;
        while (run < max_levels) {
            const int c = std::min(8, max_levels - run);
            HIP_TRY(mfd::launch_boundary_relabel(BA, 1, run, c, s));
            run += c;
            HIP_TRY(hipMemcpyAsync(ctl, g->brlctl, 5 * sizeof(unsigned), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (ctl[3] || ctl[(run + 2) % 3] == 0u) break;
        }
        BA.levels = run;
        HIP_TRY(mfd::launch_boundary_relabel(BA, 2, 0, 0, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (levels_out) *levels_out = (int64_t)ctl[4];
    return MF_OK;
}
