// Workgroup row-bitmask region discharge for 3D 6-connected 64^3 regions:
// Proc. ARD of Sec. 4.2 with the region relabel of Alg. 3, the same method as
// k_discharge_rows on regions eight times larger.
//
// One 512-thread workgroup owns a region.  Lane y of wave w owns the eight rows
// (y, z) with z = 8w .. 8w + 7, each a row of 64 vertices along x, as 64-bit
// masks in registers: residual arc present in each of the six directions,
// visited, frontier and excess.  A search level needs the frontier rows y +- 1
// and z +- 1: y +- 1 come from the neighbouring lanes (DPP wavefront shifts),
// z +- 1 from the same lane's other rows, and only the two outer z planes of a
// wave cross to the neighbouring waves through LDS.  A 64^3 region has too many
// bits for LDS (six residual masks alone are 192 KB), so LDS holds only what
// threads exchange: those z faces (double-buffered by level parity), the rows
// of vertices that received excess or were drained in a push iteration (during
// a search: the visited rows and the stage seeds), the vertices a complete
// search did not reach, and per-wave work lists.  A per-workgroup scratch area
// in HBM (mostly resident in the caches) holds the exact residual-arc and
// t-link masks, kept up to date by the pushes, the halo labels d(w) of the
// border vertices, their stage candidates, and one byte per vertex with its
// admissible arcs of the current search.  The integer state (residuals,
// t-links, excess, boundary pushes) stays in HBM and is read once per
// discharge to build the masks.
//
// * Search: the multi-level breadth-first search from the targets (stage 0
//   from t, then one stage per distinct d(w) + 1 over residual boundary arcs)
//   advances one level per workgroup barrier: a level is a few shifts and ANDs
//   of a row with its four neighbouring frontier rows.  A newly reached vertex
//   stores the arcs by which it was reached (they point exactly one level down)
//   as its admissible-arc byte; a first-level vertex of a stage k > 0 stores its
//   boundary arcs to w with d(w) + 1 = k; a vertex with a residual t-link is a
//   stage-0 seed whose only admissible arc is t.
// * Push: every excess vertex pushes along its admissible arcs, into t, to an
//   in-region neighbour, or over a boundary arc (recorded for the fusion).  All
//   excess vertices push in parallel, spread over the lanes of each wave by a
//   work list, one iteration per two barriers, until no push is possible.  Arcs
//   only go down the (stage, level) order, so an arc is changed by one side only.
// * Search and push alternate until no excess vertex reaches a target.  The
//   last search is run once more to write the labels (Alg. 3).
#include "mf_device.h"
#include "mf_launch.h"

namespace mfd {

typedef unsigned long long u64;

namespace {

constexpr int kNT = 512;                // threads per workgroup
constexpr int kW = kNT / 64;            // waves
constexpr int kRPT = 8;                 // rows per thread
constexpr int kMaxRows = kNT * kRPT;    // 4096
constexpr int kListAll = 2048;          // work-list entries per pass (whole workgroup)
constexpr int kInFlight = 4;            // push vertices per lane with loads issued together
constexpr int kRingBatch = 8;           // border vertices per thread with loads issued together

// Per-workgroup scratch in HBM (byte offsets).
struct R64Scratch {
    size_t resG, rtG, halo, slot, adm, total;
};

__host__ __device__ inline R64Scratch r64_scratch(int R, int nring) {
    R64Scratch S;
    size_t o = 0;
    S.resG = o; o += (size_t)6 * R * 8;                  // residual arc (u, u + o_k) > 0, per direction
    S.rtG = o; o += (size_t)R * 8;                       // residual t-link > 0
    S.halo = o; o += ((size_t)nring * 3 * 4 + 15) & ~(size_t)15;  // d(w) per border vertex and axis
    S.slot = o; o += ((size_t)nring * 4 + 15) & ~(size_t)15;      // stage candidate per border vertex
    S.adm = o; o += (size_t)6 * R * 8;                  // admissible arc (u, u + o_k) of the search, per direction
    S.total = o;
    return S;
}

__device__ __forceinline__ int r64_wave_min(int v) {
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

// Workgroup-wide OR / MIN with one barrier; the two halves of the buffers
// alternate between calls (a slower wave may still read the previous one).
static_assert(kW == 8, "one byte per wave in an 8-byte word");
__device__ __forceinline__ int r64_block_any(int pred, unsigned char (*anyB)[kW], int &rc) {
    const u64 b = __ballot(pred);
    const int p = rc & 1;
    rc++;
    if ((threadIdx.x & 63) == 0) anyB[p][threadIdx.x >> 6] = (b != 0ull) ? 1 : 0;
    __syncthreads();
    const uint2 v = *(const uint2 *)anyB[p];
    return (v.x | v.y) != 0u;
}

__device__ __forceinline__ int r64_block_min(int v, int (*red)[kW], int &rc) {
    v = r64_wave_min(v);
    const int p = rc & 1;
    rc++;
    if ((threadIdx.x & 63) == 0) red[p][threadIdx.x >> 6] = v;
    __syncthreads();
    int m = kInf;
#pragma unroll
    for (int w = 0; w < kW; w++) m = min(m, red[p][w]);
    return m;
}

// Workgroup barrier that orders LDS only: the global stores and atomics issued
// before it (admissible arcs, labels) need not have completed, since nothing
// reads them before a full barrier.
__device__ __forceinline__ void r64_lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ int r64_incl_scan(int v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Global-memory pointers: the scratch and label accesses stay global (not flat)
// instructions, so that the waits for LDS results never wait on them.
#define GA __attribute__((address_space(1)))

// A uniform global pointer the compiler must treat as redefined here: keeps it
// from hoisting per-row addresses out of the loops (they would stay live in
// registers across the whole discharge).
template <typename T>
__device__ __forceinline__ GA T *r64_opaque(T *p) {
    GA T *q = (GA T *)p;
    asm volatile("" : "+s"(q));
    return q;
}
template <typename T>
__device__ __forceinline__ GA T *r64_opaque(GA T *p) {
    asm volatile("" : "+s"(p));
    return p;
}

// A pointer the compiler knows to be uniform (scalar registers): a global
// access through it plus a 32-bit per-lane byte offset takes the scalar-base
// form, with no 64-bit address arithmetic in the vector ALU.
template <typename T>
__device__ __forceinline__ GA T *r64_uniform(GA T *p) {
    const u64 v = (u64)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return (GA T *)(((u64)hi << 32) | lo);
}

// Non-returning relaxed atomics on global words.
__device__ __forceinline__ void g_or(GA u64 *p, u64 v) {
    __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_and(GA u64 *p, u64 v) {
    __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Labels val for the set bits of one row per lane (slot rows rowBase + lane),
// stored by the whole wavefront one row at a time: lane x writes vertex x, so
// every row is one coalesced store however many of its bits are set.  Called
// with all lanes active; lab is the region's first label.
__device__ __forceinline__ void r64_store_labels(int *lab, int rowBase, u64 bits, int val, int lane) {
    GA int *b = r64_opaque(lab);
    u64 pend = __ballot(bits != 0ull);
    while (pend) {
        const int l = __builtin_ctzll(pend);
        pend &= pend - 1;
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)bits, l);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(bits >> 32), l);
        const u64 m = ((u64)hi << 32) | (u64)lo;
        if ((m >> lane) & 1ull) b[(size_t)(rowBase + l) * 64 + lane] = val;
    }
}

// Leaving direction of axis a at a border vertex with leaving mask mm (exactly
// one of the two directions of an axis leaves it: the tile is 64 wide on x and
// at least 2 wide on y and z).
__device__ __forceinline__ int r64_axis_dir(unsigned mm, int a) {
    return ((mm >> (2 * a)) & 1u) ? 2 * a : 2 * a + 1;
}

}  // namespace

// LDS: the frontier z faces of every wave by level parity, then the recv,
// clr and dead rows, then the work lists.
constexpr int kFaceWords = 2 * 2 * kW * 64;

size_t discharge_rows64_bytes(int ty, int tz) {
    return ((size_t)kFaceWords + (size_t)4 * ty * tz) * 8 + (size_t)kListAll * 4;
}

size_t rows64_scratch_bytes(int ty, int tz, int nring) { return r64_scratch(ty * tz, nring).total; }

bool rows64_applicable(int K, int tx, int ty, int tz) {
    return K == 6 && tx == 64 && ty == 64 && tz == 64;
}

// Frontier row of the neighbouring lane: lane i gets lane i + 1 (wavefront
// shift left; 0 for the last lane) or lane i - 1 (shift right; 0 for lane 0).
__device__ __forceinline__ u64 r64_from_next_lane(u64 v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), 0x130, 0xf, 0xf, true);
    return ((u64)(unsigned)hi << 32) | (u64)(unsigned)lo;
}
__device__ __forceinline__ u64 r64_from_prev_lane(u64 v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)v, 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(v >> 32), 0x138, 0xf, 0xf, true);
    return ((u64)(unsigned)hi << 32) | (u64)(unsigned)lo;
}

__global__ __launch_bounds__(kNT) void k_discharge_rows64(DischargeArgs A) {
    extern __shared__ __align__(16) u64 smem64[];
    __shared__ __align__(16) int red[2][kW];
    // flood level flags (bit 0: a frontier, bit 1: a live excess vertex not
    // labelled yet), OR-ed by the waves into one of three words in rotation:
    // the word of level l is read after the level's barrier, and thread 0
    // clears the word of level l + 2 then
    __shared__ int s_flood[3];
    __shared__ __align__(16) unsigned char anyB[2][kW];
    __shared__ int s_r, s_active;
    __shared__ int s_wtot[kW];     // excess vertices per wave (push list offsets)
    __shared__ long long s_tr[4];  // trace: excess out, to sink, to boundary, label sum
    if (*A.actIn == 0ull) return;
    const int stageCap = stage_cap(A);
    const int V = A.G.V, N = A.G.N;
    constexpr int R = kMaxRows;  // 64 x 64 rows
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    u64 *zF = smem64;                      // [2 parity][2 face][kW][64]: z = 8w and z = 8w + 7
    u64 *recvB = smem64 + kFaceWords;      // [R] received excess (push); visited rows (search)
    u64 *clrB = recvB + R;                 // [R] drained (push); stage seeds (search)
    u64 *deadB = clrB + R;                 // [R] not reached by the last complete search
    u64 *stuckB = deadB + R;               // [R] excess vertices with no admissible arc left (push)
    unsigned *wlist = (unsigned *)(stuckB + R);  // [kListAll]
    const R64Scratch S = r64_scratch(R, A.nring);
    unsigned char *ws = (unsigned char *)A.scratch + (size_t)blockIdx.x * 16 * (size_t)V;
    GA u64 *resG = (GA u64 *)(ws + S.resG);
    GA u64 *rtG = (GA u64 *)(ws + S.rtG);
    GA int *haloG = (GA int *)(ws + S.halo);
    GA int *slotC = (GA int *)(ws + S.slot);
    GA u64 *admG = (GA u64 *)(ws + S.adm);
    const int dinf = A.dinf;
    const int nring = A.nring;
    // row of slot j of this thread: y = lane, z = 8 wid + j
    const int row0 = lane + 64 * kRPT * wid;
    int rc = 0;
    int fl = 0;
    if (tid < 3) s_flood[tid] = 0;
    // recv and clr are contiguous and return to zero after every use
    for (int i = tid; i < 2 * R; i += kNT) recvB[i] = 0ull;

    for (;;) {
        if (tid == 0) {
            const unsigned i = atomicAdd(A.qhead, 1u);
            s_r = (i < (unsigned)A.nwork) ? A.order[i] : -1;
        }
        __syncthreads();
        const int r = s_r;
        if (r < 0) return;
        const size_t base = (size_t)r * V;
        if (tid == 0) {
            s_active = A.ractive[r];
            // a deferred region keeps its flag and is discharged in a later sweep;
            // with deferRelabel it runs its region relabel now (s_active 2)
            if (s_active && A.defer && A.defer[r]) {
                s_active = A.deferRelabel ? 2 : 0;
                if (!s_active && A.actCarry) atomicAdd(A.actCarry, 1ull);  // still active
            } else {
                A.ractive[r] = 0;
            }
        }
        __syncthreads();
        if (!s_active) {
            // skipped region (no active vertex): its border labels carry over;
            // the interior is recomputed by its next discharge
            if (A.labNew != A.labOld)
                for (int i = tid; i < A.nring; i += kNT) {
                    const int l = A.ringL[i];
                    A.labNew[base + l] = A.labOld[base + l];
                }
            __syncthreads();
            continue;
        }
        const long long t_start = wall_clock64();
        if (tid < 4) s_tr[tid] = 0;

        u64 rk[kRPT][6], vis[kRPT], F[kRPT], exM[kRPT];
        // ---------------- row masks from HBM (coalesced loads + ballots) ----------------
        // Wave w builds its own rows: one load of a plane brings one whole row
        // (one vertex per lane); the eight planes of two rows are in flight
        // before their ballots.  The residual and t-link masks go to scratch.
#pragma unroll
        for (int j = 0; j < kRPT; j++) {
            const int rowA = 64 * (kRPT * wid + j);  // rows rowA .. rowA + 63, lane l owns rowA + l
            exM[j] = 0ull;
#pragma unroll 1
            for (int l0 = 0; l0 < 64; l0 += 2) {
                int v[2][8];
#pragma unroll
                for (int i = 0; i < 2; i++) {
                    const size_t off = base + (size_t)(rowA + l0 + i) * 64 + lane;
#pragma unroll
                    for (int q = 0; q < 8; q++) {
                        const int *plane = q < 6 ? A.res + (size_t)q * N : (q == 6 ? A.rt : A.ex);
                        v[i][q] = plane[off];
                    }
                }
#pragma unroll
                for (int i = 0; i < 2; i++) {
                    const int rowb = rowA + l0 + i;
#pragma unroll
                    for (int q = 0; q < 6; q++) {
                        const u64 b = __ballot(v[i][q] > 0);
                        if (lane == 0) resG[(size_t)q * R + rowb] = b;
                    }
                    const u64 bt = __ballot(v[i][6] > 0);
                    const u64 be = __ballot(v[i][7] > 0);
                    if (lane == 0) rtG[rowb] = bt;
                    if (lane == l0 + i) exM[j] = be;
                }
            }
            deadB[row0 + 64 * j] = 0ull;
        }
        // ---------------- halo labels d(w) of the border vertices ----------------
        for (int i = tid; i < nring; i += kNT) {
            const int l = A.ringL[i];
            const unsigned mm = A.ringM[i];
            int lz, ly, lx;
            local_xyz(A.G, l, lz, ly, lx);
#pragma unroll
            for (int a = 0; a < 3; a++) {
                int h = kInf;
                if ((mm >> (2 * a)) & 3u) {
                    const int w = cross_nbr(A.G, r, lz, ly, lx, r64_axis_dir(mm, a));
                    h = w >= 0 ? A.labOld[w] : kInf;
                }
                haloG[3 * i + a] = h;
            }
        }
        __syncthreads();

        int iter = 0;
        long long levels = 0, stages = 0, pushIters = 0, t_search = 0, t_flood = 0, t_stage = 0, t_push = 0;
        const bool relabelOnly = s_active == 2;
        bool writeMode = relabelOnly;
        for (;;) {
            // ---------------- multi-level search from the targets ----------------
            const long long t0s = wall_clock64();
            // stage candidate of each border vertex: smallest d(w) + 1 over its
            // residual boundary arcs (fixed during a search)
            // (eight border vertices per thread at a time, their loads issued together)
            for (int i0 = tid; i0 < nring; i0 += kNT * kRingBatch) {
                int ll[kRingBatch], hh[kRingBatch][3];
                unsigned mmb[kRingBatch];
                u64 rr[kRingBatch][3];
#pragma unroll
                for (int b = 0; b < kRingBatch; b++) {
                    const int i = i0 + b * kNT;
                    const bool in = i < nring;
                    ll[b] = in ? A.ringL[i] : 0;
                    mmb[b] = in ? A.ringM[i] : 0u;
#pragma unroll
                    for (int a = 0; a < 3; a++) hh[b][a] = in ? haloG[3 * i + a] : kInf;
                }
#pragma unroll
                for (int b = 0; b < kRingBatch; b++)
#pragma unroll
                    for (int a = 0; a < 3; a++)
                        rr[b][a] = ((mmb[b] >> (2 * a)) & 3u)
                                       ? resG[(size_t)r64_axis_dir(mmb[b], a) * R + (ll[b] >> 6)] : 0ull;
#pragma unroll
                for (int b = 0; b < kRingBatch; b++) {
                    const int i = i0 + b * kNT;
                    if (i >= nring) continue;
                    const u64 bit = 1ull << (ll[b] & 63);
                    int c = kInf;
#pragma unroll
                    for (int a = 0; a < 3; a++)
                        if ((rr[b][a] & bit) && hh[b][a] < dinf) c = min(c, hh[b][a] + 1);
                    slotC[i] = c;
                }
            }
            int cnt = 0;  // this thread's live excess vertices not labelled yet
            {
                const GA u64 *rg = r64_opaque(resG);
                const GA u64 *tg = r64_opaque(rtG);
                GA u64 *ag = r64_opaque(admG);
#pragma unroll
                for (int j = 0; j < kRPT; j++) {
                    const int row = row0 + 64 * j;
#pragma unroll
                    for (int k = 0; k < 6; k++) {
                        rk[j][k] = rg[(unsigned)(k * R + row)];
                        ag[(unsigned)(k * R + row)] = 0ull;  // admissible arcs of this search
                    }
                    const u64 rtm = tg[(unsigned)row];
                    vis[j] = rtm;
                    F[j] = rtm;
                    cnt += __popcll(exM[j] & ~rtm & ~deadB[row]);
                }
            }
            // the labels of a writing search are stored once per stage, for the
            // vertices visited since the previous stage (recv holds the visited
            // rows at each stage's end; each thread clears and reads its own rows)
            if (writeMode) {
#pragma unroll
                for (int j = 0; j < kRPT; j++) recvB[row0 + 64 * j] = 0ull;
            }
            int p = 0;
            int stage = 0;
            bool early = false;  // stopped with every live excess vertex labelled
            for (;;) {
                // flood inside the region: u with c_f(u, u + o_k) > 0 and u + o_k in the frontier
                const long long t0f = wall_clock64();
                for (;;) {
                    u64 anyF = 0ull;
#pragma unroll
                    for (int j = 0; j < kRPT; j++) anyF |= F[j];
                    zF[((p * 2 + 0) * kW + wid) * 64 + lane] = F[0];
                    zF[((p * 2 + 1) * kW + wid) * 64 + lane] = F[kRPT - 1];
                    {
                        const u64 b = __ballot(anyF != 0ull);
                        const u64 e = __ballot(cnt > 0);
                        const int f = ((b != 0ull) ? 1 : 0) | ((e != 0ull) ? 2 : 0);
                        if (lane == 0 && f) atomicOr(&s_flood[fl], f);
                    }
                    r64_lds_barrier();
                    const int any = s_flood[fl];
                    if (tid == 0) s_flood[fl == 0 ? 2 : fl - 1] = 0;  // the word of level l + 2
                    fl = fl == 2 ? 0 : fl + 1;
                    if (!writeMode && !(any & 2)) {
                        early = true;
                        break;
                    }
                    if (!(any & 1)) break;
                    levels++;
                    // z = 8w - 1 (top face of the wave below) and z = 8w + 8 (bottom face of the wave above)
                    u64 prev = wid > 0 ? zF[((p * 2 + 1) * kW + wid - 1) * 64 + lane] : 0ull;
                    const u64 above = wid < kW - 1 ? zF[((p * 2 + 0) * kW + wid + 1) * 64 + lane] : 0ull;
                    u64 old[kRPT];
#pragma unroll
                    for (int j = 0; j < kRPT; j++) old[j] = F[j];
                    // One pass per slot (the eight slots are independent, so their
                    // instructions interleave): the new vertices nw of each row,
                    // u with c_f(u, u + o_k) > 0 and u + o_k in the frontier (y +- 1
                    // from the neighbouring lanes, z +- 1 from the neighbouring slots
                    // or waves), then the arcs by which they were reached, their
                    // admissible arcs, ORed into one plane per direction.  The level
                    // is bound by vector-ALU issue: the six ORs go out for every lane
                    // with new vertices, without a test per direction (a 64-bit
                    // compare and branch each cost more than the ORs of zero), and
                    // address the planes by scalar base and 32-bit offset.
                    GA u64 *ad0 = r64_uniform(admG), *ad1 = r64_uniform(admG + R), *ad2 = r64_uniform(admG + 2 * R);
                    GA u64 *ad3 = r64_uniform(admG + 3 * R), *ad4 = r64_uniform(admG + 4 * R), *ad5 = r64_uniform(admG + 5 * R);
#pragma unroll
                    for (int j = 0; j < kRPT; j++) {
                        const u64 cur = old[j];
                        const u64 fzp = j < kRPT - 1 ? old[j + 1] : above;
                        const u64 fzm = j > 0 ? old[j - 1] : prev;
                        const u64 fyp = r64_from_next_lane(cur), fym = r64_from_prev_lane(cur);
                        const u64 a0 = rk[j][0] & (cur >> 1), a1 = rk[j][1] & (cur << 1), a2 = rk[j][2] & fyp;
                        const u64 a3 = rk[j][3] & fym, a4 = rk[j][4] & fzp, a5 = rk[j][5] & fzm;
                        const u64 nw = (a0 | a1 | a2 | a3 | a4 | a5) & ~vis[j];
                        F[j] = nw;
                        vis[j] |= nw;
                        // a writing search is followed by no push: it needs neither the
                        // admissible arcs nor the count of unlabelled excess vertices
                        if (writeMode || __ballot(nw != 0ull) == 0ull) continue;
                        if (!nw) continue;
                        const unsigned row = (unsigned)(row0 + 64 * j);
                        if (nw & exM[j]) cnt -= __popcll(nw & exM[j] & ~deadB[row]);
                        // an opaque 32-bit offset: widened to 64 bits, it would no
                        // longer fit the scalar-base form
                        unsigned boff = row * 8u;
                        asm volatile("" : "+v"(boff));
                        g_or((GA u64 *)((GA char *)ad0 + boff), nw & a0);
                        g_or((GA u64 *)((GA char *)ad1 + boff), nw & a1);
                        g_or((GA u64 *)((GA char *)ad2 + boff), nw & a2);
                        g_or((GA u64 *)((GA char *)ad3 + boff), nw & a3);
                        g_or((GA u64 *)((GA char *)ad4 + boff), nw & a4);
                        g_or((GA u64 *)((GA char *)ad5 + boff), nw & a5);
                    }
                    p ^= 1;
                }
                const long long t1f = wall_clock64();
                t_flood += t1f - t0f;
                if (early) break;
                // next stage: smallest candidate among unvisited border vertices
                // (the visited rows go to the recv buffer, free during a search)
                if (writeMode) {
#pragma unroll
                    for (int j = 0; j < kRPT; j++)
                        r64_store_labels(A.labNew + base, 64 * (kRPT * wid + j), vis[j] & ~recvB[row0 + 64 * j],
                                         stage, lane);
                }
#pragma unroll
                for (int j = 0; j < kRPT; j++) recvB[row0 + 64 * j] = vis[j];
                __syncthreads();
                int cand = kInf;
                for (int i0 = tid; i0 < nring; i0 += kNT * kRingBatch) {
                    int cc[kRingBatch], ll[kRingBatch];
#pragma unroll
                    for (int b = 0; b < kRingBatch; b++) {
                        const int i = i0 + b * kNT;
                        cc[b] = i < nring ? slotC[i] : kInf;
                        ll[b] = i < nring ? A.ringL[i] : 0;
                    }
#pragma unroll
                    for (int b = 0; b < kRingBatch; b++) {
                        if (cc[b] == kInf) continue;
                        if ((recvB[ll[b] >> 6] >> (ll[b] & 63)) & 1ull) {
                            slotC[i0 + b * kNT] = kInf;  // labelled: no longer a seed candidate in this search
                            continue;
                        }
                        cand = min(cand, cc[b]);
                    }
                }
                const int level = r64_block_min(cand, red, rc);
                // partial discharge: stages above the cap wait for later sweeps
                if (level == kInf || (level > stageCap && !writeMode)) {
                    t_stage += wall_clock64() - t1f;
                    break;
                }
                stages++;
                stage = level;
                for (int i0 = tid; i0 < nring; i0 += kNT * kRingBatch) {
                  int cc[kRingBatch];
#pragma unroll
                  for (int b = 0; b < kRingBatch; b++) cc[b] = (i0 + b * kNT < nring) ? slotC[i0 + b * kNT] : kInf;
#pragma unroll
                  for (int b = 0; b < kRingBatch; b++) {
                    const int i = i0 + b * kNT;
                    if (cc[b] != level) continue;
                    const int l = A.ringL[i];
                    const unsigned mm = A.ringM[i];
                    const int rw = l >> 6;
                    const u64 bit = 1ull << (l & 63);
                    unsigned match = 0u;
#pragma unroll
                    for (int a = 0; a < 3; a++) {
                        if (!((mm >> (2 * a)) & 3u)) continue;
                        const int k = r64_axis_dir(mm, a);
                        if (!(resG[(size_t)k * R + rw] & bit)) continue;
                        const int d = haloG[3 * i + a];
                        if (d < dinf && d + 1 == level) match |= 1u << k;
                    }
                    // the candidate came from one of these boundary arcs
#pragma unroll
                    for (int k = 0; k < 6; k++)
                        if (((match >> k) & 1u) && !writeMode) g_or(admG + (size_t)k * R + rw, bit);
                    slotC[i] = kInf;
                    atomicOr(&clrB[rw], bit);  // seeds (clr is all zero during a search)
                  }
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < kRPT; j++) {
                    const int row = row0 + 64 * j;
                    const u64 sd = clrB[row];
                    if (!sd) continue;
                    clrB[row] = 0ull;
                    F[j] = sd & ~vis[j];
                    vis[j] |= F[j];
                    if (F[j] & exM[j]) cnt -= __popcll(F[j] & exM[j] & ~deadB[row]);
                }
                t_stage += wall_clock64() - t1f;
            }
            // a search that ended by itself (under the same stage cap) leaves the dead set
            if (!early && !writeMode) {
#pragma unroll
                for (int j = 0; j < kRPT; j++) deadB[row0 + 64 * j] = ~vis[j];
            }
            // any excess vertex that reaches a target?
            u64 reach = 0ull;
#pragma unroll
            for (int j = 0; j < kRPT; j++) reach |= exM[j] & vis[j];
            const int found = r64_block_any(reach != 0ull, anyB, rc);
            const long long t1s = wall_clock64();
            t_search += t1s - t0s;
            if (writeMode) {
#pragma unroll
                for (int j = 0; j < kRPT; j++) r64_store_labels(A.labNew + base, 64 * (kRPT * wid + j), ~vis[j], dinf, lane);
                // excess left beyond the stage cap: the region stays active
                if (found && A.actCarry && tid == 0) {
                    A.ractive[r] = 1;
                    atomicAdd(A.actCarry, 1ull);
                }
                break;
            }
            if (!found) {
                writeMode = true;  // run the last search again, writing the region relabel
                continue;
            }
            if (++iter > A.maxIter) {
                if (tid == 0) atomicOr(A.err, 4);
                writeMode = true;
                continue;
            }
            if (A.roundCap > 0 && iter > A.roundCap) {
                // round cap: the last search writes the region relabel; excess it
                // still finds waits in the region for the next sweep
                writeMode = true;
                continue;
            }

            // ---------------- push along admissible arcs until nothing moves ----------------
            // recv held the visited rows: clear it for the pushes (clr is zero)
#pragma unroll
            for (int j = 0; j < kRPT; j++) {
                recvB[row0 + 64 * j] = 0ull;
                stuckB[row0 + 64 * j] = 0ull;
            }
            __syncthreads();
            // Push from excess vertex u (local index) along its admissible arcs, with
            // its t-link bits, admissible-arc byte, excess and residuals loaded.
            auto push_apply = [&](int u, u64 rtw, unsigned a0, int e, const int *c, int cT) -> int {
                const int row = u >> 6, x = u & 63;
                const u64 bit = 1ull << x;
                const size_t gu = base + u;
                if (e <= 0) {
                    // a receipt in this iteration sets the bit again at the merge
                    atomicOr(&clrB[row], bit);
                    return 0;
                }
                // a vertex with a residual t-link was a stage-0 seed: t is its only admissible arc
                const bool tseed = (rtw & bit) != 0ull;
                const unsigned a = tseed ? 0u : a0;
                if (!tseed && !a) {
                    // every admissible arc saturated: out of the lists until the next search
                    atomicOr(&stuckB[row], bit);
                    return 0;
                }
                int rem = e;
                bool left = false;  // admissible arcs left after the pushes
                if (tseed) {
                    const int d = min(rem, cT);
                    if (d > 0) {
                        A.rt[gu] = cT - d;
                        rem -= d;
                        if (A.trace) atomicAdd((unsigned long long *)&s_tr[1], (u64)d);
                    }
                    if (cT == d) g_and(rtG + row, ~bit);  // no admissible arc left
                    left = cT > d;
                } else {
                    const int y = row & 63, z = row >> 6;
#pragma unroll
                    for (int k = 0; k < 6; k++) {
                        if (!((a >> k) & 1u) || rem <= 0) continue;
                        const int d = min(rem, c[k]);
                        const bool out = k == 0 ? x == 63 : k == 1 ? x == 0 : k == 2 ? y == 63
                                       : k == 3 ? y == 0 : k == 4 ? z == 63 : z == 0;
                        if (d > 0) {
                            A.res[(size_t)k * N + gu] = c[k] - d;
                            if (out) {
                                // first-level vertex of a stage k > 0: over the boundary arc
                                atomicAdd(&A.pushb[(size_t)k * N + gu], d);
                                if (A.trace) atomicAdd((unsigned long long *)&s_tr[2], (u64)d);
                            } else {
                                const int v = u + ((k & 1) ? -1 : 1) * (k < 2 ? 1 : (k < 4 ? 64 : 4096));
                                const size_t gv = base + v;
                                const u64 vbit = 1ull << (v & 63);
                                atomicAdd(&A.res[(size_t)(k ^ 1) * N + gv], d);
                                atomicAdd(&A.ex[gv], d);
                                g_or(resG + (size_t)(k ^ 1) * R + (v >> 6), vbit);
                                atomicOr(&recvB[v >> 6], vbit);
                            }
                            rem -= d;
                        }
                        if (c[k] == d) {
                            g_and(admG + (size_t)k * R + row, ~bit);
                            g_and(resG + (size_t)k * R + row, ~bit);
                        } else {
                            left = true;
                        }
                    }
                }
                if (rem > 0 && !left) atomicOr(&stuckB[row], bit);
                if (rem < e) {
                    // drained what it saw: cleared, unless a receipt in this
                    // iteration sets the bit again at the merge
                    atomicAdd(&A.ex[gu], rem - e);
                    if (rem == 0) atomicOr(&clrB[row], bit);
                    return 1;
                }
                return 0;
            };
            for (;;) {
                int pushed = 0;
                // one workgroup-wide list of the reached excess vertices (a
                // wave's rows may hold far more of them than another's)
                int cntP = 0;
                u64 sel[kRPT];
#pragma unroll
                for (int j = 0; j < kRPT; j++) {
                    sel[j] = exM[j] & vis[j] & ~stuckB[row0 + 64 * j];
                    cntP += __popcll(sel[j]);
                }
                const int incl = r64_incl_scan(cntP, lane);
                if (lane == 63) s_wtot[wid] = incl;
                __syncthreads();
                int first = incl - cntP, total = 0;
#pragma unroll
                for (int w = 0; w < kW; w++) {
                    const int t = s_wtot[w];
                    if (w < wid) first += t;
                    total += t;
                }
                for (int w0 = 0; w0 < total; w0 += kListAll) {
                    if (cntP && first < w0 + kListAll && first + cntP > w0) {
                        int idx = first;
#pragma unroll
                        for (int j = 0; j < kRPT; j++) {
                            u64 m = sel[j];
                            const int row = row0 + 64 * j;
                            while (m) {
                                const int x = __builtin_ctzll(m);
                                m &= m - 1;
                                if (idx >= w0 && idx < w0 + kListAll) wlist[idx - w0] = (unsigned)(row * 64 + x);
                                idx++;
                            }
                        }
                    }
                    __syncthreads();
                    const int nItems = min(total - w0, kListAll);
                    // kInFlight vertices per lane: their loads are issued together
                    for (int it0 = tid; it0 < nItems; it0 += kNT * kInFlight) {
                        int uu[kInFlight], ee[kInFlight], cT[kInFlight], cc[kInFlight][6];
                        u64 rtw[kInFlight];
                        unsigned a0[kInFlight];
#pragma unroll
                        for (int b = 0; b < kInFlight; b++) {
                            const int it = it0 + b * kNT;
                            uu[b] = it < nItems ? (int)wlist[it] : -1;
                        }
                        // every load of the kInFlight vertices issued before any is
                        // used, without a branch (an empty entry reads vertex 0 and is
                        // masked afterwards), and of each 64-bit row word only the
                        // 32-bit half that holds the vertex's bit: with branches and
                        // whole words the compiler, at this register pressure, put
                        // each load behind the previous one's wait
                        {
                            unsigned hw[kInFlight][7];
                            int ev[kInFlight];
                            GA const unsigned *rt32 = (GA const unsigned *)r64_uniform(rtG);
                            GA const unsigned *ad32 = (GA const unsigned *)r64_uniform(admG);
                            GA const int *ex32 = (GA const int *)r64_uniform((GA int *)(A.ex + base));
#pragma unroll
                            for (int b = 0; b < kInFlight; b++) {
                                const unsigned u = uu[b] >= 0 ? (unsigned)uu[b] : 0u;
                                unsigned hi = u >> 5;  // 32-bit word of the bit: 2 rr + (xb >> 5)
                                asm volatile("" : "+v"(hi));
                                hw[b][6] = rt32[hi];
#pragma unroll
                                for (int k = 0; k < 6; k++) hw[b][k] = ad32[(unsigned)(2 * k * R) + hi];
                                unsigned uo = u;
                                asm volatile("" : "+v"(uo));
                                ev[b] = ex32[uo];
                            }
#pragma unroll
                            for (int b = 0; b < kInFlight; b++) {
                                const bool in = uu[b] >= 0;
                                const unsigned sh = (unsigned)uu[b] & 31u;
                                unsigned a = 0u;
#pragma unroll
                                for (int k = 0; k < 6; k++) a |= ((hw[b][k] >> sh) & 1u) << k;
                                a0[b] = in ? a : 0u;
                                // the t-link bit in its place in the 64-bit row word
                                rtw[b] = (in && ((hw[b][6] >> sh) & 1u)) ? (1ull << ((unsigned)uu[b] & 63u)) : 0ull;
                                ee[b] = in ? ev[b] : 0;
                            }
                        }
#pragma unroll
                        for (int b = 0; b < kInFlight; b++) {
                            cT[b] = 0;
#pragma unroll
                            for (int k = 0; k < 6; k++) cc[b][k] = 0;
                            if (uu[b] < 0 || ee[b] <= 0) continue;
                            const size_t gu = base + uu[b];
                            if ((rtw[b] >> (uu[b] & 63)) & 1ull) {
                                cT[b] = A.rt[gu];
                            } else {
#pragma unroll
                                for (int k = 0; k < 6; k++)
                                    if ((a0[b] >> k) & 1u) cc[b][k] = A.res[(size_t)k * N + gu];
                            }
                        }
#pragma unroll
                        for (int b = 0; b < kInFlight; b++)
                            if (uu[b] >= 0) pushed |= push_apply(uu[b], rtw[b], a0[b], ee[b], cc[b], cT[b]);
                    }
                    __syncthreads();  // the list is rewritten by the next pass
                }
                const int any = r64_block_any(pushed, anyB, rc);
                pushIters++;
                // merge the iteration's receipts and drains into the excess rows,
                // and clear them before any push of the next iteration
#pragma unroll
                for (int j = 0; j < kRPT; j++) {
                    const int row = row0 + 64 * j;
                    const u64 rv = recvB[row], cl = clrB[row];
                    exM[j] = (exM[j] & ~cl) | rv;
                    recvB[row] = 0ull;
                    clrB[row] = 0ull;
                }
                __syncthreads();
                if (!any) break;
                // guard: pushes follow a fixed level order and end long before this
                if (pushIters > (1ll << 24)) {
                    if (tid == 0) atomicOr(A.err, 4);
                    writeMode = true;
                    break;
                }
            }
            t_push += wall_clock64() - t1s;
            if (writeMode) continue;
            // no excess left in the region (the masks may only over-report it):
            // the next search cannot find an excess vertex, so it writes the labels
            u64 left = 0ull;
#pragma unroll
            for (int j = 0; j < kRPT; j++) left |= exM[j];
            if (!r64_block_any(left != 0ull, anyB, rc)) writeMode = true;
        }
        __syncthreads();
        if (A.trace) {
            long long ex_out = 0, lsum = 0;
            for (int l = tid; l < V; l += kNT) ex_out += A.ex[base + l];
            for (int i = tid; i < nring; i += kNT) lsum += min(A.labNew[base + A.ringL[i]], 65535);
            atomicAdd((unsigned long long *)&s_tr[0], (u64)ex_out);
            atomicAdd((unsigned long long *)&s_tr[3], (u64)lsum);
        }
        __syncthreads();
        if (tid == 0 && relabelOnly) {
            atomicAdd(&A.stats[11], 1ull);
        } else if (tid == 0) {
            atomicAdd(&A.stats[0], 1ull);
            if (A.regionTicks) A.regionTicks[r] = (int)min(wall_clock64() - t_start, 0x7fffffffLL);
            atomicAdd(&A.stats[1], (u64)A.rvcount[r]);
            atomicAdd(&A.stats[2], (u64)(iter + 1));
            atomicAdd(&A.stats[3], (u64)levels);
            atomicAdd(&A.stats[4], (u64)stages);
            atomicAdd(&A.stats[6], (u64)t_search);
            atomicAdd(&A.stats[7], (u64)t_push);
            atomicAdd(&A.stats[8], (u64)t_stage);
            atomicAdd(&A.stats[9], (u64)t_flood);
            atomicAdd(&A.stats[10], (u64)pushIters);
            if (A.trace) {
                const unsigned long long idx = atomicAdd(&A.stats[5], 1ull);
                if ((long long)idx < A.traceCap) {
                    int *rec = A.trace + idx * 10;
                    rec[0] = A.sweep;
                    rec[1] = r;
                    rec[2] = iter + 1;
                    rec[3] = (int)min(levels, 0x7fffffffLL);
                    rec[4] = (int)min(stages, 0x7fffffffLL);
                    rec[5] = (int)min(wall_clock64() - t_start, 0x7fffffffLL);
                    rec[6] = (int)min(s_tr[0] + s_tr[1] + s_tr[2], 0x7fffffffLL);
                    rec[7] = (int)min(s_tr[1], 0x7fffffffLL);
                    rec[8] = (int)min(s_tr[2], 0x7fffffffLL);
                    rec[9] = (int)min(s_tr[3], 0x7fffffffLL);
                }
            }
        }
        __syncthreads();
    }
}

// Global relabel, one distance level D (see k_grelabel in mf_kernels.hip), for
// the 64^3 tiles of k_discharge_rows64, with the same row ownership: lane y of
// wave w holds the rows (y, z) with z = 8w .. 8w + 7 in registers.  At level 0
// every region builds its residual-arc masks from HBM and keeps them, with the
// mask of its unlabelled vertices, in a per-region cache (seven planes of 4096
// rows); later levels read the cache.  The flood advances one step per
// workgroup barrier, from t at level 0 and from the seed bits marked by the
// previous level otherwise; reached vertices get label D, and reached border
// vertices mark their residual predecessors across the border (unlabelled) as
// seeds of D + 1 and flag their regions.
__global__ __launch_bounds__(kNT) void k_grelabel_rows64(GRelabelArgs A) {
    __shared__ __align__(16) u64 zF[kFaceWords];  // [2 parity][2 face][kW][64]
    __shared__ __align__(16) unsigned char anyB[2][kW];
    __shared__ int s_go;
    const Geo &G = A.G;
    const int V = G.V, N = G.N, D = A.level, dinf = A.dinf;
    constexpr int R = kMaxRows;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int row0 = lane + 64 * kRPT * wid;  // row of slot j: row0 + 64 j
    int rc = 0;
    // predecessor across the border of the reached border vertex (z, y, x) in
    // direction k: u = v + o_k with residual arc (u, v) in direction k ^ 1
    auto mark = [&](int r, int z, int y, int x, int k) {
        const int ug = cross_nbr(G, r, z, y, x, k);
        if (ug < 0 || A.res[(size_t)(k ^ 1) * N + ug] <= 0 || A.lab[ug] != dinf) return;
        atomicOr(&A.candBitsOut[ug >> 5], 1u << (ug & 31));
        const int ru = ug / V;
        if (A.flagOut[ru] == 0 && atomicExch(&A.flagOut[ru], 1) == 0) atomicAdd(A.flagged, 1u);
    };
    for (int r = blockIdx.x; r < G.nreg; r += gridDim.x) {
        if (tid == 0) {
            s_go = (D == 0) ? 1 : A.flagIn[r];
            if (D > 0) A.flagIn[r] = 0;
        }
        __syncthreads();
        const int go = s_go;
        __syncthreads();
        if (!go) continue;
        const size_t base = (size_t)r * V;
        GA u64 *cr = (GA u64 *)A.cache + (size_t)r * 7 * R;
        u64 rk[kRPT][6], F[kRPT], avail[kRPT];
        if (D == 0) {
            // planes 0..5 residual arcs, plane 6 residual t-links (the seeds): one
            // load of a plane brings one row (one vertex per lane), the seven
            // planes of two rows are in flight before their ballots
#pragma unroll
            for (int j = 0; j < kRPT; j++) {
                const int rowA = 64 * (kRPT * wid + j);
#pragma unroll
                for (int q = 0; q < 6; q++) rk[j][q] = 0ull;
                F[j] = 0ull;
#pragma unroll 1
                for (int l0 = 0; l0 < 64; l0 += 2) {
                    int v[2][7];
#pragma unroll
                    for (int i = 0; i < 2; i++) {
                        const size_t off = base + (size_t)(rowA + l0 + i) * 64 + lane;
#pragma unroll
                        for (int q = 0; q < 7; q++) v[i][q] = (q < 6 ? A.res + (size_t)q * N : A.rt)[off];
                    }
#pragma unroll
                    for (int i = 0; i < 2; i++) {
#pragma unroll
                        for (int q = 0; q < 6; q++) {
                            const u64 b = __ballot(v[i][q] > 0);
                            if (lane == l0 + i) rk[j][q] = b;
                        }
                        const u64 bt = __ballot(v[i][6] > 0);
                        if (lane == l0 + i) F[j] = bt;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < kRPT; j++) {
#pragma unroll
                for (int q = 0; q < 6; q++) cr[(size_t)q * R + row0 + 64 * j] = rk[j][q];
                avail[j] = ~F[j];
            }
        } else {
            GA u64 *cb = (GA u64 *)A.candBitsIn + (base >> 6);
#pragma unroll
            for (int j = 0; j < kRPT; j++) {
                const int row = row0 + 64 * j;
#pragma unroll
                for (int q = 0; q < 6; q++) rk[j][q] = cr[(size_t)q * R + row];
                const u64 U = cr[(size_t)6 * R + row];
                const u64 c = cb[row];
                if (c) cb[row] = 0ull;
                F[j] = c & U;
                avail[j] = U & ~F[j];
            }
        }
        int p = 0;
        for (;;) {
            u64 anyF = 0ull;
#pragma unroll
            for (int j = 0; j < kRPT; j++) anyF |= F[j];
            zF[((p * 2 + 0) * kW + wid) * 64 + lane] = F[0];
            zF[((p * 2 + 1) * kW + wid) * 64 + lane] = F[kRPT - 1];
            if (!r64_block_any(anyF != 0ull, anyB, rc)) break;
            // z = 8w - 1 (top face of the wave below) and z = 8w + 8 (bottom face of the wave above)
            const u64 below = wid > 0 ? zF[((p * 2 + 1) * kW + wid - 1) * 64 + lane] : 0ull;
            const u64 above = wid < kW - 1 ? zF[((p * 2 + 0) * kW + wid + 1) * 64 + lane] : 0ull;
            u64 old[kRPT];
#pragma unroll
            for (int j = 0; j < kRPT; j++) old[j] = F[j];
#pragma unroll
            for (int j = 0; j < kRPT; j++) {
                const u64 cur = old[j];
                const u64 fzp = j < kRPT - 1 ? old[j + 1] : above;
                const u64 fzm = j > 0 ? old[j - 1] : below;
                const u64 fyp = r64_from_next_lane(cur), fym = r64_from_prev_lane(cur);
                const u64 reach = (rk[j][0] & (cur >> 1)) | (rk[j][1] & (cur << 1)) | (rk[j][2] & fyp) |
                                  (rk[j][3] & fym) | (rk[j][4] & fzp) | (rk[j][5] & fzm);
                F[j] = reach & avail[j];
                avail[j] &= ~F[j];
            }
            p ^= 1;
        }
        // reached = unlabelled before this level and not available now; the
        // unlabelled mask of the cache is written by every row at level 0
#pragma unroll
        for (int j = 0; j < kRPT; j++) {
            const int row = row0 + 64 * j;
            const u64 U0 = D == 0 ? ~0ull : cr[(size_t)6 * R + row];
            F[j] = U0 & ~avail[j];
            if (D == 0 || F[j]) cr[(size_t)6 * R + row] = avail[j];
        }
#pragma unroll
        for (int j = 0; j < kRPT; j++) r64_store_labels(A.lab + base, 64 * (kRPT * wid + j), F[j], D, lane);
        // x faces: bit 63 leaves by +x, bit 0 by -x
#pragma unroll
        for (int j = 0; j < kRPT; j++) {
            const int z = kRPT * wid + j;
            if (F[j] >> 63) mark(r, z, lane, 63, 0);
            if (F[j] & 1ull) mark(r, z, lane, 0, 1);
        }
        // y faces: the rows of lane 63 (+y) and lane 0 (-y), one vertex per lane
#pragma unroll
        for (int j = 0; j < kRPT; j++) {
            const int z = kRPT * wid + j;
            const u64 top = ((u64)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)(F[j] >> 32), 63) << 32) |
                            (u64)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)F[j], 63);
            const u64 bot = ((u64)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)(F[j] >> 32), 0) << 32) |
                            (u64)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)F[j], 0);
            if ((top >> lane) & 1ull) mark(r, z, 63, lane, 2);
            if ((bot >> lane) & 1ull) mark(r, z, 0, lane, 3);
        }
        // z faces: slot 0 of wave 0 (-z) and slot 7 of the last wave (+z), one row
        // (one y) at a time, one vertex per lane
        if (wid == 0 || wid == kW - 1) {
            const u64 m = wid == 0 ? F[0] : F[kRPT - 1];
            const int z = wid == 0 ? 0 : 64 - 1, k = wid == 0 ? 5 : 4;
            u64 pend = __ballot(m != 0ull);
            while (pend) {
                const int yy = __builtin_ctzll(pend);
                pend &= pend - 1;
                const u64 bits = ((u64)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)(m >> 32), yy) << 32) |
                                 (u64)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)m, yy);
                if ((bits >> lane) & 1ull) mark(r, z, yy, lane, k);
            }
        }
    }
}

// Residual reachability for the cuts (the region floods of k_flood, same
// marks) on the 64^3 tiles of k_discharge_rows64, with its row ownership.
// dir 0 floods forward from the excess vertices along arcs with c_f > 0 (the
// frontier is masked by the arcs at their tails and moved to their heads), dir
// 1 backward from t.  Each round every dirty region builds its residual-arc
// masks and its marks (round 0: the seeds) from HBM, floods one step per
// workgroup barrier, stores the marks of the vertices it reached, and marks
// the neighbours across the border that its reached border vertices reach
// (atomic exchange, as k_flood), flagging their regions.
__global__ __launch_bounds__(kNT) void k_flood_rows64(FloodArgs A) {
    __shared__ __align__(16) u64 zF[kFaceWords];  // [2 parity][2 face][kW][64]
    __shared__ __align__(16) unsigned char anyB[2][kW];
    __shared__ int s_go;
    const Geo &G = A.G;
    const int V = G.V, N = G.N, dir = A.dir;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int rc = 0;
    // the neighbour wg across the border of the reached border vertex (z, y, x)
    // in direction k, when the arc between them points the flood's way
    auto xmark = [&](int r, int z, int y, int x, int k) {
        const int wg = cross_nbr(G, r, z, y, x, k);
        if (wg < 0) return;
        // backward: the arc (u, v) from u = v + o_k, in direction k ^ 1, is residual
        if (dir == 1 && A.res[(size_t)(k ^ 1) * N + wg] <= 0) return;
        if (A.mark[wg] == 0 && atomicExch(&A.mark[wg], 1) == 0) {
            A.dirtyOut[wg / V] = 1;
            atomicAdd(A.changed, 1u);
        }
    };
    for (int r = blockIdx.x; r < G.nreg; r += gridDim.x) {
        if (tid == 0) {
            s_go = (A.round == 0) ? 1 : A.dirtyIn[r];
            A.dirtyIn[r] = 0;
        }
        __syncthreads();
        const int go = s_go;
        __syncthreads();
        if (!go) continue;
        const size_t base = (size_t)r * V;
        // planes 0..5 residual arcs, plane 6 the marks (round 0: the seeds, ex > 0
        // forward, r_t > 0 backward); one load of a plane brings one row
        const int *p6 = A.round > 0 ? A.mark : (dir == 0 ? A.ex : A.rt);
        u64 rk[kRPT][6], M[kRPT];
#pragma unroll
        for (int j = 0; j < kRPT; j++) {
            const int rowA = 64 * (kRPT * wid + j);
#pragma unroll
            for (int q = 0; q < 6; q++) rk[j][q] = 0ull;
            M[j] = 0ull;
#pragma unroll 1
            for (int l0 = 0; l0 < 64; l0 += 2) {
                int v[2][7];
#pragma unroll
                for (int i = 0; i < 2; i++) {
                    const size_t off = base + (size_t)(rowA + l0 + i) * 64 + lane;
#pragma unroll
                    for (int q = 0; q < 7; q++) v[i][q] = (q < 6 ? A.res + (size_t)q * N : p6)[off];
                }
#pragma unroll
                for (int i = 0; i < 2; i++) {
#pragma unroll
                    for (int q = 0; q < 6; q++) {
                        const u64 b = __ballot(v[i][q] > 0);
                        if (lane == l0 + i) rk[j][q] = b;
                    }
                    const u64 bm = __ballot(v[i][6] > 0);
                    if (lane == l0 + i) M[j] = bm;
                }
            }
        }
        u64 F[kRPT], reached[kRPT];
#pragma unroll
        for (int j = 0; j < kRPT; j++) F[j] = reached[j] = M[j];
        int p = 0;
        for (;;) {
            u64 anyF = 0ull;
#pragma unroll
            for (int j = 0; j < kRPT; j++) anyF |= F[j];
            // z faces: forward, the frontier on the arcs leaving the wave's slab
            // (-z from slot 0, +z from slot 7); backward, the frontier itself
            zF[((p * 2 + 0) * kW + wid) * 64 + lane] = dir == 0 ? (F[0] & rk[0][5]) : F[0];
            zF[((p * 2 + 1) * kW + wid) * 64 + lane] = dir == 0 ? (F[kRPT - 1] & rk[kRPT - 1][4]) : F[kRPT - 1];
            if (!r64_block_any(anyF != 0ull, anyB, rc)) break;
            const u64 below = wid > 0 ? zF[((p * 2 + 1) * kW + wid - 1) * 64 + lane] : 0ull;
            const u64 above = wid < kW - 1 ? zF[((p * 2 + 0) * kW + wid + 1) * 64 + lane] : 0ull;
            u64 old[kRPT];
#pragma unroll
            for (int j = 0; j < kRPT; j++) old[j] = F[j];
#pragma unroll
            for (int j = 0; j < kRPT; j++) {
                const u64 cur = old[j];
                u64 reach;
                if (dir == 0) {
                    // heads of the residual arcs leaving the frontier
                    const u64 fromZm = j > 0 ? (old[j - 1] & rk[j - 1][4]) : below;
                    const u64 fromZp = j < kRPT - 1 ? (old[j + 1] & rk[j + 1][5]) : above;
                    reach = ((cur & rk[j][0]) << 1) | ((cur & rk[j][1]) >> 1) | r64_from_prev_lane(cur & rk[j][2]) |
                            r64_from_next_lane(cur & rk[j][3]) | fromZm | fromZp;
                } else {
                    // tails of the residual arcs entering the frontier
                    const u64 fzp = j < kRPT - 1 ? old[j + 1] : above;
                    const u64 fzm = j > 0 ? old[j - 1] : below;
                    reach = (rk[j][0] & (cur >> 1)) | (rk[j][1] & (cur << 1)) | (rk[j][2] & r64_from_next_lane(cur)) |
                            (rk[j][3] & r64_from_prev_lane(cur)) | (rk[j][4] & fzp) | (rk[j][5] & fzm);
                }
                F[j] = reach & ~reached[j];
                reached[j] |= F[j];
            }
            p ^= 1;
        }
        // marks of this round, seeds included (stores of 1 race harmlessly with
        // the neighbours' exchanges)
#pragma unroll
        for (int j = 0; j < kRPT; j++)
            r64_store_labels(A.mark + base, 64 * (kRPT * wid + j), A.round > 0 ? reached[j] & ~M[j] : reached[j], 1,
                             lane);
        // reached border vertices; forward only those whose leaving arc is residual
        // x faces: bit 63 leaves by +x, bit 0 by -x
#pragma unroll
        for (int j = 0; j < kRPT; j++) {
            const int z = kRPT * wid + j;
            const u64 m0 = dir == 0 ? reached[j] & rk[j][0] : reached[j];
            const u64 m1 = dir == 0 ? reached[j] & rk[j][1] : reached[j];
            if (m0 >> 63) xmark(r, z, lane, 63, 0);
            if (m1 & 1ull) xmark(r, z, lane, 0, 1);
        }
        // y faces: the rows of lane 63 (+y) and lane 0 (-y), one vertex per lane
#pragma unroll
        for (int j = 0; j < kRPT; j++) {
            const int z = kRPT * wid + j;
            const u64 m2 = dir == 0 ? reached[j] & rk[j][2] : reached[j];
            const u64 m3 = dir == 0 ? reached[j] & rk[j][3] : reached[j];
            const u64 top = ((u64)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)(m2 >> 32), 63) << 32) |
                            (u64)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)m2, 63);
            const u64 bot = ((u64)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)(m3 >> 32), 0) << 32) |
                            (u64)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)m3, 0);
            if ((top >> lane) & 1ull) xmark(r, z, 63, lane, 2);
            if ((bot >> lane) & 1ull) xmark(r, z, 0, lane, 3);
        }
        // z faces: slot 0 of wave 0 (-z) and slot 7 of the last wave (+z), one row
        // (one y) at a time, one vertex per lane
        if (wid == 0 || wid == kW - 1) {
            const int k = wid == 0 ? 5 : 4, z = wid == 0 ? 0 : 64 - 1;
            const u64 rm = wid == 0 ? reached[0] : reached[kRPT - 1];
            const u64 m = dir == 0 ? rm & (wid == 0 ? rk[0][5] : rk[kRPT - 1][4]) : rm;
            u64 pend = __ballot(m != 0ull);
            while (pend) {
                const int yy = __builtin_ctzll(pend);
                pend &= pend - 1;
                const u64 bits = ((u64)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)(m >> 32), yy) << 32) |
                                 (u64)(unsigned)__builtin_amdgcn_readlane((int)(unsigned)m, yy);
                if ((bits >> lane) & 1ull) xmark(r, z, yy, lane, k);
            }
        }
    }
}

hipError_t launch_flood_rows64(const FloodArgs &A, int blocks, hipStream_t s) {
    if (!rows64_applicable(A.G.K, A.G.tx, A.G.ty, A.G.tz) || A.noCross) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_flood_rows64, dim3(blocks), dim3(kNT), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_grelabel_rows64(const GRelabelArgs &A, int blocks, hipStream_t s) {
    if (!rows64_applicable(A.G.K, A.G.tx, A.G.ty, A.G.tz) || !A.cache || !A.candBitsIn || !A.candBitsOut)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_grelabel_rows64, dim3(blocks), dim3(kNT), 0, s, A);
    return hipGetLastError();
}

size_t grelabel_rows64_cache_bytes(int nreg) { return (size_t)nreg * 7 * kMaxRows * sizeof(u64); }

void set_rows64_attributes() {
    (void)hipFuncSetAttribute((const void *)k_discharge_rows64, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
}

hipError_t launch_discharge_rows64(const DischargeArgs &A, int blocks, size_t lds, hipStream_t s) {
    if (!rows64_applicable(A.G.K, A.G.tx, A.G.ty, A.G.tz) || lds < discharge_rows64_bytes(A.G.ty, A.G.tz) ||
        rows64_scratch_bytes(A.G.ty, A.G.tz, A.nring) > (size_t)16 * A.G.V)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_discharge_rows64, dim3(blocks), dim3(kNT), lds, s, A);
    return hipGetLastError();
}

}  // namespace mfd
