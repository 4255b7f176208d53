// Single-wavefront region discharge for 2D tiles of at most 64 x 64 vertices
// (Proc. ARD of Sec. 4.2 with the region relabel of Alg. 3; same method as
// k_discharge, different execution).
//
// One wave64 owns a region.  Lane y holds row y of the tile as 64-bit masks:
// residual arc present in each direction, residual t-link, excess present,
// visited, frontier, and the arcs by which the search reached each vertex (its
// admissible arcs, pointing one search level down).  A search level is a
// handful of shifts, two cross-lane row exchanges and ORs in registers, with no
// LDS traffic and no barrier.  The integer state (residuals, t-links, excess,
// halo labels, boundary pushes) is staged in LDS, in 8-bit residuals and 16-bit
// excess when the capacities allow it (two regions per compute unit), else in
// 16- or 32-bit residuals.  The push phase moves excess along admissible arcs:
// in every iteration each excess vertex pushes as much as it can, the excess
// vertices are spread over the 64 lanes through a work list, and iterations
// repeat until nothing moves.  Search and push alternate until no excess
// vertex reaches a target; the last search is run again to write the labels.
#include "mf_device.h"
#include "mf_launch.h"

namespace mfd {

typedef unsigned long long u64;

namespace {


__host__ __device__ inline size_t al16w(size_t x) { return (x + 15) & ~(size_t)15; }

struct WaveLayout {
    size_t res, ex, rt, halo, push, resM, admM, rows, list, total;  // byte offsets
};

// rtBytes: residual and t-link width (1, 2, 4); exBytes: excess width (2, 4)
__host__ __device__ inline WaveLayout wave_layout(int V, int K, int nring, int rtBytes, int exBytes) {
    WaveLayout L;
    size_t o = 0;
    L.res = o; o = al16w(o + (size_t)V * K * rtBytes);
    L.ex = o; o = al16w(o + (size_t)(V + 1) * exBytes);
    L.rt = o; o = al16w(o + (size_t)V * rtBytes);
    L.halo = o; o = al16w(o + (size_t)nring * K * 4);
    L.push = o; o = al16w(o + (size_t)nring * K * 4);
    L.resM = o; o = al16w(o + (size_t)K * 64 * 8);        // residual arc inside the tile, per direction
    L.admM = o; o = al16w(o + (size_t)(K + 1) * 64 * 8);  // admissible arcs of the round, then t
    L.rows = o; o = al16w(o + (size_t)3 * 64 * 8);        // residual t-link, received, drained rows
    L.list = o; o = al16w(o + (size_t)V * 2);              // work list: room for every vertex
    L.total = o;
    return L;
}

__device__ __forceinline__ u64 shfl64(u64 v, int src) {
    return __shfl(v, src, 64);
}

// Bits of row mask m moved so that bit x holds bit x + dx.
__device__ __forceinline__ u64 shift_dx(u64 m, int dx) {
    return dx > 0 ? (m >> dx) : (dx < 0 ? (m << (-dx)) : m);
}

// Whole-wave lane shifts by DPP (wave_shr:1 / wave_shl:1): lane i reads lane
// i - 1 / i + 1 of v; lanes without a source read 0.
__device__ __forceinline__ u64 lane_prev(u64 v) {
    const unsigned lo = __builtin_amdgcn_update_dpp(0u, (unsigned)v, 0x138, 0xf, 0xf, true);
    const unsigned hi = __builtin_amdgcn_update_dpp(0u, (unsigned)(v >> 32), 0x138, 0xf, 0xf, true);
    return ((u64)hi << 32) | lo;
}
__device__ __forceinline__ u64 lane_next(u64 v) {
    const unsigned lo = __builtin_amdgcn_update_dpp(0u, (unsigned)v, 0x130, 0xf, 0xf, true);
    const unsigned hi = __builtin_amdgcn_update_dpp(0u, (unsigned)(v >> 32), 0x130, 0xf, 0xf, true);
    return ((u64)hi << 32) | lo;
}

// Rows y-1, y, y+1 of a per-lane row mask (0 outside the tile).  Lanes at or
// beyond the tile's last row hold 0, so the shifted-in rows are 0 there.
struct Rows3 {
    u64 up, mid, dn;  // row y-1, y, y+1
    __device__ __forceinline__ u64 at(int dy) const { return dy < 0 ? up : (dy > 0 ? dn : mid); }
};

__device__ __forceinline__ Rows3 rows3(u64 v, int y, int ty) {
    (void)y;
    (void)ty;
    Rows3 r;
    r.mid = v;
    r.up = lane_prev(v);
    r.dn = lane_next(v);
    return r;
}

__device__ __forceinline__ int wave_min_int(int v) {
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ int wave_scan_incl(int v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// LDS written by one lane and read by another lane of the same wave.
__device__ __forceinline__ void lane_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Excess in LDS: 32-bit, or 16-bit packed two to a word (every excess is at
// most c(s,v) + sum_u c(u,v) <= 32767 then, so a half never carries or borrows).
__device__ __forceinline__ int ex_get(const int *e, int i) { return e[i]; }
__device__ __forceinline__ int ex_get(const short *e, int i) { return e[i]; }
__device__ __forceinline__ void ex_add(int *e, int i, int d) { atomicAdd(&e[i], d); }
__device__ __forceinline__ void ex_add(short *e, int i, int d) {
    atomicAdd((unsigned *)(e + (i & ~1)), (unsigned)d << ((i & 1) * 16));
}
// subtract d and return the value before
__device__ __forceinline__ int ex_sub(int *e, int i, int d) { return atomicSub(&e[i], d); }
__device__ __forceinline__ int ex_sub(short *e, int i, int d) {
    const int sh = (i & 1) * 16;
    const unsigned old = atomicSub((unsigned *)(e + (i & ~1)), (unsigned)d << sh);
    return (int)((old >> sh) & 0xffffu);
}

// Add d to a residual in LDS without reading it: 8- and 16-bit residuals are
// added to their containing 32-bit word (a residual never exceeds its pair sum,
// which fits its width, so no carry leaves it).
__device__ __forceinline__ void res_add(unsigned char *r, int i, int d) {
    atomicAdd((unsigned *)(r + (i & ~3)), (unsigned)d << ((i & 3) * 8));
}
__device__ __forceinline__ void res_add(short *r, int i, int d) {
    atomicAdd((unsigned *)(r + (i & ~1)), (unsigned)d << ((i & 1) * 16));
}
__device__ __forceinline__ void res_add(int *r, int i, int d) { atomicAdd(&r[i], d); }

// The K residuals of one vertex (contiguous, K * sizeof(RT) bytes at a multiple
// of that size) in one or two vector loads.
template <int K, typename RT>
__device__ __forceinline__ void load_res_row(const RT *p, RT (&out)[K]) {
    constexpr int B = K * (int)sizeof(RT);
    static_assert(B == 4 || B == 8 || B == 16 || B == 32, "residual row of 4, 8, 16 or 32 bytes");
    if constexpr (B == 4) {
        const unsigned w = *(const unsigned *)p;
        __builtin_memcpy(out, &w, 4);
    } else if constexpr (B == 8) {
        const uint2 w = *(const uint2 *)p;
        __builtin_memcpy(out, &w, 8);
    } else if constexpr (B == 16) {
        const uint4 w = *(const uint4 *)p;
        __builtin_memcpy(out, &w, 16);
    } else {
        const uint4 a = ((const uint4 *)p)[0], b = ((const uint4 *)p)[1];
        __builtin_memcpy(out, &a, 16);
        __builtin_memcpy((char *)out + 16, &b, 16);
    }
}

template <int K, typename RT>
__device__ __forceinline__ void store_res_row(RT *p, const RT (&in)[K]) {
    constexpr int B = K * (int)sizeof(RT);
    static_assert(B == 4 || B == 8 || B == 16 || B == 32, "residual row of 4, 8, 16 or 32 bytes");
    if constexpr (B == 4) {
        unsigned w;
        __builtin_memcpy(&w, in, 4);
        *(unsigned *)p = w;
    } else if constexpr (B == 8) {
        uint2 w;
        __builtin_memcpy(&w, in, 8);
        *(uint2 *)p = w;
    } else if constexpr (B == 16) {
        uint4 w;
        __builtin_memcpy(&w, in, 16);
        *(uint4 *)p = w;
    } else {
        uint4 a, b;
        __builtin_memcpy(&a, in, 16);
        __builtin_memcpy(&b, (const char *)in + 16, 16);
        ((uint4 *)p)[0] = a;
        ((uint4 *)p)[1] = b;
    }
}

__device__ __forceinline__ void store_row_labels(int *lab, int rowBase, u64 bits, int val) {
    while (bits) {
        const int x = __ffsll(bits) - 1;
        bits &= bits - 1;
        lab[rowBase + x] = val;
    }
}

}  // namespace

size_t discharge_wave_bytes(int V, int K, int nring, int mode) {
    // mode 2: 8-bit residuals, 16-bit excess; 1: 16-bit residuals; 0: 32-bit
    return wave_layout(V, K, nring, mode == 2 ? 1 : (mode == 1 ? 2 : 4), mode == 2 ? 2 : 4).total;
}

template <int K, typename RT, typename ET>
__global__ __launch_bounds__(64) void k_discharge_wave(DischargeArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ long long s_tr[4];
    __shared__ u64 seedRows[64];
    if (*A.actIn == 0ull) return;
    const int stageCap = stage_cap(A);
    const Geo &G = A.G;
    const int V = G.V, N = G.N, nring = A.nring;
    const int TX = G.tx, TY = G.ty;
    const int lane = threadIdx.x;
    const int y = lane;  // the row this lane owns (idle lanes: y >= TY)
    seedRows[lane] = 0ull;
    const WaveLayout L = wave_layout(V, K, nring, (int)sizeof(RT), (int)sizeof(ET));
    RT *resL = (RT *)(smem + L.res);
    ET *exL = (ET *)(smem + L.ex);
    RT *rtL = (RT *)(smem + L.rt);
    int *halo = (int *)(smem + L.halo);
    int *pushL = (int *)(smem + L.push);
    u64 *resM = (u64 *)(smem + L.resM);
    u64 *admM = (u64 *)(smem + L.admM);
    u64 *rtRows = (u64 *)(smem + L.rows);
    u64 *recvRows = rtRows + 64;
    u64 *clrRows = rtRows + 128;
    unsigned short *wl = (unsigned short *)(smem + L.list);
    const int dinf = A.dinf;
    const u64 rowmask = TX == 64 ? ~0ull : ((1ull << TX) - 1);
    const bool myrow = y < TY;
    // 2D grids only: the canonical direction offsets, constants after unrolling
    int dy[K], dx[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        dy[k] = off2d_dy(k);
        dx[k] = off2d_dx(k);
    }
    // arcs of direction k that stay inside the tile, as a row mask of this lane
    u64 inside[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        const bool rowok = myrow && y + dy[k] >= 0 && y + dy[k] < TY;
        u64 m = rowok ? rowmask : 0ull;
        if (dx[k] > 0) m &= rowmask >> dx[k];
        if (dx[k] < 0) m &= (rowmask << (-dx[k])) & rowmask;
        inside[k] = m;
    }
    // border vertices of this lane: i = lane + 64 j (at most 4 * 64 >= 4 * 63 for 64 x 64 tiles)
    const int nslot = (nring + 63) / 64;
    int slotL[4], slotY[4], slotX[4];  // local index, row and column (0 for no slot)
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int i = lane + 64 * j;
        slotL[j] = (j < nslot && i < nring) ? A.ringL[i] : -1;
        const int l = slotL[j] >= 0 ? slotL[j] : 0;
        slotY[j] = l / TX;
        slotX[j] = l - slotY[j] * TX;
    }

    for (;;) {
        int r = 0;
        if (lane == 0) {
            unsigned i = atomicAdd(A.qhead, 1u);
            r = (i < (unsigned)A.nwork) ? A.order[i] : -1;
        }
        r = __shfl(r, 0, 64);
        if (r < 0) return;
        const int base = r * V;
        int active = 0;
        if (lane == 0) {
            active = A.ractive[r];
            // a deferred region keeps its flag and is discharged in a later sweep;
            // with deferRelabel it runs its region relabel now (active 2)
            if (active && A.defer && A.defer[r]) {
                active = A.deferRelabel ? 2 : 0;
                if (!active && A.actCarry) atomicAdd(A.actCarry, 1ull);  // still active
            } else {
                A.ractive[r] = 0;
            }
        }
        active = __shfl(active, 0, 64);
        if (!active) {
            // border labels only: the interior is recomputed by the next discharge
            if (A.labNew != A.labOld)
                for (int i = lane; i < A.nring; i += 64) {
                    const int l = A.ringL[i];
                    A.labNew[base + l] = A.labOld[base + l];
                }
            continue;
        }
        const long long t_start = wall_clock64();
        if (lane < 4) s_tr[lane] = 0;
        // ---------------- stage the region into LDS ----------------
        for (int l = lane; l < V; l += 64) {
            RT rv[K];
#pragma unroll
            for (int k = 0; k < K; k++) rv[k] = (RT)A.res[(size_t)k * N + base + l];
            store_res_row<K, RT>(resL + l * K, rv);
            exL[l] = (ET)A.ex[base + l];
            rtL[l] = (RT)A.rt[base + l];
        }
        if (lane == 0) exL[V] = 0;  // pad of the last packed word
        for (int i = lane; i < nring; i += 64) {
            const int l = A.ringL[i];
            const unsigned m = A.ringM[i];
            int lz, ly, lx;
            local_xyz(G, l, lz, ly, lx);
#pragma unroll
            for (int k = 0; k < K; k++) {
                int h = kInf;
                if ((m >> k) & 1u) {
                    int w = cross_nbr(G, r, lz, ly, lx, k);
                    if (w >= 0) h = A.labOld[w];
                }
                halo[i * K + k] = h;
                pushL[i * K + k] = 0;
            }
        }
        __syncthreads();
        // ---------------- row masks from LDS (coalesced, by ballot), once per discharge ----------------
        u64 EXm = 0;
        {
            u64 Rk[K], RTm = 0;
#pragma unroll
            for (int k = 0; k < K; k++) Rk[k] = 0;
            for (int row = 0; row < TY; row++) {
                const int l = row * TX + lane;
                const bool ok = lane < TX;
                RT rv[K];
#pragma unroll
                for (int k = 0; k < K; k++) rv[k] = 0;
                if (ok) load_res_row<K, RT>(resL + l * K, rv);
#pragma unroll
                for (int k = 0; k < K; k++) {
                    const u64 b = __ballot(rv[k] > 0);
                    if (lane == row) Rk[k] = b;
                }
                const u64 bt = __ballot(ok && rtL[l] > 0);
                const u64 be = __ballot(ok && ex_get(exL, l) > 0);
                if (lane == row) { RTm = bt; EXm = be; }
            }
#pragma unroll
            for (int k = 0; k < K; k++) resM[k * 64 + lane] = Rk[k] & inside[k];
            rtRows[lane] = myrow ? RTm : 0ull;
            recvRows[lane] = 0ull;
            clrRows[lane] = 0ull;
        }
        lane_sync();

        int iter = 0;
        long long levels = 0, stages = 0, pushIters = 0, t_search = 0, t_push = 0;
        const bool relabelOnly = active == 2;
        bool writeMode = relabelOnly;
        const int rowBase = base + y * TX;
        // Vertices a complete search did not reach cannot reach a target for the
        // rest of the discharge (pushes only add residual arcs between reached
        // vertices), so later push-round searches stop once every excess vertex
        // outside this set is labelled; only the final search must be complete.
        u64 dead = 0ull;
        for (;;) {
            const long long t_round = wall_clock64();
            // ---------------- multi-level search from the targets ----------------
            u64 R[K], adm[K];
#pragma unroll
            for (int k = 0; k < K; k++) {
                R[k] = resM[k * 64 + lane];
                adm[k] = 0ull;
            }
            const u64 RT0 = rtRows[lane];
            u64 VIS = RT0, F = RT0;
            const u64 admT = RT0;
            unsigned admB = 0u;  // border slot j: bit K j + k, boundary arc k to push over
            // stage candidate of each border slot: smallest d(w) + 1 over its residual boundary arcs
            int slotC[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                int c = kInf;
                const int l = slotL[j];
                if (l >= 0) {
                    const int i = lane + 64 * j;
                    RT rv[K];
                    load_res_row<K, RT>(resL + l * K, rv);
#pragma unroll
                    for (int k = 0; k < K; k++) {
                        const int h = halo[i * K + k];
                        if (h < dinf && rv[k] > 0) c = min(c, h + 1);
                    }
                }
                slotC[j] = c;
            }
            if (writeMode && myrow) store_row_labels(A.labNew, rowBase, F, 0);
            int stage = 0;
            bool early = false;  // stopped with every live excess vertex labelled
            for (;;) {
                // flood: u unvisited with a residual arc (u, u + o_k) into the frontier
                for (;;) {
                    if (!writeMode && __ballot((EXm & ~VIS & ~dead) != 0ull) == 0ull) {
                        early = true;
                        break;
                    }
                    const Rows3 FR = rows3(F, y, TY);
                    u64 t[K], nw = 0ull;
#pragma unroll
                    for (int k = 0; k < K; k++) {
                        t[k] = R[k] & shift_dx(FR.at(dy[k]), dx[k]);
                        nw |= t[k];
                    }
                    nw &= ~VIS;
                    if (!__ballot(nw != 0ull)) break;
                    levels++;
#pragma unroll
                    for (int k = 0; k < K; k++) adm[k] |= nw & t[k];
                    VIS |= nw;
                    F = nw;
                    if (writeMode && nw) store_row_labels(A.labNew, rowBase, nw, stage);
                }
                if (early) break;
                // next stage: smallest candidate over unvisited border vertices
                int best = kInf;
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    if (j >= nslot) break;
                    const int ry = slotY[j], rx = slotX[j];
                    const u64 vrow = shfl64(VIS, ry);
                    if (slotC[j] != kInf) {
                        if ((vrow >> rx) & 1ull) slotC[j] = kInf;  // labelled in this search
                        else best = min(best, slotC[j]);
                    }
                }
                const int level = wave_min_int(best);
                // partial discharge: stages above the cap wait for later sweeps
                if (level == kInf || (level > stageCap && !writeMode)) break;
                stages++;
                stage = level;
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    if (j >= nslot) break;
                    if (slotC[j] != level) continue;
                    const int l = slotL[j];
                    const int i = lane + 64 * j;
                    const int ry = slotY[j], rx = slotX[j];
                    unsigned match = 0u;
                    RT rv[K];
                    load_res_row<K, RT>(resL + l * K, rv);
#pragma unroll
                    for (int k = 0; k < K; k++) {
                        const int h = halo[i * K + k];
                        if (h < dinf && h + 1 == level && rv[k] > 0) match |= 1u << k;
                    }
                    admB |= match << (K * j);
                    slotC[j] = kInf;
                    atomicOr(&seedRows[ry], 1ull << rx);
                }
                lane_sync();
                u64 seed = seedRows[lane];
                seedRows[lane] = 0ull;
                lane_sync();
                seed &= ~VIS;
                VIS |= seed;
                F = seed;
                if (writeMode && seed) store_row_labels(A.labNew, rowBase, seed, level);
            }
            const long long t_mid = wall_clock64();
            t_search += t_mid - t_round;
            // a search that ended by itself (under the same stage cap) leaves the dead set
            if (!early && !writeMode) dead = ~VIS & rowmask;
            const bool found = __ballot((EXm & VIS) != 0ull) != 0ull;
            if (writeMode) {
                if (myrow) store_row_labels(A.labNew, rowBase, ~VIS & rowmask, dinf);
                // excess left beyond the stage cap: the region stays active
                if (found && A.actCarry && lane == 0) {
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
                if (lane == 0) atomicOr(A.err, 4);
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
#pragma unroll
            for (int k = 0; k < K; k++) admM[k * 64 + lane] = adm[k];
            admM[K * 64 + lane] = admT;
            u64 canPush = admT;
#pragma unroll
            for (int k = 0; k < K; k++) canPush |= adm[k];
            lane_sync();
            for (;;) {
                int pushed = 0;
                // push from excess vertex u (row uy, column ux) along its admissible arcs
                auto push_from = [&](int u, int uy, int ux) {
                    const u64 bit = 1ull << ux;
                    u64 am[K + 1];
#pragma unroll
                    for (int k = 0; k <= K; k++) am[k] = admM[k * 64 + uy];
                    const int e = ex_get(exL, u);
                    if (e <= 0) {
                        // a receipt in this iteration sets the bit again at the merge
                        atomicOr(&clrRows[uy], bit);
                        return;
                    }
                    int rem = e;
                    if (am[K] & bit) {
                        const int c = rtL[u];
                        const int d = min(rem, c);
                        if (d > 0) {
                            rtL[u] = (RT)(c - d);
                            rem -= d;
                            if (A.trace) atomicAdd((unsigned long long *)&s_tr[1], (u64)d);
                        }
                        if (c == d) {
                            atomicAnd(&admM[K * 64 + uy], ~bit);
                            atomicAnd(&rtRows[uy], ~bit);
                        }
                    }
                    // the residuals of u only fall through u's own pushes (an
                    // admissible arc is never pushed from both ends), so one
                    // vector load of all K is as good as K separate ones
                    RT rv[K];
                    load_res_row<K, RT>(resL + u * K, rv);
                    int c[K];
#pragma unroll
                    for (int k = 0; k < K; k++) c[k] = (am[k] & bit) ? (int)rv[k] : 0;
#pragma unroll
                    for (int k = 0; k < K; k++) {
                        if (rem <= 0 || !(am[k] & bit)) continue;
                        const int d = min(rem, c[k]);
                        if (d > 0) {
                            const int v = u + dy[k] * TX + dx[k];
                            const u64 vbit = 1ull << (ux + dx[k]);
                            resL[u * K + k] = (RT)(c[k] - d);
                            res_add(resL, v * K + (k ^ 1), d);
                            ex_add(exL, v, d);
                            atomicOr(&resM[(k ^ 1) * 64 + uy + dy[k]], vbit);
                            atomicOr(&recvRows[uy + dy[k]], vbit);
                            rem -= d;
                        }
                        if (c[k] == d) {
                            atomicAnd(&admM[k * 64 + uy], ~bit);
                            atomicAnd(&resM[k * 64 + uy], ~bit);
                        }
                    }
                    if (rem < e) {
                        // drained what it saw: cleared, unless a receipt in this
                        // iteration sets the bit again at the merge
                        ex_add(exL, u, rem - e);
                        if (rem == 0) atomicOr(&clrRows[uy], bit);
                        pushed = 1;
                    }
                };
                const u64 P = EXm & canPush;
                const int cnt = __popcll(P);
                if (__ballot(cnt > 2) == 0ull) {
                    // light iteration: every lane pushes from its own row
                    u64 m = P;
                    while (m) {
                        const int x = __ffsll(m) - 1;
                        m &= m - 1;
                        push_from(y * TX + x, y, x);
                    }
                } else {
                    // the excess vertices of all rows, spread over the lanes by a work list
                    // (the list has room for every vertex of the tile: one pass)
                    const int incl = wave_scan_incl(cnt, lane);
                    const int total = __builtin_amdgcn_readlane(incl, 63);
                    int idx = incl - cnt;
                    u64 m = P;
                    while (m) {
                        const int x = __ffsll(m) - 1;
                        m &= m - 1;
                        wl[idx++] = (unsigned short)((y << 6) | x);  // row and column (TX <= 64)
                    }
                    lane_sync();
                    for (int it = lane; it < total; it += 64) {
                        const int w = wl[it];
                        const int uy = w >> 6, ux = w & 63;
                        push_from(uy * TX + ux, uy, ux);
                    }
                    lane_sync();
                }
                // first-level vertices of stages k > 0 push over boundary arcs
                if (admB) {
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const unsigned ab = (admB >> (K * j)) & ((1u << K) - 1u);
                        if (!ab) continue;
                        const int l = slotL[j];
                        const int i = lane + 64 * j;
                        const int ly = slotY[j], lx = slotX[j];
                        const u64 bit = 1ull << lx;
                        const int e = ex_get(exL, l);
                        if (e <= 0) {
                            atomicOr(&clrRows[ly], bit);
                            continue;
                        }
                        int rem = e;
                        RT rv[K];
                        load_res_row<K, RT>(resL + l * K, rv);
#pragma unroll
                        for (int k = 0; k < K; k++) {
                            if (!((ab >> k) & 1u) || rem <= 0) continue;
                            const int c = rv[k];
                            const int d = min(rem, c);
                            if (d > 0) {
                                resL[l * K + k] = (RT)(c - d);
                                pushL[i * K + k] += d;
                                rem -= d;
                                if (A.trace) atomicAdd((unsigned long long *)&s_tr[2], (u64)d);
                            }
                            if (c == d) admB &= ~(1u << (K * j + k));
                        }
                        if (rem < e) {
                            const int D = e - rem;
                            if (ex_sub(exL, l, D) == D) atomicOr(&clrRows[ly], bit);
                            pushed = 1;
                        }
                    }
                }
                lane_sync();
                const bool any = __ballot(pushed != 0) != 0ull;
                pushIters++;
                EXm = (EXm & ~clrRows[lane]) | recvRows[lane];
                clrRows[lane] = 0ull;
                recvRows[lane] = 0ull;
                canPush = admM[K * 64 + lane];
#pragma unroll
                for (int k = 0; k < K; k++) canPush |= admM[k * 64 + lane];
                lane_sync();
                if (!any) break;
            }
            t_push += wall_clock64() - t_mid;
            // no excess left in the region (the masks may only over-report it):
            // the next search cannot find an excess vertex, so it writes the labels
            if (__ballot(EXm != 0ull) == 0ull) writeMode = true;
        }
        __syncthreads();
        // ---------------- write the region back ----------------
        for (int l = lane; l < V; l += 64) {
            RT rv[K];
            load_res_row<K, RT>(resL + l * K, rv);
#pragma unroll
            for (int k = 0; k < K; k++) A.res[(size_t)k * N + base + l] = rv[k];
            A.ex[base + l] = ex_get(exL, l);
            A.rt[base + l] = rtL[l];
        }
        for (int i = lane; i < nring; i += 64) {
            const int l = A.ringL[i];
#pragma unroll
            for (int k = 0; k < K; k++) {
                const int p = pushL[i * K + k];
                if (p) A.pushb[(size_t)k * N + base + l] = p;
            }
        }
        if (A.trace) {
            long long ex_out = 0, lsum = 0;
            for (int l = lane; l < V; l += 64) ex_out += ex_get(exL, l);
            for (int i = lane; i < nring; i += 64) lsum += min(A.labNew[base + A.ringL[i]], 65535);
            atomicAdd((unsigned long long *)&s_tr[0], (u64)ex_out);
            atomicAdd((unsigned long long *)&s_tr[3], (u64)lsum);
        }
        __syncthreads();
        if (lane == 0 && relabelOnly) {
            atomicAdd(&A.stats[11], 1ull);
        } else if (lane == 0) {
            atomicAdd(&A.stats[0], 1ull);
            if (A.regionTicks) A.regionTicks[r] = (int)min(wall_clock64() - t_start, 0x7fffffffLL);
            atomicAdd(&A.stats[1], (u64)A.rvcount[r]);
            atomicAdd(&A.stats[2], (u64)(iter + 1));
            atomicAdd(&A.stats[3], (u64)levels);
            atomicAdd(&A.stats[4], (u64)stages);
            atomicAdd(&A.stats[6], (u64)t_search);
            atomicAdd(&A.stats[7], (u64)t_push);
            atomicAdd(&A.stats[10], (u64)pushIters);
            if (A.trace) {
                unsigned long long idx = atomicAdd(&A.stats[5], 1ull);
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

#define MF_WAVE_KERNELS(X) \
    X(4, unsigned char, short) X(8, unsigned char, short) X(4, short, int) X(8, short, int) \
    X(4, int, int) X(8, int, int)

void set_wave_attributes() {
#define MF_SET(K, RT, ET)                                                                        \
    (void)hipFuncSetAttribute((const void *)k_discharge_wave<K, RT, ET>,                         \
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    MF_WAVE_KERNELS(MF_SET)
#undef MF_SET
    (void)hipGetLastError();
}

template <int K, typename RT, typename ET>
static hipError_t launch_wave_t(const DischargeArgs &A, int blocks, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_discharge_wave<K, RT, ET>), dim3(blocks), dim3(64), lds, s, A);
    return hipGetLastError();
}

hipError_t launch_discharge_wave(const DischargeArgs &A, int blocks, size_t lds, int mode,
                                 hipStream_t s) {
    const int K = A.G.K;
    if (A.G.tz != 1 || A.G.tx > 64 || A.G.ty > 64 || A.nring > 4 * 64) return hipErrorInvalidValue;
    if (mode == 2) {
        if (K == 4) return launch_wave_t<4, unsigned char, short>(A, blocks, lds, s);
        if (K == 8) return launch_wave_t<8, unsigned char, short>(A, blocks, lds, s);
    } else if (mode == 1) {
        if (K == 4) return launch_wave_t<4, short, int>(A, blocks, lds, s);
        if (K == 8) return launch_wave_t<8, short, int>(A, blocks, lds, s);
    } else {
        if (K == 4) return launch_wave_t<4, int, int>(A, blocks, lds, s);
        if (K == 8) return launch_wave_t<8, int, int>(A, blocks, lds, s);
    }
    return hipErrorInvalidValue;
}

// Global relabel, one distance level (see k_grelabel in mf_kernels.hip), for
// 2D regions of at most 64 x 64 with the row-bitmask flood of one wavefront.
// At level 0 the residual-arc masks are built from HBM by ballot and kept in a
// per-region cache with the mask of unlabelled vertices; later levels read the
// cache and take their seeds from the border vertices marked by the previous
// level.  The flood runs in registers; labels and next-level marks are written
// back.
template <int K>
__global__ __launch_bounds__(64) void k_grelabel_wave(GRelabelArgs A) {
    __shared__ u64 seedRows[64];
    const Geo &G = A.G;
    const int V = G.V, N = G.N, TX = G.tx, TY = G.ty, D = A.level, dinf = A.dinf;
    const int lane = threadIdx.x, y = lane;
    const bool myrow = y < TY;
    const u64 rowmask = TX == 64 ? ~0ull : ((1ull << TX) - 1);
    seedRows[lane] = 0ull;
    // 2D grids only: the canonical direction offsets, constants after unrolling
    int dy[K], dx[K];
    u64 inside[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        dy[k] = off2d_dy(k);
        dx[k] = off2d_dx(k);
        const bool rowok = myrow && y + dy[k] >= 0 && y + dy[k] < TY;
        u64 m = rowok ? rowmask : 0ull;
        if (dx[k] > 0) m &= rowmask >> dx[k];
        if (dx[k] < 0) m &= (rowmask << (-dx[k])) & rowmask;
        inside[k] = m;
    }
    // border vertices of this lane: i = lane + 64 j (a tile of at most 64 x 64
    // has at most 252), with their rows and columns
    int slotL[4], slotY[4], slotX[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int i = lane + 64 * j;
        slotL[j] = i < A.nring ? A.ringL[i] : -1;
        const int l = slotL[j] >= 0 ? slotL[j] : 0;
        slotY[j] = l / TX;
        slotX[j] = l - slotY[j] * TX;
    }
    for (int r = blockIdx.x; r < G.nreg; r += gridDim.x) {
        int go = 1;
        if (D > 0) {
            if (lane == 0) {
                go = A.flagIn[r];
                A.flagIn[r] = 0;
            }
            go = __shfl(go, 0, 64);
        }
        if (!go) continue;
        const int base = r * V;
        u64 *cr = (u64 *)A.cache + (size_t)r * (K + 1) * 64;
        u64 R[K], U = 0, SEED = 0;
        if (D == 0) {
            // four rows of loads in flight at a time (addresses clamped, not predicated)
            for (int row0 = 0; row0 < TY; row0 += 4) {
                int v[4][K + 1];
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const bool ok = lane < TX && row0 + j < TY;
                    const int l = ok ? (row0 + j) * TX + lane : 0;
#pragma unroll
                    for (int k = 0; k < K; k++) v[j][k] = A.res[(size_t)k * N + base + l];
                    v[j][K] = A.rt[base + l];
                }
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const int row = row0 + j;
                    const bool ok = lane < TX && row < TY;
#pragma unroll
                    for (int k = 0; k < K; k++) {
                        const u64 b = __ballot(ok && v[j][k] > 0);
                        if (lane == row) R[k] = b;
                    }
                    const u64 bs = __ballot(ok && v[j][K] > 0);
                    if (lane == row) SEED = bs;
                }
            }
            U = myrow ? rowmask : 0ull;  // every label is d_inf when a relabel starts
#pragma unroll
            for (int k = 0; k < K; k++) {
                R[k] &= inside[k];
                cr[k * 64 + lane] = R[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < K; k++) R[k] = cr[k * 64 + lane];
            U = cr[K * 64 + lane];
            // seeds: border vertices marked by the previous level
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int l = slotL[j];
                if (l >= 0 && A.candIn[base + l]) {
                    A.candIn[base + l] = 0;
                    atomicOr(&seedRows[slotY[j]], 1ull << slotX[j]);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            SEED = seedRows[lane] & U;
            seedRows[lane] = 0ull;
        }
        u64 reached = SEED, F = SEED;
        for (;;) {
            const Rows3 FR = rows3(F, y, TY);
            u64 nw = 0;
#pragma unroll
            for (int k = 0; k < K; k++) nw |= R[k] & shift_dx(FR.at(dy[k]), dx[k]);
            nw &= U & ~reached;
            if (!__ballot(nw != 0ull)) break;
            reached |= nw;
            F = nw;
        }
        if (myrow && reached) {
            store_row_labels(A.lab, base + y * TX, reached, D);
            cr[K * 64 + lane] = U & ~reached;
        } else if (D == 0) {
            cr[K * 64 + lane] = U;
        }
        // marks for D + 1: residual predecessors across the border of reached border vertices
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (64 * j >= A.nring) break;  // uniform: every lane takes part in the row exchange
            const int i = lane + 64 * j;
            const int ry = slotY[j], rx = slotX[j];
            const u64 m = shfl64(reached, ry);
            if (slotL[j] >= 0 && ((m >> rx) & 1ull)) {
                const unsigned lm = A.ringM[i];
#pragma unroll
                for (int k = 0; k < K; k++) {
                    // predecessor u = v - o_k lies across the border when direction k^1 leaves
                    if (!((lm >> (k ^ 1)) & 1u)) continue;
                    const int ug = cross_nbr(G, r, 0, ry, rx, k ^ 1);
                    if (ug < 0 || A.res[(size_t)k * N + ug] <= 0 || A.lab[ug] != dinf) continue;
                    A.candOut[ug] = 1;
                    if (atomicExch(&A.flagOut[ug / V], 1) == 0) atomicAdd(A.flagged, 1u);
                }
            }
        }
    }
}

// Residual reachability for the cuts (the region floods of k_flood, same
// marks) on 2D tiles of at most 64 x 64: one wavefront per region, lane y holds
// row y as 64-bit masks.  dir 0 floods forward from the excess vertices along
// arcs with c_f > 0 (the masks hold, at the head w of each arc, whether the arc
// w - o_k -> w is residual), dir 1 backward from t.  Reached border vertices
// mark their neighbours across the border (atomic exchange, as k_flood) and
// flag the neighbouring region for the next round.
template <int K>
__global__ __launch_bounds__(64) void k_flood_wave(FloodArgs A) {
    const Geo &G = A.G;
    const int V = G.V, N = G.N, TX = G.tx, TY = G.ty;
    const int lane = threadIdx.x, y = lane;
    const bool myrow = y < TY;
    const u64 rowmask = TX == 64 ? ~0ull : ((1ull << TX) - 1);
    // 2D grids only: the canonical direction offsets, constants after unrolling
    int dy[K], dx[K];
    u64 inside[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        dy[k] = off2d_dy(k);
        dx[k] = off2d_dx(k);
        const bool rowok = myrow && y + dy[k] >= 0 && y + dy[k] < TY;
        u64 m = rowok ? rowmask : 0ull;
        if (dx[k] > 0) m &= rowmask >> dx[k];
        if (dx[k] < 0) m &= (rowmask << (-dx[k])) & rowmask;
        inside[k] = m;
    }
    int slotL[4], slotY[4], slotX[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int i = lane + 64 * j;
        slotL[j] = i < A.nring ? A.ringL[i] : -1;
        const int l = slotL[j] >= 0 ? slotL[j] : 0;
        slotY[j] = l / TX;
        slotX[j] = l - slotY[j] * TX;
    }
    for (int r = blockIdx.x; r < G.nreg; r += gridDim.x) {
        int go = 1;
        if (lane == 0) {
            go = (A.round == 0) ? 1 : A.dirtyIn[r];
            A.dirtyIn[r] = 0;
        }
        go = __shfl(go, 0, 64);
        if (!go) continue;
        const int base = r * V;
        // row masks: residual arcs inside the tile, the marks already stored
        // (M0) and with the round-0 seeds (M)
        u64 R[K], M = 0, M0 = 0;
#pragma unroll
        for (int k = 0; k < K; k++) R[k] = 0;
        // four rows of loads in flight at a time (addresses clamped, not predicated)
        const int *seedPlane = A.dir == 0 ? A.ex : A.rt;
        for (int row0 = 0; row0 < TY; row0 += 4) {
            int v[4][K + 2];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const bool ok = lane < TX && row0 + j < TY;
                const int l = ok ? (row0 + j) * TX + lane : 0;
#pragma unroll
                for (int k = 0; k < K; k++) v[j][k] = A.res[(size_t)k * N + base + l];
                v[j][K] = A.mark[base + l];
                v[j][K + 1] = A.round == 0 ? seedPlane[base + l] : 0;
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int row = row0 + j;
                const bool ok = lane < TX && row < TY;
#pragma unroll
                for (int k = 0; k < K; k++) {
                    const u64 b = __ballot(ok && v[j][k] > 0);
                    if (lane == row) R[k] = b;
                }
                const bool m0 = ok && v[j][K] != 0;
                const bool sd = ok && v[j][K + 1] > 0;
                const u64 b0 = __ballot(m0), bm = __ballot(m0 || sd);
                if (lane == row) {
                    M0 = b0;
                    M = bm;
                }
            }
        }
        u64 Rf[K];  // the arcs the flood follows, at the vertex it reaches
#pragma unroll
        for (int k = 0; k < K; k++) {
            R[k] &= inside[k];
            // forward: w is reached over w - o_k -> w, residual at row y - dy, column x - dx
            Rf[k] = A.dir == 0 ? (shift_dx(rows3(R[k], y, TY).at(-dy[k]), -dx[k]) & (myrow ? rowmask : 0ull))
                               : R[k];
        }
        u64 reached = myrow ? M : 0ull, F = reached;
        for (;;) {
            const Rows3 FR = rows3(F, y, TY);
            u64 nw = 0;
#pragma unroll
            for (int k = 0; k < K; k++) {
                const int sy = A.dir == 0 ? -dy[k] : dy[k], sx = A.dir == 0 ? -dx[k] : dx[k];
                nw |= Rf[k] & shift_dx(FR.at(sy), sx);
            }
            nw &= ~reached;
            if (!__ballot(nw != 0ull)) break;
            reached |= nw;
            F = nw;
        }
        // marks of this round, seeds included (stores of 1 race harmlessly with
        // the neighbours' exchanges)
        if (myrow) {
            u64 nb = reached & ~M0;
            const int rowBase = base + y * TX;
            while (nb) {
                const int x = __ffsll(nb) - 1;
                nb &= nb - 1;
                A.mark[rowBase + x] = 1;
            }
        }
        // across the border
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (64 * j >= A.nring) break;  // uniform: every lane takes part in the row exchange
            const int i = lane + 64 * j;
            const int ry = slotY[j], rx = slotX[j];
            const u64 m = shfl64(reached, ry);
            if (slotL[j] < 0 || !((m >> rx) & 1ull)) continue;
            const unsigned lm = A.ringM[i];
            const int v = slotL[j];
#pragma unroll
            for (int k = 0; k < K; k++) {
                if (A.dir == 0) {
                    // forward: arc (v, v + o_k) with c_f > 0 that leaves the tile
                    if (!((lm >> k) & 1u) || A.res[(size_t)k * N + base + v] <= 0) continue;
                    const int wg = cross_nbr(G, r, 0, ry, rx, k);
                    if (wg >= 0 && atomicExch(&A.mark[wg], 1) == 0) {
                        A.dirtyOut[wg / V] = 1;
                        atomicAdd(A.changed, 1u);
                    }
                } else {
                    // backward: u = v - o_k across the border with c_f(u, v) > 0
                    if (!((lm >> (k ^ 1)) & 1u)) continue;
                    const int wg = cross_nbr(G, r, 0, ry, rx, k ^ 1);
                    if (wg >= 0 && A.res[(size_t)k * N + wg] > 0 && atomicExch(&A.mark[wg], 1) == 0) {
                        A.dirtyOut[wg / V] = 1;
                        atomicAdd(A.changed, 1u);
                    }
                }
            }
        }
    }
}

hipError_t launch_flood_wave(const FloodArgs &A, int blocks, hipStream_t s) {
    if (A.G.tz != 1 || A.G.tx > 64 || A.G.ty > 64 || A.nring > 256) return hipErrorInvalidValue;
    if (A.G.K == 4) hipLaunchKernelGGL(k_flood_wave<4>, dim3(blocks), dim3(64), 0, s, A);
    else if (A.G.K == 8) hipLaunchKernelGGL(k_flood_wave<8>, dim3(blocks), dim3(64), 0, s, A);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_grelabel_wave(const GRelabelArgs &A, int blocks, hipStream_t s) {
    if (A.G.tz != 1 || A.G.tx > 64 || A.G.ty > 64) return hipErrorInvalidValue;
    if (A.G.K == 4) hipLaunchKernelGGL(k_grelabel_wave<4>, dim3(blocks), dim3(64), 0, s, A);
    else if (A.G.K == 8) hipLaunchKernelGGL(k_grelabel_wave<8>, dim3(blocks), dim3(64), 0, s, A);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace mfd
