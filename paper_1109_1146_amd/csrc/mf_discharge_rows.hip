// Workgroup row-bitmask region discharge for 3D 6-connected regions whose rows
// along x are 32 vertices long and which have at most 1024 rows (Proc. ARD of
// Sec. 4.2 with the region relabel of Alg. 3; same method as k_discharge,
// different execution).
//
// One 1024-thread workgroup owns a region; each thread owns one row (y, z) of
// 32 vertices as 32-bit masks in registers: residual arc present in each of the
// six directions, visited, frontier, and the arcs by which the search reached
// each vertex (its admissible arcs).  The integer state (residuals, t-links,
// excess, boundary pushes) stays in HBM.  LDS holds the exact residual-arc and
// t-link masks of the region, the admissible-arc masks of the current round, the
// frontier rows a search level exchanges between neighbouring rows, the rows of
// vertices whose excess changed in a push iteration, the halo labels d(w) and
// the stage candidates of the border vertices, and per-wave work lists.
//
// * Search: the multi-level breadth-first search from the targets (stage 0
//   from t, then one stage per distinct d(w) + 1 over residual boundary arcs)
//   advances one level per workgroup barrier: a level is a few shifts and ANDs
//   of a row with the frontier rows y +- 1 and z +- 1.  A vertex keeps the arcs
//   that led it to the previous level; they point exactly one level down.
// * Push: every excess vertex pushes along its admissible arcs, into t for the
//   vertices of stage 0 and over boundary arcs for the first-level vertices of a
//   stage k > 0 (to w with d(w) + 1 = k).  All vertices push in parallel, one
//   iteration per barrier, until no push is possible; arcs only go down the
//   (stage, level) order, so an arc is changed by one side only.  The excess
//   vertices of a wave's rows are spread over its 64 lanes through a list in
//   LDS, and for 32 x 32 rows each wave owns a diagonal of (y, z), so that a
//   front of excess on a y or z plane is shared by all waves.
// * Search and push alternate until no excess vertex reaches a target.  The
//   last search is run once more to write the labels (Alg. 3).
#include "mf_device.h"
#include "mf_launch.h"

namespace mfd {

typedef unsigned long long u64;

namespace {

constexpr int kRowsNT = 1024;
constexpr int kRowsWaves = kRowsNT / 64;

constexpr int kListCap = 256;  // work-list entries per wave and pass

struct RowsLayout {
    size_t resM, F, vis, recv, clr, adm, rtm, halo, slotC, slotL, list, total;  // offsets in 32-bit words
};

// Halo labels d(w) of the boundary arcs, one array per tile face: faces -+x
// are indexed by the row (y + ty z), faces -+y by x + 32 z, faces -+z by x + 32 y.
__host__ __device__ inline int face_size(int k, int TY, int TZ) {
    return k < 2 ? TY * TZ : (k < 4 ? 32 * TZ : 32 * TY);
}

__host__ __device__ inline RowsLayout rows_layout(int R, int TY, int TZ, int nring) {
    RowsLayout L;
    size_t o = 0;
    L.resM = o; o += 6 * (size_t)R;  // residual arc (u, u + o_k) > 0, per direction
    L.F = o; o += 2 * (size_t)R;     // frontier rows, two buffers by level parity
    L.vis = o; o += (size_t)R;       // visited rows (read by the border owners)
    L.recv = o; o += 2 * (size_t)R;  // vertices that received excess, by iteration parity
    L.clr = o; o += 2 * (size_t)R;   // vertices whose excess dropped to zero
    L.adm = o; o += 7 * (size_t)R;   // admissible arcs of the round: six directions, then t
    L.rtm = o; o += (size_t)R;       // residual t-link > 0
    L.halo = o;
    for (int k = 0; k < 6; k++) o += face_size(k, TY, TZ);
    L.slotC = o; o += (size_t)nring;            // stage candidate of each border vertex
    L.slotL = o; o += ((size_t)nring + 1) / 2;  // its local index (16 bit)
    L.list = o; o += (size_t)kRowsWaves * kListCap / 2;
    L.total = o;
    return L;
}

__device__ __forceinline__ int wave_min_rows(int v) {
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

// Workgroup-wide OR / MIN with one barrier.  The two halves of red[] / anyB[]
// alternate between consecutive calls, so a call never overwrites values that a
// slower wave may still read from the previous one.  The OR keeps one byte per
// wave, read back as one 16-byte word.
static_assert(kRowsWaves == 16, "one byte per wave in a 16-byte word");
__device__ __forceinline__ int block_any(int pred, unsigned char (*anyB)[kRowsWaves], int &rc) {
    const u64 b = __ballot(pred);
    const int p = rc & 1;
    rc++;
    if ((threadIdx.x & 63) == 0) anyB[p][threadIdx.x >> 6] = (b != 0ull) ? 1 : 0;
    __syncthreads();
    const uint4 v = *(const uint4 *)anyB[p];
    return (v.x | v.y | v.z | v.w) != 0u;
}

__device__ __forceinline__ int block_min(int v, int (*red)[kRowsWaves], int &rc) {
    v = wave_min_rows(v);
    const int p = rc & 1;
    rc++;
    if ((threadIdx.x & 63) == 0) red[p][threadIdx.x >> 6] = v;
    __syncthreads();
    int m = kInf;
#pragma unroll
    for (int w = 0; w < kRowsWaves; w++) m = min(m, red[p][w]);
    return m;
}

__device__ __forceinline__ void store_labels(int *lab, size_t rowBase, unsigned bits, int val) {
    while (bits) {
        const int x = __ffs(bits) - 1;
        bits &= bits - 1;
        lab[rowBase + x] = val;
    }
}

}  // namespace

size_t discharge_rows_bytes(int ty, int tz, int nring) {
    return rows_layout(ty * tz, ty, tz, nring).total * sizeof(unsigned);
}

// Position of the boundary arc (l, k) in its face array.
__device__ __forceinline__ int face_pos(int k, int l, int TY) {
    const int x = l & 31, row = l >> 5;
    if (k < 2) return row;
    const int y = row % TY, z = row / TY;
    return k < 4 ? x + 32 * z : x + 32 * y;
}

// Row owned by thread tid.  For 32 x 32 rows, wave w holds the rows with
// (y + z) mod 16 == w (two per z), so the rows of any y or z plane are spread
// over all waves; other shapes use rows in thread order.
__device__ __forceinline__ int row_of(int tid, int TY, int TZ) {
    if (TY == 32 && TZ == 32) {
        const int w = tid >> 6, lane = tid & 63;
        const int z = lane >> 1;
        const int y = ((w - z) & 15) + 16 * (lane & 1);
        return y + 32 * z;
    }
    return tid;
}

// LDS written by one lane of a wave and read by another lane of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Leaving direction of axis a at a border vertex with leaving mask mm: exactly
// one of the two directions of an axis leaves it (tiles are at least 2 wide on
// y and z and 32 on x).
__device__ __forceinline__ int axis_dir_m(unsigned mm, int a) {
    return ((mm >> (2 * a)) & 1u) ? 2 * a : 2 * a + 1;
}

__global__ __launch_bounds__(kRowsNT) void k_discharge_rows(DischargeArgs A) {
    extern __shared__ __align__(16) unsigned smem_rows[];
    __shared__ __align__(16) int red[2][kRowsWaves];
    // flood level flags (bit 0: a frontier, bit 1: a live excess vertex not
    // labelled yet), OR-ed by the waves into one of three words in rotation: the
    // word of level l is read after the level's barrier, and thread 0 clears
    // the word of level l + 2 then (its readers passed this barrier, its
    // writers come after the next one)
    __shared__ int s_flood[3];
    __shared__ __align__(16) unsigned char anyB[2][kRowsWaves];  // block_any bytes
    __shared__ int s_r, s_active;
    __shared__ long long s_tr[4];  // trace: excess out, to sink, to boundary, label sum
    if (*A.actIn == 0ull) return;
    const int stageCap = stage_cap(A);
    const int V = A.G.V, N = A.G.N, TY = A.G.ty, TZ = A.G.tz, R = TY * TZ;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const RowsLayout L = rows_layout(R, TY, TZ, A.nring);
    unsigned *resM = smem_rows + L.resM;
    unsigned *Fb = smem_rows + L.F;
    unsigned *Vb = smem_rows + L.vis;
    unsigned *recvB = smem_rows + L.recv;
    unsigned *clrB = smem_rows + L.clr;
    unsigned *admL = smem_rows + L.adm;
    unsigned *rtmL = smem_rows + L.rtm;
    int *halo = (int *)(smem_rows + L.halo);
    int *slotC = (int *)(smem_rows + L.slotC);
    unsigned short *slotL = (unsigned short *)(smem_rows + L.slotL);
    unsigned short *wlist = (unsigned short *)(smem_rows + L.list) + wid * kListCap;
    int faceOff[6];
    faceOff[0] = 0;
#pragma unroll
    for (int k = 1; k < 6; k++) faceOff[k] = faceOff[k - 1] + face_size(k - 1, TY, TZ);
    const bool myrow = tid < R;
    const int row = myrow ? row_of(tid, TY, TZ) : 0;
    const int y = row % TY, z = row / TY;
    const int dinf = A.dinf;
    const int nring = A.nring;
    int rc = 0;
    int fl = 0;  // flood word of the next level (0, 1, 2 in rotation)
    if (tid < 3) s_flood[tid] = 0;

    // recv and clr are contiguous and return to zero after every use
    for (int i = tid; i < 4 * R; i += kRowsNT) recvB[i] = 0u;

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
                for (int i = tid; i < A.nring; i += kRowsNT) {
                    const int l = A.ringL[i];
                    A.labNew[base + l] = A.labOld[base + l];
                }
            __syncthreads();
            continue;
        }
        const long long t_start = wall_clock64();
        if (tid < 4) s_tr[tid] = 0;

        // ---------------- row masks from HBM (coalesced loads + ballots) ----------------
        // Wave w reads rows 64w .. 64w + 63: load i brings rows 64w + 2i and
        // 64w + 2i + 1 (one 32-bit half of the ballot each).  Residual masks go
        // to resM, the t-link mask to rtm, the excess mask to a frontier buffer.
        {
            const int row0 = wid * 64;
            if (row0 + 64 <= R) {
                for (int q = 0; q < 8; q++) {
                    const int *plane = q < 6 ? A.res + (size_t)q * N : (q == 6 ? A.rt : A.ex);
                    unsigned *dst = q < 6 ? resM + q * R : (q == 6 ? rtmL : Fb);
                    const int *src = plane + base + (size_t)row0 * 32 + lane;
                    // eight loads in flight before their ballots (a load
                    // followed at once by its ballot waits for each in turn)
                    for (int i0 = 0; i0 < 32; i0 += 8) {
                        int v[8];
#pragma unroll
                        for (int i = 0; i < 8; i++) v[i] = src[(i0 + i) * 64];
#pragma unroll
                        for (int i = 0; i < 8; i++) {
                            const u64 b = __ballot(v[i] > 0);
                            if (lane == 0) {
                                dst[row0 + 2 * (i0 + i)] = (unsigned)b;
                                dst[row0 + 2 * (i0 + i) + 1] = (unsigned)(b >> 32);
                            }
                        }
                    }
                }
            }
        }
        // ---------------- border vertices: halo labels into LDS ----------------
        for (int i = tid; i < nring; i += kRowsNT) {
            const int l = A.ringL[i];
            const unsigned mm = A.ringM[i];
            int lz, ly, lx;
            local_xyz(A.G, l, lz, ly, lx);
            for (int k = 0; k < 6; k++) {
                if (!((mm >> k) & 1u)) continue;
                const int w = cross_nbr(A.G, r, lz, ly, lx, k);
                halo[faceOff[k] + face_pos(k, l, TY)] = w >= 0 ? A.labOld[w] : kInf;
            }
            slotL[i] = (unsigned short)l;
        }
        __syncthreads();
        unsigned exM = myrow ? Fb[row] : 0u;

        int iter = 0;
        long long levels = 0, stages = 0, pushIters = 0, t_search = 0, t_flood = 0, t_stage = 0, t_push = 0;
        const bool relabelOnly = s_active == 2;
        bool writeMode = relabelOnly;
        const size_t rowBase = base + (size_t)row * 32;
        // Vertices a complete search did not reach cannot reach a target for the
        // rest of the discharge (pushes only add residual arcs between reached
        // vertices), so later push-round searches stop once every excess vertex
        // outside this set is labelled; only the final search must be complete.
        unsigned dead = 0u;
        for (;;) {
            // ---------------- multi-level search from the targets ----------------
            const long long t0s = wall_clock64();
            unsigned rk[6];
#pragma unroll
            for (int k = 0; k < 6; k++) rk[k] = myrow ? resM[k * R + row] : 0u;
            const unsigned rtM = myrow ? rtmL[row] : 0u;
            unsigned vis = rtM, F = rtM, admT = rtM;
            unsigned adm[6];
#pragma unroll
            for (int k = 0; k < 6; k++) adm[k] = 0u;
            u64 admB = 0ull;  // border slot j (vertex tid + 1024 j), bit 3j + axis: boundary arc to push over
            // stage candidate of each border vertex of this thread: smallest
            // d(w) + 1 over its residual boundary arcs (fixed during a search)
#pragma unroll 4
            for (int i = tid; i < nring; i += kRowsNT) {
                const int l = slotL[i];
                const unsigned mm = A.ringM[i];
                const int rw = l >> 5;
                const unsigned bit = 1u << (l & 31);
                int c = kInf;
                for (int k = 0; k < 6; k++) {
                    if (!((mm >> k) & 1u) || !(resM[k * R + rw] & bit)) continue;
                    const int d = halo[faceOff[k] + face_pos(k, l, TY)];
                    if (d < dinf) c = min(c, d + 1);
                }
                slotC[i] = c;
            }
            int p = 0;
            int stage = 0;
            bool early = false;  // stopped with every live excess vertex labelled
            if (writeMode && myrow) store_labels(A.labNew, rowBase, F, 0);
            for (;;) {
                // flood inside the region: u with c_f(u, u + o_k) > 0 and u + o_k in the frontier
                const long long t0f = wall_clock64();
                for (;;) {
                    if (myrow) {
                        Fb[p * R + row] = F;
                        Vb[row] = vis;
                    }
                    // one barrier; the level's flag word and the neighbour rows
                    // are read in the same LDS round trip
                    {
                        const u64 b = __ballot(F != 0u);
                        const u64 e = __ballot((exM & ~vis & ~dead) != 0u);
                        const int f = ((b != 0ull) ? 1 : 0) | ((e != 0ull) ? 2 : 0);
                        if (lane == 0 && f) atomicOr(&s_flood[fl], f);
                    }
                    __syncthreads();
                    const int any = s_flood[fl];
                    if (tid == 0) s_flood[fl == 0 ? 2 : fl - 1] = 0;  // the word of level l + 2
                    fl = fl == 2 ? 0 : fl + 1;
                    const unsigned *Fp = Fb + p * R;
                    unsigned fyp = 0u, fym = 0u, fzp = 0u, fzm = 0u;
                    if (myrow) {
                        fyp = (y + 1 < TY) ? Fp[row + 1] : 0u;
                        fym = (y > 0) ? Fp[row - 1] : 0u;
                        fzp = (z + 1 < TZ) ? Fp[row + TY] : 0u;
                        fzm = (z > 0) ? Fp[row - TY] : 0u;
                    }
                    if (!writeMode && !(any & 2)) {
                        early = true;
                        break;
                    }
                    if (!(any & 1)) break;
                    levels++;
                    unsigned nw = 0u;
                    if (F | fyp | fym | fzp | fzm) {
                        const unsigned t0 = rk[0] & (F >> 1), t1 = rk[1] & (F << 1);
                        const unsigned t2 = rk[2] & fyp, t3 = rk[3] & fym;
                        const unsigned t4 = rk[4] & fzp, t5 = rk[5] & fzm;
                        nw = ~vis & (t0 | t1 | t2 | t3 | t4 | t5);
                        adm[0] |= nw & t0;
                        adm[1] |= nw & t1;
                        adm[2] |= nw & t2;
                        adm[3] |= nw & t3;
                        adm[4] |= nw & t4;
                        adm[5] |= nw & t5;
                        vis |= nw;
                        if (writeMode && nw) store_labels(A.labNew, rowBase, nw, stage);
                    }
                    F = nw;
                    p ^= 1;
                }
                const long long t1f = wall_clock64();
                t_flood += t1f - t0f;
                if (early) break;
                // next stage: smallest candidate among unvisited border vertices
                int cand = kInf;
                for (int i = tid; i < nring; i += kRowsNT) {
                    const int c = slotC[i];
                    if (c == kInf) continue;
                    const int l = slotL[i];
                    if (Vb[l >> 5] & (1u << (l & 31))) {
                        slotC[i] = kInf;  // labelled: no longer a seed candidate in this search
                        continue;
                    }
                    cand = min(cand, c);
                }
                const int level = block_min(cand, red, rc);
                // partial discharge: stages above the cap wait for later sweeps
                if (level == kInf || (level > stageCap && !writeMode)) {
                    t_stage += wall_clock64() - t1f;
                    break;
                }
                stages++;
                stage = level;
                for (int j = 0, i = tid; i < nring; j++, i += kRowsNT) {
                    if (slotC[i] != level) continue;
                    const int l = slotL[i];
                    const unsigned mm = A.ringM[i];
                    const int rw = l >> 5;
                    const unsigned bit = 1u << (l & 31);
                    unsigned match = 0u;
                    for (int k = 0; k < 6; k++) {
                        if (!((mm >> k) & 1u) || !(resM[k * R + rw] & bit)) continue;
                        const int d = halo[faceOff[k] + face_pos(k, l, TY)];
                        if (d < dinf && d + 1 == level) match |= 1u << (k >> 1);
                    }
                    // match != 0: the candidate came from one of these arcs
                    admB |= (u64)match << (3 * j);
                    slotC[i] = kInf;
                    atomicOr(&Fb[p * R + rw], bit);  // this buffer is all zero: the flood just ended on it
                }
                __syncthreads();
                if (myrow) {
                    F = Fb[p * R + row] & ~vis;
                    vis |= F;
                    if (writeMode && F) store_labels(A.labNew, rowBase, F, level);
                }
                t_stage += wall_clock64() - t1f;
            }
            // a search that ended by itself (under the same stage cap) leaves the dead set
            if (!early && !writeMode) dead = ~vis;
            // any excess vertex that reaches a target?
            const int found = block_any(myrow && (exM & vis) != 0u, anyB, rc);
            const long long t1s = wall_clock64();
            t_search += t1s - t0s;
            if (writeMode) {
                if (myrow) store_labels(A.labNew, rowBase, ~vis, dinf);
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
            unsigned canPush = 0u;
            if (myrow) {
#pragma unroll
                for (int k = 0; k < 6; k++) admL[k * R + row] = adm[k];
                admL[6 * R + row] = admT;
                canPush = admT | adm[0] | adm[1] | adm[2] | adm[3] | adm[4] | adm[5];
            }
            __syncthreads();
            int q = 0;
            for (;;) {
                int pushed = 0;
                // push from excess vertex u (local index, row ur) along its admissible arcs
                auto push_from = [&](int u, int ur) {
                    const int x = u & 31;
                    const unsigned bit = 1u << x;
                    unsigned a[7];
#pragma unroll
                    for (int k = 0; k < 7; k++) a[k] = admL[k * R + ur] & bit;
                    int *const exU = A.ex + base + u;
                    int c[6];
#pragma unroll
                    for (int k = 0; k < 6; k++) c[k] = a[k] ? A.res[(size_t)k * N + base + u] : 0;
                    const int cT = a[6] ? A.rt[base + u] : 0;
                    const int e = *exU;
                    if (e <= 0) {
                        // a receipt in this iteration sets the bit again at the merge
                        atomicOr(&clrB[q * R + ur], bit);
                        return;
                    }
                    int rem = e;
                    if (a[6]) {
                        const int d = min(rem, cT);
                        if (d > 0) {
                            A.rt[base + u] = cT - d;
                            rem -= d;
                            if (A.trace) atomicAdd((unsigned long long *)&s_tr[1], (u64)d);
                        }
                        if (cT == d) {
                            atomicAnd(&admL[6 * R + ur], ~bit);
                            atomicAnd(&rtmL[ur], ~bit);
                        }
                    }
#pragma unroll
                    for (int k = 0; k < 6; k++) {
                        if (!a[k] || rem <= 0) continue;
                        const int d = min(rem, c[k]);
                        if (d > 0) {
                            A.res[(size_t)k * N + base + u] = c[k] - d;
                            const int v = u + ((k & 1) ? -1 : 1) * (k < 2 ? 1 : (k < 4 ? 32 : 32 * TY));
                            const unsigned vbit = 1u << (v & 31);
                            atomicAdd(&A.res[(size_t)(k ^ 1) * N + base + v], d);
                            atomicAdd(&A.ex[base + v], d);
                            atomicOr(&resM[(k ^ 1) * R + (v >> 5)], vbit);
                            atomicOr(&recvB[q * R + (v >> 5)], vbit);
                            rem -= d;
                        }
                        if (c[k] == d) {
                            atomicAnd(&admL[k * R + ur], ~bit);
                            atomicAnd(&resM[k * R + ur], ~bit);
                        }
                    }
                    if (rem < e) {
                        // drained what it saw: cleared, unless a receipt in this
                        // iteration sets the bit again at the merge
                        atomicAdd(exU, rem - e);
                        if (rem == 0) atomicOr(&clrB[q * R + ur], bit);
                        pushed = 1;
                    }
                };
                const unsigned P = exM & canPush;
                const int cnt = __popc(P);
                if (__ballot(cnt > 1) == 0ull) {
                    // light iteration: each thread pushes from its own row
                    if (P) push_from(row * 32 + __ffs(P) - 1, row);
                } else {
                    // the excess vertices of the wave's rows, spread over its lanes
                    const int incl = wave_incl_scan(cnt, lane);
                    const int total = __builtin_amdgcn_readlane(incl, 63);
                    for (int w0 = 0; w0 < total; w0 += kListCap) {
                        int idx = incl - cnt;
                        if (cnt && idx < w0 + kListCap && idx + cnt > w0) {
                            unsigned m = P;
                            while (m) {
                                const int x = __ffs(m) - 1;
                                m &= m - 1;
                                if (idx >= w0 && idx < w0 + kListCap) wlist[idx - w0] = (unsigned short)(row * 32 + x);
                                idx++;
                            }
                        }
                        wave_lds_sync();
                        const int nItems = min(total - w0, kListCap);
                        for (int it = lane; it < nItems; it += 64) {
                            const int u = wlist[it];
                            push_from(u, u >> 5);
                        }
                        wave_lds_sync();
                    }
                }
                // first-level vertices of stages k > 0 push over boundary arcs
                if (admB) {
                    for (int j = 0; (admB >> (3 * j)) != 0ull; j++) {
                        const unsigned ab = (unsigned)(admB >> (3 * j)) & 7u;
                        if (!ab) continue;
                        const int i = tid + j * kRowsNT;
                        const int l = slotL[i];
                        const unsigned mm = A.ringM[i];
                        const size_t gu = base + l;
                        const int rw = l >> 5;
                        const unsigned bit = 1u << (l & 31);
                        const int e = A.ex[gu];
                        if (e <= 0) {
                            atomicOr(&clrB[q * R + rw], bit);
                            continue;
                        }
                        int rem = e;
                        for (int a = 0; a < 3; a++) {
                            if (!((ab >> a) & 1u) || rem <= 0) continue;
                            const int k = axis_dir_m(mm, a);
                            const int c = A.res[(size_t)k * N + gu];
                            const int d = min(rem, c);
                            if (d > 0) {
                                A.res[(size_t)k * N + gu] = c - d;
                                atomicAdd(&A.pushb[(size_t)k * N + gu], d);
                                rem -= d;
                                if (A.trace) atomicAdd((unsigned long long *)&s_tr[2], (u64)d);
                            }
                            if (c == d) {
                                admB &= ~(1ull << (3 * j + a));
                                atomicAnd(&resM[k * R + rw], ~bit);
                            }
                        }
                        if (rem < e) {
                            atomicAdd(&A.ex[gu], rem - e);
                            if (rem == 0) atomicOr(&clrB[q * R + rw], bit);
                            pushed = 1;
                        }
                    }
                }
                const int any = block_any(pushed, anyB, rc);
                pushIters++;
                if (myrow) {
                    const unsigned rv = recvB[q * R + row], cl = clrB[q * R + row];
                    recvB[q * R + row] = 0u;
                    clrB[q * R + row] = 0u;
                    exM = (exM & ~cl) | rv;
                    canPush = admL[6 * R + row];
#pragma unroll
                    for (int k = 0; k < 6; k++) canPush |= admL[k * R + row];
                }
                q ^= 1;
                if (!any) break;
            }
            t_push += wall_clock64() - t1s;
            // no excess left in the region (the masks may only over-report it):
            // the next search cannot find an excess vertex, so it writes the labels
            if (!block_any(myrow && exM != 0u, anyB, rc)) writeMode = true;
        }
        __syncthreads();
        if (A.trace) {
            long long ex_out = 0, lsum = 0;
            for (int l = tid; l < V; l += kRowsNT) ex_out += A.ex[base + l];
            for (int i = tid; i < nring; i += kRowsNT) lsum += min(A.labNew[base + A.ringL[i]], 65535);
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

// ---------------------------------------------------------------------------
// Global relabel, one distance level D (see k_grelabel in mf_kernels.hip), for
// the tiles of k_discharge_rows.  At level 0 every region builds its residual-
// arc masks from HBM into a per-region cache (six directions, then the
// unlabelled vertices); later levels read the cache.  The flood of a level
// runs on the row masks with one barrier per step, from t at level 0 and from
// the seed bits marked by the previous level otherwise; reached vertices get
// label D, and reached border vertices mark their residual predecessors across
// the border (unlabelled) as seeds of D + 1 and flag their regions.
// ---------------------------------------------------------------------------
size_t grelabel_rows_lds(int ty, int tz) { return (size_t)9 * ty * tz * sizeof(unsigned); }

// The 64 row masks (32-bit, "value > 0") of 64 consecutive rows of one plane,
// built by one wave: src points at this lane's vertex of the first two rows.
// All 32 loads are issued before the first ballot, so they are in flight together.
__device__ __forceinline__ void build_row_masks(const int *src, unsigned *dst, int lane) {
    int v[32];
#pragma unroll
    for (int i = 0; i < 32; i++) v[i] = src[i * 64];
#pragma unroll
    for (int i = 0; i < 32; i++) {
        const u64 b = __ballot(v[i] > 0);
        if (lane == 0) {
            dst[2 * i] = (unsigned)b;
            dst[2 * i + 1] = (unsigned)(b >> 32);
        }
    }
}

__global__ __launch_bounds__(kRowsNT) void k_grelabel_rows(GRelabelArgs A) {
    extern __shared__ __align__(16) unsigned smem_rows[];
    __shared__ __align__(16) unsigned char anyB[2][kRowsWaves];  // block_any bytes
    __shared__ int s_go;
    const Geo &G = A.G;
    const int V = G.V, N = G.N, TY = G.ty, TZ = G.tz, R = TY * TZ, D = A.level, dinf = A.dinf;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const bool myrow = tid < R;
    const int row = tid, y = tid % TY, z = tid / TY;
    unsigned *tmp = smem_rows;        // [7][R]: masks built at level 0
    unsigned *Fb = smem_rows + 7 * R; // [2][R]: frontier rows
    int rc = 0;
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
        unsigned *cr = (unsigned *)A.cache + (size_t)r * 7 * R;
        unsigned rk[6], U = 0u, seed = 0u;
#pragma unroll
        for (int k = 0; k < 6; k++) rk[k] = 0u;
        if (D == 0) {
            const int row0 = wid * 64;
            if (row0 + 64 <= R) {
                for (int q = 0; q < 7; q++) {
                    const int *plane = q < 6 ? A.res + (size_t)q * N : A.rt;
                    build_row_masks(plane + base + (size_t)row0 * 32 + lane, tmp + q * R + row0, lane);
                }
            }
            __syncthreads();
            if (myrow) {
#pragma unroll
                for (int k = 0; k < 6; k++) {
                    rk[k] = tmp[k * R + row];
                    cr[k * R + row] = rk[k];
                }
                U = ~0u;
                seed = tmp[6 * R + row];
            }
        } else if (myrow) {
#pragma unroll
            for (int k = 0; k < 6; k++) rk[k] = cr[k * R + row];
            U = cr[6 * R + row];
            unsigned *cw = A.candBitsIn + (base >> 5) + row;
            seed = *cw & U;
            *cw = 0u;
        }
        unsigned reached = seed, F = seed;
        int p = 0;
        for (;;) {
            if (myrow) Fb[p * R + row] = F;
            if (!block_any(F != 0u, anyB, rc)) break;
            if (myrow) {
                const unsigned *Fp = Fb + p * R;
                const unsigned fyp = (y + 1 < TY) ? Fp[row + 1] : 0u;
                const unsigned fym = (y > 0) ? Fp[row - 1] : 0u;
                const unsigned fzp = (z + 1 < TZ) ? Fp[row + TY] : 0u;
                const unsigned fzm = (z > 0) ? Fp[row - TY] : 0u;
                const unsigned nw = U & ~reached &
                                    ((rk[0] & (F >> 1)) | (rk[1] & (F << 1)) | (rk[2] & fyp) |
                                     (rk[3] & fym) | (rk[4] & fzp) | (rk[5] & fzm));
                reached |= nw;
                F = nw;
            }
            p ^= 1;
        }
        // the unlabelled mask of the cache is written by every row at level 0
        if (myrow && (reached || D == 0)) cr[6 * R + row] = U & ~reached;
        if (myrow && reached) {
            store_labels(A.lab, base + (size_t)row * 32, reached, D);
            // predecessors across the border of the reached border vertices
            for (int k = 0; k < 6; k++) {
                // border vertices of this row that direction k leaves the tile from
                unsigned m;
                if (k == 0) m = reached & 0x80000000u;
                else if (k == 1) m = reached & 1u;
                else if (k == 2) m = (y == TY - 1) ? reached : 0u;
                else if (k == 3) m = (y == 0) ? reached : 0u;
                else if (k == 4) m = (z == TZ - 1) ? reached : 0u;
                else m = (z == 0) ? reached : 0u;
                while (m) {
                    const int x = __ffs(m) - 1;
                    m &= m - 1;
                    // u = v + o_k across the border, with residual arc (u, v) in direction k ^ 1
                    const int ug = cross_nbr(G, r, z, y, x, k);
                    if (ug < 0 || A.res[(size_t)(k ^ 1) * N + ug] <= 0 || A.lab[ug] != dinf) continue;
                    atomicOr(&A.candBitsOut[ug >> 5], 1u << (ug & 31));
                    if (atomicExch(&A.flagOut[ug / V], 1) == 0) atomicAdd(A.flagged, 1u);
                }
            }
        }
    }
}

// Residual reachability for the cuts (the region floods of k_flood, same
// marks) on the tiles of k_discharge_rows: one workgroup per region, one 32-bit
// row per thread.  dir 0 floods forward from the excess vertices along arcs
// with c_f > 0 (the masks are moved to the head of each arc), dir 1 backward
// from t.  Reached border vertices mark their neighbours across the border
// (atomic exchange, as k_flood) and flag the neighbouring region.
__global__ __launch_bounds__(kRowsNT) void k_flood_rows(FloodArgs A) {
    extern __shared__ __align__(16) unsigned smem_rows[];
    __shared__ __align__(16) unsigned char anyB[2][kRowsWaves];  // block_any bytes
    __shared__ int s_go;
    const Geo &G = A.G;
    const int V = G.V, N = G.N, TY = G.ty, TZ = G.tz, R = TY * TZ;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const bool myrow = tid < R;
    const int row = tid, y = tid % TY, z = tid / TY;
    unsigned *tmp = smem_rows;        // [7][R]: residual masks, then marks (or round-0 seeds)
    unsigned *Fb = smem_rows + 7 * R; // [2][R]: frontier rows
    int rc = 0;
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
        // masks from HBM: plane q < 6 residual arcs, plane 6 the marks (all zero
        // in round 0, when it holds the seeds instead)
        {
            const int row0 = wid * 64;
            if (row0 + 64 <= R) {
                for (int q = 0; q < 7; q++) {
                    const int *plane = q < 6 ? A.res + (size_t)q * N
                                             : (A.round > 0 ? A.mark : (A.dir == 0 ? A.ex : A.rt));
                    build_row_masks(plane + base + (size_t)row0 * 32 + lane, tmp + q * R + row0, lane);
                }
            }
        }
        __syncthreads();
        unsigned rk[6], rf[6], M = 0u;
#pragma unroll
        for (int k = 0; k < 6; k++) rk[k] = rf[k] = 0u;
        if (myrow) {
#pragma unroll
            for (int k = 0; k < 6; k++) rk[k] = tmp[k * R + row];
            M = tmp[6 * R + row];
            if (A.dir == 0) {
                // at the head w: is the arc w - o_k -> w residual (inside the tile)
                rf[0] = rk[0] << 1;
                rf[1] = rk[1] >> 1;
                rf[2] = (y > 0) ? tmp[2 * R + row - 1] : 0u;
                rf[3] = (y + 1 < TY) ? tmp[3 * R + row + 1] : 0u;
                rf[4] = (z > 0) ? tmp[4 * R + row - TY] : 0u;
                rf[5] = (z + 1 < TZ) ? tmp[5 * R + row + TY] : 0u;
            }
        }
        const unsigned M0 = A.round > 0 ? M : 0u;  // marks already stored
        unsigned reached = M, F = M;
        int p = 0;
        for (;;) {
            if (myrow) Fb[p * R + row] = F;
            if (!block_any(F != 0u, anyB, rc)) break;
            if (myrow) {
                const unsigned *Fp = Fb + p * R;
                const unsigned fyp = (y + 1 < TY) ? Fp[row + 1] : 0u;
                const unsigned fym = (y > 0) ? Fp[row - 1] : 0u;
                const unsigned fzp = (z + 1 < TZ) ? Fp[row + TY] : 0u;
                const unsigned fzm = (z > 0) ? Fp[row - TY] : 0u;
                unsigned nw;
                if (A.dir == 0)
                    nw = (rf[0] & (F << 1)) | (rf[1] & (F >> 1)) | (rf[2] & fym) | (rf[3] & fyp) |
                         (rf[4] & fzm) | (rf[5] & fzp);
                else
                    nw = (rk[0] & (F >> 1)) | (rk[1] & (F << 1)) | (rk[2] & fyp) | (rk[3] & fym) |
                         (rk[4] & fzp) | (rk[5] & fzm);
                nw &= ~reached;
                reached |= nw;
                F = nw;
            }
            p ^= 1;
        }
        if (myrow && reached) {
            // marks of this round, seeds included (stores of 1 race harmlessly
            // with the neighbours' exchanges)
            unsigned nb = reached & ~M0;
            while (nb) {
                const int x = __ffs(nb) - 1;
                nb &= nb - 1;
                A.mark[base + (size_t)row * 32 + x] = 1;
            }
            for (int k = 0; k < 6; k++) {
                // reached border vertices of this row that direction k leaves the tile from
                unsigned m;
                if (k == 0) m = reached & 0x80000000u;
                else if (k == 1) m = reached & 1u;
                else if (k == 2) m = (y == TY - 1) ? reached : 0u;
                else if (k == 3) m = (y == 0) ? reached : 0u;
                else if (k == 4) m = (z == TZ - 1) ? reached : 0u;
                else m = (z == 0) ? reached : 0u;
                if (A.dir == 0) m &= rk[k];  // forward: the arc (v, v + o_k) is residual
                while (m) {
                    const int x = __ffs(m) - 1;
                    m &= m - 1;
                    const int wg = cross_nbr(G, r, z, y, x, k);
                    if (wg < 0) continue;
                    // backward: the arc (u, v) from u = v + o_k, in direction k ^ 1, is residual
                    if (A.dir == 1 && A.res[(size_t)(k ^ 1) * N + wg] <= 0) continue;
                    if (atomicExch(&A.mark[wg], 1) == 0) {
                        A.dirtyOut[wg / V] = 1;
                        atomicAdd(A.changed, 1u);
                    }
                }
            }
        }
    }
}

hipError_t launch_flood_rows(const FloodArgs &A, int blocks, hipStream_t s) {
    const int R = A.G.ty * A.G.tz;
    if (A.G.K != 6 || A.G.tx != 32 || R % 64 != 0 || R > kRowsNT) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_flood_rows, dim3(blocks), dim3(kRowsNT), grelabel_rows_lds(A.G.ty, A.G.tz), s, A);
    return hipGetLastError();
}

hipError_t launch_grelabel_rows(const GRelabelArgs &A, int blocks, hipStream_t s) {
    hipLaunchKernelGGL(k_grelabel_rows, dim3(blocks), dim3(kRowsNT), grelabel_rows_lds(A.G.ty, A.G.tz), s, A);
    return hipGetLastError();
}

void set_rows_attributes() {
    (void)hipFuncSetAttribute((const void *)k_discharge_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    (void)hipFuncSetAttribute((const void *)k_grelabel_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                              64 * 1024);
}

// The boundary pushes keep three bits per border vertex of a thread in 64 bits.
int rows_slots(int nring) {
    const int need = (nring + kRowsNT - 1) / kRowsNT;
    return need <= 21 ? need : 0;
}

hipError_t launch_discharge_rows(const DischargeArgs &A, int blocks, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL(k_discharge_rows, dim3(blocks), dim3(kRowsNT), lds, s, A);
    return hipGetLastError();
}

}  // namespace mfd
