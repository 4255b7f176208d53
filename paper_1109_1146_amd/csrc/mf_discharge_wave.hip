// Single-wavefront region discharge for 2D tiles of at most 64 x 64 vertices
// (Proc. ARD of Sec. 4.2 with the region relabel of Alg. 3; same method as
// k_discharge_lds, different execution).
//
// One wave64 owns a region.  Lane y holds row y of the tile as 64-bit masks:
// residual arc present in each direction, residual t-link, visited, frontier,
// and the 12 bit-planes of each vertex's search level.  One level of the
// multi-level breadth-first search from the targets is then a handful of
// shifts, cross-lane row exchanges and ORs in registers, with no LDS traffic
// and no workgroup barrier.  The integer state (residuals as int16 K-vectors,
// excess, t-links, halo labels, boundary pushes) stays in LDS; the push pass
// walks the levels from the last to the first, each lane handling the
// vertices of its row at that level.
#include "mf_device.h"
#include "mf_launch.h"

namespace mfd {

typedef unsigned long long u64;

namespace {

constexpr int kPlanes = 12;  // search steps < 4096 = 64 * 64

__host__ __device__ inline size_t al16w(size_t x) { return (x + 15) & ~(size_t)15; }

struct WaveLayout {
    size_t res, ex, rt, S, stepLevel, ringIdx, halo, push, total;
};

__host__ __device__ inline WaveLayout wave_layout(int V, int K, int nring, int rtBytes) {
    WaveLayout L;
    size_t o = 0;
    L.res = o; o = al16w(o + (size_t)V * K * rtBytes);
    L.ex = o; o = al16w(o + (size_t)V * 4);
    L.rt = o; o = al16w(o + (size_t)V * rtBytes);
    L.S = o; o = al16w(o + (size_t)V * 2);
    L.stepLevel = o; o = al16w(o + (size_t)V * 4);
    L.ringIdx = o; o = al16w(o + (size_t)V * 2);
    L.halo = o; o = al16w(o + (size_t)nring * K * 4);
    L.push = o; o = al16w(o + (size_t)nring * K * 4);
    L.total = o;
    return L;
}

__device__ __forceinline__ u64 shfl64(u64 v, int src) {
    return __shfl(v, src, 64);
}

// Row (y + dy) of a per-lane row mask, 0 outside the tile.
__device__ __forceinline__ u64 row_at(u64 v, int y, int dy, int ty) {
    const int src = y + dy;
    const u64 w = shfl64(v, src < 0 ? 0 : (src > 63 ? 63 : src));
    return (src < 0 || src >= ty) ? 0ull : w;
}

// Bits of row mask m moved so that bit x holds bit x + dx.
__device__ __forceinline__ u64 shift_dx(u64 m, int dx) {
    return dx > 0 ? (m >> dx) : (dx < 0 ? (m << (-dx)) : m);
}

// Rows y-1, y, y+1 of a per-lane row mask (0 outside the tile).
struct Rows3 {
    u64 up, mid, dn;  // row y-1, y, y+1
    __device__ __forceinline__ u64 at(int dy) const { return dy < 0 ? up : (dy > 0 ? dn : mid); }
};

__device__ __forceinline__ Rows3 rows3(u64 v, int y, int ty) {
    Rows3 r;
    r.mid = v;
    r.up = row_at(v, y, -1, ty);
    r.dn = row_at(v, y, 1, ty);
    return r;
}

__device__ __forceinline__ int wave_min_int(int v) {
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

}  // namespace

size_t discharge_wave_bytes(int V, int K, int nring, int narrow) {
    return wave_layout(V, K, nring, narrow ? 2 : 4).total;
}

template <int K, typename RT>
__global__ __launch_bounds__(64) void k_discharge_wave(DischargeArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ long long s_tr[4];
    __shared__ u64 seedRows[64];
    __shared__ u64 exRows[64];  // push pass: bit x of row y set iff vertex (x, y) holds excess
    if (*A.actIn == 0ull) return;
    seedRows[threadIdx.x] = 0ull;
    const Geo &G = A.G;
    const int V = G.V, N = G.N, nring = A.nring;
    const int TX = G.tx, TY = G.ty;
    const int lane = threadIdx.x;
    const int y = lane;  // the row this lane owns (idle lanes: y >= TY)
    const WaveLayout L = wave_layout(V, K, nring, (int)sizeof(RT));
    RT *resL = (RT *)(smem + L.res);
    int *exL = (int *)(smem + L.ex);
    RT *rtL = (RT *)(smem + L.rt);
    unsigned short *S = (unsigned short *)(smem + L.S);
    int *stepLevel = (int *)(smem + L.stepLevel);
    short *ringIdx = (short *)(smem + L.ringIdx);
    int *halo = (int *)(smem + L.halo);
    int *pushL = (int *)(smem + L.push);
    const int dinf = A.dinf;
    const u64 rowmask = TX == 64 ? ~0ull : ((1ull << TX) - 1);
    const bool myrow = y < TY;
    int dy[K], dx[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        dy[k] = G.oy[k];
        dx[k] = G.ox[k];
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
            // a deferred region keeps its flag and is discharged in a later sweep
            if (active && A.defer && A.defer[r]) active = 0;
            else A.ractive[r] = 0;
        }
        active = __shfl(active, 0, 64);
        if (!active) {
            for (int l = lane; l < V; l += 64) A.labNew[base + l] = A.labOld[base + l];
            continue;
        }
        const long long t_start = wall_clock64();
        if (lane < 4) s_tr[lane] = 0;
        // ---------------- stage the region into LDS ----------------
        for (int l = lane; l < V; l += 64) {
#pragma unroll
            for (int k = 0; k < K; k++) resL[l * K + k] = (RT)A.res[(size_t)k * N + base + l];
            exL[l] = A.ex[base + l];
            rtL[l] = (RT)A.rt[base + l];
            ringIdx[l] = -1;
        }
        __syncthreads();
        for (int i = lane; i < nring; i += 64) {
            const int l = A.ringL[i];
            const unsigned m = A.ringM[i];
            ringIdx[l] = (short)i;
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

        int iter = 0;
        long long bfs_steps = 0, classes = 0, t_search = 0, t_push = 0;
        u64 VIS = 0, P[kPlanes];
        int nsteps = 0;
        for (;;) {
            const long long t_round = wall_clock64();
            // ---------------- row masks from the LDS state (coalesced, by ballot) ----------------
            u64 R[K], RTm = 0, EXm = 0;
#pragma unroll
            for (int k = 0; k < K; k++) R[k] = 0;
            for (int row = 0; row < TY; row++) {
                const int l = row * TX + lane;
                const bool ok = lane < TX;
                RT c[K];
                if (ok) {
#pragma unroll
                    for (int k = 0; k < K; k++) c[k] = resL[l * K + k];
                } else {
#pragma unroll
                    for (int k = 0; k < K; k++) c[k] = 0;
                }
#pragma unroll
                for (int k = 0; k < K; k++) {
                    const u64 b = __ballot(c[k] > 0);
                    if (lane == row) R[k] = b;
                }
                const u64 bt = __ballot(ok && rtL[l] > 0);
                const u64 be = __ballot(ok && exL[l] > 0);
                if (lane == row) { RTm = bt; EXm = be; }
            }
#pragma unroll
            for (int k = 0; k < K; k++) R[k] &= inside[k];
            // ---------------- multi-level search from the targets ----------------
#pragma unroll
            for (int j = 0; j < kPlanes; j++) P[j] = 0;
            VIS = RTm;  // step 0: residual t-links
            u64 F = RTm;
            nsteps = 0;
            int lvl = 0;
            if (__ballot(F != 0ull)) {
                if (lane == 0) stepLevel[0] = 0;
                nsteps = 1;
            }
            for (;;) {
                // flood: u unvisited with a residual arc (u, v) to a frontier vertex v
                for (;;) {
                    u64 nw = 0;
                    const Rows3 FR = rows3(F, y, TY);
#pragma unroll
                    for (int k = 0; k < K; k++) nw |= R[k] & shift_dx(FR.at(dy[k]), dx[k]);
                    nw &= ~VIS;
                    if (!__ballot(nw != 0ull)) break;
                    const int st = nsteps;
                    VIS |= nw;
#pragma unroll
                    for (int j = 0; j < kPlanes; j++)
                        if ((st >> j) & 1) P[j] |= nw;
                    if (lane == 0) stepLevel[st] = lvl;
                    nsteps = st + 1;
                    F = nw;
                }
                // next stage: smallest d(w) + 1 over residual boundary arcs of
                // unvisited border vertices; border entries are spread over the lanes
                int best = kInf;
                for (int i0 = 0; i0 < nring; i0 += 64) {
                    const int i = i0 + lane;
                    const int l = i < nring ? A.ringL[i] : 0;
                    const int ry = l / TX, rx = l - ry * TX;
                    const u64 vrow = shfl64(VIS, ry);
                    if (i < nring && !((vrow >> rx) & 1ull)) {
#pragma unroll
                        for (int k = 0; k < K; k++) {
                            const int h = halo[i * K + k];
                            if (h < dinf && resL[l * K + k] > 0) best = min(best, h + 1);
                        }
                    }
                }
                const int level = wave_min_int(best);
                if (level == kInf) break;
                classes++;
                for (int i0 = 0; i0 < nring; i0 += 64) {
                    const int i = i0 + lane;
                    const int l = i < nring ? A.ringL[i] : 0;
                    const int ry = l / TX, rx = l - ry * TX;
                    const u64 vrow = shfl64(VIS, ry);
                    if (i < nring && !((vrow >> rx) & 1ull)) {
                        bool hit = false;
#pragma unroll
                        for (int k = 0; k < K; k++) {
                            const int h = halo[i * K + k];
                            if (h < dinf && h + 1 == level && resL[l * K + k] > 0) hit = true;
                        }
                        if (hit) atomicOr(&seedRows[ry], 1ull << rx);
                    }
                }
                __syncthreads();
                u64 seed = 0;
                if (myrow) {
                    seed = seedRows[y];
                    seedRows[y] = 0ull;
                }
                __syncthreads();
                const int st = nsteps;
                VIS |= seed;
#pragma unroll
                for (int j = 0; j < kPlanes; j++)
                    if ((st >> j) & 1) P[j] |= seed;
                if (lane == 0) stepLevel[st] = level;
                nsteps = st + 1;
                lvl = level;
                F = seed;
            }
            bfs_steps += nsteps;
            const long long t_mid = wall_clock64();
            t_search += t_mid - t_round;
            if (!__ballot((EXm & VIS) != 0ull)) break;
            if (++iter > A.maxIter) {
                if (lane == 0) atomicOr(A.err, 4);
                break;
            }
            exRows[lane] = EXm;
            __syncthreads();  // stepLevel and exRows visible
            // ---------------- push excess down the search levels ----------------
            for (int s = nsteps - 1; s >= 0; s--) {
                // members of level s and s - 1 in this row
                u64 Ms = VIS, Mp = (s > 0) ? VIS : 0ull;
#pragma unroll
                for (int j = 0; j < kPlanes; j++) {
                    Ms &= ((s >> j) & 1) ? P[j] : ~P[j];
                    if (s > 0) Mp &= (((s - 1) >> j) & 1) ? P[j] : ~P[j];
                }
                u64 m = Ms & exRows[lane];
                if (!__ballot(m != 0ull)) continue;  // no excess on this level: nothing moves
                const int Lv = stepLevel[s];
                const bool seedstep = (s == 0) || (stepLevel[s - 1] != Lv);
                u64 Adm[K];
                {
                    const Rows3 MR = rows3(Mp, y, TY);  // all lanes take part in the exchange
#pragma unroll
                    for (int k = 0; k < K; k++) Adm[k] = seedstep ? 0ull : (R[k] & shift_dx(MR.at(dy[k]), dx[k]));
                }
                u64 drained = 0;
                while (m) {
                    const int x = __ffsll(m) - 1;
                    m &= m - 1;
                    const int u = y * TX + x;
                    int e = exL[u];
                    if (e <= 0) continue;
                    if (seedstep) {
                        if (Lv == 0) {
                            const int t = rtL[u];
                            if (t > 0) {
                                const int d = min(e, t);
                                rtL[u] = (RT)(t - d);
                                e -= d;
                                if (A.trace) atomicAdd((unsigned long long *)&s_tr[1], (u64)d);
                            }
                        } else {
                            const int ri = ringIdx[u];
#pragma unroll
                            for (int k = 0; k < K; k++) {
                                if (e <= 0 || ri < 0) break;
                                const int h = halo[ri * K + k];
                                if (h >= dinf || h + 1 != Lv) continue;
                                const int c = resL[u * K + k];
                                if (c <= 0) continue;
                                const int d = min(e, c);
                                resL[u * K + k] = (RT)(c - d);
                                pushL[ri * K + k] += d;
                                e -= d;
                            }
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < K; k++) {
                            if (e <= 0 || !((Adm[k] >> x) & 1ull)) continue;
                            const int v = u + dy[k] * TX + dx[k];
                            const int c = resL[u * K + k];
                            if (c <= 0) continue;
                            const int d = min(e, c);
                            resL[u * K + k] = (RT)(c - d);
                            resL[v * K + (k ^ 1)] = (RT)(resL[v * K + (k ^ 1)] + d);
                            atomicAdd(&exL[v], d);
                            atomicOr(&exRows[y + dy[k]], 1ull << (x + dx[k]));
                            e -= d;
                        }
                    }
                    exL[u] = e;
                    if (e == 0) drained |= 1ull << x;
                }
                if (drained) atomicAnd(&exRows[y], ~drained);
                __syncthreads();
            }
            t_push += wall_clock64() - t_mid;
        }
        // ---------------- levels of the last search -> labels ----------------
        // store each vertex's step (or 0xffff when unreached) in S, row by row
        for (int row = 0; row < TY; row++) {
            const u64 vis = shfl64(VIS, row);
            int stp = 0;
#pragma unroll
            for (int j = 0; j < kPlanes; j++) {
                const u64 pj = shfl64(P[j], row);
                if (lane < TX && ((pj >> lane) & 1ull)) stp |= 1 << j;
            }
            if (lane < TX) S[row * TX + lane] = ((vis >> lane) & 1ull) ? (unsigned short)stp : 0xffffu;
        }
        __syncthreads();
        // ---------------- write the region back ----------------
        for (int l = lane; l < V; l += 64) {
#pragma unroll
            for (int k = 0; k < K; k++) A.res[(size_t)k * N + base + l] = resL[l * K + k];
            A.ex[base + l] = exL[l];
            A.rt[base + l] = rtL[l];
            const int s = S[l];
            A.labNew[base + l] = (s == 0xffff) ? dinf : min(stepLevel[s], dinf);
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
            long long ex_out = 0, to_b = 0, lsum = 0;
            for (int l = lane; l < V; l += 64) ex_out += exL[l];
            for (int i = lane; i < nring; i += 64) {
#pragma unroll
                for (int k = 0; k < K; k++) to_b += pushL[i * K + k];
                const int s = S[A.ringL[i]];
                lsum += (s == 0xffff) ? 65535 : min(stepLevel[s], 65535);
            }
            atomicAdd((unsigned long long *)&s_tr[0], (u64)ex_out);
            atomicAdd((unsigned long long *)&s_tr[2], (u64)to_b);
            atomicAdd((unsigned long long *)&s_tr[3], (u64)lsum);
        }
        __syncthreads();
        if (lane == 0) {
            atomicAdd(&A.stats[0], 1ull);
            atomicAdd(&A.stats[1], (u64)A.rvcount[r]);
            atomicAdd(&A.stats[2], (u64)(iter + 1));
            atomicAdd(&A.stats[3], (u64)bfs_steps);
            atomicAdd(&A.stats[4], (u64)classes);
            atomicAdd(&A.stats[6], (u64)t_search);
            atomicAdd(&A.stats[7], (u64)t_push);
            if (A.trace) {
                unsigned long long idx = atomicAdd(&A.stats[5], 1ull);
                if ((long long)idx < A.traceCap) {
                    int *rec = A.trace + idx * 10;
                    const long long ex_in = s_tr[0] + s_tr[1] + s_tr[2];
                    rec[0] = A.sweep;
                    rec[1] = r;
                    rec[2] = iter + 1;
                    rec[3] = (int)min(bfs_steps, 0x7fffffffLL);
                    rec[4] = (int)min(classes, 0x7fffffffLL);
                    rec[5] = (int)min(wall_clock64() - t_start, 0x7fffffffLL);
                    rec[6] = (int)min(ex_in, 0x7fffffffLL);
                    rec[7] = (int)min(s_tr[1], 0x7fffffffLL);
                    rec[8] = (int)min(s_tr[2], 0x7fffffffLL);
                    rec[9] = (int)min(s_tr[3], 0x7fffffffLL);
                }
            }
        }
        __syncthreads();
    }
}

void set_wave_attributes() {
    (void)hipFuncSetAttribute((const void *)k_discharge_wave<4, short>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute((const void *)k_discharge_wave<8, short>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute((const void *)k_discharge_wave<4, int>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute((const void *)k_discharge_wave<8, int>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();
}

template <int K, typename RT>
static hipError_t launch_wave_t(const DischargeArgs &A, int blocks, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_discharge_wave<K, RT>), dim3(blocks), dim3(64), lds, s, A);
    return hipGetLastError();
}

hipError_t launch_discharge_wave(const DischargeArgs &A, int blocks, size_t lds, int narrow,
                                 hipStream_t s) {
    const int K = A.G.K;
    if (A.G.tz != 1 || A.G.tx > 64 || A.G.ty > 64) return hipErrorInvalidValue;
    if (narrow) {
        if (K == 4) return launch_wave_t<4, short>(A, blocks, lds, s);
        if (K == 8) return launch_wave_t<8, short>(A, blocks, lds, s);
    } else {
        if (K == 4) return launch_wave_t<4, int>(A, blocks, lds, s);
        if (K == 8) return launch_wave_t<8, int>(A, blocks, lds, s);
    }
    return hipErrorInvalidValue;
}

// Global relabel, one distance level (see k_grelabel in mf_kernels.hip), for
// 2D regions of at most 64 x 64 with the row-bitmask flood of one wavefront:
// masks are built from HBM by ballot, the flood runs in registers, labels and
// next-level marks are written back.
template <int K>
__global__ __launch_bounds__(64) void k_grelabel_wave(GRelabelArgs A) {
    const Geo &G = A.G;
    const int V = G.V, N = G.N, TX = G.tx, TY = G.ty, D = A.level, dinf = A.dinf;
    const int lane = threadIdx.x, y = lane;
    const bool myrow = y < TY;
    const u64 rowmask = TX == 64 ? ~0ull : ((1ull << TX) - 1);
    int dy[K], dx[K];
    u64 inside[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        dy[k] = G.oy[k];
        dx[k] = G.ox[k];
        const bool rowok = myrow && y + dy[k] >= 0 && y + dy[k] < TY;
        u64 m = rowok ? rowmask : 0ull;
        if (dx[k] > 0) m &= rowmask >> dx[k];
        if (dx[k] < 0) m &= (rowmask << (-dx[k])) & rowmask;
        inside[k] = m;
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
        u64 R[K], U = 0, SEED = 0;
        for (int row = 0; row < TY; row++) {
            const int l = row * TX + lane;
            const bool ok = lane < TX;
#pragma unroll
            for (int k = 0; k < K; k++) {
                const u64 b = __ballot(ok && A.res[(size_t)k * N + base + l] > 0);
                if (lane == row) R[k] = b;
            }
            const int lv = ok ? A.lab[base + l] : 0;
            const bool unl = ok && lv == dinf;
            bool sd;
            if (D == 0) {
                sd = unl && A.rt[base + l] > 0;
            } else {
                const bool c = ok && A.candIn[base + l] != 0;
                if (c) A.candIn[base + l] = 0;
                sd = unl && c;
            }
            const u64 bu = __ballot(unl), bs = __ballot(sd);
            if (lane == row) { U = bu; SEED = bs; }
        }
#pragma unroll
        for (int k = 0; k < K; k++) R[k] &= inside[k];
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
        for (int row = 0; row < TY; row++) {
            const u64 m = shfl64(reached, row);
            if (lane < TX && ((m >> lane) & 1ull)) A.lab[base + row * TX + lane] = D;
        }
        // marks for D + 1: residual predecessors across the border of reached border vertices
        for (int i0 = 0; i0 < A.nring; i0 += 64) {
            const int i = i0 + lane;
            const int l = i < A.nring ? A.ringL[i] : 0;
            const int ry = l / TX, rx = l - ry * TX;
            const u64 m = shfl64(reached, ry);
            if (i < A.nring && ((m >> rx) & 1ull)) {
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

hipError_t launch_grelabel_wave(const GRelabelArgs &A, int blocks, hipStream_t s) {
    if (A.G.tz != 1 || A.G.tx > 64 || A.G.ty > 64) return hipErrorInvalidValue;
    if (A.G.K == 4) hipLaunchKernelGGL(k_grelabel_wave<4>, dim3(blocks), dim3(64), 0, s, A);
    else if (A.G.K == 8) hipLaunchKernelGGL(k_grelabel_wave<8>, dim3(blocks), dim3(64), 0, s, A);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace mfd
