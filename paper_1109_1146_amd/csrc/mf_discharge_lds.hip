// LDS-resident region discharge (Proc. ARD of Sec. 4.2 with the region
// relabel of Alg. 3) for regions whose whole working state fits in the 160 KB
// of LDS of a gfx950 compute unit.
//
// Same method as k_discharge in mf_kernels.hip (multi-level search from the
// targets, excess pushed down the search levels, repeated until no excess
// vertex of the region reaches a target), but the region is copied into LDS
// once, worked on there, and written back once: residuals as an array of
// per-vertex K-vectors (int16 when every pair sum c(u,v) + c(v,u) fits, else
// int32), excess, residual t-links, the labels of the neighbouring boundary
// vertices and the pushes over the region's outgoing boundary arcs.
#include "mf_device.h"
#include "mf_launch.h"

namespace mfd {

typedef unsigned long long u64;

static __host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~(size_t)15; }

struct LdsLayout {
    size_t res, ex, rt, S, Q, stepEnd, stepLevel, ringIdx, halo, push, total;
};

__host__ __device__ inline LdsLayout lds_layout(int V, int K, int nring, int rtBytes) {
    LdsLayout L;
    size_t o = 0;
    L.res = o; o = al16(o + (size_t)V * K * rtBytes);
    L.ex = o; o = al16(o + (size_t)V * 4);
    L.rt = o; o = al16(o + (size_t)V * rtBytes);
    L.S = o; o = al16(o + (size_t)V * 2 + 4);
    L.Q = o; o = al16(o + (size_t)V * 2);
    L.stepEnd = o; o = al16(o + (size_t)V * 2);
    L.stepLevel = o; o = al16(o + (size_t)V * 4);
    L.ringIdx = o; o = al16(o + (size_t)V * 2);
    L.halo = o; o = al16(o + (size_t)nring * K * 4);
    L.push = o; o = al16(o + (size_t)nring * K * 4);
    L.total = o;
    return L;
}

size_t discharge_lds_bytes(int V, int K, int nring, int narrow) {
    return lds_layout(V, K, nring, narrow ? 2 : 4).total;
}

constexpr short kSInf = 0x7fff;

__device__ __forceinline__ int wmin64(int v) {
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

// Slots for n items of this lane in a queue whose tail counter is *cnt, with
// one LDS atomic per wave: an inclusive scan of n over the wave, the last lane
// reserves the wave's total.  All 64 lanes of the wave must call it.
__device__ __forceinline__ int wave_reserve(int *cnt, int n) {
    const int lane = threadIdx.x & 63;
    int x = n;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    int base = 0;
    if (lane == 63 && x > 0) base = atomicAdd(cnt, x);
    base = __shfl(base, 63, 64);
    return base + x - n;
}

// Claim S[u] (int16) for `step` if it is still unlabeled; 32-bit CAS on the
// word that holds it.  Returns true for exactly one caller.
__device__ __forceinline__ bool claim16(short *S, int u, short step) {
    unsigned *word = (unsigned *)((char *)S + ((size_t)u * 2 & ~(size_t)3));
    const int shift = (u & 1) * 16;
    unsigned old = *(volatile unsigned *)word;
    for (;;) {
        if ((short)((old >> shift) & 0xffffu) != kSInf) return false;
        unsigned nw = (old & ~(0xffffu << shift)) | ((unsigned)(unsigned short)step << shift);
        unsigned seen = atomicCAS(word, old, nw);
        if (seen == old) return true;
        old = seen;
    }
}

// Tile-local index arithmetic; P2: power-of-two extents along x and y, so
// decoding needs shifts and masks instead of integer division.
template <bool P2>
struct TileIx {
    int tx, ty, tz, sx, sxy;
    __device__ __forceinline__ void decode(int l, int &z, int &y, int &x) const {
        if (P2) {
            x = l & (tx - 1);
            y = (l >> sx) & (ty - 1);
            z = l >> sxy;
        } else {
            x = l % tx;
            const int t = l / tx;
            y = t % ty;
            z = t / ty;
        }
    }
    __device__ __forceinline__ bool inside(int z, int y, int x) const {
        return (unsigned)x < (unsigned)tx && (unsigned)y < (unsigned)ty && (unsigned)z < (unsigned)tz;
    }
};

template <int K, typename RT, int NT, bool P2>
__global__ __launch_bounds__(NT) void k_discharge_lds(DischargeArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_r, s_active, s_found, s_min;
    __shared__ int s_cnt[3];
    __shared__ int s_wmin[NT / 64];
    __shared__ long long s_tr[4];  // excess in, to sink, to boundary, label sum
    if (*A.actIn == 0ull) return;
    const int stageCap = stage_cap(A);
    const Geo &G = A.G;
    const int V = G.V, N = G.N, tid = threadIdx.x, nring = A.nring;
    const LdsLayout L = lds_layout(V, K, nring, (int)sizeof(RT));
    RT *resL = (RT *)(smem + L.res);
    int *exL = (int *)(smem + L.ex);
    RT *rtL = (RT *)(smem + L.rt);
    short *S = (short *)(smem + L.S);
    unsigned short *Q = (unsigned short *)(smem + L.Q);
    unsigned short *stepEnd = (unsigned short *)(smem + L.stepEnd);
    int *stepLevel = (int *)(smem + L.stepLevel);
    short *ringIdx = (short *)(smem + L.ringIdx);
    int *halo = (int *)(smem + L.halo);
    int *pushL = (int *)(smem + L.push);
    const int dinf = A.dinf;

    TileIx<P2> T;
    T.tx = G.tx; T.ty = G.ty; T.tz = G.tz;
    T.sx = 31 - __clz(G.tx);
    T.sxy = T.sx + (31 - __clz(G.ty));
    int dl[K];  // index offset of direction k inside the tile
#pragma unroll
    for (int k = 0; k < K; k++) dl[k] = (G.oz[k] * G.ty + G.oy[k]) * G.tx + G.ox[k];

    for (;;) {
        if (tid == 0) {
            unsigned i = atomicAdd(A.qhead, 1u);
            s_r = (i < (unsigned)A.nwork) ? A.order[i] : -1;
        }
        __syncthreads();
        const int r = s_r;
        if (r < 0) return;
        const int base = r * V;
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
            // border labels only: the interior is recomputed by the next discharge
            if (A.labNew != A.labOld)
                for (int i = tid; i < A.nring; i += NT) {
                    const int l = A.ringL[i];
                    A.labNew[base + l] = A.labOld[base + l];
                }
            __syncthreads();
            continue;
        }
        // ---------------- stage the region into LDS ----------------
        const long long t_start = wall_clock64();
        if (tid < 4) s_tr[tid] = 0;
        for (int l = tid; l < V; l += NT) {
#pragma unroll
            for (int k = 0; k < K; k++) resL[l * K + k] = (RT)A.res[(size_t)k * N + base + l];
            exL[l] = A.ex[base + l];
            rtL[l] = (RT)A.rt[base + l];
            ringIdx[l] = -1;
        }
        __syncthreads();
        for (int i = tid; i < nring; i += NT) {
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
        long long bfs_steps = 0, classes = 0, t_search = 0, t_push = 0, t_setup = 0, t_flood = 0;
        int nsteps = 0;
        // partial discharge: the searches of the push rounds stop at the stage
        // cap; the labels come from a complete search (full)
        // region relabel only (Alg. 3 on the current state, no pushes): one
        // complete search, whose labels are written
        const bool relabelOnly = s_active == 2;
        bool full = !A.partial || relabelOnly;
        bool roundCapped = false;  // the round cap was reached: one more complete search
        for (;;) {
            const long long t_round = wall_clock64();
            bool capped = false;
            // ---------------- multi-level search from the targets ----------------
            // Every thread keeps identical copies of qtail / nsteps / fs; new
            // vertices of step st are appended through counter s_cnt[st % 3], so
            // one barrier per level suffices (the counter read after a barrier is
            // not the one the next level appends to or resets).
            for (int l = tid; l < V; l += NT) S[l] = kSInf;
            if (tid == 0) {
                s_found = 0;
                s_cnt[0] = 0; s_cnt[1] = 0; s_cnt[2] = 0;
            }
            __syncthreads();
            {
                int found = 0;
                for (int l0 = 0; l0 < V; l0 += NT) {
                    const int l = l0 + tid;
                    const bool want = l < V && rtL[l] > 0;
                    const int slot = wave_reserve(&s_cnt[0], want ? 1 : 0);
                    if (want) {
                        S[l] = 0;
                        Q[slot] = (unsigned short)l;
                        found |= exL[l] > 0;
                    }
                }
                if (found) s_found = 1;
            }
            __syncthreads();
            int qtail = s_cnt[0];
            int fs = 0;
            nsteps = 0;
            int lvl = 0;
            if (qtail > 0) {
                if (tid == 0) { stepEnd[0] = (unsigned short)qtail; stepLevel[0] = 0; }
                nsteps = 1;
            }
            if (tid == 0) s_cnt[1] = 0;  // counter of step 1 (step 0 used s_cnt[0])
            __syncthreads();
            t_setup += wall_clock64() - t_round;
            for (;;) {
                // flood inside the region: u with c_f(u, v) > 0 to a frontier v
                const long long t_f0 = wall_clock64();
                while (fs < qtail) {
                    const int st = nsteps;
                    int *cnt = &s_cnt[st % 3];
                    int found = 0;
                    for (int i0 = fs; i0 < qtail; i0 += NT) {
                        const int i = i0 + tid;
                        unsigned got = 0;
                        int v = 0;
                        if (i < qtail) {
                            v = Q[i];
                            int vz, vy, vx;
                            T.decode(v, vz, vy, vx);
                            unsigned cand = 0;
#pragma unroll
                            for (int k = 0; k < K; k++) {
                                // u = v - o_k, arc (u, v) in direction k
                                if (!T.inside(vz - G.oz[k], vy - G.oy[k], vx - G.ox[k])) continue;
                                const int u = v - dl[k];
                                if (resL[u * K + k] > 0 && S[u] == kSInf) cand |= 1u << k;
                            }
                            while (cand) {
                                const int k = __ffs(cand) - 1;
                                cand &= cand - 1;
                                if (claim16(S, v - dl[k], (short)st)) got |= 1u << k;
                            }
                        }
                        int slot = qtail + wave_reserve(cnt, __popc(got));
                        while (got) {
                            const int k = __ffs(got) - 1;
                            got &= got - 1;
                            const int u = v - dl[k];
                            Q[slot++] = (unsigned short)u;
                            found |= exL[u] > 0;
                        }
                    }
                    if (found) s_found = 1;
                    if (tid == 0) s_cnt[(st + 1) % 3] = 0;
                    __syncthreads();
                    const int nnew = *cnt;
                    fs = qtail;
                    qtail += nnew;
                    if (nnew > 0) {
                        if (tid == 0) { stepEnd[st] = (unsigned short)qtail; stepLevel[st] = lvl; }
                        nsteps = st + 1;
                    }
                }
                t_flood += wall_clock64() - t_f0;
                // next stage: smallest d(w) + 1 over residual boundary arcs of unlabeled vertices
                int best = kInf;
                for (int i = tid; i < nring; i += NT) {
                    const int l = A.ringL[i];
                    if (S[l] != kSInf) continue;
#pragma unroll
                    for (int k = 0; k < K; k++) {
                        const int h = halo[i * K + k];
                        if (h < dinf && resL[l * K + k] > 0) best = min(best, h + 1);
                    }
                }
                best = wmin64(best);
                if ((tid & 63) == 0) s_wmin[tid >> 6] = best;
                __syncthreads();
                if (tid == 0) {
                    int b = kInf;
                    for (int w = 0; w < NT / 64; w++) b = min(b, s_wmin[w]);
                    s_min = b;
                }
                __syncthreads();
                const int level = s_min;
                if (level == kInf) break;
                if (!full && level > stageCap) {
                    capped = true;
                    break;
                }
                classes++;
                {
                    const int st = nsteps;
                    int *cnt = &s_cnt[st % 3];  // zero: the last flood level appended nothing to it
                    int found = 0;
                    for (int i0 = 0; i0 < nring; i0 += NT) {
                        const int i = i0 + tid;
                        bool want = false;
                        int l = 0;
                        if (i < nring) {
                            l = A.ringL[i];
                            if (S[l] == kSInf) {
#pragma unroll
                                for (int k = 0; k < K; k++) {
                                    const int h = halo[i * K + k];
                                    if (h < dinf && h + 1 == level && resL[l * K + k] > 0) want = true;
                                }
                            }
                        }
                        const int slot = qtail + wave_reserve(cnt, want ? 1 : 0);
                        if (want) {
                            S[l] = (short)st;
                            Q[slot] = (unsigned short)l;
                            found |= exL[l] > 0;
                        }
                    }
                    if (found) s_found = 1;
                    if (tid == 0) s_cnt[(st + 1) % 3] = 0;
                    __syncthreads();
                    const int nnew = *cnt;  // >= 1: the level came from an unlabeled border vertex
                    fs = qtail;
                    qtail += nnew;
                    if (tid == 0) { stepEnd[st] = (unsigned short)qtail; stepLevel[st] = level; }
                    nsteps = st + 1;
                    lvl = level;
                }
            }
            bfs_steps += nsteps;
            __syncthreads();
            const long long t_mid = wall_clock64();
            t_search += t_mid - t_round;
            if (relabelOnly) break;
            if (!s_found) {
                if (capped) {
                    full = true;  // search again, complete, for the region relabel
                    continue;
                }
                break;
            }
            if (full && (A.partial || roundCapped)) {
                // complete search after capped rounds: the excess it reaches lies
                // beyond the cap and stays; the region stays active
                if (tid == 0) {
                    A.ractive[r] = 1;
                    atomicAdd(A.actCarry, 1ull);
                }
                break;
            }
            if (++iter > A.maxIter) {
                if (tid == 0) atomicOr(A.err, 4);
                break;
            }
            if (A.roundCap > 0 && iter > A.roundCap) {
                roundCapped = true;  // search once more, complete, for the region relabel
                full = true;
                continue;
            }
            // ---------------- push excess down the search levels ----------------
            for (int s = nsteps - 1; s >= 0; s--) {
                const int lo = s > 0 ? stepEnd[s - 1] : 0, hi = stepEnd[s];
                const int Lv = stepLevel[s];
                const bool seed = (s == 0) || (stepLevel[s - 1] != Lv);
                for (int i = lo + tid; i < hi; i += NT) {
                    const int u = Q[i];
                    int e = exL[u];
                    if (e <= 0) continue;
                    if (seed) {
                        if (Lv == 0) {
                            const int t = rtL[u];
                            if (t > 0) {
                                const int d = min(e, t);
                                rtL[u] = (RT)(t - d);
                                e -= d;
                                if (A.trace) atomicAdd((unsigned long long *)&s_tr[1], (u64)d);
                            }
                        } else {
                            // stage seeds are border vertices; ri >= 0
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
                        int uz, uy, ux;
                        T.decode(u, uz, uy, ux);
                        int cap[K];
                        unsigned adm = 0;
#pragma unroll
                        for (int k = 0; k < K; k++) {
                            cap[k] = 0;
                            if (!T.inside(uz + G.oz[k], uy + G.oy[k], ux + G.ox[k])) continue;
                            const int v = u + dl[k];
                            cap[k] = resL[u * K + k];
                            if (cap[k] > 0 && S[v] == s - 1) adm |= 1u << k;
                        }
#pragma unroll
                        for (int k = 0; k < K; k++) {
                            if (!((adm >> k) & 1u) || e <= 0) continue;
                            const int v = u + dl[k];
                            const int d = min(e, cap[k]);
                            resL[u * K + k] = (RT)(cap[k] - d);
                            resL[v * K + (k ^ 1)] = (RT)(resL[v * K + (k ^ 1)] + d);
                            atomicAdd(&exL[v], d);
                            e -= d;
                        }
                    }
                    exL[u] = e;
                }
                __syncthreads();
            }
            t_push += wall_clock64() - t_mid;
        }
        // ---------------- write the region back ----------------
        for (int l = tid; l < V; l += NT) {
#pragma unroll
            for (int k = 0; k < K; k++) A.res[(size_t)k * N + base + l] = resL[l * K + k];
            A.ex[base + l] = exL[l];
            A.rt[base + l] = rtL[l];
            const int s = S[l];
            A.labNew[base + l] = (s == kSInf) ? dinf : min(stepLevel[s], dinf);
        }
        for (int i = tid; i < nring; i += NT) {
            const int l = A.ringL[i];
#pragma unroll
            for (int k = 0; k < K; k++) {
                const int p = pushL[i * K + k];
                if (p) A.pushb[(size_t)k * N + base + l] = p;
            }
        }
        if (A.trace) {
            // excess in = excess out + flow to t + flow over boundary arcs
            long long ex_out = 0, to_b = 0, lsum = 0;
            for (int l = tid; l < V; l += NT) ex_out += exL[l];
            for (int i = tid; i < nring; i += NT) {
#pragma unroll
                for (int k = 0; k < K; k++) to_b += pushL[i * K + k];
                const int s = S[A.ringL[i]];
                lsum += (s == kSInf) ? 65535 : min(stepLevel[s], 65535);
            }
            atomicAdd((unsigned long long *)&s_tr[0], (u64)ex_out);
            atomicAdd((unsigned long long *)&s_tr[2], (u64)to_b);
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
            atomicAdd(&A.stats[3], (u64)bfs_steps);
            atomicAdd(&A.stats[4], (u64)classes);
            atomicAdd(&A.stats[6], (u64)t_search);
            atomicAdd(&A.stats[7], (u64)t_push);
            atomicAdd(&A.stats[8], (u64)t_setup);
            atomicAdd(&A.stats[9], (u64)t_flood);
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

template <int K, typename RT>
static void set_attr_k() {
    (void)hipFuncSetAttribute((const void *)k_discharge_lds<K, RT, 512, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute((const void *)k_discharge_lds<K, RT, 512, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

void set_lds_attributes() {
    set_attr_k<4, short>(); set_attr_k<6, short>(); set_attr_k<8, short>();
    set_attr_k<4, int>(); set_attr_k<6, int>(); set_attr_k<8, int>();
    (void)hipGetLastError();
}

template <int K, typename RT, bool P2>
static hipError_t launch_lds_t(const DischargeArgs &A, int blocks, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_discharge_lds<K, RT, 512, P2>), dim3(blocks), dim3(512), lds, s, A);
    return hipGetLastError();
}

template <int K, typename RT>
static hipError_t launch_lds_k(const DischargeArgs &A, int blocks, size_t lds, hipStream_t s) {
    const int tx = A.G.tx, ty = A.G.ty;
    const bool p2 = (tx & (tx - 1)) == 0 && (ty & (ty - 1)) == 0;
    return p2 ? launch_lds_t<K, RT, true>(A, blocks, lds, s) : launch_lds_t<K, RT, false>(A, blocks, lds, s);
}

hipError_t launch_discharge_lds(const DischargeArgs &A, int blocks, size_t lds, int narrow,
                                hipStream_t s) {
    const int K = A.G.K;
    if (narrow) {
        if (K == 4) return launch_lds_k<4, short>(A, blocks, lds, s);
        if (K == 6) return launch_lds_k<6, short>(A, blocks, lds, s);
        if (K == 8) return launch_lds_k<8, short>(A, blocks, lds, s);
    } else {
        if (K == 4) return launch_lds_k<4, int>(A, blocks, lds, s);
        if (K == 6) return launch_lds_k<6, int>(A, blocks, lds, s);
        if (K == 8) return launch_lds_k<8, int>(A, blocks, lds, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace mfd
