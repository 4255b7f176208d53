// General networks in region pages (Sec. 5.3): the splitter, parallel region
// discharge (Alg. 2 with Proc. ARD and the region relabel of Alg. 3) over the
// pages, with the pages either all resident in HBM or streamed through a fixed
// number of device page slots, and the two extremal cuts.
//
// The splitter numbers the vertices region by region and writes one page per
// region: its arcs in compressed rows with 32-bit offsets inside the page, and
// its part of the preflow state.  Pairs whose ends lie in different regions
// are withheld from the pages into a resident boundary table (the shared part
// of Sec. 5.3: O(|B| + |(B, B)|)); a page refers to them by index.  Every
// kernel below reads and writes only its own region's page and the resident
// boundary table, so a region page is the unit of transfer between host and
// device memory.
//
// Page of a region with nv vertices and na arcs (int32 words):
//   off[nv + 1]  arc range of each local vertex
//   head[na]     local head vertex, or -(x + 1) for boundary arc x (below)
//   rev[na]      local index of the reverse arc (-1 for boundary arcs)
//   gid[nv]      the vertex's number in the caller's network
//   -- state (written back when a streamed page leaves the device) --
//   res[na]      residual capacity of an arc inside the region
//   rres[na]     residual capacity of its reverse arc (res[rev[a]], kept beside
//                the arc so that a backward search reads it with the head)
//   ex[nv], rt[nv], lab[nv], mk[nv]  excess, residual t-link, label, cut mark
//
// Boundary table: boundary vertices get slots numbered region by region; pair
// c across two regions owns arcs x = 2c (first to second end) and 2c + 1;
// cr[x] is the arc's residual, cp[x] the flow a discharge of its tail's region
// sent over it in this sweep, cslot[x] the boundary slot of its tail.  labB
// (two buffers) holds the boundary labels, exIn the excess the flow fusion
// delivered to a boundary vertex and no discharge has taken in yet.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "mf.h"
#include "mf_device.h"
#include "mf_launch.h"

namespace mfg {

using mfd::kInf;
typedef unsigned long long u64;

struct Layout {
    int off, head, rev, gid, res, rres, ex, rt, lab, mk, words;
};

__host__ __device__ inline Layout layout_of(int nv, int na) {
    Layout L;
    L.off = 0;
    L.head = nv + 1;
    L.rev = L.head + na;
    L.gid = L.rev + na;
    L.res = L.gid + nv;
    L.rres = L.res + na;
    L.ex = L.rres + na;
    L.rt = L.ex + nv;
    L.lab = L.rt + nv;
    L.mk = L.lab + nv;
    L.words = L.mk + nv;
    return L;
}

struct Args {
    int *pool;          // device page slots
    long long stride;   // words per slot
    const int4 *rinfo;  // per region: nv, na, first boundary slot, boundary count
    const int *blocal;  // boundary slot -> local vertex of its region
    const int *labOld;  // boundary labels of the previous sweep
    int *labNew;        // boundary labels written by this sweep
    int *exIn;
    int *cr, *cp;
    const int *cslot;
    const int *order;   // regions to process: order[listLo ..]
    const int *cnt;     // their number, when listN < 0
    int listLo, listN;
    int slotBase;       // < 0: region r lives in slot r; else the i-th region in slot slotBase + i
    unsigned *qhead;
    int *scratch;       // kScratchInts * nvmax ints per workgroup
    int nvmax;
    int dinf, maxIter;
    int *err;
    u64 *stats;         // [0] discharges [1] push rounds [2] search steps [3] vertices [4] arcs
    const u64 *actIn;
    int roundCap;       // > 0: at most this many push rounds per discharge and sweep
    u64 *actCarry;      // regions a capped discharge left active (counted into the next sweep)
    int *ractive;       // region flags of the next sweep
    int mode;           // flood: 0 = backward from t, 1 = forward from the excess
    int first;          // flood: first round
    int *markB;         // flood marks of the boundary vertices
    unsigned *changed;
    unsigned char *cut; // cut output, indexed by the caller's vertex numbers
    u64 *sum;
};

__device__ __forceinline__ int wsum(int v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ int wmin(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

// Takes the next region of the list; its slot into *slot.  Block-uniform.
template <int NT>
__device__ __forceinline__ int next_region(const Args &A, int *s_r, int *s_slot) {
    if (threadIdx.x == 0) {
        const unsigned i = atomicAdd(A.qhead, 1u);
        const int n = A.listN >= 0 ? A.listN : *A.cnt;
        const int r = (i < (unsigned)n) ? A.order[A.listLo + (int)i] : -1;
        *s_r = r;
        *s_slot = A.slotBase < 0 ? r : A.slotBase + (int)i;
    }
    __syncthreads();
    return *s_r;
}

// Sums and minima over a group of G consecutive lanes (G divides 64).
template <int G>
__device__ __forceinline__ long long gscan(long long x, int lane) {
    for (int o = 1; o < G; o <<= 1) {
        const long long y = __shfl_up(x, o, G);
        if (lane >= o) x += y;
    }
    return x;
}
template <int G>
__device__ __forceinline__ int gmin(int x) {
    for (int o = G / 2; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, G));
    return x;
}

constexpr int kScratchInts = 6;  // per vertex of the largest region, per workgroup

// ---------------------------------------------------------------------------
// Region discharge, Proc. ARD (Sec. 4.2) on a region page.  As on grids, the
// staged Augment(R, T_k) runs as pushes along the levels of a multi-level
// breadth-first search from the targets: t first (stage 0), then the boundary
// arcs to vertices w of other regions in increasing d(w) + 1 (stage k).  A
// vertex's stage is the smallest k with a residual path to T_k, and the last
// (complete) search gives the labels of the region relabel (Alg. 3).  Search
// and push rounds alternate until no excess vertex of the region reaches a
// target.  Arcs from other regions into R are not used (capacity 0 in G^R);
// flow sent over a boundary arc waits in cp for the fusion.
//
// A group of G lanes takes one vertex and its arcs G at a time: in the search
// every lane tests one arc; in a push the lanes split the vertex's excess over
// its admissible arcs in arc order by a prefix sum of their capacities.  The
// search marks S, the queue Q, the smallest halo level M of every boundary
// vertex (fixed during a search) and the row offsets live in LDS when the
// region fits (LDS), else in per-workgroup scratch.
// ---------------------------------------------------------------------------
template <int NT, int G, bool LDS>
__global__ __launch_bounds__(NT) void k_gdischarge(Args A) {
    extern __shared__ int smem[];
    __shared__ int s_r, s_slot, s_qtail, s_fe, s_nsteps, s_min, s_found, s_live, s_hit, s_stop;
    __shared__ int s_wmin[NT / 64];
    constexpr int kDead = kInf - 1;  // not reached by a complete search of this discharge
    constexpr int NG = NT / G;
    if (*A.actIn == 0ull) return;
    const int tid = threadIdx.x, lane = tid % G, grp = tid / G;
    const int nvmax = A.nvmax;
    int *gs = A.scratch + (size_t)blockIdx.x * kScratchInts * nvmax;
    int *stepEnd = gs, *stepLevel = gs + nvmax;
    int *S, *Q, *M, *offL;
    unsigned *XB;  // excess vertices at the start of the search, one bit each
    if (LDS) {
        S = smem;
        Q = S + nvmax;
        M = Q + nvmax;
        offL = M + nvmax;
        XB = (unsigned *)(offL + nvmax + 1);
    } else {
        S = gs + 2 * nvmax;
        Q = gs + 3 * nvmax;
        M = gs + 4 * nvmax;
        offL = nullptr;
        XB = (unsigned *)(gs + 5 * nvmax);
    }
    const int dinf = A.dinf;
    const int *labOld = A.labOld, *cslot = A.cslot, *blocal = A.blocal;
    int *cr = A.cr, *cp = A.cp;
    for (;;) {
        const int r = next_region<NT>(A, &s_r, &s_slot);
        if (r < 0) return;
        const int4 info = A.rinfo[r];
        const int nv = info.x, na = info.y, b0 = info.z, nb = info.w;
        const Layout L = layout_of(nv, na);
        int *P = A.pool + (long long)s_slot * A.stride;
        const int *head = P + L.head, *rev = P + L.rev;
        int *res = P + L.res, *rres = P + L.rres, *ex = P + L.ex, *rt = P + L.rt, *lab = P + L.lab;
        const int *off = P + L.off;
        if (LDS) {
            for (int l = tid; l <= nv; l += NT) offL[l] = off[l];
            off = offL;
        }
        for (int i = tid; i < nb; i += NT) {
            const int e = A.exIn[b0 + i];
            if (e) {
                ex[blocal[b0 + i]] += e;
                A.exIn[b0 + i] = 0;
            }
        }
        __syncthreads();
        long long iter = 0, steps = 0;
        bool firstSearch = true, lastComplete = false;
        // round cap: after roundCap push rounds one more complete search writes
        // the region relabel on the current state; excess it still finds reaching
        // a target stays in the region, which stays active
        bool finalSearch = false;
        for (;;) {
            bool early = false;
            if (tid == 0) {
                s_qtail = 0;
                s_nsteps = 0;
                s_found = 0;
                s_live = 0;
                s_hit = 0;
            }
            __syncthreads();
            // first level (c_f(u, t) > 0), dead marks, live excess count, and the
            // excess bitmap (the excess does not change during a search)
            for (int i = tid; i < (nv + 31) / 32; i += NT) XB[i] = 0u;
            __syncthreads();
            int live = 0, hit = 0;
            for (int l = tid; l < nv; l += NT) {
                const int prev = firstSearch ? kInf : S[l];
                const bool dead = prev == kDead || (lastComplete && prev == kInf);
                const bool hasEx = ex[l] > 0;
                if (hasEx) atomicOr(&XB[l >> 5], 1u << (l & 31));
                const bool lv = !dead && hasEx;
                if (!dead && rt[l] > 0) {
                    S[l] = 0;
                    Q[atomicAdd(&s_qtail, 1)] = l;
                    hit |= lv ? 1 : 0;
                } else {
                    S[l] = dead ? kDead : kInf;
                    live += lv ? 1 : 0;
                }
            }
            live = wsum(live);
            if ((tid & 63) == 0 && live) atomicAdd(&s_live, live);
            if (hit) s_hit = 1;
            // every boundary vertex: the smallest d(w) + 1 over its residual boundary arcs
            for (int i = grp; i < nb; i += NG) {
                const int l = blocal[b0 + i];
                int best = kInf;
                const int a1 = off[l + 1];
                for (int a = off[l] + lane; a < a1; a += G) {
                    const int h = head[a];
                    if (h >= 0) continue;
                    const int x = -h - 1;
                    if (cr[x] <= 0) continue;
                    const int d = labOld[cslot[x ^ 1]];
                    if (d < dinf) best = min(best, d + 1);
                }
                best = gmin<G>(best);
                if (lane == 0) M[i] = best;
            }
            __syncthreads();
            if (tid == 0) {
                if (s_qtail > 0) {
                    stepEnd[0] = s_qtail;
                    stepLevel[0] = 0;
                    s_nsteps = 1;
                }
                s_fe = s_qtail;
                s_stop = !finalSearch && s_hit && s_live == 0;
            }
            __syncthreads();
            int fs = 0;
            for (;;) {
                // breadth-first levels inside the region: u joins when c_f(u, v) > 0
                // for a frontier vertex v
                for (;;) {
                    const int fe = s_fe;
                    if (s_stop) {
                        early = true;  // every live excess vertex has a level
                        break;
                    }
                    if (fs == fe) break;
                    const int step = s_nsteps;
                    // u joins the level through arc a = (v, u) when c_f(u, v) > 0
                    auto visit = [&](int u, int c) {
                        if (u < 0 || c <= 0 || S[u] != kInf) return;
                        if (atomicCAS(&S[u], kInf, step) == kInf) {
                            Q[atomicAdd(&s_qtail, 1)] = u;
                            if ((XB[u >> 5] >> (u & 31)) & 1u) {
                                atomicSub(&s_live, 1);
                                s_hit = 1;
                            }
                        }
                    };
                    // two frontier vertices per group, their first G arcs loaded together
                    for (int i = fs + grp; i < fe; i += 2 * NG) {
                        const int v0 = Q[i], v1 = i + NG < fe ? Q[i + NG] : -1;
                        const int b0 = off[v0], e0 = off[v0 + 1];
                        const int b1 = v1 >= 0 ? off[v1] : 0, e1 = v1 >= 0 ? off[v1 + 1] : 0;
                        int u0 = -1, c0 = 0, u1 = -1, c1 = 0;
                        if (b0 + lane < e0) {
                            u0 = head[b0 + lane];
                            c0 = rres[b0 + lane];
                        }
                        if (b1 + lane < e1) {
                            u1 = head[b1 + lane];
                            c1 = rres[b1 + lane];
                        }
                        visit(u0, c0);
                        visit(u1, c1);
                        for (int a = b0 + G + lane; a < e0; a += G) visit(head[a], rres[a]);
                        for (int a = b1 + G + lane; a < e1; a += G) visit(head[a], rres[a]);
                    }
                    __syncthreads();
                    if (tid == 0) {
                        if (s_qtail > fe) {
                            stepEnd[step] = s_qtail;
                            stepLevel[step] = step > 0 ? stepLevel[step - 1] : 0;
                            s_nsteps = step + 1;
                        }
                        s_fe = s_qtail;
                        s_stop = !finalSearch && s_hit && s_live == 0;
                    }
                    fs = fe;
                    __syncthreads();
                }
                if (early) break;
                // next stage: the smallest halo level of a boundary vertex without a level
                int best = kInf;
                for (int i = tid; i < nb; i += NT)
                    if (S[blocal[b0 + i]] == kInf) best = min(best, M[i]);
                best = wmin(best);
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
                const int step = s_nsteps;
                for (int i = tid; i < nb; i += NT) {
                    const int l = blocal[b0 + i];
                    if (S[l] != kInf || M[i] != level) continue;
                    S[l] = step;
                    Q[atomicAdd(&s_qtail, 1)] = l;
                    if ((XB[l >> 5] >> (l & 31)) & 1u) {
                        atomicSub(&s_live, 1);
                        s_hit = 1;
                    }
                }
                __syncthreads();
                if (tid == 0) {
                    stepEnd[step] = s_qtail;  // level came from a vertex without a level: one seed at least
                    stepLevel[step] = level;
                    s_nsteps = step + 1;
                    s_fe = s_qtail;
                    s_stop = !finalSearch && s_hit && s_live == 0;
                }
                __syncthreads();
            }
            steps += s_nsteps;
            firstSearch = false;
            lastComplete = !early;
            // does an excess vertex reach a target?
            int found = early ? 1 : 0;
            if (!early)
                for (int l = tid; l < nv; l += NT)
                    if (S[l] < kDead && ex[l] > 0) found = 1;
            if (found) s_found = 1;
            __syncthreads();
            if (!s_found) break;
            if (finalSearch) {
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
            // push the excess down the levels, the last level first
            const int nsteps = s_nsteps;
            for (int s = nsteps - 1; s >= 0; s--) {
                const int lo = s > 0 ? stepEnd[s - 1] : 0, hi = stepEnd[s];
                const int Lv = stepLevel[s];
                const bool seed = s == 0 || stepLevel[s - 1] != Lv;
                for (int i = lo + grp; i < hi; i += NG) {
                    const int u = Q[i];
                    int e = ex[u];
                    if (e <= 0) continue;  // uniform over the group
                    if (seed && Lv == 0) {
                        if (lane == 0) {
                            const int t = rt[u];
                            const int d = min(e, t);
                            rt[u] = t - d;
                            ex[u] = e - d;
                        }
                        continue;
                    }
                    const int a1 = off[u + 1];
                    for (int base = off[u]; base < a1 && e > 0; base += G) {
                        const int a = base + lane;
                        int c = 0, x = -1, h = -1;
                        if (a < a1) {
                            h = head[a];
                            if (seed) {
                                if (h < 0) {
                                    x = -h - 1;
                                    const int cc = cr[x];
                                    if (cc > 0) {
                                        const int dw = labOld[cslot[x ^ 1]];
                                        if (dw < dinf && dw + 1 == Lv) c = cc;
                                    }
                                }
                            } else if (h >= 0) {
                                const int cc = res[a];
                                if (cc > 0 && S[h] == s - 1) c = cc;
                            }
                        }
                        // the lanes take the excess in arc order
                        const long long incl = gscan<G>((long long)c, lane);
                        const long long before = incl - c;
                        const int d = (int)std::min<long long>(c, std::max<long long>(0, (long long)e - before));
                        if (d > 0) {
                            if (seed) {
                                cr[x] -= d;
                                cp[x] += d;
                            } else {
                                const int ra = rev[a];
                                res[a] -= d;
                                rres[a] += d;
                                res[ra] += d;
                                rres[ra] -= d;
                                atomicAdd(&ex[h], d);
                            }
                        }
                        const long long tot = __shfl(incl, G - 1, G);
                        e -= (int)std::min<long long>(e, tot);
                    }
                    if (lane == 0) ex[u] = e;
                }
                __syncthreads();
            }
            if (A.roundCap > 0 && iter >= A.roundCap) finalSearch = true;
        }
        // region relabel (Alg. 3): a vertex's label is its stage, d_inf without one
        for (int l = tid; l < nv; l += NT) {
            const int s = S[l];
            lab[l] = (s >= kDead) ? dinf : min(stepLevel[s], dinf);
        }
        __syncthreads();
        for (int i = tid; i < nb; i += NT) A.labNew[b0 + i] = lab[blocal[b0 + i]];
        if (tid == 0) {
            atomicAdd(&A.stats[0], 1ull);
            atomicAdd(&A.stats[1], (u64)(iter + 1));
            atomicAdd(&A.stats[2], (u64)steps);
            atomicAdd(&A.stats[3], (u64)nv);
            atomicAdd(&A.stats[4], (u64)na);
        }
        __syncthreads();
    }
}

// Labels of boundary vertices whose region is not discharged this sweep carry
// over; also resets the region list of the sweep.
__global__ void k_gcarry(const int *ractive, const int *bregion, const int *labOld, int *labNew, int nB,
                         int *cnt, unsigned *qhead, const u64 *actIn) {
    if (*actIn == 0ull) return;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b == 0) {
        *cnt = 0;
        *qhead = 0u;
    }
    if (b < nB && !ractive[bregion[b]]) labNew[b] = labOld[b];
}

// The regions to discharge this sweep: those with an active vertex.
__global__ void k_gqueue(int *ractive, int K, int *order, int *cnt, const u64 *actIn) {
    if (*actIn == 0ull) return;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < K && ractive[r]) {
        order[atomicAdd(cnt, 1)] = r;
        ractive[r] = 0;
    }
}

// Flow fusion of Alg. 2 on the boundary pairs: a push u -> v stays iff
// d'(v) <= d'(u) + 1, otherwise it returns to u.  The flow that stays or
// returns becomes excess of a boundary vertex through exIn.
__global__ void k_gfuse(int *cr, int *cp, const int *cslot, const int *lab, int *exIn, long long nC,
                        const u64 *actIn) {
    if (*actIn == 0ull) return;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nC) return;
    const long long x0 = 2 * c, x1 = x0 + 1;
    const int p0 = cp[x0], p1 = cp[x1];
    if ((p0 | p1) == 0) return;
    const int bu = cslot[x0], bv = cslot[x1];
    const int du = lab[bu], dv = lab[bv];
    cp[x0] = 0;
    cp[x1] = 0;
    if (p0) {
        if (dv <= du + 1) {
            cr[x1] += p0;
            atomicAdd(&exIn[bv], p0);
        } else {
            cr[x0] += p0;
            atomicAdd(&exIn[bu], p0);
        }
    }
    if (p1) {
        if (du <= dv + 1) {
            cr[x0] += p1;
            atomicAdd(&exIn[bu], p1);
        } else {
            cr[x1] += p1;
            atomicAdd(&exIn[bv], p1);
        }
    }
}

// Global gap (Sec. 5.1) on the boundary labels, then the activity of the next
// sweep: after a complete discharge only boundary vertices that received flow
// can be active.
__global__ void k_gapply(int *lab, const int *exIn, const int *bregion, int *ractive, int nB,
                         const int *gap, int dinf, u64 *actOut, const u64 *actIn) {
    __shared__ int s_w[4];
    if (*actIn == 0ull) return;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    int act = 0;
    if (b < nB) {
        int d = lab[b];
        const int g = *gap;
        if (g >= 0 && d > g && d < dinf) {
            d = dinf;
            lab[b] = d;
        }
        if (exIn[b] > 0 && d < dinf) {
            act = 1;
            ractive[bregion[b]] = 1;
        }
    }
    act = wsum(act);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = act;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int t = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        if (t) atomicAdd(actOut, (u64)t);
    }
}

// Residual reachability inside a region page, one round: mode 0 marks the
// vertices with a residual path to t (backward search), mode 1 the vertices an
// excess vertex reaches (forward search).  Paths that cross regions go through
// the boundary marks; rounds repeat until no boundary mark changes.
template <int NT>
__global__ __launch_bounds__(NT) void k_gflood(Args A) {
    __shared__ int s_r, s_slot, s_qtail, s_fe;
    const int tid = threadIdx.x;
    int *Q = A.scratch + (size_t)blockIdx.x * kScratchInts * A.nvmax;
    const int *cslot = A.cslot, *blocal = A.blocal;
    const int *cr = A.cr;
    const bool back = A.mode == 0;
    for (;;) {
        const int r = next_region<NT>(A, &s_r, &s_slot);
        if (r < 0) return;
        const int4 info = A.rinfo[r];
        const int nv = info.x, na = info.y, b0 = info.z, nb = info.w;
        const Layout L = layout_of(nv, na);
        int *P = A.pool + (long long)s_slot * A.stride;
        const int *off = P + L.off, *head = P + L.head;
        const int *res = P + L.res, *rres = P + L.rres, *ex = P + L.ex, *rt = P + L.rt;
        int *mk = P + L.mk;
        if (tid == 0) s_qtail = 0;
        __syncthreads();
        if (A.first) {
            for (int l = tid; l < nv; l += NT) {
                const int m = back ? (rt[l] > 0) : (ex[l] > 0);
                mk[l] = m;
                if (m) Q[atomicAdd(&s_qtail, 1)] = l;
            }
            __syncthreads();
            if (!back)  // excess the fusion delivered and no discharge took in yet
                for (int i = tid; i < nb; i += NT) {
                    const int l = blocal[b0 + i];
                    if (A.exIn[b0 + i] > 0 && atomicCAS(&mk[l], 0, 1) == 0) Q[atomicAdd(&s_qtail, 1)] = l;
                }
        }
        __syncthreads();
        // boundary vertices joined by a residual boundary arc to a marked vertex
        for (int i = tid; i < nb; i += NT) {
            const int l = blocal[b0 + i];
            if (mk[l]) continue;
            const int a1 = off[l + 1];
            for (int a = off[l]; a < a1; a++) {
                const int h = head[a];
                if (h >= 0) continue;
                const int x = -h - 1;
                const int c = back ? cr[x] : cr[x ^ 1];
                if (c > 0 && A.markB[cslot[x ^ 1]]) {
                    if (atomicCAS(&mk[l], 0, 1) == 0) Q[atomicAdd(&s_qtail, 1)] = l;
                    break;
                }
            }
        }
        __syncthreads();
        if (tid == 0) s_fe = s_qtail;
        __syncthreads();
        int fs = 0;
        for (;;) {
            const int fe = s_fe;
            if (fs == fe) break;
            for (int i = fs + tid; i < fe; i += NT) {
                const int v = Q[i];
                const int a1 = off[v + 1];
                for (int a = off[v]; a < a1; a++) {
                    const int w = head[a];
                    if (w < 0 || mk[w]) continue;
                    const int c = back ? rres[a] : res[a];
                    if (c > 0 && atomicCAS(&mk[w], 0, 1) == 0) Q[atomicAdd(&s_qtail, 1)] = w;
                }
            }
            __syncthreads();
            if (tid == 0) s_fe = s_qtail;
            fs = fe;
            __syncthreads();
        }
        int ch = 0;
        for (int i = tid; i < nb; i += NT)
            if (mk[blocal[b0 + i]] && !A.markB[b0 + i]) {
                A.markB[b0 + i] = 1;
                ch = 1;
            }
        if (ch) atomicOr(A.changed, 1u);
        __syncthreads();
    }
}

// Per region page: the cut side of every vertex (mode 0: the maximal source
// side, the vertices without a mark; mode 1: the minimal one, the marked
// vertices), and the sum of the residual t-links.
template <int NT>
__global__ __launch_bounds__(NT) void k_gcollect(Args A) {
    __shared__ int s_r, s_slot;
    __shared__ long long s_w[NT / 64];
    const int tid = threadIdx.x;
    for (;;) {
        const int r = next_region<NT>(A, &s_r, &s_slot);
        if (r < 0) return;
        const int4 info = A.rinfo[r];
        const int nv = info.x, na = info.y;
        const Layout L = layout_of(nv, na);
        const int *P = A.pool + (long long)s_slot * A.stride;
        const int *gid = P + L.gid, *rt = P + L.rt, *mk = P + L.mk;
        long long t = 0;
        for (int l = tid; l < nv; l += NT) {
            if (A.cut) A.cut[gid[l]] = (unsigned char)(A.mode == 0 ? !mk[l] : (mk[l] != 0));
            t += rt[l];
        }
        for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
        if ((tid & 63) == 0) s_w[tid >> 6] = t;
        __syncthreads();
        if (tid == 0) {
            long long s = 0;
            for (int w = 0; w < NT / 64; w++) s += s_w[w];
            if (s) atomicAdd(A.sum, (u64)s);
        }
        __syncthreads();
    }
}

constexpr int kNT = 512;    // floods and collection
constexpr int kDNT = 1024;  // discharge: a few regions at a time are active, each gets a whole compute unit

}  // namespace mfg

// ---------------------------------------------------------------------------
// Host side: the splitter, page transfers, the sweep driver.
// ---------------------------------------------------------------------------
using mfg::Layout;
using mfg::layout_of;
typedef unsigned long long u64;

struct mf_graph {
    int device = 0, numCU = 0;
    int32_t n = 0;
    int64_t np = 0;
    int K = 0;
    int nB = 0;
    long long nC = 0;
    int dinf = 1;
    int nvmax = 0;
    long long stride = 0;  // words per page slot
    int P = 0;             // device page slots
    bool resident = true;
    int half = 0;          // streamed: regions per transfer batch
    int nhalves = 1;       // streamed: 2 alternating halves of the slots (1 with a single slot)
    int blocks = 1;        // workgroups of the page kernels
    std::vector<int4> rinfo;
    std::vector<long long> pair_loc;  // >= 0: (region << 32) | local arc of pu -> pv; < 0: ~cross pair
    std::vector<int> blocal_h;
    int *hpages = nullptr;            // streamed: pinned host page store, region r at r * stride
    // device
    int *pool = nullptr, *blocal = nullptr, *bregion = nullptr, *lab[2] = {nullptr, nullptr};
    int4 *drinfo = nullptr;
    int *exIn = nullptr, *cr = nullptr, *cp = nullptr, *cslot = nullptr, *order = nullptr;
    int *allreg = nullptr, *cnt = nullptr, *ractive = nullptr, *scratch = nullptr, *markB = nullptr;
    int *err = nullptr, *maxlab = nullptr, *gap = nullptr;
    unsigned *qhead = nullptr, *changed = nullptr, *hist = nullptr;
    u64 *act = nullptr, *counters = nullptr, *stats = nullptr, *sum = nullptr;
    u64 *carry = nullptr;             // regions left active by capped discharges, per sweep
    int roundCap = 0;                 // push rounds per discharge and sweep, 0: no cap
    unsigned char *cutbuf = nullptr;
    void *pinned = nullptr;           // mailbox: [0..7] words, then the region list
    hipStream_t s = nullptr, sc = nullptr, sd = nullptr;  // solve, page loads, page write-backs
    hipEvent_t evLoad[2] = {nullptr, nullptr}, evComp[2] = {nullptr, nullptr}, evWB[2] = {nullptr, nullptr};
    long long sum_ct = 0, flow = 0;
    long long sweeps = 0;
    int cur = 0;                      // lab[cur] holds the current boundary labels
    int cut_cached = -1;
    bool solved = false;
    long long pages_in = 0, pages_out = 0, bytes_h2d = 0, bytes_d2h = 0;
    int group = 8;                    // lanes per vertex in the discharge (8 or 32, from the mean degree)
    size_t ldsBytes = 0;              // dynamic LDS of the discharge, 0: search arrays in scratch
    bool profile = false;             // time every discharge launch with HIP events
    std::vector<hipEvent_t> evProf;   // start and end event per launch
    size_t nprof = 0;
};

namespace {

bool ok(hipError_t e) { return e == hipSuccess; }
#define GTRY(x)                          \
    do {                                 \
        if (!ok(x)) return MF_E_DEVICE;  \
    } while (0)

template <typename T>
hipError_t dalloc(T **p, size_t count) {
    if (count == 0) count = 1;
    return hipMalloc((void **)p, count * sizeof(T));
}

void free_graph(mf_graph *g) {
    void *d[] = {g->pool, g->blocal, g->bregion, g->lab[0], g->lab[1], g->drinfo, g->exIn, g->cr,
                 g->cp, g->cslot, g->order, g->allreg, g->cnt, g->ractive, g->scratch, g->markB,
                 g->err, g->maxlab, g->gap, g->qhead, g->changed, g->hist, g->act, g->counters,
                 g->stats, g->sum, g->carry, g->cutbuf};
    for (void *p : d)
        if (p) (void)hipFree(p);
    if (g->hpages) (void)hipHostFree(g->hpages);
    if (g->pinned) (void)hipHostFree(g->pinned);
    for (hipEvent_t e : g->evProf) (void)hipEventDestroy(e);
    for (int h = 0; h < 2; h++) {
        if (g->evLoad[h]) (void)hipEventDestroy(g->evLoad[h]);
        if (g->evComp[h]) (void)hipEventDestroy(g->evComp[h]);
        if (g->evWB[h]) (void)hipEventDestroy(g->evWB[h]);
    }
    if (g->s) (void)hipStreamDestroy(g->s);
    if (g->sc) (void)hipStreamDestroy(g->sc);
    if (g->sd) (void)hipStreamDestroy(g->sd);
}

int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }

mfg::Args base_args(mf_graph *g) {
    mfg::Args A;
    memset(&A, 0, sizeof(A));
    A.pool = g->pool;
    A.stride = g->stride;
    A.rinfo = g->drinfo;
    A.blocal = g->blocal;
    A.exIn = g->exIn;
    A.cr = g->cr;
    A.cp = g->cp;
    A.cslot = g->cslot;
    A.scratch = g->scratch;
    A.nvmax = std::max(g->nvmax, 1);
    A.dinf = g->dinf;
    A.maxIter = 1 << 18;
    A.err = g->err;
    A.stats = g->stats;
    A.markB = g->markB;
    A.changed = g->changed;
    A.sum = g->sum;
    A.slotBase = -1;
    A.listN = -1;
    A.roundCap = g->roundCap;
    A.actCarry = g->carry;
    A.ractive = g->ractive;
    return A;
}

// Runs a page kernel over a list of regions.  Resident pages: one launch over
// the device list (order, count on the device).  Streamed pages: the host list
// `list` (n regions) in batches of g->half regions, alternating between the
// two halves of the page slots (a single slot is one half), with the next
// batch's pages loaded on one copy stream while the current batch runs, and
// the state part of each page written back after its kernel on another (when
// `writeBack`), so that the two directions of the link overlap.
template <class Launch>
mf_status page_pass(mf_graph *g, const int *dlist, const int *hlist, int n, bool writeBack,
                    Launch launch) {
    if (g->resident) {
        GTRY(hipMemsetAsync(g->qhead, 0, sizeof(unsigned), g->s));
        GTRY(launch(dlist, 0, n, -1, g->s));
        return MF_OK;
    }
    int pending[2] = {0, 0};          // regions of the last batch on each half
    int pendLo[2] = {0, 0};
    const int nb = (n + g->half - 1) / g->half;
    auto write_back = [&](int h) -> mf_status {
        if (!writeBack || pending[h] == 0) return MF_OK;
        GTRY(hipStreamWaitEvent(g->sd, g->evComp[h], 0));
        for (int i = 0; i < pending[h]; i++) {
            const int r = hlist[pendLo[h] + i];
            const Layout L = layout_of(g->rinfo[r].x, g->rinfo[r].y);
            const size_t slot = (size_t)h * g->half + i;
            const size_t bytes = (size_t)(L.words - L.res) * sizeof(int);
            GTRY(hipMemcpyAsync(g->hpages + (size_t)r * g->stride + L.res,
                                g->pool + slot * g->stride + L.res, bytes, hipMemcpyDeviceToHost, g->sd));
            g->pages_out++;
            g->bytes_d2h += (long long)bytes;
        }
        GTRY(hipEventRecord(g->evWB[h], g->sd));
        pending[h] = 0;
        return MF_OK;
    };
    for (int j = 0; j < nb; j++) {
        const int h = j % g->nhalves, lo = j * g->half, cnt = std::min(g->half, n - lo);
        mf_status st = write_back(h);
        if (st != MF_OK) return st;
        // the slots of this half are free once the kernel that used them ended
        // and their state was written back
        GTRY(hipStreamWaitEvent(g->sc, g->evComp[h], 0));
        GTRY(hipStreamWaitEvent(g->sc, g->evWB[h], 0));
        for (int i = 0; i < cnt;) {
            // consecutive regions in consecutive slots: one copy (the last page without its padding)
            int j = i + 1;
            while (j < cnt && hlist[lo + j] == hlist[lo + j - 1] + 1) j++;
            const int r0 = hlist[lo + i], rl = hlist[lo + j - 1];
            const Layout L = layout_of(g->rinfo[rl].x, g->rinfo[rl].y);
            const size_t slot = (size_t)h * g->half + i;
            const size_t words = (size_t)(j - 1 - i) * g->stride + L.words;
            GTRY(hipMemcpyAsync(g->pool + slot * g->stride, g->hpages + (size_t)r0 * g->stride,
                                words * sizeof(int), hipMemcpyHostToDevice, g->sc));
            g->pages_in += j - i;
            g->bytes_h2d += (long long)(words * sizeof(int));
            i = j;
        }
        GTRY(hipEventRecord(g->evLoad[h], g->sc));
        GTRY(hipStreamWaitEvent(g->s, g->evLoad[h], 0));
        GTRY(hipMemsetAsync(g->qhead, 0, sizeof(unsigned), g->s));
        GTRY(launch(dlist, lo, cnt, h * g->half, g->s));
        GTRY(hipEventRecord(g->evComp[h], g->s));
        pending[h] = cnt;
        pendLo[h] = lo;
    }
    for (int h = 0; h < g->nhalves; h++) {
        mf_status st = write_back(h);
        if (st != MF_OK) return st;
    }
    // later work on the compute stream comes after the write-backs
    for (int h = 0; h < g->nhalves; h++) GTRY(hipStreamWaitEvent(g->s, g->evWB[h], 0));
    return MF_OK;
}

mf_status launch_discharge(mf_graph *g, const mfg::Args &base, const int *dlist, int lo, int n,
                           int slotBase, hipStream_t s) {
    if (g->profile) {
        if (g->evProf.size() < 2 * (g->nprof + 1)) {
            hipEvent_t e0 = nullptr, e1 = nullptr;
            GTRY(hipEventCreate(&e0));
            GTRY(hipEventCreate(&e1));
            g->evProf.push_back(e0);
            g->evProf.push_back(e1);
        }
        GTRY(hipEventRecord(g->evProf[2 * g->nprof], s));
    }
    mfg::Args A = base;
    A.order = dlist;
    A.cnt = g->cnt;
    A.listLo = lo;
    A.listN = n;
    A.slotBase = slotBase;
    A.qhead = g->qhead;
    const int blocks = n >= 0 ? std::max(1, std::min(n, g->blocks)) : g->blocks;
    const size_t lds = g->ldsBytes;
    if (g->group == 32) {
        if (lds) hipLaunchKernelGGL((mfg::k_gdischarge<mfg::kDNT, 32, true>), dim3(blocks), dim3(mfg::kDNT), lds, s, A);
        else hipLaunchKernelGGL((mfg::k_gdischarge<mfg::kDNT, 32, false>), dim3(blocks), dim3(mfg::kDNT), 0, s, A);
    } else {
        if (lds) hipLaunchKernelGGL((mfg::k_gdischarge<mfg::kDNT, 8, true>), dim3(blocks), dim3(mfg::kDNT), lds, s, A);
        else hipLaunchKernelGGL((mfg::k_gdischarge<mfg::kDNT, 8, false>), dim3(blocks), dim3(mfg::kDNT), 0, s, A);
    }
    if (!ok(hipGetLastError())) return MF_E_DEVICE;
    if (g->profile) {
        GTRY(hipEventRecord(g->evProf[2 * g->nprof + 1], s));
        g->nprof++;
    }
    return MF_OK;
}

// One sweep of Alg. 2 over the active regions.  Resident pages: enqueued
// without a host round trip.  Streamed pages: the region list comes to the
// host, whose page transfers follow it.
mf_status enqueue_sweep(mf_graph *g, long long i, bool gapOn, int *regionsOut) {
    const u64 *actIn = g->act + (i & 1);
    u64 *actOut = g->act + ((i + 1) & 1);
    int *labOld = g->lab[i & 1], *labNew = g->lab[(i + 1) & 1];
    hipStream_t s = g->s;
    hipLaunchKernelGGL(mfg::k_gcarry, dim3(cdiv(std::max(g->nB, 1), 256)), dim3(256), 0, s, g->ractive,
                       g->bregion, labOld, labNew, g->nB, g->cnt, g->qhead, actIn);
    hipLaunchKernelGGL(mfg::k_gqueue, dim3(cdiv(std::max(g->K, 1), 256)), dim3(256), 0, s, g->ractive, g->K,
                       g->order, g->cnt, actIn);
    GTRY(hipGetLastError());
    mfg::Args A = base_args(g);
    A.labOld = labOld;
    A.labNew = labNew;
    A.actIn = actIn;
    if (g->resident) {
        mf_status st = launch_discharge(g, A, g->order, 0, -1, -1, s);
        if (st != MF_OK) return st;
    } else {
        int *mb = (int *)g->pinned;
        GTRY(hipMemcpyAsync(mb, g->cnt, sizeof(int), hipMemcpyDeviceToHost, s));
        GTRY(hipMemcpyAsync(mb + 16, g->order, sizeof(int) * (size_t)g->K, hipMemcpyDeviceToHost, s));
        GTRY(hipStreamSynchronize(s));
        u64 a = 0;
        GTRY(hipMemcpy(&a, actIn, sizeof(u64), hipMemcpyDeviceToHost));
        const int n = a ? mb[0] : 0;
        if (regionsOut) *regionsOut = n;
        if (n > 0) {
            // regions in increasing order: neighbouring pages load in one copy
            std::sort(mb + 16, mb + 16 + n);
            GTRY(hipMemcpyAsync(g->order, mb + 16, sizeof(int) * (size_t)n, hipMemcpyHostToDevice, s));
            mf_status st = page_pass(g, g->order, mb + 16, n, true,
                                     [&](const int *dl, int lo, int cnt, int sb, hipStream_t ss) {
                                         return launch_discharge(g, A, dl, lo, cnt, sb, ss) == MF_OK
                                                    ? hipSuccess : hipErrorUnknown;
                                     });
            if (st != MF_OK) return st;
        }
    }
    if (g->nC > 0)
        hipLaunchKernelGGL(mfg::k_gfuse, dim3(cdiv(g->nC, 256)), dim3(256), 0, s, g->cr, g->cp, g->cslot,
                           labNew, g->exIn, g->nC, actIn);
    GTRY(hipGetLastError());
    if (g->nB > 0) GTRY(mfd::launch_label_hist(labNew, g->nB, g->dinf, g->hist, g->maxlab, actIn, s));
    mfd::GapArgs G;
    memset(&G, 0, sizeof(G));
    G.hist = g->hist;
    G.maxlab = g->maxlab;
    G.gap = g->gap;
    G.gapOn = gapOn ? 1 : 0;
    G.actIn = actIn;
    G.actOut = actOut;
    G.qheadNext = g->qhead;
    G.counters = g->counters;
    G.actCarry = g->carry;  // zero unless a capped discharge left its region active
    GTRY(mfd::launch_gap_find(G, s));
    hipLaunchKernelGGL(mfg::k_gapply, dim3(cdiv(std::max(g->nB, 1), 256)), dim3(256), 0, s, labNew, g->exIn,
                       g->bregion, g->ractive, g->nB, g->gap, g->dinf, actOut, actIn);
    GTRY(hipGetLastError());
    return MF_OK;
}

// Runs a page kernel over every region (the flood rounds and the collection).
template <class Fill>
mf_status all_regions(mf_graph *g, bool writeBack, Fill fill) {
    std::vector<int> hl;
    if (!g->resident) {
        hl.resize(g->K);
        for (int r = 0; r < g->K; r++) hl[r] = r;
    }
    return page_pass(g, g->allreg, hl.data(), g->K, writeBack,
                     [&](const int *dl, int lo, int cnt, int sb, hipStream_t ss) {
                         mfg::Args A = base_args(g);
                         A.order = dl;
                         A.listLo = lo;
                         A.listN = cnt;
                         A.slotBase = sb;
                         A.qhead = g->qhead;
                         fill(A);
                         return A.listN == -2 ? hipErrorUnknown : hipSuccess;
                     });
}

mf_status flood(mf_graph *g, int kind) {
    if (g->cut_cached == kind) return MF_OK;
    g->cut_cached = -1;
    const int mode = kind == MF_CUT_MAX_SOURCE ? 0 : 1;
    GTRY(hipMemsetAsync(g->markB, 0, sizeof(int) * (size_t)std::max(g->nB, 1), g->s));
    for (long long round = 0;; round++) {
        GTRY(hipMemsetAsync(g->changed, 0, sizeof(unsigned), g->s));
        mf_status st = all_regions(g, true, [&](mfg::Args &A) {
            A.mode = mode;
            A.first = round == 0 ? 1 : 0;
            const int blocks = std::max(1, std::min(A.listN, g->blocks));
            hipLaunchKernelGGL(mfg::k_gflood<mfg::kNT>, dim3(blocks), dim3(mfg::kNT), 0, g->s, A);
            if (!ok(hipGetLastError())) A.listN = -2;
        });
        if (st != MF_OK) return st;
        GTRY(hipMemcpyAsync(g->pinned, g->changed, sizeof(unsigned), hipMemcpyDeviceToHost, g->s));
        GTRY(hipStreamSynchronize(g->s));
        if (*(unsigned *)g->pinned == 0u) break;
        if (round > (long long)g->nB + 2) return MF_E_DEVICE;  // a round that changes adds a boundary mark
    }
    g->cut_cached = kind;
    return MF_OK;
}

// Sum of the residual t-links and, with cut != null, the cut side per vertex.
mf_status collect(mf_graph *g, int mode, unsigned char *cut, long long *sumRt) {
    GTRY(hipMemsetAsync(g->sum, 0, sizeof(u64), g->s));
    mf_status st = all_regions(g, false, [&](mfg::Args &A) {
        A.mode = mode;
        A.cut = cut;
        const int blocks = std::max(1, std::min(A.listN, g->blocks));
        hipLaunchKernelGGL(mfg::k_gcollect<mfg::kNT>, dim3(blocks), dim3(mfg::kNT), 0, g->s, A);
        if (!ok(hipGetLastError())) A.listN = -2;
    });
    if (st != MF_OK) return st;
    GTRY(hipMemcpyAsync(g->pinned, g->sum, sizeof(u64), hipMemcpyDeviceToHost, g->s));
    GTRY(hipStreamSynchronize(g->s));
    if (sumRt) *sumRt = (long long)*(u64 *)g->pinned;
    return MF_OK;
}

}  // namespace

static mf_status mf_create_graph_impl(int32_t n, int64_t npairs, const int32_t *pu, const int32_t *pv,
                                     const int32_t *cuv, const int32_t *cvu, const int32_t *cs,
                                     const int32_t *ct, const int32_t *region, int32_t region_size,
                                     int64_t device_pages, mf_graph **out) {
    if (!out) return MF_E_INVAL;
    *out = nullptr;
    if (n < 0 || npairs < 0 || device_pages < 0) return MF_E_INVAL;
    if (npairs > 0 && (!pu || !pv || !cuv || !cvu)) return MF_E_INVAL;
    if (n > 0 && (!cs || !ct)) return MF_E_INVAL;
    if (!region && region_size < 1) return MF_E_INVAL;
    if (npairs > (1LL << 30)) return MF_E_INVAL;  // arcs are numbered with 32 bits
    // ---- validation: vertex numbers, capacities, int32 bounds of every residual and excess
    std::vector<long long> inflow((size_t)n, 0);
    for (int32_t v = 0; v < n; v++) {
        if (cs[v] < 0 || ct[v] < 0) return MF_E_INVAL;
        inflow[v] = cs[v];
    }
    for (int64_t i = 0; i < npairs; i++) {
        const int32_t u = pu[i], v = pv[i];
        if (u < 0 || v < 0 || u >= n || v >= n || u == v) return MF_E_INVAL;
        if (cuv[i] < 0 || cvu[i] < 0) return MF_E_INVAL;
        if ((long long)cuv[i] + cvu[i] > 0x7fffffffLL) return MF_E_OVERFLOW;
        inflow[v] += cuv[i];
        inflow[u] += cvu[i];
    }
    for (int32_t v = 0; v < n; v++)
        if (inflow[v] > 0x7fffffffLL) return MF_E_OVERFLOW;  // bounds the excess of v
    // ---- regions: the caller's region numbers renumbered densely in increasing
    // order (any numbers >= 0 are allowed), or blocks of region_size vertices
    std::vector<int> reg((size_t)n);
    int K = 0;
    if (region) {
        std::vector<int32_t> ids(region, region + n);
        std::sort(ids.begin(), ids.end());
        ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
        if (!ids.empty() && ids[0] < 0) return MF_E_INVAL;
        K = (int)ids.size();
        for (int32_t v = 0; v < n; v++)
            reg[v] = (int)(std::lower_bound(ids.begin(), ids.end(), region[v]) - ids.begin());
    } else {
        for (int32_t v = 0; v < n; v++) reg[v] = v / region_size;
        K = n > 0 ? (int)((n - 1) / region_size + 1) : 0;
    }
    mf_graph *g = new (std::nothrow) mf_graph;
    if (!g) return MF_E_NOMEM;
    // a host allocation that fails below throws: the handle is released on the way out
    struct Guard {
        mf_graph *g;
        ~Guard() {
            if (g) {
                free_graph(g);
                delete g;
            }
        }
    } guard{g};
    g->n = n;
    g->np = npairs;
    g->K = K;
    // local numbering: the vertices of a region in increasing order
    std::vector<int> nv(K, 0), loc((size_t)n), deg((size_t)n, 0), nb(K, 0);
    for (int32_t v = 0; v < n; v++) loc[v] = nv[reg[v]]++;
    std::vector<char> inB((size_t)n, 0);
    long long nC = 0;
    for (int64_t i = 0; i < npairs; i++) {
        deg[pu[i]]++;
        deg[pv[i]]++;
        if (reg[pu[i]] != reg[pv[i]]) {
            inB[pu[i]] = 1;
            inB[pv[i]] = 1;
            nC++;
        }
    }
    // boundary slots, region by region in local order
    std::vector<std::vector<int>> members(K);
    for (int r = 0; r < K; r++) members[r].reserve(nv[r]);
    for (int32_t v = 0; v < n; v++) members[reg[v]].push_back(v);
    std::vector<int> bslot((size_t)n, -1), bbase(K + 1, 0);
    int nB = 0;
    g->blocal_h.clear();
    std::vector<int> bregion_h;
    for (int r = 0; r < K; r++) {
        bbase[r] = nB;
        for (int v : members[r])
            if (inB[v]) {
                bslot[v] = nB++;
                g->blocal_h.push_back(loc[v]);
                bregion_h.push_back(r);
                nb[r]++;
            }
    }
    bbase[K] = nB;
    g->nB = nB;
    g->nC = nC;
    g->dinf = std::max(nB, 1);
    // pages
    std::vector<long long> na(K, 0);
    long long maxWords = 1;
    g->rinfo.resize(K);
    for (int r = 0; r < K; r++) {
        for (int v : members[r]) na[r] += deg[v];
        if (na[r] > 0x3fffffffLL / 4) {
            return MF_E_INVAL;  // 32-bit offsets inside a page
        }
        const Layout L = layout_of(nv[r], (int)na[r]);
        maxWords = std::max(maxWords, (long long)L.words);
        g->rinfo[r] = make_int4(nv[r], (int)na[r], bbase[r], nb[r]);
        g->nvmax = std::max(g->nvmax, nv[r]);
    }
    g->stride = (maxWords + 63) / 64 * 64;
    g->resident = device_pages == 0 || device_pages >= K;
    g->P = g->resident ? K : (int)device_pages;
    g->nhalves = (!g->resident && g->P >= 2) ? 2 : 1;
    g->half = g->resident ? 0 : g->P / g->nhalves;
    const size_t storeWords = (size_t)K * (size_t)g->stride;
    std::vector<int> store;
    int *hp = nullptr;
    if (g->resident) {
        store.assign(std::max(storeWords, (size_t)1), 0);
        hp = store.data();
    } else {
        if (!ok(hipHostMalloc((void **)&g->hpages, std::max(storeWords, (size_t)1) * sizeof(int), 0))) {
            return MF_E_NOMEM;
        }
        memset(g->hpages, 0, storeWords * sizeof(int));
        hp = g->hpages;
    }
    // fill the pages: rows of arcs in pair order
    std::vector<int> fillpos((size_t)n, 0);
    std::vector<int> cr_h((size_t)(2 * nC)), cslot_h((size_t)(2 * nC));
    std::vector<int> ract(K, 0);
    long long sumCt = 0;
    for (int r = 0; r < K; r++) {
        int *pg = hp + (size_t)r * g->stride;
        const Layout L = layout_of(nv[r], (int)na[r]);
        int a = 0;
        for (int v : members[r]) {
            const int l = loc[v];
            pg[L.off + l] = a;
            fillpos[v] = a;
            a += deg[v];
            pg[L.gid + l] = v;
            pg[L.ex + l] = cs[v];
            pg[L.rt + l] = ct[v];
            sumCt += ct[v];
            if (cs[v] > 0) ract[r] = 1;
        }
        pg[L.off + nv[r]] = a;
    }
    g->pair_loc.resize((size_t)npairs);
    long long c = 0;
    for (int64_t i = 0; i < npairs; i++) {
        const int u = pu[i], v = pv[i];
        const int ru = reg[u], rv = reg[v];
        const int au = fillpos[u]++, av = fillpos[v]++;
        int *pgu = hp + (size_t)ru * g->stride, *pgv = hp + (size_t)rv * g->stride;
        const Layout Lu = layout_of(nv[ru], (int)na[ru]), Lv = layout_of(nv[rv], (int)na[rv]);
        if (ru == rv) {
            pgu[Lu.head + au] = loc[v];
            pgu[Lu.head + av] = loc[u];
            pgu[Lu.rev + au] = av;
            pgu[Lu.rev + av] = au;
            pgu[Lu.res + au] = cuv[i];
            pgu[Lu.res + av] = cvu[i];
            pgu[Lu.rres + au] = cvu[i];
            pgu[Lu.rres + av] = cuv[i];
            g->pair_loc[i] = ((long long)ru << 32) | (long long)au;
        } else {
            pgu[Lu.head + au] = -(int)(2 * c) - 1;
            pgv[Lv.head + av] = -(int)(2 * c + 1) - 1;
            pgu[Lu.rev + au] = -1;
            pgv[Lv.rev + av] = -1;
            cr_h[2 * c] = cuv[i];
            cr_h[2 * c + 1] = cvu[i];
            cslot_h[2 * c] = bslot[u];
            cslot_h[2 * c + 1] = bslot[v];
            g->pair_loc[i] = ~c;
            c++;
        }
    }
    g->sum_ct = sumCt;
    // ---- device
    hipDeviceProp_t prop;
    if (!ok(hipGetDevice(&g->device)) || !ok(hipGetDeviceProperties(&prop, g->device))) {
        return MF_E_DEVICE;
    }
    g->numCU = prop.multiProcessorCount;
    // a group of lanes per vertex: 32 when vertices have a dozen arcs or more
    g->group = (n > 0 && 2 * npairs >= 12LL * n) ? 32 : 8;
    // the search arrays and row offsets in LDS while two workgroups fit a compute unit
    {
        const size_t nvm = (size_t)std::max(g->nvmax, 1);
        const size_t need = sizeof(int) * (4 * nvm + 1 + (nvm + 31) / 32);
        const size_t cap = std::min<size_t>(80 * 1024, (size_t)prop.sharedMemPerBlock);
        g->ldsBytes = need <= cap ? need : 0;
        static bool attrs = false;
        if (!attrs) {
            (void)hipFuncSetAttribute((const void *)mfg::k_gdischarge<mfg::kDNT, 32, true>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 80 * 1024);
            (void)hipFuncSetAttribute((const void *)mfg::k_gdischarge<mfg::kDNT, 8, true>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, 80 * 1024);
            attrs = true;
        }
    }
    // workgroups: two per compute unit, as many as the scratch budget allows
    const long long perBlock = 4LL * mfg::kScratchInts * std::max(g->nvmax, 1);
    const int budgetBlocks = (int)std::max(1LL, (1LL << 30) / perBlock);
    const int listMax = g->resident ? K : g->half;
    g->blocks = std::max(1, std::min({std::max(listMax, 1), 2 * g->numCU, budgetBlocks}));
    bool good = ok(hipStreamCreateWithFlags(&g->s, hipStreamNonBlocking)) &&
                ok(hipStreamCreateWithFlags(&g->sc, hipStreamNonBlocking)) &&
                ok(hipStreamCreateWithFlags(&g->sd, hipStreamNonBlocking));
    for (int h = 0; h < 2 && good; h++)
        good = ok(hipEventCreateWithFlags(&g->evLoad[h], hipEventDisableTiming)) &&
               ok(hipEventCreateWithFlags(&g->evComp[h], hipEventDisableTiming)) &&
               ok(hipEventCreateWithFlags(&g->evWB[h], hipEventDisableTiming));
    const size_t poolWords = (size_t)g->P * (size_t)g->stride;
    good = good && ok(dalloc(&g->pool, poolWords)) && ok(dalloc(&g->drinfo, (size_t)K)) &&
           ok(dalloc(&g->blocal, (size_t)nB)) && ok(dalloc(&g->bregion, (size_t)nB)) &&
           ok(dalloc(&g->lab[0], (size_t)nB)) && ok(dalloc(&g->lab[1], (size_t)nB)) &&
           ok(dalloc(&g->exIn, (size_t)nB)) && ok(dalloc(&g->markB, (size_t)nB)) &&
           ok(dalloc(&g->cr, (size_t)(2 * nC))) && ok(dalloc(&g->cp, (size_t)(2 * nC))) &&
           ok(dalloc(&g->cslot, (size_t)(2 * nC))) && ok(dalloc(&g->order, (size_t)K)) &&
           ok(dalloc(&g->allreg, (size_t)K)) && ok(dalloc(&g->cnt, 1)) &&
           ok(dalloc(&g->ractive, (size_t)K)) &&
           ok(dalloc(&g->scratch, (size_t)g->blocks * mfg::kScratchInts * (size_t)std::max(g->nvmax, 1))) &&
           ok(dalloc(&g->err, 4)) && ok(dalloc(&g->maxlab, 1)) && ok(dalloc(&g->gap, 1)) &&
           ok(dalloc(&g->qhead, 2)) && ok(dalloc(&g->changed, 1)) &&
           ok(dalloc(&g->hist, (size_t)mfd::kHistBins)) && ok(dalloc(&g->act, 2)) &&
           ok(dalloc(&g->counters, 4)) && ok(dalloc(&g->stats, 8)) && ok(dalloc(&g->sum, 1)) &&
           ok(dalloc(&g->carry, 1)) &&
           ok(dalloc(&g->cutbuf, (size_t)n)) &&
           ok(hipHostMalloc(&g->pinned, sizeof(int) * (16 + (size_t)K), 0));
    if (!good) {
        return MF_E_NOMEM;
    }
    std::vector<int> allreg_h(K);
    for (int r = 0; r < K; r++) allreg_h[r] = r;
    long long act0 = 0;
    for (int r = 0; r < K; r++) act0 += ract[r];
    const u64 actInit[2] = {(u64)act0, 0ull};
    const int minus1 = -1;
    hipStream_t s = g->s;
    good = ok(hipMemcpyAsync(g->drinfo, g->rinfo.data(), sizeof(int4) * (size_t)K, hipMemcpyHostToDevice, s)) &&
           ok(hipMemcpyAsync(g->blocal, g->blocal_h.data(), sizeof(int) * (size_t)nB, hipMemcpyHostToDevice, s)) &&
           ok(hipMemcpyAsync(g->bregion, bregion_h.data(), sizeof(int) * (size_t)nB, hipMemcpyHostToDevice, s)) &&
           ok(hipMemsetAsync(g->lab[0], 0, sizeof(int) * (size_t)std::max(nB, 1), s)) &&
           ok(hipMemsetAsync(g->lab[1], 0, sizeof(int) * (size_t)std::max(nB, 1), s)) &&
           ok(hipMemsetAsync(g->exIn, 0, sizeof(int) * (size_t)std::max(nB, 1), s)) &&
           ok(hipMemcpyAsync(g->cr, cr_h.data(), sizeof(int) * (size_t)(2 * nC), hipMemcpyHostToDevice, s)) &&
           ok(hipMemsetAsync(g->cp, 0, sizeof(int) * (size_t)std::max(2 * nC, 1LL), s)) &&
           ok(hipMemcpyAsync(g->cslot, cslot_h.data(), sizeof(int) * (size_t)(2 * nC), hipMemcpyHostToDevice, s)) &&
           ok(hipMemcpyAsync(g->allreg, allreg_h.data(), sizeof(int) * (size_t)K, hipMemcpyHostToDevice, s)) &&
           ok(hipMemcpyAsync(g->ractive, ract.data(), sizeof(int) * (size_t)K, hipMemcpyHostToDevice, s)) &&
           ok(hipMemsetAsync(g->err, 0, sizeof(int) * 4, s)) &&
           ok(hipMemcpyAsync(g->maxlab, &minus1, sizeof(int), hipMemcpyHostToDevice, s)) &&
           ok(hipMemsetAsync(g->hist, 0, sizeof(unsigned) * (size_t)mfd::kHistBins, s)) &&
           ok(hipMemcpyAsync(g->act, actInit, sizeof(actInit), hipMemcpyHostToDevice, s)) &&
           ok(hipMemsetAsync(g->counters, 0, sizeof(u64) * 4, s)) &&
           ok(hipMemsetAsync(g->carry, 0, sizeof(u64), s)) &&
           ok(hipMemsetAsync(g->stats, 0, sizeof(u64) * 8, s));
    if (good && g->resident && storeWords > 0)
        good = ok(hipMemcpyAsync(g->pool, hp, storeWords * sizeof(int), hipMemcpyHostToDevice, s));
    good = good && ok(hipStreamSynchronize(s));
    if (!good) {
        return MF_E_DEVICE;
    }
    guard.g = nullptr;
    *out = g;
    return MF_OK;
}

extern "C" void mf_graph_destroy(mf_graph *g) {
    if (!g) return;
    (void)hipSetDevice(g->device);
    if (g->s) (void)hipStreamSynchronize(g->s);
    if (g->sc) (void)hipStreamSynchronize(g->sc);
    if (g->sd) (void)hipStreamSynchronize(g->sd);
    free_graph(g);
    delete g;
}

extern "C" mf_status mf_graph_get_info(const mf_graph *g, mf_graph_info *info) {
    if (!g || !info) return MF_E_INVAL;
    info->n = g->n;
    info->npairs = g->np;
    info->regions = g->K;
    info->boundary_size = g->nB;
    info->boundary_pairs = g->nC;
    info->page_words = g->stride;
    info->device_pages = g->P;
    info->resident = g->resident ? 1 : 0;
    info->max_region_vertices = g->nvmax;
    return MF_OK;
}

static mf_status mf_graph_solve_impl(mf_graph *g, const mf_graph_opts *opts, mf_graph_stats *st) {
    if (!g) return MF_E_INVAL;
    mf_graph_opts o;
    memset(&o, 0, sizeof(o));
    o.gap = 1;
    if (opts) o = *opts;
    if (o.max_sweeps < 0 || o.check_every < 0 || o.round_cap < 0) return MF_E_INVAL;
    GTRY(hipSetDevice(g->device));
    g->roundCap = o.round_cap;
    // capped rounds spread one discharge over several sweeps, so the bound of
    // full discharges does not hold: the default guard is then at least 2^20
    const long long bound = o.round_cap > 0 ? std::max(2LL * g->nB * g->nB + 1, 1LL << 20) : 2LL * g->nB * g->nB + 1;
    const long long maxSweeps = o.max_sweeps > 0 ? o.max_sweeps : bound;
    const int every = o.check_every > 0 ? o.check_every : 8;
    const long long pin0 = g->pages_in, pout0 = g->pages_out, h2d0 = g->bytes_h2d, d2h0 = g->bytes_d2h;
    g->profile = o.profile != 0;
    g->nprof = 0;
    u64 stt0[8];
    GTRY(hipMemcpy(stt0, g->stats, sizeof(stt0), hipMemcpyDeviceToHost));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    GTRY(hipEventCreate(&e0));
    GTRY(hipEventCreate(&e1));
    GTRY(hipEventRecord(e0, g->s));
    mf_status status = MF_OK;
    bool done = false;
    long long enq = 0;  // sweeps enqueued by this call
    const long long startSweeps = g->sweeps;
    while (!done) {
        u64 ctl[2];
        GTRY(hipMemcpy(ctl, g->counters, sizeof(u64), hipMemcpyDeviceToHost));
        const long long executed = (long long)ctl[0];
        GTRY(hipMemcpy(&ctl[1], g->act + (executed & 1), sizeof(u64), hipMemcpyDeviceToHost));
        int e4[4];
        GTRY(hipMemcpy(e4, g->err, sizeof(e4), hipMemcpyDeviceToHost));
        if (e4[0]) {
            status = MF_E_DEVICE;
            break;
        }
        if (ctl[1] == 0ull) {
            done = true;
            break;
        }
        if (executed - startSweeps >= maxSweeps) {
            status = MF_E_SWEEPS;
            break;
        }
        const long long batch = g->resident ? std::min<long long>(every, maxSweeps - (executed - startSweeps)) : 1;
        for (long long j = 0; j < batch; j++) {
            mf_status s2 = enqueue_sweep(g, executed + j, o.gap != 0, nullptr);
            if (s2 != MF_OK) {
                status = s2;
                break;
            }
        }
        enq += batch;
        if (status != MF_OK) break;
        GTRY(hipStreamSynchronize(g->s));
    }
    GTRY(hipEventRecord(e1, g->s));
    GTRY(hipStreamSynchronize(g->s));
    GTRY(hipStreamSynchronize(g->sc));
    GTRY(hipStreamSynchronize(g->sd));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    u64 ctl[4], stt[8];
    GTRY(hipMemcpy(ctl, g->counters, sizeof(ctl), hipMemcpyDeviceToHost));
    GTRY(hipMemcpy(stt, g->stats, sizeof(stt), hipMemcpyDeviceToHost));
    for (int i = 0; i < 8; i++) stt[i] -= stt0[i];
    double dms = 0.0;
    for (size_t i = 0; i < g->nprof; i++) {
        float t = 0.f;
        if (ok(hipEventElapsedTime(&t, g->evProf[2 * i], g->evProf[2 * i + 1]))) dms += t;
    }
    const long long nlaunch = (long long)g->nprof;
    g->profile = false;
    g->nprof = 0;
    g->sweeps = (long long)ctl[0];
    g->cur = (int)(g->sweeps & 1);
    g->cut_cached = -1;
    (void)enq;
    if (st) {
        memset(st, 0, sizeof(*st));
        st->sweeps = g->sweeps;
        st->discharges = (int64_t)stt[0];
        st->push_rounds = (int64_t)stt[1];
        st->search_steps = (int64_t)stt[2];
        st->pages_in = g->pages_in - pin0;
        st->pages_out = g->pages_out - pout0;
        st->bytes_h2d = g->bytes_h2d - h2d0;
        st->bytes_d2h = g->bytes_d2h - d2h0;
        st->ms = ms;
        st->discharged_vertices = (int64_t)stt[3];
        st->discharged_arcs = (int64_t)stt[4];
        st->discharge_launches = nlaunch;
        st->discharge_ms = dms;
    }
    if (status != MF_OK) {
        g->solved = false;
        return status;
    }
    long long sumRt = 0;
    mf_status s3 = collect(g, 0, nullptr, &sumRt);
    if (s3 != MF_OK) return s3;
    g->flow = g->sum_ct - sumRt;
    g->solved = true;
    return MF_OK;
}

extern "C" mf_status mf_graph_flow_value(const mf_graph *g, int64_t *out) {
    if (!g || !out) return MF_E_INVAL;
    if (!g->solved) return MF_E_STATE;
    *out = g->flow;
    return MF_OK;
}

static mf_status mf_graph_min_cut_impl(mf_graph *g, int32_t kind, uint8_t *out_source_side) {
    if (!g || !out_source_side) return MF_E_INVAL;
    if (kind != MF_CUT_MIN_SOURCE && kind != MF_CUT_MAX_SOURCE) return MF_E_INVAL;
    if (!g->solved) return MF_E_STATE;
    GTRY(hipSetDevice(g->device));
    mf_status st = flood(g, kind);
    if (st != MF_OK) return st;
    st = collect(g, kind == MF_CUT_MAX_SOURCE ? 0 : 1, g->cutbuf, nullptr);
    if (st != MF_OK) return st;
    if (g->n > 0) {
        GTRY(hipMemcpyAsync(out_source_side, g->cutbuf, (size_t)g->n, hipMemcpyDeviceToHost, g->s));
        GTRY(hipStreamSynchronize(g->s));
    }
    return MF_OK;
}

static mf_status mf_graph_state_impl(mf_graph *g, int64_t *r_uv, int64_t *r_vu, int64_t *rt, int64_t *ex,
                                    int32_t *labels) {
    if (!g) return MF_E_INVAL;
    GTRY(hipSetDevice(g->device));
    GTRY(hipStreamSynchronize(g->s));
    GTRY(hipStreamSynchronize(g->sc));
    GTRY(hipStreamSynchronize(g->sd));
    const size_t storeWords = (size_t)g->K * (size_t)g->stride;
    std::vector<int> store;
    const int *hp = g->hpages;
    if (g->resident) {
        store.resize(std::max(storeWords, (size_t)1));
        if (storeWords) GTRY(hipMemcpy(store.data(), g->pool, storeWords * sizeof(int), hipMemcpyDeviceToHost));
        hp = store.data();
    }
    std::vector<int> crh((size_t)(2 * g->nC)), exInH((size_t)g->nB), labB((size_t)g->nB);
    if (g->nC) GTRY(hipMemcpy(crh.data(), g->cr, sizeof(int) * crh.size(), hipMemcpyDeviceToHost));
    if (g->nB) {
        GTRY(hipMemcpy(exInH.data(), g->exIn, sizeof(int) * exInH.size(), hipMemcpyDeviceToHost));
        GTRY(hipMemcpy(labB.data(), g->lab[g->sweeps & 1], sizeof(int) * labB.size(), hipMemcpyDeviceToHost));
    }
    for (int64_t i = 0; i < g->np; i++) {
        const long long loc = g->pair_loc[i];
        long long a = 0, b = 0;
        if (loc >= 0) {
            const int r = (int)(loc >> 32), au = (int)(loc & 0xffffffffLL);
            const int *pg = hp + (size_t)r * g->stride;
            const Layout L = layout_of(g->rinfo[r].x, g->rinfo[r].y);
            a = pg[L.res + au];
            b = pg[L.res + pg[L.rev + au]];
        } else {
            const long long c = ~loc;
            a = crh[2 * c];
            b = crh[2 * c + 1];
        }
        if (r_uv) r_uv[i] = a;
        if (r_vu) r_vu[i] = b;
    }
    for (int r = 0; r < g->K; r++) {
        const int *pg = hp + (size_t)r * g->stride;
        const Layout L = layout_of(g->rinfo[r].x, g->rinfo[r].y);
        for (int l = 0; l < g->rinfo[r].x; l++) {
            const int v = pg[L.gid + l];
            if (rt) rt[v] = pg[L.rt + l];
            if (ex) ex[v] = pg[L.ex + l];
            if (labels) labels[v] = pg[L.lab + l];
        }
        const int b0 = g->rinfo[r].z;
        for (int i = 0; i < g->rinfo[r].w; i++) {
            const int v = pg[L.gid + g->blocal_h[b0 + i]];
            if (ex) ex[v] += exInH[b0 + i];
            if (labels) labels[v] = labB[b0 + i];
        }
    }
    return MF_OK;
}

extern "C" int64_t mf_graph_discharge_bytes(int64_t nv, int64_t na) {
    if (nv < 0 || na < 0) return 0;
    // read: off (nv + 1), head and rev (2 na); read and written: res (na), ex and rt (2 nv);
    // written: lab (nv)
    return 4 * ((nv + 1) + 2 * na + 2 * (na + 2 * nv) + nv);
}

// ---------------------------------------------------------------------------
// DIMACS max-flow files (the format of the paper's instances).
// ---------------------------------------------------------------------------
#include <cstdio>
#include <cstdlib>

namespace {

void free_dimacs_arrays(mf_dimacs *d) {
    if (!d) return;
    free(d->pu);
    free(d->pv);
    free(d->cuv);
    free(d->cvu);
    free(d->cs);
    free(d->ct);
    free(d->vertex_id);
}

// Reads the next integer of line p (after whitespace); false at the end.
bool next_int(const char *&p, long long &v) {
    while (*p == ' ' || *p == '\t') p++;
    if (!(*p == '-' || (*p >= '0' && *p <= '9'))) return false;
    char *end = nullptr;
    v = strtoll(p, &end, 10);
    if (end == p) return false;
    p = end;
    return true;
}

}  // namespace

static mf_status mf_read_dimacs_impl(const char *path, mf_dimacs **out) {
    if (!path || !out) return MF_E_INVAL;
    *out = nullptr;
    FILE *f = fopen(path, "r");
    if (!f) return MF_E_INVAL;
    long long N = -1, M = -1, src = -1, snk = -1;
    std::vector<long long> au, av, ac;
    char *line = nullptr;
    size_t cap = 0;
    mf_status st = MF_OK;
    while (st == MF_OK && getline(&line, &cap, f) >= 0) {
        const char *p = line;
        while (*p == ' ' || *p == '\t') p++;
        if (*p == 'c' || *p == '\n' || *p == '\r' || *p == '\0') continue;
        const char kind = *p++;
        if (kind == 'p') {
            while (*p == ' ' || *p == '\t') p++;
            if (strncmp(p, "max", 3) != 0 || N >= 0) { st = MF_E_INVAL; break; }
            p += 3;
            if (!next_int(p, N) || !next_int(p, M) || N < 2 || M < 0 || N > 0x7fffffffLL) st = MF_E_INVAL;
        } else if (kind == 'n') {
            long long id;
            if (N < 0 || !next_int(p, id) || id < 1 || id > N) { st = MF_E_INVAL; break; }
            while (*p == ' ' || *p == '\t') p++;
            if (*p == 's') src = id;
            else if (*p == 't') snk = id;
            else st = MF_E_INVAL;
        } else if (kind == 'a') {
            long long u, v, c;
            if (N < 0 || !next_int(p, u) || !next_int(p, v) || !next_int(p, c) || u < 1 || u > N || v < 1 ||
                v > N || c < 0) {
                st = MF_E_INVAL;
                break;
            }
            if (c > 0x7fffffffLL) { st = MF_E_OVERFLOW; break; }
            au.push_back(u);
            av.push_back(v);
            ac.push_back(c);
        } else {
            st = MF_E_INVAL;
        }
    }
    free(line);
    fclose(f);
    if (st != MF_OK) return st;
    if (N < 0 || src < 0 || snk < 0 || src == snk || (long long)au.size() != M) return MF_E_INVAL;
    // vertices other than s and t, numbered in increasing file id
    const int32_t n = (int32_t)(N - 2);
    std::vector<int32_t> idx((size_t)N + 1, -1);
    mf_dimacs *d = (mf_dimacs *)calloc(1, sizeof(mf_dimacs));
    if (!d) return MF_E_NOMEM;
    d->n = n;
    d->vertex_id = (int64_t *)malloc(sizeof(int64_t) * (size_t)std::max(n, 1));
    d->cs = (int32_t *)calloc((size_t)std::max(n, 1), sizeof(int32_t));
    d->ct = (int32_t *)calloc((size_t)std::max(n, 1), sizeof(int32_t));
    if (!d->vertex_id || !d->cs || !d->ct) {
        free_dimacs_arrays(d);
        free(d);
        return MF_E_NOMEM;
    }
    for (long long id = 1, k = 0; id <= N; id++)
        if (id != src && id != snk) {
            idx[id] = (int32_t)k;
            d->vertex_id[k++] = id;
        }
    std::vector<long long> cs64((size_t)std::max(n, 1), 0), ct64((size_t)std::max(n, 1), 0);
    std::vector<int32_t> pu, pv, cuv;
    long long st_cap = 0;
    for (size_t i = 0; i < au.size(); i++) {
        const long long u = au[i], v = av[i], c = ac[i];
        if (u == v || u == snk || v == src) continue;  // arcs that carry no s-t flow
        if (u == src && v == snk) st_cap += c;
        else if (u == src) cs64[idx[v]] += c;
        else if (v == snk) ct64[idx[u]] += c;
        else {
            pu.push_back(idx[u]);
            pv.push_back(idx[v]);
            cuv.push_back((int32_t)c);
        }
    }
    for (int32_t v = 0; v < n; v++) {
        if (cs64[v] > 0x7fffffffLL || ct64[v] > 0x7fffffffLL) {
            free_dimacs_arrays(d);
            free(d);
            return MF_E_OVERFLOW;
        }
        d->cs[v] = (int32_t)cs64[v];
        d->ct[v] = (int32_t)ct64[v];
    }
    const size_t m = pu.size();
    d->npairs = (int64_t)m;
    d->st_capacity = st_cap;
    d->pu = (int32_t *)malloc(sizeof(int32_t) * std::max(m, (size_t)1));
    d->pv = (int32_t *)malloc(sizeof(int32_t) * std::max(m, (size_t)1));
    d->cuv = (int32_t *)malloc(sizeof(int32_t) * std::max(m, (size_t)1));
    d->cvu = (int32_t *)calloc(std::max(m, (size_t)1), sizeof(int32_t));
    if (!d->pu || !d->pv || !d->cuv || !d->cvu) {
        free_dimacs_arrays(d);
        free(d);
        return MF_E_NOMEM;
    }
    if (m) {
        memcpy(d->pu, pu.data(), sizeof(int32_t) * m);
        memcpy(d->pv, pv.data(), sizeof(int32_t) * m);
        memcpy(d->cuv, cuv.data(), sizeof(int32_t) * m);
    }
    *out = d;
    return MF_OK;
}

extern "C" void mf_free_dimacs(mf_dimacs *d) {
    free_dimacs_arrays(d);
    free(d);
}

extern "C" mf_status mf_create_graph(int32_t n, int64_t npairs, const int32_t *pu, const int32_t *pv, const int32_t *cuv,
                                     const int32_t *cvu, const int32_t *cs, const int32_t *ct, const int32_t *region,
                                     int32_t region_size, int64_t device_pages, mf_graph **out) {
    // host allocations throw on failure; no exception leaves the C ABI
    try {
        return mf_create_graph_impl(n, npairs, pu, pv, cuv, cvu, cs, ct, region, region_size, device_pages, out);
    } catch (const std::bad_alloc &) {
        if (out) *out = nullptr;
        return MF_E_NOMEM;
    } catch (...) {
        if (out) *out = nullptr;
        return MF_E_DEVICE;
    }
}

extern "C" mf_status mf_graph_solve(mf_graph *g, const mf_graph_opts *opts, mf_graph_stats *stats) {
    // host allocations throw on failure; no exception leaves the C ABI
    try {
        return mf_graph_solve_impl(g, opts, stats);
    } catch (const std::bad_alloc &) {
        return MF_E_NOMEM;
    } catch (...) {
        return MF_E_DEVICE;
    }
}

extern "C" mf_status mf_graph_state(mf_graph *g, int64_t *r_uv, int64_t *r_vu, int64_t *rt, int64_t *ex,
                                    int32_t *labels) {
    // host allocations throw on failure; no exception leaves the C ABI
    try {
        return mf_graph_state_impl(g, r_uv, r_vu, rt, ex, labels);
    } catch (const std::bad_alloc &) {
        return MF_E_NOMEM;
    } catch (...) {
        return MF_E_DEVICE;
    }
}

extern "C" mf_status mf_graph_min_cut(mf_graph *g, int32_t kind, uint8_t *out_source_side) {
    // host allocations throw on failure; no exception leaves the C ABI
    try {
        return mf_graph_min_cut_impl(g, kind, out_source_side);
    } catch (const std::bad_alloc &) {
        return MF_E_NOMEM;
    } catch (...) {
        return MF_E_DEVICE;
    }
}

extern "C" mf_status mf_read_dimacs(const char *path, mf_dimacs **out) {
    // host allocations throw on failure; no exception leaves the C ABI
    try {
        return mf_read_dimacs_impl(path, out);
    } catch (const std::bad_alloc &) {
        if (out) *out = nullptr;
        return MF_E_NOMEM;
    } catch (...) {
        if (out) *out = nullptr;
        return MF_E_DEVICE;
    }
}
