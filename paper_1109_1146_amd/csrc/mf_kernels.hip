// HIP kernels of the region-discharge max-flow solver for gfx950 (wave64).
//
// Data layout (HBM), all int32, blocked (region-major, see mf_device.h):
//   res[k*N + g]   residual capacity c_f(g, g + o_k)
//   rt[g]          residual t-link c_f(g, t)
//   ex[g]          excess e_f(g)
//   lab[p][g]      labels, two buffers: a sweep reads p and writes p ^ 1
//   pushb[k*N + g] flow a discharge sent over the boundary arc (g, g + o_k),
//                  consumed (and zeroed) by the fuse kernel
#include <algorithm>

#include "mf_device.h"
#include "mf_launch.h"

namespace mfd {

typedef unsigned long long u64;

__device__ __forceinline__ int wave_sum_i(int v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ long long wave_sum_ll(long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ int wave_min_i(int v) {
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

// ---------------------------------------------------------------------------
// Input validation (row-major inputs, before anything is written).
// ---------------------------------------------------------------------------
__global__ void k_validate(Geo G, const int *cs, const int *ct, const int *nbr, int n, int *err) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = v < n;
    if (!live) v = n - 1;  // duplicate the last vertex so every lane joins the reductions
    int x = v % G.dx, t = v / G.dx, y = t % G.dy, z = t / G.dy;
    int bad = 0, maxpair = 0;
    if (cs[v] < 0 || ct[v] < 0) bad |= 1;
    long long inflow = cs[v] < 0 ? 0 : cs[v];
    for (int k = 0; k < G.K; k++) {
        int c = nbr[(size_t)k * n + v];
        if (c < 0) { bad |= 1; continue; }
        int zz = z + G.oz[k], yy = y + G.oy[k], xx = x + G.ox[k];
        bool in = (unsigned)xx < (unsigned)G.dx && (unsigned)yy < (unsigned)G.dy &&
                  (unsigned)zz < (unsigned)G.dz;
        if (!in) {
            if (c != 0) bad |= 1;
            continue;
        }
        int w = (zz * G.dy + yy) * G.dx + xx;
        int crev = nbr[(size_t)(k ^ 1) * n + w];  // c(w, v)
        if (crev < 0) { bad |= 1; continue; }
        long long pair = (long long)c + crev;
        if (pair > 0x7fffffffLL) bad |= 2;
        else maxpair = max(maxpair, (int)pair);
        inflow += crev;
    }
    if (inflow > 0x7fffffffLL) bad |= 2;
    if (bad) atomicOr(err, bad);
    // largest pair sum and t-link, one atomic per wavefront
    maxpair = wave_max_i(maxpair);
    const int mct = wave_max_i(ct[v] > 0 ? ct[v] : 0);
    // c(s,v) + sum_u c(u,v) bounds the excess of v in every preflow
    const int min_ = wave_max_i((int)(inflow < 0x7fffffffLL ? inflow : 0x7fffffffLL));
    if ((threadIdx.x & 63) == 0) {
        if (maxpair > 0) atomicMax(&err[1], maxpair);
        if (mct > 0) atomicMax(&err[2], mct);
        if (min_ > 0) atomicMax(&err[3], min_);
    }
}

// Sums of the s- and t-links (int64) for the flow value and the certificate.
__global__ void k_sum_links(const int *cs, const int *ct, int n, u64 *out2) {
    long long a = 0, b = 0;
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        a += cs[v];
        b += ct[v];
    }
    a = wave_sum_ll(a);
    b = wave_sum_ll(b);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&out2[0], (u64)a);
        atomicAdd(&out2[1], (u64)b);
    }
}

// ---------------------------------------------------------------------------
// Init (Sec. 2): saturate s-links into the excess, f := 0, d := 0.
// ---------------------------------------------------------------------------
// Grid-stride loops with one atomic per workgroup for the active count (one
// per wave made the launch wait on same-address atomics).
constexpr int kCountBlocks = 2048;

__device__ __forceinline__ void block_count_add(int v, u64 *out) {
    __shared__ int s_w[4];  // blockDim.x == 256
    v = wave_sum_i(v);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int t = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        if (t) atomicAdd(out, (u64)t);
    }
}

__global__ void k_init(Geo G, const int *cs, const int *ct, const int *nbr, int n, int *res,
                       int *rt, int *ex, int *lab0, int *lab1, int *pushb, int *ractive,
                       u64 *act0) {
    int active = 0;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < G.N; g += gridDim.x * blockDim.x) {
        int z, y, x;
        bool real = blocked_to_grid(G, g, z, y, x);
        int e = 0, t = 0;
        if (real) {
            int v = (z * G.dy + y) * G.dx + x;
            e = cs[v];
            t = ct[v];
            for (int k = 0; k < G.K; k++) res[(size_t)k * G.N + g] = nbr[(size_t)k * n + v];
        } else {
            for (int k = 0; k < G.K; k++) res[(size_t)k * G.N + g] = 0;
        }
        for (int k = 0; k < G.K; k++) pushb[(size_t)k * G.N + g] = 0;
        ex[g] = e;
        rt[g] = t;
        lab0[g] = 0;
        lab1[g] = 0;
        if (e > 0) {
            active++;
            ractive[g / G.V] = 1;
        }
    }
    block_count_add(active, act0);
}

// ---------------------------------------------------------------------------
// Region discharge (Proc. ARD of Sec. 4.2 with region relabel, Alg. 3).
//
// One workgroup owns one region at a time and takes regions from a queue.
// ARD's staged Augment(R, T_k) is carried out as push-relabel with the
// lexicographic label (k, hops): a multi-level breadth-first search from the
// targets (t first, then boundary vertices w in increasing d(w) + 1; the
// search never relabels a vertex twice, exactly as Alg. 3) yields for every
// vertex u of R the smallest stage k with u -> T_k and its hop distance to
// T_k.  Excess then flows downhill through the search levels, from the last
// level to the first, along arcs that drop exactly one level inside a stage;
// first-level vertices of stage 0 push to t, of stage k > 0 over boundary
// arcs to w with d(w) + 1 = k.  Search and push alternate until no excess
// vertex of R reaches T_{d_inf}.  The last search is the region relabel.
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(NT) void k_discharge(DischargeArgs A) {
    extern __shared__ int smem[];
    __shared__ int s_r, s_active, s_qtail, s_nsteps, s_min, s_found, s_live, s_hit;
    __shared__ int s_wmin[NT / 64];
    // search marks: a step index, kInf (not reached yet) or kDead (not reached by
    // a complete search earlier in this discharge: it cannot reach a target for
    // the rest of the discharge, since pushes only add residual arcs between
    // reached vertices)
    constexpr int kDead = kInf - 1;
    __shared__ long long s_tr[4];  // trace: excess out, to sink, to boundary, label sum
    if (*A.actIn == 0ull) return;
    const int stageCap = stage_cap(A);
    const Geo &G = A.G;
    const int V = G.V, N = G.N, tid = threadIdx.x;
    int *S, *Q, *stepEnd, *stepLevel;
    if (A.useLDS) {
        S = smem;
    } else {
        S = A.scratch + (size_t)blockIdx.x * 4 * V;
    }
    Q = S + V;
    stepEnd = Q + V;
    stepLevel = stepEnd + V;
    int *res = A.res, *rt = A.rt, *ex = A.ex, *pushb = A.pushb;
    const int *labOld = A.labOld;
    const int dinf = A.dinf;

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
            // skipped region (no active vertex): labels carry over unchanged.
            // Other regions read only its border labels, and its own next
            // discharge recomputes the rest, so ARD copies the border only (the
            // other buffer holds older, never larger labels; the solve ends by
            // merging the two buffers).  The PRD gap reads every label.
            if (A.labNew != labOld) {
                if (A.prd) {
                    for (int l = tid; l < V; l += NT) A.labNew[base + l] = labOld[base + l];
                } else {
                    for (int i = tid; i < A.nring; i += NT) {
                        const int l = A.ringL[i];
                        A.labNew[base + l] = labOld[base + l];
                    }
                }
            }
            __syncthreads();
            continue;
        }

        int iter = 0;
        long long bfs_steps = 0, classes = 0;
        const long long t_start = wall_clock64();
        if (tid < 4) s_tr[tid] = 0;
        // partial discharge: the searches of the push rounds stop at the stage
        // cap; the labels come from a complete search (full)
        // region relabel only (Alg. 3 on the current state, no pushes): one
        // complete search, whose labels are written
        const bool relabelOnly = s_active == 2;
        bool full = !A.partial || relabelOnly;
        bool roundCapped = false;  // the round cap was reached: one more complete search
        bool firstSearch = true, lastComplete = false;
        for (;;) {
            bool capped = false, early = false;
            // a push-round search stops once every live excess vertex is labelled;
            // the search whose labels are written must be complete (with partial
            // discharges or after the round cap, the full one after the capped rounds)
            const bool earlyOk = !((A.partial || roundCapped) && full) && !relabelOnly;
            // ---------------- multi-level search from the targets ----------------
            if (tid == 0) {
                s_qtail = 0;
                s_nsteps = 0;
                s_found = 0;
                s_live = 0;
                s_hit = 0;
            }
            __syncthreads();
            // one pass: dead marks, live excess count, and the first level (r_t > 0;
            // such a vertex is reached by every search, so it is never dead)
            int live = 0, hit = 0;
            for (int l = tid; l < V; l += NT) {
                const int prev = firstSearch ? kInf : S[l];
                const bool dead = prev == kDead || (lastComplete && prev == kInf);
                const bool lv = !dead && ex[base + l] > 0;
                if (!dead && rt[base + l] > 0) {
                    S[l] = 0;
                    Q[atomicAdd(&s_qtail, 1)] = l;
                    hit |= lv ? 1 : 0;
                } else {
                    S[l] = dead ? kDead : kInf;
                    live += lv ? 1 : 0;
                }
            }
            live = wave_sum_i(live);
            if ((tid & 63) == 0 && live) atomicAdd(&s_live, live);
            if (hit) s_hit = 1;
            __syncthreads();
            if (A.prd) {
                // Proc. PRD: exact distance labels of the region network, d(t) = 0
                // and every arc of length 1, with the boundary labels fixed: a
                // border vertex is a seed at d(w) + 1 over its residual boundary
                // arcs.  Steps are consecutive distances, with a jump to the next
                // seed distance when the frontier runs dry.
                auto seed_dist = [&](int i) -> int {
                    const int l = A.ringL[i];
                    const unsigned m = A.ringM[i];
                    int lz, ly, lx;
                    local_xyz(G, l, lz, ly, lx);
                    int best = kInf;
                    for (int k = 0; k < G.K; k++) {
                        if (!((m >> k) & 1u)) continue;
                        if (res[(size_t)k * N + base + l] <= 0) continue;
                        const int w = cross_nbr(G, r, lz, ly, lx, k);
                        if (w < 0) continue;
                        const int d = labOld[w];
                        if (d < dinf) best = min(best, d + 1);
                    }
                    return best;
                };
                // smallest seed distance of a border vertex not reached yet (block-uniform)
                auto ring_min = [&]() -> int {
                    int best = kInf;
                    for (int i = tid; i < A.nring; i += NT)
                        if (S[A.ringL[i]] == kInf) best = min(best, seed_dist(i));
                    best = wave_min_i(best);
                    if ((tid & 63) == 0) s_wmin[tid >> 6] = best;
                    __syncthreads();
                    if (tid == 0) {
                        int b = kInf;
                        for (int w = 0; w < NT / 64; w++) b = min(b, s_wmin[w]);
                        s_min = b;
                    }
                    __syncthreads();
                    return s_min;
                };
                auto add_seeds = [&](int dist, int step) {
                    for (int i = tid; i < A.nring; i += NT) {
                        const int l = A.ringL[i];
                        if (S[l] != kInf || seed_dist(i) != dist) continue;
                        if (atomicCAS(&S[l], kInf, step) == kInf) {
                            Q[atomicAdd(&s_qtail, 1)] = l;
                            if (ex[base + l] > 0) {
                                atomicSub(&s_live, 1);
                                s_hit = 1;
                            }
                        }
                    }
                };
                // step 0 is distance 1: the vertices with c_f(u, t) > 0 (queued by the
                // pass above) and the seeds at distance 1
                int nextSeed = ring_min();
                if (nextSeed == 1) {
                    add_seeds(1, 0);
                    __syncthreads();
                    nextSeed = ring_min();
                }
                if (tid == 0 && s_qtail > 0) {
                    stepEnd[0] = s_qtail;
                    stepLevel[0] = 1;
                    s_nsteps = 1;
                }
                __syncthreads();
                int fs = 0;
                for (;;) {
                    // every thread reads the level's bounds before any thread appends
                    const bool stop = earlyOk && s_hit && s_live == 0;
                    const int fe = s_qtail;
                    const int step = s_nsteps;
                    __syncthreads();
                    if (stop) {
                        early = true;
                        break;
                    }
                    int Dn;
                    if (fs == fe) {
                        if (nextSeed == kInf) break;
                        Dn = nextSeed;  // jump to the next seed distance
                    } else {
                        Dn = stepLevel[step - 1] + 1;
                        for (int i = fs + tid; i < fe; i += NT) {
                            const int v = Q[i];
                            int vz, vy, vx;
                            local_xyz(G, v, vz, vy, vx);
                            for (int k = 0; k < G.K; k++) {
                                const int u = local_nbr(G, vz, vy, vx, k ^ 1);  // u + o_k = v
                                if (u < 0) continue;
                                if (res[(size_t)k * N + base + u] > 0 && S[u] == kInf &&
                                    atomicCAS(&S[u], kInf, step) == kInf) {
                                    Q[atomicAdd(&s_qtail, 1)] = u;
                                    if (ex[base + u] > 0) {
                                        atomicSub(&s_live, 1);
                                        s_hit = 1;
                                    }
                                }
                            }
                        }
                    }
                    if (nextSeed == Dn) add_seeds(Dn, step);
                    __syncthreads();
                    if (tid == 0 && s_qtail > fe) {
                        stepEnd[step] = s_qtail;
                        stepLevel[step] = Dn;
                        s_nsteps = step + 1;
                    }
                    if (nextSeed == Dn) nextSeed = ring_min();
                    fs = fe;
                    __syncthreads();
                }
            } else {
                if (tid == 0 && s_qtail > 0) {
                    stepEnd[0] = s_qtail;
                    stepLevel[0] = 0;
                    s_nsteps = 1;
                }
                __syncthreads();
                int fs = 0;
                for (;;) {
                    // flood inside the region: u with c_f(u, v) > 0 to a frontier v
                    for (;;) {
                        // every thread reads the level's bounds before any thread appends
                        const bool stop = earlyOk && s_hit && s_live == 0;
                        const int fe = s_qtail;
                        __syncthreads();
                        if (stop) {
                            early = true;
                            break;
                        }
                        if (fs == fe) break;
                        const int step = s_nsteps;
                        for (int i = fs + tid; i < fe; i += NT) {
                            int v = Q[i];
                            int vz, vy, vx;
                            local_xyz(G, v, vz, vy, vx);
                            for (int k = 0; k < G.K; k++) {
                                int u = local_nbr(G, vz, vy, vx, k ^ 1);  // u + o_k = v
                                if (u < 0) continue;
                                if (res[(size_t)k * N + base + u] > 0 && S[u] == kInf) {
                                    if (atomicCAS(&S[u], kInf, step) == kInf) {
                                        Q[atomicAdd(&s_qtail, 1)] = u;
                                        if (ex[base + u] > 0) {
                                            atomicSub(&s_live, 1);
                                            s_hit = 1;
                                        }
                                    }
                                }
                            }
                        }
                        __syncthreads();
                        if (tid == 0 && s_qtail > fe) {
                            stepEnd[step] = s_qtail;
                            stepLevel[step] = step > 0 ? stepLevel[step - 1] : 0;
                            s_nsteps = step + 1;
                        }
                        fs = fe;
                        __syncthreads();
                    }
                    if (early) break;
                    // next stage: smallest d(w) + 1 over residual boundary arcs of unlabeled u
                    int best = kInf;
                    for (int i = tid; i < A.nring; i += NT) {
                        int l = A.ringL[i];
                        if (S[l] != kInf) continue;
                        unsigned m = A.ringM[i];
                        int lz, ly, lx;
                        local_xyz(G, l, lz, ly, lx);
                        for (int k = 0; k < G.K; k++) {
                            if (!((m >> k) & 1u)) continue;
                            if (res[(size_t)k * N + base + l] <= 0) continue;
                            int w = cross_nbr(G, r, lz, ly, lx, k);
                            if (w < 0) continue;
                            int d = labOld[w];
                            if (d < dinf) best = min(best, d + 1);
                        }
                    }
                    best = wave_min_i(best);
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
                    const int step = s_nsteps;
                    for (int i = tid; i < A.nring; i += NT) {
                        int l = A.ringL[i];
                        if (S[l] != kInf) continue;
                        unsigned m = A.ringM[i];
                        int lz, ly, lx;
                        local_xyz(G, l, lz, ly, lx);
                        for (int k = 0; k < G.K; k++) {
                            if (!((m >> k) & 1u)) continue;
                            if (res[(size_t)k * N + base + l] <= 0) continue;
                            int w = cross_nbr(G, r, lz, ly, lx, k);
                            if (w < 0) continue;
                            int d = labOld[w];
                            if (d < dinf && d + 1 == level) {
                                S[l] = step;
                                Q[atomicAdd(&s_qtail, 1)] = l;
                                if (ex[base + l] > 0) {
                                    atomicSub(&s_live, 1);
                                    s_hit = 1;
                                }
                                break;
                            }
                        }
                    }
                    __syncthreads();
                    if (tid == 0) {
                        // at least one seed exists: level came from an unlabeled ring vertex
                        stepEnd[step] = s_qtail;
                        stepLevel[step] = level;
                        s_nsteps = step + 1;
                    }
                    __syncthreads();
                }
            }
            bfs_steps += s_nsteps;
            firstSearch = false;
            lastComplete = !early && !capped;
            if (relabelOnly) break;
            // ---------------- any excess vertex that reaches a target? ----------------
            int found = 0;
            if (early) {
                found = 1;  // every live excess vertex is labelled
            } else {
                for (int l = tid; l < V; l += NT)
                    if (S[l] < kDead && ex[base + l] > 0) found = 1;
            }
            if (found) s_found = 1;
            __syncthreads();
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
            const int nsteps = s_nsteps;
            for (int s = nsteps - 1; s >= 0; s--) {
                const int lo = s > 0 ? stepEnd[s - 1] : 0, hi = stepEnd[s];
                const int L = stepLevel[s];
                if (A.prd) {
                    // Push along admissible arcs, d(u) = d(v) + 1: into t at distance
                    // 1, to the previous step when it is distance L - 1, and over
                    // boundary arcs to w with d(w) + 1 = L
                    const bool adjPrev = s > 0 && stepLevel[s - 1] == L - 1;
                    for (int i = lo + tid; i < hi; i += NT) {
                        const int u = Q[i];
                        int e = ex[base + u];
                        if (e <= 0) continue;
                        int uz, uy, ux;
                        local_xyz(G, u, uz, uy, ux);
                        if (L == 1) {
                            const int t = rt[base + u];
                            if (t > 0) {
                                const int d = min(e, t);
                                rt[base + u] = t - d;
                                e -= d;
                                if (A.trace) atomicAdd((unsigned long long *)&s_tr[1], (u64)d);
                            }
                        }
                        for (int k = 0; k < G.K && e > 0; k++) {
                            const size_t a = (size_t)k * N + base + u;
                            const int c = res[a];
                            if (c <= 0) continue;
                            const int v = local_nbr(G, uz, uy, ux, k);
                            if (v >= 0) {
                                if (!adjPrev || S[v] != s - 1) continue;
                                const int d = min(e, c);
                                res[a] = c - d;
                                res[(size_t)(k ^ 1) * N + base + v] += d;
                                atomicAdd(&ex[base + v], d);
                                e -= d;
                            } else {
                                const int w = cross_nbr(G, r, uz, uy, ux, k);
                                if (w < 0) continue;
                                const int dw = labOld[w];
                                if (dw >= dinf || dw + 1 != L) continue;
                                const int d = min(e, c);
                                res[a] = c - d;
                                pushb[a] += d;
                                e -= d;
                                if (A.trace) atomicAdd((unsigned long long *)&s_tr[2], (u64)d);
                            }
                        }
                        ex[base + u] = e;
                    }
                    __syncthreads();
                    continue;
                }
                const bool seed = (s == 0) || (stepLevel[s - 1] != L);
                for (int i = lo + tid; i < hi; i += NT) {
                    const int u = Q[i];
                    int e = ex[base + u];
                    if (e <= 0) continue;
                    int uz, uy, ux;
                    local_xyz(G, u, uz, uy, ux);
                    if (seed) {
                        if (L == 0) {
                            int t = rt[base + u];
                            if (t > 0) {
                                int d = min(e, t);
                                rt[base + u] = t - d;
                                e -= d;
                                if (A.trace) atomicAdd((unsigned long long *)&s_tr[1], (u64)d);
                            }
                        } else {
                            for (int k = 0; k < G.K && e > 0; k++) {
                                if (local_nbr(G, uz, uy, ux, k) >= 0) continue;
                                const size_t a = (size_t)k * N + base + u;
                                int c = res[a];
                                if (c <= 0) continue;
                                int w = cross_nbr(G, r, uz, uy, ux, k);
                                if (w < 0) continue;
                                int dw = labOld[w];
                                if (dw >= dinf || dw + 1 != L) continue;
                                int d = min(e, c);
                                res[a] = c - d;
                                pushb[a] += d;
                                e -= d;
                                if (A.trace) atomicAdd((unsigned long long *)&s_tr[2], (u64)d);
                            }
                        }
                    } else {
                        for (int k = 0; k < G.K && e > 0; k++) {
                            int v = local_nbr(G, uz, uy, ux, k);
                            if (v < 0) continue;
                            const size_t a = (size_t)k * N + base + u;
                            int c = res[a];
                            if (c <= 0 || S[v] != s - 1) continue;
                            int d = min(e, c);
                            res[a] = c - d;
                            res[(size_t)(k ^ 1) * N + base + v] += d;
                            atomicAdd(&ex[base + v], d);
                            e -= d;
                        }
                    }
                    ex[base + u] = e;
                }
                __syncthreads();
            }
        }
        // ---------------- region relabel result ----------------
        for (int l = tid; l < V; l += NT) {
            int s = S[l];
            A.labNew[base + l] = (s >= kDead) ? dinf : min(stepLevel[s], dinf);
        }
        if (A.trace) {
            long long ex_out = 0, lsum = 0;
            for (int l = tid; l < V; l += NT) ex_out += ex[base + l];
            for (int i = tid; i < A.nring; i += NT) {
                const int s = S[A.ringL[i]];
                lsum += (s >= kDead) ? 65535 : min(stepLevel[s], 65535);
            }
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
            atomicAdd(&A.stats[3], (u64)bfs_steps);
            atomicAdd(&A.stats[4], (u64)classes);
            if (A.trace) {
                unsigned long long idx = atomicAdd(&A.stats[5], 1ull);
                if ((long long)idx < A.traceCap) {
                    int *rec = A.trace + idx * 10;
                    rec[0] = A.sweep;
                    rec[1] = r;
                    rec[2] = iter + 1;
                    rec[3] = (int)min(bfs_steps, 0x7fffffffLL);
                    rec[4] = (int)min(classes, 0x7fffffffLL);
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
// Flow fusion (Alg. 2): for every inter-region pair {u, v} a push u -> v stays
// iff d'(v) <= d'(u) + 1, otherwise it returns to u; same for v -> u.  One
// thread per boundary vertex handles its pairs in the canonical (even)
// directions, so every pair has exactly one owner.  Also builds the histogram
// of boundary labels for the gap heuristic.
// ---------------------------------------------------------------------------
// Adds one label per thread (-1: none) to the boundary-label histogram of the
// gap heuristic through block-privatised bins in LDS (zeroed and synchronised
// by the caller), and the block's largest label to maxlab.  256 threads.
__device__ void boundary_hist(unsigned int *lh, int *s_wmax, int mylab, unsigned int *hist,
                              int *maxlab) {
    if (mylab >= 0) {
        if (mylab < kHistLds) atomicAdd(&lh[mylab], 1u);
        else if (mylab < kHistBins) atomicAdd(&hist[mylab], 1u);
    }
    int m = wave_max_i(mylab);
    if ((threadIdx.x & 63) == 0) s_wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    for (int b = threadIdx.x; b < kHistLds; b += blockDim.x)
        if (lh[b]) atomicAdd(&hist[b], lh[b]);
    if (threadIdx.x == 0) {
        int mm = -1;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) mm = max(mm, s_wmax[w]);
        if (mm >= 0) atomicMax(maxlab, mm);
    }
}

__global__ void k_fuse(FuseArgs A) {
    __shared__ unsigned int lh[kHistLds];
    __shared__ int s_wmax[4];
    if (*A.actIn == 0ull) return;
    const Geo &G = A.G;
    const int N = G.N;
    for (int i = threadIdx.x; i < kHistLds; i += blockDim.x) lh[i] = 0;
    __syncthreads();
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int mylab = -1;
    if (i < A.nB) {
        const int u = A.bidx[i];
        const int r = u / G.V, l = u - r * G.V;
        int lz, ly, lx;
        local_xyz(G, l, lz, ly, lx);
        const int du = A.lab[u];
        int addu = 0;
        for (int k = 0; k < G.K; k += 2) {
            if (local_nbr(G, lz, ly, lx, k) >= 0) continue;
            int v = cross_nbr(G, r, lz, ly, lx, k);
            if (v < 0) continue;
            const size_t auv = (size_t)k * N + u, avu = (size_t)(k ^ 1) * N + v;
            int pout = A.pushb[auv], pin = A.pushb[avu];
            if ((pout | pin) == 0) continue;
            const int dv = A.lab[v];
            A.pushb[auv] = 0;
            A.pushb[avu] = 0;
            int addv = 0;
            if (pout) {
                if (dv <= du + 1) { A.res[avu] += pout; addv += pout; }
                else { A.res[auv] += pout; addu += pout; }
            }
            if (pin) {
                if (du <= dv + 1) { A.res[auv] += pin; addu += pin; }
                else { A.res[avu] += pin; addv += pin; }
            }
            if (addv) atomicAdd(&A.ex[v], addv);
        }
        if (addu) atomicAdd(&A.ex[u], addu);
        if (du < A.dinf) mylab = du;
    }
    if (A.histOn) boundary_hist(lh, s_wmax, mylab, A.hist, A.maxlab);
}

// Global gap (Sec. 5.1, over boundary labels): the smallest g >= 1 below the
// highest boundary label with no boundary vertex labelled g.  Also closes the
// sweep: counts it, resets the next sweep's queue and active counter.
__global__ void k_gap_find(GapArgs A) {
    __shared__ int s_wmin[16];
    const int tid = threadIdx.x;
    if (*A.actIn == 0ull) {
        if (tid == 0) {
            *A.actOut = 0ull;
            *A.qheadNext = 0u;
        }
        return;
    }
    int top = *A.maxlab;
    int lim = min(top, kHistBins);
    int g = kInf;
    if (A.gapOn) {
        for (int l = 1 + tid; l < lim; l += blockDim.x)
            if (A.hist[l] == 0u) { g = l; break; }
    }
    g = wave_min_i(g);
    if ((tid & 63) == 0) s_wmin[tid >> 6] = g;
    __syncthreads();
    if (tid == 0) {
        int b = kInf;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) b = min(b, s_wmin[w]);
        *A.gap = (b == kInf) ? -1 : b;
        // the boundary kernel adds the active boundary vertices; regions that a
        // partial discharge left active come from the carry
        if (A.actCarry) {
            *A.actOut = *A.actCarry;
            *A.actCarry = 0ull;
        } else {
            *A.actOut = 0ull;
        }
        *A.qheadNext = 0u;
        *A.maxlab = -1;
        A.counters[0] += 1ull;  // sweeps
    }
    __syncthreads();
    int clr = min(top + 1, kHistBins);
    for (int l = tid; l < clr; l += blockDim.x) A.hist[l] = 0u;
}

__global__ void k_gap_apply(GapApplyArgs A) {
    __shared__ int s_w[4];
    if (*A.actIn == 0ull) return;
    const Geo &G = A.G;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int act = 0;
    if (i < A.nB) {
        const int u = A.bidx[i];
        const int g = *A.gap;
        int d = A.lab[u];
        if (g >= 0 && d > g && d < A.dinf) {
            d = A.dinf;
            A.lab[u] = d;
        }
        if (A.ex[u] > 0 && d < A.dinf) {
            act = 1;
            A.ractive[u / G.V] = 1;
        }
    }
    act = wave_sum_i(act);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = act;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) t += s_w[w];
        if (t) atomicAdd(A.actOut, (u64)t);
    }
}

// Histogram of all labels below dinf (the global gap of push-relabel region
// discharge, whose labels count every arc: a gap must be empty over all
// vertices, not only over B) and the largest such label.
__global__ void k_label_hist(const int *lab, int N, int dinf, unsigned int *hist, int *maxlab,
                             const unsigned long long *actIn) {
    __shared__ unsigned int lh[kHistLds];
    __shared__ int s_wmax[4];
    if (*actIn == 0ull) return;
    for (int b = threadIdx.x; b < kHistLds; b += blockDim.x) lh[b] = 0u;
    __syncthreads();
    int mx = -1;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const int d = lab[i];
        if (d >= dinf) continue;
        if (d < kHistLds) atomicAdd(&lh[d], 1u);
        else if (d < kHistBins) atomicAdd(&hist[d], 1u);
        mx = max(mx, d);
    }
    mx = wave_max_i(mx);
    if ((threadIdx.x & 63) == 0) s_wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    for (int b = threadIdx.x; b < kHistLds; b += blockDim.x)
        if (lh[b]) atomicAdd(&hist[b], lh[b]);
    if (threadIdx.x == 0) {
        int mm = -1;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) mm = max(mm, s_wmax[w]);
        if (mm >= 0) atomicMax(maxlab, mm);
    }
}

// The gap over all vertices (push-relabel region discharge): with distance
// labels a raised boundary vertex may have a residual arc into an interior
// vertex above the gap, which must be raised too for the labeling to stay valid.
__global__ void k_gap_raise_all(int *lab, int N, const int *gap, int dinf,
                                const unsigned long long *actIn) {
    if (*actIn == 0ull) return;
    const int g = *gap;
    if (g < 0) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const int d = lab[i];
        if (d > g && d < dinf) lab[i] = dinf;
    }
}

// ---------------------------------------------------------------------------
// Boundary relabel heuristic (Sec. 6.1).  Groups are the (region, label)
// classes of the boundary vertices labelled below dinf; a group reaches the
// group of every larger label of its region at length 0 (a chain of
// consecutive labels) and, through each residual arc (u, w) between regions,
// the group of w at length 1.  d' is the distance to a label-0 group.
// Searched level by level from the label-0 vertices: level D + 1 of region R
// is every unreached vertex of R labelled at most M, where M is the largest
// label of an unreached vertex of R with a residual arc into a vertex at
// distance D (the zero-length arcs lead from a label to all larger ones).
// ctl: [0..2] vertices reached per level, rotating (level D counts into D % 3,
// reads D - 1 from (D + 2) % 3 and clears (D + 1) % 3 for the next level);
// [3] the search has ended; [4] levels that reached a vertex.
// ---------------------------------------------------------------------------
__global__ void k_brl_init(BrlArgs A) {
    if (A.actIn && *A.actIn == 0ull) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0)
        for (int c = 0; c < 5; c++) A.ctl[c] = 0u;
    if (i < A.nB) {
        const int u = A.bidx[i];
        A.dist[u] = A.lab[u] == 0 ? 0 : kInf;
    }
}

__global__ __launch_bounds__(256) void k_brl_level(BrlArgs A, int D) {
    __shared__ int s_m, s_c;
    if (A.actIn && *A.actIn == 0ull) return;
    if (A.ctl[3]) return;
    if (D > 0 && A.ctl[(D + 2) % 3] == 0u) {
        // the previous level reached nothing: no vertex is at distance D
        if (threadIdx.x == 0) A.ctl[3] = 1u;
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) A.ctl[(D + 1) % 3] = 0u;
    const Geo &G = A.G;
    const int r = blockIdx.x;
    const int b0 = A.bstart[r], b1 = A.bstart[r + 1];
    if (b0 == b1) return;
    if (threadIdx.x == 0) {
        s_m = -1;
        s_c = 0;
    }
    __syncthreads();
    int m = -1;
    for (int i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
        const int u = A.bidx[i];
        if (A.dist[u] != kInf) continue;
        const int du = A.lab[u];
        if (du >= A.dinf || du <= m) continue;  // only a larger label can raise M
        int lz, ly, lx;
        local_xyz(G, u - r * G.V, lz, ly, lx);
        for (int k = 0; k < G.K; k++) {
            if (local_nbr(G, lz, ly, lx, k) >= 0) continue;
            const int w = cross_nbr(G, r, lz, ly, lx, k);
            if (w < 0) continue;
            if (A.res[(size_t)k * G.N + u] > 0 && A.dist[w] == D) {
                m = du;
                break;
            }
        }
    }
    m = wave_max_i(m);
    if ((threadIdx.x & 63) == 0 && m >= 0) atomicMax(&s_m, m);
    __syncthreads();
    const int M = s_m;
    if (M < 0) return;
    int c = 0;
    for (int i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
        const int u = A.bidx[i];
        if (A.dist[u] != kInf) continue;
        const int du = A.lab[u];
        if (du <= M) {  // M < dinf, so du < dinf
            A.dist[u] = D + 1;
            c++;
        }
    }
    c = wave_sum_i(c);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(&s_c, c);
    __syncthreads();
    if (threadIdx.x == 0 && s_c) {
        atomicAdd(&A.ctl[D % 3], (unsigned)s_c);
        atomicMax(&A.ctl[4], (unsigned)(D + 1));
    }
}

// d := max(d, d') on B, with d' = dinf where the search ended without reaching
// the vertex and levels + 1 where the level budget ran out first; optionally
// builds the boundary-label histogram of the gap heuristic.
__global__ __launch_bounds__(256) void k_brl_apply(BrlArgs A) {
    __shared__ unsigned int lh[kHistLds];
    __shared__ int s_wmax[4];
    if (A.actIn && *A.actIn == 0ull) return;
    if (A.hist) {
        for (int b = threadIdx.x; b < kHistLds; b += blockDim.x) lh[b] = 0u;
        __syncthreads();
    }
    const bool ended = A.ctl[3] != 0u || A.ctl[(A.levels + 2) % 3] == 0u;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int mylab = -1;
    if (i < A.nB) {
        const int u = A.bidx[i];
        const int d = A.lab[u];
        if (d < A.dinf) {
            int dp = A.dist[u];
            if (dp == kInf) dp = ended ? A.dinf : A.levels + 1;
            const int nd = max(d, min(dp, A.dinf));
            if (nd != d) A.lab[u] = nd;
            if (nd < A.dinf) mylab = nd;
        }
    }
    if (A.hist) boundary_hist(lh, s_wmax, mylab, A.hist, A.maxlab);
}

// ---------------------------------------------------------------------------
// Results
// ---------------------------------------------------------------------------
__global__ void k_sum_i32(const int *a, int n, u64 *out) {
    long long s = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) s += a[i];
    s = wave_sum_ll(s);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(out, (u64)s);
}

// blocked -> row-major copy of one int32 plane
__global__ void k_gather_plane(Geo G, const int *src, int *dst, int n) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int x = v % G.dx, t = v / G.dx, y = t % G.dy, z = t / G.dy;
    dst[v] = src[grid_to_blocked(G, z, y, x)];
}

// Label trace of one step: the labels of the last step that ran.  Step k of a
// solve writes buffer (k + 1) & 1 and the step counter counts the steps that
// ran, so the current labels are in buffer (count & 1), also after steps that
// found no active vertex and exited at once (one buffer: lab0 == lab1).
// The labels after a step: the larger entry of the two buffers (labels never
// decrease, and a region skipped by a sweep refreshes only its border labels
// in the new buffer, so the other buffer may hold its current interior).
__global__ void k_trace_labels(Geo G, const int *lab0, const int *lab1,
                               const unsigned long long *count, int *dst, int n) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    (void)count;
    int x = v % G.dx, t = v / G.dx, y = t % G.dy, z = t / G.dy;
    const int g = grid_to_blocked(G, z, y, x);
    dst[v] = max(lab0[g], lab1[g]);
}

// dst[g] = max(dst[g], other[g]): the current labels into one buffer.
__global__ void k_label_max(int *dst, const int *other, int N) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < N; g += gridDim.x * blockDim.x) {
        const int o = other[g];
        if (o > dst[g]) dst[g] = o;
    }
}

// Residual reachability by region floods: each workgroup floods its region
// from the marked vertices, marks across the region border and flags the
// neighbouring region for the next round.  dir 0: forward from the excess
// vertices (minimal source side); dir 1: backward from t (the sink side T).
template <int NT>
__global__ __launch_bounds__(NT) void k_flood(FloodArgs A) {
    __shared__ int s_qtail, s_go;
    const Geo &G = A.G;
    const int V = G.V, N = G.N, tid = threadIdx.x;
    int *Q = A.scratch + (size_t)blockIdx.x * V;
    for (int r = blockIdx.x; r < G.nreg; r += gridDim.x) {
        const int base = r * V;
        if (tid == 0) {
            s_go = (A.round == 0) ? 1 : A.dirtyIn[r];
            A.dirtyIn[r] = 0;
            s_qtail = 0;
        }
        __syncthreads();
        if (!s_go) { __syncthreads(); continue; }
        for (int l = tid; l < V; l += NT) {
            int m = A.mark[base + l];
            if (A.round == 0) {
                int seed = (A.dir == 0) ? (A.ex[base + l] > 0) : (A.rt[base + l] > 0);
                if (seed) { A.mark[base + l] = 1; m = 1; }
            }
            if (m) Q[atomicAdd(&s_qtail, 1)] = l;
        }
        __syncthreads();
        int fs = 0;
        for (;;) {
            const int fe = s_qtail;
            __syncthreads();  // every thread has the level's end before any thread appends
            if (fs == fe) break;
            for (int i = fs + tid; i < fe; i += NT) {
                const int v = Q[i];
                int vz, vy, vx;
                local_xyz(G, v, vz, vy, vx);
                for (int k = 0; k < G.K; k++) {
                    if (A.dir == 0) {
                        // forward: arc (v, v + o_k) with c_f > 0
                        if (A.res[(size_t)k * N + base + v] <= 0) continue;
                        int w = local_nbr(G, vz, vy, vx, k);
                        if (w >= 0) {
                            if (atomicExch(&A.mark[base + w], 1) == 0) Q[atomicAdd(&s_qtail, 1)] = w;
                        } else if (!A.noCross) {
                            int wg = cross_nbr(G, r, vz, vy, vx, k);
                            if (wg >= 0 && atomicExch(&A.mark[wg], 1) == 0) {
                                A.dirtyOut[wg / V] = 1;
                                atomicAdd(A.changed, 1u);
                            }
                        }
                    } else {
                        // backward: arc (u, v) with u = v - o_k and c_f(u, v) > 0
                        int w = local_nbr(G, vz, vy, vx, k ^ 1);
                        if (w >= 0) {
                            if (A.res[(size_t)k * N + base + w] > 0 && atomicExch(&A.mark[base + w], 1) == 0)
                                Q[atomicAdd(&s_qtail, 1)] = w;
                        } else if (!A.noCross) {
                            int wg = cross_nbr(G, r, vz, vy, vx, k ^ 1);
                            if (wg >= 0 && A.res[(size_t)k * N + wg] > 0 && atomicExch(&A.mark[wg], 1) == 0) {
                                A.dirtyOut[wg / V] = 1;
                                atomicAdd(A.changed, 1u);
                            }
                        }
                    }
                }
            }
            __syncthreads();
            fs = fe;
            __syncthreads();
        }
    }
}

// Region reduction (Alg. 5, Sec. 8): the auxiliary problem with every boundary
// vertex a source without bound, for every region at once.  After Init, each
// vertex u with a neighbour w in another region takes the whole capacity
// c(w, u) into its excess, and its residual c_f(u, w) becomes c(u, w) + c(w, u).
// Each thread changes only its own vertex, and a region discharge never reads
// the residuals of arcs entering its region, so every region sees its own
// network.
__global__ void k_saturate_inflow(Geo G, const int *nbr, int n, int *res, int *ex) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < G.N; g += gridDim.x * blockDim.x) {
        int z, y, x;
        if (!blocked_to_grid(G, g, z, y, x)) continue;
        const int r = g / G.V;
        const int v = (z * G.dy + y) * G.dx + x;
        int add = 0;
        for (int k = 0; k < G.K; k++) {
            const int wz = z + G.oz[k], wy = y + G.oy[k], wx = x + G.ox[k];
            if ((unsigned)wz >= (unsigned)G.dz || (unsigned)wy >= (unsigned)G.dy || (unsigned)wx >= (unsigned)G.dx)
                continue;
            if (grid_to_blocked(G, wz, wy, wx) / G.V == r) continue;
            const int w = (wz * G.dy + wy) * G.dx + wx;
            const int cwu = nbr[(size_t)(k ^ 1) * n + w];
            add += cwu;
            res[(size_t)k * G.N + g] = nbr[(size_t)k * n + v] + cwu;
        }
        ex[g] += add;
    }
}

// Class bits of one auxiliary problem from its maximum preflow: the region
// labels (dinf = reaches no target) and the marks of the in-region forward
// search from the excess vertices (the minimal source side).
__global__ void k_reduce_classes(Geo G, const int *lab, const int *mark, unsigned char *cls, int dinf,
                                 int sinkSide) {
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < G.N; g += gridDim.x * blockDim.x) {
        const bool reached = mark[g] != 0, noTarget = lab[g] >= dinf;
        unsigned c = sinkSide ? cls[g] : 0u;
        if (!sinkSide) {
            // boundary joined to t: strong source = minimal source side; weak
            // source = maximal minus minimal source side
            if (reached) c |= 1u;
            if (noTarget && !reached) c |= 4u;
        } else {
            // boundary supplied from s: strong sink = outside the maximal source
            // side; weak sink = maximal minus minimal source side
            if (!noTarget) c |= 2u;
            if (noTarget && !reached) c |= 8u;
        }
        cls[g] = (unsigned char)c;
    }
}

// blocked bytes -> row-major bytes
__global__ void k_gather_bytes(Geo G, const unsigned char *src, unsigned char *out, int n) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int x = v % G.dx, t = v / G.dx, y = t % G.dy, z = t / G.dy;
    out[v] = src[grid_to_blocked(G, z, y, x)];
}

// blocked marks -> row-major source-side indicator
__global__ void k_cut_out(Geo G, const int *mark, unsigned char *out, int n, int invert) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int x = v % G.dx, t = v / G.dx, y = t % G.dy, z = t / G.dy;
    int m = mark[grid_to_blocked(G, z, y, x)] ? 1 : 0;
    out[v] = (unsigned char)(invert ? 1 - m : m);
}

__global__ void k_fill_i32(int *p, int n, int val) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = val;
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
static inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }

hipError_t launch_validate(const Geo &G, const int *cs, const int *ct, const int *nbr, int n,
                           int *err, hipStream_t s) {
    hipLaunchKernelGGL(k_validate, dim3(cdiv(n, 256)), dim3(256), 0, s, G, cs, ct, nbr, n, err);
    return hipGetLastError();
}

hipError_t launch_sum_links(const int *cs, const int *ct, int n, unsigned long long *out2,
                            hipStream_t s) {
    int blocks = min(cdiv(n, 256), 1024);
    hipLaunchKernelGGL(k_sum_links, dim3(blocks), dim3(256), 0, s, cs, ct, n, out2);
    return hipGetLastError();
}

hipError_t launch_init(const Geo &G, const int *cs, const int *ct, const int *nbr, int n, int *res,
                       int *rt, int *ex, int *lab0, int *lab1, int *pushb, int *ractive,
                       unsigned long long *act0, hipStream_t s) {
    hipLaunchKernelGGL(k_init, dim3(std::min(cdiv(G.N, 256), kCountBlocks)), dim3(256), 0, s, G, cs, ct,
                       nbr, n, res, rt, ex, lab0, lab1, pushb, ractive, act0);
    return hipGetLastError();
}

void set_hbm_attributes() {
    (void)hipFuncSetAttribute((const void *)k_discharge<256>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute((const void *)k_discharge<512>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();
}

hipError_t launch_discharge(const DischargeArgs &A, int blocks, int threads, size_t lds,
                            hipStream_t s) {
    if (threads == 256)
        hipLaunchKernelGGL(k_discharge<256>, dim3(blocks), dim3(256), lds, s, A);
    else if (threads == 512)
        hipLaunchKernelGGL(k_discharge<512>, dim3(blocks), dim3(512), lds, s, A);
    else if (threads == 1024)
        hipLaunchKernelGGL(k_discharge<1024>, dim3(blocks), dim3(1024), lds, s, A);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_fuse(const FuseArgs &A, hipStream_t s) {
    if (A.nB == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fuse, dim3(cdiv(A.nB, 256)), dim3(256), 0, s, A);
    return hipGetLastError();
}

// stage 0: init; 1: levels [first, first + count); 2: apply with A.levels levels run
hipError_t launch_boundary_relabel(const BrlArgs &A, int stage, int first, int count, hipStream_t s) {
    if (A.nB == 0) return hipSuccess;
    if (stage == 0) {
        hipLaunchKernelGGL(k_brl_init, dim3(cdiv(A.nB, 256)), dim3(256), 0, s, A);
    } else if (stage == 1) {
        for (int D = first; D < first + count; D++)
            hipLaunchKernelGGL(k_brl_level, dim3(A.G.nreg), dim3(256), 0, s, A, D);
    } else {
        if (A.levels <= 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_brl_apply, dim3(cdiv(A.nB, 256)), dim3(256), 0, s, A);
    }
    return hipGetLastError();
}

hipError_t launch_label_hist(const int *lab, int N, int dinf, unsigned int *hist, int *maxlab,
                             const unsigned long long *actIn, hipStream_t s) {
    hipLaunchKernelGGL(k_label_hist, dim3(min(cdiv(N, 256), 1024)), dim3(256), 0, s, lab, N, dinf,
                       hist, maxlab, actIn);
    return hipGetLastError();
}

hipError_t launch_gap_raise_all(int *lab, int N, const int *gap, int dinf,
                                const unsigned long long *actIn, hipStream_t s) {
    hipLaunchKernelGGL(k_gap_raise_all, dim3(min(cdiv(N, 256), 1024)), dim3(256), 0, s, lab, N, gap,
                       dinf, actIn);
    return hipGetLastError();
}

hipError_t launch_gap_find(const GapArgs &A, hipStream_t s) {
    hipLaunchKernelGGL(k_gap_find, dim3(1), dim3(1024), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_gap_apply(const GapApplyArgs &A, hipStream_t s) {
    if (A.nB == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gap_apply, dim3(cdiv(A.nB, 256)), dim3(256), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_sum_i32(const int *a, int n, unsigned long long *out, hipStream_t s) {
    int blocks = min(cdiv(n, 256), 1024);
    hipLaunchKernelGGL(k_sum_i32, dim3(blocks), dim3(256), 0, s, a, n, out);
    return hipGetLastError();
}

hipError_t launch_gather_plane(const Geo &G, const int *src, int *dst, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_plane, dim3(cdiv(n, 256)), dim3(256), 0, s, G, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_trace_labels(const Geo &G, const int *lab0, const int *lab1,
                               const unsigned long long *count, int *dst, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_trace_labels, dim3(cdiv(n, 256)), dim3(256), 0, s, G, lab0, lab1, count, dst, n);
    return hipGetLastError();
}

hipError_t launch_label_max(int *dst, const int *other, int N, hipStream_t s) {
    if (N <= 0 || dst == other) return hipSuccess;
    hipLaunchKernelGGL(k_label_max, dim3(std::min(cdiv(N, 256), kCountBlocks)), dim3(256), 0, s, dst, other, N);
    return hipGetLastError();
}

hipError_t launch_saturate_inflow(const Geo &G, const int *nbr, int n, int *res, int *ex, hipStream_t s) {
    hipLaunchKernelGGL(k_saturate_inflow, dim3(std::min(cdiv(G.N, 256), kCountBlocks)), dim3(256), 0, s, G,
                       nbr, n, res, ex);
    return hipGetLastError();
}

hipError_t launch_reduce_classes(const Geo &G, const int *lab, const int *mark, unsigned char *cls,
                                 int dinf, int sinkSide, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_classes, dim3(std::min(cdiv(G.N, 256), kCountBlocks)), dim3(256), 0, s, G,
                       lab, mark, cls, dinf, sinkSide);
    return hipGetLastError();
}

hipError_t launch_gather_bytes(const Geo &G, const unsigned char *src, unsigned char *out, int n,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_gather_bytes, dim3(cdiv(n, 256)), dim3(256), 0, s, G, src, out, n);
    return hipGetLastError();
}

hipError_t launch_flood(const FloodArgs &A, int blocks, hipStream_t s) {
    // regions of 8K vertices and more: bound by memory latency, more loads in flight
    if (A.G.V >= 8192)
        hipLaunchKernelGGL(k_flood<1024>, dim3(blocks), dim3(1024), 0, s, A);
    else
        hipLaunchKernelGGL(k_flood<256>, dim3(blocks), dim3(256), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_cut_out(const Geo &G, const int *mark, unsigned char *out, int n, int invert,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_cut_out, dim3(cdiv(n, 256)), dim3(256), 0, s, G, mark, out, n, invert);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *p, int n, int val, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(cdiv(n, 256)), dim3(256), 0, s, p, n, val);
    return hipGetLastError();
}

}  // namespace mfd

namespace mfd {

// ---------------------------------------------------------------------------
// Global relabel: exact region distance d*B (Sec. 4.1) by a breadth-first
// search from t in which arcs inside a region have length 0 and arcs between
// regions length 1.  One launch per distance D: every flagged region floods
// backwards over its residual arcs from its seeds (D = 0: vertices with a
// residual t-link; D > 0: vertices marked by a neighbouring region at D - 1),
// labelling the unlabelled vertices it reaches with D; a labelled border
// vertex marks its residual predecessors across the region border as seeds of
// D + 1 and flags their regions.  d*B is a valid labeling and an upper bound
// of every valid labeling (Sec. 4.1), so it may replace the labels at any time.
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(NT) void k_grelabel(GRelabelArgs A) {
    __shared__ int s_qtail, s_go;
    const Geo &G = A.G;
    const int V = G.V, N = G.N, tid = threadIdx.x, D = A.level;
    int *Q = A.scratch + (size_t)blockIdx.x * V;
    for (int r = blockIdx.x; r < G.nreg; r += gridDim.x) {
        const int base = r * V;
        if (tid == 0) {
            s_go = (D == 0) ? 1 : A.flagIn[r];
            A.flagIn[r] = 0;
            s_qtail = 0;
        }
        __syncthreads();
        if (!s_go) { __syncthreads(); continue; }
        if (D == 0) {
            for (int l = tid; l < V; l += NT)
                if (A.rt[base + l] > 0) {
                    A.lab[base + l] = 0;
                    Q[atomicAdd(&s_qtail, 1)] = l;
                }
        } else {
            for (int i = tid; i < A.nring; i += NT) {
                const int l = A.ringL[i];
                if (A.candIn[base + l]) {
                    A.candIn[base + l] = 0;
                    if (A.lab[base + l] == A.dinf) {
                        A.lab[base + l] = D;
                        Q[atomicAdd(&s_qtail, 1)] = l;
                    }
                }
            }
        }
        __syncthreads();
        int fs = 0;
        for (;;) {
            const int fe = s_qtail;
            __syncthreads();  // every thread has the level's end before any thread appends
            if (fs == fe) break;
            for (int i = fs + tid; i < fe; i += NT) {
                const int v = Q[i];
                int vz, vy, vx;
                local_xyz(G, v, vz, vy, vx);
                for (int k = 0; k < G.K; k++) {
                    // predecessor u = v - o_k with residual arc (u, v) in direction k
                    const int u = local_nbr(G, vz, vy, vx, k ^ 1);
                    if (u >= 0) {
                        if (A.res[(size_t)k * N + base + u] > 0 && A.lab[base + u] == A.dinf &&
                            atomicCAS(&A.lab[base + u], A.dinf, D) == A.dinf)
                            Q[atomicAdd(&s_qtail, 1)] = u;
                    } else {
                        const int ug = cross_nbr(G, r, vz, vy, vx, k ^ 1);
                        if (ug >= 0 && A.res[(size_t)k * N + ug] > 0 && A.lab[ug] == A.dinf) {
                            A.candOut[ug] = 1;
                            if (atomicExch(&A.flagOut[ug / V], 1) == 0) atomicAdd(A.flagged, 1u);
                        }
                    }
                }
            }
            __syncthreads();
            fs = fe;
            __syncthreads();
        }
    }
}

// Active regions and the active-vertex count after new labels.
__global__ void k_activity(Geo G, const int *ex, const int *lab, int dinf, int *ractive,
                           unsigned long long *act) {
    int a = 0;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < G.N; g += gridDim.x * blockDim.x) {
        if (ex[g] > 0 && lab[g] < dinf) {
            a++;
            ractive[g / G.V] = 1;
        }
    }
    block_count_add(a, act);
}

hipError_t launch_grelabel(const GRelabelArgs &A, int blocks, hipStream_t s) {
    // regions of 8K vertices and more: bound by memory latency, more loads in flight
    if (A.G.V >= 8192)
        hipLaunchKernelGGL(k_grelabel<1024>, dim3(blocks), dim3(1024), 0, s, A);
    else
        hipLaunchKernelGGL(k_grelabel<256>, dim3(blocks), dim3(256), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_activity(const Geo &G, const int *ex, const int *lab, int dinf, int *ractive,
                           unsigned long long *act, hipStream_t s) {
    hipLaunchKernelGGL(k_activity, dim3(std::min(cdiv(G.N, 256), kCountBlocks)), dim3(256), 0, s, G, ex, lab,
                       dinf, ractive, act);
    return hipGetLastError();
}

}  // namespace mfd

namespace mfd {

// ---------------------------------------------------------------------------
// Batches: independent instances packed on one canvas (region-aligned, no
// arcs between instances), so the canvas solve is the union of the instance
// solves.
// ---------------------------------------------------------------------------
__global__ void k_scatter_instance(const int *cs, const int *ct, const int *nbr, int h, int w,
                                   int Ki, int *ccs, int *cct, int *cnbr, int Wc, long long nc,
                                   int y0, int x0) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = h * w;
    if (v >= n) return;
    const int y = v / w, x = v - (v / w) * w;
    const long long cv = (long long)(y0 + y) * Wc + (x0 + x);
    ccs[cv] = cs[v];
    cct[cv] = ct[v];
    for (int k = 0; k < Ki; k++) cnbr[(size_t)k * nc + cv] = nbr[(size_t)k * n + v];
}

// sum of residual t-links per instance (one workgroup per region)
__global__ void k_instance_rt(Geo G, const int *rt, const int *reginst, unsigned long long *instRt) {
    __shared__ long long s_w[4];
    const int r = blockIdx.x;
    const int inst = reginst[r];
    if (inst < 0) return;
    long long a = 0;
    for (int l = threadIdx.x; l < G.V; l += blockDim.x) a += rt[(size_t)r * G.V + l];
    a = wave_sum_ll(a);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long t = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        if (t) atomicAdd(&instRt[inst], (unsigned long long)t);
    }
}

// source-side indicator of one instance's rectangle from the canvas marks
__global__ void k_cut_rect(Geo G, const int *mark, unsigned char *out, int h, int w, int y0, int x0,
                           int invert) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= h * w) return;
    const int y = v / w, x = v - (v / w) * w;
    const int m = mark[grid_to_blocked(G, 0, y0 + y, x0 + x)] ? 1 : 0;
    out[v] = (unsigned char)(invert ? 1 - m : m);
}

hipError_t launch_scatter_instance(const int *cs, const int *ct, const int *nbr, int h, int w, int Ki,
                                   int *ccs, int *cct, int *cnbr, int Wc, long long nc, int y0,
                                   int x0, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_instance, dim3(cdiv((long long)h * w, 256)), dim3(256), 0, s, cs, ct,
                       nbr, h, w, Ki, ccs, cct, cnbr, Wc, nc, y0, x0);
    return hipGetLastError();
}

hipError_t launch_instance_rt(const Geo &G, const int *rt, const int *reginst,
                              unsigned long long *instRt, hipStream_t s) {
    hipLaunchKernelGGL(k_instance_rt, dim3(G.nreg), dim3(256), 0, s, G, rt, reginst, instRt);
    return hipGetLastError();
}

hipError_t launch_cut_rect(const Geo &G, const int *mark, unsigned char *out, int h, int w, int y0,
                           int x0, int invert, hipStream_t s) {
    hipLaunchKernelGGL(k_cut_rect, dim3(cdiv((long long)h * w, 256)), dim3(256), 0, s, G, mark, out, h,
                       w, y0, x0, invert);
    return hipGetLastError();
}

}  // namespace mfd
