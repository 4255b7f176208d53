// Workgroup row-bitmask region discharge for 3D 6-connected regions whose rows
// along x are 32 vertices long and which have at most 1024 rows (Proc. ARD of
// Sec. 4.2 with the region relabel of Alg. 3; same method as k_discharge,
// different execution).
//
// One 1024-thread workgroup owns a region; thread t owns row t = y + ty * z as
// 32-bit masks in registers: residual arc present in each of the six
// directions, residual t-link, excess present, visited, frontier, and the arcs
// by which the search reached each vertex (its admissible arcs).  The integer
// state (residuals, t-links, excess, boundary pushes) stays in HBM; LDS holds
// the exact residual-arc masks of the region, the frontier rows that a search
// level exchanges between neighbouring rows, and the per-row lists of vertices
// whose excess changed in a push iteration, and the halo labels d(w).
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
//   (stage, level) order, so an arc is changed by one side only.
// * Search and push alternate until no excess vertex reaches a target.  The
//   last search is run once more to write the labels (Alg. 3).
#include "mf_device.h"
#include "mf_launch.h"

namespace mfd {

typedef unsigned long long u64;

namespace {

constexpr int kRowsNT = 1024;
constexpr int kRowsWaves = kRowsNT / 64;

struct RowsLayout {
    size_t resM, F, vis, recv, clr, halo, slot, total;  // offsets in 32-bit words
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
    L.halo = o;
    for (int k = 0; k < 6; k++) o += face_size(k, TY, TZ);
    L.slot = o; o += (size_t)nring;  // border vertex: local index | live leaving directions << 16
    L.total = o;
    return L;
}

__device__ __forceinline__ int wave_min_rows(int v) {
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

// Workgroup-wide OR / MIN with one barrier.  The two halves of red[] alternate
// between consecutive calls, so a call never overwrites values that a slower
// wave may still read from the previous one.
__device__ __forceinline__ int block_any(int pred, int (*red)[kRowsWaves], int &rc) {
    const u64 b = __ballot(pred);
    const int p = rc & 1;
    rc++;
    if ((threadIdx.x & 63) == 0) red[p][threadIdx.x >> 6] = (b != 0ull) ? 1 : 0;
    __syncthreads();
    int a = 0;
#pragma unroll
    for (int w = 0; w < kRowsWaves; w++) a |= red[p][w];
    return a;
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

// Direction k of axis a that leaves the tile at a border vertex: exactly one of
// the two directions of an axis leaves it (tiles are at least 2 wide on y and z
// and 32 on x).
__device__ __forceinline__ int axis_dir(unsigned keep, int a) {
    return ((keep >> (2 * a)) & 1u) ? 2 * a : 2 * a + 1;
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

__global__ __launch_bounds__(kRowsNT) void k_discharge_rows(DischargeArgs A) {
    extern __shared__ __align__(16) unsigned smem_rows[];
    __shared__ int red[2][kRowsWaves];
    __shared__ int s_r, s_active;
    __shared__ long long s_tr[4];  // trace: excess out, to sink, to boundary, label sum
    if (*A.actIn == 0ull) return;
    const int V = A.G.V, N = A.G.N, TY = A.G.ty, TZ = A.G.tz, R = TY * TZ;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const RowsLayout L = rows_layout(R, TY, TZ, A.nring);
    unsigned *resM = smem_rows + L.resM;
    unsigned *Fb = smem_rows + L.F;
    unsigned *Vb = smem_rows + L.vis;
    unsigned *recvB = smem_rows + L.recv;
    unsigned *clrB = smem_rows + L.clr;
    int *halo = (int *)(smem_rows + L.halo);
    int *slot = (int *)(smem_rows + L.slot);
    int faceOff[6];
    faceOff[0] = 0;
#pragma unroll
    for (int k = 1; k < 6; k++) faceOff[k] = faceOff[k - 1] + face_size(k - 1, TY, TZ);
    const bool myrow = tid < R;
    const int y = tid % TY, z = tid / TY;
    const int dinf = A.dinf;
    int rc = 0;

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
            // a deferred region keeps its flag and is discharged in a later sweep
            if (s_active && A.defer && A.defer[r]) s_active = 0;
            else A.ractive[r] = 0;
        }
        __syncthreads();
        if (!s_active) {
            // skipped region (no active vertex): labels carry over unchanged
            const int4 *src = (const int4 *)(A.labOld + base);
            int4 *dst = (int4 *)(A.labNew + base);
            for (int i = tid; i < V / 4; i += kRowsNT) dst[i] = src[i];
            __syncthreads();
            continue;
        }
        const long long t_start = wall_clock64();
        if (tid < 4) s_tr[tid] = 0;

        // ---------------- row masks from HBM (coalesced loads + ballots) ----------------
        // Wave w covers rows 64w .. 64w + 63: load i brings rows 64w + 2i and
        // 64w + 2i + 1 (one 32-bit half of the ballot each).  Residual masks go
        // to resM, the t-link and excess masks to the two frontier buffers.
        {
            const int row0 = wid * 64;
            if (row0 + 64 <= R) {
                for (int q = 0; q < 8; q++) {
                    const int *plane = q < 6 ? A.res + (size_t)q * N : (q == 6 ? A.rt : A.ex);
                    unsigned *dst = q < 6 ? resM + q * R : Fb + (q - 6) * R;
                    const int *src = plane + base + (size_t)row0 * 32 + lane;
#pragma unroll 8
                    for (int i = 0; i < 32; i++) {
                        const u64 b = __ballot(src[i * 64] > 0);
                        if (lane == 0) {
                            dst[row0 + 2 * i] = (unsigned)b;
                            dst[row0 + 2 * i + 1] = (unsigned)(b >> 32);
                        }
                    }
                }
            }
        }
        // ---------------- border vertices: halo labels into LDS ----------------
        // slot[i] for border vertex i (handled by thread i mod 1024): local index
        // | (leaving directions with a finite halo label) << 16, or -1
        for (int i = tid; i < A.nring; i += kRowsNT) {
            const int l = A.ringL[i];
            const unsigned mm = A.ringM[i];
            int lz, ly, lx;
            local_xyz(A.G, l, lz, ly, lx);
            unsigned keep = 0u;
            for (int k = 0; k < 6; k++) {
                if (!((mm >> k) & 1u)) continue;
                const int w = cross_nbr(A.G, r, lz, ly, lx, k);
                const int d = w >= 0 ? A.labOld[w] : kInf;
                halo[faceOff[k] + face_pos(k, l, TY)] = d;
                if (d < dinf) keep |= 1u << k;  // otherwise never a target
            }
            slot[i] = keep ? (l | (int)(keep << 16)) : -1;
        }
        __syncthreads();
        unsigned rtM = myrow ? Fb[tid] : 0u;
        unsigned exM = myrow ? Fb[R + tid] : 0u;

        int iter = 0;
        long long levels = 0, stages = 0;
        bool writeMode = false;
        const size_t rowBase = base + (size_t)tid * 32;
        for (;;) {
            // ---------------- multi-level search from the targets ----------------
            unsigned rk[6];
#pragma unroll
            for (int k = 0; k < 6; k++) rk[k] = myrow ? resM[k * R + tid] : 0u;
            unsigned vis = rtM, F = rtM, admT = rtM;
            unsigned adm[6];
#pragma unroll
            for (int k = 0; k < 6; k++) adm[k] = 0u;
            u64 admB = 0ull;  // border slot j (vertex tid + 1024 j), bit 3j + axis: boundary arc to push over
            int p = 0;
            int stage = 0;
            if (writeMode && myrow) store_labels(A.labNew, rowBase, F, 0);
            for (;;) {
                // flood inside the region: u with c_f(u, u + o_k) > 0 and u + o_k in the frontier
                for (;;) {
                    if (myrow) {
                        Fb[p * R + tid] = F;
                        Vb[tid] = vis;
                    }
                    if (!block_any(F != 0u, red, rc)) break;
                    levels++;
                    if (myrow) {
                        const unsigned *Fp = Fb + p * R;
                        const unsigned fyp = (y + 1 < TY) ? Fp[tid + 1] : 0u;
                        const unsigned fym = (y > 0) ? Fp[tid - 1] : 0u;
                        const unsigned fzp = (z + 1 < TZ) ? Fp[tid + TY] : 0u;
                        const unsigned fzm = (z > 0) ? Fp[tid - TY] : 0u;
                        const unsigned t0 = rk[0] & (F >> 1), t1 = rk[1] & (F << 1);
                        const unsigned t2 = rk[2] & fyp, t3 = rk[3] & fym;
                        const unsigned t4 = rk[4] & fzp, t5 = rk[5] & fzm;
                        const unsigned nw = ~vis & (t0 | t1 | t2 | t3 | t4 | t5);
                        adm[0] |= nw & t0;
                        adm[1] |= nw & t1;
                        adm[2] |= nw & t2;
                        adm[3] |= nw & t3;
                        adm[4] |= nw & t4;
                        adm[5] |= nw & t5;
                        vis |= nw;
                        F = nw;
                        if (writeMode && nw) store_labels(A.labNew, rowBase, nw, stage);
                    }
                    p ^= 1;
                }
                // next stage: smallest d(w) + 1 over residual boundary arcs of unvisited border vertices
                int cand = kInf;
                for (int i = tid; i < A.nring; i += kRowsNT) {
                    const int sv = slot[i];
                    if (sv < 0) continue;
                    const int l = sv & 0xffff;
                    const unsigned keep = (unsigned)sv >> 16;
                    const int row = l >> 5;
                    const unsigned bit = 1u << (l & 31);
                    if (Vb[row] & bit) continue;
                    for (int a = 0; a < 3; a++) {
                        if (!((keep >> (2 * a)) & 3u)) continue;
                        const int k = axis_dir(keep, a);
                        if (resM[k * R + row] & bit) cand = min(cand, halo[faceOff[k] + face_pos(k, l, TY)] + 1);
                    }
                }
                const int level = block_min(cand, red, rc);
                if (level == kInf) break;
                stages++;
                stage = level;
                for (int j = 0, i = tid; i < A.nring; j++, i += kRowsNT) {
                    const int sv = slot[i];
                    if (sv < 0) continue;
                    const int l = sv & 0xffff;
                    const unsigned keep = (unsigned)sv >> 16;
                    const int row = l >> 5;
                    const unsigned bit = 1u << (l & 31);
                    if (Vb[row] & bit) continue;
                    unsigned match = 0u;
                    for (int a = 0; a < 3; a++) {
                        if (!((keep >> (2 * a)) & 3u)) continue;
                        const int k = axis_dir(keep, a);
                        if ((resM[k * R + row] & bit) && halo[faceOff[k] + face_pos(k, l, TY)] + 1 == level)
                            match |= 1u << a;
                    }
                    if (match) {
                        admB |= (u64)match << (3 * j);
                        atomicOr(&Fb[p * R + row], bit);  // this buffer is all zero: the flood just ended on it
                    }
                }
                __syncthreads();
                if (myrow) {
                    F = Fb[p * R + tid] & ~vis;
                    vis |= F;
                    if (writeMode && F) store_labels(A.labNew, rowBase, F, level);
                }
            }
            // any excess vertex that reaches a target?
            const int found = block_any(myrow && (exM & vis) != 0u, red, rc);
            if (writeMode) {
                if (myrow) store_labels(A.labNew, rowBase, ~vis, dinf);
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

            // ---------------- push along admissible arcs until nothing moves ----------------
            const unsigned canPush = admT | adm[0] | adm[1] | adm[2] | adm[3] | adm[4] | adm[5];
            int q = 0;
            for (;;) {
                int pushed = 0;
                if (myrow) {
                    unsigned P = exM & canPush;
                    while (P) {
                        const int x = __ffs(P) - 1;
                        const unsigned bit = 1u << x;
                        P &= P - 1;
                        const int u = tid * 32 + x;
                        const size_t gu = base + u;
                        int c[6];
#pragma unroll
                        for (int k = 0; k < 6; k++) c[k] = (adm[k] & bit) ? A.res[(size_t)k * N + gu] : 0;
                        const int cT = (admT & bit) ? A.rt[gu] : 0;
                        const int e = A.ex[gu];
                        if (e <= 0) {
                            // a later receipt in this iteration sets the bit again
                            exM &= ~bit;
                            continue;
                        }
                        int rem = e;
                        if (admT & bit) {
                            const int d = min(rem, cT);
                            if (d > 0) {
                                A.rt[gu] = cT - d;
                                rem -= d;
                                if (A.trace) atomicAdd((unsigned long long *)&s_tr[1], (u64)d);
                            }
                            if (cT == d) {
                                admT &= ~bit;
                                rtM &= ~bit;
                            }
                        }
#pragma unroll
                        for (int k = 0; k < 6; k++) {
                            if (!(adm[k] & bit) || rem <= 0) continue;
                            const int d = min(rem, c[k]);
                            if (d > 0) {
                                A.res[(size_t)k * N + gu] = c[k] - d;
                                const int v = u + ((k & 1) ? -1 : 1) * (k < 2 ? 1 : (k < 4 ? 32 : 32 * TY));
                                const unsigned vbit = 1u << (v & 31);
                                atomicAdd(&A.res[(size_t)(k ^ 1) * N + base + v], d);
                                atomicAdd(&A.ex[base + v], d);
                                atomicOr(&resM[(k ^ 1) * R + (v >> 5)], vbit);
                                atomicOr(&recvB[q * R + (v >> 5)], vbit);
                                rem -= d;
                            }
                            if (c[k] == d) {
                                adm[k] &= ~bit;
                                atomicAnd(&resM[k * R + tid], ~bit);
                            }
                        }
                        if (rem < e) {
                            const int D = e - rem;
                            if (atomicAdd(&A.ex[gu], -D) == D) atomicOr(&clrB[q * R + tid], bit);
                            pushed = 1;
                        }
                    }
                }
                // first-level vertices of stages k > 0 push over boundary arcs
                if (admB) {
                    for (int j = 0; (admB >> (3 * j)) != 0ull; j++) {
                        const unsigned ab = (unsigned)(admB >> (3 * j)) & 7u;
                        if (!ab) continue;
                        const int sv = slot[tid + j * kRowsNT];
                        const int l = sv & 0xffff;
                        const unsigned keep = (unsigned)sv >> 16;
                        const size_t gu = base + l;
                        const int row = l >> 5;
                        const unsigned bit = 1u << (l & 31);
                        const int e = A.ex[gu];
                        if (e <= 0) {
                            atomicOr(&clrB[q * R + row], bit);
                            continue;
                        }
                        int rem = e;
                        for (int a = 0; a < 3; a++) {
                            if (!((ab >> a) & 1u) || rem <= 0) continue;
                            const int k = axis_dir(keep, a);
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
                                atomicAnd(&resM[k * R + row], ~bit);
                            }
                        }
                        if (rem < e) {
                            const int D = e - rem;
                            if (atomicAdd(&A.ex[gu], -D) == D) atomicOr(&clrB[q * R + row], bit);
                            pushed = 1;
                        }
                    }
                }
                const int any = block_any(pushed, red, rc);
                if (myrow) {
                    const unsigned rv = recvB[q * R + tid], cl = clrB[q * R + tid];
                    recvB[q * R + tid] = 0u;
                    clrB[q * R + tid] = 0u;
                    exM = (exM & ~cl) | rv;
                }
                q ^= 1;
                if (!any) break;
            }
        }
        __syncthreads();
        if (A.trace) {
            long long ex_out = 0, lsum = 0;
            for (int l = tid; l < V; l += kRowsNT) ex_out += A.ex[base + l];
            for (int i = tid; i < A.nring; i += kRowsNT) lsum += min(A.labNew[base + A.ringL[i]], 65535);
            atomicAdd((unsigned long long *)&s_tr[0], (u64)ex_out);
            atomicAdd((unsigned long long *)&s_tr[3], (u64)lsum);
        }
        __syncthreads();
        if (tid == 0) {
            atomicAdd(&A.stats[0], 1ull);
            atomicAdd(&A.stats[1], (u64)A.rvcount[r]);
            atomicAdd(&A.stats[2], (u64)(iter + 1));
            atomicAdd(&A.stats[3], (u64)levels);
            atomicAdd(&A.stats[4], (u64)stages);
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

void set_rows_attributes() {
    (void)hipFuncSetAttribute((const void *)k_discharge_rows, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
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
