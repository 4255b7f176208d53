// Learned region scheduler: per-region features, a small 3D CNN over the
// region grid (forward in BF16 with FP32 accumulation, FP32 training with its
// own backward and Adam kernels), and the queue builder that orders region
// discharges by score and defers regions the network predicts to do no useful
// work.  Exactness does not depend on the scores: a deferred region keeps its
// active flag, is forced after a bounded number of deferrals, and a solve
// only ends when no vertex is active.
#include "mf_device.h"
#include "mf_launch.h"

namespace mfd {

typedef unsigned long long u64;

// ---------------------------------------------------------------------------
// Features (one workgroup per region), FEAT floats per region:
//   0  log1p(total excess of active vertices) / 8
//   1  log1p(mean label of the region's border vertices with a finite label) / 8
//   2  fraction of outgoing boundary arcs with positive residual
//   3  1 if the region holds an active vertex
//   4  sum over border vertices of min(label, 65535) (same statistic the trace
//      records after a discharge, to detect label changes)
//   5  total excess of active vertices (raw)
// ---------------------------------------------------------------------------
__global__ void k_region_features(FeatArgs A) {
    __shared__ double s_acc[6][4];
    const Geo &G = A.G;
    const int r = blockIdx.x, tid = threadIdx.x, V = G.V, N = G.N;
    const int base = r * V;
    double ex_act = 0, lsum = 0, lcnt = 0, arcs = 0, open = 0, ring_clip = 0;
    int any = 0;
    int rz, ry, rx;
    region_xyz(G, r, rz, ry, rx);
    // after the first sweep only border vertices can be active: every region has
    // been discharged once, a discharge leaves no active vertex inside, and only
    // the fusion adds excess (at border vertices); labels never decrease
    if (!A.ringOnly) {
        for (int l = tid; l < V; l += blockDim.x) {
            const int e = A.ex[base + l];
            const int d = A.lab2 ? max(A.lab[base + l], A.lab2[base + l]) : A.lab[base + l];
            if (e > 0 && d < A.dinf) {
                ex_act += e;
                any = 1;
            }
        }
    }
    for (int i = tid; i < A.nring; i += blockDim.x) {
        const int l = A.ringL[i];
        const int d = A.lab[base + l];
        if (A.ringOnly) {
            const int e = A.ex[base + l];
            if (e > 0 && d < A.dinf) {
                ex_act += e;
                any = 1;
            }
        }
        ring_clip += d < 65535 ? d : 65535;
        if (d < A.dinf) {
            lsum += d;
            lcnt += 1;
        }
        const unsigned m = A.ringM[i];
        for (int k = 0; k < G.K; k++) {
            if (!((m >> k) & 1u)) continue;
            // the arc counts if it leads into a region of the grid
            const unsigned c = A.ringX[(size_t)i * G.K + k];
            const int nx = rx + ((c & 3u) == 1u) - ((c & 3u) == 2u);
            const int ny = ry + (((c >> 2) & 3u) == 1u) - (((c >> 2) & 3u) == 2u);
            const int nz = rz + (((c >> 4) & 3u) == 1u) - (((c >> 4) & 3u) == 2u);
            if ((unsigned)nx >= (unsigned)G.rx || (unsigned)ny >= (unsigned)G.ry || (unsigned)nz >= (unsigned)G.rz)
                continue;
            arcs += 1;
            open += A.res[(size_t)k * N + base + l] > 0 ? 1 : 0;
        }
    }
    double vals[6] = {ex_act, lsum, lcnt, arcs, open, ring_clip};
    for (int j = 0; j < 6; j++) {
        double v = vals[j];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((tid & 63) == 0) s_acc[j][tid >> 6] = v;
    }
    any = __any(any);
    __shared__ int s_any[4];
    if ((tid & 63) == 0) s_any[tid >> 6] = any;
    __syncthreads();
    if (tid == 0) {
        double t[6];
        for (int j = 0; j < 6; j++) t[j] = s_acc[j][0] + s_acc[j][1] + s_acc[j][2] + s_acc[j][3];
        const int act = s_any[0] | s_any[1] | s_any[2] | s_any[3];
        float *f = A.out + (size_t)r * kFeat;
        f[0] = (float)(log1p(t[0]) / 8.0);
        f[1] = (float)(t[2] > 0 ? log1p(t[1] / t[2]) / 8.0 : log1p((double)A.dinf) / 8.0);
        f[2] = (float)(t[3] > 0 ? t[4] / t[3] : 0.0);
        f[3] = act ? 1.f : 0.f;
        f[4] = (float)t[5];
        f[5] = (float)t[0];
    }
}

hipError_t launch_region_features(const FeatArgs &A, hipStream_t s) {
    hipLaunchKernelGGL(k_region_features, dim3(A.G.nreg), dim3(256), 0, s, A);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CNN over the region grid (D x H x W, channels last): three 3x3x3 convolutions
// with zero padding, 3 -> C -> C -> 1 channels, ReLU after the first two.
// Parameter layout (floats): w1[C][3][27], b1[C], w2[C][C][27], b2[C],
// w3[1][C][27], b3[1]; weight index (co, ci, tap) with tap = (dz+1)*9 + (dy+1)*3 + (dx+1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bf16_round(float x) {
    // round to nearest even at 8 mantissa bits (bfloat16), finite inputs
    unsigned u = __float_as_uint(x);
    const unsigned lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return __uint_as_float(u & 0xffff0000u);
}

// y[v][co] = b[co] + sum_ci sum_tap w[co][ci][tap] * x[v + tap][ci]; optional ReLU;
// bf16: weights and inputs rounded to bfloat16, products accumulated in fp32,
// the output rounded to bfloat16.  The block stages the (rounded) weights in
// LDS; inputs already rounded by the previous layer (roundIn == 0) are used as
// they are (rounding is idempotent).
__global__ void k_conv3_fwd(const float *x, int xs, int cin, const float *w, const float *b, int cout,
                            float *y, int D, int H, int W, int relu, int bf16, int roundIn) {
    extern __shared__ float wl[];  // [cout][cin][27]
    const int nw = cout * cin * 27;
    for (int i = threadIdx.x; i < nw; i += blockDim.x) wl[i] = bf16 ? bf16_round(w[i]) : w[i];
    __syncthreads();
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int nv = D * H * W;
    if (idx >= nv * cout) return;
    const bool rin = bf16 && roundIn;
    const int co = idx % cout, v = idx / cout;
    const int z = v / (H * W), t = v - z * H * W, yy = t / W, xx = t - yy * W;
    float acc = b[co];
    for (int dz = -1; dz <= 1; dz++) {
        const int zz = z + dz;
        if (zz < 0 || zz >= D) continue;
        for (int dy = -1; dy <= 1; dy++) {
            const int y2 = yy + dy;
            if (y2 < 0 || y2 >= H) continue;
            for (int dx = -1; dx <= 1; dx++) {
                const int x2 = xx + dx;
                if (x2 < 0 || x2 >= W) continue;
                const int tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                const float *xv = x + (size_t)((zz * H + y2) * W + x2) * xs;
                const float *wv = wl + co * cin * 27 + tap;
                for (int ci = 0; ci < cin; ci++) {
                    const float a = rin ? bf16_round(xv[ci]) : xv[ci];
                    acc += a * wv[ci * 27];
                }
            }
        }
    }
    if (relu) acc = fmaxf(acc, 0.f);
    if (bf16) acc = bf16_round(acc);
    y[idx] = acc;
}

// gradient w.r.t. the input: gx[v][ci] = sum_co sum_tap w[co][ci][tap] * gy[v - tap][co]
__global__ void k_conv3_bwd_x(const float *gy, int cout, const float *w, int cin, float *gx, int D,
                              int H, int W) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int nv = D * H * W;
    if (idx >= nv * cin) return;
    const int ci = idx % cin, v = idx / cin;
    const int z = v / (H * W), t = v - z * H * W, yy = t / W, xx = t - yy * W;
    float acc = 0.f;
    for (int dz = -1; dz <= 1; dz++) {
        const int zz = z - dz;
        if (zz < 0 || zz >= D) continue;
        for (int dy = -1; dy <= 1; dy++) {
            const int y2 = yy - dy;
            if (y2 < 0 || y2 >= H) continue;
            for (int dx = -1; dx <= 1; dx++) {
                const int x2 = xx - dx;
                if (x2 < 0 || x2 >= W) continue;
                const int tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1);
                const float *g = gy + (size_t)((zz * H + y2) * W + x2) * cout;
                for (int co = 0; co < cout; co++) acc += w[((size_t)co * cin + ci) * 27 + tap] * g[co];
            }
        }
    }
    gx[idx] = acc;
}

// gradient w.r.t. weights and bias: one thread per (co, ci, tap) (+ bias threads)
__global__ void k_conv3_bwd_w(const float *x, int xs, int cin, const float *gy, int cout, float *gw,
                              float *gb, int D, int H, int W) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = cout * cin * 27;
    const int nv = D * H * W;
    if (idx < nw) {
        const int tap = idx % 27, ci = (idx / 27) % cin, co = idx / (27 * cin);
        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
        float acc = 0.f;
        for (int v = 0; v < nv; v++) {
            const int z = v / (H * W), t = v - z * H * W, yy = t / W, xx = t - yy * W;
            const int zz = z + dz, y2 = yy + dy, x2 = xx + dx;
            if (zz < 0 || zz >= D || y2 < 0 || y2 >= H || x2 < 0 || x2 >= W) continue;
            acc += x[(size_t)((zz * H + y2) * W + x2) * xs + ci] * gy[(size_t)v * cout + co];
        }
        gw[idx] = acc;
    } else if (idx < nw + cout) {
        const int co = idx - nw;
        float acc = 0.f;
        for (int v = 0; v < nv; v++) acc += gy[(size_t)v * cout + co];
        gb[co] = acc;
    }
}

// ReLU backward in place: g *= (y > 0)
__global__ void k_relu_bwd(float *g, const float *y, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(y[i] > 0.f)) g[i] = 0.f;
}

// Binary cross-entropy with logits, averaged over masked voxels:
// loss = mean(max(z,0) - z*t + log(1 + exp(-|z|))); dz = (sigmoid(z) - t) * m / sum(m)
__global__ void k_bce(const float *z, const float *t, const float *m, int n, float *gz, float *loss) {
    __shared__ float s_l[4], s_m[4];
    float lsum = 0.f, msum = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) msum += m[i];
    for (int off = 32; off > 0; off >>= 1) msum += __shfl_xor(msum, off, 64);
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = msum;
    __syncthreads();
    const float mtot = s_m[0] + s_m[1] + s_m[2] + s_m[3];
    const float inv = mtot > 0.f ? 1.f / mtot : 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const float zi = z[i], ti = t[i], mi = m[i];
        lsum += mi * (fmaxf(zi, 0.f) - zi * ti + log1pf(expf(-fabsf(zi))));
        gz[i] = (1.f / (1.f + expf(-zi)) - ti) * mi * inv;
    }
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if ((threadIdx.x & 63) == 0) s_l[threadIdx.x >> 6] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) *loss = (s_l[0] + s_l[1] + s_l[2] + s_l[3]) * inv;
}

// Adam (bias-corrected), one thread per parameter
__global__ void k_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Queue of a learned sweep, one workgroup: an active region whose predicted
// probability of progress is below the threshold is deferred, unless it was
// deferred max_defer times in a row.  A counting sort over classes (largest
// first) then lists the regions to discharge by their previous discharge time
// (log2 buckets, longest first), then the deferred regions (skipped at once),
// then the inactive ones.  Order inside a class is arbitrary; the result of a
// sweep does not depend on the order.
constexpr int kQueueBuckets = 34;  // 0 inactive, 1 deferred, 2 + log2(ticks) active

__global__ void k_sched_queue(SchedArgs A) {
    extern __shared__ unsigned char smem[];
    __shared__ int hist[kQueueBuckets], off[kQueueBuckets];
    const int n = A.nreg;
    unsigned char *cls = smem;
    for (int i = threadIdx.x; i < kQueueBuckets; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const bool act = A.feat[(size_t)i * kFeat + 3] > 0.5f;
        const float prob = 1.f / (1.f + expf(-A.score[i]));
        int d = 0;
        if (act && prob < A.threshold && A.deferCount[i] < A.maxDefer) d = 1;
        A.defer[i] = d;
        A.deferCount[i] = d ? A.deferCount[i] + 1 : 0;
        int c = 0;
        if (act) {
            const unsigned lt = (unsigned)max(A.regionTicks[i], 0);
            c = d ? 1 : 2 + (lt ? 32 - __clz(lt) : 0);
        }
        cls[i] = (unsigned char)c;
        atomicAdd(&hist[c], 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int c = kQueueBuckets - 1; c >= 0; c--) {
            off[c] = acc;
            acc += hist[c];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) A.order[atomicAdd(&off[cls[i]], 1)] = i;
}

// Phase lists of the learned colour phases (Alg. 1), one workgroup: the
// colours in descending order of the predicted progress summed over their
// active regions (ties keep the colour order), and for phase q the regions of
// its colour followed by -1 up to the longest colour (a region kernel stops at
// the first -1).  Sums in a fixed order, so the phase order is reproducible.
__global__ void k_phase_lists(PhaseArgs A) {
    __shared__ float s_part[kMaxColours][16];
    __shared__ int s_perm[kMaxColours];
    const int tid = threadIdx.x, nw = blockDim.x >> 6;
    for (int c = 0; c < A.ncol; c++) {
        float acc = 0.f;
        for (int i = A.cstart[c] + tid; i < A.cstart[c + 1]; i += blockDim.x) {
            const int r = A.corder[i];
            if (A.ractive[r]) acc += 1.f / (1.f + expf(-A.score[r]));
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((tid & 63) == 0) s_part[c][tid >> 6] = acc;
    }
    __syncthreads();
    if (tid == 0) {
        float prog[kMaxColours];
        for (int c = 0; c < A.ncol; c++) {
            float t = 0.f;
            for (int w = 0; w < nw; w++) t += s_part[c][w];
            prog[c] = t;
            s_perm[c] = c;
        }
        // insertion sort, descending, stable
        for (int a = 1; a < A.ncol; a++) {
            const int c = s_perm[a];
            int b = a - 1;
            while (b >= 0 && prog[s_perm[b]] < prog[c]) {
                s_perm[b + 1] = s_perm[b];
                b--;
            }
            s_perm[b + 1] = c;
        }
    }
    __syncthreads();
    for (int q = 0; q < A.ncol; q++) {
        const int c = s_perm[q], lo = A.cstart[c], len = A.cstart[c + 1] - lo;
        for (int i = tid; i < A.maxC; i += blockDim.x) A.out[q * A.maxC + i] = i < len ? A.corder[lo + i] : -1;
    }
}

static inline int cdiv_s(long long a, int b) { return (int)((a + b - 1) / b); }

hipError_t launch_phase_lists(const PhaseArgs &A, hipStream_t s) {
    if (A.ncol < 1 || A.ncol > kMaxColours) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_phase_lists, dim3(1), dim3(1024), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_conv3_fwd(const float *x, int xs, int cin, const float *w, const float *b, int cout,
                            float *y, int D, int H, int W, int relu, int bf16, int roundIn, hipStream_t s) {
    const size_t lds = sizeof(float) * (size_t)cout * cin * 27;
    hipLaunchKernelGGL(k_conv3_fwd, dim3(cdiv_s((long long)D * H * W * cout, 256)), dim3(256), lds, s, x,
                       xs, cin, w, b, cout, y, D, H, W, relu, bf16, roundIn);
    return hipGetLastError();
}

hipError_t launch_conv3_bwd(const float *x, int xs, int cin, const float *w, const float *gy, int cout,
                            float *gx, float *gw, float *gb, int D, int H, int W, hipStream_t s) {
    if (gx)
        hipLaunchKernelGGL(k_conv3_bwd_x, dim3(cdiv_s((long long)D * H * W * cin, 256)), dim3(256), 0, s,
                           gy, cout, w, cin, gx, D, H, W);
    hipLaunchKernelGGL(k_conv3_bwd_w, dim3(cdiv_s((long long)cout * cin * 27 + cout, 256)), dim3(256), 0,
                       s, x, xs, cin, gy, cout, gw, gb, D, H, W);
    return hipGetLastError();
}

hipError_t launch_relu_bwd(float *g, const float *y, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_relu_bwd, dim3(cdiv_s(n, 256)), dim3(256), 0, s, g, y, n);
    return hipGetLastError();
}

hipError_t launch_bce(const float *z, const float *t, const float *m, int n, float *gz, float *loss,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_bce, dim3(1), dim3(256), 0, s, z, t, m, n, gz, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(cdiv_s(n, 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

void set_sched_attributes() {
    (void)hipFuncSetAttribute((const void *)k_sched_queue, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    (void)hipGetLastError();
}

hipError_t launch_sched_queue(const SchedArgs &A, hipStream_t s) {
    const size_t lds = (size_t)A.nreg;  // one class byte per region
    if (lds > 64 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sched_queue, dim3(1), dim3(1024), lds, s, A);
    return hipGetLastError();
}

}  // namespace mfd
