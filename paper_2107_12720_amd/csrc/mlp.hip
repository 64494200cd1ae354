// mlp.hip -- learned successor order for AC-6 (BF16 MFMA, FP32 accumulation).
//
// AC-6 checks successors in CSR order and keeps the first live one as the
// support (Section 6.1); a live vertex costs (index of its first live
// successor + 1) checks.  A small network scores every edge u -> w by how
// likely w is to stay live, and each adjacency list is then reordered by that
// score, so AC-6 tries likely supports first.  The order changes only the
// traversed edges, never the live set (every order reaches the same greatest
// fixed point).
//
// Network: 8 edge features -> 32 -> 32 -> 1, ReLU, BF16 weights, BF16 inputs
// and layer-1 activations as MFMA operands (the FP32 layer-2 activations feed
// the 32-term output dot product directly), FP32 accumulation, FP32 master
// weights, Adam.  The backward pass rounds dZ2 and dZ1 to BF16 where they
// enter an MFMA.
// Features of u -> w at position i of u's list:
//   log1p(outdeg u), log1p(indeg u), log1p(outdeg w), log1p(indeg w),
//   log1p(outdeg u) - log1p(outdeg w)  (= log of the degree ratio),
//   three +-1 bits of a hash of i.
// Loss: binary cross-entropy of "w is live" over edges whose source is live
// (only those edges decide a support).
//
// MFMA layout (v_mfma_f32_32x32x8 bf16, 64 lanes): A[i][k] sits in lane
// i%32 + 32*(k/4), item k%4; B[k][j] in lane j + 32*(k/4), item k%4; D[i][j]
// in lane j + 32*((i/4)%2), register 4*(i/8) + i%4.  A 32-edge tile is
// computed transposed (hidden units x edges), so layer 1's output registers
// 4j..4j+3 are exactly the B operand of layer 2's k-block j.
// Contractions over 32 (layer 2 and its backward pass, the weight gradients
// over a tile's edges) use gfx950's double-K form v_mfma_f32_32x32x16 bf16:
// 8 items per lane, A[i][k] in lane i%32 + 32*(k/8), item k%8, the same D.
// Where its operands are two 8-deep blocks side by side (cat), both operands
// see the same order of k, and a sum over k does not depend on that order.
#include "trim_device.h"
#include "trim_internal.h"

namespace trim {

namespace {

typedef __attribute__((__vector_size__(4 * sizeof(short)))) short bf16x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kW1 = 0, kB1 = 256, kW2 = 288, kB2 = 1312, kW3 = 1344, kB3 = 1376;

__device__ __forceinline__ short f2bf(float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ __forceinline__ float bf2f(short h) {
    return __uint_as_float(((uint32_t)(uint16_t)h) << 16);
}
__device__ __forceinline__ float rbf(float f) { return bf2f(f2bf(f)); }
// row of D register r held by lane l
__device__ __forceinline__ int drow(int r, int l) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }
__device__ __forceinline__ f32x16 mfma(bf16x4 a, bf16x4 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
}
typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __bf16 bf16v8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f32x16 mfma16(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16v8, a),
                                                   __builtin_bit_cast(bf16v8, b), c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 cat(bf16x4 lo, bf16x4 hi) {
    return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

struct Graph {
    const int* row_off;
    const int* col;
    const int* indeg;
    const int* src;
    long long m;
    // per-vertex (log1p(outdeg), log1p(indeg)) when precomputed, else NULL
    const float2* vf;
};

// (log1p(outdeg v), log1p(indeg v)) in FP32, the same expressions the edge
// features use.
__global__ void vertex_features(const int* row_off, const int* indeg, int n, float2* vf) {
    for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        vf[v] = make_float2(log1pf((float)(row_off[v + 1] - row_off[v])),
                            log1pf((float)indeg[v]));
}

// This lane's four features (half 0: features 0-3, half 1: 4-7) of edge e.
__device__ __forceinline__ void features(const Graph& g, long long e, int half, float f[4],
                                         int& u, int& w) {
    u = g.src[e];
    w = g.col[e];
    float lu, lw, iu, iw;
    if (g.vf) {   // one 8-byte gather per endpoint
        const float2 a = g.vf[u], b = g.vf[w];
        lu = a.x;
        iu = a.y;
        lw = b.x;
        iw = b.y;
    } else {
        lu = log1pf((float)(g.row_off[u + 1] - g.row_off[u]));
        lw = log1pf((float)(g.row_off[w + 1] - g.row_off[w]));
        iu = log1pf((float)g.indeg[u]);
        iw = log1pf((float)g.indeg[w]);
    }
    if (half == 0) {
        f[0] = lu;
        f[1] = iu;
        f[2] = lw;
        f[3] = iw;
    } else {
        const uint64_t h = mix64((uint64_t)(e - g.row_off[u]));
        f[0] = lu - lw;
        f[1] = (h & 1) ? 1.f : -1.f;
        f[2] = (h & 2) ? 1.f : -1.f;
        f[3] = (h & 4) ? 1.f : -1.f;
    }
}

// Weights staged per wave as MFMA operands.
struct Weights {
    bf16x4 w1;        // A of layer 1: W1[l%32][4(l/32)+t]
    bf16x4 w2[4];     // A of layer 2, k-block j: W2[l%32][8j+4(l/32)+t]
    bf16x4 w2t[4];    // A of dH1 = W2^T dZ2, k-block j: W2[8j+4(l/32)+t][l%32]
    float b1[16], b2[16], w3[16];   // per D register
    float b3;
};

__device__ __forceinline__ void load_weights(const short* p, Weights& W) {
    const int l = lane_id();
    for (int t = 0; t < 4; ++t) W.w1[t] = p[kW1 + (l & 31) * 8 + 4 * (l >> 5) + t];
    for (int j = 0; j < 4; ++j)
        for (int t = 0; t < 4; ++t) {
            const int k = 8 * j + 4 * (l >> 5) + t;
            W.w2[j][t] = p[kW2 + (l & 31) * 32 + k];
            W.w2t[j][t] = p[kW2 + k * 32 + (l & 31)];
        }
    for (int r = 0; r < 16; ++r) {
        const int h = drow(r, l);
        W.b1[r] = bf2f(p[kB1 + h]);
        W.b2[r] = bf2f(p[kB2 + h]);
        W.w3[r] = bf2f(p[kW3 + h]);
    }
    W.b3 = bf2f(p[kB3]);
}

// Forward pass of a 32-edge tile (edge = l%32).  Returns the logit of this
// lane's edge; z1/z2 hold pre-activations, h1 the BF16 layer-1 activations.
__device__ __forceinline__ float forward(const Weights& W, const float f[4], f32x16& z1,
                                         f32x16& z2, bf16x4 h1[4], float h2[16]) {
    bf16x4 x;
    for (int t = 0; t < 4; ++t) x[t] = f2bf(f[t]);
    const f32x16 zero = {};
    z1 = mfma(W.w1, x, zero);
    for (int r = 0; r < 16; ++r) {
        z1[r] += W.b1[r];
        h1[r >> 2][r & 3] = f2bf(fmaxf(z1[r], 0.f));
    }
    z2 = mfma16(cat(W.w2[0], W.w2[1]), cat(h1[0], h1[1]), zero);
    z2 = mfma16(cat(W.w2[2], W.w2[3]), cat(h1[2], h1[3]), z2);
    float s = 0.f;
    for (int r = 0; r < 16; ++r) {
        z2[r] += W.b2[r];
        h2[r] = fmaxf(z2[r], 0.f);
        s += W.w3[r] * h2[r];
    }
    s += __shfl_xor(s, 32);   // the other half of the hidden units
    return s + W.b3;
}

__device__ __forceinline__ bool bit(const uint32_t* bm, int v) { return (bm[v >> 5] >> (v & 31)) & 1u; }

__device__ __forceinline__ long long sample_edge(const long long* ids, uint64_t seed, int step,
                                                 long long idx, long long m) {
    if (ids) return ids[idx];
    return (long long)(mix64(seed ^ ((uint64_t)step << 40) ^ (uint64_t)idx) % (uint64_t)m);
}

// Per-wave LDS tiles for the weight gradients (32 hidden x 32 edges, padded).
struct Tiles {
    float a[32][33];
    float b[32][33];
    float x[32][8];
};

// Gradients of the mean loss over `count` sampled edges, accumulated into
// grad[0..1376]; grad[1377] accumulates the loss.  Edges are ids[k] when ids
// is given, else hashed samples.  Loss weight 1/count per edge, 0 when the
// source is not live.
__global__ __launch_bounds__(256) void mlp_grad(Graph g, const uint32_t* live, const short* p,
                                                const long long* ids, long long count,
                                                uint64_t seed, int step, float* grad) {
    __shared__ Tiles tiles[4];
    Tiles& T = tiles[threadIdx.x / kWave];
    const int l = lane_id(), half = l >> 5, col = l & 31;
    Weights W;
    load_weights(p, W);
    const f32x16 zero = {};
    f32x16 gw2 = zero, gw1 = zero;
    float gb1[16] = {}, gb2[16] = {}, gw3[16] = {};
    float gb3 = 0.f, loss = 0.f;
    const float inv = 1.f / (float)count;
    const long long tiles_total = (count + 31) / 32;
    const long long wave = (blockIdx.x * (long long)blockDim.x + threadIdx.x) / kWave;
    const long long nwaves = (gridDim.x * (long long)blockDim.x) / kWave;
    for (long long t = wave; t < tiles_total; t += nwaves) {
        const long long k = t * 32 + col;
        float f[4] = {0.f, 0.f, 0.f, 0.f};
        float wgt = 0.f, y = 0.f;
        if (k < count) {
            const long long e = sample_edge(ids, seed, step, k, g.m);
            int u, w;
            features(g, e, half, f, u, w);
            wgt = bit(live, u) ? inv : 0.f;
            y = bit(live, w) ? 1.f : 0.f;
        }
        f32x16 z1, z2;
        bf16x4 h1[4];
        float h2[16];
        const float s = forward(W, f, z1, z2, h1, h2);
        // d(loss)/d(logit) for binary cross-entropy
        const float pr = 1.f / (1.f + expf(-s));
        const float gs = wgt * (pr - y);
        if (half == 0 && wgt != 0.f)
            loss += wgt * (fmaxf(s, 0.f) - s * y + log1pf(expf(-fabsf(s))));
        if (half == 0) gb3 += gs;
        float dz2[16];
        bf16x4 dz2b[4];
        for (int r = 0; r < 16; ++r) {
            gw3[r] += gs * h2[r];
            dz2[r] = z2[r] > 0.f ? gs * W.w3[r] : 0.f;
            gb2[r] += dz2[r];
            dz2b[r >> 2][r & 3] = f2bf(dz2[r]);
        }
        // dH1 = W2^T dZ2 (dZ2 registers 4j..4j+3 are the B operand of k-block j)
        f32x16 dh1 = mfma16(cat(W.w2t[0], W.w2t[1]), cat(dz2b[0], dz2b[1]), zero);
        dh1 = mfma16(cat(W.w2t[2], W.w2t[3]), cat(dz2b[2], dz2b[3]), dh1);
        // stage dZ2, H1 and X for the weight gradients (contraction over edges)
        for (int r = 0; r < 16; ++r) {
            T.a[drow(r, l)][col] = bf2f(dz2b[r >> 2][r & 3]);
            T.b[drow(r, l)][col] = bf2f(h1[r >> 2][r & 3]);
        }
        for (int t4 = 0; t4 < 4; ++t4) T.x[col][4 * half + t4] = rbf(f[t4]);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int j = 0; j < 2; ++j) {
            bf16x8 a, b;
            for (int t8 = 0; t8 < 8; ++t8) {
                const int e = 16 * j + 8 * half + t8;
                a[t8] = f2bf(T.a[col][e]);
                b[t8] = f2bf(T.b[col][e]);
            }
            gw2 = mfma16(a, b, gw2);   // dW2[h_out][h_in] += sum_e dZ2[h_out][e] H1[h_in][e]
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // dZ1 = dH1 * relu'(Z1)
        for (int r = 0; r < 16; ++r) {
            const float dz1 = z1[r] > 0.f ? dh1[r] : 0.f;
            gb1[r] += dz1;
            T.a[drow(r, l)][col] = rbf(dz1);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int j = 0; j < 2; ++j) {
            bf16x8 a, b;
            for (int t8 = 0; t8 < 8; ++t8) {
                const int e = 16 * j + 8 * half + t8;
                a[t8] = f2bf(T.a[col][e]);
                b[t8] = col < 8 ? f2bf(T.x[e][col]) : (short)0;
            }
            gw1 = mfma16(a, b, gw1);   // dW1[h][f] += sum_e dZ1[h][e] X[e][f]
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    // reduce over the 32 edges of each half, then one atomic per parameter
    for (int r = 0; r < 16; ++r) {
        float a = gb1[r], b = gb2[r], c = gw3[r];
        for (int off = 16; off > 0; off >>= 1) {
            a += __shfl_xor(a, off);
            b += __shfl_xor(b, off);
            c += __shfl_xor(c, off);
        }
        if (col == 0) {
            atomicAdd(grad + kB1 + drow(r, l), a);
            atomicAdd(grad + kB2 + drow(r, l), b);
            atomicAdd(grad + kW3 + drow(r, l), c);
        }
        atomicAdd(grad + kW2 + drow(r, l) * 32 + col, gw2[r]);
        if (col < 8) atomicAdd(grad + kW1 + drow(r, l) * 8 + col, gw1[r]);
    }
    for (int off = 16; off > 0; off >>= 1) {
        gb3 += __shfl_xor(gb3, off);
        loss += __shfl_xor(loss, off);
    }
    if (l == 0) {
        atomicAdd(grad + kB3, gb3);
        atomicAdd(grad + 1377, loss);
    }
}

// Adam on the FP32 master weights; writes the BF16 copy and clears the
// gradients.  c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ void mlp_adam(float* p32, short* pbf, float* m1, float* m2, float* grad, float lr,
                         float beta1, float beta2, float eps, float c1, float c2) {
    for (int i = threadIdx.x; i < 1377; i += blockDim.x) {
        const float gi = grad[i];
        const float a = beta1 * m1[i] + (1.f - beta1) * gi;
        const float b = beta2 * m2[i] + (1.f - beta2) * gi * gi;
        m1[i] = a;
        m2[i] = b;
        const float w = p32[i] - lr * (a * c1) / (sqrtf(b * c2) + eps);
        p32[i] = w;
        pbf[i] = f2bf(w);
        grad[i] = 0.f;
    }
    if (threadIdx.x == 0) grad[1377] = 0.f;
}

// The network's logit that the target of every edge stays live, in CSR
// order.  The logit, not the probability, is what the lists are ordered by:
// the logistic function saturates to exactly 1 in FP32 for logits above about
// 17, which would tie most live targets.
__global__ __launch_bounds__(256) void mlp_score(Graph g, const short* p, float* score) {
    const int l = lane_id(), half = l >> 5, col = l & 31;
    Weights W;
    load_weights(p, W);
    const long long tiles_total = (g.m + 31) / 32;
    const long long wave = (blockIdx.x * (long long)blockDim.x + threadIdx.x) / kWave;
    const long long nwaves = (gridDim.x * (long long)blockDim.x) / kWave;
    for (long long t = wave; t < tiles_total; t += nwaves) {
        const long long e = t * 32 + col;
        float f[4] = {0.f, 0.f, 0.f, 0.f};
        if (e < g.m) {
            int u, w;
            features(g, e, half, f, u, w);
        }
        f32x16 z1, z2;
        bf16x4 h1[4];
        float h2[16];
        const float s = forward(W, f, z1, z2, h1, h2);
        if (half == 0 && e < g.m) score[e] = s;
    }
}

inline int grid_for(long long n, int block, int max_blocks) {
    long long b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > max_blocks) b = max_blocks;
    return (int)b;
}

}  // namespace

hipError_t mlp_grad_launch(const int* row_off, const int* col, const int* indeg, const int* src,
                           long long m, const uint32_t* live, const short* pbf,
                           const long long* ids, long long count, uint64_t seed, int step,
                           float* grad, int cus, hipStream_t s) {
    Graph g{row_off, col, indeg, src, m, nullptr};
    const int blocks = grid_for((count + 31) / 32, 4, cus * 8);
    hipLaunchKernelGGL(mlp_grad, dim3(blocks), dim3(256), 0, s, g, live, pbf, ids, count, seed,
                       step, grad);
    return hipGetLastError();
}

hipError_t mlp_adam_launch(float* p32, short* pbf, float* m1, float* m2, float* grad, float lr,
                           float beta1, float beta2, float eps, int step, hipStream_t s) {
    // the bias corrections in double: 1 - beta2^t cancels badly in FP32
    // (beta2 = 0.999 loses about 15 bits at t = 2)
    const float c1 = (float)(1.0 / (1.0 - pow((double)beta1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - pow((double)beta2, (double)step)));
    hipLaunchKernelGGL(mlp_adam, dim3(1), dim3(256), 0, s, p32, pbf, m1, m2, grad, lr, beta1,
                       beta2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_score_launch(const int* row_off, const int* col, const int* indeg, const int* src,
                            int n, long long m, const short* pbf, float* score, float2* vf,
                            int cus, hipStream_t s) {
    Graph g{row_off, col, indeg, src, m, vf};
    if (m > 0) {
        hipLaunchKernelGGL(vertex_features, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s,
                           row_off, indeg, n, vf);
        hipLaunchKernelGGL(mlp_score, dim3(grid_for((m + 31) / 32, 4, cus * 16)), dim3(256), 0, s,
                           g, pbf, score);
    }
    return hipGetLastError();
}

}  // namespace trim
