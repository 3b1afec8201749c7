// kd_mlp.hip -- the radius-prediction MLP (3 -> 64 -> 64 -> 1, ReLU):
// bfloat16 operands, float32 accumulation.  The 64x64 contractions run on
// the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16); the 3-wide input layer
// and the 64-wide output dot product run on the vector ALU.
//
// Model (per query q, with the tree's bounding box lo/extent):
//   x  = bf16(fl((q - lo) * inv))       inv = fl(1 / extent), 0 on a flat axis
//   a1 = W1b x + b1,  h1 = bf16(relu(a1))
//   a2 = W2b h1 + b2, h2 = bf16(relu(a2))
//   y  = w3b . h2 + b3                  y predicts ln(k-th neighbour distance)
// W1b, W2b, w3b are bfloat16 roundings (nearest-even) of the float32 master
// weights; biases stay float32.  Parameters are one float32 vector:
//   W1[64][3] | b1[64] | W2[64][64] | b2[64] | w3[64] | b3    (4481 floats)
//
// Training: loss = mean (y - t)^2 with t = 0.5 ln(max(d2_k, 1e-14)) from the
// plain traversal; gradients straight through the bfloat16 casts, with the
// output-layer-2 gradient rounded to bfloat16 before both matrix-core
// products (dW2 = da2b^T h1, dh1 = da2b W2b).  Each wave reduces its 64
// samples into one partial gradient vector; a second kernel sums the wave
// partials in a fixed order (deterministic) and applies Adam.
//
// Matrix-core layout (16x16x32 bf16, wave64): for C[m][n] = sum_k A[m][k] B[k][n]
// lane l supplies A[m0 + l%16][k0 + 8*(l/16) + e] and B[k0 + 8*(l/16) + e][n0 + l%16]
// (e = 0..7) and receives C[m0 + 4*(l/16) + r][n0 + l%16] (r = 0..3).  Both
// operands are staged in LDS K-contiguous (A as [m][k], B as B^T [n][k]), so
// every fragment is one 16-byte LDS read.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kd_internal.h"

namespace kd {

namespace {

constexpr int HID = 64;
constexpr int OFF_W1 = 0, OFF_B1 = 192, OFF_W2 = 256, OFF_B2 = 4352, OFF_W3 = 4416, OFF_B3 = 4480;
constexpr int NPARAM = 4481;

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// bfloat16 rounding (nearest, ties to even) of a finite float, as raw bits
__device__ __forceinline__ uint16_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf16_round(float f) { return __uint_as_float(uint32_t(bf16_bits(f)) << 16); }

// LDS buffers one wave works in (64 samples).  W2b / W2b^T may be shared by
// several waves of a workgroup; the rest is private to the wave.
struct MlpBufs {
    uint16_t* w2;     // W2b [o][i]
    uint16_t* w2t;    // W2b^T [i][o]       (training only)
    uint16_t* h1;     // [q][i]
    uint16_t* h1t;    // [i][q]             (training only)
    uint16_t* h2;     // [q][o]  bfloat16 h2; reused for da2 [q][o] in training
    uint16_t* da2t;   // [o][q]             (training only)
    float (*red)[HID][4];
    float (*x)[3];
    float* dy;
    uint64_t* a1pos;  // bit i: a1[q][i] > 0
};

struct TrainSmem {
    uint16_t w2[HID * HID], w2t[HID * HID], h1[HID * HID], h1t[HID * HID], h2[HID * HID], da2t[HID * HID];
    float red[4][HID][4];
    float x[HID][3];
    float dy[HID];
    uint64_t a1pos[HID];
};

// Orders this wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ bf16x8 frag(const uint16_t* base, int row, int col0) {
    return *reinterpret_cast<const bf16x8*>(base + row * HID + col0);
}

// acc[mi][ni] = C tile (16x16) of C[m][n] = sum_k A[m][k] * BT[n][k], 64x64x64
__device__ __forceinline__ void gemm64_nt(const uint16_t* A, const uint16_t* BT, f32x4 (&acc)[4][4], int lane) {
    const int r16 = lane & 15, kg = (lane >> 4) * 8;
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
        bf16x8 a[4], b[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            a[t] = frag(A, t * 16 + r16, kk * 32 + kg);
            b[t] = frag(BT, t * 16 + r16, kk * 32 + kg);
        }
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int ni = 0; ni < 4; ++ni)
                acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mi], b[ni], acc[mi][ni], 0, 0, 0);
    }
}

struct Norm {
    float lo[3];
    float inv[3];
};

// W2b (and optionally its transpose) into LDS, cooperatively by nthreads.
__device__ __forceinline__ void stage_w2(const float* __restrict__ P, uint16_t* w2, uint16_t* w2t, int tid,
                                         int nthreads) {
    for (int e = tid; e < HID * HID; e += nthreads) {
        const uint16_t b = bf16_bits(P[OFF_W2 + e]);
        w2[e] = b;
        if (w2t) w2t[(e % HID) * HID + e / HID] = b;
    }
}

// Forward pass for the wave's 64 samples (lane = sample); W2b must already be
// staged.  Leaves h1 in B.h1 (and B.h1t, B.x when training), a1 signs in
// B.a1pos, the layer-2 pre-activations in acc (matrix-core layout), bfloat16
// h2 in B.h2, and returns y for the lane.
__device__ __forceinline__ float mlp_forward(const float* __restrict__ P, const Norm& nm, const float (&q)[3],
                                             const MlpBufs& B, f32x4 (&acc)[4][4], bool train, int lane) {
    float x[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const float t = q[j] - nm.lo[j];
        x[j] = bf16_round(t * nm.inv[j]);
        if (train) B.x[lane][j] = x[j];
    }
    uint64_t pos = 0;
#pragma unroll 8
    for (int i = 0; i < HID; ++i) {
        float a = P[OFF_B1 + i];
        a += bf16_round(P[OFF_W1 + 3 * i + 0]) * x[0];
        a += bf16_round(P[OFF_W1 + 3 * i + 1]) * x[1];
        a += bf16_round(P[OFF_W1 + 3 * i + 2]) * x[2];
        pos |= uint64_t(a > 0.0f) << i;
        const uint16_t h = bf16_bits(a > 0.0f ? a : 0.0f);
        B.h1[lane * HID + i] = h;
        if (train) B.h1t[i * HID + lane] = h;
    }
    B.a1pos[lane] = pos;
    wave_sync();
    gemm64_nt(B.h1, B.w2, acc, lane);  // C[q][o] = sum_i h1[q][i] W2b[o][i]
    const int r16 = lane & 15, rg = (lane >> 4) * 4;
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
            const int o = ni * 16 + r16;
            const float b2 = P[OFF_B2 + o];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float a2 = acc[mi][ni][r] + b2;
                acc[mi][ni][r] = a2;
                B.h2[(mi * 16 + rg + r) * HID + o] = bf16_bits(a2 > 0.0f ? a2 : 0.0f);
            }
        }
    wave_sync();
    float y = P[OFF_B3];
#pragma unroll 8
    for (int o = 0; o < HID; ++o)
        y += bf16_round(P[OFF_W3 + o]) * __uint_as_float(uint32_t(B.h2[lane * HID + o]) << 16);
    wave_sync();
    return y;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// ---------------------------------------------------------------- kernels

// ------------------------------------------------------------ inference
//
// Register-resident forward for 64 queries per wave and tile, no LDS.  Both
// layers run transposed on the matrix cores, queries along N:
//   GEMM1  a1^T[i][q] = W1b[i][x] . X^T[x][q] + b1[i]    (K = 3, zero-padded to 32)
//   GEMM2  a2^T[o][q] = W2b[o][i] . h1^T[i][q] + b2[o]   (K = 64, two 32-slices)
// with the biases preloaded as the accumulators.  GEMM1's output layout
// (lane l holds rows i = 16 mi + 4 (l/16) + r, r = 0..3, of column q) is fed
// to GEMM2 directly as its B operand by ordering GEMM2's contraction index:
// slice kk, element e of lane l's fragment is hidden unit
//   i = 16 (2 kk + e/4) + 4 (l/16) + e%4,
// and W2b's fragments use the same order (a contraction does not depend on
// the order of its index).  Layer 3 is a per-lane bfloat16 dot product over
// the 16 outputs a lane holds plus two cross-lane sums.  Weights are read
// into registers once per wave.
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(2))) short s16x2;

__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
    const bf16x2 v = {static_cast<__bf16>(lo), static_cast<__bf16>(hi)};  // round to nearest even
    return __builtin_bit_cast(uint32_t, v);
}
// bf16(relu(.)) of a pair: rounding keeps the sign, so relu is applied to the
// rounded values as a packed 16-bit integer max with 0 (negative bfloat16
// patterns, -0 included, are negative int16)
__device__ __forceinline__ uint32_t pack_bf16_relu(float lo, float hi) {
    const s16x2 v = __builtin_bit_cast(s16x2, pack_bf16(lo, hi));
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(v, s16x2{0, 0}));
}

struct InferWeights {
    bf16x8 a1[4];      // W1b fragments (lanes 0..15: i = 16 mi + l, x = e < 3; else 0)
    bf16x8 a2[4][2];   // W2b fragments [mo][kk]
    f32x4 b1[4];       // b1[16 mi + 4 (l/16) + r]
    f32x4 b2[4];       // b2[16 mo + 4 (l/16) + r]
    uint32_t w3[4][2]; // w3b pairs for o = 16 mo + 4 (l/16) + {0,1}, {2,3}
    float b3;
};

__device__ __forceinline__ void load_weights(const float* __restrict__ P, int lane, InferWeights& W) {
    const int c = lane & 15, g = lane >> 4;
#pragma unroll
    for (int mi = 0; mi < 4; ++mi) {
        const int i = 16 * mi + c;
        uint32_t u[4] = {0u, 0u, 0u, 0u};
        if (g == 0) {
            u[0] = pack_bf16(P[OFF_W1 + 3 * i + 0], P[OFF_W1 + 3 * i + 1]);
            u[1] = pack_bf16(P[OFF_W1 + 3 * i + 2], 0.0f);
        }
        W.a1[mi] = __builtin_bit_cast(bf16x8, make_uint4(u[0], u[1], u[2], u[3]));
        const float4 bb1 = *reinterpret_cast<const float4*>(P + OFF_B1 + 16 * mi + 4 * g);
        W.b1[mi] = f32x4{bb1.x, bb1.y, bb1.z, bb1.w};
    }
#pragma unroll
    for (int mo = 0; mo < 4; ++mo) {
        const int o = 16 * mo + c;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            // e = 0..3: i = 16 (2 kk) + 4 g + e;  e = 4..7: i = 16 (2 kk + 1) + 4 g + e - 4
            const float* r = P + OFF_W2 + o * HID + 4 * g;
            const float4 lo = *reinterpret_cast<const float4*>(r + 16 * (2 * kk));
            const float4 hi = *reinterpret_cast<const float4*>(r + 16 * (2 * kk + 1));
            W.a2[mo][kk] = __builtin_bit_cast(
                bf16x8, make_uint4(pack_bf16(lo.x, lo.y), pack_bf16(lo.z, lo.w), pack_bf16(hi.x, hi.y),
                                   pack_bf16(hi.z, hi.w)));
        }
        const float4 bb2 = *reinterpret_cast<const float4*>(P + OFF_B2 + 16 * mo + 4 * g);
        W.b2[mo] = f32x4{bb2.x, bb2.y, bb2.z, bb2.w};
        const float4 ww3 = *reinterpret_cast<const float4*>(P + OFF_W3 + 16 * mo + 4 * g);
        W.w3[mo][0] = pack_bf16(ww3.x, ww3.y);
        W.w3[mo][1] = pack_bf16(ww3.z, ww3.w);
    }
    W.b3 = P[OFF_B3];
}

// y for the 64 queries of a tile; lanes 0..15 pass the normalised inputs
// xs[nq] of queries 16 nq + lane (other lanes' xs are ignored).  Returns y of
// query `lane`.
__device__ __forceinline__ float mlp_tile(const InferWeights& W, const float (&xs)[4][3], int lane) {
    const int g = lane >> 4;
    float y_mine = 0.0f;
#pragma unroll
    for (int nq = 0; nq < 4; ++nq) {
        uint32_t u[4] = {0u, 0u, 0u, 0u};
        if (g == 0) {
            u[0] = pack_bf16(xs[nq][0], xs[nq][1]);
            u[1] = pack_bf16(xs[nq][2], 0.0f);
        }
        const bf16x8 bx = __builtin_bit_cast(bf16x8, make_uint4(u[0], u[1], u[2], u[3]));
        // layer 1: a1^T rows 16 mi + 4 g + r of column q = 16 nq + (lane % 16)
        f32x4 a1[4];
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) a1[mi] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.a1[mi], bx, W.b1[mi], 0, 0, 0);
        // h1 = bf16(relu(a1)) as GEMM2's B fragments
        bf16x8 h1[2];
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            const f32x4 p = a1[2 * kk], q = a1[2 * kk + 1];
            h1[kk] = __builtin_bit_cast(bf16x8, make_uint4(pack_bf16_relu(p[0], p[1]), pack_bf16_relu(p[2], p[3]),
                                                           pack_bf16_relu(q[0], q[1]), pack_bf16_relu(q[2], q[3])));
        }
        // layer 2 and the lane's part of layer 3
        float part = 0.0f;
#pragma unroll
        for (int mo = 0; mo < 4; ++mo) {
            f32x4 a2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.a2[mo][0], h1[0], W.b2[mo], 0, 0, 0);
            a2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(W.a2[mo][1], h1[1], a2, 0, 0, 0);
            const uint32_t h01 = pack_bf16_relu(a2[0], a2[1]);
            const uint32_t h23 = pack_bf16_relu(a2[2], a2[3]);
            part = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, h01), __builtin_bit_cast(bf16x2, W.w3[mo][0]),
                                                   part, false);
            part = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, h23), __builtin_bit_cast(bf16x2, W.w3[mo][1]),
                                                   part, false);
        }
        // sum over the four lane groups holding column q
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (g == nq) y_mine = part + W.b3;
    }
    return y_mine;
}

template <bool RECORDS>
__device__ __forceinline__ void load_tile_x(const void* __restrict__ src, uint32_t n, uint32_t tile, int lane,
                                            const Norm& nm, float (&xs)[4][3]) {
#pragma unroll
    for (int nq = 0; nq < 4; ++nq) {
        xs[nq][0] = xs[nq][1] = xs[nq][2] = 0.0f;
        const uint32_t i = tile * 64u + 16u * nq + uint32_t(lane);
        if (lane < 16 && i < n) {
            float q[3];
            if (RECORDS) {
                const float4 v = static_cast<const float4*>(src)[i];
                q[0] = v.x;
                q[1] = v.y;
                q[2] = v.z;
            } else {
                const float* p = static_cast<const float*>(src) + size_t(i) * 3;
                q[0] = p[0];
                q[1] = p[1];
                q[2] = p[2];
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) xs[nq][j] = (q[j] - nm.lo[j]) * nm.inv[j];
        }
    }
}

// Inference: worst0[slot] = min(R2, fl(r0 * r0)), r0 = exp(y + margin);
// a non-finite or negative r0 leaves R2.  Queries are the traversal-order
// records (16 bytes: x, y, z, row).  Persistent over 64-query tiles.
__global__ __launch_bounds__(256) void mlp_worst0(const float* __restrict__ P, Norm nm, float margin, float R2,
                                                  const float4* __restrict__ sq, uint32_t Q,
                                                  float* __restrict__ worst0) {
    const int lane = threadIdx.x & 63;
    InferWeights W;
    load_weights(P, lane, W);
    const uint32_t ntiles = (Q + 63) / 64;
    const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
    for (uint32_t tile = wave; tile < ntiles; tile += nwaves) {
        float xs[4][3];
        load_tile_x<true>(sq, Q, tile, lane, nm, xs);
        const float y = mlp_tile(W, xs, lane);
        const uint32_t slot = tile * 64u + uint32_t(lane);
        if (slot < Q) {
            const float r0 = expf(y + margin);
            float wv = R2;
            if (__builtin_isfinite(r0) && r0 >= 0.0f) {
                const float r2 = r0 * r0;
                wv = r2 < R2 ? r2 : R2;
            }
            worst0[slot] = wv;
        }
    }
}

// Inference for batched class records (32 bytes: x, y, z, w, row, job, pad),
// one table entry per 3-D job with a model: tile t of the table (ascending
// tile_base) covers that job's records slot_base + 64 (t - tile_base) ...;
// the wave loads the job's weights when its model differs from the last.
__global__ __launch_bounds__(256) void mlp_worst0_jobs(const MlpJob* __restrict__ jobs, int njobs, uint32_t ntiles,
                                                       const float4* __restrict__ recs, float* __restrict__ worst0) {
    const int lane = threadIdx.x & 63;
    InferWeights W;
    const float* loaded = nullptr;
    const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
    for (uint32_t tile = wave; tile < ntiles; tile += nwaves) {
        int lo = 0, hi = njobs - 1;  // last job with tile_base <= tile
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile_base <= tile) lo = mid;
            else hi = mid - 1;
        }
        const MlpJob& J = jobs[lo];
        if (J.P != loaded) {
            load_weights(J.P, lane, W);
            loaded = J.P;
        }
        Norm nm;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            nm.lo[j] = J.lo[j];
            nm.inv[j] = J.inv[j];
        }
        const uint32_t first = J.slot_base + (tile - J.tile_base) * 64u;
        const uint32_t end = J.slot_base + J.Q;
        float xs[4][3];
#pragma unroll
        for (int nq = 0; nq < 4; ++nq) {
            xs[nq][0] = xs[nq][1] = xs[nq][2] = 0.0f;
            const uint32_t i = first + 16u * nq + uint32_t(lane);
            if (lane < 16 && i < end) {
                const float4 v = recs[2 * size_t(i)];
                xs[nq][0] = (v.x - nm.lo[0]) * nm.inv[0];
                xs[nq][1] = (v.y - nm.lo[1]) * nm.inv[1];
                xs[nq][2] = (v.z - nm.lo[2]) * nm.inv[2];
            }
        }
        const float y = mlp_tile(W, xs, lane);
        const uint32_t slot = first + uint32_t(lane);
        if (slot < end) {
            const float r0 = expf(y + J.margin);
            float wv = J.R2;
            if (__builtin_isfinite(r0) && r0 >= 0.0f) {
                const float r2 = r0 * r0;
                wv = r2 < J.R2 ? r2 : J.R2;
            }
            worst0[slot] = wv;
        }
    }
}

// Raw forward for tests: y[i] for caller-layout queries [n][3].
__global__ __launch_bounds__(256) void mlp_predict(const float* __restrict__ P, Norm nm, const float* __restrict__ qs,
                                                   uint32_t n, float* __restrict__ y) {
    const int lane = threadIdx.x & 63;
    InferWeights W;
    load_weights(P, lane, W);
    const uint32_t ntiles = (n + 63) / 64;
    const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint32_t nwaves = gridDim.x * (blockDim.x >> 6);
    for (uint32_t tile = wave; tile < ntiles; tile += nwaves) {
        float xs[4][3];
        load_tile_x<false>(qs, n, tile, lane, nm, xs);
        const float yy = mlp_tile(W, xs, lane);
        const uint32_t i = tile * 64u + uint32_t(lane);
        if (i < n) y[i] = yy;
    }
}

// Forward + backward for one batch: block w covers batch entries
// [64w, 64w + 64); sample b is row idx[b0 + b] of (qs, t).  Writes the wave's
// partial gradient (parameter order) to part[w][*] and its partial loss
// sum((y - t)^2) to part_loss[w].  scale = 2 / batch.
__global__ __launch_bounds__(64) void mlp_fwd_bwd(const float* __restrict__ P, Norm nm,
                                                  const float* __restrict__ qs, const float* __restrict__ t,
                                                  const uint32_t* __restrict__ idx, uint32_t b0, uint32_t batch,
                                                  float scale, float* __restrict__ part,
                                                  float* __restrict__ part_loss) {
    __shared__ TrainSmem sm;
    const int lane = threadIdx.x;
    stage_w2(P, sm.w2, sm.w2t, lane, 64);
    const MlpBufs B{sm.w2, sm.w2t, sm.h1, sm.h1t, sm.h2, sm.da2t, sm.red, sm.x, sm.dy, sm.a1pos};
    wave_sync();
    const uint32_t b = blockIdx.x * 64u + lane;
    const bool valid = b < batch;
    float q[3] = {0.f, 0.f, 0.f};
    float tgt = 0.f;
    if (valid) {
        const uint32_t row = idx ? idx[b0 + b] : b0 + b;
        q[0] = qs[size_t(row) * 3 + 0];
        q[1] = qs[size_t(row) * 3 + 1];
        q[2] = qs[size_t(row) * 3 + 2];
        tgt = t[row];
    }
    f32x4 acc[4][4];
    const float y = mlp_forward(P, nm, q, B, acc, true, lane);
    const float err = valid ? y - tgt : 0.0f;
    const float dy = scale * err;
    sm.dy[lane] = dy;
    float* out = part + size_t(blockIdx.x) * NPARAM;
    const float lsum = wave_sum(err * err);
    const float gb3 = wave_sum(dy);
    if (lane == 0) {
        part_loss[blockIdx.x] = lsum;
        out[OFF_B3] = gb3;
    }
    wave_sync();

    // layer-2 output gradient in the matrix-core layout of acc
    const int r16 = lane & 15, rg = (lane >> 4) * 4, grp = lane >> 4;
    float gb2p[4] = {0, 0, 0, 0}, gw3p[4] = {0, 0, 0, 0};
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
        const int o = ni * 16 + r16;
        const float w3b = bf16_round(P[OFF_W3 + o]);
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int qq = mi * 16 + rg + r;
                const float a2 = acc[mi][ni][r];
                const float h2 = bf16_round(a2 > 0.0f ? a2 : 0.0f);
                const float dyq = sm.dy[qq];
                gw3p[ni] += dyq * h2;
                const float da2 = a2 > 0.0f ? dyq * w3b : 0.0f;
                gb2p[ni] += da2;
                const uint16_t db = bf16_bits(da2);
                sm.h2[qq * HID + o] = db;  // h2 is no longer needed: reuse as da2 [q][o]
                sm.da2t[o * HID + qq] = db;
            }
    }
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
        sm.red[grp][ni * 16 + r16][0] = gb2p[ni];
        sm.red[grp][ni * 16 + r16][1] = gw3p[ni];
    }
    wave_sync();
    {
        const int o = lane;
        float s0 = 0, s1 = 0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            s0 += sm.red[g][o][0];
            s1 += sm.red[g][o][1];
        }
        out[OFF_B2 + o] = s0;
        out[OFF_W3 + o] = s1;
    }
    wave_sync();

    // dW2[o][i] = sum_q da2b[q][o] h1[q][i]
    gemm64_nt(sm.da2t, sm.h1t, acc, lane);
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) out[OFF_W2 + (mi * 16 + rg + r) * HID + ni * 16 + r16] = acc[mi][ni][r];

    // dh1[q][i] = sum_o da2b[q][o] W2b[o][i];  da1 = dh1 * [a1 > 0]
    gemm64_nt(sm.h2, sm.w2t, acc, lane);
    float gb1p[4] = {0, 0, 0, 0}, gw1p[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int qq = mi * 16 + rg + r;
            const uint64_t pos = sm.a1pos[qq];
            const float x0 = sm.x[qq][0], x1 = sm.x[qq][1], x2 = sm.x[qq][2];
#pragma unroll
            for (int ni = 0; ni < 4; ++ni) {
                const int i = ni * 16 + r16;
                const float da1 = ((pos >> i) & 1u) ? acc[mi][ni][r] : 0.0f;
                gb1p[ni] += da1;
                gw1p[ni][0] += da1 * x0;
                gw1p[ni][1] += da1 * x1;
                gw1p[ni][2] += da1 * x2;
            }
        }
    wave_sync();
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
        sm.red[grp][ni * 16 + r16][0] = gb1p[ni];
        sm.red[grp][ni * 16 + r16][1] = gw1p[ni][0];
        sm.red[grp][ni * 16 + r16][2] = gw1p[ni][1];
        sm.red[grp][ni * 16 + r16][3] = gw1p[ni][2];
    }
    wave_sync();
    {
        const int i = lane;
        float s[4] = {0, 0, 0, 0};
#pragma unroll
        for (int g = 0; g < 4; ++g)
#pragma unroll
            for (int c = 0; c < 4; ++c) s[c] += sm.red[g][i][c];
        out[OFF_B1 + i] = s[0];
        out[OFF_W1 + 3 * i + 0] = s[1];
        out[OFF_W1 + 3 * i + 1] = s[2];
        out[OFF_W1 + 3 * i + 2] = s[3];
    }
}

// Sum of the wave partials in a fixed order, then (step > 0) one Adam step on
// the float32 master weights.  bc1 = 1 - beta1^step and bc2 = 1 - beta2^step
// come from the host (computed in double and rounded once: at small steps
// 1 - beta2^step cancels, and a fast power would lose most of its digits).
// grad (nullable) receives the summed gradient; loss (nullable, thread 0) the
// batch loss.
__global__ void mlp_reduce_adam(const float* __restrict__ part, const float* __restrict__ part_loss, int nparts,
                                float inv_batch, float* __restrict__ P, float* __restrict__ m,
                                float* __restrict__ v, int step, float lr, float beta1, float beta2, float eps,
                                float bc1, float bc2, float* __restrict__ grad, float* __restrict__ loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && loss) {
        float s = 0;
        for (int w = 0; w < nparts; ++w) s += part_loss[w];
        *loss = s * inv_batch;
    }
    if (p >= NPARAM) return;
    float g = 0;
    for (int w = 0; w < nparts; ++w) g += part[size_t(w) * NPARAM + p];
    if (grad) grad[p] = g;
    if (step > 0) {
        const float mm = beta1 * m[p] + (1.0f - beta1) * g;
        const float vv = beta2 * v[p] + (1.0f - beta2) * g * g;
        m[p] = mm;
        v[p] = vv;
        const float mhat = mm / bc1;
        const float vhat = vv / bc2;
        P[p] -= lr * mhat / (__fsqrt_rn(vhat) + eps);
    }
}

// t[i] = 0.5 ln(max(d2_k, 1e-14)) from the k-th column of a kNN result
__global__ void knn_label(const float* __restrict__ d2, int k, uint32_t n, float* __restrict__ t) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v = d2[size_t(i) * k + (k - 1)];
    v = v > 1e-14f ? v : 1e-14f;
    t[i] = 0.5f * logf(v);
}

// Caller-layout queries [n][3] as traversal records (x, y, z, row = i).
__global__ void caller_records3(const float* __restrict__ q, uint32_t n, float4* __restrict__ rec) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    rec[i] = make_float4(q[size_t(i) * 3 + 0], q[size_t(i) * 3 + 1], q[size_t(i) * 3 + 2], __uint_as_float(i));
}

Norm make_norm(const float* lo, const float* inv) {
    Norm nm;
    for (int j = 0; j < 3; ++j) {
        nm.lo[j] = lo[j];
        nm.inv[j] = inv[j];
    }
    return nm;
}

}  // namespace

// Inference grid: workgroups of 4 waves, each wave looping over 64-query
// tiles (weights are loaded once per wave); at most 768 workgroups, three
// waves per SIMD at 148 VGPRs on 256 CUs.
static uint32_t infer_grid(uint32_t n) {
    const uint32_t tiles = (n + 63) / 64;
    uint32_t grid = (tiles + 3) / 4;
    return grid > 768 ? 768 : grid;
}

hipError_t launch_mlp_worst0(const float* P, const float* lo, const float* inv, float margin, float R2,
                             const void* sq, uint32_t Q, float* worst0, hipStream_t st) {
    if (Q == 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_worst0, dim3(infer_grid(Q)), dim3(256), 0, st, P, make_norm(lo, inv), margin, R2,
                       reinterpret_cast<const float4*>(sq), Q, worst0);
    return hipGetLastError();
}

hipError_t launch_mlp_worst0_jobs(const MlpJob* jobs, int njobs, uint32_t ntiles, const void* recs, float* worst0,
                                  hipStream_t st) {
    if (ntiles == 0 || njobs == 0) return hipSuccess;
    uint32_t grid = (ntiles + 3) / 4;
    if (grid > 768) grid = 768;
    hipLaunchKernelGGL(mlp_worst0_jobs, dim3(grid), dim3(256), 0, st, jobs, njobs, ntiles,
                       static_cast<const float4*>(recs), worst0);
    return hipGetLastError();
}

hipError_t launch_mlp_worst0_rows(const float* P, const float* lo, const float* inv, float margin, float R2,
                                  const float* queries, uint32_t n, void* recs, float* worst0, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(caller_records3, dim3((n + 255) / 256), dim3(256), 0, st, queries, n,
                       static_cast<float4*>(recs));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_mlp_worst0(P, lo, inv, margin, R2, recs, n, worst0, st);
}

hipError_t launch_mlp_predict(const float* P, const float* lo, const float* inv, const float* qs, uint32_t n,
                              float* y, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_predict, dim3(infer_grid(n)), dim3(256), 0, st, P, make_norm(lo, inv), qs, n, y);
    return hipGetLastError();
}

hipError_t launch_mlp_fwd_bwd(const float* P, const float* lo, const float* inv, const float* qs, const float* t,
                              const uint32_t* idx, uint32_t b0, uint32_t batch, float* part, float* part_loss,
                              hipStream_t st) {
    hipLaunchKernelGGL(mlp_fwd_bwd, dim3((batch + 63) / 64), dim3(64), 0, st, P, make_norm(lo, inv), qs, t, idx, b0,
                       batch, 2.0f / float(batch), part, part_loss);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce_adam(const float* part, const float* part_loss, int nparts, uint32_t batch, float* P,
                                  float* m, float* v, int step, float lr, float* grad, float* loss, hipStream_t st) {
    const float beta1 = MLP_ADAM_BETA1, beta2 = MLP_ADAM_BETA2;
    const float bc1 = step > 0 ? float(1.0 - std::pow(double(beta1), double(step))) : 1.0f;
    const float bc2 = step > 0 ? float(1.0 - std::pow(double(beta2), double(step))) : 1.0f;
    hipLaunchKernelGGL(mlp_reduce_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, st, part, part_loss, nparts,
                       1.0f / float(batch), P, m, v, step, lr, beta1, beta2, MLP_ADAM_EPS, bc1, bc2, grad, loss);
    return hipGetLastError();
}

hipError_t launch_knn_label(const float* d2, int k, uint32_t n, float* t, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(knn_label, dim3((n + 255) / 256), dim3(256), 0, st, d2, k, n, t);
    return hipGetLastError();
}

}  // namespace kd
