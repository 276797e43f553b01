// mlp.hip -- the learned flip-proposal network on gfx950: bf16 operands on
// the MFMA matrix cores with fp32 accumulation.
//
//   z1 = X W1 + b1, h1 = bf16(relu(z1)); z2 = h1 W2 + b2, h2 = bf16(relu(z2));
//   logit = h2 . w3 + b3;  loss = mean(softplus(logit) - y logit)
//
// The three dense products of the forward pass and the three of the backward
// pass run through one tiled GEMM kernel (64x128 output tile per workgroup,
// four wavefronts of 32x64 on v_mfma_f32_32x32x16_bf16, K staged through LDS
// 64 at a time) with fused epilogues: bias + ReLU + bf16 rounding (forward),
// ReLU mask + bf16 rounding (backpropagated deltas), plain fp32 (weight
// gradients).
#include <hip/hip_runtime.h>

#include "../../include/tsf.h"
#include "tsf_internal.h"

#include <cstring>

namespace {

typedef float v16f32 __attribute__((ext_vector_type(16)));

constexpr int IN = TSF_MLP_IN, HID = TSF_MLP_HID;
// offsets into the fp32 parameter vector
constexpr int O_W1T = 0;                   // W1^T: HID x IN (row n holds W1[:, n])
constexpr int O_B1 = O_W1T + HID * IN;     // HID
constexpr int O_W2T = O_B1 + HID;          // W2^T: HID x HID
constexpr int O_B2 = O_W2T + HID * HID;    // HID
constexpr int O_W3 = O_B2 + HID;           // HID
constexpr int O_B3 = O_W3 + HID;           // 1 (padded to 4)
static_assert(O_B3 + 4 == TSF_MLP_NPARAM, "parameter layout");
// offsets into the bf16 compute copies
constexpr int Q_W1T = 0;                   // HID x IN
constexpr int Q_W2T = Q_W1T + HID * IN;    // HID x HID (W2^T)
constexpr int Q_W2 = Q_W2T + HID * HID;    // HID x HID (W2, for the backward)
constexpr int Q_W3 = Q_W2 + HID * HID;     // HID
static_assert(Q_W3 + HID == TSF_MLP_NBF16, "bf16 layout");

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    // round to nearest, ties to even (finite inputs)
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

enum Epilogue { EP_BIAS_RELU_BF16 = 0, EP_MASK_BF16 = 1, EP_F32 = 2 };

struct GemmArgs {
    // C[m][n] = sum_k A(m,k) B(n,k); element (r,c) of an operand at
    // ptr[r * s_row + c * s_col] (bf16)
    const uint16_t *A;
    int64_t a_row, a_col;
    const uint16_t *B;
    int64_t b_row, b_col;
    int M, N, K;
    int ep;
    const float *bias;      // EP_BIAS_RELU_BF16: N
    const uint16_t *mask;   // EP_MASK_BF16: M x N, row-major (keep where > 0)
    uint16_t *out_bf16;     // M x N row-major
    float *out_f32;         // M x N row-major
};

typedef __bf16 v8bf16 __attribute__((ext_vector_type(8)));

// Output tile BM x BN per workgroup of four wavefronts (2 x 2 of WM x 64);
// K is staged through LDS 64 at a time.
constexpr int BM = 64, BN = 128, BK = 64, LDK = BK + 8;
// wavefront sub-tile: WM x 64, AM blocks of 32 rows
constexpr int WM = BM / 2, AM = WM / 32;

// Stage a 128 x BK tile of an operand (rows r0.., cols k0..) into LDS as
// tile[r][k], zero outside the matrix.  When the operand's k is contiguous,
// each thread moves 8 consecutive elements (16 bytes) at a time; otherwise
// threads walk the contiguous row dimension so reads still coalesce.
template <int R>
__device__ __forceinline__ void stage(uint16_t (*tile)[LDK], const uint16_t *P, int64_t s_row,
                                      int64_t s_col, int rows, int K, int r0, int k0)
{
    const int tid = threadIdx.x;
    if (s_col == 1) {
        for (int e = tid; e < R * BK / 8; e += 256) {
            const int r = e / (BK / 8), kc = (e % (BK / 8)) * 8;
            const int gr = r0 + r, gk = k0 + kc;
            const uint16_t *src = P + gr * s_row + gk;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (gr < rows) {
                if (gk + 8 <= K && ((reinterpret_cast<uintptr_t>(src) & 15) == 0)) {
                    v = *reinterpret_cast<const uint4 *>(src);
                } else {
                    uint16_t tmp[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) tmp[q] = (gk + q < K) ? src[q] : (uint16_t)0;
                    v = make_uint4(tmp[0] | (uint32_t)tmp[1] << 16, tmp[2] | (uint32_t)tmp[3] << 16,
                                   tmp[4] | (uint32_t)tmp[5] << 16, tmp[6] | (uint32_t)tmp[7] << 16);
                }
            }
            *reinterpret_cast<uint4 *>(&tile[r][kc]) = v;
        }
    } else {
        for (int e = tid; e < R * BK; e += 256) {
            const int k = e / R, r = e % R;
            const int gr = r0 + r, gk = k0 + k;
            tile[r][k] = (gr < rows && gk < K) ? P[gr * s_row + gk * s_col] : (uint16_t)0;
        }
    }
}

// The same staging split in two for operands whose k is contiguous: each
// thread's two 16-byte pieces of the next tile are read into registers while
// the current tile is multiplied, then written to LDS.
template <int R>
struct Frag {
    static_assert(R * BK % (8 * 256) == 0, "whole 16-byte pieces per thread");
    uint4 v[R * BK / 8 / 256];
};
template <int R>
__device__ __forceinline__ void load_frag(Frag<R> &f, const uint16_t *P, int64_t s_row, int rows,
                                          int K, int r0, int k0)
{
#pragma unroll
    for (int t = 0; t < R * BK / 8 / 256; ++t) {
        const int e = threadIdx.x + 256 * t;
        const int r = e / (BK / 8), kc = (e % (BK / 8)) * 8;
        const int gr = r0 + r, gk = k0 + kc;
        const uint16_t *src = P + gr * s_row + gk;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (gr < rows) {
            if (gk + 8 <= K && ((reinterpret_cast<uintptr_t>(src) & 15) == 0)) {
                v = *reinterpret_cast<const uint4 *>(src);
            } else {
                uint16_t tmp[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) tmp[q] = (gk + q < K) ? src[q] : (uint16_t)0;
                v = make_uint4(tmp[0] | (uint32_t)tmp[1] << 16, tmp[2] | (uint32_t)tmp[3] << 16,
                               tmp[4] | (uint32_t)tmp[5] << 16, tmp[6] | (uint32_t)tmp[7] << 16);
            }
        }
        f.v[t] = v;
    }
}
template <int R>
__device__ __forceinline__ void store_frag(uint16_t (*tile)[LDK], const Frag<R> &f)
{
#pragma unroll
    for (int t = 0; t < R * BK / 8 / 256; ++t) {
        const int e = threadIdx.x + 256 * t;
        const int r = e / (BK / 8), kc = (e % (BK / 8)) * 8;
        *reinterpret_cast<uint4 *>(&tile[r][kc]) = f.v[t];
    }
}

__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g)
{
    // one LDS buffer: the A and B tiles during the products, the output tile
    // of the forward epilogue afterwards
    constexpr int kTiles = (BM + BN) * LDK, kOut = BM * (BN + 8);
    __shared__ __attribute__((aligned(16))) uint16_t smem[kTiles > kOut ? kTiles : kOut];
    uint16_t (*As)[LDK] = reinterpret_cast<uint16_t (*)[LDK]>(smem);
    uint16_t (*Bs)[LDK] = reinterpret_cast<uint16_t (*)[LDK]>(smem + BM * LDK);
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm = (wave >> 1) * WM, wn = (wave & 1) * 64;  // this wave's WM x 64 sub-tile
    v16f32 acc[AM][2];
#pragma unroll
    for (int a = 0; a < AM; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[a][b][q] = 0.0f;
    const int row = lane & 31, kh = 8 * (lane >> 5);
    // both operands k-contiguous (the forward pass): the next tile's reads
    // overlap this tile's products
    const bool piped = g.a_col == 1 && g.b_col == 1;
    Frag<BM> fa;
    Frag<BN> fb;
    if (piped) {
        load_frag(fa, g.A, g.a_row, g.M, g.K, m0, 0);
        load_frag(fb, g.B, g.b_row, g.N, g.K, n0, 0);
    }
    for (int k0 = 0; k0 < g.K; k0 += BK) {
        if (piped) {
            store_frag(As, fa);
            store_frag(Bs, fb);
        } else {
            stage<BM>(As, g.A, g.a_row, g.a_col, g.M, g.K, m0, k0);
            stage<BN>(Bs, g.B, g.b_row, g.b_col, g.N, g.K, n0, k0);
        }
        __syncthreads();
        if (piped && k0 + BK < g.K) {
            load_frag(fa, g.A, g.a_row, g.M, g.K, m0, k0 + BK);
            load_frag(fb, g.B, g.b_row, g.N, g.K, n0, k0 + BK);
        }
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            // 32x32x16: lane l holds A[l%32][8*(l/32) + 0..7] and B[l%32][same k]
            v8bf16 av[AM], bv[2];
#pragma unroll
            for (int a = 0; a < AM; ++a)
                av[a] = *reinterpret_cast<const v8bf16 *>(&As[wm + 32 * a + row][kk + kh]);
#pragma unroll
            for (int b = 0; b < 2; ++b)
                bv[b] = *reinterpret_cast<const v8bf16 *>(&Bs[wn + 32 * b + row][kk + kh]);
#pragma unroll
            for (int a = 0; a < AM; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
    }
    // accumulator register q of lane l: row 8*(q/4) + 4*(l/32) + q%4, column l%32
    if (g.ep == EP_BIAS_RELU_BF16 && m0 + BM <= g.M && n0 + BN <= g.N && (g.N & 7) == 0 &&
        (reinterpret_cast<uintptr_t>(g.out_bf16) & 15) == 0) {
        // full tile of the forward pass: bias + ReLU + bf16 into LDS, then
        // 16-byte row-contiguous stores
        uint16_t (*Cs)[BN + 8] = reinterpret_cast<uint16_t (*)[BN + 8]>(smem);
#pragma unroll
        for (int a = 0; a < AM; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int cl = wn + 32 * b + (lane & 31);
                const float bias = g.bias[n0 + cl];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int rl = wm + 32 * a + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                    const float v = acc[a][b][q] + bias;
                    Cs[rl][cl] = to_bf16(v > 0.0f ? v : 0.0f);
                }
            }
        __syncthreads();
        for (int e = threadIdx.x; e < BM * BN / 8; e += 256) {
            const int r = e / (BN / 8), c = (e % (BN / 8)) * 8;
            *reinterpret_cast<uint4 *>(g.out_bf16 + (int64_t)(m0 + r) * g.N + n0 + c) =
                *reinterpret_cast<const uint4 *>(&Cs[r][c]);
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < AM; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int col = n0 + wn + 32 * b + (lane & 31);
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int rr = m0 + wm + 32 * a + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                if (rr >= g.M || col >= g.N) continue;
                float v = acc[a][b][q];
                const int64_t o = (int64_t)rr * g.N + col;
                if (g.ep == EP_BIAS_RELU_BF16) {
                    v += g.bias[col];
                    g.out_bf16[o] = to_bf16(v > 0.0f ? v : 0.0f);
                } else if (g.ep == EP_MASK_BF16) {
                    const bool keep = from_bf16(g.mask[o]) > 0.0f;
                    g.out_bf16[o] = to_bf16(keep ? v : 0.0f);
                } else {
                    g.out_f32[o] = v;
                }
            }
        }
}

// logit = h2 . w3 + b3; one wavefront per row
__global__ void __launch_bounds__(256) logit_kernel(const uint16_t *h2, const uint16_t *w3,
                                                    const float *b3, int M, float *logit)
{
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= M) return;
    float s = 0.0f;
    for (int n = lane; n < HID; n += 64)
        s += from_bf16(h2[(int64_t)row * HID + n]) * from_bf16(w3[n]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) logit[row] = s + b3[0];
}

// delta3 = (sigmoid(logit) - y) / M; delta2 = bf16(delta3 w3 [h2 > 0]); loss
__global__ void __launch_bounds__(256) delta_kernel(const float *logit, const float *y,
                                                    const uint16_t *h2, const uint16_t *w3, int M,
                                                    float *d3, uint16_t *d2, float *loss)
{
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= M) return;
    const float z = logit[row];
    const float sig = 1.0f / (1.0f + __expf(-z));
    const float dz = (sig - y[row]) / (float)M;
    if (lane == 0) {
        d3[row] = dz;
        // softplus(z) - y z, computed stably
        const float sp = z > 0.0f ? z + log1pf(__expf(-z)) : log1pf(__expf(z));
        atomicAdd(loss, (sp - y[row] * z) / (float)M);
    }
    for (int n = lane; n < HID; n += 64) {
        const int64_t o = (int64_t)row * HID + n;
        const bool keep = from_bf16(h2[o]) > 0.0f;
        d2[o] = to_bf16(keep ? dz * from_bf16(w3[n]) : 0.0f);
    }
}

// column sums: out[n] += sum over this block's rows of A[m][n] (bf16 A), or
// of w[m] A[m][n] when w is given; out must be zeroed first
__global__ void __launch_bounds__(256) colsum_kernel(const uint16_t *A, const float *w, int M,
                                                     int N, float *out)
{
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    const int m_begin = blockIdx.y * 64, m_end = min(M, m_begin + 64);
    float s = 0.0f;
    for (int m = m_begin; m < m_end; ++m) {
        const float a = from_bf16(A[(int64_t)m * N + n]);
        s += w ? w[m] * a : a;
    }
    atomicAdd(&out[n], s);
}

__global__ void sum_kernel(const float *v, int M, float *out)
{
    __shared__ float sh[256];
    float s = 0.0f;
    for (int m = threadIdx.x; m < M; m += 256) s += v[m];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

__global__ void zero_kernel(float *p, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// Adam (Kingma & Ba) on the fp32 masters
__global__ void adam_kernel(float *p, const float *g, float *m, float *v, int n, float lr, float b1,
                            float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bf16 compute copies from the fp32 masters: W1^T, W2^T, W2, w3
__global__ void sync_kernel(const float *p, uint16_t *q)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < HID * IN) q[Q_W1T + i] = to_bf16(p[O_W1T + i]);
    if (i < HID * HID) {
        q[Q_W2T + i] = to_bf16(p[O_W2T + i]);
        const int n = i / HID, k = i % HID;  // W2[k][n] = W2^T[n][k]
        q[Q_W2 + k * HID + n] = to_bf16(p[O_W2T + i]);
    }
    if (i < HID) q[Q_W3 + i] = to_bf16(p[O_W3 + i]);
}

tsf_status launch_gemm(const GemmArgs &g, hipStream_t s)
{
    dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM);
    if (grid.y > 65535u) return tsf_fail(TSF_E_ARG, "GEMM with %d rows exceeds the grid", g.M);
    hipLaunchKernelGGL(gemm_kernel, grid, dim3(256), 0, s, g);
    if (hipGetLastError() != hipSuccess) return tsf_fail(TSF_E_DEVICE, "GEMM launch failed");
    return TSF_OK;
}

tsf_status check_net(const tsf_mlp *net)
{
    if (!net || !net->param || !net->wbf) return tsf_fail(TSF_E_ARG, "null network buffers");
    return TSF_OK;
}

}  // namespace

extern "C" {

tsf_status tsf_mlp_sync(const tsf_mlp *net, void *hip_stream)
{
    tsf_status st = check_net(net);
    if (st) return st;
    hipLaunchKernelGGL(sync_kernel, dim3((HID * IN + 255) / 256), dim3(256), 0,
                       (hipStream_t)hip_stream, net->param, net->wbf);
    if (hipGetLastError() != hipSuccess) return tsf_fail(TSF_E_DEVICE, "sync launch failed");
    return TSF_OK;
}

tsf_status tsf_mlp_fwd(const tsf_mlp *net, const uint16_t *X, int32_t M, uint16_t *h1,
                       uint16_t *h2, float *logit, void *hip_stream)
{
    tsf_status st = check_net(net);
    if (st) return st;
    if (M < 0 || (M > 0 && (!X || !h1 || !h2 || !logit))) return tsf_fail(TSF_E_ARG, "bad forward arguments");
    if (M == 0) return TSF_OK;
    hipStream_t s = (hipStream_t)hip_stream;
    GemmArgs g;
    std::memset(&g, 0, sizeof g);
    g.A = X; g.a_row = IN; g.a_col = 1;
    g.B = net->wbf + Q_W1T; g.b_row = IN; g.b_col = 1;
    g.M = M; g.N = HID; g.K = IN;
    g.ep = EP_BIAS_RELU_BF16; g.bias = net->param + O_B1; g.out_bf16 = h1;
    if ((st = launch_gemm(g, s))) return st;
    g.A = h1; g.a_row = HID;
    g.B = net->wbf + Q_W2T; g.b_row = HID;
    g.K = HID; g.bias = net->param + O_B2; g.out_bf16 = h2;
    if ((st = launch_gemm(g, s))) return st;
    hipLaunchKernelGGL(logit_kernel, dim3((M + 3) / 4), dim3(256), 0, s, h2, net->wbf + Q_W3,
                       net->param + O_B3, M, logit);
    if (hipGetLastError() != hipSuccess) return tsf_fail(TSF_E_DEVICE, "logit launch failed");
    return TSF_OK;
}

tsf_status tsf_mlp_bwd(const tsf_mlp *net, const uint16_t *X, const float *y, int32_t M,
                       const uint16_t *h1, const uint16_t *h2, const float *logit, uint16_t *d2,
                       uint16_t *d1, float *d3, float *loss, void *hip_stream)
{
    tsf_status st = check_net(net);
    if (st) return st;
    if (!net->grad) return tsf_fail(TSF_E_ARG, "null gradient buffer");
    if (M <= 0 || !X || !y || !h1 || !h2 || !logit || !d2 || !d1 || !d3 || !loss)
        return tsf_fail(TSF_E_ARG, "bad backward arguments");
    hipStream_t s = (hipStream_t)hip_stream;
    float *gp = net->grad;
    hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(256), 0, s, loss, 1);
    hipLaunchKernelGGL(delta_kernel, dim3((M + 3) / 4), dim3(256), 0, s, logit, y, h2,
                       net->wbf + Q_W3, M, d3, d2, loss);
    // dW3 = h2^T d3, db3 = sum d3, db2 = colsum d2
    const dim3 cs_grid(1, (M + 63) / 64);
    hipLaunchKernelGGL(zero_kernel, dim3((TSF_MLP_NPARAM + 255) / 256), dim3(256), 0, s, gp,
                       TSF_MLP_NPARAM);
    hipLaunchKernelGGL(colsum_kernel, cs_grid, dim3(256), 0, s, h2, d3, M, HID, gp + O_W3);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, d3, M, gp + O_B3);
    hipLaunchKernelGGL(colsum_kernel, cs_grid, dim3(256), 0, s, d2, (const float *)nullptr, M, HID,
                       gp + O_B2);
    GemmArgs g;
    std::memset(&g, 0, sizeof g);
    // dW2^T[n][k] = sum_m d2[m][n] h1[m][k]
    g.A = d2; g.a_row = 1; g.a_col = HID;
    g.B = h1; g.b_row = 1; g.b_col = HID;
    g.M = HID; g.N = HID; g.K = M;
    g.ep = EP_F32; g.out_f32 = gp + O_W2T;
    if ((st = launch_gemm(g, s))) return st;
    // d1 = (d2 W2^T) [h1 > 0]: d1[m][k] = sum_n d2[m][n] W2[k][n]
    g.A = d2; g.a_row = HID; g.a_col = 1;
    g.B = net->wbf + Q_W2; g.b_row = HID; g.b_col = 1;
    g.M = M; g.N = HID; g.K = HID;
    g.ep = EP_MASK_BF16; g.mask = h1; g.out_bf16 = d1; g.out_f32 = nullptr;
    if ((st = launch_gemm(g, s))) return st;
    hipLaunchKernelGGL(colsum_kernel, cs_grid, dim3(256), 0, s, d1, (const float *)nullptr, M, HID,
                       gp + O_B1);
    // dW1^T[n][k] = sum_m d1[m][n] X[m][k]
    g.A = d1; g.a_row = 1; g.a_col = HID;
    g.B = X; g.b_row = 1; g.b_col = IN;
    g.M = HID; g.N = IN; g.K = M;
    g.ep = EP_F32; g.mask = nullptr; g.out_bf16 = nullptr; g.out_f32 = gp + O_W1T;
    if ((st = launch_gemm(g, s))) return st;
    if (hipGetLastError() != hipSuccess) return tsf_fail(TSF_E_DEVICE, "backward launch failed");
    return TSF_OK;
}

tsf_status tsf_mlp_step(const tsf_mlp *net, float lr, float beta1, float beta2, float eps,
                        int32_t step, void *hip_stream)
{
    tsf_status st = check_net(net);
    if (st) return st;
    if (!net->grad || !net->adam_m || !net->adam_v || step < 1)
        return tsf_fail(TSF_E_ARG, "bad optimiser arguments");
    hipStream_t s = (hipStream_t)hip_stream;
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((TSF_MLP_NPARAM + 255) / 256), dim3(256), 0, s,
                       net->param, net->grad, net->adam_m, net->adam_v, TSF_MLP_NPARAM, lr, beta1,
                       beta2, eps, c1, c2);
    if (hipGetLastError() != hipSuccess) return tsf_fail(TSF_E_DEVICE, "adam launch failed");
    return tsf_mlp_sync(net, hip_stream);
}

}  // extern "C"
