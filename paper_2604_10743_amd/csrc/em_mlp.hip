// Learned screen: a small MLP (16 -> 256 -> 256 -> 256 -> 1, exact GELU)
// predicting log10 of a tree's nucleation time from per-tree features, with
// hand-written BF16 MFMA GEMMs (FP32 accumulation), backward pass and Adam.
//
// Precision contract: every hidden-layer GEMM operand is
// rounded to BF16 (round to nearest even) when it is staged into LDS; the
// accumulation, bias, GELU, the output layer, the loss and the optimiser are
// FP32, with an FP32 master copy of every weight.
#include "em_internal.h"
#include "../../include/em.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int NF = 16;       // features
constexpr int KF = 16;       // padded feature width (MFMA K granularity)
constexpr int HID = 256;     // hidden width
constexpr int NPARAM = HID * NF + HID + HID * HID + HID + HID * HID + HID + HID + 1;

// parameter offsets (FP32 master layout, exported order)
constexpr int OW1 = 0, OB1 = OW1 + HID * NF, OW2 = OB1 + HID, OB2 = OW2 + HID * HID, OW3 = OB2 + HID,
              OB3 = OW3 + HID * HID, OW4 = OB3 + HID, OB4 = OW4 + HID;

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }   // RNE

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

enum Epi { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_GELU_BWD = 2 };

struct GemmArgs {
    const float *A;          // element (m, k) at A[m*sam + k*sak]
    const float *B;          // element (k, n) at B[k*sbk + n*sbn]
    float *C;                // (m, n) at C[m*ldc + n]
    float *H;                // EPI_BIAS_GELU: activations out (m, n) at H[m*ldc + n]
    const float *bias;       // EPI_BIAS_GELU: [N]
    const float *Z;          // EPI_GELU_BWD: pre-activations (m, n) at Z[m*ldc + n]
    long long sam, sak, sbk, sbn;
    int M, N, K, ldc;
};

// C[MxN] = A[MxK] B[KxN] on BF16 matrix cores.  A 256-thread block computes
// a 128x128 tile, each of its four waves a 64x64 quarter as 2x2 sub-tiles of
// the 32x32x16 BF16 MFMA, over K in steps of 32 staged through LDS (k
// contiguous, so every lane reads its 8 operand values with one 16-byte
// load).  Operand layout of the 32x32x16 MFMA: lane l supplies
// A[l%32][8*(l/32) .. +7] and B[8*(l/32) .. +7][l%32]; the 16 accumulator
// registers of lane l hold C[8*(r/4) + 4*(l/32) + r%4][l%32].  Blocks along
// grid z split K (partial tiles to a workspace, summed in a fixed order by
// k_splitk_sum) when the output is small and K long.
constexpr int TB = 128, BK = 32, LDK = BK + 8;

// Stage rows [r0, r0+128) x k [k0, k0+32) of a strided FP32 operand, element
// (r, k) at P[r*sr + k*sk], into T[row][k] as BF16 (zero outside R x K).
__device__ inline void stage_tile(__bf16 (*T)[LDK], const float *P, long long sr, long long sk, int r0, int R,
                                  int k0, int K, int tid)
{
    if (sk == 1) {
        const int r = tid >> 1, kk = (tid & 1) * 16;
        const int gr = r0 + r, gk = k0 + kk;
        const float *src = P + (long long)gr * sr + gk;
        if (gr < R && gk + 16 <= K && ((reinterpret_cast<uintptr_t>(src) & 15) == 0)) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 v = reinterpret_cast<const float4 *>(src)[q];
                T[r][kk + 4 * q + 0] = to_bf16(v.x); T[r][kk + 4 * q + 1] = to_bf16(v.y);
                T[r][kk + 4 * q + 2] = to_bf16(v.z); T[r][kk + 4 * q + 3] = to_bf16(v.w);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e)
                T[r][kk + e] = to_bf16((gr < R && gk + e < K) ? P[(long long)gr * sr + gk + e] : 0.0f);
        }
    } else {
        const int kk = tid >> 3, rr = (tid & 7) * 16;
        const int gk = k0 + kk, gr = r0 + rr;
        const float *src = P + (long long)gr * sr + (long long)gk * sk;
        if (sr == 1 && gk < K && gr + 16 <= R && ((reinterpret_cast<uintptr_t>(src) & 15) == 0)) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float4 v = reinterpret_cast<const float4 *>(src)[q];
                T[rr + 4 * q + 0][kk] = to_bf16(v.x); T[rr + 4 * q + 1][kk] = to_bf16(v.y);
                T[rr + 4 * q + 2][kk] = to_bf16(v.z); T[rr + 4 * q + 3][kk] = to_bf16(v.w);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e)
                T[rr + e][kk] = to_bf16((gk < K && gr + e < R) ? P[(long long)(gr + e) * sr + (long long)gk * sk]
                                                               : 0.0f);
        }
    }
}

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g, float *ws, int kchunk)
{
    __shared__ __attribute__((aligned(16))) __bf16 As[TB][LDK];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[TB][LDK];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m0 = blockIdx.y * TB, n0 = blockIdx.x * TB;
    const int wm = (wv >> 1) * 64, wn = (wv & 1) * 64;
    const int kbeg = blockIdx.z * kchunk, kend = min(g.K, kbeg + kchunk);
    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        stage_tile(As, g.A, g.sam, g.sak, m0, g.M, k0, kend, tid);
        stage_tile(Bs, g.B, g.sbn, g.sbk, n0, g.N, k0, kend, tid);
        __syncthreads();
#pragma unroll
        for (int kc = 0; kc < BK; kc += 16) {
            const int kb = kc + 8 * (lane >> 5);
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                a[i] = *reinterpret_cast<const bf16x8 *>(&As[wm + 32 * i + (lane & 31)][kb]);
                b[i] = *reinterpret_cast<const bf16x8 *>(&Bs[wn + 32 * i + (lane & 31)][kb]);
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int col = n0 + wn + 32 * j + (lane & 31);
                if (row >= g.M || col >= g.N) continue;
                float v = acc[i][j][r];
                if (ws) {                                   // split-K partial
                    ws[((size_t)blockIdx.z * g.M + row) * g.N + col] = v;
                    continue;
                }
                const long long o = (long long)row * g.ldc + col;
                if (EPI == EPI_BIAS_GELU) {
                    v += g.bias[col];
                    g.C[o] = v;
                    g.H[o] = gelu(v);
                } else if (EPI == EPI_GELU_BWD) {
                    g.C[o] = v * gelu_d(g.Z[o]);
                } else {
                    g.C[o] = v;
                }
            }
}

// C = sum over the splits of the workspace partials (fixed order)
__global__ __launch_bounds__(256) void k_splitk_sum(const float *ws, int splits, float *C, int M, int N, int ldc)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)M * N) return;
    float acc = 0.0f;
    for (int z = 0; z < splits; ++z) acc += ws[(size_t)z * M * N + i];
    C[(i / N) * ldc + (i % N)] = acc;
}

// y = H3 w4 + b4, one wave per row (fixed summation order)
__global__ __launch_bounds__(256) void k_out(const float *H3, const float *w4, const float *b4, float *y, int n)
{
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= n) return;
    float s = 0.f;
    for (int c = lane; c < HID; c += 64) s += H3[(long long)row * HID + c] * w4[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) y[row] = s + b4[0];
}

// dy = 2 (y - t) / n ; per-block partial losses
__global__ __launch_bounds__(256) void k_loss(const float *y, const float *t, float *dy, float *part, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    float e = 0.f;
    if (i < n) {
        float d = y[i] - t[i];
        dy[i] = 2.0f * d / (float)n;
        e = d * d;
    }
    __shared__ float red[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// dZ3 = dy w4 * gelu'(Z3)
__global__ __launch_bounds__(256) void k_out_bwd(const float *dy, const float *w4, const float *Z3, float *dZ3, int n)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)n * HID) return;
    const int row = (int)(i / HID), c = (int)(i % HID);
    dZ3[i] = dy[row] * w4[c] * gelu_d(Z3[i]);
}

// column sums over n rows: out[c] = sum_r X[r*ld + c] (w: optional row weights)
__global__ __launch_bounds__(256) void k_colsum(const float *X, const float *w, float *out, int n, int ncol, int ld)
{
    const int c = blockIdx.x;
    if (c >= ncol) return;
    float s = 0.f;
    for (int r = threadIdx.x; r < n; r += 256) s += X[(long long)r * ld + c] * (w ? w[r] : 1.0f);
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
}

// Adam on the FP32 master copy (bias-corrected moments)
__global__ __launch_bounds__(256) void k_adam(float *p, const float *gr, float *m, float *v, int n, float lr,
                                              float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// pack the [n][NF] feature rows into [n][KF] with zero padding (a copy while NF == KF)
__global__ __launch_bounds__(256) void k_pad_x(const float *X, float *Xp, int n)
{
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= (long long)n * KF) return;
    const int r = (int)(i / KF), c = (int)(i % KF);
    Xp[i] = c < NF ? X[(long long)r * NF + c] : 0.0f;
}

inline int cdiv(long long a, int b) { return (int)((a + b - 1) / b); }

}  // namespace

struct em_mlp {
    hipStream_t stream = nullptr;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // [NPARAM]
    float *W1p = nullptr;      // [HID][KF] padded first layer (rebuilt from p before use)
    float *gW1p = nullptr;
    float *ws = nullptr;       // split-K partials of the weight gradients [32][HID][HID]
    int cap = 0;               // rows allocated
    float *Xp = nullptr, *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *Z3 = nullptr, *H3 = nullptr;
    float *y = nullptr, *dy = nullptr, *dZ3 = nullptr, *dZ2 = nullptr, *dZ1 = nullptr, *part = nullptr;
    long long t = 0;           // Adam step
    std::string err;
};

namespace {

em_status mfail(em_mlp *m, em_status s, const std::string &msg)
{
    if (m) m->err = msg;
    return s;
}

#define MCHK(m, call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return mfail((m), EM_ERR_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

__global__ __launch_bounds__(256) void k_w1_pad(const float *p, float *W1p)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= HID * KF) return;
    const int r = i / KF, c = i % KF;
    W1p[i] = c < NF ? p[OW1 + r * NF + c] : 0.0f;
}

__global__ __launch_bounds__(256) void k_w1_unpad(const float *gW1p, float *g)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= HID * NF) return;
    const int r = i / NF, c = i % NF;
    g[OW1 + i] = gW1p[r * KF + c];
}

em_status ensure_rows(em_mlp *m, int n)
{
    if (n <= m->cap) return EM_OK;
    float **bufs[] = {&m->Xp, &m->Z1, &m->H1, &m->Z2, &m->H2, &m->Z3, &m->H3, &m->y, &m->dy, &m->dZ3, &m->dZ2,
                      &m->dZ1, &m->part};
    for (float **b : bufs)
        if (*b) { (void)hipFree(*b); *b = nullptr; }
    const size_t nr = (size_t)n;
    size_t sz[] = {nr * KF, nr * HID, nr * HID, nr * HID, nr * HID, nr * HID, nr * HID, nr, nr, nr * HID,
                   nr * HID, nr * HID, nr / 256 + 2};
    for (int k = 0; k < 13; ++k)
        if (hipMalloc((void **)bufs[k], sz[k] * sizeof(float)) != hipSuccess)
            return mfail(m, EM_ERR_OOM, "MLP activation buffers");
    m->cap = n;
    return EM_OK;
}

constexpr int SPLITK_MAX = 32;

void gemm(em_mlp *m, int epi, const float *A, long long sam, long long sak, const float *B, long long sbk,
          long long sbn, float *C, int ldc, int M, int N, int K, const float *bias, float *H, const float *Z,
          hipStream_t st)
{
    GemmArgs g;
    g.A = A; g.B = B; g.C = C; g.H = H; g.bias = bias; g.Z = Z;
    g.sam = sam; g.sak = sak; g.sbk = sbk; g.sbn = sbn;
    g.M = M; g.N = N; g.K = K; g.ldc = ldc;
    const int tiles = cdiv(N, TB) * cdiv(M, TB);
    int splits = 1;
    if (epi == EPI_STORE && tiles < 64 && K >= 2048 && (long long)M * N <= (long long)HID * HID)
        splits = std::min(SPLITK_MAX, K / 1024);
    const int kchunk = splits > 1 ? ((K + splits - 1) / splits + BK - 1) / BK * BK : K;
    splits = (K + kchunk - 1) / kchunk;
    dim3 grid(cdiv(N, TB), cdiv(M, TB), splits);
    float *ws = splits > 1 ? m->ws : nullptr;
    if (epi == EPI_BIAS_GELU) k_gemm_bf16<EPI_BIAS_GELU><<<grid, 256, 0, st>>>(g, nullptr, kchunk);
    else if (epi == EPI_GELU_BWD) k_gemm_bf16<EPI_GELU_BWD><<<grid, 256, 0, st>>>(g, nullptr, kchunk);
    else k_gemm_bf16<EPI_STORE><<<grid, 256, 0, st>>>(g, ws, kchunk);
    if (ws) k_splitk_sum<<<cdiv((long long)M * N, 256), 256, 0, st>>>(ws, splits, C, M, N, ldc);
}

// Activation buffers of one forward pass: padded input, pre-activations Z
// (kept for the backward pass; one shared buffer when only y is wanted) and
// post-activations H of the three hidden layers, output y.
struct Act {
    float *Xp, *Z1, *H1, *Z2, *H2, *Z3, *H3, *y;
};

// forward pass into the given activation buffers (X: device [n][NF])
void forward_into(em_mlp *m, const float *X, int n, const Act &a, hipStream_t st)
{
    k_pad_x<<<cdiv((long long)n * KF, 256), 256, 0, st>>>(X, a.Xp, n);
    k_w1_pad<<<cdiv(HID * KF, 256), 256, 0, st>>>(m->p, m->W1p);
    // Z1 = X W1^T + b1 : B(k, n) = W1p[n][k]
    gemm(m, EPI_BIAS_GELU, a.Xp, KF, 1, m->W1p, 1, KF, a.Z1, HID, n, HID, KF, m->p + OB1, a.H1, nullptr, st);
    gemm(m, EPI_BIAS_GELU, a.H1, HID, 1, m->p + OW2, 1, HID, a.Z2, HID, n, HID, HID, m->p + OB2, a.H2, nullptr, st);
    gemm(m, EPI_BIAS_GELU, a.H2, HID, 1, m->p + OW3, 1, HID, a.Z3, HID, n, HID, HID, m->p + OB3, a.H3, nullptr, st);
    k_out<<<cdiv(n, 4), 256, 0, st>>>(a.H3, m->p + OW4, m->p + OB4, a.y, n);
}

// forward pass into the model's own activation buffers
void forward(em_mlp *m, const float *X, int n, hipStream_t st)
{
    forward_into(m, X, n, Act{m->Xp, m->Z1, m->H1, m->Z2, m->H2, m->Z3, m->H3, m->y}, st);
}

// gradient of the mean squared error into m->g; the loss (when asked for)
// synchronises the stream
em_status backward(em_mlp *m, const float *t, int n, float *loss)
{
    hipStream_t st = m->stream;
    const int nb = cdiv(n, 256);
    k_loss<<<nb, 256, 0, st>>>(m->y, t, m->dy, m->part, n);
    // output layer
    k_colsum<<<HID, 256, 0, st>>>(m->H3, m->dy, m->g + OW4, n, HID, HID);
    k_colsum<<<1, 256, 0, st>>>(m->dy, nullptr, m->g + OB4, n, 1, 1);
    k_out_bwd<<<cdiv((long long)n * HID, 256), 256, 0, st>>>(m->dy, m->p + OW4, m->Z3, m->dZ3, n);
    // layer 3: dW3[o][i] = sum_r dZ3[r][o] H2[r][i]  (A(m=o,k=r) = dZ3[r][o])
    gemm(m, EPI_STORE, m->dZ3, 1, HID, m->H2, HID, 1, m->g + OW3, HID, HID, HID, n, nullptr, nullptr, nullptr, st);
    k_colsum<<<HID, 256, 0, st>>>(m->dZ3, nullptr, m->g + OB3, n, HID, HID);
    // dZ2 = (dZ3 W3) * gelu'(Z2) : B(k=o, n=i) = W3[o][i]
    gemm(m, EPI_GELU_BWD, m->dZ3, HID, 1, m->p + OW3, HID, 1, m->dZ2, HID, n, HID, HID, nullptr, nullptr, m->Z2, st);
    gemm(m, EPI_STORE, m->dZ2, 1, HID, m->H1, HID, 1, m->g + OW2, HID, HID, HID, n, nullptr, nullptr, nullptr, st);
    k_colsum<<<HID, 256, 0, st>>>(m->dZ2, nullptr, m->g + OB2, n, HID, HID);
    gemm(m, EPI_GELU_BWD, m->dZ2, HID, 1, m->p + OW2, HID, 1, m->dZ1, HID, n, HID, HID, nullptr, nullptr, m->Z1, st);
    // dW1[o][c] = sum_r dZ1[r][o] X[r][c]
    gemm(m, EPI_STORE, m->dZ1, 1, HID, m->Xp, KF, 1, m->gW1p, KF, HID, KF, n, nullptr, nullptr, nullptr, st);
    k_w1_unpad<<<cdiv(HID * NF, 256), 256, 0, st>>>(m->gW1p, m->g);
    k_colsum<<<HID, 256, 0, st>>>(m->dZ1, nullptr, m->g + OB1, n, HID, HID);
    MCHK(m, hipGetLastError());
    if (loss) {
        std::vector<float> parts(nb);
        MCHK(m, hipMemcpyAsync(parts.data(), m->part, sizeof(float) * nb, hipMemcpyDeviceToHost, st));
        MCHK(m, hipStreamSynchronize(st));
        double s = 0;
        for (float x : parts) s += x;
        *loss = (float)(s / n);
    }
    return EM_OK;
}

}  // namespace

namespace em {
int mlp_reserve(em_mlp *m, int n)
{
    if (!m || n <= 0) return EM_ERR_ARG;
    return ensure_rows(m, n);
}

int mlp_forward_async(em_mlp *m, const float *X, int n, float *y, hipStream_t st)
{
    if (!m || !X || !y || n <= 0) return EM_ERR_ARG;
    em_status s = ensure_rows(m, n);
    if (s != EM_OK) return s;
    forward(m, X, n, st);
    if (hipGetLastError() != hipSuccess) return EM_ERR_HIP;
    if (hipMemcpyAsync(y, m->y, sizeof(float) * n, hipMemcpyDeviceToDevice, st) != hipSuccess) return EM_ERR_HIP;
    return EM_OK;
}
}  // namespace em

// ---------------------------------------------------------------------------
// Allocation-free forward pass.  The activations live in a file-scope device
// array instead of the model's row-sized buffers (which em_mlp_forward grows
// with hipMalloc): padded input, one pre-activation buffer shared by the three
// layers (the backward pass is not run here), and the three post-activation
// buffers, each sized for NOALLOC_MAX_ROWS rows.  Every kernel guards its row
// loads and stores with n, so the array needs no clearing between calls.  In
// host code `scratch` names a host-side stand-in: kernels receive the device
// address that hipGetSymbolAddress returns, looked up once per device.
// ---------------------------------------------------------------------------
constexpr int NOALLOC_MAX_ROWS = 4096;
constexpr size_t NOALLOC_FLOATS = (size_t)NOALLOC_MAX_ROWS * (KF + 4 * HID);   // 17.0 MB
static __device__ __align__(256) float scratch[NOALLOC_FLOATS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float *g_scratch_dev[MAX_DEVICES] = {};     // device address of `scratch`, per device

// The scratch array of the device that runs `st`, set up on the first call
// on that device (with that device current, restored afterwards).
hipError_t scratch_of_stream(hipStream_t st, float **out)
{
    int dev = 0;
    hipError_t e = st ? hipStreamGetDevice(st, &dev) : hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        int cur = 0;
        if ((e = hipGetDevice(&cur)) != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) {
            hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = (float *)p;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}
}  // namespace

extern "C" {

int32_t em_mlp_noalloc_max_rows(void) { return NOALLOC_MAX_ROWS; }

em_status em_mlp_forward_noalloc(em_mlp *m, const float *X, int32_t n, float *y)
{
    if (!m || !X || !y || n <= 0) return mfail(m, EM_ERR_ARG, "bad forward arguments");
    if (n > NOALLOC_MAX_ROWS)
        return mfail(m, EM_ERR_ARG, "em_mlp_forward_noalloc: more rows than its scratch holds "
                                    "(em_mlp_noalloc_max_rows)");
    float *base = nullptr;
    MCHK(m, scratch_of_stream(m->stream, &base));
    const size_t R = NOALLOC_MAX_ROWS;
    float *Xp = base, *Z = Xp + R * KF, *H1 = Z + R * HID, *H2 = H1 + R * HID, *H3 = H2 + R * HID;
    forward_into(m, X, n, Act{Xp, Z, H1, Z, H2, Z, H3, y}, m->stream);
    MCHK(m, hipGetLastError());
    return EM_OK;
}

em_status em_mlp_create(void *hip_stream, em_mlp **out)
{
    if (!out) return EM_ERR_ARG;
    em_mlp *m = new (std::nothrow) em_mlp();
    if (!m) return EM_ERR_OOM;
    *out = m;
    m->stream = (hipStream_t)hip_stream;
    float **bufs[] = {&m->p, &m->g, &m->m, &m->v};
    for (float **b : bufs) {
        if (hipMalloc((void **)b, sizeof(float) * NPARAM) != hipSuccess) return mfail(m, EM_ERR_OOM, "MLP params");
        MCHK(m, hipMemsetAsync(*b, 0, sizeof(float) * NPARAM, m->stream));
    }
    MCHK(m, hipMalloc((void **)&m->W1p, sizeof(float) * HID * KF));
    MCHK(m, hipMalloc((void **)&m->ws, sizeof(float) * 32 * HID * HID));
    MCHK(m, hipMalloc((void **)&m->gW1p, sizeof(float) * HID * KF));
    MCHK(m, hipStreamSynchronize(m->stream));
    return EM_OK;
}

em_status em_mlp_destroy(em_mlp *m)
{
    if (!m) return EM_OK;
    (void)hipStreamSynchronize(m->stream);
    float *bufs[] = {m->p, m->g, m->m, m->v, m->W1p, m->gW1p, m->ws, m->Xp, m->Z1, m->H1, m->Z2, m->H2, m->Z3, m->H3,
                     m->y, m->dy, m->dZ3, m->dZ2, m->dZ1, m->part};
    for (float *b : bufs)
        if (b) (void)hipFree(b);
    delete m;
    return EM_OK;
}

const char *em_mlp_last_error(const em_mlp *m) { return m ? m->err.c_str() : "null MLP"; }

int32_t em_mlp_num_params(void) { return NPARAM; }

em_status em_mlp_set_params(em_mlp *m, const float *host, int32_t n)
{
    if (!m || !host || n != NPARAM) return mfail(m, EM_ERR_ARG, "expected em_mlp_num_params() floats");
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(host[i])) return mfail(m, EM_ERR_ARG, "non-finite parameter");
    MCHK(m, hipMemcpyAsync(m->p, host, sizeof(float) * NPARAM, hipMemcpyHostToDevice, m->stream));
    MCHK(m, hipMemsetAsync(m->m, 0, sizeof(float) * NPARAM, m->stream));
    MCHK(m, hipMemsetAsync(m->v, 0, sizeof(float) * NPARAM, m->stream));
    MCHK(m, hipStreamSynchronize(m->stream));
    m->t = 0;
    return EM_OK;
}

em_status em_mlp_get_params(em_mlp *m, float *host, int32_t n)
{
    if (!m || !host || n != NPARAM) return mfail(m, EM_ERR_ARG, "expected em_mlp_num_params() floats");
    MCHK(m, hipMemcpyAsync(host, m->p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, m->stream));
    MCHK(m, hipStreamSynchronize(m->stream));
    return EM_OK;
}

em_status em_mlp_forward(em_mlp *m, const float *X, int32_t n, float *y)
{
    if (!m || !X || !y || n <= 0) return mfail(m, EM_ERR_ARG, "bad forward arguments");
    em_status s = ensure_rows(m, n);
    if (s != EM_OK) return s;
    forward(m, X, n, m->stream);
    MCHK(m, hipGetLastError());
    MCHK(m, hipMemcpyAsync(y, m->y, sizeof(float) * n, hipMemcpyDeviceToDevice, m->stream));
    MCHK(m, hipStreamSynchronize(m->stream));
    return EM_OK;
}

em_status em_mlp_grad(em_mlp *m, const float *X, const float *t, int32_t n, float *grad_host, float *loss)
{
    if (!m || !X || !t || n <= 0) return mfail(m, EM_ERR_ARG, "bad gradient arguments");
    em_status s = ensure_rows(m, n);
    if (s != EM_OK) return s;
    forward(m, X, n, m->stream);
    s = backward(m, t, n, loss);
    if (s != EM_OK) return s;
    if (grad_host) {
        MCHK(m, hipMemcpyAsync(grad_host, m->g, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, m->stream));
        MCHK(m, hipStreamSynchronize(m->stream));
    }
    return EM_OK;
}

em_status em_mlp_train_step(em_mlp *m, const float *X, const float *t, int32_t n, float lr, float *loss)
{
    if (!m || !X || !t || n <= 0 || !(lr > 0)) return mfail(m, EM_ERR_ARG, "bad training arguments");
    em_status s = ensure_rows(m, n);
    if (s != EM_OK) return s;
    forward(m, X, n, m->stream);
    s = backward(m, t, n, loss);
    if (s != EM_OK) return s;
    m->t += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, (float)m->t), c2 = 1.0f - powf(b2, (float)m->t);
    k_adam<<<cdiv(NPARAM, 256), 256, 0, m->stream>>>(m->p, m->g, m->m, m->v, NPARAM, lr, b1, b2, eps, c1, c2);
    MCHK(m, hipGetLastError());
    return EM_OK;
}

}  // extern "C"
