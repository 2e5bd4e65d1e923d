// lb_mlp: the restoring-force surrogate's forward, backward and Adam kernels for gfx950, and the
// C ABI declared in include/lb_mlp.h.
//
// Products run on the matrix cores: v_mfma_f32_16x16x16_bf16 with BF16 operands rounded (nearest
// even) from FP32 while a 64x64 output tile's operands are staged through LDS, FP32 accumulation,
// and fused epilogues (bias, tanh, tanh derivative).  Master weights, gradients and Adam moments
// are FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "lb.h"
#include "lb_launch.h"
#include "lb_mlp.h"

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_rne(float x) {
    unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (short)(u >> 16);   // inf / nan kept
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

enum Epi { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_TANH = 2, EPI_TANH_GRAD = 3 };

constexpr int TM = 64, TN = 64, TK = 16;

// D(m, n) = epilogue( sum_k A(m, k) B(k, n) ) with A(m, k) = A[m*sam + k*sak] and
// B(k, n) = B[k*sbk + n*sbn] (strides express transposes).  Epilogues: + bias[n]; tanh(+ bias);
// times (1 - aux(m, n)^2) with aux row-major M x N (the tanh derivative from stored activations).
// Block: 256 threads = 4 waves, 64x64 tile; each wave owns 32x32 = 2x2 MFMA tiles of 16x16.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(const float *__restrict__ A, long sam, long sak, const float *__restrict__ B,
                                              long sbk, long sbn, float *__restrict__ D, int M, int N, int K,
                                              const float *__restrict__ bias, const float *__restrict__ aux) {
    __shared__ short As[TM][TK + 4];
    __shared__ short Bs[TK][TN + 4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += TK) {
        // stage 64x16 of A and 16x64 of B as BF16 (4 elements per thread each), zero outside
        for (int e = tid; e < TM * TK; e += 256) {
            int mm = e / TK, kk = e % TK;
            int m = m0 + mm, k = k0 + kk;
            float v = (m < M && k < K) ? A[(long)m * sam + (long)k * sak] : 0.f;
            As[mm][kk] = bf16_rne(v);
        }
        for (int e = tid; e < TK * TN; e += 256) {
            int kk = e / TN, nn = e % TN;
            int k = k0 + kk, n = n0 + nn;
            float v = (k < K && n < N) ? B[(long)k * sbk + (long)n * sbn] : 0.f;
            Bs[kk][nn] = bf16_rne(v);
        }
        __syncthreads();
        // operand layout of the 16x16x16 BF16 MFMA: lane l holds A(l%16, 4*(l/16)+0..3) and
        // B(4*(l/16)+0..3, l%16)
        const int r = lane & 15, kq = (lane >> 4) * 4;
        bf16x4 a[2], b[2];
        for (int i = 0; i < 2; ++i) {
            const short *ap = &As[wm + 16 * i + r][kq];
            a[i] = bf16x4{ap[0], ap[1], ap[2], ap[3]};
        }
        for (int j = 0; j < 2; ++j) {
            const int c = wn + 16 * j + r;
            b[j] = bf16x4{Bs[kq][c], Bs[kq + 1][c], Bs[kq + 2][c], Bs[kq + 3][c]};
        }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // result layout: lane l holds D(4*(l/16)+q, l%16), q = 0..3
    const int c = lane & 15, rq = (lane >> 4) * 4;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn + 16 * j + c;
            if (n >= N) continue;
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + wm + 16 * i + rq + q;
                if (m >= M) continue;
                float v = acc[i][j][q];
                if (EPI == EPI_BIAS || EPI == EPI_BIAS_TANH) v += bias[n];
                if (EPI == EPI_BIAS_TANH) v = tanhf(v);
                if (EPI == EPI_TANH_GRAD) {
                    const float a = aux[(long)m * N + n];
                    v *= 1.0f - a * a;
                }
                D[(long)m * N + n] = v;
            }
        }
}

// db[n] = sum over rows of dZ(m, n); one block per 64 columns, fixed summation order
// zero n bytes (n a multiple of 4, 4-byte aligned): a kernel rather than a memset node, so a caller
// may capture the calls that clear state into a graph
__global__ __launch_bounds__(256) void k_zero(unsigned *__restrict__ p, size_t n_words) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n_words; i += (size_t)gridDim.x * 256) p[i] = 0u;
}

static hipError_t zero_async(void *p, size_t bytes, hipStream_t st) {
    const size_t words = bytes / 4;
    if (words == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 4096);
    k_zero<<<blocks, 256, 0, st>>>(static_cast<unsigned *>(p), words);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_colsum(const float *__restrict__ dZ, int M, int N, float *__restrict__ db) {
    __shared__ float part[4][64];
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    float s = 0.f;
    if (n < N)
        for (int m = g; m < M; m += 4) s += dZ[(long)m * N + n];
    part[g][c] = s;
    __syncthreads();
    if (g == 0 && n < N) db[n] = (part[0][c] + part[1][c]) + (part[2][c] + part[3][c]);
}

// per row i: r_i = |yhat_i - y_i|^2 / |y_i|^2; dYhat = 2 (yhat - y) / (|y|^2 batch); row loss out
__global__ __launch_bounds__(64) void k_rel_loss(const float *__restrict__ Yh, const float *__restrict__ Y, int B, int N,
                                                 float *__restrict__ dY, float *__restrict__ row_loss) {
    const int i = blockIdx.x, l = threadIdx.x;
    float e2 = 0.f, y2 = 0.f;
    for (int n = l; n < N; n += 64) {
        float d = Yh[(long)i * N + n] - Y[(long)i * N + n];
        float y = Y[(long)i * N + n];
        e2 += d * d;
        y2 += y * y;
    }
    for (int o = 32; o > 0; o >>= 1) {
        e2 += __shfl_xor(e2, o);
        y2 += __shfl_xor(y2, o);
    }
    const float inv = 1.0f / fmaxf(y2, 1e-30f);
    for (int n = l; n < N; n += 64)
        dY[(long)i * N + n] = 2.0f * (Yh[(long)i * N + n] - Y[(long)i * N + n]) * inv / (float)B;
    if (l == 0) row_loss[i] = e2 * inv;
}

__global__ __launch_bounds__(256) void k_mean(const float *__restrict__ v, int n, float *__restrict__ out) {
    __shared__ float part[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += v[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0] / (float)n;
}

__global__ __launch_bounds__(256) void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
                                              float *__restrict__ m2, long n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
    long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float a = b1 * m1[i] + (1.0f - b1) * gi;
    float b = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    p[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    lbk::set_last_error(buf);
    return code;
}
#define HIPCHK(expr)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return fail(LB_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct Layout {
    int L = 0;
    std::vector<int> w;
    std::vector<size_t> oW, oB;   // offsets (floats) of W_l and b_l in the parameter array
    size_t n_params = 0, acts = 0;
    size_t bytes = 0, oP = 0, oG = 0, oM1 = 0, oM2 = 0, oAct = 0, oGrad = 0, oRow = 0, oLoss = 0;
};

int layout(const lb_mlp_config *c, Layout &lo) {
    if (!c) return fail(LB_EINVAL, "config is NULL");
    if (c->n_layers < 1 || c->n_layers > 8) return fail(LB_EINVAL, "n_layers must be 1..8");
    if (c->max_batch < 1 || c->max_batch > (1 << 20)) return fail(LB_EINVAL, "max_batch out of range");
    lo.L = c->n_layers;
    lo.w.assign(c->widths, c->widths + c->n_layers + 1);
    for (int x : lo.w)
        if (x < 1 || x > 4096) return fail(LB_EINVAL, "layer widths must be 1..4096");
    size_t off = 0, acts = 0;
    for (int l = 0; l < lo.L; ++l) {
        lo.oW.push_back(off);
        off += (size_t)lo.w[l + 1] * lo.w[l];
        lo.oB.push_back(off);
        off += (size_t)lo.w[l + 1];
        acts += (size_t)lo.w[l + 1];
    }
    lo.n_params = off;
    lo.acts = acts;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t o = 0;
    lo.oP = o;  o += al(4 * off);
    lo.oG = o;  o += al(4 * off);
    lo.oM1 = o; o += al(4 * off);
    lo.oM2 = o; o += al(4 * off);
    lo.oAct = o; o += al(4 * acts * (size_t)c->max_batch);           // activations of every layer
    size_t wmax = *std::max_element(lo.w.begin(), lo.w.end());
    lo.oGrad = o; o += al(4 * 2 * wmax * (size_t)c->max_batch);      // two gradient buffers
    lo.oRow = o; o += al(4 * (size_t)c->max_batch);
    lo.oLoss = o; o += al(4);
    lo.bytes = o + 256;
    return LB_OK;
}

}  // namespace

struct lb_mlp {
    lb_mlp_config cfg;
    Layout lo;
    char *base = nullptr;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    long step = 0;
    // waits for the stream and releases it if the library created it (also when lb_mlp_create
    // fails part way); the arena belongs to the caller
    ~lb_mlp() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
    float *P() { return reinterpret_cast<float *>(base + lo.oP); }
    float *G() { return reinterpret_cast<float *>(base + lo.oG); }
    float *M1() { return reinterpret_cast<float *>(base + lo.oM1); }
    float *M2() { return reinterpret_cast<float *>(base + lo.oM2); }
    float *act(int l) {   // output of layer l (batch x w[l+1]) at max_batch stride
        size_t off = 0;
        for (int i = 0; i < l; ++i) off += (size_t)lo.w[i + 1];
        return reinterpret_cast<float *>(base + lo.oAct) + off * (size_t)cfg.max_batch;
    }
    float *grad(int i) {
        size_t wmax = *std::max_element(lo.w.begin(), lo.w.end());
        return reinterpret_cast<float *>(base + lo.oGrad) + (size_t)i * wmax * cfg.max_batch;
    }
    float *rows() { return reinterpret_cast<float *>(base + lo.oRow); }
    float *loss() { return reinterpret_cast<float *>(base + lo.oLoss); }
};

namespace {

hipError_t gemm(int epi, const float *A, long sam, long sak, const float *B, long sbk, long sbn, float *D, int M, int N,
                int K, const float *bias, const float *aux, hipStream_t st) {
    dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM);
    switch (epi) {
    case EPI_STORE: k_gemm<EPI_STORE><<<grid, 256, 0, st>>>(A, sam, sak, B, sbk, sbn, D, M, N, K, bias, aux); break;
    case EPI_BIAS: k_gemm<EPI_BIAS><<<grid, 256, 0, st>>>(A, sam, sak, B, sbk, sbn, D, M, N, K, bias, aux); break;
    case EPI_BIAS_TANH: k_gemm<EPI_BIAS_TANH><<<grid, 256, 0, st>>>(A, sam, sak, B, sbk, sbn, D, M, N, K, bias, aux); break;
    default: k_gemm<EPI_TANH_GRAD><<<grid, 256, 0, st>>>(A, sam, sak, B, sbk, sbn, D, M, N, K, bias, aux); break;
    }
    return hipGetLastError();
}

// ---- forward pass without allocation ------------------------------------------------------
// The hidden activations of lb_mlp_forward_noalloc live in this file-scope device array, two
// ping-pong halves of kScratchFloats / 2 floats.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol): each device's copy is looked up once
// with hipGetSymbolAddress and its address kept per device.
constexpr size_t kScratchFloats = size_t(1) << 20;   // 4 MiB per GPU, held until the process ends
constexpr int kMaxDevices = 64;
__device__ __align__(256) float scratch[kScratchFloats];
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};

int scratch_on_current_device(float **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LB_EINVAL, "device index %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(LB_EDEVICE, "no device address for the scratch array");
        g_scratch_ptr[dev] = static_cast<float *>(p);
    }
    *out = g_scratch_ptr[dev];
    return LB_OK;
}

// forward into the activation buffers; returns the output pointer (batch x w[L])
int forward(lb_mlp *m, const float *X, int B) {
    const Layout &lo = m->lo;
    const float *in = X;
    for (int l = 0; l < lo.L; ++l) {
        const int K = lo.w[l], N = lo.w[l + 1];
        const float *W = m->P() + lo.oW[l], *b = m->P() + lo.oB[l];
        // Z = A_prev W^T + b: A_prev(m, k) = in[m*K + k], B(k, n) = W[n*K + k]
        HIPCHK(gemm(l + 1 < lo.L ? EPI_BIAS_TANH : EPI_BIAS, in, K, 1, W, 1, K, m->act(l), B, N, K, b, nullptr, m->stream));
        in = m->act(l);
    }
    return LB_OK;
}

// gradients of the mean squared relative error into G(); loss of the batch into loss()
int backward(lb_mlp *m, const float *X, const float *Y, int B) {
    const Layout &lo = m->lo;
    const int L = lo.L, NL = lo.w[L];
    float *dA = m->grad(0), *dZ = m->grad(1);
    k_rel_loss<<<B, 64, 0, m->stream>>>(m->act(L - 1), Y, B, NL, dZ, m->rows());
    HIPCHK(hipGetLastError());
    k_mean<<<1, 256, 0, m->stream>>>(m->rows(), B, m->loss());
    HIPCHK(hipGetLastError());
    for (int l = L - 1; l >= 0; --l) {
        const int K = lo.w[l], N = lo.w[l + 1];
        const float *Aprev = l > 0 ? m->act(l - 1) : X;
        float *gW = m->G() + lo.oW[l], *gb = m->G() + lo.oB[l];
        // dW = dZ^T A_prev: A(m=n_out, k=row) = dZ[row*N + n_out], B(k=row, n=in) = Aprev[row*K + in]
        HIPCHK(gemm(EPI_STORE, dZ, 1, N, Aprev, K, 1, gW, N, K, B, nullptr, nullptr, m->stream));
        k_colsum<<<(N + 63) / 64, 256, 0, m->stream>>>(dZ, B, N, gb);
        HIPCHK(hipGetLastError());
        if (l > 0) {
            // dZ_prev = (dZ W) * (1 - A_prev^2): A(m=row, k=out) = dZ[row*N + out], B(k=out, n=in) = W[out*K + in]
            const float *W = m->P() + lo.oW[l];
            HIPCHK(gemm(EPI_TANH_GRAD, dZ, N, 1, W, K, 1, dA, B, K, N, nullptr, Aprev, m->stream));
            std::swap(dA, dZ);
        }
    }
    return LB_OK;
}

}  // namespace

extern "C" {

int lb_mlp_query_bytes(const lb_mlp_config *cfg, size_t *bytes) {
    if (!bytes) return fail(LB_EINVAL, "bytes is NULL");
    Layout lo;
    int rc = layout(cfg, lo);
    if (rc) return rc;
    *bytes = lo.bytes;
    return LB_OK;
}

int lb_mlp_n_params(const lb_mlp_config *cfg, size_t *n) {
    if (!n) return fail(LB_EINVAL, "n is NULL");
    Layout lo;
    int rc = layout(cfg, lo);
    if (rc) return rc;
    *n = lo.n_params;
    return LB_OK;
}

int lb_mlp_create(const lb_mlp_config *cfg, void *arena, size_t arena_bytes, void *stream, lb_mlp **out) {
    if (!out || !arena) return fail(LB_EINVAL, "NULL argument");
    if ((uintptr_t)arena & 255) return fail(LB_EINVAL, "arena must be 256-byte aligned");
    try {
        std::unique_ptr<lb_mlp> m(new lb_mlp());
        int rc = layout(cfg, m->lo);
        if (rc) return rc;
        if (arena_bytes < m->lo.bytes) return fail(LB_ENOMEM, "arena too small: %zu < %zu", arena_bytes, m->lo.bytes);
        m->cfg = *cfg;
        if (m->cfg.beta1 == 0.f) m->cfg.beta1 = 0.9f;
        if (m->cfg.beta2 == 0.f) m->cfg.beta2 = 0.999f;
        if (m->cfg.eps == 0.f) m->cfg.eps = 1e-8f;
        m->base = static_cast<char *>(arena);
        if (stream) {
            m->stream = static_cast<hipStream_t>(stream);
        } else {
            HIPCHK(hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking));
            m->own_stream = true;
        }
        HIPCHK(zero_async(m->base, m->lo.oAct, m->stream));
        HIPCHK(hipStreamSynchronize(m->stream));
        *out = m.release();
        return LB_OK;
    } catch (...) {
        return fail(LB_ENOMEM, "host allocation failed");
    }
}

int lb_mlp_set_params(lb_mlp *m, const float *host) {
    if (!m || !host) return fail(LB_EINVAL, "NULL argument");
    HIPCHK(hipMemcpyAsync(m->P(), host, 4 * m->lo.n_params, hipMemcpyHostToDevice, m->stream));
    HIPCHK(zero_async(m->M1(), 4 * m->lo.n_params, m->stream));
    HIPCHK(zero_async(m->M2(), 4 * m->lo.n_params, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    m->step = 0;
    return LB_OK;
}

int lb_mlp_get_params(lb_mlp *m, float *host) {
    if (!m || !host) return fail(LB_EINVAL, "NULL argument");
    HIPCHK(hipMemcpyAsync(host, m->P(), 4 * m->lo.n_params, hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    return LB_OK;
}

int lb_mlp_forward(lb_mlp *m, const float *X, int32_t batch, float *Y) {
    if (!m || !X || !Y) return fail(LB_EINVAL, "NULL argument");
    if (batch < 1 || batch > m->cfg.max_batch) return fail(LB_ERANGE, "batch out of range");
    int rc = forward(m, X, batch);
    if (rc) return rc;
    const int NL = m->lo.w[m->lo.L];
    HIPCHK(hipMemcpyAsync(Y, m->act(m->lo.L - 1), 4 * (size_t)batch * NL, hipMemcpyDeviceToDevice, m->stream));
    return LB_OK;
}

int lb_mlp_gradients(lb_mlp *m, const float *X, const float *Y, int32_t batch, float *host_loss, float *host_grads) {
    if (!m || !X || !Y) return fail(LB_EINVAL, "NULL argument");
    if (batch < 1 || batch > m->cfg.max_batch) return fail(LB_ERANGE, "batch out of range");
    int rc = forward(m, X, batch);
    if (rc) return rc;
    rc = backward(m, X, Y, batch);
    if (rc) return rc;
    if (host_loss) HIPCHK(hipMemcpyAsync(host_loss, m->loss(), 4, hipMemcpyDeviceToHost, m->stream));
    if (host_grads) HIPCHK(hipMemcpyAsync(host_grads, m->G(), 4 * m->lo.n_params, hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    return LB_OK;
}

int lb_mlp_train_step(lb_mlp *m, const float *X, const float *Y, int32_t batch, float lr, float *device_loss) {
    if (!m || !X || !Y) return fail(LB_EINVAL, "NULL argument");
    if (batch < 1 || batch > m->cfg.max_batch) return fail(LB_ERANGE, "batch out of range");
    int rc = forward(m, X, batch);
    if (rc) return rc;
    rc = backward(m, X, Y, batch);
    if (rc) return rc;
    m->step += 1;
    const float c1 = 1.0f - std::pow(m->cfg.beta1, (float)m->step);
    const float c2 = 1.0f - std::pow(m->cfg.beta2, (float)m->step);
    const long n = (long)m->lo.n_params;
    k_adam<<<(unsigned)((n + 255) / 256), 256, 0, m->stream>>>(m->P(), m->G(), m->M1(), m->M2(), n, lr, m->cfg.beta1,
                                                               m->cfg.beta2, m->cfg.eps, c1, c2);
    HIPCHK(hipGetLastError());
    if (device_loss) HIPCHK(hipMemcpyAsync(device_loss, m->loss(), 4, hipMemcpyDeviceToDevice, m->stream));
    return LB_OK;
}

int lb_mlp_destroy(lb_mlp *m) {
    if (!m) return fail(LB_EINVAL, "NULL argument");
    delete m;
    return LB_OK;
}

int lb_mlp_forward_noalloc(const lb_mlp_config *cfg, const float *params, const float *X, int32_t batch, float *Y,
                           void *hip_stream) {
    if (!cfg || !params || !X || !Y) return fail(LB_EINVAL, "NULL argument");
    const int L = cfg->n_layers;
    if (L < 1 || L > 8) return fail(LB_EINVAL, "n_layers must be 1..8");
    int wmax_hidden = 0;
    for (int l = 0; l <= L; ++l) {
        if (cfg->widths[l] < 1 || cfg->widths[l] > 4096) return fail(LB_EINVAL, "layer widths must be 1..4096");
        if (l > 0 && l < L) wmax_hidden = std::max(wmax_hidden, cfg->widths[l]);
    }
    if (batch < 1) return fail(LB_ERANGE, "batch must be positive");
    if ((size_t)batch * (size_t)wmax_hidden > kScratchFloats / 2)
        return fail(LB_ERANGE, "batch %d x hidden width %d exceeds the scratch limit of %zu values", batch, wmax_hidden,
                    kScratchFloats / 2);
    float *buf = nullptr;
    int rc = scratch_on_current_device(&buf);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const float *in = X;
    size_t off = 0;   // parameter offset of W_l
    for (int l = 0; l < L; ++l) {
        const int K = cfg->widths[l], N = cfg->widths[l + 1];
        const float *W = params + off, *b = params + off + (size_t)N * K;
        off += (size_t)N * K + N;
        float *out = l + 1 < L ? buf + (size_t)(l & 1) * (kScratchFloats / 2) : Y;
        HIPCHK(gemm(l + 1 < L ? EPI_BIAS_TANH : EPI_BIAS, in, K, 1, W, 1, K, out, batch, N, K, b, nullptr, st));
        in = out;
    }
    return LB_OK;
}

int lb_mlp_gemm_bf16(const float *A, const float *B, float *D, int32_t M, int32_t N, int32_t K, void *stream) {
    if (!A || !B || !D) return fail(LB_EINVAL, "NULL argument");
    if (M < 1 || N < 1 || K < 1) return fail(LB_EINVAL, "sizes must be positive");
    HIPCHK(gemm(EPI_STORE, A, K, 1, B, N, 1, D, M, N, K, nullptr, nullptr, static_cast<hipStream_t>(stream)));
    return LB_OK;
}

}  // extern "C"
