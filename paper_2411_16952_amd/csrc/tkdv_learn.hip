// Learned proposal: the network that maps (beta', E0, C3/C2) to the mixture
// of a point, and its training on the GPU (FP64 throughout).
//
// One training step (all on one stream):
//   k_mlp_fwd       per point: z -> h1 -> h2 -> o (tanh layers)
//   k_mix_prep      per point: o -> log d, V; A = D^-1, G^-1, log|L0| and
//                   the gradient of log|L0|
//   k_mix_fwd_mm    per chunk of rows: the y products of all S shifts on the
//                   FP64 matrix cores, log q_net and log q_mix
//   k_loss_max      per point maximum of r_s = log f - log q_mix
//   k_loss_chunk    per chunk of a point's rows: sum of exp(r_s/T - max), NLL
//   k_loss_final    per point: chunk partials in order -> soft maximum, loss
//   k_mix_bwd_mm    per chunk: dL/d(log d, V) of the point from a second
//                   product X^T C and per-mode rotations
//   k_param_grad    per point: chunk partials in order, the log|L0| term,
//                   dL/do
//   k_mlp_bwd_*     back through the layers; dL/dweights summed over points
//   k_adam          the update
// Rows are grouped by point (an index order) and cut into chunks of at most
// kChunk rows of one point; every sum runs in a fixed order, so a step is
// deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/tkdv.h"
#include "tkdv_device.h"
#include "tkdv_internal.h"
#include "tkdv_kernels.h"
#include "tkdv_runtime.h"

namespace tkdv {

constexpr int kLKMax = 32;        // largest K of the learned proposal
constexpr int kMaxHidden = 256;
constexpr int kChunk = 32;        // rows per chunk of the reductions

struct LearnPoint {
    double z[3];
    double logs2[kLKMax];  // log s_k^2 of the Sigma plan
    double E0, beta_p, c32;
    double lng, gc;        // sum_k ln(1 + gc k^2), gc = alpha beta'/K^3
    double inv_n_acc;      // 1 / (accepted rows of the point), 0 if none
    uint32_t chunk0, chunk1;  // the point's chunks [chunk0, chunk1)
};

constexpr int kMixCols = 2 * kMixS;  // columns (shift j, q) -> 2 j + q of the y products

struct LearnParam {
    double logd[kLKMax], a[kLKMax];
    double V[2 * kLKMax][2];
    double gi[2][2];
    double logdet;
    double dld_logd[kLKMax];   // d log|L0| / d log d_k
    double dld_V[2 * kLKMax][2];
    // y_j = V^T A R_j^T x = B_j^T x for every shift at once: B[n][2 j + q] = (R_j A V)_nq
    double B[2 * kLKMax][kMixCols];
};

__constant__ double c_cs[kMixS], c_sn[kMixS];

struct LearnStats {
    unsigned long long maxkey;  // order-preserving key of max_s r_s/T
    double sum;                 // sum_s exp(r_s/T - max)
    double nll;                 // sum over accepted rows of -log q_net
    double loss;
};

// Partials of one chunk: [sum, nll, csum, gd (K), gv (2K x 2)], csum = sum of
// c_s = dL/d log q_net(x_s), gd/gv = sum of c_s d log q_net/d(log d, V)
// without the log|L0| term.
constexpr int chunk_part_len(int K) { return 3 + 5 * K; }

struct LearnArgs {
    const double *X;         // rows [n][2K]
    const int *row_point;    // [n]
    const uint8_t *kind;     // [n]
    const double *lf;        // log f of the rows
    double *lnet, *lmix;     // [n]
    unsigned long long n;
    const LearnPoint *pts;
    const LearnParam *par;
    LearnStats *st;
    const uint32_t *order;        // row indices grouped by point
    const uint32_t *chunk_start;  // [n_chunks + 1] offsets into order
    const int *chunk_point;       // [n_chunks]
    unsigned n_chunks;
    double *part;                 // [n_chunks][pt_len]
    int pt_len;                   // 3 + 5K
    double T, lambda, log_eps, log_1m_eps;
};

__device__ __forceinline__ unsigned long long dkey(double d)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double dkey_inv(unsigned long long k)
{
    const unsigned long long b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    return __longlong_as_double((long long)b);
}
__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Network
// ---------------------------------------------------------------------------
struct MlpView {
    const double *W1, *b1, *W2, *b2, *W3, *b3;
    __host__ __device__ MlpView(const double *W, int H, int n_out)
        : W1(W), b1(W + 3 * H), W2(W + 4 * H), b2(W + 4 * H + H * H), W3(W + 5 * H + H * H),
          b3(W + 5 * H + H * H + H * n_out) {}
};
inline int64_t mlp_n_weights(int H, int n_out) { return 5ll * H + (int64_t)H * H + (int64_t)H * n_out + n_out; }

__global__ void __launch_bounds__(kMaxHidden) k_mlp_fwd(const double *W, int H, int n_out, const double *z,
                                                        double *h1, double *h2, double *out)
{
    __shared__ double s1[kMaxHidden], s2[kMaxHidden];
    const int p = blockIdx.x, i = threadIdx.x;
    const MlpView w(W, H, n_out);
    const double *zp = z + 3 * p;
    if (i < H) {
        const double a = w.b1[i] + w.W1[i] * zp[0] + w.W1[H + i] * zp[1] + w.W1[2 * H + i] * zp[2];
        s1[i] = tanh(a);
        h1[(size_t)p * H + i] = s1[i];
    }
    __syncthreads();
    if (i < H) {
        double a = w.b2[i];
        for (int j = 0; j < H; ++j) a += w.W2[(size_t)j * H + i] * s1[j];
        s2[i] = tanh(a);
        h2[(size_t)p * H + i] = s2[i];
    }
    __syncthreads();
    for (int o = i; o < n_out; o += blockDim.x) {
        double a = w.b3[o];
        for (int j = 0; j < H; ++j) a += w.W3[(size_t)j * n_out + o] * s2[j];
        out[(size_t)p * n_out + o] = a;
    }
}

// dh2 = (W3 dout) * (1 - h2^2), dh1 = (W2 dh2) * (1 - h1^2), per point.
__global__ void __launch_bounds__(kMaxHidden) k_mlp_bwd_hidden(const double *W, int H, int n_out,
                                                               const double *h1, const double *h2,
                                                               const double *dout, double *dh1, double *dh2)
{
    __shared__ double s2[kMaxHidden];
    const int p = blockIdx.x, j = threadIdx.x;
    const MlpView w(W, H, n_out);
    if (j < H) {
        double a = 0.0;
        for (int o = 0; o < n_out; ++o) a += w.W3[(size_t)j * n_out + o] * dout[(size_t)p * n_out + o];
        const double h = h2[(size_t)p * H + j];
        s2[j] = a * (1.0 - h * h);
        dh2[(size_t)p * H + j] = s2[j];
    }
    __syncthreads();
    if (j < H) {
        double a = 0.0;
        for (int k = 0; k < H; ++k) a += w.W2[(size_t)j * H + k] * s2[k];
        const double h = h1[(size_t)p * H + j];
        dh1[(size_t)p * H + j] = a * (1.0 - h * h);
    }
}

// dL/dweights = sum over points of the outer products (one thread per weight).
__global__ void k_mlp_bwd_weights(int H, int n_out, int n_points, const double *z, const double *h1,
                                  const double *h2, const double *dh1, const double *dh2, const double *dout,
                                  double *gW)
{
    const long long nW = 5ll * H + (long long)H * H + (long long)H * n_out + n_out;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < nW;
         idx += (long long)gridDim.x * blockDim.x) {
        double g = 0.0;
        long long r = idx;
        if (r < 3ll * H) {  // W1[c][i]
            const int c = (int)(r / H), i = (int)(r % H);
            for (int p = 0; p < n_points; ++p) g += z[3 * p + c] * dh1[(size_t)p * H + i];
        } else if ((r -= 3ll * H) < H) {  // b1
            for (int p = 0; p < n_points; ++p) g += dh1[(size_t)p * H + r];
        } else if ((r -= H) < (long long)H * H) {  // W2[j][i]
            const int j = (int)(r / H), i = (int)(r % H);
            for (int p = 0; p < n_points; ++p) g += h1[(size_t)p * H + j] * dh2[(size_t)p * H + i];
        } else if ((r -= (long long)H * H) < H) {  // b2
            for (int p = 0; p < n_points; ++p) g += dh2[(size_t)p * H + r];
        } else if ((r -= H) < (long long)H * n_out) {  // W3[j][o]
            const int j = (int)(r / n_out), o = (int)(r % n_out);
            for (int p = 0; p < n_points; ++p) g += h2[(size_t)p * H + j] * dout[(size_t)p * n_out + o];
        } else {  // b3
            r -= (long long)H * n_out;
            for (int p = 0; p < n_points; ++p) g += dout[(size_t)p * n_out + r];
        }
        gW[idx] = g;
    }
}

__global__ void k_adam(double *W, const double *gW, double *m1, double *m2, long long n, double lr, double b1,
                       double b2, double eps, double c1, double c2)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const double g = gW[i];
        const double a = b1 * m1[i] + (1.0 - b1) * g;
        const double b = b2 * m2[i] + (1.0 - b2) * g * g;
        m1[i] = a;
        m2[i] = b;
        W[i] -= lr * (a / c1) / (sqrt(b / c2) + eps);
    }
}

// ---------------------------------------------------------------------------
// Mixture parameters of each point from the network output (one wave per point)
// ---------------------------------------------------------------------------
template <int K>
__global__ void __launch_bounds__(64) k_mix_prep(const double *out, int n_out, const LearnPoint *pts,
                                                 LearnParam *par, double v_amp, double v_scale)
{
    const int p = blockIdx.x, m = threadIdx.x;
    const LearnPoint &L = pts[p];
    LearnParam &Q = par[p];
    const double *o = out + (size_t)p * n_out;
    const bool act = m < 2 * K;
    const int k = m % K;
    const double logd = act ? L.logs2[k] + o[k] : 0.0;
    const double a = act ? exp(-logd) : 0.0;
    const double v00 = v_amp / sqrt((double)K);
    double V0 = 0.0, V1 = 0.0;
    if (act) {
        V0 = (m < K ? v00 : 0.0) + v_scale * o[K + 2 * m];
        V1 = (m >= K ? v00 : 0.0) + v_scale * o[K + 2 * m + 1];
        Q.V[m][0] = V0;
        Q.V[m][1] = V1;
    }
    if (m < K) {
        Q.logd[m] = logd;
        Q.a[m] = a;
    }
    const double G00 = 1.0 + wsum(a * V0 * V0), G01 = wsum(a * V0 * V1), G11 = 1.0 + wsum(a * V1 * V1);
    const double det = G00 * G11 - G01 * G01;
    const double i00 = G11 / det, i01 = -G01 / det, i11 = G00 / det;
    const double ldD = wsum(m < K ? 2.0 * logd : 0.0);
    // V_m G^-1
    const double u0 = V0 * i00 + V1 * i01, u1 = V0 * i01 + V1 * i11;
    if (act) {
        Q.dld_V[m][0] = 2.0 * a * u0;
        Q.dld_V[m][1] = 2.0 * a * u1;
    }
    // d log|L0| / d log d_k = sum over the mode's two coordinates of 1 - a_m V_m G^-1 V_m^T
    const double own = act ? 1.0 - a * (u0 * V0 + u1 * V1) : 0.0;
    const double partner = __shfl(own, (m + K) & 63, 64);
    if (m < K) Q.dld_logd[m] = own + partner;
    // the y-product matrix: coordinate n of x enters w = R_j^T x at n (cos c) and at
    // its partner n +- K (sin s): B[n][2j + q] = a (c V_nq +- s V_{n -+ K, q})
    const int src = act ? (m < K ? m + K : m - K) : m;
    const double P0 = __shfl(V0, src, 64), P1 = __shfl(V1, src, 64);
    if (act) {
        const double sg = m < K ? 1.0 : -1.0;
        for (int j = 0; j < kMixS; ++j) {
            const int mi = ((k + 1) * j) & (kMixS - 1);
            const double c = c_cs[mi], sn = sg * c_sn[mi];
            Q.B[m][2 * j] = a * (c * V0 + sn * P0);
            Q.B[m][2 * j + 1] = a * (c * V1 + sn * P1);
        }
    }
    if (m == 0) {
        Q.gi[0][0] = i00;
        Q.gi[0][1] = i01;
        Q.gi[1][0] = i01;
        Q.gi[1][1] = i11;
        Q.logdet = ldD + log(det);
    }
}

// log f of the training rows (thread per row).
template <int K>
__global__ void k_rows_log_f(const double *X, const int *row_point, const LearnPoint *pts, double *lf,
                             unsigned long long r0, unsigned long long n)
{
    for (unsigned long long r = r0 + (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; r < r0 + n;
         r += (unsigned long long)gridDim.x * blockDim.x) {
        const LearnPoint &L = pts[row_point[r]];
        double x[2 * K];
        double t = 0.0;
        for (int m = 0; m < 2 * K; ++m) x[m] = X[r * 2 * K + m];
        for (int k = 1; k <= K; ++k) t += (double)k * k * (x[k - 1] * x[k - 1] + x[K + k - 1] * x[K + k - 1]);
        lf[r] = log_f_fp64(K, L.E0, L.beta_p, L.c32, x, t);
    }
}

// FP32 rows (row stride in floats) -> FP64 unit rows appended at r0.
template <int K>
__global__ void k_rows_append(const float *src, unsigned long long stride, unsigned long long n, double *X,
                              int *row_point, uint8_t *kind, unsigned long long r0, int point, int kd)
{
    for (unsigned long long r = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (unsigned long long)gridDim.x * blockDim.x) {
        double x[2 * K], r2 = 0.0;
        for (int m = 0; m < 2 * K; ++m) {
            x[m] = (double)src[r * stride + m];
            r2 += x[m] * x[m];
        }
        const double inv = 1.0 / sqrt(r2);
        for (int m = 0; m < 2 * K; ++m) X[(r0 + r) * 2 * K + m] = x[m] * inv;
        row_point[r0 + r] = point;
        kind[r0 + r] = (uint8_t)kd;
    }
}

__global__ void k_loss_max(LearnArgs A)
{
    for (unsigned long long r = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; r < A.n;
         r += (unsigned long long)gridDim.x * blockDim.x)
        if (A.kind[r] != 2)  // kind 2: likelihood term only
            atomicMax(&A.st[A.row_point[r]].maxkey, dkey((A.lf[r] - A.lmix[r]) / A.T));
}

// Sum of exp(r_s/T - max) and of -log q_net over the accepted rows, per chunk
// (one wave; lane-strided then a fixed butterfly).
__global__ void __launch_bounds__(256) k_loss_chunk(LearnArgs A)
{
    const int m = threadIdx.x & 63;
    const unsigned c = __builtin_amdgcn_readfirstlane((blockIdx.x * 256 + threadIdx.x) >> 6);
    if (c >= A.n_chunks) return;
    const int p = A.chunk_point[c];
    const double mx = dkey_inv(A.st[p].maxkey);
    double se = 0.0, nll = 0.0;
    for (unsigned q = A.chunk_start[c] + m; q < A.chunk_start[c + 1]; q += 64) {
        const unsigned r = A.order[q];
        const uint8_t kd = A.kind[r];
        se += kd != 2 ? exp((A.lf[r] - A.lmix[r]) / A.T - mx) : 0.0;
        nll += kd != 1 ? -A.lnet[r] : 0.0;
    }
    se = wsum(se);
    nll = wsum(nll);
    if (m == 0) {
        A.part[(size_t)c * A.pt_len + 0] = se;
        A.part[(size_t)c * A.pt_len + 1] = nll;
    }
}

// Per point: chunk partials in chunk order -> soft maximum and loss.
__global__ void k_loss_final(LearnArgs A, int n_points)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_points) return;
    LearnStats &S = A.st[p];
    const LearnPoint &L = A.pts[p];
    double se = 0.0, nll = 0.0;
    for (unsigned c = L.chunk0; c < L.chunk1; ++c) {
        se += A.part[(size_t)c * A.pt_len + 0];
        nll += A.part[(size_t)c * A.pt_len + 1];
    }
    S.sum = se;
    S.nll = nll;
    S.loss = se > 0.0 ? A.T * (dkey_inv(S.maxkey) + log(se)) + A.lambda * nll * L.inv_n_acc
                      : A.lambda * nll * L.inv_n_acc;
}

// ---------------------------------------------------------------------------
// Mixture densities of the rows and their gradients, as products on the FP64
// matrix cores, one wave per chunk (at most 32 rows of one point, two tiles
// of 16 rows).  log q_net = LSE_j(-K ln qf_j) - ln S - log|L0|/2 over the S
// shifts; c_s = dL/d log q_net(x_s) = -w_s rho_s [kinds 0, 1] - lambda/n_acc
// [kinds 0, 2] with w_s = softmax_s(r_s/T), rho_s = (1 - eps) q_net/q_mix.
//   Forward: Y = X B (rows x 64, column 2j + q holds y_jq) by 16x16x4 FP64
//   instructions; qf_j = Q - y_j^T G^-1 y_j with Q = x^T A x (Woodbury; A is
//   constant on each mode pair, so Q does not depend on the shift); l_j =
//   -K ln qf_j and the log-sum-exp over the 32 shifts across lanes.
//   Backward: with f_j = c_s pi_j K/qf_j (pi_j = softmax_j l_j) and
//   g_j = G^-1 y_j, the chunk's sums
//     M = X^T C,  C[s][2j + q] = f_sj g_sjq     (a second product),
//     S = sum_sj f_sj g_sj g_sj^T,  E_m = sum_s (sum_j f_sj) x_sm^2,
//   and P_mq = sum_j (R_j^T M_(j,q))_m give, per coordinate m of mode k,
//     dL/dV_mq  = 2 a_k (P_mq - (V_m S)_q),
//     dL/dlog d_k = a_k sum_{m in k} (E_m - 2 V_m . P_m + V_m S V_m^T)
//   (with e_j = R_j^T x - V g_j, dqf_j/dV_mq = -2 a_k e_jm g_jq and
//   dqf_j/dlog d_k = -sum_{m in k} a_k e_jm^2, expanded over the sums).
// Matrix instruction layout: lane l supplies A[l%16][l/16] and B[l/16][l%16],
// and element v of its result is D[4v + l/16][l%16].  The backward's C is
// formed in the D layout of the first product, which is the B layout of the
// second.
// ---------------------------------------------------------------------------
typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4_t mma_f64(double a, double b, d4_t c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row i of chunk c (rows past the chunk's end repeat its first row; their
// results are not used).
__device__ __forceinline__ unsigned chunk_row(const LearnArgs &A, unsigned c0, unsigned nc, int i)
{
    return A.order[c0 + (i < (int)nc ? i : 0)];
}

// y products of 16 rows (this lane's A-operand row: rowA) into acc[t] (column
// tile t), and the row's Q = x^T A x and t = sum k^2 x_k^2 (lanes l % 16 = i).
template <int K>
__device__ __forceinline__ void mix_products(const LearnArgs &A, const LearnParam &Q, unsigned rowA, int lane,
                                             d4_t (&acc)[4], double &Qr, double &tr)
{
    const int g = lane >> 4, i16 = lane & 15;
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = d4_t{0.0, 0.0, 0.0, 0.0};
    double qa = 0.0, ta = 0.0;
    const double *x = A.X + (size_t)rowA * 2 * K;
#pragma unroll
    for (int s = 0; s < K / 2; ++s) {  // k-steps of 4 coordinates
        const int m = 4 * s + g, k = m % K;
        const double xv = x[m];
        qa += Q.a[k] * xv * xv;
        ta += (double)((k + 1) * (k + 1)) * xv * xv;
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = mma_f64(xv, Q.B[m][16 * t + i16], acc[t]);
    }
    qa += __shfl_xor(qa, 16, 64);
    qa += __shfl_xor(qa, 32, 64);
    ta += __shfl_xor(ta, 16, 64);
    ta += __shfl_xor(ta, 32, 64);
    Qr = qa;
    tr = ta;
}

template <int K>
__global__ void __launch_bounds__(256) k_mix_fwd_mm(LearnArgs A)
{
    const int lane = threadIdx.x & 63, g = lane >> 4, i16 = lane & 15;
    const unsigned c = __builtin_amdgcn_readfirstlane((blockIdx.x * 256 + threadIdx.x) >> 6);
    if (c >= A.n_chunks) return;
    const int p = A.chunk_point[c];
    const LearnPoint &L = A.pts[p];
    const LearnParam &Q = A.par[p];
    const unsigned c0 = A.chunk_start[c], nc = A.chunk_start[c + 1] - c0;
    const double gi00 = Q.gi[0][0], gi01 = Q.gi[0][1], gi11 = Q.gi[1][1];
    const double cst = -log((double)kMixS) - 0.5 * Q.logdet;
    for (int rt = 0; rt * 16 < (int)nc; ++rt) {
        d4_t acc[4];
        double Qa, ta;
        mix_products<K>(A, Q, chunk_row(A, c0, nc, rt * 16 + i16), lane, acc, Qa, ta);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ri = 4 * v + g;  // the tile row of this lane's results
            const double Qr = __shfl(Qa, ri, 64), tr = __shfl(ta, ri, 64);
            double lj[4], mx = -INFINITY;
#pragma unroll
            for (int t = 0; t < 4; ++t) {  // shift j = 8t + i16/2; lanes l, l^1 hold q = 0, 1
                const double y = acc[t][v], yo = __shfl_xor(y, 1, 64);
                const double y0 = (lane & 1) ? yo : y, y1 = (lane & 1) ? y : yo;
                const double qf = Qr - (gi00 * y0 * y0 + 2.0 * gi01 * y0 * y1 + gi11 * y1 * y1);
                lj[t] = -K * log(qf);
                mx = fmax(mx, lj[t]);
            }
            double se = 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t) se += exp(lj[t] - mx);
#pragma unroll
            for (int o = 2; o <= 8; o <<= 1) {  // the other shifts of the row (lane bits 1..3)
                const double m2 = __shfl_xor(mx, o, 64), s2 = __shfl_xor(se, o, 64);
                const double mm = fmax(mx, m2);
                se = se * exp(mx - mm) + s2 * exp(m2 - mm);
                mx = mm;
            }
            const double lnet = mx + log(se) + cst;
            const double lg = L.lng - K * log1p(L.gc * tr);
            const double a1 = A.log_eps + lg, b1 = A.log_1m_eps + lnet;
            const double hi = fmax(a1, b1);
            const double lm = hi + log(exp(a1 - hi) + exp(b1 - hi));
            const int rr = rt * 16 + ri;
            if (i16 == 0 && rr < (int)nc) {
                const unsigned row = A.order[c0 + rr];
                A.lnet[row] = lnet;
                A.lmix[row] = lm;
            }
        }
    }
}

template <int K>
__global__ void __launch_bounds__(256) k_mix_bwd_mm(LearnArgs A)
{
    constexpr int MT = 2 * K / 16;  // 16-coordinate tiles of M
    const int lane = threadIdx.x & 63, g = lane >> 4, i16 = lane & 15, q = lane & 1;
    const unsigned c = __builtin_amdgcn_readfirstlane((blockIdx.x * 256 + threadIdx.x) >> 6);
    if (c >= A.n_chunks) return;
    const int p = A.chunk_point[c];
    const LearnPoint &L = A.pts[p];
    const LearnParam &Q = A.par[p];
    const LearnStats &St = A.st[p];
    const double mxL = dkey_inv(St.maxkey), inv_sum = 1.0 / St.sum;
    const unsigned c0 = A.chunk_start[c], nc = A.chunk_start[c + 1] - c0;
    const double gi00 = Q.gi[0][0], gi01 = Q.gi[0][1], gi11 = Q.gi[1][1];
    const double lse0 = log((double)kMixS) + 0.5 * Q.logdet;
    d4_t macc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int t = 0; t < 4; ++t) macc[mt][t] = d4_t{0.0, 0.0, 0.0, 0.0};
    double S00 = 0.0, S01 = 0.0, S11 = 0.0, cs_acc = 0.0;
    double Epart[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) Epart[mt] = 0.0;
    for (int rt = 0; rt * 16 < (int)nc; ++rt) {
        // the row coefficient of this lane's A-operand row
        const bool valid = rt * 16 + i16 < (int)nc;
        const unsigned rowA = chunk_row(A, c0, nc, rt * 16 + i16);
        const double lnet = A.lnet[rowA], lmix = A.lmix[rowA];
        const uint8_t kd = A.kind[rowA];
        const double ws = kd != 2 ? exp((A.lf[rowA] - lmix) / A.T - mxL) * inv_sum : 0.0;
        const double rho = exp(A.log_1m_eps + lnet - lmix);
        const double cf = valid ? -ws * rho - (kd != 1 ? A.lambda * L.inv_n_acc : 0.0) : 0.0;
        const double lse = lnet + lse0;
        if (g == 0) cs_acc += cf;
        d4_t acc[4];
        double Qa, ta;
        mix_products<K>(A, Q, rowA, lane, acc, Qa, ta);
        double Cv[4][4], Fv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int ri = 4 * v + g;
            const double Qr = __shfl(Qa, ri, 64), cfr = __shfl(cf, ri, 64), lser = __shfl(lse, ri, 64);
            double fsum = 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double y = acc[t][v], yo = __shfl_xor(y, 1, 64);
                const double y0 = q ? yo : y, y1 = q ? y : yo;
                const double qf = Qr - (gi00 * y0 * y0 + 2.0 * gi01 * y0 * y1 + gi11 * y1 * y1);
                const double g0 = gi00 * y0 + gi01 * y1, g1 = gi01 * y0 + gi11 * y1;
                const double pi = exp(-K * log(qf) - lser);
                const double f = cfr * pi * K / qf;
                Cv[v][t] = f * (q ? g1 : g0);
                if (!q) {  // each (row, shift) once
                    S00 += f * g0 * g0;
                    S01 += f * g0 * g1;
                    S11 += f * g1 * g1;
                    fsum += f;
                }
            }
#pragma unroll
            for (int o = 1; o <= 8; o <<= 1) fsum += __shfl_xor(fsum, o, 64);
            Fv[v] = fsum;  // sum_j f of tile row 4v + g
        }
        // M += X^T C over the tile's rows: k-step s covers rows 4s .. 4s + 3
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const double *xr = A.X + (size_t)chunk_row(A, c0, nc, rt * 16 + 4 * s + g) * 2 * K;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const double xa = xr[16 * mt + i16];
                Epart[mt] += Fv[s] * xa * xa;
#pragma unroll
                for (int t = 0; t < 4; ++t) macc[mt][t] = mma_f64(xa, Cv[s][t], macc[mt][t]);
            }
        }
    }
    // P_mq = sum_j (R_j^T M_(j,q))_m for m = 16 mt + 4v + g
    double P[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int m = 16 * mt + 4 * v + g, k1 = m % K + 1;
            // cos coordinate (m < K; a compile-time fact: 4v + g < 16), and the partner
            // coordinate m -+ K: another tile (K >= 16) or another v (K = 8)
            constexpr bool big = K >= 16;
            const bool cosc = big ? mt < K / 16 : v < 2;
            const int mtp = big ? (cosc ? mt + K / 16 : mt - K / 16) : mt;
            const int vp = big ? v : (cosc ? v + 2 : v - 2);
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int j = 8 * t + (i16 >> 1), mi = (k1 * j) & (kMixS - 1);
                const double Mv = macc[mt][t][v], Mp = macc[mtp][t][vp];
                acc += cosc ? c_cs[mi] * Mv - c_sn[mi] * Mp : c_cs[mi] * Mv + c_sn[mi] * Mp;
            }
#pragma unroll
            for (int o = 2; o <= 8; o <<= 1) acc += __shfl_xor(acc, o, 64);
            P[mt][v] = acc;  // lanes with lane & 1 = q
        }
#pragma unroll
    for (int o = 1; o <= 32; o <<= 1) {
        S00 += __shfl_xor(S00, o, 64);
        S01 += __shfl_xor(S01, o, 64);
        S11 += __shfl_xor(S11, o, 64);
        cs_acc += __shfl_xor(cs_acc, o, 64);
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        Epart[mt] += __shfl_xor(Epart[mt], 16, 64);
        Epart[mt] += __shfl_xor(Epart[mt], 32, 64);  // E of coordinate 16 mt + i16
    }
    double *o = A.part + (size_t)c * A.pt_len;
    if (lane == 0) o[2] = cs_acc;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int m = 16 * mt + 4 * v + g, k = m % K;
            const double ak = Q.a[k];
            const double Pq = P[mt][v], Po = __shfl_xor(Pq, 1, 64);
            const double P0 = q ? Po : Pq, P1 = q ? Pq : Po;
            const double V0 = Q.V[m][0], V1 = Q.V[m][1];
            // dL/dV_mq
            if ((i16 >> 1) == 0) o[3 + K + 2 * m + q] = 2.0 * ak * (Pq - (q ? V0 * S01 + V1 * S11 : V0 * S00 + V1 * S01));
            // this coordinate's share of dL/dlog d_k, summed with its partner's in the cos lane
            const double Em = __shfl(Epart[mt], 4 * v + g, 64);
            const double term = Em - 2.0 * (V0 * P0 + V1 * P1) + V0 * V0 * S00 + 2.0 * V0 * V1 * S01 + V1 * V1 * S11;
            constexpr bool big = K >= 16;
            const bool cosc = big ? mt < K / 16 : v < 2;
            const int mtp = big ? (cosc ? mt + K / 16 : mt - K / 16) : mt;
            const int vp = big ? v : (cosc ? v + 2 : v - 2);
            const int mp = cosc ? m + K : m - K;
            const double Ppq = P[mtp][vp], Ppo = __shfl_xor(Ppq, 1, 64);
            const double Pp0 = q ? Ppo : Ppq, Pp1 = q ? Ppq : Ppo;
            const double W0 = Q.V[mp][0], W1 = Q.V[mp][1];
            const double Ep = __shfl(Epart[mtp], (16 * mtp + 4 * vp + g) % 16, 64);
            const double termp = Ep - 2.0 * (W0 * Pp0 + W1 * Pp1) + W0 * W0 * S00 + 2.0 * W0 * W1 * S01 + W1 * W1 * S11;
            if (cosc && i16 == 0) o[3 + k] = ak * (term + termp);
        }
}

// Per point: dL/dtheta = chunk sums (in order) - (1/2) csum d log|L0|/dtheta; dL/do.
template <int K>
__global__ void __launch_bounds__(64) k_param_grad(const LearnArgs A, int n_out, double v_scale, double *dout,
                                                   double *gmix)
{
    const int p = blockIdx.x, m = threadIdx.x;
    const LearnParam &Q = A.par[p];
    const LearnPoint &L = A.pts[p];
    double cs = 0.0, gd = 0.0, g0 = 0.0, g1 = 0.0;
    for (unsigned c = L.chunk0; c < L.chunk1; ++c) {
        const double *o = A.part + (size_t)c * A.pt_len;
        cs += o[2];
        if (m < K) gd += o[3 + m];
        if (m < 2 * K) {
            g0 += o[3 + K + 2 * m];
            g1 += o[3 + K + 2 * m + 1];
        }
    }
    double *d = dout + (size_t)p * n_out;
    double *g = gmix + (size_t)p * 5 * K;
    if (m < K) {
        const double v = gd - 0.5 * cs * Q.dld_logd[m];
        d[m] = v;
        g[m] = v;
    }
    if (m < 2 * K) {
        const double v0 = g0 - 0.5 * cs * Q.dld_V[m][0], v1 = g1 - 0.5 * cs * Q.dld_V[m][1];
        g[K + 2 * m] = v0;
        g[K + 2 * m + 1] = v1;
        d[K + 2 * m] = v_scale * v0;
        d[K + 2 * m + 1] = v_scale * v1;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
namespace {

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t b)
    {
        if (p && bytes >= b) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
        }
        bytes = std::max<size_t>(b, 256);
        return hipMalloc(&p, bytes);
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T>
    T *as() const { return reinterpret_cast<T *>(p); }
};

}  // namespace
}  // namespace tkdv

using namespace tkdv;

struct tkdv_learner {
    int device = 0;
    tkdv_learner_cfg cfg{};
    int K = 0, H = 0, n_out = 0;
    int64_t nW = 0;
    int n_points = 0;
    std::vector<LearnPoint> hpts;
    std::vector<uint64_t> n_acc;
    Buf W, gW, m1, m2, z, h1, h2, out, dh1, dh2, dout, gmix, par, pts, st;
    Buf X, row_point, kind, lf, lnet, lmix;
    Buf order, chunk_start, chunk_point, part;  // rows grouped by point, chunks, chunk partials
    Buf shift_src;                              // base rows and phases of tkdv_learner_add_shifted_rows
    std::vector<int> h_row_point;
    unsigned n_chunks = 0;
    unsigned long long n_rows = 0, cap_rows = 0;
    long long step = 0;
    int n_cu = 256;
};

namespace {

#define LTRY(expr)                                                                                   \
    do {                                                                                             \
        hipError_t _e = (expr);                                                                      \
        if (_e != hipSuccess) return record_error(TKDV_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

void features(const tkdv_point &pt, double *z)
{
    z[0] = (pt.beta_p - 40.0) / 20.0;
    z[1] = std::log(pt.E0);
    z[2] = pt.c32 * std::sqrt(pt.E0) * pt.beta_p / 1e4 - 1.0;
}

tkdv_status make_learn_point(const tkdv_learner *L, const tkdv_point &pt, const tkdv_plan &sp, LearnPoint &lp)
{
    if (pt.K != L->K) return record_error(TKDV_E_ARG, "point K differs from the learner's K");
    if (sp.proposal != TKDV_PROP_SIGMA) return record_error(TKDV_E_ARG, "the learner needs Sigma plans");
    if (!(pt.E0 > 0.0) || !std::isfinite(pt.beta_p) || !std::isfinite(pt.c32))
        return record_error(TKDV_E_ARG, "invalid point");
    std::memset(&lp, 0, sizeof(lp));
    features(pt, lp.z);
    const int K = pt.K;
    for (int k = 0; k < K; ++k) {
        if (!(sp.sigma2[k] > 0.0)) return record_error(TKDV_E_ARG, "plan has non-positive s_k^2");
        lp.logs2[k] = std::log(sp.sigma2[k]);
    }
    lp.E0 = pt.E0;
    lp.beta_p = pt.beta_p;
    lp.c32 = pt.c32;
    lp.gc = sp.alpha_star * pt.beta_p / ((double)K * K * K);
    lp.lng = 0.0;
    for (int k = 1; k <= K; ++k) lp.lng += std::log1p(lp.gc * k * k);
    return TKDV_OK;
}

template <int K>
hipError_t launch_prep(tkdv_learner *L, const double *out, const LearnPoint *pts, LearnParam *par, int np,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_mix_prep<K>, dim3(np), dim3(64), 0, st, out, L->n_out, pts, par, L->cfg.v_amp,
                       L->cfg.v_scale);
    return hipGetLastError();
}

hipError_t prep(tkdv_learner *L, const double *out, const LearnPoint *pts, LearnParam *par, int np, hipStream_t st)
{
    switch (L->K) {
    case 8: return launch_prep<8>(L, out, pts, par, np, st);
    case 16: return launch_prep<16>(L, out, pts, par, np, st);
    default: return launch_prep<32>(L, out, pts, par, np, st);
    }
}

LearnArgs args(tkdv_learner *L)
{
    LearnArgs A;
    A.X = L->X.as<double>();
    A.row_point = L->row_point.as<int>();
    A.kind = L->kind.as<uint8_t>();
    A.lf = L->lf.as<double>();
    A.lnet = L->lnet.as<double>();
    A.lmix = L->lmix.as<double>();
    A.n = L->n_rows;
    A.pts = L->pts.as<LearnPoint>();
    A.par = L->par.as<LearnParam>();
    A.st = L->st.as<LearnStats>();
    A.order = L->order.as<uint32_t>();
    A.chunk_start = L->chunk_start.as<uint32_t>();
    A.chunk_point = L->chunk_point.as<int>();
    A.n_chunks = L->n_chunks;
    A.part = L->part.as<double>();
    A.pt_len = chunk_part_len(L->K);
    A.T = L->cfg.temperature;
    A.lambda = L->cfg.nll_weight;
    const uint64_t E = (uint64_t)TKDV_MIX_S * (uint64_t)std::floor(L->cfg.eps * 4294967296.0 / TKDV_MIX_S);
    const double eps = std::ldexp((double)E, -32);
    A.log_eps = std::log(eps);
    A.log_1m_eps = std::log1p(-eps);
    return A;
}

template <int K>
hipError_t launch_rows(tkdv_learner *L, const LearnArgs &A, hipStream_t st, bool bwd)
{
    if (A.n == 0) return hipSuccess;
    if (!bwd)
        hipLaunchKernelGGL(k_mix_fwd_mm<K>, dim3((A.n_chunks + 3) / 4), dim3(256), 0, st, A);
    else
        hipLaunchKernelGGL(k_mix_bwd_mm<K>, dim3((A.n_chunks + 3) / 4), dim3(256), 0, st, A);
    return hipGetLastError();
}

hipError_t rows_pass(tkdv_learner *L, const LearnArgs &A, hipStream_t st, bool bwd)
{
    switch (L->K) {
    case 8: return launch_rows<8>(L, A, st, bwd);
    case 16: return launch_rows<16>(L, A, st, bwd);
    default: return launch_rows<32>(L, A, st, bwd);
    }
}

template <int K>
hipError_t launch_pgrad(tkdv_learner *L, hipStream_t st)
{
    hipLaunchKernelGGL(k_param_grad<K>, dim3(L->n_points), dim3(64), 0, st, args(L), L->n_out, L->cfg.v_scale,
                       L->dout.as<double>(), L->gmix.as<double>());
    return hipGetLastError();
}

// Loss and gradients at the current weights (gW holds dL/dweights after it).
tkdv_status evaluate(tkdv_learner *L, hipStream_t st)
{
    const int np = L->n_points, H = L->H, no = L->n_out;
    hipLaunchKernelGGL(k_mlp_fwd, dim3(np), dim3(kMaxHidden), 0, st, L->W.as<double>(), H, no, L->z.as<double>(),
                       L->h1.as<double>(), L->h2.as<double>(), L->out.as<double>());
    LTRY(hipGetLastError());
    LTRY(prep(L, L->out.as<double>(), L->pts.as<LearnPoint>(), L->par.as<LearnParam>(), np, st));
    LTRY(launch_fill_u32(L->st.p, sizeof(LearnStats) * np / 4, 0u, st));
    LearnArgs A = args(L);
    LTRY(rows_pass(L, A, st, false));
    const unsigned long long g = std::min<unsigned long long>((L->n_rows + 255) / 256 + 1, 4096);
    hipLaunchKernelGGL(k_loss_max, dim3((unsigned)g), dim3(256), 0, st, A);
    LTRY(hipGetLastError());
    hipLaunchKernelGGL(k_loss_chunk, dim3((A.n_chunks + 3) / 4), dim3(256), 0, st, A);
    LTRY(hipGetLastError());
    hipLaunchKernelGGL(k_loss_final, dim3((np + 63) / 64), dim3(64), 0, st, A, np);
    LTRY(hipGetLastError());
    LTRY(rows_pass(L, A, st, true));
    switch (L->K) {
    case 8: LTRY(launch_pgrad<8>(L, st)); break;
    case 16: LTRY(launch_pgrad<16>(L, st)); break;
    default: LTRY(launch_pgrad<32>(L, st)); break;
    }
    hipLaunchKernelGGL(k_mlp_bwd_hidden, dim3(np), dim3(kMaxHidden), 0, st, L->W.as<double>(), H, no,
                       L->h1.as<double>(), L->h2.as<double>(), L->dout.as<double>(), L->dh1.as<double>(),
                       L->dh2.as<double>());
    LTRY(hipGetLastError());
    const unsigned long long gw = std::min<unsigned long long>((L->nW + 255) / 256, 2048);
    hipLaunchKernelGGL(k_mlp_bwd_weights, dim3((unsigned)gw), dim3(256), 0, st, H, no, np, L->z.as<double>(),
                       L->h1.as<double>(), L->h2.as<double>(), L->dh1.as<double>(), L->dh2.as<double>(),
                       L->dout.as<double>(), L->gW.as<double>());
    LTRY(hipGetLastError());
    return TKDV_OK;
}

tkdv_status read_loss(tkdv_learner *L, double *h_loss, hipStream_t st)
{
    if (!h_loss) return TKDV_OK;
    std::vector<LearnStats> s(L->n_points);
    LTRY(hipMemcpyAsync(s.data(), L->st.p, sizeof(LearnStats) * L->n_points, hipMemcpyDeviceToHost, st));
    LTRY(hipStreamSynchronize(st));
    for (int p = 0; p < L->n_points; ++p) h_loss[p] = s[p].loss;
    return TKDV_OK;
}

tkdv_status grow_rows(tkdv_learner *L, unsigned long long need, hipStream_t st)
{
    if (need <= L->cap_rows) return TKDV_OK;
    unsigned long long cap = std::max<unsigned long long>(need, 2 * L->cap_rows);
    cap = std::max<unsigned long long>(cap, 4096);
    const int K = L->K;
    Buf X2, rp2, kd2, lf2;
    LTRY(X2.ensure(cap * 2 * K * sizeof(double)));
    LTRY(rp2.ensure(cap * sizeof(int)));
    LTRY(kd2.ensure(cap));
    LTRY(lf2.ensure(cap * sizeof(double)));
    if (L->n_rows) {
        LTRY(hipMemcpyAsync(X2.p, L->X.p, L->n_rows * 2 * K * sizeof(double), hipMemcpyDeviceToDevice, st));
        LTRY(hipMemcpyAsync(rp2.p, L->row_point.p, L->n_rows * sizeof(int), hipMemcpyDeviceToDevice, st));
        LTRY(hipMemcpyAsync(kd2.p, L->kind.p, L->n_rows, hipMemcpyDeviceToDevice, st));
        LTRY(hipMemcpyAsync(lf2.p, L->lf.p, L->n_rows * sizeof(double), hipMemcpyDeviceToDevice, st));
        LTRY(hipStreamSynchronize(st));
    }
    L->X.release();
    L->row_point.release();
    L->kind.release();
    L->lf.release();
    L->X = X2;
    L->row_point = rp2;
    L->kind = kd2;
    L->lf = lf2;
    LTRY(L->lnet.ensure(cap * sizeof(double)));
    LTRY(L->lmix.ensure(cap * sizeof(double)));
    L->cap_rows = cap;
    return TKDV_OK;
}

// Rows grouped by point in insertion order, cut into chunks of at most kChunk
// rows of one point; uploads the index order, the chunk table and the
// points' chunk ranges.
tkdv_status build_chunks(tkdv_learner *L, hipStream_t st)
{
    const int np = L->n_points;
    std::vector<std::vector<uint32_t>> by(np);
    for (uint32_t r = 0; r < (uint32_t)L->h_row_point.size(); ++r) by[L->h_row_point[r]].push_back(r);
    std::vector<uint32_t> order, cstart;
    std::vector<int> cpoint;
    for (int p = 0; p < np; ++p) {
        L->hpts[p].chunk0 = (uint32_t)cpoint.size();
        for (size_t q = 0; q < by[p].size(); q += kChunk) {
            cstart.push_back((uint32_t)(order.size() + q));
            cpoint.push_back(p);
        }
        order.insert(order.end(), by[p].begin(), by[p].end());
        L->hpts[p].chunk1 = (uint32_t)cpoint.size();
    }
    cstart.push_back((uint32_t)order.size());
    L->n_chunks = (unsigned)cpoint.size();
    LTRY(L->order.ensure(std::max<size_t>(order.size(), 1) * 4));
    LTRY(L->chunk_start.ensure(cstart.size() * 4));
    LTRY(L->chunk_point.ensure(std::max<size_t>(cpoint.size(), 1) * 4));
    LTRY(L->part.ensure(std::max<size_t>(cpoint.size(), 1) * chunk_part_len(L->K) * 8));
    if (!order.empty())
        LTRY(hipMemcpyAsync(L->order.p, order.data(), order.size() * 4, hipMemcpyHostToDevice, st));
    LTRY(hipMemcpyAsync(L->chunk_start.p, cstart.data(), cstart.size() * 4, hipMemcpyHostToDevice, st));
    if (!cpoint.empty())
        LTRY(hipMemcpyAsync(L->chunk_point.p, cpoint.data(), cpoint.size() * 4, hipMemcpyHostToDevice, st));
    LTRY(hipStreamSynchronize(st));
    return TKDV_OK;
}

tkdv_status upload_points(tkdv_learner *L, hipStream_t st)
{
    {
        tkdv_status s = build_chunks(L, st);
        if (s != TKDV_OK) return s;
    }
    for (int p = 0; p < L->n_points; ++p) L->hpts[p].inv_n_acc = L->n_acc[p] ? 1.0 / (double)L->n_acc[p] : 0.0;
    LTRY(hipMemcpyAsync(L->pts.p, L->hpts.data(), sizeof(LearnPoint) * L->n_points, hipMemcpyHostToDevice, st));
    LTRY(hipStreamSynchronize(st));
    return TKDV_OK;
}

template <int K>
hipError_t launch_append(tkdv_learner *L, const float *src, unsigned long long stride, unsigned long long n,
                         unsigned long long r0, int point, int kd, hipStream_t st)
{
    const unsigned long long g = std::min<unsigned long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_rows_append<K>, dim3((unsigned)g), dim3(256), 0, st, src, stride, n, L->X.as<double>(),
                       L->row_point.as<int>(), L->kind.as<uint8_t>(), r0, point, kd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rows_log_f<K>, dim3((unsigned)g), dim3(256), 0, st, L->X.as<double>(),
                       L->row_point.as<int>(), L->pts.as<LearnPoint>(), L->lf.as<double>(), r0, n);
    return hipGetLastError();
}

// Row (r, q) of n x n_phi new rows = base row r with the field translated by
// phi_q, u(xi) -> u(xi + phi_q): the (cos, sin) pair (a, b) of mode k becomes
// (a cos k phi + b sin k phi, b cos k phi - a sin k phi).  One thread per
// (row, mode); the rows are appended at r0 + r n_phi + q with their point and kind.
__global__ void k_rows_shift(int K, const double *base, const double *phi, unsigned long long n, int n_phi,
                             double *X, int *row_point, uint8_t *kind, unsigned long long r0, int point, int kd)
{
    const unsigned long long total = n * (unsigned long long)n_phi * K;
    for (unsigned long long v = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; v < total;
         v += (unsigned long long)gridDim.x * blockDim.x) {
        const int k = (int)(v % K) + 1;
        const unsigned long long rq = v / K, r = rq / n_phi;
        const int q = (int)(rq % n_phi);
        double sn, cs;
        sincos((double)k * phi[q], &sn, &cs);
        const double a = base[r * 2 * K + k - 1], b = base[r * 2 * K + K + k - 1];
        double *o = X + (r0 + rq) * 2 * K;
        o[k - 1] = a * cs + b * sn;
        o[K + k - 1] = b * cs - a * sn;
        if (k == 1) {
            row_point[r0 + rq] = point;
            kind[r0 + rq] = (uint8_t)kd;
        }
    }
}

template <int K>
hipError_t launch_log_f(tkdv_learner *L, unsigned long long r0, unsigned long long n, hipStream_t st)
{
    const unsigned long long g = std::min<unsigned long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_rows_log_f<K>, dim3((unsigned)g), dim3(256), 0, st, L->X.as<double>(),
                       L->row_point.as<int>(), L->pts.as<LearnPoint>(), L->lf.as<double>(), r0, n);
    return hipGetLastError();
}

}  // namespace

extern "C" {

tkdv_status tkdv_learner_create(tkdv_ctx *ctx, const tkdv_learner_cfg *cfg, tkdv_learner **out)
{
    if (!ctx || !cfg || !out) return record_error(TKDV_E_ARG, "NULL argument");
    *out = nullptr;
    const tkdv_learner_cfg &c = *cfg;
    if (c.K != 8 && c.K != 16 && c.K != 32) return record_error(TKDV_E_UNSUPPORTED, "the learner supports K in {8,16,32}");
    if (c.hidden < 1 || c.hidden > kMaxHidden) return record_error(TKDV_E_ARG, "hidden must be in 1..256");
    if (!(c.eps > 0.0 && c.eps < 1.0) || !(c.temperature > 0.0) || !(c.nll_weight >= 0.0) || !(c.lr > 0.0) ||
        !(c.beta1 >= 0.0 && c.beta1 < 1.0) || !(c.beta2 >= 0.0 && c.beta2 < 1.0) || !(c.adam_eps > 0.0) ||
        !std::isfinite(c.v_amp) || !std::isfinite(c.v_scale))
        return record_error(TKDV_E_ARG, "invalid learner configuration");
    LTRY(hipSetDevice(ctx_device(ctx)));
    tkdv_learner *L = new tkdv_learner();
    L->device = ctx_device(ctx);
    L->cfg = c;
    L->K = c.K;
    L->H = c.hidden;
    L->n_out = 5 * c.K;
    L->nW = mlp_n_weights(L->H, L->n_out);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, L->device) == hipSuccess) L->n_cu = prop.multiProcessorCount;
    // initial weights: Glorot uniform for W1, W2; W3 and biases 0 (the
    // network starts at D = Sigma, V = V0 for every point)
    std::vector<double> w((size_t)L->nW, 0.0);
    std::mt19937_64 rng(c.seed);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    const int H = L->H;
    const double a1 = std::sqrt(6.0 / (3 + H)), a2 = std::sqrt(6.0 / (2.0 * H));
    for (int i = 0; i < 3 * H; ++i) w[i] = a1 * U(rng);
    for (int i = 0; i < H * H; ++i) w[4 * H + i] = a2 * U(rng);
    tkdv_status s = TKDV_OK;
    auto fail = [&](hipError_t e) {
        s = record_error(TKDV_E_DEVICE, std::string("learner allocation: ") + hipGetErrorString(e));
    };
    hipError_t e;
    if ((e = L->W.ensure(L->nW * 8)) != hipSuccess || (e = L->gW.ensure(L->nW * 8)) != hipSuccess ||
        (e = L->m1.ensure(L->nW * 8)) != hipSuccess || (e = L->m2.ensure(L->nW * 8)) != hipSuccess)
        fail(e);
    if (s == TKDV_OK) {
        if ((e = hipMemcpy(L->W.p, w.data(), L->nW * 8, hipMemcpyHostToDevice)) != hipSuccess) fail(e);
        std::fill(w.begin(), w.end(), 0.0);
        if (s == TKDV_OK && (e = hipMemcpy(L->m1.p, w.data(), L->nW * 8, hipMemcpyHostToDevice)) != hipSuccess) fail(e);
        if (s == TKDV_OK && (e = hipMemcpy(L->m2.p, w.data(), L->nW * 8, hipMemcpyHostToDevice)) != hipSuccess) fail(e);
    }
    if (s != TKDV_OK) {
        tkdv_learner_destroy(L);
        return s;
    }
    *out = L;
    return TKDV_OK;
}

tkdv_status tkdv_learner_destroy(tkdv_learner *L)
{
    if (!L) return TKDV_OK;
    (void)hipSetDevice(L->device);
    Buf *bs[] = {&L->W, &L->gW, &L->m1, &L->m2, &L->z, &L->h1, &L->h2, &L->out, &L->dh1, &L->dh2, &L->dout,
                 &L->gmix, &L->par, &L->pts, &L->st, &L->X, &L->row_point, &L->kind, &L->lf, &L->lnet, &L->lmix,
                 &L->order, &L->chunk_start, &L->chunk_point, &L->part, &L->shift_src};
    for (Buf *b : bs) b->release();
    delete L;
    return TKDV_OK;
}

tkdv_status tkdv_learner_set_points(tkdv_learner *L, int32_t n_points, const tkdv_point *pts,
                                    const tkdv_plan *sigma_plans)
{
    if (!L || !pts || !sigma_plans || n_points < 1) return record_error(TKDV_E_ARG, "invalid points");
    LTRY(hipSetDevice(L->device));
    std::vector<LearnPoint> hp(n_points);
    for (int p = 0; p < n_points; ++p) {
        tkdv_status s = make_learn_point(L, pts[p], sigma_plans[p], hp[p]);
        if (s != TKDV_OK) return s;
    }
    L->n_points = n_points;
    L->hpts = hp;
    L->n_acc.assign(n_points, 0);
    L->n_rows = 0;
    L->h_row_point.clear();
    const size_t np = n_points, H = L->H, no = L->n_out;
    LTRY(L->z.ensure(np * 3 * 8));
    LTRY(L->h1.ensure(np * H * 8));
    LTRY(L->h2.ensure(np * H * 8));
    LTRY(L->dh1.ensure(np * H * 8));
    LTRY(L->dh2.ensure(np * H * 8));
    LTRY(L->out.ensure(np * no * 8));
    LTRY(L->dout.ensure(np * no * 8));
    LTRY(L->gmix.ensure(np * 5 * L->K * 8));
    LTRY(L->par.ensure(np * sizeof(LearnParam)));
    LTRY(L->pts.ensure(np * sizeof(LearnPoint)));
    LTRY(L->st.ensure(np * sizeof(LearnStats)));
    std::vector<double> z(np * 3);
    for (size_t p = 0; p < np; ++p)
        for (int c = 0; c < 3; ++c) z[p * 3 + c] = hp[p].z[c];
    LTRY(hipMemcpy(L->z.p, z.data(), z.size() * 8, hipMemcpyHostToDevice));
    double cs[kMixS], sn[kMixS];
    for (int m = 0; m < kMixS; ++m) {
        cs[m] = std::cos(2.0 * 3.14159265358979323846 * m / kMixS);
        sn[m] = std::sin(2.0 * 3.14159265358979323846 * m / kMixS);
    }
    LTRY(hipMemcpyToSymbol(HIP_SYMBOL(c_cs), cs, sizeof(cs)));
    LTRY(hipMemcpyToSymbol(HIP_SYMBOL(c_sn), sn, sizeof(sn)));
    return upload_points(L, nullptr);
}

tkdv_status tkdv_learner_add_rows(tkdv_learner *L, int32_t point, const float *d_xhat, uint64_t row_stride,
                                  uint64_t n, int32_t kind, void *stream)
{
    if (!L || (n > 0 && !d_xhat) || point < 0 || point >= L->n_points || (kind < 0 || kind > 2) ||
        row_stride < (uint64_t)(2 * L->K))
        return record_error(TKDV_E_ARG, "invalid rows");
    if (n == 0) return TKDV_OK;
    LTRY(hipSetDevice(L->device));
    hipStream_t st = (hipStream_t)stream;
    tkdv_status s = grow_rows(L, L->n_rows + n, st);
    if (s != TKDV_OK) return s;
    hipError_t e;
    switch (L->K) {
    case 8: e = launch_append<8>(L, d_xhat, row_stride, n, L->n_rows, point, kind, st); break;
    case 16: e = launch_append<16>(L, d_xhat, row_stride, n, L->n_rows, point, kind, st); break;
    default: e = launch_append<32>(L, d_xhat, row_stride, n, L->n_rows, point, kind, st); break;
    }
    LTRY(e);
    LTRY(hipStreamSynchronize(st));
    L->n_rows += n;
    L->h_row_point.insert(L->h_row_point.end(), n, point);
    if (kind != 1) L->n_acc[point] += n;
    return upload_points(L, st);
}

tkdv_status tkdv_learner_add_rows_host(tkdv_learner *L, int32_t point, const double *h_xhat, uint64_t n,
                                       int32_t kind)
{
    if (!L || (n > 0 && !h_xhat) || point < 0 || point >= L->n_points || (kind < 0 || kind > 2))
        return record_error(TKDV_E_ARG, "invalid rows");
    if (n == 0) return TKDV_OK;
    LTRY(hipSetDevice(L->device));
    const int K = L->K;
    std::vector<double> x(h_xhat, h_xhat + n * 2 * K);
    for (uint64_t r = 0; r < n; ++r) {
        double r2 = 0.0;
        for (int m = 0; m < 2 * K; ++m) r2 += x[r * 2 * K + m] * x[r * 2 * K + m];
        if (!(r2 > 0.0) || !std::isfinite(r2)) return record_error(TKDV_E_ARG, "row of zero or non-finite norm");
        const double inv = 1.0 / std::sqrt(r2);
        for (int m = 0; m < 2 * K; ++m) x[r * 2 * K + m] *= inv;
    }
    tkdv_status s = grow_rows(L, L->n_rows + n, nullptr);
    if (s != TKDV_OK) return s;
    std::vector<int> rp(n, point);
    std::vector<uint8_t> kd(n, (uint8_t)kind);
    LTRY(hipMemcpy(L->X.as<double>() + L->n_rows * 2 * K, x.data(), n * 2 * K * 8, hipMemcpyHostToDevice));
    LTRY(hipMemcpy(L->row_point.as<int>() + L->n_rows, rp.data(), n * sizeof(int), hipMemcpyHostToDevice));
    LTRY(hipMemcpy(L->kind.as<uint8_t>() + L->n_rows, kd.data(), n, hipMemcpyHostToDevice));
    hipError_t e;
    switch (K) {
    case 8: e = launch_log_f<8>(L, L->n_rows, n, nullptr); break;
    case 16: e = launch_log_f<16>(L, L->n_rows, n, nullptr); break;
    default: e = launch_log_f<32>(L, L->n_rows, n, nullptr); break;
    }
    LTRY(e);
    LTRY(hipDeviceSynchronize());
    L->n_rows += n;
    L->h_row_point.insert(L->h_row_point.end(), n, point);
    if (kind != 1) L->n_acc[point] += n;
    return upload_points(L, nullptr);
}

tkdv_status tkdv_learner_add_shifted_rows(tkdv_learner *L, int32_t point, const double *h_xhat, uint64_t n,
                                          const double *h_phi, int32_t n_phi, int32_t kind)
{
    if (!L || (n > 0 && (!h_xhat || !h_phi)) || point < 0 || point >= L->n_points || (kind < 0 || kind > 2) ||
        n_phi < 1 || n_phi > 4096 || n > (1ull << 32))
        return record_error(TKDV_E_ARG, "invalid rows or phases");
    if (n == 0) return TKDV_OK;
    for (int q = 0; q < n_phi; ++q)
        if (!std::isfinite(h_phi[q])) return record_error(TKDV_E_ARG, "non-finite phase");
    LTRY(hipSetDevice(L->device));
    const int K = L->K;
    std::vector<double> x(h_xhat, h_xhat + n * 2 * K);
    for (uint64_t r = 0; r < n; ++r) {
        double r2 = 0.0;
        for (int m = 0; m < 2 * K; ++m) r2 += x[r * 2 * K + m] * x[r * 2 * K + m];
        if (!(r2 > 0.0) || !std::isfinite(r2)) return record_error(TKDV_E_ARG, "row of zero or non-finite norm");
        const double inv = 1.0 / std::sqrt(r2);
        for (int m = 0; m < 2 * K; ++m) x[r * 2 * K + m] *= inv;
    }
    const unsigned long long n_new = n * (unsigned long long)n_phi;
    tkdv_status s = grow_rows(L, L->n_rows + n_new, nullptr);
    if (s != TKDV_OK) return s;
    const size_t base_bytes = n * 2 * K * sizeof(double);
    LTRY(L->shift_src.ensure(base_bytes + (size_t)n_phi * sizeof(double)));
    double *d_base = L->shift_src.as<double>();
    double *d_phi = d_base + n * 2 * K;
    LTRY(hipMemcpy(d_base, x.data(), base_bytes, hipMemcpyHostToDevice));
    LTRY(hipMemcpy(d_phi, h_phi, (size_t)n_phi * sizeof(double), hipMemcpyHostToDevice));
    const unsigned long long g = std::min<unsigned long long>((n_new * K + 255) / 256, 4096);
    hipLaunchKernelGGL(k_rows_shift, dim3((unsigned)g), dim3(256), 0, nullptr, K, d_base, d_phi,
                       (unsigned long long)n, n_phi, L->X.as<double>(), L->row_point.as<int>(),
                       L->kind.as<uint8_t>(), L->n_rows, point, kind);
    LTRY(hipGetLastError());
    hipError_t e;
    switch (K) {
    case 8: e = launch_log_f<8>(L, L->n_rows, n_new, nullptr); break;
    case 16: e = launch_log_f<16>(L, L->n_rows, n_new, nullptr); break;
    default: e = launch_log_f<32>(L, L->n_rows, n_new, nullptr); break;
    }
    LTRY(e);
    LTRY(hipDeviceSynchronize());
    L->n_rows += n_new;
    L->h_row_point.insert(L->h_row_point.end(), n_new, point);
    if (kind != 1) L->n_acc[point] += n_new;
    return upload_points(L, nullptr);
}

tkdv_status tkdv_learner_train(tkdv_learner *L, int32_t n_steps, double *h_loss, void *stream)
{
    if (!L || n_steps < 0) return record_error(TKDV_E_ARG, "invalid argument");
    if (L->n_points < 1 || L->n_rows == 0) return record_error(TKDV_E_ARG, "no training rows");
    LTRY(hipSetDevice(L->device));
    hipStream_t st = (hipStream_t)stream;
    const tkdv_learner_cfg &c = L->cfg;
    for (int it = 0; it < n_steps; ++it) {
        tkdv_status s = evaluate(L, st);
        if (s != TKDV_OK) return s;
        ++L->step;
        const double c1 = 1.0 - std::pow(c.beta1, (double)L->step), c2 = 1.0 - std::pow(c.beta2, (double)L->step);
        const unsigned long long g = std::min<unsigned long long>((L->nW + 255) / 256, 2048);
        hipLaunchKernelGGL(k_adam, dim3((unsigned)g), dim3(256), 0, st, L->W.as<double>(), L->gW.as<double>(),
                           L->m1.as<double>(), L->m2.as<double>(), (long long)L->nW, c.lr, c.beta1, c.beta2,
                           c.adam_eps, c1, c2);
        LTRY(hipGetLastError());
    }
    if (n_steps > 0) return read_loss(L, h_loss, st);
    LTRY(hipStreamSynchronize(st));
    return TKDV_OK;
}

tkdv_status tkdv_learner_gradients(tkdv_learner *L, double *h_loss, double *h_grad_mix, double *h_grad_weights,
                                   void *stream)
{
    if (!L) return record_error(TKDV_E_ARG, "invalid argument");
    if (L->n_points < 1 || L->n_rows == 0) return record_error(TKDV_E_ARG, "no training rows");
    LTRY(hipSetDevice(L->device));
    hipStream_t st = (hipStream_t)stream;
    tkdv_status s = evaluate(L, st);
    if (s != TKDV_OK) return s;
    if (h_grad_mix)
        LTRY(hipMemcpyAsync(h_grad_mix, L->gmix.p, (size_t)L->n_points * 5 * L->K * 8, hipMemcpyDeviceToHost, st));
    if (h_grad_weights) LTRY(hipMemcpyAsync(h_grad_weights, L->gW.p, L->nW * 8, hipMemcpyDeviceToHost, st));
    LTRY(hipStreamSynchronize(st));
    return read_loss(L, h_loss, st);
}

tkdv_status tkdv_learner_mixture(tkdv_learner *L, const tkdv_point *pt, const tkdv_plan *sigma_plan,
                                 tkdv_mixture *out)
{
    if (!L || !pt || !sigma_plan || !out) return record_error(TKDV_E_ARG, "NULL argument");
    LTRY(hipSetDevice(L->device));
    LearnPoint lp;
    tkdv_status s = make_learn_point(L, *pt, *sigma_plan, lp);
    if (s != TKDV_OK) return s;
    const int H = L->H, no = L->n_out, K = L->K;
    Buf z, h1, h2, o, pts, par;
    LTRY(z.ensure(3 * 8));
    LTRY(h1.ensure(H * 8));
    LTRY(h2.ensure(H * 8));
    LTRY(o.ensure(no * 8));
    LTRY(pts.ensure(sizeof(LearnPoint)));
    LTRY(par.ensure(sizeof(LearnParam)));
    tkdv_status rs = TKDV_OK;
    LearnParam hp;
    do {
        hipError_t e;
        if ((e = hipMemcpy(z.p, lp.z, 3 * 8, hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(pts.p, &lp, sizeof(lp), hipMemcpyHostToDevice)) != hipSuccess) {
            rs = record_error(TKDV_E_DEVICE, hipGetErrorString(e));
            break;
        }
        hipLaunchKernelGGL(k_mlp_fwd, dim3(1), dim3(kMaxHidden), 0, nullptr, L->W.as<double>(), H, no,
                           z.as<double>(), h1.as<double>(), h2.as<double>(), o.as<double>());
        if ((e = hipGetLastError()) != hipSuccess ||
            (e = prep(L, o.as<double>(), pts.as<LearnPoint>(), par.as<LearnParam>(), 1, nullptr)) != hipSuccess ||
            (e = hipMemcpy(&hp, par.p, sizeof(hp), hipMemcpyDeviceToHost)) != hipSuccess) {
            rs = record_error(TKDV_E_DEVICE, hipGetErrorString(e));
            break;
        }
    } while (false);
    Buf *bs[] = {&z, &h1, &h2, &o, &pts, &par};
    for (Buf *b : bs) b->release();
    if (rs != TKDV_OK) return rs;
    std::memset(out, 0, sizeof(*out));
    out->K = K;
    out->eps = L->cfg.eps;
    for (int k = 0; k < K; ++k) out->logd[k] = hp.logd[k];
    for (int m = 0; m < 2 * K; ++m)
        for (int q = 0; q < 2; ++q) out->V[m][q] = hp.V[m][q];
    return TKDV_OK;
}

int64_t tkdv_learner_n_weights(const tkdv_learner *L) { return L ? L->nW : -1; }

tkdv_status tkdv_learner_get_weights(const tkdv_learner *L, double *h_out, int64_t n)
{
    if (!L || !h_out || n != L->nW) return record_error(TKDV_E_ARG, "invalid argument");
    LTRY(hipSetDevice(L->device));
    LTRY(hipMemcpy(h_out, L->W.p, n * 8, hipMemcpyDeviceToHost));
    return TKDV_OK;
}

tkdv_status tkdv_learner_set_weights(tkdv_learner *L, const double *h_in, int64_t n)
{
    if (!L || !h_in || n != L->nW) return record_error(TKDV_E_ARG, "invalid argument");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(h_in[i])) return record_error(TKDV_E_ARG, "non-finite weight");
    LTRY(hipSetDevice(L->device));
    LTRY(hipMemcpy(L->W.p, h_in, n * 8, hipMemcpyHostToDevice));
    std::vector<double> zero((size_t)n, 0.0);
    LTRY(hipMemcpy(L->m1.p, zero.data(), n * 8, hipMemcpyHostToDevice));
    LTRY(hipMemcpy(L->m2.p, zero.data(), n * 8, hipMemcpyHostToDevice));
    L->step = 0;
    return TKDV_OK;
}

}  // extern "C"
