// Learned proposal: the network that maps (beta', E0, C3/C2) to the mixture
// of a point, and its training on the GPU (FP64 throughout).
//
// One training step (all on one stream):
//   k_mlp_fwd       per point: z -> h1 -> h2 -> o (tanh layers)
//   k_mix_prep      per point: o -> log d, V; A = D^-1, G^-1, log|L0| and
//                   the gradient of log|L0|
//   k_mix_fwd       per row (one wave, a lane per coordinate): log q_net and
//                   log q_mix over the S shifts (online log-sum-exp)
//   k_loss_max      per point maximum of r_s = log f - log q_mix
//   k_loss_chunk    per chunk of a point's rows: sum of exp(r_s/T - max), NLL
//   k_loss_final    per point: chunk partials in order -> soft maximum, loss
//   k_mix_bwd       per chunk: dL/d(log d, V) of the point, accumulated over
//                   the rows' shifts in row order
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

struct LearnParam {
    double logd[kLKMax], a[kLKMax];
    double V[2 * kLKMax][2];
    double gi[2][2];
    double logdet;
    double dld_logd[kLKMax];   // d log|L0| / d log d_k
    double dld_V[2 * kLKMax][2];
};

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

// ---------------------------------------------------------------------------
// Mixture density of a row, one wave per row, lane m = coordinate m (2K <= 64).
//   w = R_j^T x, y = V^T A w, g = G^-1 y, e = w - V g, qf_j = e^T A e + |g|^2,
//   l_j = -K ln qf_j; log q_net = LSE_j(l_j) - ln S - log|L0|/2.
// ---------------------------------------------------------------------------
template <int K>
struct RowMix {
    double xm, xp;   // own coordinate and the other one of the mode pair
    double am, v0, v1;
    int k;           // mode of the lane (1..K)
    bool act, sinb;

    __device__ void load(const LearnArgs &A, const LearnParam &Q, unsigned long long r, int m)
    {
        act = m < 2 * K;
        sinb = m >= K;
        k = m % K + 1;
        const int mp = sinb ? m - K : m + K;
        xm = act ? A.X[r * 2 * K + m] : 0.0;
        xp = act ? A.X[r * 2 * K + mp] : 0.0;
        am = act ? Q.a[k - 1] : 0.0;
        v0 = act ? Q.V[m][0] : 0.0;
        v1 = act ? Q.V[m][1] : 0.0;
    }
    // shift j: own coordinate of w = R_j^T x, e and qf (all lanes get qf, g)
    __device__ void shift(const LearnParam &Q, const double *cs, const double *sn, int j, double &w, double &e,
                          double &qf, double &g0, double &g1) const
    {
        const int mi = (k * j) & (kMixS - 1);
        const double c = cs[mi], s = sn[mi];
        w = act ? (sinb ? xm * c + xp * s : xm * c - xp * s) : 0.0;
        const double aw = am * w;
        const double y0 = wsum(v0 * aw), y1 = wsum(v1 * aw);
        g0 = Q.gi[0][0] * y0 + Q.gi[0][1] * y1;
        g1 = Q.gi[1][0] * y0 + Q.gi[1][1] * y1;
        e = w - (v0 * g0 + v1 * g1);
        qf = wsum(am * e * e) + g0 * g0 + g1 * g1;
    }
};

__constant__ double c_cs[kMixS], c_sn[kMixS];

template <int K>
__global__ void __launch_bounds__(256) k_mix_fwd(LearnArgs A)
{
    const int m = threadIdx.x & 63;
    const unsigned long long nw = (unsigned long long)gridDim.x * 4;
    for (unsigned long long r = ((unsigned long long)blockIdx.x * 256 + threadIdx.x) >> 6; r < A.n; r += nw) {
        const int p = __builtin_amdgcn_readfirstlane(A.row_point[r]);
        const LearnPoint &L = A.pts[p];
        const LearnParam &Q = A.par[p];
        RowMix<K> R;
        R.load(A, Q, r, m);
        double mx = -INFINITY, se = 0.0;
        for (int j = 0; j < kMixS; ++j) {
            double w, e, qf, g0, g1;
            R.shift(Q, c_cs, c_sn, j, w, e, qf, g0, g1);
            const double l = -K * log(qf);
            if (l > mx) {
                se = se * exp(mx - l) + 1.0;
                mx = l;
            } else {
                se += exp(l - mx);
            }
        }
        const double t = wsum(R.act ? (double)R.k * R.k * R.xm * R.xm : 0.0);
        const double lnet = mx + log(se) - log((double)kMixS) - 0.5 * Q.logdet;
        const double lg = L.lng - K * log1p(L.gc * t);
        const double a1 = A.log_eps + lg, b1 = A.log_1m_eps + lnet;
        const double hi = a1 > b1 ? a1 : b1;
        const double lm = hi + log(exp(a1 - hi) + exp(b1 - hi));
        if (m == 0) {
            A.lnet[r] = lnet;
            A.lmix[r] = lm;
        }
    }
}

__global__ void k_loss_max(LearnArgs A)
{
    for (unsigned long long r = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; r < A.n;
         r += (unsigned long long)gridDim.x * blockDim.x)
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
        se += exp((A.lf[r] - A.lmix[r]) / A.T - mx);
        nll += A.kind[r] == 0 ? -A.lnet[r] : 0.0;
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

// dL/d(log d, V) per chunk (one wave, rows in order).  c_s = dL/d log q_net(x_s):
//   -w_s rho_s - lambda/n_acc [kind 0],  w_s = softmax_s(r_s/T),
//   rho_s = (1 - eps) q_net/q_mix.
// d log q_net/dV_mq = sum_j pi_j (2K/qf_j) (A e_j)_m g_jq,
// d log q_net/d log d_k = sum_j pi_j (K/qf_j) sum_{m in k} a_m e_jm^2
// (pi_j = softmax_j l_j), without the -log|L0|/2 term (added per point).
template <int K>
__global__ void __launch_bounds__(256) k_mix_bwd(LearnArgs A)
{
    const int m = threadIdx.x & 63;
    const unsigned c = __builtin_amdgcn_readfirstlane((blockIdx.x * 256 + threadIdx.x) >> 6);
    if (c >= A.n_chunks) return;
    const int p = A.chunk_point[c];
    const LearnPoint &L = A.pts[p];
    const LearnParam &Q = A.par[p];
    const LearnStats &S = A.st[p];
    const double mx = dkey_inv(S.maxkey);
    double gv0 = 0.0, gv1 = 0.0, gd = 0.0, cs_acc = 0.0;
    for (unsigned q = A.chunk_start[c]; q < A.chunk_start[c + 1]; ++q) {
        const unsigned r = A.order[q];
        const double ws = exp((A.lf[r] - A.lmix[r]) / A.T - mx) / S.sum;
        const double rho = exp(A.log_1m_eps + A.lnet[r] - A.lmix[r]);
        const double cf = -ws * rho - (A.kind[r] == 0 ? A.lambda * L.inv_n_acc : 0.0);
        cs_acc += cf;
        RowMix<K> R;
        R.load(A, Q, r, m);
        // log-sum-exp of l_j: ln(sum_j qf_j^-K) relative to the row's q_net
        const double lse = A.lnet[r] + log((double)kMixS) + 0.5 * Q.logdet;
        for (int j = 0; j < kMixS; ++j) {
            double w, e, qf, g0, g1;
            R.shift(Q, c_cs, c_sn, j, w, e, qf, g0, g1);
            const double pi = exp(-K * log(qf) - lse);
            const double f = cf * pi * K / qf;
            const double ae = R.am * e;
            gv0 += 2.0 * f * ae * g0;
            gv1 += 2.0 * f * ae * g1;
            gd += f * ae * e;
        }
    }
    // the two coordinates of mode m + 1
    const double gd_pair = gd + __shfl(gd, (m + K) & 63, 64);
    double *o = A.part + (size_t)c * A.pt_len;
    if (m == 0) o[2] = cs_acc;
    if (m < K) o[3 + m] = gd_pair;
    if (m < 2 * K) {
        o[3 + K + 2 * m] = gv0;
        o[3 + K + 2 * m + 1] = gv1;
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
    const unsigned long long n = A.n;
    if (n == 0) return hipSuccess;
    if (!bwd) {
        unsigned long long g = (n + 3) / 4;
        g = std::min<unsigned long long>(g, 64ull * L->n_cu);
        hipLaunchKernelGGL(k_mix_fwd<K>, dim3((unsigned)g), dim3(256), 0, st, A);
    } else {
        hipLaunchKernelGGL(k_mix_bwd<K>, dim3((A.n_chunks + 3) / 4), dim3(256), 0, st, A);
    }
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
    if (!L || (n > 0 && !d_xhat) || point < 0 || point >= L->n_points || (kind != 0 && kind != 1) ||
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
    if (kind == 0) L->n_acc[point] += n;
    return upload_points(L, st);
}

tkdv_status tkdv_learner_add_rows_host(tkdv_learner *L, int32_t point, const double *h_xhat, uint64_t n,
                                       int32_t kind)
{
    if (!L || (n > 0 && !h_xhat) || point < 0 || point >= L->n_points || (kind != 0 && kind != 1))
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
    if (kind == 0) L->n_acc[point] += n;
    return upload_points(L, nullptr);
}

tkdv_status tkdv_learner_add_shifted_rows(tkdv_learner *L, int32_t point, const double *h_xhat, uint64_t n,
                                          const double *h_phi, int32_t n_phi, int32_t kind)
{
    if (!L || (n > 0 && (!h_xhat || !h_phi)) || point < 0 || point >= L->n_points || (kind != 0 && kind != 1) ||
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
    if (kind == 0) L->n_acc[point] += n_new;
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
