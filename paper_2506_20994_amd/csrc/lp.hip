// Learned per-element preconditioner: an (n + 6)-256-256-n MLP, n = lx^3 (518-256-
// 256-512 at lx = 8), applied to each element's normalised residual plus six
// geometric features, trained on the GPU with Adam.  The dense contractions run on bf16 MFMA
// (v_mfma_f32_16x16x32_bf16) with float32 accumulation; master weights, Adam
// moments, the loss and the bias gradients are float32.
//
// GEMM form used throughout: C[M][N] = A[M][K] . B[N][K]^T with both operands
// k-contiguous (row-major bf16); the other products of backpropagation are
// brought to this form with explicit transposes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "sem_internal.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

// the lx = 8 sizes (the weight-stationary linear product is written for them);
// a network's own sizes are lx^3 outputs, lx^3 + 6 inputs padded to 16
constexpr int kIn = 518, kInPad = 528, kHid = 256, kOut = 512;
constexpr int kBlock = 256;

__device__ __forceinline__ u16 bf16_rne(float f) {
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7fffffffu) > 0x7f800000u) return (u16)((b >> 16) | 0x40u);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (u16)(b >> 16);
}
__device__ __forceinline__ float bf16_f(u16 h) { return __uint_as_float((uint32_t)h << 16); }

enum { EPI_BIAS = 1, EPI_RELU = 2, EPI_MASK = 4 };
constexpr int BM = 128, BN = 128, BK = 64, LDK = BK + 8;

// C = A . B^T (+bias[n]) (relu) (*(mask[m][n] > 0)); Cf float and/or Cb bf16.
// With pos, the float output of (m, n) goes to Cf[pos[m * ldc + n]], scaled by
// rowscale[m].
// Requires K % 8 == 0, lda % 8 == 0, ldb % 8 == 0 and 16-byte aligned bases.
// 128 x 128 tile per 256-thread workgroup, each wave 64 x 64 as 4 x 4
// 16x16x32 MFMA blocks; the next 64-wide k-slab is fetched into registers
// while the current one is multiplied out of LDS.
__global__ void __launch_bounds__(256)
gemm_nt(int M, int N, int K, const u16* __restrict__ A, int lda, const u16* __restrict__ B, int ldb,
        const float* __restrict__ bias, const u16* __restrict__ mask, int ldm,
        float* __restrict__ Cf, u16* __restrict__ Cb, int ldc, int epi, const int* __restrict__ skip,
        const float* __restrict__ rowscale, const int32_t* __restrict__ pos) {
    if (skip && *skip) return;
    __shared__ __attribute__((aligned(16))) u16 sA[BM * LDK];
    __shared__ __attribute__((aligned(16))) u16 sB[BN * LDK];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // each thread moves 4 chunks of 8 bf16 of A and of B per slab
    constexpr int CH = BM * BK / 8 / 256;
    uint4 ra[CH], rb[CH];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int c = tid + q * 256;
            const int row = c >> 3, kc = (c & 7) * 8;
            const int gk = k0 + kc;
            const int gm = m0 + row, gn = n0 + row;
            ra[q] = (gm < M && gk < K) ? *reinterpret_cast<const uint4*>(A + (int64_t)gm * lda + gk)
                                       : uint4{0u, 0u, 0u, 0u};
            rb[q] = (gn < N && gk < K) ? *reinterpret_cast<const uint4*>(B + (int64_t)gn * ldb + gk)
                                       : uint4{0u, 0u, 0u, 0u};
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int q = 0; q < CH; ++q) {
            const int c = tid + q * 256;
            const int row = c >> 3, kc = (c & 7) * 8;
            *reinterpret_cast<uint4*>(sA + row * LDK + kc) = ra[q];
            *reinterpret_cast<uint4*>(sB + row * LDK + kc) = rb[q];
        }
        __syncthreads();
        if (k0 + BK < K) fetch(k0 + BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 32) {
            bf16x8 af[4], bfv[4];
            const int ko = kk + (lane >> 4) * 8;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                af[i] = *reinterpret_cast<const bf16x8*>(sA + (wm * 64 + i * 16 + (lane & 15)) * LDK + ko);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                bfv[j] = *reinterpret_cast<const bf16x8*>(sB + (wn * 64 + j * 16 + (lane & 15)) * LDK + ko);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfv[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // acc[i][j][q] = C[wm*64 + i*16 + 4*(lane/16) + q][wn*64 + j*16 + lane%16]
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + wn * 64 + j * 16 + (lane & 15);
            if (n >= N) continue;
            const float bv = (epi & EPI_BIAS) ? bias[n] : 0.f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + q;
                if (m >= M) continue;
                float v = acc[i][j][q] + bv;
                if (epi & EPI_RELU) v = fmaxf(v, 0.f);
                if ((epi & EPI_MASK) && !(bf16_f(mask[(int64_t)m * ldm + n]) > 0.f)) v = 0.f;
                if (pos) Cf[pos[(int64_t)m * ldc + n]] = v * rowscale[m];
                else if (Cf) Cf[(int64_t)m * ldc + n] = v;
                if (Cb) Cb[(int64_t)m * ldc + n] = bf16_rne(v);
            }
        }
}

// C[r][c] = sum_k A[r][k] B[k][c] in float32 (small products of the weights)
__global__ void matmul_f32(float* __restrict__ C, const float* __restrict__ A, const float* __restrict__ B,
                           int rows, int inner, int cols, int lda, int ldb, int ldc) {
    const int r = blockIdx.y, c = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows || c >= cols) return;
    float s = 0.f;
    for (int k = 0; k < inner; ++k) s += A[(int64_t)r * lda + k] * B[(int64_t)k * ldb + c];
    C[(int64_t)r * ldc + c] = s;
}

__global__ void f32_to_bf16(u16* __restrict__ out, const float* __restrict__ in, int64_t n) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        out[q] = bf16_rne(in[q]);
}

// out[c][r] = in[r][c] (bf16), rows x cols, leading dims ldi / ldo
// out = bf16((in + in^T) / 2) for an n x n row-major matrix
__global__ void sym_to_bf16(u16* __restrict__ out, const float* __restrict__ in, int n) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n * n; q += gridDim.x * blockDim.x) {
        const int i = q / n, j = q % n;
        out[q] = bf16_rne(0.5f * (in[q] + in[j * n + i]));
    }
}

__global__ void transpose_bf16(u16* __restrict__ out, int ldo, const u16* __restrict__ in, int ldi,
                               int rows, int cols) {
    __shared__ u16 t[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 32 x 8
    for (int y = ty; y < 32; y += 8) {
        const int r = r0 + y, c = c0 + tx;
        t[y][tx] = (r < rows && c < cols) ? in[(int64_t)r * ldi + c] : (u16)0;
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int c = c0 + y, r = r0 + tx;
        if (c < cols && r < rows) out[(int64_t)c * ldo + r] = t[tx][y];
    }
}

// float32 master (rows x cols) -> bf16 copy with leading dim ldo (zero pad)
// and, if outT != null, its bf16 transpose (cols x rows)
__global__ void weights_to_bf16(u16* __restrict__ out, int ldo, u16* __restrict__ outT,
                                const float* __restrict__ w, int rows, int cols) {
    const int64_t n = (int64_t)rows * ldo;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(q / ldo), c = (int)(q % ldo);
        const u16 v = c < cols ? bf16_rne(w[(int64_t)r * cols + c]) : (u16)0;
        out[q] = v;
        if (outT && c < cols) outT[(int64_t)c * rows + r] = v;
    }
}

// batch gather: Xb[i] = X[rows[i]] (bf16, nip wide), Tb[i] = T[rows[i]] (float, no)
__global__ void gather_rows(u16* __restrict__ Xb, float* __restrict__ Tb, const u16* __restrict__ X,
                            const float* __restrict__ T, const int64_t* __restrict__ rows, int B, int nip, int no) {
    const int i = blockIdx.x;
    if (i >= B) return;
    const int64_t r = rows[i];
    for (int c = threadIdx.x; c < nip; c += blockDim.x) Xb[(int64_t)i * nip + c] = X[r * nip + c];
    for (int c = threadIdx.x; c < no; c += blockDim.x) Tb[(int64_t)i * no + c] = T[r * no + c];
}

// d3 = 2 (Y3 - T) / (B * kOut) as float and bf16; per-block partial of sum (Y3 - T)^2
__global__ void mse_grad(float* __restrict__ d3f, u16* __restrict__ d3b, const float* __restrict__ Y3,
                         const float* __restrict__ T, int64_t n, float scale, double* __restrict__ part) {
    __shared__ double s[kBlock / 64];
    double acc = 0.0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const float d = Y3[q] - T[q];
        acc += (double)d * d;
        const float g = scale * d;
        d3f[q] = g;
        d3b[q] = bf16_rne(g);
    }
    acc = sem::wave_sum(acc);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kBlock / 64; ++q) t += s[q];
        part[blockIdx.x] = t;
    }
}

// d = Y3 - T as float and bf16 (the metric loss's residual)
__global__ void diff_kernel(float* __restrict__ df, u16* __restrict__ db, const float* __restrict__ Y3,
                            const float* __restrict__ T, int64_t n) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const float d = Y3[q] - T[q];
        df[q] = d;
        db[q] = bf16_rne(d);
    }
}

// loss partials sum d.Kd; gradient d3 = scale * Kd (float and bf16)
__global__ void metric_grad(float* __restrict__ d3f, u16* __restrict__ d3b, const float* __restrict__ df,
                            const float* __restrict__ Kd, int64_t n, float scale, double* __restrict__ part) {
    __shared__ double s[kBlock / 64];
    double acc = 0.0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const float k = Kd[q];
        acc += (double)df[q] * k;
        const float g = scale * k;
        d3f[q] = g;
        d3b[q] = bf16_rne(g);
    }
    acc = sem::wave_sum(acc);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < kBlock / 64; ++q) t += s[q];
        part[blockIdx.x] = t;
    }
}

// one 256-thread block: strided partial sums, then a fixed-order tree
__global__ void loss_final(float* __restrict__ loss, const double* __restrict__ part, int nb, double inv_n) {
    __shared__ double s_red[256];
    double t = 0.0;
    for (int q = threadIdx.x; q < nb; q += 256) t += part[q];
    s_red[threadIdx.x] = t;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_red[threadIdx.x] += s_red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(s_red[0] * inv_n);
}

// out[c] = sum_r d[r][c] (float), fixed order
// column sums of a (rows x cols) row-major matrix in two deterministic passes:
// part[chunk][c] = sum over the 64 rows of the chunk (256 threads: 4 row groups
// x 64 columns, combined in a fixed order), then out[c] = sum over the chunks
constexpr int kColRows = 64;
__global__ void colsum_part(float* __restrict__ part, const float* __restrict__ d, int rows, int cols) {
    __shared__ float s_red[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), rg = threadIdx.x >> 6;
    const int r0 = blockIdx.y * kColRows;
    float s = 0.f;
    if (c < cols)
        for (int r = r0 + rg; r < r0 + kColRows && r < rows; r += 4) s += d[(int64_t)r * cols + c];
    s_red[rg][threadIdx.x & 63] = s;
    __syncthreads();
    if (rg == 0 && c < cols)
        part[(int64_t)blockIdx.y * cols + c] = (s_red[0][threadIdx.x] + s_red[1][threadIdx.x]) +
                                              (s_red[2][threadIdx.x] + s_red[3][threadIdx.x]);
}

__global__ void colsum_final(float* __restrict__ out, const float* __restrict__ part, int chunks, int cols) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int q = 0; q < chunks; ++q) s += part[(int64_t)q * cols + c];
    out[c] = s;
}

// Adam on a (rows x cols) parameter whose gradient has leading dim ldg
__global__ void adam_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int rows, int cols, int ldg, float lr,
                            float b1, float omb1, float b2, float omb2, float eps, float c1, float c2) {
    const int64_t n = (int64_t)rows * cols;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = q / cols, c = q % cols;
        const float gv = g[r * ldg + c];
        const float mv = b1 * m[q] + omb1 * gv;
        const float vv = b2 * v[q] + omb2 * gv * gv;
        m[q] = mv;
        v[q] = vv;
        p[q] -= lr * (mv / c1) / (sqrtf(vv / c2) + eps);
    }
}

// per-element geometric features (six means of h1 g_ab over kappa), kappa and 1/kappa
__global__ void geo_kernel(float* __restrict__ geo, float* __restrict__ kappa, float* __restrict__ kappa_inv,
                           const double* __restrict__ h1, const double* __restrict__ g11,
                           const double* __restrict__ g22, const double* __restrict__ g33,
                           const double* __restrict__ g12, const double* __restrict__ g13,
                           const double* __restrict__ g23, int64_t nel, int no) {
    const int64_t e = blockIdx.x;
    if (e >= nel) return;
    const double* G[6] = {g11, g22, g33, g12, g13, g23};
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int q = threadIdx.x; q < no; q += 64) {
        const int64_t L = e * no + q;
        const double h = h1 ? h1[L] : 1.0;
        for (int a = 0; a < 6; ++a) s[a] += h * G[a][L];
    }
    for (int a = 0; a < 6; ++a) s[a] = sem::wave_sum(s[a]);
    if (threadIdx.x == 0) {
        const double kap = (s[0] + s[1] + s[2]) / (3.0 * no);
        kappa[e] = (float)kap;
        kappa_inv[e] = (float)(1.0 / kap);
        for (int a = 0; a < 6; ++a) geo[e * 6 + a] = (float)(s[a] / no / kap);
    }
}

// X[row] = [bf16(r_e / s_e) (no), geo (6), 0 (to nip)]; scale[row] = s_e / kappa_e;
// optionally T[row] = err_e * kappa_e / s_e.  With uoff (unique layout) or mult
// (local layout) the residual is first weighted by S = mult^-1/2 (the linear
// form's symmetric apply).  One wave per element, NC = ceil(no / 64) nodes per lane.
template <typename T, int NC>
__global__ void features_kernel(u16* __restrict__ X, float* __restrict__ scale, float* __restrict__ Tt,
                                const T* __restrict__ r, const double* __restrict__ err,
                                const double* __restrict__ minv,
                                const float* __restrict__ geo, const float* __restrict__ kappa,
                                const int64_t* __restrict__ elems, int64_t count, int64_t row0,
                                const int* __restrict__ skip, const int32_t* __restrict__ lid,
                                const int32_t* __restrict__ uoff, const double* __restrict__ mult,
                                int no, int nip) {
    if (skip && *skip) return;
    const int64_t q = blockIdx.x;
    if (q >= count) return;
    const int64_t e = elems ? elems[q] : q;
    const int64_t row = row0 + q;
    const int lane = threadIdx.x;
    double v[NC];
    double ss = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int n = c * 64 + lane;
        const int64_t L = e * no + n;
        const int64_t u = n >= no ? -1 : lid ? (int64_t)lid[L] : L;
        if (u < 0) v[c] = 0.0;                                         // Dirichlet node (or past no)
        else if (uoff) v[c] = (double)r[u] * rsqrt((double)(uoff[u + 1] - uoff[u]));  // S = mult^-1/2
        else if (mult) v[c] = (double)r[u] * rsqrt(mult[L]);
        else v[c] = (double)r[u];
        ss += v[c] * v[c];
    }
    ss = sem::wave_sum(ss);
    const double s = sqrt(ss) + 1e-30;
    const double kap = (double)kappa[e];
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (c * 64 + lane < no) X[row * nip + c * 64 + lane] = bf16_rne((float)(v[c] / s));
    if (lane < nip - no)
        X[row * nip + no + lane] = (lane < 6 && geo) ? bf16_rne(geo[e * 6 + lane]) : (u16)0;
    if (lane == 0 && scale) scale[row] = (float)(s / kap);
    if (Tt) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int n = c * 64 + lane;
            if (n >= no) continue;
            const int64_t L = e * no + n;
            const double ev = minv ? err[L] - minv[L] * v[c] : err[L];   // Jacobi base removed
            Tt[row * no + n] = (float)(ev * kap / s);
        }
    }
}

// z_L = (scale[e] * Y3[e][node] (+ minv_L r_L)) / mult_L, or with sym
// z_L = scale[e] * Y3[e][node] / sqrt(mult_L) (+ minv_L r_L / mult_L)
template <typename T>
__global__ void lp_output_kernel(T* __restrict__ z, const float* __restrict__ Y3,
                                 const float* __restrict__ scale, const double* __restrict__ mult,
                                 const double* __restrict__ minv, const T* __restrict__ r,
                                 int64_t n, const int* __restrict__ skip, bool sym, int no) {
    if (skip && *skip) return;
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x) {
        double v = (double)scale[L / no] * (double)Y3[L];
        if (sym) {     // S y + Minv r / mult; the gather-scatter sums the copies
            v *= rsqrt(mult[L]);
            if (minv) v += minv[L] * (double)r[L] / mult[L];
            z[L] = (T)v;
            continue;
        }
        if (minv) v += minv[L] * (double)r[L];
        z[L] = (T)(v / mult[L]);
    }
}

// unique layout: z_u = mean over the copies L of u of scale[e(L)] Y3[L], or with
// sym their sum weighted by mult_u^-1/2 (+ Minv_u r_u with the Jacobi base)
template <typename T>
__global__ void lp_output_unique_kernel(T* __restrict__ z, const float* __restrict__ Y3,
                                        const float* __restrict__ scale, const double* __restrict__ minv,
                                        const T* __restrict__ r, const int32_t* __restrict__ uoff,
                                        const int32_t* __restrict__ uidx, int64_t nu,
                                        const int* __restrict__ skip, bool sym, int no) {
    if (skip && *skip) return;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < nu;
         u += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = uoff[u], e = uoff[u + 1];
        double s = 0.0;
        for (int32_t q = b; q < e; ++q) {
            const int32_t L = uidx[q];
            s += (double)scale[L / no] * (double)Y3[L];
        }
        s *= sym ? rsqrt((double)(e - b)) : 1.0 / (double)(e - b);
        if (minv) s += minv[uidx[b]] * (double)r[u];
        z[u] = (T)s;
    }
}

// ---- linear form on unique-layout vectors ----------------------------------
// zl[upos[L]] = (1/kappa_e) sum_k Ws[n][k] S_k r_k for every local node
// L = (e, n) of an element, with S = mult^-1/2 (sl, per local node) and Ws the
// symmetric folded matrix, so that summing zl over the copies of a node and
// weighting by S gives the symmetric additive preconditioner.  Three passes:
// a gather of S r into element-major bf16 rows (many waves, so the dependent
// index -> value loads overlap), the product, and the assembly.  The product
// takes 64 elements per 256-thread block, 16 per wave as the rows of 16x16x32
// bf16 MFMA blocks: a wave keeps its 16 x 512 residual block in registers and
// its 16 x 512 outputs in 32 accumulator tiles while Ws streams through LDS in
// 32-wide k-slabs, the next slab fetched into registers during the current
// one's products.  The outputs land in CSR order, where the assembly reads
// each node's copies contiguously.
constexpr int kLinBK = 32, kLinSlabs = kOut / kLinBK;

__device__ __forceinline__ bf16x8 pack_bf16x8(const float* v) {
    uint4 w;
    w.x = (uint32_t)bf16_rne(v[0]) | ((uint32_t)bf16_rne(v[1]) << 16);
    w.y = (uint32_t)bf16_rne(v[2]) | ((uint32_t)bf16_rne(v[3]) << 16);
    w.z = (uint32_t)bf16_rne(v[4]) | ((uint32_t)bf16_rne(v[5]) << 16);
    w.w = (uint32_t)bf16_rne(v[6]) | ((uint32_t)bf16_rne(v[7]) << 16);
    return __builtin_bit_cast(bf16x8, w);
}

// r[u], or 0 for a Dirichlet node (u < 0)
template <typename T>
__device__ __forceinline__ float ld_free(const T* __restrict__ r, int32_t u) {
    return u >= 0 ? (float)r[u] : 0.0f;
}

// X[e][n] = bf16(S r) at the unique node of local node (e, n); 8 nodes per
// thread.  S comes per local node (sl, a coalesced stream), so r is the only
// gathered array.
template <typename T>
__global__ void lin_gather_kernel(u16* __restrict__ X, const T* __restrict__ r, const float* __restrict__ sl,
                                  const int32_t* __restrict__ lid, int64_t n8, const int* __restrict__ skip,
                                  int no, int nip) {
    if (skip && *skip) return;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n8;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t L = t * 8;
        const int4 i0 = *reinterpret_cast<const int4*>(lid + L);
        const int4 i1 = *reinterpret_cast<const int4*>(lid + L + 4);
        const float4 s0 = *reinterpret_cast<const float4*>(sl + L);
        const float4 s1 = *reinterpret_cast<const float4*>(sl + L + 4);
        float v[8];
        v[0] = ld_free(r, i0.x) * s0.x;
        v[1] = ld_free(r, i0.y) * s0.y;
        v[2] = ld_free(r, i0.z) * s0.z;
        v[3] = ld_free(r, i0.w) * s0.w;
        v[4] = ld_free(r, i1.x) * s1.x;
        v[5] = ld_free(r, i1.y) * s1.y;
        v[6] = ld_free(r, i1.z) * s1.z;
        v[7] = ld_free(r, i1.w) * s1.w;
        *reinterpret_cast<bf16x8*>(X + (L / no) * nip + (L % no)) = pack_bf16x8(v);
    }
}

// sl[L] = mult^-1/2 of local node L (0 on Dirichlet nodes)
__global__ void sl_kernel(float* __restrict__ sl, const int32_t* __restrict__ lid, const int32_t* __restrict__ uoff,
                          int64_t n) {
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x) {
        const int32_t u = lid[L];
        sl[L] = u >= 0 ? (float)(1.0 / sqrt((double)(uoff[u + 1] - uoff[u]))) : 0.0f;
    }
}

// zl[upos[L]] = (1/kappa_e) (Ws X_e)_n for every local node L = (e, n).
// Weight-stationary: block b owns half of Ws's rows (256 output nodes), each of
// its 8 waves 32 of them, held for the whole kernel as the B fragments of
// 16x16x32 bf16 MFMA blocks (128 registers).  The block walks over 16-element
// chunks of X (chunks g, g + groups, ...), staged through a double-buffered LDS
// tile with a two-chunk register prefetch.  The two halves of a group run 8 block
// indices apart, on the same XCD, so a chunk of X is read from HBM once.
constexpr int kWsChunk = 16, kWsLd = kOut + 8, kWsGroupsMax = 128;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));

// 16 bf16 of chunk c (element se of the chunk, columns sk .. sk + 15), zero past
// the end; the load always reads a valid row (clamped) and the select zeroes it
__device__ __forceinline__ u32x8 ws_load_chunk(const u16* __restrict__ X, int64_t c, int64_t nchunks, int64_t nel,
                                               int se, int sk) {
    const int64_t e = c * kWsChunk + se;
    const bool ok = c < nchunks && e < nel;
    const u16* p = X + (ok ? e : 0) * kInPad + sk;
    const u32x4 a = *reinterpret_cast<const u32x4*>(p), b = *reinterpret_cast<const u32x4*>(p + 8);
    const u32x8 v = u32x8{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    return ok ? v : u32x8{0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
}

__device__ __forceinline__ void ws_stage(u16* __restrict__ dst, u32x8 v) {
    *reinterpret_cast<u32x4*>(dst) = u32x4{v[0], v[1], v[2], v[3]};
    *reinterpret_cast<u32x4*>(dst + 8) = u32x4{v[4], v[5], v[6], v[7]};
}

__device__ __forceinline__ void ws_load_pos(int32_t (&pos)[2][4], float (&kinv)[4], const int32_t* __restrict__ upos,
                                            const float* __restrict__ kappa_inv, int64_t c, int64_t nel, int grp,
                                            int col) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        int64_t e = c * kWsChunk + 4 * grp + j;
        e = e < nel ? e : nel - 1;        // rows past the end read valid data and are not stored
        kinv[j] = kappa_inv[e];
        pos[0][j] = upos[e * kOut + col];
        pos[1][j] = upos[e * kOut + col + 16];
    }
}

// One chunk c.  Loads are issued in the order they are needed, because the
// vector-memory counter is waited on in order: first the next chunk's CSR
// positions and scales, then (after this chunk's products out of LDS buffer
// `buf` and its stores, which use positions fetched one step ago) the chunk
// `groups` ahead goes from its registers (fetched two steps ago) to the other
// buffer, and those registers start fetching the chunk three steps ahead.
// Two register sets alternate between consecutive steps.
__device__ __forceinline__ void ws_step(float* __restrict__ zl, const u16* __restrict__ X,
                                        const int32_t* __restrict__ upos, const float* __restrict__ kappa_inv,
                                        u16 (*sx)[kWsChunk * kWsLd], const bf16x8 (&w)[kLinSlabs][2],
                                        int64_t c, int buf, int64_t groups, int64_t nchunks, int64_t nel,
                                        u32x8& nx, const int32_t (&pos)[2][4], const float (&kinv)[4],
                                        int32_t (&pnext)[2][4], float (&knext)[4], int row, int grp, int col,
                                        int se, int sk) {
    ws_load_pos(pnext, knext, upos, kappa_inv, c + groups, nel, grp, col);
    f32x4 acc0 = f32x4{0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
    const u16* xs = sx[buf] + row * kWsLd + 8 * grp;
#pragma unroll
    for (int kb = 0; kb < kLinSlabs; ++kb) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(xs + kb * kLinBK);
        acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w[kb][0], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, w[kb][1], acc1, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (c * kWsChunk + 4 * grp + j < nel) {
            zl[pos[0][j]] = acc0[j] * kinv[j];
            zl[pos[1][j]] = acc1[j] * kinv[j];
        }
    }
    ws_stage(sx[buf ^ 1] + se * kWsLd + sk, nx);
    nx = ws_load_chunk(X, c + 3 * groups, nchunks, nel, se, sk);
    __syncthreads();
}

__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
lin_gemm_kernel(float* __restrict__ zl, const u16* __restrict__ X, const int32_t* __restrict__ upos,
                const float* __restrict__ kappa_inv, const u16* __restrict__ Ws, int64_t nel, int groups,
                const int* __restrict__ skip) {
    if (skip && *skip) return;
    __shared__ __attribute__((aligned(16))) u16 sx[2][kWsChunk * kWsLd];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int row = lane & 15, grp = lane >> 4;
    const int b = blockIdx.x;
    const int half = (b >> 3) & 1;
    const int64_t g = (b & 7) + 8 * (b >> 4);
    const int64_t nchunks = (nel + kWsChunk - 1) / kWsChunk;
    if (g >= nchunks) return;                 // uniform over the block, before any barrier
    const int col = half * 256 + wave * 32 + row;   // this lane's output node (and col + 16)

    bf16x8 w[kLinSlabs][2];
#pragma unroll
    for (int kb = 0; kb < kLinSlabs; ++kb)
#pragma unroll
        for (int t = 0; t < 2; ++t)
            w[kb][t] = *reinterpret_cast<const bf16x8*>(Ws + (int64_t)(col + 16 * t) * kOut + kb * kLinBK +
                                                        8 * grp);

    const int se = tid >> 5, sk = (tid & 31) * 16;   // staging: element se, columns sk .. sk + 15
    int32_t pos0[2][4], pos1[2][4];
    float kinv0[4], kinv1[4];
    ws_stage(sx[0] + se * kWsLd + sk, ws_load_chunk(X, g, nchunks, nel, se, sk));
    ws_load_pos(pos0, kinv0, upos, kappa_inv, g, nel, grp, col);
    // everything loaded so far (the W fragments above all) has arrived: the loop
    // below then carries no pending-load state for W, and its only waits are for
    // loads issued one (positions) or two (chunks) steps earlier
    __builtin_amdgcn_s_waitcnt(0);
    u32x8 nx0 = ws_load_chunk(X, g + groups, nchunks, nel, se, sk);
    u32x8 nx1 = ws_load_chunk(X, g + 2 * groups, nchunks, nel, se, sk);
    __syncthreads();

    for (int64_t c = g; c < nchunks; c += 2 * groups) {
        ws_step(zl, X, upos, kappa_inv, sx, w, c, 0, groups, nchunks, nel, nx0, pos0, kinv0, pos1, kinv1, row,
                grp, col, se, sk);
        if (c + groups >= nchunks) break;     // uniform over the block
        ws_step(zl, X, upos, kappa_inv, sx, w, c + groups, 1, groups, nchunks, nel, nx1, pos1, kinv1, pos0,
                kinv0, row, grp, col, se, sk);
    }
}

// z_u = S_u sum over the CSR segment of u of zl (+ Minv_u r_u with the Jacobi
// base, Minv on unique nodes)
template <typename T>
__global__ void lin_assemble_kernel(T* __restrict__ z, const float* __restrict__ zl,
                                    const double* __restrict__ minvu, const T* __restrict__ r,
                                    const int32_t* __restrict__ uoff, int64_t nu,
                                    const int* __restrict__ skip) {
    if (skip && *skip) return;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < nu;
         u += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = uoff[u], e = uoff[u + 1];
        float s = 0.f;
        for (int32_t q = b; q < e; ++q) s += zl[q];
        double v = (double)s * rsqrt((double)(e - b));
        if (minvu) v += minvu[u] * (double)r[u];
        z[u] = (T)v;
    }
}

// unique-layout copy of a continuous local field: out[u] = in[uidx[uoff[u]]]
__global__ void first_copy_kernel(double* __restrict__ out, const double* __restrict__ in,
                                  const int32_t* __restrict__ uoff, const int32_t* __restrict__ uidx,
                                  int64_t nu) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < nu;
         u += (int64_t)gridDim.x * blockDim.x)
        out[u] = in[uidx[uoff[u]]];
}

__global__ void zero_f32(float* __restrict__ x, int n) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) x[q] = 0.f;
}

// x = 1 / x, with 0 kept at 0 (Dirichlet nodes, zeroed by the gather-scatter)
__global__ void inv_kernel(double* __restrict__ x, int64_t n) {
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n;
         L += (int64_t)gridDim.x * blockDim.x)
        x[L] = x[L] != 0.0 ? 1.0 / x[L] : 0.0;
}

unsigned grid_of(int64_t n, int64_t cap = 4096) {
    int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

namespace {

// u[L] = 1 where ids[L] == g, else 0
__global__ void unit_id_kernel(double* __restrict__ u, const int64_t* __restrict__ ids, int64_t g, int64_t n) {
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n; L += (int64_t)gridDim.x * blockDim.x)
        u[L] = ids[L] == g ? 1.0 : 0.0;
}

}  // namespace

struct sem_lp_s {
    sem_ctx_t ctx = nullptr;
    int64_t max_rows = 0;
    // element size: lx, no = lx^3 outputs, ni = no + 6 inputs, nip = ni padded to 16;
    // nh the width of the two hidden layers
    int lx = 8, no = kOut, ni = kIn, nip = kInPad, nh = kHid;
    // the linear form's unique-layout product: 0 automatic (weight-stationary at
    // lx = 8, the general product otherwise), 1 weight-stationary, 2 general
    int product = 0;
    // float32 masters, Adam moments, gradients (W1 gradient is 256 x nip)
    float *W[3] = {}, *b[3] = {}, *mW[3] = {}, *mb[3] = {}, *vW[3] = {}, *vb[3] = {};
    float *gW[3] = {}, *gb[3] = {};
    int64_t step = 0;
    // bf16 copies: W1 (256 x nip), W2 (256 x 256), W3 (no x 256), W2^T, W3^T
    u16 *W1b = nullptr, *W2b = nullptr, *W3b = nullptr, *W2t = nullptr, *W3t = nullptr;
    double mu = -1.0;         // training metric (< 0: mean squared error)
    bool dirty = true;        // bf16 copies of the weights out of date
    bool fold_dirty = true;   // folded matrix of the linear form out of date
    float* colpart = nullptr; // column-sum partials (bias gradients)
    // activations / work for up to max_rows rows
    u16 *X = nullptr, *Y1 = nullptr, *Y2 = nullptr, *d3b = nullptr, *d2b = nullptr, *d1b = nullptr;
    float *Y3 = nullptr, *T = nullptr, *d3f = nullptr, *d2f = nullptr, *d1f = nullptr, *scale = nullptr;
    u16 *tA = nullptr, *tB = nullptr;   // transposes (nip x max_rows each)
    double* part = nullptr;
    float* loss = nullptr;
    // bound operator (inference)
    int64_t nel = 0, geo_cap = 0;
    float *geo = nullptr, *kappa = nullptr, *kappa_inv = nullptr;
    bool bound = false;
    sem_gs_t gs = nullptr;
    sem::AxArgs A64{};        // the bound operator (float64 arrays of the caller)
    const int* skip = nullptr;   // set by the solver: kernels return when *skip != 0
    // energy-norm loss: metric K (no x no, bf16) and work arrays
    u16* K = nullptr;
    float *dF = nullptr, *Kd = nullptr;
    u16* dB = nullptr;
    // linear form: identity activations, no biases, geometric inputs zeroed;
    // inference then uses the folded matrix (W3 W2 W1)[:, :no] (bf16)
    bool linear = false;
    float *T32 = nullptr, *Wf32 = nullptr;
    u16* Wfb = nullptr;
    // Jacobi base: z = Minv r + network correction (Minv of the bound operator)
    bool jacobi_base = false;
    double* minv = nullptr;
    int64_t minv_n = 0;
    float* sl = nullptr;      // mult^-1/2 per local node of the bound plan
    int64_t sl_n = 0;
    double* minvu = nullptr;  // Minv on the unique nodes of the bound plan (Jacobi base)
    int64_t minvu_n = 0;
    std::vector<void*> allocs;
};

namespace {

int param_rows(const sem_lp_s* lp, int layer) { return layer == 2 ? lp->no : lp->nh; }
int param_cols(const sem_lp_s* lp, int layer) { return layer == 0 ? lp->ni : lp->nh; }

int lp_alloc(sem_lp_t lp, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return sem::check_hip(lp->ctx, e, "sem_lp: hipMalloc");
    lp->allocs.push_back(*p);
    SEM_HIP(lp->ctx, hipMemsetAsync(*p, 0, bytes, lp->ctx->stream));
    return SEM_OK;
}

int gemm(sem_lp_t lp, int M, int N, int K, const u16* A, int lda, const u16* B, int ldb,
         const float* bias, const u16* mask, int ldm, float* Cf, u16* Cb, int ldc, int epi,
         const float* rowscale = nullptr, const int32_t* pos = nullptr) {
    if (M == 0 || N == 0) return SEM_OK;
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM);
    gemm_nt<<<grid, 256, 0, lp->ctx->stream>>>(M, N, K, A, lda, B, ldb, bias, mask, ldm, Cf, Cb, ldc, epi,
                                               lp->skip, rowscale, pos);
    SEM_LAUNCH_CHECK(lp->ctx);
    return SEM_OK;
}

// features_kernel for this network's element size (ceil(no / 64) nodes per lane)
template <typename T>
int launch_features(sem_lp_t lp, int64_t count, u16* X, float* scale, float* Tt, const T* r, const double* err,
                    const double* minv, const float* geo, const int64_t* elems, int64_t row0, const int* skip,
                    const int32_t* lid, const int32_t* uoff, const double* mult) {
    hipStream_t st = lp->ctx->stream;
    const unsigned g = (unsigned)count;
#define LP_FEAT(NC) features_kernel<T, NC><<<g, 64, 0, st>>>(X, scale, Tt, r, err, minv, geo, lp->kappa, elems, \
                                                              count, row0, skip, lid, uoff, mult, lp->no, lp->nip)
    switch ((lp->no + 63) / 64) {
        case 1: LP_FEAT(1); break;
        case 4: LP_FEAT(4); break;
        case 8: LP_FEAT(8); break;
        case 16: LP_FEAT(16); break;
        case 27: LP_FEAT(27); break;
        default: return sem::fail(lp->ctx, SEM_EUNSUPPORTED_LX, "sem_lp: element size %d", lp->no);
    }
#undef LP_FEAT
    SEM_LAUNCH_CHECK(lp->ctx);
    return SEM_OK;
}

int transpose(sem_lp_t lp, u16* out, int ldo, const u16* in, int ldi, int rows, int cols) {
    dim3 grid((cols + 31) / 32, (rows + 31) / 32);
    transpose_bf16<<<grid, 256, 0, lp->ctx->stream>>>(out, ldo, in, ldi, rows, cols);
    SEM_LAUNCH_CHECK(lp->ctx);
    return SEM_OK;
}

int refresh_bf16(sem_lp_t lp) {
    const int kHid = lp->nh;     // this network's hidden width
    if (!lp->dirty) return SEM_OK;
    hipStream_t st = lp->ctx->stream;
    weights_to_bf16<<<256, kBlock, 0, st>>>(lp->W1b, lp->nip, nullptr, lp->W[0], kHid, lp->ni);
    weights_to_bf16<<<256, kBlock, 0, st>>>(lp->W2b, kHid, lp->W2t, lp->W[1], kHid, kHid);
    weights_to_bf16<<<256, kBlock, 0, st>>>(lp->W3b, kHid, lp->W3t, lp->W[2], lp->no, kHid);
    SEM_LAUNCH_CHECK(lp->ctx);
    lp->dirty = false;
    return SEM_OK;
}

// symmetric part of the folded (W3 W2 W1)[:, :no] of the linear form, in bf16;
// needed by inference only, so training steps do not recompute it
int refresh_fold(sem_lp_t lp) {
    const int kHid = lp->nh;     // this network's hidden width
    int rc = refresh_bf16(lp);
    if (rc || !lp->fold_dirty || !lp->linear || !lp->Wfb) return rc;
    hipStream_t st = lp->ctx->stream;
    const int no = lp->no;
    matmul_f32<<<dim3((kHid + 255) / 256, no), 256, 0, st>>>(lp->T32, lp->W[2], lp->W[1], no, kHid,
                                                             kHid, kHid, kHid, kHid);
    matmul_f32<<<dim3((no + 255) / 256, no), 256, 0, st>>>(lp->Wf32, lp->T32, lp->W[0], no, kHid,
                                                           no, kHid, lp->ni, no);
    sym_to_bf16<<<256, kBlock, 0, st>>>(lp->Wfb, lp->Wf32, no);
    SEM_LAUNCH_CHECK(lp->ctx);
    lp->fold_dirty = false;
    return SEM_OK;
}

// forward of rows [0, M) of lp->X into Y1, Y2 (bf16) and Y3 (float)
int forward(sem_lp_t lp, const u16* X, int64_t M) {
    const int kHid = lp->nh;     // this network's hidden width
    int rc = refresh_bf16(lp);
    if (rc) return rc;
    if (M > 0x7fffffff) return sem::fail(lp->ctx, SEM_EINVAL, "sem_lp: too many rows");
    const int m = (int)M;
    const int hid = lp->linear ? 0 : EPI_BIAS | EPI_RELU, out = lp->linear ? 0 : EPI_BIAS;
    rc = gemm(lp, m, kHid, lp->nip, X, lp->nip, lp->W1b, lp->nip, lp->b[0], nullptr, 0, nullptr, lp->Y1, kHid, hid);
    if (!rc) rc = gemm(lp, m, kHid, kHid, lp->Y1, kHid, lp->W2b, kHid, lp->b[1], nullptr, 0, nullptr, lp->Y2, kHid, hid);
    if (!rc) rc = gemm(lp, m, lp->no, kHid, lp->Y2, kHid, lp->W3b, kHid, lp->b[2], nullptr, 0, lp->Y3, nullptr, lp->no, out);
    return rc;
}

float** param_slot(sem_lp_t lp, int which, int64_t* count, int* ld) {
    // 0..5 params, 6..11 first moments, 12..17 second moments, 18..23 gradients
    const int kind = which / 6, idx = which % 6, layer = idx / 2;
    const bool isW = (idx % 2) == 0;
    *count = isW ? (int64_t)param_rows(lp, layer) * param_cols(lp, layer) : param_rows(lp, layer);
    *ld = isW ? param_cols(lp, layer) : 1;
    if (kind == 3 && isW && layer == 0) *ld = lp->nip;
    switch (kind) {
        case 0: return isW ? &lp->W[layer] : &lp->b[layer];
        case 1: return isW ? &lp->mW[layer] : &lp->mb[layer];
        case 2: return isW ? &lp->vW[layer] : &lp->vb[layer];
        case 3: return isW ? &lp->gW[layer] : &lp->gb[layer];
    }
    return nullptr;
}

}  // namespace

extern "C" int sem_lp_create_lx(sem_ctx_t ctx, int lx, int hidden, int64_t max_rows, sem_lp_t* out) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!out) return sem::fail(ctx, SEM_EINVAL, "sem_lp_create: null output");
    *out = nullptr;
    if (lx < 4 || lx > SEM_LX_MAX || lx % 2)
        return sem::fail(ctx, SEM_EUNSUPPORTED_LX, "sem_lp_create: lx=%d (the network takes even lx in [4, %d])", lx,
                         SEM_LX_MAX);
    if (max_rows < 1 || max_rows > (1ll << 26))
        return sem::fail(ctx, SEM_EINVAL, "sem_lp_create: max_rows=%lld outside [1, 2^26]", (long long)max_rows);
    if (hidden == 0) hidden = kHid;
    if (hidden < 16 || hidden > 1024 || hidden % 16)
        return sem::fail(ctx, SEM_EINVAL, "sem_lp_create: hidden width %d (a multiple of 16 in [16, 1024])", hidden);
    auto* lp = new sem_lp_s();
    lp->ctx = ctx;
    lp->max_rows = max_rows;
    lp->lx = lx;
    lp->nh = hidden;
    const int kHid = hidden;
    lp->no = lx * lx * lx;
    lp->ni = lp->no + 6;
    lp->nip = (lp->ni + 15) / 16 * 16;
    const int no = lp->no, nip = lp->nip;
    auto bail = [&](int code) { sem_lp_destroy(lp); return code; };
#define LP_ALLOC(ptr, bytes) do { int rc_ = lp_alloc(lp, (void**)&(ptr), (bytes)); if (rc_) return bail(rc_); } while (0)
    for (int l = 0; l < 3; ++l) {
        const size_t nw = (size_t)param_rows(lp, l) * param_cols(lp, l), nb = param_rows(lp, l);
        LP_ALLOC(lp->W[l], 4 * nw); LP_ALLOC(lp->mW[l], 4 * nw); LP_ALLOC(lp->vW[l], 4 * nw);
        LP_ALLOC(lp->b[l], 4 * nb); LP_ALLOC(lp->mb[l], 4 * nb); LP_ALLOC(lp->vb[l], 4 * nb);
        LP_ALLOC(lp->gW[l], 4 * (size_t)param_rows(lp, l) * (l == 0 ? nip : param_cols(lp, l)));
        LP_ALLOC(lp->gb[l], 4 * nb);
    }
    LP_ALLOC(lp->W1b, 2 * (size_t)kHid * nip);
    LP_ALLOC(lp->W2b, 2 * (size_t)kHid * kHid);
    LP_ALLOC(lp->W3b, 2 * (size_t)no * kHid);
    LP_ALLOC(lp->W2t, 2 * (size_t)kHid * kHid);
    LP_ALLOC(lp->W3t, 2 * (size_t)kHid * no);
    const size_t R = (size_t)max_rows;
    LP_ALLOC(lp->X, 2 * R * nip);
    LP_ALLOC(lp->Y1, 2 * R * kHid);
    LP_ALLOC(lp->Y2, 2 * R * kHid);
    LP_ALLOC(lp->Y3, 4 * R * no);
    LP_ALLOC(lp->T, 4 * R * no);
    LP_ALLOC(lp->scale, 4 * R);
    LP_ALLOC(lp->part, 8 * 4096);
    LP_ALLOC(lp->loss, 4);
#undef LP_ALLOC
    SEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *out = lp;
    return SEM_OK;
}

extern "C" int sem_lp_create(sem_ctx_t ctx, int64_t max_rows, sem_lp_t* out) {
    return sem_lp_create_lx(ctx, 8, kHid, max_rows, out);
}

extern "C" int sem_lp_lx(sem_lp_t lp, int* lx, int* hidden) {
    if (!lp || !lx) return sem::fail(lp ? lp->ctx : nullptr, SEM_EINVAL, "sem_lp_lx: null argument");
    *lx = lp->lx;
    if (hidden) *hidden = lp->nh;
    return SEM_OK;
}

extern "C" int sem_lp_destroy(sem_lp_t lp) {
    if (!lp) return SEM_OK;
    if (lp->ctx) {
        (void)hipSetDevice(lp->ctx->device);
        (void)hipStreamSynchronize(lp->ctx->stream);
    }
    for (void* p : lp->allocs) (void)hipFree(p);
    delete lp;
    return SEM_OK;
}

extern "C" int sem_lp_set(sem_lp_t lp, int which, const float* host, int64_t count) {
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_set: null network");
    int rc = sem::enter(lp->ctx);
    if (rc) return rc;
    if (which < 0 || which >= 24 || !host) return sem::fail(lp->ctx, SEM_EINVAL, "sem_lp_set: bad slot %d", which);
    int64_t n;
    int ld;
    float** slot = param_slot(lp, which, &n, &ld);
    if (count != n) return sem::fail(lp->ctx, SEM_EINVAL, "sem_lp_set: slot %d holds %lld values, got %lld",
                                     which, (long long)n, (long long)count);
    SEM_HIP(lp->ctx, hipStreamSynchronize(lp->ctx->stream));
    if (which == 18) {   // W1 gradient: nh x ni values into an nh x nip array
        for (int r = 0; r < lp->nh; ++r)
            SEM_HIP(lp->ctx, hipMemcpy(*slot + (size_t)r * ld, host + (size_t)r * lp->ni, 4 * (size_t)lp->ni,
                                       hipMemcpyHostToDevice));
    } else {
        SEM_HIP(lp->ctx, hipMemcpy(*slot, host, 4 * (size_t)n, hipMemcpyHostToDevice));
    }
    if (which < 6) lp->dirty = lp->fold_dirty = true;
    return SEM_OK;
}

extern "C" int sem_lp_get(sem_lp_t lp, int which, float* host, int64_t count) {
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_get: null network");
    int rc = sem::enter(lp->ctx);
    if (rc) return rc;
    if (which < 0 || which >= 24 || !host) return sem::fail(lp->ctx, SEM_EINVAL, "sem_lp_get: bad slot %d", which);
    int64_t n;
    int ld;
    float** slot = param_slot(lp, which, &n, &ld);
    if (count != n) return sem::fail(lp->ctx, SEM_EINVAL, "sem_lp_get: slot %d holds %lld values, got %lld",
                                     which, (long long)n, (long long)count);
    SEM_HIP(lp->ctx, hipStreamSynchronize(lp->ctx->stream));
    if (which == 18) {
        for (int r = 0; r < lp->nh; ++r)
            SEM_HIP(lp->ctx, hipMemcpy(host + (size_t)r * lp->ni, *slot + (size_t)r * ld, 4 * (size_t)lp->ni,
                                       hipMemcpyDeviceToHost));
    } else {
        SEM_HIP(lp->ctx, hipMemcpy(host, *slot, 4 * (size_t)n, hipMemcpyDeviceToHost));
    }
    return SEM_OK;
}

extern "C" int sem_lp_set_step(sem_lp_t lp, int64_t step) {
    if (!lp || step < 0) return sem::fail(lp ? lp->ctx : nullptr, SEM_EINVAL, "sem_lp_set_step: bad argument");
    lp->step = step;
    return SEM_OK;
}

extern "C" int sem_lp_get_step(sem_lp_t lp, int64_t* step) {
    if (!lp || !step) return sem::fail(lp ? lp->ctx : nullptr, SEM_EINVAL, "sem_lp_get_step: bad argument");
    *step = lp->step;
    return SEM_OK;
}

extern "C" int sem_lp_set_metric(sem_lp_t lp, double mu) {
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_set_metric: null network");
    sem_ctx_t ctx = lp->ctx;
    int rc = sem::enter(ctx);
    if (rc) return rc;
    lp->mu = mu < 0 ? -1.0 : mu;
    if (mu < 0) {            // back to the plain mean squared error
        lp->K = nullptr;
        return SEM_OK;
    }
    const int lx = lp->lx, kOut = lp->no;
    std::vector<double> xi(lx), w(lx), D((size_t)lx * lx);   // D[m*lx + i] = l_i'(xi_m)
    sem::gll_host(lx, xi.data(), w.data(), D.data());
    std::vector<double> Kh((size_t)lx * lx);   // 1-D stiffness sum_m w_m l_i'(xi_m) l_i''(xi_m)
    for (int i = 0; i < lx; ++i)
        for (int ip = 0; ip < lx; ++ip) {
            double s = 0.0;
            for (int m = 0; m < lx; ++m) s += w[m] * D[m * lx + i] * D[m * lx + ip];
            Kh[(size_t)i * lx + ip] = s;
        }
    double wsum = 0.0;
    for (int i = 0; i < lx; ++i) wsum += w[i];
    const double kappa = std::pow(wsum / lx, 3);     // mean of w_i w_j w_k
    std::vector<u16> Kb((size_t)kOut * kOut);
    for (int p = 0; p < kOut; ++p) {
        const int i = p % lx, j = (p / lx) % lx, k = p / (lx * lx);
        for (int q = 0; q < kOut; ++q) {
            const int ip = q % lx, jp = (q / lx) % lx, kp = q / (lx * lx);
            double v = 0.0;
            if (j == jp && k == kp) v += Kh[(size_t)i * lx + ip] * w[j] * w[k];
            if (i == ip && k == kp) v += w[i] * Kh[(size_t)j * lx + jp] * w[k];
            if (i == ip && j == jp) v += w[i] * w[j] * Kh[(size_t)k * lx + kp];
            v /= kappa;
            if (p == q) v += mu * w[i] * w[j] * w[k] / kappa;
            const float f = (float)v;
            uint32_t b;
            std::memcpy(&b, &f, 4);
            b += 0x7fffu + ((b >> 16) & 1u);
            Kb[(size_t)p * kOut + q] = (u16)(b >> 16);
        }
    }
    if (!lp->K) {
        const size_t R = (size_t)lp->max_rows;
        void* p = nullptr;
        rc = lp_alloc(lp, &p, 2 * (size_t)kOut * kOut);
        if (rc) return rc;
        lp->K = (u16*)p;
        rc = lp_alloc(lp, &p, 4 * R * kOut);
        if (rc) return rc;
        lp->dF = (float*)p;
        rc = lp_alloc(lp, &p, 4 * R * kOut);
        if (rc) return rc;
        lp->Kd = (float*)p;
        rc = lp_alloc(lp, &p, 2 * R * kOut);
        if (rc) return rc;
        lp->dB = (u16*)p;
    }
    SEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    SEM_HIP(ctx, hipMemcpy(lp->K, Kb.data(), 2 * Kb.size(), hipMemcpyHostToDevice));
    return SEM_OK;
}

extern "C" int sem_lp_set_linear(sem_lp_t lp, int on) {
    const int kHid = lp->nh;     // this network's hidden width
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_set_linear: null network");
    int rc = sem::enter(lp->ctx);
    if (rc) return rc;
    lp->linear = on != 0;
    if (lp->linear && !lp->Wfb) {
        const size_t no = (size_t)lp->no;
        void* p = nullptr;
        rc = lp_alloc(lp, &p, 4 * no * kHid);
        if (rc) return rc;
        lp->T32 = (float*)p;
        rc = lp_alloc(lp, &p, 4 * no * no);
        if (rc) return rc;
        lp->Wf32 = (float*)p;
        rc = lp_alloc(lp, &p, 2 * no * no);
        if (rc) return rc;
        lp->Wfb = (u16*)p;
    }
    lp->dirty = lp->fold_dirty = true;
    return SEM_OK;
}

extern "C" int sem_lp_set_jacobi_base(sem_lp_t lp, int on) {
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_set_jacobi_base: null network");
    lp->jacobi_base = on != 0;
    lp->bound = false;    // a new bind is required
    return SEM_OK;
}

extern "C" int sem_lp_bind(sem_lp_t lp, const sem_operator_t* A, sem_gs_t gs) {
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_bind: null network");
    sem_ctx_t ctx = lp->ctx;
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!A || !gs) return sem::fail(ctx, SEM_EINVAL, "sem_lp_bind: null operator or plan");
    if (A->lx != lp->lx)
        return sem::fail(ctx, SEM_EUNSUPPORTED_LX, "sem_lp_bind: the network is built for lx = %d, got %d", lp->lx, A->lx);
    if (A->nel < 1 || A->nel > lp->max_rows)
        return sem::fail(ctx, SEM_EINVAL, "sem_lp_bind: nel=%lld outside [1, max_rows=%lld]",
                         (long long)A->nel, (long long)lp->max_rows);
    if (gs->n_local != A->nel * lp->no) return sem::fail(ctx, SEM_EINVAL, "sem_lp_bind: plan size mismatch");
    if (!A->g11 || !A->g22 || !A->g33 || !A->g12 || !A->g13 || !A->g23)
        return sem::fail(ctx, SEM_EINVAL, "sem_lp_bind: null geometric factor");
    if (lp->geo_cap < A->nel) {
        lp->geo_cap = A->nel;
        void* p = nullptr;
        rc = lp_alloc(lp, &p, 4 * 6 * (size_t)A->nel);
        if (rc) return rc;
        lp->geo = (float*)p;
        rc = lp_alloc(lp, &p, 4 * (size_t)A->nel);
        if (rc) return rc;
        lp->kappa = (float*)p;
        rc = lp_alloc(lp, &p, 4 * (size_t)A->nel);
        if (rc) return rc;
        lp->kappa_inv = (float*)p;
    }
    lp->nel = A->nel;
    lp->gs = gs;
    lp->bound = true;
    lp->A64 = sem::AxArgs{};
    {
        const double* Dp[6] = {A->dx, A->dy, A->dz, A->dxt, A->dyt, A->dzt};
        const double* Gp[6] = {A->g11, A->g22, A->g33, A->g12, A->g13, A->g23};
        for (int q = 0; q < 6; ++q) { lp->A64.D[q] = Dp[q]; lp->A64.G[q] = Gp[q]; }
    }
    lp->A64.h1 = A->h1;
    lp->A64.nel = A->nel;
    lp->A64.lx = A->lx;
    geo_kernel<<<(unsigned)A->nel, 64, 0, ctx->stream>>>(lp->geo, lp->kappa, lp->kappa_inv, A->h1, A->g11, A->g22, A->g33,
                                                         A->g12, A->g13, A->g23, A->nel, lp->no);
    SEM_LAUNCH_CHECK(ctx);
    if (lp->sl_n < gs->n_local) {
        void* p = nullptr;
        rc = lp_alloc(lp, &p, 4 * (size_t)gs->n_local);
        if (rc) return rc;
        lp->sl = (float*)p;
        lp->sl_n = gs->n_local;
    }
    sl_kernel<<<grid_of(gs->n_local), kBlock, 0, ctx->stream>>>(lp->sl, gs->lid, gs->uoff, gs->n_local);
    SEM_LAUNCH_CHECK(ctx);
    if (lp->jacobi_base) {
        const int64_t n = A->nel * lp->no;
        if (lp->minv_n < n) {
            void* p = nullptr;
            rc = lp_alloc(lp, &p, 8 * (size_t)n);
            if (rc) return rc;
            lp->minv = (double*)p;
            lp->minv_n = n;
        }
        rc = sem_ax_diag(ctx, lp->minv, A->dx, A->h1, A->g11, A->g22, A->g33, A->g12, A->g13, A->g23,
                         A->nel, A->lx);
        if (rc) return rc;
        rc = sem_gs(gs, lp->minv, SEM_F64);
        if (rc) return rc;
        inv_kernel<<<grid_of(n), kBlock, 0, ctx->stream>>>(lp->minv, n);
        SEM_LAUNCH_CHECK(ctx);
        if (lp->minvu_n < gs->n_unique) {
            void* p = nullptr;
            rc = lp_alloc(lp, &p, 8 * (size_t)gs->n_unique);
            if (rc) return rc;
            lp->minvu = (double*)p;
            lp->minvu_n = gs->n_unique;
        }
        first_copy_kernel<<<grid_of(gs->n_unique), kBlock, 0, ctx->stream>>>(lp->minvu, lp->minv, gs->uoff,
                                                                             gs->uidx, gs->n_unique);
        SEM_LAUNCH_CHECK(ctx);
    }
    return SEM_OK;
}

extern "C" int sem_lp_samples(sem_lp_t lp, const double* r, const double* err, const int64_t* elems,
                              int64_t count, uint16_t* X, float* T, int64_t row0) {
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_samples: null network");
    sem_ctx_t ctx = lp->ctx;
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!lp->bound) return sem::fail(ctx, SEM_EINVAL, "sem_lp_samples: bind an operator first");
    if (!r || !X || !elems || count < 0 || row0 < 0 || (T && !err))
        return sem::fail(ctx, SEM_EINVAL, "sem_lp_samples: bad argument");
    if (count == 0) return SEM_OK;
    return launch_features<double>(lp, count, X, nullptr, T, r, err, lp->jacobi_base ? lp->minv : nullptr,
                                   lp->linear ? nullptr : lp->geo, elems, row0, nullptr, nullptr, nullptr, nullptr);
}

namespace {

// r = b - r (r holds the assembled A x), err = xstar - x
__global__ void pair_kernel(double* __restrict__ r, double* __restrict__ err, const double* __restrict__ b,
                            const double* __restrict__ x, const double* __restrict__ xstar, int64_t n) {
    for (int64_t L = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; L < n; L += (int64_t)gridDim.x * blockDim.x) {
        r[L] = b[L] - r[L];
        err[L] = xstar[L] - x[L];
    }
}

}  // namespace

extern "C" int sem_lp_snapshot(sem_lp_t lp, const double* x, const double* xstar, const double* b,
                               double* r_out, double* err_out, const int64_t* elems, int64_t count,
                               uint16_t* X, float* T, int64_t row0) {
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_snapshot: null network");
    sem_ctx_t ctx = lp->ctx;
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!lp->bound) return sem::fail(ctx, SEM_EINVAL, "sem_lp_snapshot: bind an operator first");
    if (!x || !xstar || !b || !r_out || !err_out || !X || !T || !elems || count < 0 || row0 < 0)
        return sem::fail(ctx, SEM_EINVAL, "sem_lp_snapshot: bad argument");
    const double* outs[2] = {r_out, err_out};
    const double* ins[3] = {x, xstar, b};
    for (const double* o : outs)
        for (const double* i : ins)
            if (o == i) return sem::fail(ctx, SEM_EINVAL, "sem_lp_snapshot: an output aliases an input");
    if (r_out == err_out) return sem::fail(ctx, SEM_EINVAL, "sem_lp_snapshot: r_out aliases err_out");
    const int64_t n = lp->gs->n_local;
    rc = sem::launch_ax(ctx, sem::AxKind::F64, lp->A64, r_out, x, nullptr, nullptr, nullptr);
    if (rc) return rc;
    rc = sem::gs_launch(lp->gs, r_out, SEM_F64, nullptr);
    if (rc) return rc;
    pair_kernel<<<grid_of(n, 8192), kBlock, 0, ctx->stream>>>(r_out, err_out, b, x, xstar, n);
    SEM_LAUNCH_CHECK(ctx);
    return sem_lp_samples(lp, r_out, err_out, elems, count, X, T, row0);
}

extern "C" int sem_lp_reference_block(sem_ctx_t ctx, int lx, double* W) {
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!sem::lx_ok(lx)) return sem::fail(ctx, SEM_EUNSUPPORTED_LX, "sem_lp_reference_block: lx=%d", lx);
    if (!W) return sem::fail(ctx, SEM_EINVAL, "sem_lp_reference_block: null output");
    const int n = 3, ecen = 13;                     // the centre element of the undeformed periodic 3^3 box
    const int nel = n * n * n, l2 = lx * lx, nloc = l2 * lx;
    const int64_t nl = (int64_t)nel * nloc;
    hipStream_t st = ctx->stream;
    std::vector<void*> tmp;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);
        for (void* p : tmp) (void)hipFree(p);
    };
    auto alloc = [&](void** p, size_t bytes) -> int {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) return sem::check_hip(ctx, e, "sem_lp_reference_block: hipMalloc");
        tmp.push_back(*p);
        return SEM_OK;
    };
#define RB_TRY(call) do { int rc_ = (call); if (rc_) { cleanup(); return rc_; } } while (0)
    double *x, *y, *z, *u, *w, *cols, *Dd;
    double* G[6];
    int64_t* ids;
    RB_TRY(alloc((void**)&x, 8 * nl));
    RB_TRY(alloc((void**)&y, 8 * nl));
    RB_TRY(alloc((void**)&z, 8 * nl));
    RB_TRY(alloc((void**)&u, 8 * nl));
    RB_TRY(alloc((void**)&w, 8 * nl));
    RB_TRY(alloc((void**)&cols, 8 * (size_t)nloc * nloc));
    RB_TRY(alloc((void**)&Dd, 8 * 2 * (size_t)l2));
    RB_TRY(alloc((void**)&ids, 8 * nl));
    for (int a = 0; a < 6; ++a) RB_TRY(alloc((void**)&G[a], 8 * nl));
    RB_TRY(sem_box_mesh(ctx, n, lx, 0.0, x, y, z, ids));
    RB_TRY(sem_geometry(ctx, x, y, z, nel, lx, G[0], G[1], G[2], G[3], G[4], G[5], nullptr, nullptr));
    std::vector<int64_t> hids(nl);
    RB_TRY(sem::check_hip(ctx, hipStreamSynchronize(st), "sem_lp_reference_block: sync"));
    RB_TRY(sem::check_hip(ctx, hipMemcpy(hids.data(), ids, 8 * nl, hipMemcpyDeviceToHost), "hipMemcpy"));
    sem_gs_t gs = nullptr;
    RB_TRY(sem_gs_setup(ctx, hids.data(), nl, &gs));
    std::vector<double> dx(l2), dxt(l2);
    sem_gll(lx, nullptr, nullptr, dx.data(), dxt.data());
    RB_TRY(sem::check_hip(ctx, hipMemcpy(Dd, dx.data(), 8 * l2, hipMemcpyHostToDevice), "hipMemcpy"));
    RB_TRY(sem::check_hip(ctx, hipMemcpy(Dd + l2, dxt.data(), 8 * l2, hipMemcpyHostToDevice), "hipMemcpy"));
    sem::AxArgs a{};
    for (int q = 0; q < 3; ++q) { a.D[q] = Dd; a.D[3 + q] = Dd + l2; }
    for (int q = 0; q < 6; ++q) a.G[q] = G[q];
    a.nel = nel;
    a.lx = lx;
    // column j: A_G applied to the unit vector of the centre element's node j
    // (every local copy set), read back on the centre element
    for (int j = 0; j < nloc; ++j) {
        unit_id_kernel<<<grid_of(nl, 8192), kBlock, 0, st>>>(u, ids, hids[(int64_t)ecen * nloc + j], nl);
        rc = sem::launch_ax(ctx, sem::AxKind::F64, a, w, u, nullptr, nullptr, nullptr);
        if (!rc) rc = sem::gs_launch(gs, w, SEM_F64, nullptr);
        if (rc) { sem_gs_destroy(gs); cleanup(); return rc; }
        rc = sem::check_hip(ctx, hipMemcpyAsync(cols + (size_t)j * nloc, w + (int64_t)ecen * nloc, 8 * (size_t)nloc,
                                                hipMemcpyDeviceToDevice, st), "hipMemcpyAsync");
        if (rc) { sem_gs_destroy(gs); cleanup(); return rc; }
    }
    sem_gs_destroy(gs);
    std::vector<double> A((size_t)nloc * nloc), g(3 * (size_t)nloc);
    RB_TRY(sem::check_hip(ctx, hipStreamSynchronize(st), "sem_lp_reference_block: sync"));
    RB_TRY(sem::check_hip(ctx, hipMemcpy(A.data(), cols, 8 * (size_t)nloc * nloc, hipMemcpyDeviceToHost), "hipMemcpy"));
    for (int q = 0; q < 3; ++q)
        RB_TRY(sem::check_hip(ctx, hipMemcpy(g.data() + (size_t)q * nloc, G[q] + (int64_t)ecen * nloc, 8 * (size_t)nloc,
                                             hipMemcpyDeviceToHost), "hipMemcpy"));
    cleanup();
#undef RB_TRY
    // A is stored by columns; it is symmetric up to rounding: symmetrise
    for (int i = 0; i < nloc; ++i)
        for (int j = i + 1; j < nloc; ++j) {
            const double v = 0.5 * (A[(size_t)i * nloc + j] + A[(size_t)j * nloc + i]);
            A[(size_t)i * nloc + j] = A[(size_t)j * nloc + i] = v;
        }
    double kappa = 0.0;
    for (int L = 0; L < nloc; ++L) kappa += g[L] + g[nloc + L] + g[2 * nloc + L];
    kappa /= 3.0 * nloc;
    if (!sem::spd_inverse(A, nloc))
        return sem::fail(ctx, SEM_EBREAKDOWN, "sem_lp_reference_block: element matrix not positive definite");
    for (size_t q = 0; q < A.size(); ++q) W[q] = kappa * A[q];
    return SEM_OK;
}

extern "C" int sem_lp_forward(sem_lp_t lp, const uint16_t* X, int64_t rows, float* Y) {
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_forward: null network");
    sem_ctx_t ctx = lp->ctx;
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!X || !Y || rows < 0 || rows > lp->max_rows) return sem::fail(ctx, SEM_EINVAL, "sem_lp_forward: bad argument");
    if (rows == 0) return SEM_OK;
    rc = forward(lp, X, rows);
    if (rc) return rc;
    SEM_HIP(ctx, hipMemcpyAsync(Y, lp->Y3, 4 * (size_t)rows * lp->no, hipMemcpyDeviceToDevice, ctx->stream));
    return SEM_OK;
}

static void colsum(sem_lp_t lp, float* out, const float* d, int rows, int cols) {
    hipStream_t st = lp->ctx->stream;
    const int chunks = (rows + kColRows - 1) / kColRows;
    colsum_part<<<dim3((cols + 63) / 64, chunks), 256, 0, st>>>(lp->colpart, d, rows, cols);
    colsum_final<<<(cols + 255) / 256, 256, 0, st>>>(out, lp->colpart, chunks, cols);
}

// gradients of the batch loss into the gradient slots (and the loss into *loss_dev)
static int lp_backward(sem_lp_t lp, const uint16_t* Xb, const float* Tb, int B) {
    const int kHid = lp->nh;     // this network's hidden width
    sem_ctx_t ctx = lp->ctx;
    hipStream_t st = ctx->stream;
    int rc = forward(lp, Xb, B);
    if (rc) return rc;
    const int kOut = lp->no, kInPad = lp->nip;     // this network's sizes
    const int64_t n3 = (int64_t)B * kOut;
    const unsigned g = grid_of(n3);
    if (lp->K) {
        // loss = mean_b d_b^T K d_b, gradient 2 K d / B
        diff_kernel<<<g, kBlock, 0, st>>>(lp->dF, lp->dB, lp->Y3, Tb, n3);
        rc = gemm(lp, B, kOut, kOut, lp->dB, kOut, lp->K, kOut, nullptr, nullptr, 0, lp->Kd, nullptr, kOut, 0);
        if (rc) return rc;
        metric_grad<<<g, kBlock, 0, st>>>(lp->d3f, lp->d3b, lp->dF, lp->Kd, n3, 2.0f / (float)B, lp->part);
        loss_final<<<1, 256, 0, st>>>(lp->loss, lp->part, (int)g, 1.0 / (double)B);
    } else {
        mse_grad<<<g, kBlock, 0, st>>>(lp->d3f, lp->d3b, lp->Y3, Tb, n3, 2.0f / (float)n3, lp->part);
        loss_final<<<1, 256, 0, st>>>(lp->loss, lp->part, (int)g, 1.0 / (double)n3);
    }
    SEM_LAUNCH_CHECK(ctx);
    // layer 3: gW3 = d3^T Y2, gb3 = colsum d3, d2 = (d3 W3) * (Y2 > 0)
    rc = transpose(lp, lp->tA, B, lp->d3b, kOut, B, kOut);           // d3^T: no x B
    if (!rc) rc = transpose(lp, lp->tB, B, lp->Y2, kHid, B, kHid);   // Y2^T: 256 x B
    if (!rc) rc = gemm(lp, kOut, kHid, B, lp->tA, B, lp->tB, B, nullptr, nullptr, 0, lp->gW[2], nullptr, kHid, 0);
    const int mask = lp->linear ? 0 : EPI_MASK;
    if (!lp->linear) colsum(lp, lp->gb[2], lp->d3f, B, kOut);
    if (!rc) rc = gemm(lp, B, kHid, kOut, lp->d3b, kOut, lp->W3t, kOut, nullptr, lp->Y2, kHid, lp->d2f, lp->d2b, kHid, mask);
    // layer 2
    if (!rc) rc = transpose(lp, lp->tA, B, lp->d2b, kHid, B, kHid);
    if (!rc) rc = transpose(lp, lp->tB, B, lp->Y1, kHid, B, kHid);
    if (!rc) rc = gemm(lp, kHid, kHid, B, lp->tA, B, lp->tB, B, nullptr, nullptr, 0, lp->gW[1], nullptr, kHid, 0);
    if (!lp->linear) colsum(lp, lp->gb[1], lp->d2f, B, kHid);
    if (!rc) rc = gemm(lp, B, kHid, kHid, lp->d2b, kHid, lp->W2t, kHid, nullptr, lp->Y1, kHid, lp->d1f, lp->d1b, kHid, mask);
    // layer 1
    if (!rc) rc = transpose(lp, lp->tA, B, lp->d1b, kHid, B, kHid);
    if (!rc) rc = transpose(lp, lp->tB, B, Xb, kInPad, B, kInPad);
    if (!rc) rc = gemm(lp, kHid, kInPad, B, lp->tA, B, lp->tB, B, nullptr, nullptr, 0, lp->gW[0], nullptr, kInPad, 0);
    if (!lp->linear) colsum(lp, lp->gb[0], lp->d1f, B, kHid);
    if (lp->linear) {   // the biases are not used: their gradients are zero
        zero_f32<<<1, 256, 0, st>>>(lp->gb[0], kHid);
        zero_f32<<<1, 256, 0, st>>>(lp->gb[1], kHid);
        zero_f32<<<2, 256, 0, st>>>(lp->gb[2], kOut);
    }
    SEM_LAUNCH_CHECK(ctx);
    return rc;
}

static int lp_train_buffers(sem_lp_t lp, int B) {
    const int kHid = lp->nh;     // this network's hidden width
    if (lp->d3f) return SEM_OK;
    const size_t R = (size_t)lp->max_rows;
    const size_t kOut = (size_t)lp->no, kInPad = (size_t)lp->nip;
    void* p = nullptr;
    int rc;
#define LP_ALLOC2(ptr, bytes) do { rc = lp_alloc(lp, &p, (bytes)); if (rc) return rc; ptr = (decltype(ptr))p; } while (0)
    LP_ALLOC2(lp->d3f, 4 * R * kOut);
    LP_ALLOC2(lp->d3b, 2 * R * kOut);
    LP_ALLOC2(lp->d2f, 4 * R * kHid);
    LP_ALLOC2(lp->d2b, 2 * R * kHid);
    LP_ALLOC2(lp->d1f, 4 * R * kHid);
    LP_ALLOC2(lp->d1b, 2 * R * kHid);
    // the transposes hold no x B, 256 x B or nip x B values, the column-sum
    // partials chunks x no or chunks x 256 (no < 256 for lx < 8)
    const size_t wide = std::max<size_t>(kInPad, (size_t)kHid), cols = std::max<size_t>(kOut, (size_t)kHid);
    LP_ALLOC2(lp->tA, 2 * R * wide);
    LP_ALLOC2(lp->tB, 2 * R * wide);
    LP_ALLOC2(lp->colpart, 4 * ((R + kColRows - 1) / kColRows) * cols);
#undef LP_ALLOC2
    (void)B;
    return SEM_OK;
}

extern "C" int sem_lp_gradients(sem_lp_t lp, const uint16_t* X, const float* T, int64_t B, float* loss) {
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_gradients: null network");
    sem_ctx_t ctx = lp->ctx;
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!X || !T || B < 1 || B > lp->max_rows || B % 8)
        return sem::fail(ctx, SEM_EINVAL, "sem_lp_gradients: batch %lld must be in [1, max_rows], a multiple of 8",
                         (long long)B);
    rc = lp_train_buffers(lp, (int)B);
    if (!rc) rc = lp_backward(lp, X, T, (int)B);
    if (rc) return rc;
    if (loss) {
        SEM_HIP(ctx, hipMemcpyAsync(loss, lp->loss, 4, hipMemcpyDeviceToHost, ctx->stream));
        SEM_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    return SEM_OK;
}

extern "C" int sem_lp_adam(sem_lp_t lp, double lr, double beta1, double beta2, double eps) {
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_adam: null network");
    sem_ctx_t ctx = lp->ctx;
    int rc = sem::enter(ctx);
    if (rc) return rc;
    lp->step += 1;
    const double c1 = 1.0 - std::pow(beta1, (double)lp->step);
    const double c2 = 1.0 - std::pow(beta2, (double)lp->step);
    for (int l = 0; l < 3; ++l) {
        const int rows = param_rows(lp, l), cols = param_cols(lp, l);
        adam_kernel<<<grid_of((int64_t)rows * cols), kBlock, 0, ctx->stream>>>(
            lp->W[l], lp->mW[l], lp->vW[l], lp->gW[l], rows, cols, l == 0 ? lp->nip : cols, (float)lr,
            (float)beta1, (float)(1.0 - beta1), (float)beta2, (float)(1.0 - beta2), (float)eps,
            (float)c1, (float)c2);
        adam_kernel<<<grid_of(rows), kBlock, 0, ctx->stream>>>(
            lp->b[l], lp->mb[l], lp->vb[l], lp->gb[l], 1, rows, rows, (float)lr, (float)beta1,
            (float)(1.0 - beta1), (float)beta2, (float)(1.0 - beta2), (float)eps, (float)c1, (float)c2);
    }
    SEM_LAUNCH_CHECK(ctx);
    lp->dirty = lp->fold_dirty = true;
    return SEM_OK;
}

extern "C" int sem_lp_train_step(sem_lp_t lp, const uint16_t* X, const float* T, const int64_t* rows,
                                 int64_t B, double lr, float* loss) {
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_train_step: null network");
    sem_ctx_t ctx = lp->ctx;
    int rc = sem::enter(ctx);
    if (rc) return rc;
    if (!X || !T || !rows || B < 8 || B > lp->max_rows || B % 8)
        return sem::fail(ctx, SEM_EINVAL, "sem_lp_train_step: bad batch (%lld)", (long long)B);
    rc = lp_train_buffers(lp, (int)B);
    if (rc) return rc;
    gather_rows<<<(unsigned)B, 256, 0, ctx->stream>>>(lp->X, lp->T, X, T, rows, (int)B, lp->nip, lp->no);
    SEM_LAUNCH_CHECK(ctx);
    rc = lp_backward(lp, lp->X, lp->T, (int)B);
    if (rc) return rc;
    rc = sem_lp_adam(lp, lr, 0.9, 0.999, 1e-8);
    if (rc) return rc;
    if (loss) SEM_HIP(ctx, hipMemcpyAsync(loss, lp->loss, 4, hipMemcpyDeviceToDevice, ctx->stream));
    return SEM_OK;
}

namespace sem {

// z = Q Q^T (mult^-1 (s/kappa) NN(features(r))) for the bound operator
// linear form, unique layout: gather of S r and the product into lp->Y3 (CSR order)
template <typename T>
int lin_product(sem_lp_t lp, const T* r) {
    int rc = refresh_fold(lp);
    if (rc) return rc;
    sem_ctx_t ctx = lp->ctx;
    hipStream_t st = ctx->stream;
    const int64_t nel = lp->nel;
    lin_gather_kernel<T><<<grid_of(nel * lp->no / 8, 8192), kBlock, 0, st>>>(lp->X, r, lp->sl, lp->gs->lid,
                                                                         nel * lp->no / 8, lp->skip, lp->no,
                                                                         lp->nip);
    SEM_LAUNCH_CHECK(ctx);
    if (lp->no != kOut || lp->product == 2) {   // the general product, outputs scattered to CSR order
        if (nel > 0x7fffffff) return sem::fail(ctx, SEM_EINVAL, "sem_lp: too many elements");
        return gemm(lp, (int)nel, lp->no, lp->no, lp->X, lp->nip, lp->Wfb, lp->no, nullptr, nullptr, 0, lp->Y3,
                    nullptr, lp->no, 0, lp->kappa_inv, lp->gs->upos);
    }
    const int64_t nchunks = (nel + kWsChunk - 1) / kWsChunk;
    const int groups = (int)std::min<int64_t>(kWsGroupsMax, (nchunks + 7) / 8 * 8);
    lin_gemm_kernel<<<(unsigned)(2 * groups), 512, 0, st>>>(lp->Y3, lp->X, lp->gs->upos, lp->kappa_inv, lp->Wfb,
                                                            nel, groups, lp->skip);
    SEM_LAUNCH_CHECK(ctx);
    return SEM_OK;
}

template <typename T>
int lp_apply_t(sem_lp_t lp, T* z, const T* r, bool unique) {
    sem_ctx_t ctx = lp->ctx;
    hipStream_t st = ctx->stream;
    const int64_t nel = lp->nel;
    if (unique && lp->linear) {   // product with CSR-ordered output, then assembly
        int rc = lin_product(lp, r);
        if (rc) return rc;
        const int64_t nu = lp->gs->n_unique;
        lin_assemble_kernel<T><<<grid_of(nu, 8192), kBlock, 0, st>>>(z, lp->Y3,
                                                                     lp->jacobi_base ? lp->minvu : nullptr, r,
                                                                     lp->gs->uoff, nu, lp->skip);
        SEM_LAUNCH_CHECK(ctx);
        return SEM_OK;
    }
    int rc = launch_features<T>(lp, nel, lp->X, lp->scale, nullptr, r, nullptr, nullptr,
                                lp->linear ? nullptr : lp->geo, nullptr, 0, lp->skip,
                                unique ? lp->gs->lid : nullptr, lp->linear && unique ? lp->gs->uoff : nullptr,
                                lp->linear && !unique ? lp->gs->mult : nullptr);
    if (rc) return rc;
    if (lp->linear) {   // one product with the folded matrix
        rc = refresh_fold(lp);
        if (!rc) rc = gemm(lp, (int)nel, lp->no, lp->no, lp->X, lp->nip, lp->Wfb, lp->no, nullptr, nullptr, 0,
                           lp->Y3, nullptr, lp->no, 0);
    } else {
        rc = forward(lp, lp->X, nel);
    }
    if (rc) return rc;
    if (unique) {
        const int64_t nu = lp->gs->n_unique;
        lp_output_unique_kernel<T><<<grid_of(nu), kBlock, 0, st>>>(
            z, lp->Y3, lp->scale, lp->jacobi_base ? lp->minv : nullptr, r, lp->gs->uoff, lp->gs->uidx,
            nu, lp->skip, lp->linear, lp->no);
        SEM_LAUNCH_CHECK(ctx);
        return SEM_OK;
    }
    const int64_t n = nel * lp->no;
    lp_output_kernel<T><<<grid_of(n), kBlock, 0, st>>>(z, lp->Y3, lp->scale, lp->gs->mult,
                                                       lp->jacobi_base ? lp->minv : nullptr, r, n, lp->skip,
                                                       lp->linear, lp->no);
    SEM_LAUNCH_CHECK(ctx);
    return gs_launch(lp->gs, z, sizeof(T) == 8 ? SEM_F64 : SEM_F32, lp->skip);
}

int lp_apply_partial(sem_lp_t lp, const void* r, bool f64, const int* skip, const float** zl, bool* jacobi_base) {
    if (!lp->bound || !lp->gs) return fail(lp->ctx, SEM_EINVAL, "learned preconditioner has no bound operator");
    if (!lp->linear) return SEM_EUNSUPPORTED_LX;
    lp->skip = skip;
    const int rc = f64 ? lin_product<double>(lp, (const double*)r) : lin_product<float>(lp, (const float*)r);
    lp->skip = nullptr;
    *zl = lp->Y3;
    *jacobi_base = lp->jacobi_base;
    return rc;
}

int lp_apply(sem_lp_t lp, void* z, const void* r, bool f64, const int* skip, bool unique) {
    if (!lp->bound || !lp->gs) return fail(lp->ctx, SEM_EINVAL, "learned preconditioner has no bound operator");
    lp->skip = skip;
    const int rc = f64 ? lp_apply_t<double>(lp, (double*)z, (const double*)r, unique)
                       : lp_apply_t<float>(lp, (float*)z, (const float*)r, unique);
    lp->skip = nullptr;
    return rc;
}

int64_t lp_rows(sem_lp_t lp) { return lp->nel; }
sem_gs_t lp_plan(sem_lp_t lp) { return lp->gs; }

}  // namespace sem

extern "C" int sem_lp_apply(sem_lp_t lp, void* z, const void* r, sem_dtype_t dtype) {
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_apply: null network");
    int rc = sem::enter(lp->ctx);
    if (rc) return rc;
    if (!z || !r || (dtype != SEM_F64 && dtype != SEM_F32))
        return sem::fail(lp->ctx, SEM_EINVAL, "sem_lp_apply: bad argument");
    return sem::lp_apply(lp, z, r, dtype == SEM_F64, nullptr, false);
}

extern "C" int sem_lp_apply_unique(sem_lp_t lp, void* z, const void* r, sem_dtype_t dtype) {
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_apply_unique: null network");
    int rc = sem::enter(lp->ctx);
    if (rc) return rc;
    if (!z || !r || z == r || (dtype != SEM_F64 && dtype != SEM_F32))
        return sem::fail(lp->ctx, SEM_EINVAL, "sem_lp_apply_unique: bad argument");
    return sem::lp_apply(lp, z, r, dtype == SEM_F64, nullptr, true);
}

// ---- checkpoint file -------------------------------------------------------
// "SEMLP001", int32 version 1, int32 linear, int32 jacobi_base, double mu,
// int64 Adam step, then for each of the 18 slots 0..17 (parameters, first and
// second moments, in sem_lp_set order) int64 count + count float32 values.
namespace {
constexpr char kMagic[8] = {'S', 'E', 'M', 'L', 'P', '0', '0', '1'};
}

extern "C" int sem_lp_save(sem_lp_t lp, const char* path) {
    if (!lp || !path) return sem::fail(lp ? lp->ctx : nullptr, SEM_EINVAL, "sem_lp_save: null argument");
    int rc = sem::enter(lp->ctx);
    if (rc) return rc;
    std::vector<std::vector<float>> slots(18);
    for (int w = 0; w < 18; ++w) {
        int64_t n;
        int ld;
        param_slot(lp, w, &n, &ld);
        slots[w].resize((size_t)n);
        rc = sem_lp_get(lp, w, slots[w].data(), n);
        if (rc) return rc;
    }
    FILE* f = std::fopen(path, "wb");
    if (!f) return sem::fail(lp->ctx, SEM_EINVAL, "sem_lp_save: cannot open %s", path);
    const int32_t hdr[3] = {1, lp->linear ? 1 : 0, lp->jacobi_base ? 1 : 0};
    const int64_t step = lp->step;
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(hdr, 4, 3, f) == 3 &&
              std::fwrite(&lp->mu, 8, 1, f) == 1 && std::fwrite(&step, 8, 1, f) == 1;
    for (int w = 0; ok && w < 18; ++w) {
        const int64_t n = (int64_t)slots[w].size();
        ok = std::fwrite(&n, 8, 1, f) == 1 && std::fwrite(slots[w].data(), 4, (size_t)n, f) == (size_t)n;
    }
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return sem::fail(lp->ctx, SEM_EINVAL, "sem_lp_save: write to %s failed", path);
    return SEM_OK;
}

extern "C" int sem_lp_load(sem_lp_t lp, const char* path) {
    if (!lp || !path) return sem::fail(lp ? lp->ctx : nullptr, SEM_EINVAL, "sem_lp_load: null argument");
    int rc = sem::enter(lp->ctx);
    if (rc) return rc;
    FILE* f = std::fopen(path, "rb");
    if (!f) return sem::fail(lp->ctx, SEM_EINVAL, "sem_lp_load: cannot open %s", path);
    char magic[8];
    int32_t hdr[3];
    double mu;
    int64_t step;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 &&
              std::fread(hdr, 4, 3, f) == 3 && hdr[0] == 1 && std::fread(&mu, 8, 1, f) == 1 &&
              std::fread(&step, 8, 1, f) == 1 && step >= 0;
    std::vector<std::vector<float>> slots(18);
    for (int w = 0; ok && w < 18; ++w) {
        int64_t n, want;
        int ld;
        param_slot(lp, w, &want, &ld);
        ok = std::fread(&n, 8, 1, f) == 1 && n == want;
        if (ok) {
            slots[w].resize((size_t)n);
            ok = std::fread(slots[w].data(), 4, (size_t)n, f) == (size_t)n;
        }
    }
    std::fclose(f);
    if (!ok) return sem::fail(lp->ctx, SEM_EINVAL, "sem_lp_load: %s is not a network checkpoint of this shape", path);
    // nothing is changed before the whole file has been read and checked
    rc = sem_lp_set_linear(lp, hdr[1]);
    if (!rc) rc = sem_lp_set_jacobi_base(lp, hdr[2]);
    if (!rc) rc = sem_lp_set_metric(lp, mu);
    for (int w = 0; !rc && w < 18; ++w) rc = sem_lp_set(lp, w, slots[w].data(), (int64_t)slots[w].size());
    if (!rc) rc = sem_lp_set_step(lp, step);
    return rc;
}

extern "C" int sem_lp_set_product(sem_lp_t lp, int kind) {
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_set_product: null network");
    if (kind < 0 || kind > 2 || (kind == 1 && lp->no != kOut))
        return sem::fail(lp->ctx, SEM_EINVAL, "sem_lp_set_product: kind %d (the weight-stationary product needs lx = 8)",
                         kind);
    lp->product = kind;
    return SEM_OK;
}

extern "C" int sem_lp_set_block(sem_lp_t lp, const float* W, int64_t count) {
    if (!lp) return sem::fail(nullptr, SEM_EINVAL, "sem_lp_set_block: null network");
    int rc = sem::enter(lp->ctx);
    if (rc) return rc;
    if (!W || count != (int64_t)lp->no * lp->no)
        return sem::fail(lp->ctx, SEM_EINVAL, "sem_lp_set_block: need %d x %d values", lp->no, lp->no);
    rc = sem_lp_set_linear(lp, 1);
    if (rc) return rc;
    rc = refresh_bf16(lp);
    if (rc) return rc;
    SEM_HIP(lp->ctx, hipStreamSynchronize(lp->ctx->stream));
    SEM_HIP(lp->ctx, hipMemcpy(lp->Wf32, W, 4 * (size_t)count, hipMemcpyHostToDevice));
    sym_to_bf16<<<256, kBlock, 0, lp->ctx->stream>>>(lp->Wfb, lp->Wf32, lp->no);
    SEM_LAUNCH_CHECK(lp->ctx);
    lp->fold_dirty = false;      // until the weights change again
    return SEM_OK;
}
