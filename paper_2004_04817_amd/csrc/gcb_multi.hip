// Multiple right-hand sides on one support set (many deformation modes or
// time steps; Eqs. 4-6 with a matrix of displacements): weights by the FP64
// inverse factor, W = M^T (M D_S), and the volume sweep
// out = Phi(targets, S) W as a dense contraction on FP64 matrix cores.
#include "gcb_internal.h"
#include "gcb_kernels.h"
#include "gcb_device.h"

namespace gcb {

typedef double d4 __attribute__((ext_vector_type(4)));

// D_S[s][c] = modes[orig[s]][c] for the n supports (R columns, first rc real).
__global__ __launch_bounds__(kBlock) void k_gather_modes(int n, int rc, int R, const int32_t* __restrict__ orig,
                                                         const double* __restrict__ modes, double* __restrict__ D) {
    const int64_t x = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (x >= (int64_t)n * R) return;
    const int s = (int)(x / R), c = (int)(x % R);
    D[x] = c < rc ? modes[(int64_t)orig[s] * rc + c] : 0.0;
}

// One workgroup per row of the result; thread t handles column c = t % R of
// the R right-hand sides and every J-th term of the row (J = kBlock / R, at
// least 1), and the J partial sums are added in a fixed order.  With few
// right-hand sides (the 3 displacement components of the weights) every
// thread still has work.
// Y[i][c] = sum_{j <= i} M[i][j] D[j][c], M by packed rows.
__global__ __launch_bounds__(kBlock) void k_trmm_lower(int n, int R, const double* __restrict__ M,
                                                       const double* __restrict__ D, double* __restrict__ Y) {
    __shared__ double part[kBlock];
    const int i = blockIdx.x;
    const int J = max(1, kBlock / R);
    const int t = threadIdx.x, c = t % R, jl = t / R;
    const double* Mi = M + (size_t)i * (i + 1) / 2;
    double a0 = 0.0, a1 = 0.0;
    if (jl < J) {
        int j = jl;
        for (; j + J <= i; j += 2 * J) {
            a0 = fma(Mi[j], D[(size_t)j * R + c], a0);
            a1 = fma(Mi[j + J], D[(size_t)(j + J) * R + c], a1);
        }
        if (j <= i) a0 = fma(Mi[j], D[(size_t)j * R + c], a0);
    }
    part[t] = a0 + a1;
    __syncthreads();
    if (t < R) {
        double sum = 0.0;
        for (int q = 0; q < J; ++q) sum += part[q * R + t];
        Y[(size_t)i * R + t] = sum;
    }
}

// W[j][c] = sum_{i >= j} M[i][j] Y[i][c], M read by columns from Mc.
__global__ __launch_bounds__(kBlock) void k_trmm_upper(int n, int R, const double* __restrict__ Mc, int64_t cap,
                                                       const double* __restrict__ Y, double* __restrict__ W) {
    __shared__ double part[kBlock];
    const int j = blockIdx.x;
    const int J = max(1, kBlock / R);
    const int t = threadIdx.x, c = t % R, il = t / R;
    const double* col = Mc + (size_t)j * cap - (size_t)j * (j - 1) / 2;
    double a0 = 0.0, a1 = 0.0;
    if (il < J) {
        int i = j + il;
        for (; i + J < n; i += 2 * J) {
            a0 = fma(col[i - j], Y[(size_t)i * R + c], a0);
            a1 = fma(col[i + J - j], Y[(size_t)(i + J) * R + c], a1);
        }
        if (i < n) a0 = fma(col[i - j], Y[(size_t)i * R + c], a0);
    }
    part[t] = a0 + a1;
    __syncthreads();
    if (t < R) {
        double sum = 0.0;
        for (int q = 0; q < J; ++q) sum += part[q * R + t];
        W[(size_t)j * R + t] = sum;
    }
}

// Volume sweep with R right-hand sides (R a multiple of 16, at most kMaxR).
// Block: kMWaves waves, each owning 16 targets and all R columns; supports in
// chunks of kMChunk staged in LDS (coordinates and the chunk of W).  Per step
// of 4 supports a lane evaluates one phi (target l%16, support l/16): the A
// operand of v_mfma_f64_16x16x4f64; B is W[support][16 t + l%16]; the
// accumulator of tile t holds out[target (l/16) + 4 r][16 t + l%16].
constexpr int kMWaves = 16;
constexpr int kMChunk = 32;
constexpr int kMaxR = 192;

template <typename TIn, typename TOut>
__global__ __launch_bounds__(kMWaves * 64) void k_volume_multi(int64_t nv, const TIn* __restrict__ xyz, double inv_r,
                                                                int n, const double* __restrict__ sx,
                                                                const double* __restrict__ sy,
                                                                const double* __restrict__ sz,
                                                                const double* __restrict__ W, int R, int rc,
                                                                TOut* __restrict__ out) {
    __shared__ double lw[kMChunk][kMaxR];
    __shared__ double lc[3][kMChunk];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int nt = R / 16;
    const int64_t tbase = ((int64_t)blockIdx.x * kMWaves + wave) * 16;
    const int64_t tgt = min(tbase + (lane & 15), nv - 1);
    // points scaled by 1/(2R): phi from the quarter squared distance (one square-root Newton step)
    const double h = 0.5 * inv_r;
    const double tx = (double)xyz[3 * tgt] * h, ty = (double)xyz[3 * tgt + 1] * h, tz = (double)xyz[3 * tgt + 2] * h;
    d4 acc[kMaxR / 16];
#pragma unroll
    for (int t = 0; t < kMaxR / 16; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    const int kq = lane >> 4;   // support within a step of 4 (A row / B column index k)
    const int jl = lane & 15;
    for (int c0 = 0; c0 < n; c0 += kMChunk) {
        const int cn = min(kMChunk, n - c0);
        __syncthreads();
        for (int x = threadIdx.x; x < kMChunk * R; x += kMWaves * 64) {
            const int s = x / R, c = x % R;
            lw[s][c] = s < cn ? W[(size_t)(c0 + s) * R + c] : 0.0;
        }
        if (threadIdx.x < kMChunk) {
            const int s = threadIdx.x;
            lc[0][s] = s < cn ? 0.5 * sx[c0 + s] : 1e3;
            lc[1][s] = s < cn ? 0.5 * sy[c0 + s] : 1e3;
            lc[2][s] = s < cn ? 0.5 * sz[c0 + s] : 1e3;
        }
        __syncthreads();
#pragma unroll 1
        for (int s0 = 0; s0 < kMChunk; s0 += 4) {
            const int s = s0 + kq;
            const double a = wendland_quarter(dist2(tx, ty, tz, lc[0][s], lc[1][s], lc[2][s]));
#pragma unroll
            for (int t = 0; t < kMaxR / 16; ++t) {
                if (t < nt) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, lw[s][16 * t + jl], acc[t], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < kMaxR / 16; ++t) {
        if (t < nt) {
            const int c = 16 * t + jl;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t row = tbase + kq + 4 * r;
                if (row < nv && c < rc) out[row * rc + c] = (TOut)acc[t][r];
            }
        }
    }
}

int multi_padded_r(int rc) { return (rc + 15) / 16 * 16; }

bool launch_deform_multi(hipStream_t s, const Support& sp, int n, int rc, const double* modes_dev, double* Dbuf,
                         double* Ybuf, double* Wbuf, int64_t nv, const void* xyz, int in_f64, double inv_r, void* out,
                         int out_f64) {
    const int R = multi_padded_r(rc);
    if (R > kMaxR || n <= 0) return false;
    const int64_t cnt = (int64_t)n * R;
    hipLaunchKernelGGL(k_gather_modes, dim3((unsigned)((cnt + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n, rc, R,
                       sp.orig, modes_dev, Dbuf);
    hipLaunchKernelGGL(k_trmm_lower, dim3((unsigned)n), dim3(kBlock), 0, s, n, R, sp.M, Dbuf, Ybuf);
    hipLaunchKernelGGL(k_trmm_upper, dim3((unsigned)n), dim3(kBlock), 0, s, n, R, sp.Mc, sp.cap, Ybuf, Wbuf);
    if (nv <= 0) return true;
    const unsigned gv = (unsigned)((nv + kMWaves * 16 - 1) / (kMWaves * 16));
    if (in_f64 && out_f64)
        hipLaunchKernelGGL((k_volume_multi<double, double>), dim3(gv), dim3(kMWaves * 64), 0, s, nv,
                           (const double*)xyz, inv_r, n, sp.sx, sp.sy, sp.sz, Wbuf, R, rc, (double*)out);
    else if (in_f64)
        hipLaunchKernelGGL((k_volume_multi<double, float>), dim3(gv), dim3(kMWaves * 64), 0, s, nv,
                           (const double*)xyz, inv_r, n, sp.sx, sp.sy, sp.sz, Wbuf, R, rc, (float*)out);
    else if (out_f64)
        hipLaunchKernelGGL((k_volume_multi<float, double>), dim3(gv), dim3(kMWaves * 64), 0, s, nv,
                           (const float*)xyz, inv_r, n, sp.sx, sp.sy, sp.sz, Wbuf, R, rc, (double*)out);
    else
        hipLaunchKernelGGL((k_volume_multi<float, float>), dim3(gv), dim3(kMWaves * 64), 0, s, nv,
                           (const float*)xyz, inv_r, n, sp.sx, sp.sy, sp.sz, Wbuf, R, rc, (float*)out);
    return true;
}

// Sum over the 64 lanes of a wave (every lane active): a butterfly over the lane masks 32, 16, ..., 1; both
// lanes of a pair add the same two values, so every lane ends with the same total.
__device__ __forceinline__ double wave_total(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// The weights' three displacement columns (Eq. 4 for x, y and z): Y = M D with D = Delta_S (n x 3, row-major),
// one wave per row of M (packed rows), the lanes over the row's entries with two partial sums per column, then a
// wave tree.  Every row reads only its own entries of M and of D.
__global__ __launch_bounds__(kBlock) void k_trmv3_lower(int n, const double* __restrict__ M,
                                                        const double* __restrict__ D, double* __restrict__ Y) {
    const int i = blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= n) return;   // the whole wave
    const double* Mi = M + (size_t)i * (i + 1) / 2;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0;
    int j = lane;
    for (; j + 64 <= i; j += 128) {
        const double m0 = Mi[j], m1 = Mi[j + 64];
        const double* d0 = D + 3 * (size_t)j;
        const double* d1 = D + 3 * (size_t)(j + 64);
        a0 = fma(m0, d0[0], a0);
        a1 = fma(m0, d0[1], a1);
        a2 = fma(m0, d0[2], a2);
        b0 = fma(m1, d1[0], b0);
        b1 = fma(m1, d1[1], b1);
        b2 = fma(m1, d1[2], b2);
    }
    if (j <= i) {
        const double m0 = Mi[j];
        const double* d0 = D + 3 * (size_t)j;
        a0 = fma(m0, d0[0], a0);
        a1 = fma(m0, d0[1], a1);
        a2 = fma(m0, d0[2], a2);
    }
    const double y0 = wave_total(a0 + b0), y1 = wave_total(a1 + b1), y2 = wave_total(a2 + b2);
    if (lane == 0) {
        Y[3 * (size_t)i] = y0;
        Y[3 * (size_t)i + 1] = y1;
        Y[3 * (size_t)i + 2] = y2;
    }
}

// W = M^T Y for the same three columns, one wave per column j of M (the column-major copy: rows j.. of column j
// at j cap - j (j - 1) / 2), written straight into the support's weight arrays.
__global__ __launch_bounds__(kBlock) void k_trmv3_upper(int n, const double* __restrict__ Mc, int64_t cap,
                                                        const double* __restrict__ Y, double* __restrict__ wx,
                                                        double* __restrict__ wy, double* __restrict__ wz) {
    const int j = blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (j >= n) return;   // the whole wave
    const double* col = Mc + (size_t)j * cap - (size_t)j * (j - 1) / 2;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, b0 = 0.0, b1 = 0.0, b2 = 0.0;
    int i = j + lane;
    for (; i + 64 < n; i += 128) {
        const double m0 = col[i - j], m1 = col[i + 64 - j];
        const double* y0 = Y + 3 * (size_t)i;
        const double* y1 = Y + 3 * (size_t)(i + 64);
        a0 = fma(m0, y0[0], a0);
        a1 = fma(m0, y0[1], a1);
        a2 = fma(m0, y0[2], a2);
        b0 = fma(m1, y1[0], b0);
        b1 = fma(m1, y1[1], b1);
        b2 = fma(m1, y1[2], b2);
    }
    if (i < n) {
        const double m0 = col[i - j];
        const double* y0 = Y + 3 * (size_t)i;
        a0 = fma(m0, y0[0], a0);
        a1 = fma(m0, y0[1], a1);
        a2 = fma(m0, y0[2], a2);
    }
    const double w0 = wave_total(a0 + b0), w1 = wave_total(a1 + b1), w2 = wave_total(a2 + b2);
    if (lane == 0) {
        wx[j] = w0;
        wy[j] = w1;
        wz[j] = w2;
    }
}

bool launch_support_weights(hipStream_t s, Support& sp, int n, const double* disp, double* Dbuf, double* Ybuf) {
    if (n <= 0) return false;
    const int64_t cnt = 3 * (int64_t)n;
    hipLaunchKernelGGL(k_gather_modes, dim3((unsigned)((cnt + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n, 3, 3,
                       sp.orig, disp, Dbuf);
    const unsigned g = (unsigned)((n + kBlock / 64 - 1) / (kBlock / 64));
    hipLaunchKernelGGL(k_trmv3_lower, dim3(g), dim3(kBlock), 0, s, n, sp.M, Dbuf, Ybuf);
    hipLaunchKernelGGL(k_trmv3_upper, dim3(g), dim3(kBlock), 0, s, n, sp.Mc, sp.cap, Ybuf, sp.wx, sp.wy, sp.wz);
    return true;
}

}  // namespace gcb
