// Dense FP64 refactorisation of the support system: Phi_S = L L^T (blocked
// right-looking Cholesky) and M = L^-1 (blocked triangular inverse), with the
// block products on the FP64 matrix cores (v_mfma_f64_16x16x4f64).  Used to
// rebuild the inverse factor of a given support set, and to re-certify the
// incrementally grown factor against rounding drift.
//
// Matrices are dense row-major np x np with np = n rounded up to kDB; the
// padding is the identity, so every block step is full-sized:
// chol([[Phi, 0], [0, I]]) = [[L, 0], [0, I]] and its inverse is [[M, 0], [0, I]].
#include <hip/hip_runtime.h>

#include "gcb_device.h"
#include "gcb_internal.h"
#include "gcb_kernels.h"

namespace gcb {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int kDB = 32;   // block size of the blocked algorithms

// A = Phi_S (lower triangle, zero above) in the np x np padded layout.
__global__ __launch_bounds__(kBlock) void k_assemble(int n, int np, const double* __restrict__ sx,
                                                     const double* __restrict__ sy, const double* __restrict__ sz,
                                                     double* __restrict__ A) {
    const int64_t x = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (x >= (int64_t)np * np) return;
    const int i = (int)(x / np), j = (int)(x % np);
    double v = 0.0;
    if (i < n && j < n) {
        if (j <= i) v = wendland_r2(dist2(sx[i], sy[i], sz[i], sx[j], sy[j], sz[j]));
    } else if (i == j) {
        v = 1.0;
    }
    A[x] = v;
}

// The value of v held by lane `lane` (a constant), broadcast through scalar registers.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Step k0 of the Cholesky factorisation.  Wave 0 factors the diagonal block
// (already updated by the earlier steps) in registers, one row per lane, with
// the column entries broadcast across lanes; the factored block goes to LDS
// and, from workgroup 0, to Dbuf (the diagonal blocks of L are read from there
// later; A's own diagonal block is only read in this launch, so no workgroup
// overwrites what another still reads).  Then each workgroup solves kBlock
// rows of the panel below: x L_kk^T = a.
__global__ __launch_bounds__(kBlock) void k_chol_step(int np, int k0, double* __restrict__ A,
                                                      double* __restrict__ Dbuf, int32_t* __restrict__ bad) {
    __shared__ double D[kDB][kDB + 1];
    __shared__ double Rd[kDB];
    const int tid = threadIdx.x;
    if (tid < 64) {
        const int lane = tid;
        const int row = lane < kDB ? lane : kDB - 1;
        double a[kDB];
        const double* Ar = A + (size_t)(k0 + row) * np + k0;
#pragma unroll
        for (int c = 0; c < kDB; ++c) a[c] = (c <= lane && lane < kDB) ? Ar[c] : 0.0;
        int sing = 0;
#pragma unroll
        for (int c = 0; c < kDB; ++c) {
            double d = readlane_f64(a[c], c);
            if (!(d > kSingularTol)) {
                sing = 1;
                d = 1.0;
            }
            // 1/sqrt(d) by two Newton steps on the hardware estimate; L_cc = d / sqrt(d)
            double rs = __builtin_amdgcn_rsq(d);
            rs = fma(0.5 * rs, fma(-d * rs, rs, 1.0), rs);
            rs = fma(0.5 * rs, fma(-d * rs, rs, 1.0), rs);
            if (lane == c) a[c] = d * rs;
            if (lane > c) a[c] *= rs;
#pragma unroll
            for (int j = c + 1; j < kDB; ++j) {
                const double ljc = readlane_f64(a[c], j);
                if (lane >= j) a[j] = fma(-a[c], ljc, a[j]);
            }
        }
        if (lane < kDB) {
#pragma unroll
            for (int c = 0; c < kDB; ++c) D[lane][c] = c <= lane ? a[c] : 0.0;
            if (blockIdx.x == 0) {
                double* Db = Dbuf + (size_t)(k0 / kDB) * kDB * kDB + (size_t)lane * kDB;
#pragma unroll
                for (int c = 0; c < kDB; ++c) Db[c] = c <= lane ? a[c] : 0.0;
            }
        }
        if (lane == 0 && sing) bad[0] = 1;
    }
    __syncthreads();
    if (tid < kDB) Rd[tid] = 1.0 / D[tid][tid];
    __syncthreads();
    const int r = k0 + kDB + blockIdx.x * kBlock + tid;
    if (r >= np) return;
    double* Ar = A + (size_t)r * np + k0;
    double x[kDB];
#pragma unroll
    for (int c = 0; c < kDB; ++c) x[c] = Ar[c];
    // right-looking: once x_c is known, every later entry is updated (independent FMAs)
#pragma unroll
    for (int c = 0; c < kDB; ++c) {
        x[c] *= Rd[c];
#pragma unroll
        for (int t = c + 1; t < kDB; ++t) x[t] = fma(-x[c], D[t][c], x[t]);
    }
#pragma unroll
    for (int c = 0; c < kDB; ++c) Ar[c] = x[c];
}

// lower block index pair (ti >= tj) of linear index b
__device__ __forceinline__ void tri_index(int b, int& ti, int& tj) {
    int i = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= b) ++i;
    while (i * (i + 1) / 2 > b) --i;
    ti = i;
    tj = b - i * (i + 1) / 2;
}

// Trailing update after step k0: A[k1:, k1:] -= P P^T (lower blocks) with
// P = A[k1:, k0:k1], k1 = k0 + kDB.  One workgroup per kDB x kDB block, one
// wave per 16 x 16 quarter, K = kDB on the matrix cores.
__global__ __launch_bounds__(kBlock) void k_chol_update(int np, int k0, double* __restrict__ A) {
    const int k1 = k0 + kDB;
    int ti, tj;
    tri_index(blockIdx.x, ti, tj);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int R0 = k1 + kDB * ti + 16 * (wave >> 1);
    const int C0 = k1 + kDB * tj + 16 * (wave & 1);
    if (ti == tj && (wave >> 1) < (wave & 1)) return;   // strictly upper quarter of a diagonal block
    const int li = lane & 15, lk = lane >> 4;
    const double* Pa = A + (size_t)(R0 + li) * np + k0;
    const double* Pb = A + (size_t)(C0 + li) * np + k0;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < kDB; s += 4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Pa[s + lk], Pb[s + lk], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) A[(size_t)(R0 + lk + 4 * r) * np + C0 + li] -= acc[r];
}

// Diagonal blocks of M: M_jj = L_jj^-1 (L_jj from Dbuf), one workgroup per
// block; thread c forms column c by forward substitution.
__global__ __launch_bounds__(kBlock) void k_trtri_diag(int np, const double* __restrict__ Dbuf, double* __restrict__ M) {
    __shared__ double Ld[kDB][kDB + 1];
    __shared__ double X[kDB][kDB + 1];
    const int j0 = blockIdx.x * kDB;
    const double* Db = Dbuf + (size_t)blockIdx.x * kDB * kDB;
    for (int x = threadIdx.x; x < kDB * kDB; x += kBlock) Ld[x / kDB][x % kDB] = Db[x];
    __syncthreads();
    const int c = threadIdx.x;
    if (c < kDB) {
        for (int i = 0; i < kDB; ++i) {
            if (i < c) {
                X[i][c] = 0.0;
                continue;
            }
            double v = i == c ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) v -= Ld[i][k] * X[k][c];
            X[i][c] = v / Ld[i][i];
        }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < kDB * kDB; x += kBlock)
        M[(size_t)(j0 + x / kDB) * np + j0 + x % kDB] = X[x / kDB][x % kDB];
}

// Blocks of M at distance s below the diagonal, all in parallel:
// M_ij = -M_ii (sum_{k=j}^{i-1} L_ik M_kj), i = j + s; the blocks M_kj with
// k - j < s come from earlier launches.  16 waves per block: four per 16 x 16
// quarter of the tile, each summing every fourth 16-wide slice of the K range
// (four accumulator chains), the slices added in order through LDS.
constexpr int kTriWaves = 16;

__global__ __launch_bounds__(kTriWaves * 64) void k_trtri_off(int np, int s, const double* __restrict__ L,
                                                              double* __restrict__ M) {
    __shared__ double part[4][kDB][kDB + 1];
    __shared__ double T[kDB][kDB + 1];
    const int j = blockIdx.x, i = j + s;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int quarter = wave & 3, slice = wave >> 2;
    const int qi = quarter >> 1, qj = quarter & 1;
    const int li = lane & 15, lk = lane >> 4;
    d4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
    const double* La = L + (size_t)(kDB * i + 16 * qi + li) * np;
    const double* Mb = M + kDB * j + 16 * qj + li;
    // four 16-wide slices in flight per round (loads first, then their products)
    const int kend = kDB * i;
    int k = kDB * j + 16 * slice;
    for (; k + 192 < kend; k += 256) {
        double a[4][4], b[4][4];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[c][q] = La[k + 64 * c + 4 * q + lk];
                b[c][q] = Mb[(size_t)(k + 64 * c + 4 * q + lk) * np];
            }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][q], b[c][q], acc[q], 0, 0, 0);
    }
    for (; k < kend; k += 64) {
        double a[4], b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a[q] = La[k + 4 * q + lk];
            b[q] = Mb[(size_t)(k + 4 * q + lk) * np];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[q], acc[q], 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        part[slice][16 * qi + lk + 4 * r][16 * qj + li] = (acc[0][r] + acc[1][r]) + (acc[2][r] + acc[3][r]);
    __syncthreads();
    for (int x = threadIdx.x; x < kDB * kDB; x += kTriWaves * 64) {
        const int r = x / kDB, c = x % kDB;
        T[r][c] = (part[0][r][c] + part[1][r][c]) + (part[2][r][c] + part[3][r][c]);
    }
    __syncthreads();
    if (wave >= 4) return;
    d4 out = {0.0, 0.0, 0.0, 0.0};
    const double* Mi = M + (size_t)(kDB * i + 16 * qi + li) * np + kDB * i;
#pragma unroll
    for (int k = 0; k < kDB; k += 4)
        out = __builtin_amdgcn_mfma_f64_16x16x4f64(Mi[k + lk], T[k + lk][16 * qj + li], out, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) M[(size_t)(kDB * i + 16 * qi + lk + 4 * r) * np + kDB * j + 16 * qj + li] = -out[r];
}

// Packed rows of the first n rows (row i at i(i+1)/2), and the largest
// |new - old| and |old| against a previous packed factor (per workgroup).
__global__ __launch_bounds__(kBlock) void k_pack_rows(int n, int np, const double* __restrict__ Md,
                                                      double* Mp, const double* old,   // Mp may be old
                                                      double* __restrict__ red) {
    __shared__ double sd[kBlock], so[kBlock];
    const int64_t tri = (int64_t)n * (n + 1) / 2;
    double dmax = 0.0, omax = 0.0;
    for (int64_t x = blockIdx.x * (int64_t)kBlock + threadIdx.x; x < tri; x += (int64_t)gridDim.x * kBlock) {
        int i = (int)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
        while ((int64_t)(i + 1) * (i + 2) / 2 <= x) ++i;
        while ((int64_t)i * (i + 1) / 2 > x) --i;
        const int j = (int)(x - (int64_t)i * (i + 1) / 2);
        const double v = Md[(size_t)i * np + j];
        if (old) {
            const double o = old[x];
            dmax = fmax(dmax, fabs(v - o));
            omax = fmax(omax, fabs(o));
        }
        Mp[x] = v;
    }
    sd[threadIdx.x] = dmax;
    so[threadIdx.x] = omax;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + h]);
            so[threadIdx.x] = fmax(so[threadIdx.x], so[threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        red[2 * blockIdx.x] = sd[0];
        red[2 * blockIdx.x + 1] = so[0];
    }
}

// Scaled coordinates of a given support set (original indices orig[0..n)).
__global__ __launch_bounds__(kBlock) void k_gather_support(int n, const int32_t* __restrict__ orig,
                                                           const double* __restrict__ xyz0, double inv_r,
                                                           double* __restrict__ sx, double* __restrict__ sy,
                                                           double* __restrict__ sz) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const int o = orig[j];
    sx[j] = xyz0[3 * (size_t)o] * inv_r;
    sy[j] = xyz0[3 * (size_t)o + 1] * inv_r;
    sz[j] = xyz0[3 * (size_t)o + 2] * inv_r;
}

}  // namespace

void launch_gather_support(hipStream_t s, Support& sp, int n, const double* xyz0, double inv_r) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_support, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n, sp.orig,
                       xyz0, inv_r, sp.sx, sp.sy, sp.sz);
}

int dense_padded(int n) { return (n + kDB - 1) / kDB * kDB; }

int dense_pack_blocks() { return 256; }

void launch_inverse_factor(hipStream_t s, const Support& sp, int n, double* A, double* Md, double* Dbuf,
                           int32_t* bad) {
    const int np = dense_padded(n);
    const int nbk = np / kDB;
    const int64_t cnt = (int64_t)np * np;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)((cnt + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n, np, sp.sx,
                       sp.sy, sp.sz, A);
    for (int kb = 0; kb < nbk; ++kb) {
        const int k0 = kb * kDB;
        const int rows = np - k0 - kDB;
        const unsigned g = (unsigned)std::max(1, (rows + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_chol_step, dim3(g), dim3(kBlock), 0, s, np, k0, A, Dbuf, bad);
        const int nt = nbk - kb - 1;
        if (nt > 0) hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(kBlock), 0, s, np, k0, A);
    }
    // blocks of Md above the diagonal are never read: no clearing needed
    hipLaunchKernelGGL(k_trtri_diag, dim3((unsigned)nbk), dim3(kBlock), 0, s, np, Dbuf, Md);
    for (int d = 1; d < nbk; ++d)
        hipLaunchKernelGGL(k_trtri_off, dim3((unsigned)(nbk - d)), dim3(kTriWaves * 64), 0, s, np, d, A, Md);
}

void launch_pack_factor(hipStream_t s, int n, const double* Md, double* Mp, const double* old, double* red) {
    hipLaunchKernelGGL(k_pack_rows, dim3((unsigned)dense_pack_blocks()), dim3(kBlock), 0, s, n, dense_padded(n), Md, Mp,
                       old, red);
}

}  // namespace gcb
