// Dense FP64 refactorisation of the support system: Phi_S = L L^T (blocked
// right-looking Cholesky) and, in the same block steps, M = L^-1, with the
// block products on the FP64 matrix cores (v_mfma_f64_16x16x4f64).  Used to
// rebuild the inverse factor of a given support set, and to re-certify the
// incrementally grown factor against rounding drift.
//
// The inverse follows from L M = I by blocks: M_kk = L_kk^-1 and, for j < k,
// M_kj = -M_kk T_kj with T_kj = sum_{l=j}^{k-1} L_kl M_lj.  Step k of the
// Cholesky produces the panel L_{.,k}; the same step's update adds
// L_ik M_kj to T_ij for every i > k and j <= k, so T_kj is complete when
// step k starts and the inverse costs no launches of its own.
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
// the column entries broadcast across lanes; the factored block goes to LDS.
// A's diagonal block is only read in this launch and never written, so no
// workgroup overwrites what another still reads.  In workgroup 0, 32 lanes of
// wave 1 then form M_kk = L_kk^-1 (lane c: column c by forward substitution)
// into Md.  Each workgroup solves kBlock rows of the panel below:
// x L_kk^T = a.
__global__ __launch_bounds__(kBlock) void k_chol_step(int np, int k0, double* __restrict__ A,
                                                      double* __restrict__ Md, int32_t* __restrict__ bad) {
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
        }
        if (lane == 0 && sing) bad[0] = 1;
    }
    __syncthreads();
    if (tid < kDB) Rd[tid] = 1.0 / D[tid][tid];
    __syncthreads();
    if (blockIdx.x == 0 && tid >= 64 && tid < 64 + kDB) {
        const int c = tid - 64;
        double x[kDB];
#pragma unroll
        for (int i = 0; i < kDB; ++i) x[i] = i == c ? 1.0 : 0.0;
        // L_kk x = e_c, right-looking: x_t is final once the earlier columns are applied
#pragma unroll
        for (int t = 0; t < kDB; ++t) {
            x[t] *= Rd[t];
#pragma unroll
            for (int i = t + 1; i < kDB; ++i) x[i] = fma(-D[i][t], x[t], x[i]);
        }
#pragma unroll
        for (int i = 0; i < kDB; ++i) Md[(size_t)(k0 + i) * np + k0 + c] = x[i];
    }
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

// M_kj = -M_kk T_kj (j < k) or M_kk (j = k) into Ms, one 16 x 16 quarter per
// wave (K = kDB on the matrix cores); block row k starts at k0.
__device__ __forceinline__ void inverse_row_block(int np, int k0, int jb, const double* __restrict__ Tb,
                                                  const double* __restrict__ Md, double (*Ms)[kDB + 1]) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int qi = wave >> 1, qj = wave & 1, li = lane & 15, lk = lane >> 4;
    if (jb * kDB == k0) {
        for (int x = threadIdx.x; x < kDB * kDB; x += kBlock) Ms[x / kDB][x % kDB] = Md[(size_t)(k0 + x / kDB) * np + k0 + x % kDB];
        return;
    }
    const double* Mkk = Md + (size_t)(k0 + 16 * qi + li) * np + k0;
    const double* Tkj = Tb + (size_t)k0 * np + kDB * jb + 16 * qj + li;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < kDB; s += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Mkk[s + lk], Tkj[(size_t)(s + lk) * np], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) Ms[16 * qi + lk + 4 * r][16 * qj + li] = -acc[r];
}

// Update after step k0 (k1 = k0 + kDB), one workgroup per kDB x kDB block,
// one wave per 16 x 16 quarter, K = kDB on the matrix cores:
//   blocks [0, nA): A[k1:, k1:] -= P P^T (lower blocks), P = A[k1:, k0:k1];
//   blocks [nA, ...): T_ij += L_ik M_kj for block rows i > k and columns
//   j <= k, with M_kj formed from T_kj first; the blocks of row k + 1 also
//   store M_kj into Md (T_kj is read by other blocks of this launch, so M
//   lives apart from T).
__global__ __launch_bounds__(kBlock) void k_chol_update(int np, int k0, int nA, double* __restrict__ A,
                                                        double* __restrict__ Tb, double* __restrict__ Md) {
    const int k1 = k0 + kDB;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    if ((int)blockIdx.x >= nA) {
        __shared__ double Ms[kDB][kDB + 1];
        const int kb = k0 / kDB;
        const int b = (int)blockIdx.x - nA;
        const int ti = b / (kb + 1), jb = b % (kb + 1);
        inverse_row_block(np, k0, jb, Tb, Md, Ms);
        __syncthreads();
        if (ti == 0 && jb < kb)
            for (int x = threadIdx.x; x < kDB * kDB; x += kBlock)
                Md[(size_t)(k0 + x / kDB) * np + kDB * jb + x % kDB] = Ms[x / kDB][x % kDB];
        const int qi = wave >> 1, qj = wave & 1;
        const int R0 = k1 + kDB * ti + 16 * qi, C0 = kDB * jb + 16 * qj;
        d4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r] = Tb[(size_t)(R0 + lk + 4 * r) * np + C0 + li];
        const double* Lik = A + (size_t)(R0 + li) * np + k0;
#pragma unroll
        for (int s = 0; s < kDB; s += 4)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Lik[s + lk], Ms[s + lk][16 * qj + li], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) Tb[(size_t)(R0 + lk + 4 * r) * np + C0 + li] = acc[r];
        return;
    }
    int ti, tj;
    tri_index(blockIdx.x, ti, tj);
    const int R0 = k1 + kDB * ti + 16 * (wave >> 1);
    const int C0 = k1 + kDB * tj + 16 * (wave & 1);
    if (ti == tj && (wave >> 1) < (wave & 1)) return;   // strictly upper quarter of a diagonal block
    const double* Pa = A + (size_t)(R0 + li) * np + k0;
    const double* Pb = A + (size_t)(C0 + li) * np + k0;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < kDB; s += 4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Pa[s + lk], Pb[s + lk], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) A[(size_t)(R0 + lk + 4 * r) * np + C0 + li] -= acc[r];
}

// The last block row of M (no update follows the last step): M_kj for j < k.
__global__ __launch_bounds__(kBlock) void k_inverse_last_row(int np, int k0, const double* __restrict__ Tb,
                                                             double* __restrict__ Md) {
    __shared__ double Ms[kDB][kDB + 1];
    const int jb = blockIdx.x;
    inverse_row_block(np, k0, jb, Tb, Md, Ms);
    __syncthreads();
    for (int x = threadIdx.x; x < kDB * kDB; x += kBlock)
        Md[(size_t)(k0 + x / kDB) * np + kDB * jb + x % kDB] = Ms[x / kDB][x % kDB];
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

void launch_inverse_factor(hipStream_t s, const Support& sp, int n, double* A, double* Md, double* Tb,
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
        hipLaunchKernelGGL(k_chol_step, dim3(g), dim3(kBlock), 0, s, np, k0, A, Md, bad);
        const int nt = nbk - kb - 1;
        if (nt > 0) {
            const int nA = nt * (nt + 1) / 2, nT = nt * (kb + 1);
            hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(nA + nT)), dim3(kBlock), 0, s, np, k0, nA, A, Tb, Md);
        }
    }
    if (nbk > 1)
        hipLaunchKernelGGL(k_inverse_last_row, dim3((unsigned)(nbk - 1)), dim3(kBlock), 0, s, np, (nbk - 1) * kDB,
                           Tb, Md);
}

void launch_pack_factor(hipStream_t s, int n, const double* Md, double* Mp, const double* old, double* red) {
    hipLaunchKernelGGL(k_pack_rows, dim3((unsigned)dense_pack_blocks()), dim3(kBlock), 0, s, n, dense_padded(n), Md, Mp,
                       old, red);
}

}  // namespace gcb
