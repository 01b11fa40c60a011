// Dense FP64 refactorisation of the support system: Phi_S = L L^T and M = L^-1
// (the inverse factor), by recursive halving, with the block products on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64).  Used to rebuild the inverse
// factor of a given support set, and to re-certify the incrementally grown
// factor against rounding drift.
//
// For Phi = [[A11, A21^T], [A21, A22]] split at a multiple of 64:
//   (L11, M11) from A11 (recursively);
//   L21 = A21 L11^-T = A21 M11^T (refined once against L11 for large A11);
//   S = A22 - L21 L21^T = L22 L22^T, and (L22, M22) from S (recursively);
//   M21 = -M22 L21 M11, formed as X = L21 M11, then M21 = -M22 X.
// Nearly all flops sit in the four products, whose depth is the size of the
// split (a few thousand at the top), so they run near the matrix cores' rate;
// only the 64 x 64 leaves are factored one workgroup at a time.
//
// Matrices are dense row-major np x np with np = n rounded up to 64; the
// padding is the identity, so every leaf is full-sized:
// chol([[Phi, 0], [0, I]]) = [[L, 0], [0, I]] and its inverse is [[M, 0], [0, I]].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <initializer_list>
#include <vector>

#include "gcb_device.h"
#include "gcb_internal.h"
#include "gcb_kernels.h"

namespace gcb {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int kLeaf = 64;   // leaf size of the recursion and tile size of the products

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

// One wave factors a 32 x 32 SPD block and inverts its factor in the same
// column loop.  On entry lane i < 32 holds row i of the block (entries t <= i,
// zero above) and lane 32 + t holds column t of the identity.  On exit lane i
// holds row i of L in its entries t <= i (the entries above are left with
// values that are never read) and lane 32 + t column t of L^-1.
// Column c (right-looking): every lane scales its entry c by 1 / sqrt(a_cc)
// (L_ic below the diagonal; in the upper half row c of the inverse,
// R_c / L_cc, final once the earlier columns are applied), then for k > c
// every lane takes a_k -= a_c L_kc: the lower half's a_ik -= L_ic L_kc and
// the upper half's R_k -= L_kc M_c, one broadcast of L_kc serving both.
// The broadcasts are read in groups of eight into separate registers before
// their products, so that their latency overlaps (also across columns).
__device__ __forceinline__ void chol_inv32(double (&a)[32], int& sing) {
#pragma unroll
    for (int c = 0; c < 32; ++c) {
        const double d0 = readlane_f64(a[c], c);
        const bool ok = d0 > kSingularTol;
        sing |= ok ? 0 : 1;
        const double d = ok ? d0 : 1.0;
        // 1/sqrt(d) by two Newton steps on the hardware estimate (good to about 2^-24)
        double rs = __builtin_amdgcn_rsq(d);
        rs = fma(0.5 * rs, fma(-d * rs, rs, 1.0), rs);
        rs = fma(0.5 * rs, fma(-d * rs, rs, 1.0), rs);
        a[c] *= rs;
#pragma unroll
        for (int k0 = c + 1; k0 < 32; k0 += 8) {
            double b[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + u < 32) b[u] = readlane_f64(a[c], k0 + u);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + u < 32) a[k0 + u] = fma(-a[c], b[u], a[k0 + u]);
        }
    }
}

// D (16 x 16 tile of one wave, d4 layout: row lk + 4 r, column li) += X Y over depth 32, both from LDS:
// X[i][k] at x[(xr + i) * xs + xc + k]; Y[k][j] at y[(yk + k) * ys + yc + j] or, transposed
// (Y given as rows j), at y[(yc + j) * ys + yk + k].
template <bool YT>
__device__ __forceinline__ d4 mm16x32(d4 acc, double sgn, const double* x, int xs, int xr, int xc, const double* y,
                                      int ys, int yk, int yc, int li, int lk) {
#pragma unroll
    for (int s = 0; s < 32; s += 4) {
        const double av = sgn * x[(xr + li) * xs + xc + s + lk];
        const double bv = YT ? y[(yc + li) * ys + yk + s + lk] : y[(yk + s + lk) * ys + yc + li];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    return acc;
}

// Leaf: the 64 x 64 diagonal block at (o, o) of A (lower triangle, already
// reduced by the earlier blocks) gives the same block of L (into Tb) and of
// Md = L^-1, both with zeros above the diagonal, by one halving step inside
// the workgroup: two 32-wide factorisations with inverse (wave 0) and the
// products between them on the matrix cores (all four waves).
constexpr int kLs = kLeaf + 1;   // LDS row strides
constexpr int kHs = 33;

__global__ __launch_bounds__(kBlock) void k_leaf64(int np, int o, const double* __restrict__ A,
                                                   double* __restrict__ Md, double* __restrict__ Lt,
                                                   int32_t* __restrict__ bad) {
    __shared__ double sA[kLeaf * kLs], sLb[kLeaf * kLs];
    __shared__ double sM1[32 * kHs], sM2[32 * kHs], sL[32 * kHs], sX[32 * kHs];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    for (int x = tid; x < kLeaf * kLeaf; x += kBlock) sA[(x >> 6) * kLs + (x & 63)] = A[(size_t)(o + (x >> 6)) * np + o + (x & 63)];
    __syncthreads();
    int sing = 0;
    if (wave == 0) {
        double a[32];
        const int i = lane & 31;
#pragma unroll
        for (int t = 0; t < 32; ++t) {   // every lane reads (in bounds); v * keep + one is exact: no branch
            const double v = sA[i * kLs + t];
            a[t] = fma(v, (lane < 32 && t <= i) ? 1.0 : 0.0, (lane >= 32 && t == i) ? 1.0 : 0.0);
        }
        chol_inv32(a, sing);
        if (lane >= 32)   // column i of M11
#pragma unroll
            for (int t = 0; t < 32; ++t) sM1[t * kHs + i] = a[t];
        else   // row i of L11 and the zeros beside it
#pragma unroll
            for (int t = 0; t < 32; ++t) {
                sLb[i * kLs + t] = t <= i ? a[t] : 0.0;
                sLb[i * kLs + 32 + t] = 0.0;
            }
    }
    __syncthreads();
    const int wi = wave >> 1, wj = wave & 1;
    {   // L21 = A21 M11^T
        d4 acc = {0.0, 0.0, 0.0, 0.0};
        acc = mm16x32<true>(acc, 1.0, sA, kLs, 32 + 16 * wi, 0, sM1, kHs, 0, 16 * wj, li, lk);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            sL[(16 * wi + lk + 4 * r) * kHs + 16 * wj + li] = acc[r];
            sLb[(32 + 16 * wi + lk + 4 * r) * kLs + 16 * wj + li] = acc[r];
        }
    }
    __syncthreads();
    // S = A22 - L21 L21^T (lower tiles 0..2) and X = L21 M11 (tiles 3..6)
    for (int job = wave; job < 7; job += 4) {
        if (job < 3) {
            const int ti = job == 0 ? 0 : 1, tj = job == 2 ? 1 : 0;
            double* s = sA + (32 + 16 * ti) * kLs + 32 + 16 * tj;
            d4 acc;
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = s[(lk + 4 * r) * kLs + li];
            acc = mm16x32<true>(acc, -1.0, sL, kHs, 16 * ti, 0, sL, kHs, 0, 16 * tj, li, lk);
#pragma unroll
            for (int r = 0; r < 4; ++r) s[(lk + 4 * r) * kLs + li] = acc[r];
        } else {
            const int ti = (job - 3) >> 1, tj = (job - 3) & 1;
            d4 acc = {0.0, 0.0, 0.0, 0.0};
            acc = mm16x32<false>(acc, 1.0, sL, kHs, 16 * ti, 0, sM1, kHs, 0, 16 * tj, li, lk);
#pragma unroll
            for (int r = 0; r < 4; ++r) sX[(16 * ti + lk + 4 * r) * kHs + 16 * tj + li] = acc[r];
        }
    }
    __syncthreads();
    if (wave == 0) {
        double a[32];
        const int i = lane & 31;
#pragma unroll
        for (int t = 0; t < 32; ++t) {
            const double v = sA[(32 + i) * kLs + 32 + t];
            a[t] = fma(v, (lane < 32 && t <= i) ? 1.0 : 0.0, (lane >= 32 && t == i) ? 1.0 : 0.0);
        }
        chol_inv32(a, sing);
        if (lane >= 32)   // column i of M22
#pragma unroll
            for (int t = 0; t < 32; ++t) sM2[t * kHs + i] = a[t];
        else   // row i of L22
#pragma unroll
            for (int t = 0; t < 32; ++t) sLb[(32 + i) * kLs + 32 + t] = t <= i ? a[t] : 0.0;
        if (lane == 0 && sing) bad[0] = 1;
    }
    __syncthreads();
    {   // M21 = -M22 X
        d4 acc = {0.0, 0.0, 0.0, 0.0};
        acc = mm16x32<false>(acc, -1.0, sM2, kHs, 16 * wi, 0, sX, kHs, 0, 16 * wj, li, lk);
#pragma unroll
        for (int r = 0; r < 4; ++r) Md[(size_t)(o + 32 + 16 * wi + lk + 4 * r) * np + o + 16 * wj + li] = acc[r];
    }
    for (int x = tid; x < 64 * 32; x += kBlock) {
        const int r = x >> 5, c = x & 31;
        if (r < 32) {   // M11 and the zero block beside it
            Md[(size_t)(o + r) * np + o + c] = sM1[r * kHs + c];
            Md[(size_t)(o + r) * np + o + 32 + c] = 0.0;
        } else {
            Md[(size_t)(o + r) * np + o + 32 + c] = sM2[(r - 32) * kHs + c];
        }
    }
    for (int x = tid; x < kLeaf * kLeaf; x += kBlock) Lt[(size_t)(o + (x >> 6)) * np + o + (x & 63)] = sLb[(x >> 6) * kLs + (x & 63)];
}

// ---------------------------------------------------------------------------
// Block products C (m x n) = alpha X Y (+ C), all matrices row-major with the
// leading dimension np.  X[i][k] at X + i np + k; Y[k][j] at Y + k np + j, or
// (y_rows) Y given by its rows j: Y[k][j] at Y + j np + k.  Output tiles of
// TL x TL (64, or 32 for small products; four waves of TL/2 x TL/2); a tile's
// depth range may be split into
// slices, one workgroup each (the work items of a launch, built on the host),
// so that tiles of very different depth (triangular factors) spread evenly
// over the chip and small products still fill it.  Slice 0 writes C itself
// (alpha p_0, plus C for accumulate), slice s > 0 writes alpha p_s to a
// partial buffer, and a second launch adds the partials to C in slice order,
// so a plan always gives the same bits.
//
// Depth in chunks of 32 staged in LDS (two stages), with the global loads of
// the next two chunks in flight in two register sets while a chunk is
// multiplied; operands stored in LDS depth-major so that each wave reads its
// matrix-core operands as 16 consecutive doubles.  Rows of the staged chunk
// are not padded; instead the column index is XOR-ed with a function of the
// depth row (lds_swizzle), which keeps both the transposing stores and the
// operand reads free of LDS bank conflicts.
struct GemmSide {
    const double* X;
    const double* Y;
    double* C;
    double alpha;
    int accumulate;  // C = alpha X Y + C
    int y_rows;      // Y given by its rows j (Y^T row-major)
};
struct GemmItem {
    int32_t ti, tj;  // output tile
    int32_t kb, ke;  // depth slice (multiples of 64)
    int32_t s;       // slice index
    int32_t part;    // partial slot of this slice (s > 0)
    int32_t side;    // 0 or 1: which product of the launch
    int32_t pad;
};
struct GemmReduce {   // a sliced tile: C += partials part .. part + P - 2, in order
    int32_t ti, tj, side, P, part, pad[3];
};
struct GemmLaunch {
    GemmSide side[2];
    const GemmItem* items;
    int total;
    int np;
    double* part;
};
struct ReduceLaunch {
    double* C[2];
    const GemmReduce* tiles;
    int np;
    const double* part;
};

constexpr int kKc = 32;            // depth chunk
constexpr int kTile = kLeaf * kLeaf;   // doubles per partial slot

// One chunk's global loads of one thread (TL / 16 d2 of each operand): X rows rr + 16 u, depth rk, rk + 1; Y
// likewise, or depth-major: depth ck + (512 / TL) u, columns cj, cj + 1.
template <int TL>
struct ChunkRegs {
    d2 x[TL / 16], y[TL / 16];
};

// Column swizzle of depth row k of a staged chunk (row length TL, a multiple of 32): bits 1-3 are bits 1-3 of k
// and bit 4 is bit 0 of k XOR bit 4 of k.  XOR with it permutes the columns within aligned blocks of 32
// (so the 16 consecutive doubles of a matrix-core operand stay one permuted block of 16).  Operand reads: the two
// rows a half-wave reads (k even, k + 1) fall in opposite halves of the banks.  Transposing stores: the 32 lanes
// of a half-wave (two rows r, 16 depths 2m) land on 32 distinct double slots.  Pairs of columns (even, odd) stay
// adjacent, so 16-byte stores of a depth-major chunk keep working.
__device__ __forceinline__ int lds_swizzle(int k) { return (k & 14) | ((((k >> 4) ^ k) & 1) << 4); }

// TL x TL output tiles (TL = 64 or 32); each wave computes a (TL / 2) x (TL / 2) quadrant of TW x TW matrix-core
// tiles of 16 x 16.
template <int TL>
__global__ __launch_bounds__(kBlock) void k_gemm(GemmLaunch g) {
    constexpr int TW = TL / 32, NU = TL / 16, kTs = TL, CW = TL / 2;
    __shared__ __align__(16) double sX[2][kKc * kTs];
    __shared__ __align__(16) double sY[2][kKc * kTs];
    // consecutive items on one XCD (workgroups are dealt to the 8 XCDs in turn), so that items sharing a row
    // panel share its L2
    const int b = blockIdx.x, T = g.total;
    const int xcd = b & 7, q = T >> 3, rem = T & 7;
    const GemmItem it = g.items[xcd * q + min(xcd, rem) + (b >> 3)];
    const GemmSide& op = it.side ? g.side[1] : g.side[0];
    const double* __restrict__ X = op.X;
    const double* __restrict__ Y = op.Y;
    const int y_rows = op.y_rows;
    const int i0 = it.ti * TL, j0 = it.tj * TL, np = g.np, kb = it.kb, ke = it.ke;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4, qi = wave >> 1, qj = wave & 1;
    // staging: a row-major chunk (TL rows x 32 depth): thread -> rows rr + 16 u, depth rk, rk + 1; a depth-major
    // one (32 depth x TL columns): thread -> depth ck + (512 / TL) u, columns cj, cj + 1
    const int rr = tid >> 4, rk = (tid & 15) * 2;
    const int ck = tid / CW, cj = (tid % CW) * 2;
    const double* Xp = X + (size_t)(i0 + rr) * np + rk;
    const double* Yp = y_rows ? Y + (size_t)(j0 + rr) * np + rk : Y + (size_t)ck * np + j0 + cj;
    auto load = [&](ChunkRegs<TL>& R, int kc) {
#pragma unroll
        for (int u = 0; u < NU; ++u) R.x[u] = *reinterpret_cast<const d2*>(Xp + (size_t)(16 * u) * np + kc);
        if (y_rows) {
#pragma unroll
            for (int u = 0; u < NU; ++u) R.y[u] = *reinterpret_cast<const d2*>(Yp + (size_t)(16 * u) * np + kc);
        } else {
#pragma unroll
            for (int u = 0; u < NU; ++u) R.y[u] = *reinterpret_cast<const d2*>(Yp + (size_t)(kc + (512 / TL) * u) * np);
        }
    };
    auto store = [&](const ChunkRegs<TL>& R, int buf) {
        double* x = sX[buf];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            x[rk * kTs + ((rr + 16 * u) ^ lds_swizzle(rk))] = R.x[u].x;
            x[(rk + 1) * kTs + ((rr + 16 * u) ^ lds_swizzle(rk + 1))] = R.x[u].y;
        }
        double* y = sY[buf];
        if (y_rows) {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                y[rk * kTs + ((rr + 16 * u) ^ lds_swizzle(rk))] = R.y[u].x;
                y[(rk + 1) * kTs + ((rr + 16 * u) ^ lds_swizzle(rk + 1))] = R.y[u].y;
            }
        } else {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int k = ck + (512 / TL) * u;
                *reinterpret_cast<d2*>(y + k * kTs + (cj ^ lds_swizzle(k))) = R.y[u];
            }
        }
    };
    d4 acc[TW][TW];
#pragma unroll
    for (int a = 0; a < TW; ++a)
#pragma unroll
        for (int c = 0; c < TW; ++c) acc[a][c] = d4{0.0, 0.0, 0.0, 0.0};
    auto compute = [&](int buf) {
        const double* x = sX[buf];
        const double* y = sY[buf];
#pragma unroll
        for (int s = 0; s < kKc; s += 4) {
            double av[TW], bv[TW];
#pragma unroll
            for (int a = 0; a < TW; ++a) av[a] = x[(s + lk) * kTs + ((CW * qi + 16 * a + li) ^ lds_swizzle(s + lk))];
#pragma unroll
            for (int c = 0; c < TW; ++c) bv[c] = y[(s + lk) * kTs + ((CW * qj + 16 * c + li) ^ lds_swizzle(s + lk))];
#pragma unroll
            for (int a = 0; a < TW; ++a)
#pragma unroll
                for (int c = 0; c < TW; ++c)
                    acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[c], acc[a][c], 0, 0, 0);
        }
    };
    if (kb < ke) {
        ChunkRegs<TL> RA, RB;
        load(RA, kb);
        if (kb + kKc < ke) load(RB, kb + kKc);
        store(RA, 0);
        __syncthreads();
        // stage 0 holds chunk kc (from RA), RB holds chunk kc + 32; the loop body handles two chunks so that the
        // register sets keep fixed names (depth ranges are multiples of 64)
        for (int kc = kb;; kc += 2 * kKc) {
            if (kc + 2 * kKc < ke) load(RA, kc + 2 * kKc);
            compute(0);
            if (kc + kKc >= ke) break;
            store(RB, 1);
            __syncthreads();
            if (kc + 3 * kKc < ke) load(RB, kc + 3 * kKc);
            compute(1);
            if (kc + 2 * kKc >= ke) break;
            store(RA, 0);
            __syncthreads();
        }
    }
    double* C = op.C;
    const double alpha = op.alpha;
    if (it.s == 0) {
        const int accumulate = op.accumulate;
#pragma unroll
        for (int a = 0; a < TW; ++a)
#pragma unroll
            for (int c = 0; c < TW; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double* p = C + (size_t)(i0 + CW * qi + 16 * a + lk + 4 * r) * np + j0 + CW * qj + 16 * c + li;
                    const double v = alpha * acc[a][c][r];
                    *p = accumulate ? *p + v : v;
                }
    } else {
        double* pp = g.part + (size_t)it.part * kTile;
#pragma unroll
        for (int a = 0; a < TW; ++a)
#pragma unroll
            for (int c = 0; c < TW; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    pp[(CW * qi + 16 * a + lk + 4 * r) * TL + CW * qj + 16 * c + li] = alpha * acc[a][c][r];
    }
}

// C += the partials of each sliced tile, in slice order (one element per thread; TL x TL tiles).
template <int TL>
__global__ __launch_bounds__(kBlock) void k_gemm_reduce(ReduceLaunch g) {
    constexpr int per = TL * TL / kBlock;   // workgroups per tile
    const GemmReduce t = g.tiles[blockIdx.x / per];
    double* C = t.side ? g.C[1] : g.C[0];
    const int x = (blockIdx.x % per) * kBlock + threadIdx.x;
    double* p = C + (size_t)(t.ti * TL + x / TL) * g.np + t.tj * TL + x % TL;
    double v = *p;
    for (int sl = 0; sl < t.P - 1; ++sl) v += g.part[(size_t)(t.part + sl) * kTile + x];
    *p = v;
}

// Packed rows of the first n rows (row i at i(i+1)/2), and the largest
// |new - old| and |old| against a previous packed factor (per workgroup).
// Workgroup b copies rows b, b + G, b + 2G, ... (G workgroups), its threads
// along the row.
__global__ __launch_bounds__(kBigBlock) void k_pack_rows(int n, int np, const double* __restrict__ Md,
                                                         double* Mp, const double* old,   // Mp may be old
                                                         double* __restrict__ red) {
    __shared__ double sd[kBigBlock], so[kBigBlock];
    double dmax = 0.0, omax = 0.0;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        const double* src = Md + (size_t)i * np;
        const size_t r0 = (size_t)i * (i + 1) / 2;
        for (int j = threadIdx.x; j <= i; j += kBigBlock) {
            const double v = src[j];
            if (old) {
                const double o = old[r0 + j];
                dmax = fmax(dmax, fabs(v - o));
                omax = fmax(omax, fabs(o));
            }
            Mp[r0 + j] = v;
        }
    }
    sd[threadIdx.x] = dmax;
    so[threadIdx.x] = omax;
    __syncthreads();
    for (int h = kBigBlock / 2; h > 0; h >>= 1) {
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

// One product of the recursion: shape, depth rule and operands (offsets into A, Md, Tb).
enum DenseBuf { kA = 0, kM = 1, kT = 2 };
struct ProdSpec {
    int m, n, k;
    int krule;   // depth range of tile (ti, tj): 0 all; 1 k < 64 (tj + 1) (Y^T lower); 2 k >= 64 tj (Y lower);
                 // 3 k < 64 (ti + 1) (X lower)
    int lower;   // only the tiles with tj <= ti
    int xb, yb, cb;
    size_t xo, yo, co;
    double alpha;
    int accumulate, y_rows;
};

}  // namespace

// The launches of a refactorisation of one padded size: leaves and products in
// order, each product's work items (tile, depth slice) in a device table.
struct DensePlan {
    struct Step {
        int leaf;       // >= 0: leaf at this offset; else a product launch
        int nspec;
        ProdSpec spec[2];
        int64_t item0;  // first work item
        int total;      // work items
        int64_t red0;   // first sliced tile
        int nred;       // sliced tiles (a reduction launch follows when > 0)
        int tl;         // output tile size of the product launch (64, or 32 for small products)
    };
    int np = 0;
    std::vector<Step> steps;
    GemmItem* items = nullptr;
    GemmReduce* red = nullptr;
    double* part = nullptr;
    int64_t nitems = 0, nred = 0, npart = 0;
    // the whole sequence captured once for one set of buffers (key), then replayed
    std::vector<const void*> key;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
};

namespace {

// Multiplying by the explicit inverse M11 gives L21 with an error that grows like kappa(L11)^2 u; one step of
// refinement against L11 itself brings it back to the level of a triangular solve.  Below this size the diagonal
// blocks are small enough that the product alone is as accurate.
constexpr int kRefineFrom = 256;

void plan_rec(std::vector<DensePlan::Step>& steps, int np, int o, int nl) {
    if (nl == 1) {
        DensePlan::Step st{};
        st.leaf = o * kLeaf;
        steps.push_back(st);
        return;
    }
    const int h = (nl + 1) / 2;
    plan_rec(steps, np, o, h);
    const int o1 = o * kLeaf, n1 = h * kLeaf, o2 = (o + h) * kLeaf, n2 = (nl - h) * kLeaf;
    const size_t p11 = (size_t)o1 * np + o1, p21 = (size_t)o2 * np + o1, p22 = (size_t)o2 * np + o2;
    auto step = [&](std::initializer_list<ProdSpec> sp) {
        DensePlan::Step st{};
        st.leaf = -1;
        for (const ProdSpec& x : sp) st.spec[st.nspec++] = x;
        steps.push_back(st);
    };
    // L21 = A21 M11^T into Tb
    step({ProdSpec{n2, n1, n1, 1, 0, kA, kM, kT, p21, p11, p21, 1.0, 0, 1}});
    if (n1 >= kRefineFrom) {
        // one refinement step: R = A21 - L21 L11^T into A21's place, then L21 += R M11^T
        step({ProdSpec{n2, n1, n1, 1, 0, kT, kT, kA, p21, p11, p21, -1.0, 1, 1}});
        step({ProdSpec{n2, n1, n1, 1, 0, kA, kM, kT, p21, p11, p21, 1.0, 1, 1}});
    }
    // S = A22 - L21 L21^T (lower tiles) and X = L21 M11 into A21's place, in one launch
    step({ProdSpec{n2, n2, n1, 0, 1, kT, kT, kA, p21, p21, p22, -1.0, 1, 1},
          ProdSpec{n2, n1, n1, 2, 0, kT, kM, kA, p21, p11, p21, 1.0, 0, 0}});
    plan_rec(steps, np, o + h, nl - h);
    // M21 = -M22 X
    step({ProdSpec{n2, n1, n2, 3, 0, kM, kA, kM, p22, p21, p21, -1.0, 0, 0}});
}

// Depth range of output tile (ti, tj) of size tl, in multiples of 64 (the products' chunk loop takes 64 at a time):
// the triangular rules hold per element and the leaves store exact zeros above the diagonal, so a range that also
// covers some of those zeros gives the same sums.
void depth_range(const ProdSpec& p, int tl, int ti, int tj, int& kb, int& ke) {
    kb = 0;
    ke = p.k;
    const int cj = tj * tl / kLeaf * kLeaf, ci = ti * tl / kLeaf * kLeaf;   // 64-block of the tile's first column / row
    if (p.krule == 1) ke = std::min(p.k, cj + kLeaf);
    else if (p.krule == 2) kb = cj;
    else if (p.krule == 3) ke = std::min(p.k, ci + kLeaf);
}

// Work items of one launch: tiles of 64, or of 32 when there are fewer than 128 tiles of 64 (so that a small
// product still spreads over many CUs); the slice depth (a multiple of 64) is chosen so that the launch has about
// eight items per workgroup slot of the chip (2 slots per CU with 64-tiles, 4 with 32-tiles at their LDS use; 2
// and 4 items per slot measured 4 % and 1 % slower at Nc = 4,000, 16 and 32 no faster), and is at least 256: a
// shallower tile gains less from splitting than the reduction launch costs.
void plan_items(DensePlan::Step& st, std::vector<GemmItem>& items, std::vector<GemmReduce>& red, int64_t& npart) {
    int64_t tiles64 = 0;
    for (int q = 0; q < st.nspec; ++q) {
        const ProdSpec& p = st.spec[q];
        const int64_t mt = p.m / kLeaf, nt = p.n / kLeaf;
        tiles64 += p.lower ? mt * (mt + 1) / 2 : mt * nt;
    }
    const int tl = tiles64 < 128 ? 32 : kLeaf;
    st.tl = tl;
    int64_t depth = 0;
    for (int q = 0; q < st.nspec; ++q) {
        const ProdSpec& p = st.spec[q];
        for (int ti = 0; ti < p.m / tl; ++ti)
            for (int tj = 0; tj < p.n / tl; ++tj) {
                if (p.lower && tj * tl / kLeaf > ti * tl / kLeaf) continue;
                int kb, ke;
                depth_range(p, tl, ti, tj, kb, ke);
                depth += std::max(0, ke - kb);
            }
    }
    const int64_t target = 8 * (tl == kLeaf ? 2 : 4) * 256;
    int ks = (int)std::min<int64_t>(1 << 20, (depth + target - 1) / target);
    ks = std::max(4 * kLeaf, (ks + kLeaf - 1) / kLeaf * kLeaf);
    int32_t part = 0;
    for (int q = 0; q < st.nspec; ++q) {
        const ProdSpec& p = st.spec[q];
        for (int ti = 0; ti < p.m / tl; ++ti)
            for (int tj = 0; tj < p.n / tl; ++tj) {
                if (p.lower && tj * tl / kLeaf > ti * tl / kLeaf) continue;
                int kb, ke;
                depth_range(p, tl, ti, tj, kb, ke);
                const int P = std::max(1, (ke - kb + ks - 1) / ks);
                for (int sl = 0; sl < P; ++sl) {
                    GemmItem it{};
                    it.ti = ti;
                    it.tj = tj;
                    it.kb = kb + sl * ks;
                    it.ke = std::min(ke, kb + (sl + 1) * ks);
                    it.s = sl;
                    it.part = sl > 0 ? part + sl - 1 : 0;
                    it.side = q;
                    items.push_back(it);
                }
                if (P > 1) {
                    red.push_back(GemmReduce{ti, tj, q, P, part, {0, 0, 0}});
                    part += P - 1;
                }
            }
    }
    npart = std::max<int64_t>(npart, part);
}

}  // namespace

void free_dense_plan(DensePlan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    if (p->items) (void)hipFree(p->items);
    if (p->red) (void)hipFree(p->red);
    if (p->part) (void)hipFree(p->part);
    delete p;
}

size_t dense_plan_bytes(const DensePlan* p) {
    if (!p) return 0;
    return sizeof(GemmItem) * (size_t)p->nitems + sizeof(GemmReduce) * (size_t)p->nred +
           sizeof(double) * kTile * (size_t)p->npart;
}

hipError_t dense_plan_for(DensePlan*& plan, int n, hipStream_t s) {
    const int np = dense_padded(n);
    if (plan && plan->np == np) return hipSuccess;
    free_dense_plan(plan);
    plan = nullptr;
    DensePlan* p = new DensePlan();
    p->np = np;
    plan_rec(p->steps, np, 0, np / kLeaf);
    std::vector<GemmItem> items;
    std::vector<GemmReduce> red;
    for (DensePlan::Step& st : p->steps) {
        if (st.leaf >= 0) continue;
        st.item0 = (int64_t)items.size();
        st.red0 = (int64_t)red.size();
        plan_items(st, items, red, p->npart);
        st.total = (int)((int64_t)items.size() - st.item0);
        st.nred = (int)((int64_t)red.size() - st.red0);
    }
    p->nitems = (int64_t)items.size();
    p->nred = (int64_t)red.size();

    hipError_t e = hipMalloc(&p->items, sizeof(GemmItem) * std::max<size_t>(1, items.size()));
    if (e == hipSuccess) e = hipMalloc(&p->red, sizeof(GemmReduce) * std::max<size_t>(1, red.size()));
    if (e == hipSuccess && p->npart > 0) e = hipMalloc(&p->part, sizeof(double) * kTile * (size_t)p->npart);
    if (e == hipSuccess && !items.empty())
        e = hipMemcpyAsync(p->items, items.data(), sizeof(GemmItem) * items.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !red.empty())
        e = hipMemcpyAsync(p->red, red.data(), sizeof(GemmReduce) * red.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host tables go out of scope
    if (e != hipSuccess) {
        free_dense_plan(p);
        return e;
    }
    plan = p;
    return hipSuccess;
}

void launch_gather_support(hipStream_t s, Support& sp, int n, const double* xyz0, double inv_r) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_support, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n, sp.orig,
                       xyz0, inv_r, sp.sx, sp.sy, sp.sz);
}

int dense_padded(int n) { return (n + kLeaf - 1) / kLeaf * kLeaf; }

int dense_pack_blocks() { return 256; }

namespace {

// The plan's launches on stream s.
void issue_plan(hipStream_t s, const Support& sp, int n, double* A, double* Md, double* Tb, int32_t* bad,
                const DensePlan* plan) {
    const int np = plan->np;
    const int64_t cnt = (int64_t)np * np;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)((cnt + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n, np, sp.sx,
                       sp.sy, sp.sz, A);
    double* bufs[3] = {A, Md, Tb};
    for (const DensePlan::Step& st : plan->steps) {
        if (st.leaf >= 0) {
            hipLaunchKernelGGL(k_leaf64, dim3(1), dim3(kBlock), 0, s, np, st.leaf, A, Md, Tb, bad);
            continue;
        }
        GemmLaunch g{};
        ReduceLaunch r{};
        for (int k = 0; k < st.nspec; ++k) {
            const ProdSpec& p = st.spec[k];
            g.side[k] = GemmSide{bufs[p.xb] + p.xo, bufs[p.yb] + p.yo, bufs[p.cb] + p.co, p.alpha, p.accumulate, p.y_rows};
            r.C[k] = bufs[p.cb] + p.co;
        }
        g.items = plan->items + st.item0;
        g.total = st.total;
        g.np = np;
        g.part = plan->part;
        if (st.tl == kLeaf) hipLaunchKernelGGL(k_gemm<kLeaf>, dim3((unsigned)st.total), dim3(kBlock), 0, s, g);
        else hipLaunchKernelGGL(k_gemm<32>, dim3((unsigned)st.total), dim3(kBlock), 0, s, g);
        if (st.nred > 0) {
            r.tiles = plan->red + st.red0;
            r.np = np;
            r.part = plan->part;
            const unsigned per = (unsigned)(st.tl * st.tl / kBlock);
            if (st.tl == kLeaf) hipLaunchKernelGGL(k_gemm_reduce<kLeaf>, dim3((unsigned)st.nred * per), dim3(kBlock), 0, s, r);
            else hipLaunchKernelGGL(k_gemm_reduce<32>, dim3((unsigned)st.nred * per), dim3(kBlock), 0, s, r);
        }
    }
}

}  // namespace

hipError_t launch_inverse_factor(hipStream_t s, const Support& sp, int n, double* A, double* Md, double* Tb,
                                 int32_t* bad, DensePlan* plan) {
    const std::vector<const void*> key = {A, Md, Tb, bad, sp.sx, sp.sy, sp.sz, reinterpret_cast<const void*>((intptr_t)n)};
    if (!plan->exec || plan->key != key) {
        if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
        plan->exec = nullptr;
        plan->key.clear();
        hipError_t e = hipSuccess;
        if (!plan->cap) e = hipStreamCreateWithFlags(&plan->cap, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        issue_plan(plan->cap, sp, n, A, Md, Tb, bad, plan);
        e = hipStreamEndCapture(plan->cap, &graph);
        if (e != hipSuccess) return e;
        e = hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            plan->exec = nullptr;
            return e;
        }
        plan->key = key;
    }
    return hipGraphLaunch(plan->exec, s);
}

void launch_pack_factor(hipStream_t s, int n, const double* Md, double* Mp, const double* old, double* red) {
    hipLaunchKernelGGL(k_pack_rows, dim3((unsigned)dense_pack_blocks()), dim3(kBigBlock), 0, s, n, dense_padded(n), Md,
                       Mp, old, red);
}

}  // namespace gcb
