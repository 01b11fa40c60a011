// HIP kernels for gfx950: RBF interpolant sweeps (Eq. 1 / Eq. 6), group
// argmax (Algorithm 1), starting-node rule, inverse-factor append and the
// FP64 certificate.  In the volume sweeps, the certificate and the
// large-group sweep every lane owns one target point and the support data is
// wave-uniform, read through the scalar cache (SGPR operands of the VALU
// ops) with no LDS staging; the group sweeps of smaller groups split each
// target's supports over the lanes of a wave and stage windows of supports
// in LDS between barriers.
#include "gcb_internal.h"
#include "gcb_kernels.h"
#include "gcb_device.h"

#include <algorithm>
#include <mutex>

namespace gcb {

#define GCB_LAUNCH(kern, grid, block, stream, ...) hipLaunchKernelGGL(kern, grid, block, 0, stream, __VA_ARGS__)

// Accumulate sum_{j in [s0, s1)} w_j phi(|t - s_j|) for one target per lane
// (full-accuracy phi: the greedy's certificate and monitor).
__device__ __forceinline__ void accumulate64(double tx, double ty, double tz, int s0, int s1,
                                             const double* __restrict__ sx, const double* __restrict__ sy,
                                             const double* __restrict__ sz, const double* __restrict__ wx,
                                             const double* __restrict__ wy, const double* __restrict__ wz,
                                             double& ax, double& ay, double& az) {
    int j = s0;
#pragma unroll 1
    for (; j + 4 <= s1; j += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double phi = wendland_r2(dist2(tx, ty, tz, sx[j + u], sy[j + u], sz[j + u]));
            ax = fma(wx[j + u], phi, ax);
            ay = fma(wy[j + u], phi, ay);
            az = fma(wz[j + u], phi, az);
        }
    }
#pragma unroll 1
    for (; j < s1; ++j) {
        const double phi = wendland_r2(dist2(tx, ty, tz, sx[j], sy[j], sz[j]));
        ax = fma(wx[j], phi, ax);
        ay = fma(wy[j], phi, ay);
        az = fma(wz[j], phi, az);
    }
}

// Volume form of the same sum (Eq. 6).  Points are scaled by 1/(2R) and
// centred at the first support; with u the target and v_j the supports
// (table vt), d = |u|^2 + |v_j|^2 - 2 u.v_j = |u - v_j|^2 costs three FMAs
// and an add per pair, the phi of wendland_quarter eleven more operations and
// the quarter-rate rsq, and the three weights three FMAs.  m = -2 u, uu = |u|^2.
__device__ __forceinline__ void accumulate_vol(double mx, double my, double mz, double uu, int n, const VolTable& vt,
                                               const double* __restrict__ wx, const double* __restrict__ wy,
                                               const double* __restrict__ wz, double& ax, double& ay, double& az) {
    const double* __restrict__ qx = vt.qx;
    const double* __restrict__ qy = vt.qy;
    const double* __restrict__ qz = vt.qz;
    const double* __restrict__ qq = vt.qq;
    int j = 0;
#pragma unroll 1
    for (; j + 8 <= n; j += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double d = fma(mx, qx[j + u], fma(my, qy[j + u], fma(mz, qz[j + u], uu + qq[j + u])));
            const double phi = wendland_quarter(d);
            ax = fma(wx[j + u], phi, ax);
            ay = fma(wy[j + u], phi, ay);
            az = fma(wz[j + u], phi, az);
        }
    }
#pragma unroll 1
    for (; j < n; ++j) {
        const double d = fma(mx, qx[j], fma(my, qy[j], fma(mz, qz[j], uu + qq[j])));
        const double phi = wendland_quarter(d);
        ax = fma(wx[j], phi, ax);
        ay = fma(wy[j], phi, ay);
        az = fma(wz[j], phi, az);
    }
}

// Target of a volume sweep: scaled by 1/(2R), centred at the first support
// (whose coordinates are kept scaled by 1/R).
struct VolTarget {
    double mx, my, mz, uu;
};

__device__ __forceinline__ VolTarget vol_target(double x, double y, double z, double inv_r, const SupportView& sv) {
    const double h = 0.5 * inv_r;
    const double ux = fma(x, h, -0.5 * sv.sx[0]), uy = fma(y, h, -0.5 * sv.sy[0]), uz = fma(z, h, -0.5 * sv.sz[0]);
    return VolTarget{-2.0 * ux, -2.0 * uy, -2.0 * uz, fma(uz, uz, fma(uy, uy, ux * ux))};
}

// ---------------------------------------------------------------- reductions
struct Best {
    double v;
    int32_t idx;   // decides ties (lowest wins)
    int32_t aux;
};

__device__ __forceinline__ bool better(double v, int32_t i, double bv, int32_t bi) {
    return v > bv || (v == bv && i < bi);
}

// Wave reductions (every lane of the wave active), with no LDS round trip.  The first four steps pair
// lanes inside each row of 16 with DPP lane moves: swaps within quads (xor 1, xor 2), then the half-row and
// row mirrors.  The last two combine rows 16 and 32 lanes apart with the permlane swaps: swapping a value
// with itself leaves the even and the odd rows (or the lower and the upper 32 lanes) in the two results of
// every lane.  Every step pairs each lane with a partner that pairs back with it, and both combine the same
// two values, so all lanes end with one identical result in a fixed order.
constexpr int kDppXor1 = 0xB1;          // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;          // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;   // lane i of each half row of 8 reads lane 7 - i
constexpr int kDppMirror = 0x140;       // lane i of each row of 16 reads lane 15 - i

template <int CTRL>
__device__ __forceinline__ int32_t dpp_i32(int32_t v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)dpp_i32<CTRL>((int32_t)(uint32_t)b);
    const uint32_t hi = (uint32_t)dpp_i32<CTRL>((int32_t)(uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// lo / hi: the value of the lower / upper partner (rows 16 apart with K32 = false, halves 32 apart with true)
template <bool K32>
__device__ __forceinline__ void swap_rows_u32(uint32_t x, uint32_t& lo, uint32_t& hi) {
    if constexpr (K32) {
        const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        lo = r[0];
        hi = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        lo = r[0];
        hi = r[1];
    }
}

template <bool K32>
__device__ __forceinline__ void swap_rows_f64(double x, double& lo, double& hi) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    uint32_t l0, h0, l1, h1;
    swap_rows_u32<K32>((uint32_t)b, l0, h0);
    swap_rows_u32<K32>((uint32_t)(b >> 32), l1, h1);
    lo = __longlong_as_double((long long)(((uint64_t)l1 << 32) | l0));
    hi = __longlong_as_double((long long)(((uint64_t)h1 << 32) | h0));
}

template <bool K32>
__device__ __forceinline__ double sum_rows_f64(double v) {
    double lo, hi;
    swap_rows_f64<K32>(v, lo, hi);
    return lo + hi;
}

template <bool K32>
__device__ __forceinline__ int32_t sum_rows_i32(int32_t v) {
    uint32_t lo, hi;
    swap_rows_u32<K32>((uint32_t)v, lo, hi);
    return (int32_t)(lo + hi);
}

template <bool K32>
__device__ __forceinline__ void best_step_rows(Best& b) {
    Best lo, hi;
    swap_rows_f64<K32>(b.v, lo.v, hi.v);
    uint32_t il, ih, al, ah;
    swap_rows_u32<K32>((uint32_t)b.idx, il, ih);
    swap_rows_u32<K32>((uint32_t)b.aux, al, ah);
    lo.idx = (int32_t)il; hi.idx = (int32_t)ih;
    lo.aux = (int32_t)al; hi.aux = (int32_t)ah;
    b = better(hi.v, hi.idx, lo.v, lo.idx) ? hi : lo;
}

template <int CTRL>
__device__ __forceinline__ void best_step_dpp(Best& b) {
    const double v = dpp_f64<CTRL>(b.v);
    const int32_t i = dpp_i32<CTRL>(b.idx);
    const int32_t a = dpp_i32<CTRL>(b.aux);
    if (better(v, i, b.v, b.idx)) { b.v = v; b.idx = i; b.aux = a; }
}

// Every lane ends with the same (v, idx); aux comes with it when that pair is held by a single lane (equal
// pairs keep the aux of whichever lane the pairing order reaches first).
__device__ __forceinline__ Best wave_best(Best b) {
    best_step_dpp<kDppXor1>(b);
    best_step_dpp<kDppXor2>(b);
    best_step_dpp<kDppHalfMirror>(b);
    best_step_dpp<kDppMirror>(b);
    best_step_rows<false>(b);
    best_step_rows<true>(b);
    return b;
}

// Block of kBlock threads: best over the block, valid in thread 0.
__device__ Best block_best(Best b) {
    __shared__ Best sh[kBlock / 64];
    b = wave_best(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kBlock / 64; ++i)
            if (better(sh[i].v, sh[i].idx, b.v, b.idx)) b = sh[i];
    }
    __syncthreads();
    return b;
}

template <int NT>
__device__ Best block_best_n(Best b) {
    __shared__ Best sh[NT / 64];
    b = wave_best(b);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < NT / 64; ++i)
            if (better(sh[i].v, sh[i].idx, b.v, b.idx)) b = sh[i];
    }
    __syncthreads();
    return b;
}

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<kDppXor1>(v);
    v += dpp_f64<kDppXor2>(v);
    v += dpp_f64<kDppHalfMirror>(v);
    v += dpp_f64<kDppMirror>(v);
    v = sum_rows_f64<false>(v);
    return sum_rows_f64<true>(v);
}

__device__ __forceinline__ double wave_min(double v) {
    v = fmin(v, dpp_f64<kDppXor1>(v));
    v = fmin(v, dpp_f64<kDppXor2>(v));
    v = fmin(v, dpp_f64<kDppHalfMirror>(v));
    v = fmin(v, dpp_f64<kDppMirror>(v));
    double lo, hi;
    swap_rows_f64<false>(v, lo, hi);
    v = fmin(lo, hi);
    swap_rows_f64<true>(v, lo, hi);
    return fmin(lo, hi);
}

__device__ __forceinline__ double wave_max(double v) { return -wave_min(-v); }

template <int NT>
__device__ double block_sum(double v) {
    __shared__ double sh[NT / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / 64; ++i) r += sh[i];
    __syncthreads();
    return r;   // valid in thread 0
}

__device__ __forceinline__ int32_t wave_isum(int32_t v) {
    v += dpp_i32<kDppXor1>(v);
    v += dpp_i32<kDppXor2>(v);
    v += dpp_i32<kDppHalfMirror>(v);
    v += dpp_i32<kDppMirror>(v);
    v = sum_rows_i32<false>(v);
    return sum_rows_i32<true>(v);
}

__device__ Best big_block_best(Best b) { return block_best_n<kBigBlock>(b); }

// Integer sum over a kBigBlock block, valid in thread 0.
__device__ int32_t big_block_isum(int32_t v) {
    __shared__ int32_t sh[kBigBlock / 64];
    v = wave_isum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    int32_t r = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBigBlock / 64; ++i) r += sh[i];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- iteration kernels
// One greedy iteration is three kernels; kernel boundaries are the only
// grid-wide synchronisation (no atomics, no spin waits), and every reduction
// runs in a fixed order, so results never depend on scheduling.
//   k_sweep    group sweep (a3): lanes of a block split the supports of a
//              few targets of the active group; one best record per block.
//   k_factor_l decision (a4) from the block records, b and l = M b (a5).
//   k_factor_u u = M^T l, new row of M, W update, commit of the iteration.
// The active group (g, its first permuted position t0, its size T) is a
// kernel argument: k advances by one every iteration, so the host knows it.
// Loads that do not depend on the decision are issued before it.

// Layout of a group sweep of T targets: `lpt` lanes share one target,
// each lane holds `tpl` targets; a block of kBlock threads holds
// (kBlock / lpt) * tpl targets.
Tuning g_tuning;

// lanes per target (lpt <= the tuning cap) and targets per lane for a group of T targets
inline void sweep_layout(int T, int& lpt, int& tpl) {
    // one wave per target measured fastest for groups of ~10^3 (each target reads every support
    // once, so wider layouts only add reduction work); groups of 4,097 to 8,192 hold 2 targets per
    // lane; above that k_sweep_lanes runs instead, and the 4-per-lane layout only bounds its record count
    if (T <= 512) { lpt = 128; tpl = 1; }
    else if (T <= 4096) { lpt = 64; tpl = 1; }
    else if (T <= 8192) { lpt = 64; tpl = 2; }
    else { lpt = 64; tpl = 4; }
    if (lpt > g_tuning.sweep_lpt_max) lpt = g_tuning.sweep_lpt_max;
}

__host__ __device__ inline int sweep_nblocks_dev(int T, int lpt, int tpl) {
    const int per = (kBlock / lpt) * tpl;
    return T > 0 ? (T + per - 1) / per : 1;
}

inline int sweep_nblocks(int T) {
    int lpt, tpl;
    sweep_layout(T, lpt, tpl);
    const int per = (kBlock / lpt) * tpl;
    return T > 0 ? (T + per - 1) / per : 1;
}

// Algorithm 1's decision for the iteration from the group's best candidate.
struct Decision {
    int32_t app, done, quiet;
    double E;
};

__device__ __forceinline__ Decision decide_local(int32_t done, int32_t quiet, int n, int32_t m, double e2,
                                                 double tol_abs, int64_t nc_max, int64_t cap) {
    Decision d;
    const bool have = e2 >= 0.0;
    d.E = have ? sqrt(e2) : 0.0;
    d.app = 0;
    d.done = done;
    d.quiet = quiet;
    if (have && d.E > tol_abs) {
        if (n < nc_max && n < cap) {
            d.app = 1;
            d.quiet = 0;
        } else if (n >= nc_max) {
            d.done = 2;
        } else {
            d.done = 4;   // factor capacity exhausted: the host reports an internal error
        }
    } else {
        d.quiet += 1;
    }
    if (d.done == 0 && !d.app && d.quiet >= m) d.done = 1;
    return d;
}

__device__ __forceinline__ bool better_rec(const ArgRec& a, const ArgRec& b) { return better(a.e2, a.orig, b.e2, b.orig); }


// Block variant: the wave's best `np` candidates (one per lane at most), in rank order on (e^2 descending,
// original index ascending), written as np consecutive records; a record with e2 = -1 marks no further
// candidate.  The first record carries the count of live candidates.  Every lane of the wave takes part.
__device__ __forceinline__ void write_top_records(ArgRec* __restrict__ out, int np, double e2, int32_t orig,
                                                  int32_t count, int32_t pos, double x, double y, double z,
                                                  double dx, double dy, double dz) {
    const int lane = threadIdx.x & 63;
    double v = e2;
    for (int r = 0; r < np; ++r) {
        const Best b = wave_best(Best{v, v >= 0.0 ? orig : 0x7fffffff, lane});
        const bool have = b.v >= 0.0;
        if (lane == (have ? b.aux : 0)) {
            ArgRec& o = out[r];
            o.e2 = have ? v : -1.0;
            o.orig = have ? orig : 0x7fffffff;
            o.pos = pos;
            o.count = r == 0 ? count : 0;
            o.x = x;
            o.y = y;
            o.z = z;
            o.dx = dx;
            o.dy = dy;
            o.dz = dz;
        }
        if (have && lane == b.aux) v = -1.0;   // taken
    }
}

// Supports staged in LDS per window: all loads of a window are issued at once.
constexpr int kStage = 1280;
// batched launches hold many more blocks: a smaller window keeps several blocks per CU
constexpr int kStageBatch = 256;

template <int STAGE, bool TOPK = false>
__device__ __forceinline__ void sweep_body(const SweepArgs& A, const int bid) {
    const GState* __restrict__ st = A.st;
    const int t0 = A.t0, T = A.T, lpt = A.lpt, tpl = A.tpl;
    const double* __restrict__ px = A.px;
    const double* __restrict__ py = A.py;
    const double* __restrict__ pz = A.pz;
    const double* __restrict__ pdx = A.pdx;
    const double* __restrict__ pdy = A.pdy;
    const double* __restrict__ pdz = A.pdz;
    const uint8_t* __restrict__ inS = A.inS;
    const int32_t* __restrict__ perm = A.perm;
    const SupportView sv = A.sv;
    const int64_t nub = A.nub;
    ArgRec* __restrict__ rec = A.rec;
    __shared__ double ls[6][STAGE];
    __shared__ double red[3][4][kBlock / 64];
    __shared__ int32_t s_n, s_done;
    const int groups = kBlock / lpt;                // target groups per block
    const int grp = threadIdx.x / lpt;
    const int gl = threadIdx.x % lpt;               // lane within the group
    const int tbase = (bid * groups + grp) * tpl;
    // |S| and the status, loaded by every lane with a zero offset held in a vector register (so they
    // issue as vector loads and nothing waits for them here); thread 0 publishes its values after the
    // other loads are issued
    int zero = 0;
    asm volatile("" : "+v"(zero));
    const int32_t st_n = st[zero].n, st_done = st[zero].done;
    // everything below is independent of |S| and is loaded in one round with the state:
    // the group's targets, what the candidate threads need, and the first window of supports
    double tx[4], ty[4], tz[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int t = min(tbase + q, T - 1);
        tx[q] = px[t0 + t];
        ty[q] = py[t0 + t];
        tz[q] = pz[t0 + t];
    }
    // candidate threads (one per target of the block) load what the record needs; the others repeat
    // thread 0's loads (same addresses, no traffic), so the loads carry no branch, and the membership byte
    // is tested only after the barrier (nothing waits for it here)
    const int ncand = groups * 4;
    const int tcand = (int)threadIdx.x < ncand ? (int)threadIdx.x : 0;
    const int ct = (bid * groups + tcand / 4) * tpl + tcand % 4;
    const int tc = min(ct, T - 1);
    const uint8_t cins = inS[t0 + tc];
    const double cdx = pdx[t0 + tc], cdy = pdy[t0 + tc], cdz = pdz[t0 + tc];
    const double cx = px[t0 + tc], cy = py[t0 + tc], cz = pz[t0 + tc];
    const int32_t corig = perm[t0 + tc];
    // the first 256 supports are staged with the state load; the rest of the first window once |S| is
    // known (a window of up to STAGE supports staged before |S| is known wastes bandwidth while |S| is small)
    const int w0eager = (int)min((int64_t)min(STAGE, 256), nub);
    for (int j = threadIdx.x; j < w0eager; j += kBlock) {
        ls[0][j] = sv.sx[j];
        ls[1][j] = sv.sy[j];
        ls[2][j] = sv.sz[j];
        ls[3][j] = sv.wx[j];
        ls[4][j] = sv.wy[j];
        ls[5][j] = sv.wz[j];
    }
    if (threadIdx.x == 0) {
        s_n = st_n;
        s_done = st_done;
    }
    __syncthreads();
    if (s_done) return;
    const int n = s_n;
    const bool clive = (int)threadIdx.x < ncand && tcand % 4 < tpl && ct < T && !cins;
    const int w0end = min(STAGE, n);
    if (w0end > w0eager) {
        for (int j = w0eager + threadIdx.x; j < w0end; j += kBlock) {
            ls[0][j] = sv.sx[j];
            ls[1][j] = sv.sy[j];
            ls[2][j] = sv.sz[j];
            ls[3][j] = sv.wx[j];
            ls[4][j] = sv.wy[j];
            ls[5][j] = sv.wz[j];
        }
        __syncthreads();
    }
    double ax[4] = {0, 0, 0, 0}, ay[4] = {0, 0, 0, 0}, az[4] = {0, 0, 0, 0};
    // windows after the first: each thread's share of window w + 1 is loaded into registers
    // while window w is evaluated, and stored to LDS between the two barriers
    constexpr int kPer = (STAGE + kBlock - 1) / kBlock;
    double nx[kPer], ny[kPer], nz[kPer], nwx[kPer], nwy[kPer], nwz[kPer];
    for (int w0 = 0; w0 < n; w0 += STAGE) {
        const int w1 = min(n, w0 + STAGE);
        if (w0 > 0) {
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int jj = threadIdx.x + kBlock * u;
                if (jj < STAGE && w0 + jj < w1) {
                    ls[0][jj] = nx[u];
                    ls[1][jj] = ny[u];
                    ls[2][jj] = nz[u];
                    ls[3][jj] = nwx[u];
                    ls[4][jj] = nwy[u];
                    ls[5][jj] = nwz[u];
                }
            }
            __syncthreads();
        }
        if (w1 < n) {
            const int w2 = min(n, w1 + STAGE);
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int jj = threadIdx.x + kBlock * u;
                const int j = min(w1 + jj, w2 - 1);
                nx[u] = sv.sx[j];
                ny[u] = sv.sy[j];
                nz[u] = sv.sz[j];
                nwx[u] = sv.wx[j];
                nwy[u] = sv.wy[j];
                nwz[u] = sv.wz[j];
            }
        }
        // four supports per step: independent dependency chains keep a lone wave busy
        int j = w0 + gl;
        if (tpl == 1) {
            double bx[4] = {0, 0, 0, 0}, by[4] = {0, 0, 0, 0}, bz[4] = {0, 0, 0, 0};
            for (; j + 3 * lpt < w1; j += 4 * lpt) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int jj = j + u * lpt - w0;
                    const double phi = wendland_r2(dist2(tx[0], ty[0], tz[0], ls[0][jj], ls[1][jj], ls[2][jj]));
                    bx[u] = fma(ls[3][jj], phi, bx[u]);
                    by[u] = fma(ls[4][jj], phi, by[u]);
                    bz[u] = fma(ls[5][jj], phi, bz[u]);
                }
            }
            ax[0] += (bx[0] + bx[1]) + (bx[2] + bx[3]);
            ay[0] += (by[0] + by[1]) + (by[2] + by[3]);
            az[0] += (bz[0] + bz[1]) + (bz[2] + bz[3]);
        }
        for (; j < w1; j += lpt) {
            const int jj = j - w0;
            const double sx = ls[0][jj], sy = ls[1][jj], sz = ls[2][jj];
            const double wx = ls[3][jj], wy = ls[4][jj], wz = ls[5][jj];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q < tpl) {
                    const double phi = wendland_r2(dist2(tx[q], ty[q], tz[q], sx, sy, sz));
                    ax[q] = fma(wx, phi, ax[q]);
                    ay[q] = fma(wy, phi, ay[q]);
                    az[q] = fma(wz, phi, az[q]);
                }
            }
        }
    }
    // sum over the lpt lanes of each target: a tree per wave, then the waves of a group in order
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q < tpl) {
            ax[q] = wave_sum(ax[q]);
            ay[q] = wave_sum(ay[q]);
            az[q] = wave_sum(az[q]);
            if (lane == 0) {
                red[0][q][wave] = ax[q];
                red[1][q][wave] = ay[q];
                red[2][q][wave] = az[q];
            }
        }
    }
    __syncthreads();
    // Every candidate is a lane of wave 0 (at most 16 per block): one lane per (group, q) forms the error of
    // target tbase + q, the wave takes the best on (e^2, original index) only (a total order over live
    // candidates), and its lane writes the full record (lane 0 when the block has no live candidate).
    if (wave != 0) return;
    double e2 = -1.0;
    if ((int)threadIdx.x < ncand && clive) {
        const int gq = threadIdx.x / 4, q = threadIdx.x % 4;
        const int wpg = lpt / 64;   // waves per group
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int w = 0; w < wpg; ++w) {
            fx += red[0][q][gq * wpg + w];
            fy += red[1][q][gq * wpg + w];
            fz += red[2][q][gq * wpg + w];
        }
        const double ex = fx - cdx, ey = fy - cdy, ez = fz - cdz;
        e2 = fma(ez, ez, fma(ey, ey, ex * ex));
    }
    const int32_t orig = clive ? corig : 0x7fffffff;
    if constexpr (TOPK) {
        write_top_records(rec + (size_t)bid * A.ptop, A.ptop, e2, orig, wave_isum(clive ? 1 : 0), t0 + ct, cx, cy,
                          cz, cdx, cdy, cdz);
        return;
    }
    const Best b = wave_best(Best{e2, orig, lane});
    const int32_t tot = wave_isum(clive ? 1 : 0);
    if (lane == (tot > 0 ? b.aux : 0)) {
        ArgRec& o = rec[bid];
        o.e2 = e2;
        o.orig = orig;
        o.pos = t0 + ct;
        o.count = tot;
        o.x = cx;
        o.y = cy;
        o.z = cz;
        o.dx = cdx;
        o.dy = cdy;
        o.dz = cdz;
    }
}

__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs A) { sweep_body<kStage>(A, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void k_sweep_top(SweepArgs A) { sweep_body<kStage, true>(A, blockIdx.x); }
// Groups of 4,097 to 8,192 targets (two targets per lane): many more blocks, so the small window keeps several
// blocks resident per CU.  With more than one target per lane every lane sums its supports in one sequence
// across windows, so the window size does not change any result.
__global__ __launch_bounds__(kBlock) void k_sweep_wide(SweepArgs A) { sweep_body<kStageBatch>(A, blockIdx.x); }
__global__ __launch_bounds__(kBlock) void k_sweep_wide_top(SweepArgs A) {
    sweep_body<kStageBatch, true>(A, blockIdx.x);
}
// Groups above 8,192 targets: one target per lane and 64 targets per block; the block's four waves take contiguous quarters
// of the supports, read through the scalar cache (no staging, no barrier until the end), and the quarter sums
// are added in a fixed order.  One best record per block, as in k_sweep.
constexpr int kLaneTargets = 64;

int sweep_lanes_blocks(int T) { return T > 0 ? (T + kLaneTargets - 1) / kLaneTargets : 1; }

template <bool TOPK>
__device__ __forceinline__ void sweep_lanes_body(const SweepArgs& A) {
    __shared__ double part[3][4][kLaneTargets];
    const GState st = *A.st;
    if (st.done) return;
    const int n = st.n;
    // wave-uniform quarter of the supports (readfirstlane: scalar loads of the supports)
    const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), tl = threadIdx.x & 63;
    const int t = blockIdx.x * kLaneTargets + tl;   // target within the group
    const int p = A.t0 + min(t, A.T - 1);
    const int s0 = (int)((int64_t)n * q / 4), s1 = (int)((int64_t)n * (q + 1) / 4);
    double ax = 0.0, ay = 0.0, az = 0.0;
    accumulate64(A.px[p], A.py[p], A.pz[p], s0, s1, A.sv.sx, A.sv.sy, A.sv.sz, A.sv.wx, A.sv.wy, A.sv.wz, ax, ay,
                 az);
    part[0][q][tl] = ax;
    part[1][q][tl] = ay;
    part[2][q][tl] = az;
    __syncthreads();
    if (q != 0) return;
    const bool live = t < A.T && !A.inS[p];
    double e2 = -1.0;
    if (live) {
        const double fx = (part[0][0][tl] + part[0][1][tl]) + (part[0][2][tl] + part[0][3][tl]);
        const double fy = (part[1][0][tl] + part[1][1][tl]) + (part[1][2][tl] + part[1][3][tl]);
        const double fz = (part[2][0][tl] + part[2][1][tl]) + (part[2][2][tl] + part[2][3][tl]);
        const double ex = fx - A.pdx[p], ey = fy - A.pdy[p], ez = fz - A.pdz[p];
        e2 = fma(ez, ez, fma(ey, ey, ex * ex));
    }
    const int32_t orig = live ? A.perm[p] : 0x7fffffff;
    if constexpr (TOPK) {
        write_top_records(A.rec + (size_t)blockIdx.x * A.ptop, A.ptop, e2, orig, wave_isum(live ? 1 : 0), p, A.px[p],
                          A.py[p], A.pz[p], A.pdx[p], A.pdy[p], A.pdz[p]);
        return;
    }
    const Best b = wave_best(Best{e2, orig, tl});
    const int32_t count = wave_isum(live ? 1 : 0);
    // live targets have distinct original indices, so the best lane is unique; with none, lane 0 writes
    if (count > 0 ? tl == b.aux : tl == 0) {
        ArgRec& o = A.rec[blockIdx.x];
        o.e2 = e2;
        o.orig = orig;
        o.pos = p;
        o.count = count;
        o.x = A.px[p];
        o.y = A.py[p];
        o.z = A.pz[p];
        o.dx = A.pdx[p];
        o.dy = A.pdy[p];
        o.dz = A.pdz[p];
    }
}

__global__ __launch_bounds__(kBlock) void k_sweep_lanes(SweepArgs A) { sweep_lanes_body<false>(A); }
__global__ __launch_bounds__(kBlock) void k_sweep_lanes_top(SweepArgs A) { sweep_lanes_body<true>(A); }

// l = M b, one wave per row of M (kRowsL rows per block); b_j = phi(|r_new -
// s_j| / R) staged in LDS windows.  Block partials Pb[blk] = (b.W over
// columns [i0, i0 + kRowsL), l.l over rows [i0, i0 + kRowsL)).  Before that,
// every block reduces the sweep records (nrec of them) to the group maximum
// and takes the decision; block 0 stores it.  With init_t >= 0 the node is
// the starting node init[init_t] instead.
template <int RPW>
__device__ __forceinline__ void factor_l_body(const FactorLArgs& A, const int bid) {
    GState* __restrict__ st = A.st;
    IterRec* __restrict__ irec = A.irec;
    const ArgRec* __restrict__ srec = A.srec;
    const int nrec = A.nrec;
    const int32_t m = A.m;
    const int g = A.g;
    const int init_t = A.init_t;
    const int32_t* __restrict__ init = A.init;
    const int32_t* __restrict__ pos_of = A.pos_of;
    const double* __restrict__ px = A.px;
    const double* __restrict__ py = A.py;
    const double* __restrict__ pz = A.pz;
    const double* __restrict__ pdx = A.pdx;
    const double* __restrict__ pdy = A.pdy;
    const double* __restrict__ pdz = A.pdz;
    const SupportView sv = A.sv;
    const double* __restrict__ Mr = A.Mr;
    double* __restrict__ l = A.l;
    double* __restrict__ Pb = A.Pb;
    const double tol_abs = A.tol_abs;
    const int64_t nc_max = A.nc_max, cap = A.cap;
    int32_t* __restrict__ log_group = A.log_group;
    int32_t* __restrict__ log_node = A.log_node;
    double* __restrict__ log_err = A.log_err;
    int8_t* __restrict__ log_app = A.log_app;
    const int64_t log_cap = A.log_cap;
    __shared__ double bw[kBWindow];
    __shared__ double sl[kRowsL * RPW];
    __shared__ int32_t s_n, s_done;
    __shared__ double s_we2[kBigBlock / 64];
    __shared__ int32_t s_wor[kBigBlock / 64], s_cnt[kBigBlock / 64];
    __shared__ double s_win[6];
    __shared__ int32_t s_winpos;
    __shared__ int32_t s_app;
    __shared__ double s_q[3];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    constexpr int rpw = RPW;             // rows of M per wave
    constexpr int rpb = kRowsL * rpw;    // rows of M per block
    // Thread 0 reads the fields of the state it needs into registers and publishes |S| and the status to
    // the block only after the other loads are issued: loads that depend neither on |S| nor on the
    // decision (support coordinates of the first b window and of this block's b.W slice) then arrive in
    // the round trip of the state and the records.
    // (Every lane loads them with a zero offset held in a vector register, so they issue as vector loads
    // and no wait is placed before the other loads; only thread 0's values are used.)
    int zero = 0;
    asm volatile("" : "+v"(zero));
    const GState& stv = st[zero];
    const int32_t st_n = stv.n, st_done = stv.done, st_quiet = stv.quiet;
    const int64_t st_log = stv.log_len;
    const uint64_t st_pairs = stv.pairs_group;
    constexpr int kBPre = 1;
    double pbx[kBPre], pby[kBPre], pbz[kBPre];
#pragma unroll
    for (int u = 0; u < kBPre; ++u) {
        const int j = min((int)threadIdx.x + kBigBlock * u, (int)cap - 1);
        pbx[u] = sv.sx[j];
        pby[u] = sv.sy[j];
        pbz[u] = sv.sz[j];
    }
    double wsx = 0.0, wsy = 0.0, wsz = 0.0, wwx = 0.0, wwy = 0.0, wwz = 0.0;
    if (wave == 0 && lane < kRowsL) {
        const int j = min((int)bid * rpb + lane, (int)cap - 1);
        wsx = sv.sx[j]; wsy = sv.sy[j]; wsz = sv.sz[j];
        wwx = sv.wx[j]; wwy = sv.wy[j]; wwz = sv.wz[j];
    }
    // each thread keeps the best of its records on (e^2, original index), with its fields
    double be2 = -1.0, bx = 0.0, by = 0.0, bz = 0.0, bdx = 0.0, bdy = 0.0, bdz = 0.0;
    int32_t bor = 0x7fffffff, bpos = -1, c = 0;
    if (init_t < 0) {
        for (int i = threadIdx.x; i < nrec; i += kBigBlock) {
            // whole records with selects: every field is loaded at once, nothing stays in flight
            const ArgRec x = srec[i];
            const bool bt = better(x.e2, x.orig, be2, bor);
            be2 = bt ? x.e2 : be2; bor = bt ? x.orig : bor; bpos = bt ? x.pos : bpos;
            bx = bt ? x.x : bx; by = bt ? x.y : by; bz = bt ? x.z : bz;
            bdx = bt ? x.dx : bdx; bdy = bt ? x.dy : bdy; bdz = bt ? x.dz : bdz;
            c += x.count;
        }
    }
    if (threadIdx.x == 0) {
        s_n = st_n;
        s_done = st_done;
    }
    // Everything loaded so far has arrived (the records came last); waiting for it here, where it costs
    // nothing, keeps the loads of M below free to stay in flight through the decision.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (init_t < 0 && s_done) {
        if (bid == 0 && threadIdx.x == 0) {
            irec->app = 0;
            irec->ran = 0;
        }
        return;
    }
    const int n = init_t >= 0 ? init_t : s_n;
    const int i0 = bid * rpb;
    const int i = i0 + wave;   // first of this wave's rows i, i + kRowsL, ...
    // this wave's row of M, loaded while the decision is taken
    constexpr int kRowPre = 16;
    double mrow[kRowPre];
    const double* Mi = Mr + (size_t)i * (i + 1) / 2;
#pragma unroll
    for (int u = 0; u < kRowPre; ++u) {
        const int j = lane + 64 * u;
        mrow[u] = (i < n && j <= i) ? Mi[j] : 0.0;
    }
    if (init_t >= 0) {
        if (threadIdx.x == 0) {
            const int o = init[init_t];
            const int p = pos_of[o];
            s_app = 1;
            s_q[0] = px[p];
            s_q[1] = py[p];
            s_q[2] = pz[p];
            if (bid == 0) {
                irec->n = init_t;
                irec->app = 1;
                irec->init = 1;
                irec->ran = 0;
                irec->node_pos = p;
                irec->node_orig = o;
                irec->E = 0.0;
                irec->x = px[p];
                irec->y = py[p];
                irec->z = pz[p];
                irec->dx = pdx[p];
                irec->dy = pdy[p];
                irec->dz = pdz[p];
            }
        }
    } else {
        // block-wide best: per wave, then waves in order (a total order, so the result is unique)
        const Best wb = wave_best(Best{be2, bor, 0});
        const double we2 = wb.v;
        const int32_t wor = wb.idx;
        c = wave_isum(c);
        if (lane == 0) {
            s_we2[wave] = we2;
            s_wor[wave] = wor;
            s_cnt[wave] = c;
        }
        __syncthreads();
        // every wave reduces the per-wave bests itself (its first lanes read them), so all threads know the
        // block's best and count with no serial pass and no further barrier
        const bool has = lane < kBigBlock / 64;
        const Best bb = wave_best(Best{has ? s_we2[lane] : -1.0, has ? s_wor[lane] : 0x7fffffff, 0});
        const int32_t total = wave_isum(has ? s_cnt[lane] : 0);
        // the thread holding the winning record publishes its fields (original indices are unique)
        if (be2 >= 0.0 && bor == bb.idx) {
            s_win[0] = bx; s_win[1] = by; s_win[2] = bz; s_win[3] = bdx; s_win[4] = bdy; s_win[5] = bdz;
            s_winpos = bpos;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            ArgRec b;
            b.e2 = bb.v;
            b.orig = bb.idx;
            if (b.e2 >= 0.0) {
                b.pos = s_winpos;
                b.x = s_win[0]; b.y = s_win[1]; b.z = s_win[2];
                b.dx = s_win[3]; b.dy = s_win[4]; b.dz = s_win[5];
            } else {
                b.pos = -1;
                b.x = b.y = b.z = b.dx = b.dy = b.dz = 0.0;
            }
            const Decision d = decide_local(st_done, st_quiet, n, m, b.e2, tol_abs, nc_max, cap);   // thread 0
            s_app = d.app;
            s_q[0] = b.x;
            s_q[1] = b.y;
            s_q[2] = b.z;
            if (bid == 0) {
                if (d.done != 4) {
                    const int64_t it = st_log;
                    if (it < log_cap) {
                        log_group[it] = g;
                        log_node[it] = b.e2 >= 0.0 ? b.orig : -1;
                        log_err[it] = d.E;
                        log_app[it] = (int8_t)d.app;
                    }
                    st->log_len = it + 1;
                    st->pairs_group = st_pairs + (uint64_t)total * (uint64_t)n;
                }
                st->quiet = d.quiet;
                st->done = d.done;
                irec->n = n;
                irec->app = d.app;
                irec->init = 0;
                irec->ran = d.done != 4;
                irec->node_pos = d.app ? b.pos : -1;
                irec->node_orig = d.app ? b.orig : -1;
                irec->E = d.E;
                irec->x = b.x;
                irec->y = b.y;
                irec->z = b.z;
                irec->dx = b.dx;
                irec->dy = b.dy;
                irec->dz = b.dz;
            }
        }
    }
    __syncthreads();
    if (!s_app) return;
    const int nblk = max(1, (n + rpb - 1) / rpb);
    if ((int)bid >= nblk) return;
    const int i1 = min(n, i0 + rpb);
    const double qx = s_q[0], qy = s_q[1], qz = s_q[2];
    double acc[RPW];
#pragma unroll
    for (int r = 0; r < RPW; ++r) acc[r] = 0.0;
    for (int w0 = 0; w0 < i1; w0 += kBWindow) {
        const int w1 = min(i1, w0 + kBWindow);
        __syncthreads();
        if (w0 == 0) {
#pragma unroll
            for (int u = 0; u < kBPre; ++u) {
                const int j = threadIdx.x + kBigBlock * u;
                if (j < w1) bw[j] = wendland_r2(dist2(qx, qy, qz, pbx[u], pby[u], pbz[u]));
            }
            for (int j = threadIdx.x + kBigBlock * kBPre; j < w1; j += kBigBlock)
                bw[j] = wendland_r2(dist2(qx, qy, qz, sv.sx[j], sv.sy[j], sv.sz[j]));
        } else {
            for (int j = w0 + threadIdx.x; j < w1; j += kBigBlock)
                bw[j - w0] = wendland_r2(dist2(qx, qy, qz, sv.sx[j], sv.sy[j], sv.sz[j]));
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int ir = i + kRowsL * r;
            if (ir < i1) {
                const double* Mir = Mr + (size_t)ir * (ir + 1) / 2;
                const int je = min(w1, ir + 1);
                int j = w0 + lane;
                double a0 = 0.0, a1 = 0.0;
                if (w0 == 0) {
                    // the same summation order for every row, whichever wave and round holds it
#pragma unroll
                    for (int u = 0; u < kRowPre; ++u) {
                        const int jj = lane + 64 * u;
                        if (jj < je) a0 = fma(r == 0 ? mrow[u] : Mir[jj], bw[jj], a0);
                    }
                    j = lane + 64 * kRowPre;
                }
                for (; j + 64 < je; j += 128) {
                    const double m0 = Mir[j], m1 = Mir[j + 64];
                    a0 = fma(m0, bw[j - w0], a0);
                    a1 = fma(m1, bw[j + 64 - w0], a1);
                }
                if (j < je) a0 = fma(Mir[j], bw[j - w0], a0);
                acc[r] += a0 + a1;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int ir = i + kRowsL * r;
        const double li = wave_sum(acc[r]);
        if (lane == 0 && ir < i1) {
            l[ir] = li;
            sl[kRowsL * r + wave] = li;
        }
    }
    __syncthreads();
    if (wave == 0) {
        // shares of b.W and l.l per chunk of kRowsL rows (chunk index i / kRowsL, whatever
        // the rows per block), each in the wave-tree order, so the sums do not depend on rpw
        for (int r = 0; r < rpw; ++r) {
            const int c0 = i0 + kRowsL * r;
            if (r > 0 && c0 >= i1) break;   // chunk 0 is always written (zeros while |S| = 0)
            double fx = 0.0, fy = 0.0, fz = 0.0, ll = 0.0;
            const int j = c0 + lane;
            if (lane < kRowsL && j < i1) {
                double sx = wsx, sy = wsy, sz = wsz, wx = wwx, wy = wwy, wz = wwz;
                if (r > 0) {
                    sx = sv.sx[j]; sy = sv.sy[j]; sz = sv.sz[j];
                    wx = sv.wx[j]; wy = sv.wy[j]; wz = sv.wz[j];
                }
                const double bj = wendland_r2(dist2(qx, qy, qz, sx, sy, sz));
                fx = bj * wx;
                fy = bj * wy;
                fz = bj * wz;
                ll = sl[kRowsL * r + lane] * sl[kRowsL * r + lane];
            }
            fx = wave_sum(fx);
            fy = wave_sum(fy);
            fz = wave_sum(fz);
            ll = wave_sum(ll);
            if (lane == 0) {
                const int cb = c0 / kRowsL;
                Pb[4 * cb + 0] = fx;
                Pb[4 * cb + 1] = fy;
                Pb[4 * cb + 2] = fz;
                Pb[4 * cb + 3] = ll;
            }
        }
    }
}

__global__ __launch_bounds__(kBigBlock) void k_factor_l(FactorLArgs A) { factor_l_body<1>(A, blockIdx.x); }

// u = M^T l, one wave per column j of M read from the column-major copy Mc
// (column j holds rows j.. at offset j*cap - j(j-1)/2).  Every block first
// sums the k_factor_l partials in block order to s = 1 - l.l and
// e = d_new - b.W.  Writes the new row [-u^T/sqrt(s), 1/sqrt(s)] into both
// copies of M and W <- [W - u e/s; e/s]; block 0 commits the iteration.
template <int RPW, bool PREW = false>
__device__ __forceinline__ void factor_u_body(const FactorUArgs& A, const int bid) {
    GState* __restrict__ st = A.st;
    const IterRec* __restrict__ irec = A.irec;
    uint8_t* __restrict__ inS = A.inS;
    const SupportMut sm = A.sm;
    double* __restrict__ Mc = A.Mc;
    const int64_t cap = A.cap;
    const double* __restrict__ l = A.l;
    const double* __restrict__ Pb = A.Pb;
    __shared__ double part[4][kBigBlock / 64];
    __shared__ double sh[4];
    __shared__ int32_t s_bad;
    constexpr int rpw = RPW;             // columns of M per wave
    constexpr int rpb = kRowsL * rpw;    // columns of M per block (as in k_factor_l)
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int j = bid * rpb + wave;   // first of this wave's columns j, j + kRowsL, ...
    // With PREW, the W entries of this wave's columns are loaded with the iteration record (bounded by the
    // capacity; used only for columns below n), so that the update at the end needs no further round
    // trip; the batched kernels, short of registers, read them at the end.
    double wox[RPW], woy[RPW], woz[RPW];
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
        const int jq = j + kRowsL * q;
        const bool ok = PREW && lane == 0 && jq < cap;
        wox[q] = ok ? sm.wx[jq] : 0.0;
        woy[q] = ok ? sm.wy[jq] : 0.0;
        woz[q] = ok ? sm.wz[jq] : 0.0;
    }
    // the iteration record is only read here (k_factor_l wrote it), so every block sees the same values
    const IterRec r = *irec;
    // this thread's share of the k_factor_l partials (masked once n is known)
    double pv[4] = {0.0, 0.0, 0.0, 0.0};
    const int nbl_cap = (int)((cap + kRowsL - 1) / kRowsL);   // partials come per chunk of kRowsL rows
    if ((int)threadIdx.x < nbl_cap) {
#pragma unroll
        for (int c = 0; c < 4; ++c) pv[c] = Pb[4 * threadIdx.x + c];
    }
    if (!r.app) return;
    const int n = r.n;
    const int ncb = max(1, (n + kRowsL - 1) / kRowsL);
    if ((int)bid >= max(1, (n + rpb - 1) / rpb)) return;
    // column j of M and the matching entries of l, loaded before s is known
    constexpr int kColPre = 16;
    double mc[kColPre], lv[kColPre];
    const double* col = Mc + (size_t)j * cap - (size_t)j * (j - 1) / 2;   // rows j.. of column j
#pragma unroll
    for (int u = 0; u < kColPre; ++u) {
        const int ii = j + lane + 64 * u;
        const bool ok = j < n && ii < n;
        mc[u] = ok ? col[ii - j] : 0.0;
        lv[u] = ok ? l[ii] : 0.0;
    }
    {
        // fixed-order reduction: per thread in block order, a tree per wave, waves in order (thread 0 reads
        // the 16 wave sums with independent loads)
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        if ((int)threadIdx.x < ncb) {
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] = pv[c];
        }
        for (int b = threadIdx.x + kBigBlock; b < ncb; b += kBigBlock)
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] += Pb[4 * b + c];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            v[c] = wave_sum(v[c]);
            if (lane == 0) part[c][wave] = v[c];
        }
        __syncthreads();
        // lanes 0..3 form 1 / sqrt(s) and the three e / s side by side (each sums the wave totals in block
        // order, as one thread would): one sum chain, one square root and one division deep
        if (threadIdx.x < 4) {
            const int k = threadIdx.x;
            const int c = k > 0 ? k - 1 : 0;
            double fc = 0.0, f3 = 0.0;
            for (int t = 0; t < kBigBlock / 64; ++t) {
                fc += part[c][t];
                f3 += part[3][t];
            }
            const double s = 1.0 - f3;
            const double dk = k == 1 ? r.dx : (k == 2 ? r.dy : r.dz);
            sh[k] = k == 0 ? 1.0 / sqrt(s) : (dk - fc) / s;
            if (k == 0) s_bad = !(s > kSingularTol);
        }
        __syncthreads();
    }
    if (s_bad) {
        if (bid == 0 && threadIdx.x == 0) {
            st->done = 3;
            st->singular_node = r.node_orig;
        }
        return;
    }
    const double rs = sh[0], cx = sh[1], cy = sh[2], cz = sh[3];
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
        const int jq = j + kRowsL * q;
        if (jq < n) {
            double* cq = Mc + (size_t)jq * cap - (size_t)jq * (jq - 1) / 2;
            double a0 = 0.0, a1 = 0.0;
            // an accumulator defined here keeps the first products from being folded into the prefetch
            // above, where they would wait for its first loads before the others are issued
            asm volatile("" : "+v"(a0));
            // the same summation order for every column, whichever wave and round holds it
#pragma unroll
            for (int u = 0; u < kColPre; ++u) {
                if (q == 0) {
                    a0 = fma(mc[u], lv[u], a0);
                } else {
                    const int ii = jq + lane + 64 * u;
                    if (ii < n) a0 = fma(cq[ii - jq], l[ii], a0);
                }
            }
            int ii = jq + lane + 64 * kColPre;
            for (; ii + 64 < n; ii += 128) {
                a0 = fma(cq[ii - jq], l[ii], a0);
                a1 = fma(cq[ii + 64 - jq], l[ii + 64], a1);
            }
            if (ii < n) a0 = fma(cq[ii - jq], l[ii], a0);
            const double u = wave_sum(a0 + a1);
            if (lane == 0) {
                const double v = -u * rs;
                sm.M[(size_t)n * (n + 1) / 2 + jq] = v;
                cq[n - jq] = v;
                sm.wx[jq] = fma(-u, cx, PREW ? wox[q] : sm.wx[jq]);
                sm.wy[jq] = fma(-u, cy, PREW ? woy[q] : sm.wy[jq]);
                sm.wz[jq] = fma(-u, cz, PREW ? woz[q] : sm.wz[jq]);
            }
        }
    }
    if (bid == 0 && threadIdx.x == 0) {
        const int p = r.node_pos;
        sm.M[(size_t)n * (n + 1) / 2 + n] = rs;
        Mc[(size_t)n * cap - (size_t)n * (n - 1) / 2] = rs;
        sm.wx[n] = cx;
        sm.wy[n] = cy;
        sm.wz[n] = cz;
        sm.sx[n] = r.x;
        sm.sy[n] = r.y;
        sm.sz[n] = r.z;
        sm.orig[n] = r.node_orig;
        inS[p] = 1;
        st->n = n + 1;
        if (r.init) st->init_left -= 1;   // starting nodes are not loop appends
        else st->pairs_append += (uint64_t)n;
    }
}

__global__ __launch_bounds__(kBigBlock) void k_factor_u(FactorUArgs A) { factor_u_body<1, true>(A, blockIdx.x); }

// ---------------------------------------------------------------- several nodes per iteration (block variant)
// The peak-selection idea cited in Section 1 in block form: one sweep ranks the active group's nodes over E*
// and up to p of them are appended together.  With Phi_S = L L^T, M = L^-1, B = phi(S, new) (n x q) and
// C = phi(new, new) (q x q), the bordered factor is [[L, 0], [Lambda^T, L22]] with Lambda = M B and
// L22 L22^T = C - Lambda^T Lambda; the new rows of M are [-L22^-1 U^T, L22^-1] with U = M^T Lambda, and
// W' = [W - U Z ; Z] with Z = L22^-T L22^-1 (D_new - B^T W).  The pivots of L22 are the values 1 - l.l that
// q single appends in rank order would meet, checked against the same threshold.
//   k_sweep_top / _wide_top / _lanes_top  each block's best candidates in rank order (SweepArgs.ptop records)
//   k_factor_l_blk  every block: the group's best p over all records and the decision (block 0 logs it);
//                   Lambda = M B by rows (B staged in LDS windows), per-chunk partials of B^T W, Lambda^T Lambda
//   k_factor_u_blk  partials summed, the q x q Cholesky and inverse, U = M^T Lambda by columns, new rows, W

// Order LDS accesses of one wave (its DS instructions complete in order).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// The best `np` of the candidates the wave's lanes hold (KPL each; e2 < 0 marks none), in rank order, written
// to out_*[0..np) by the winning lanes (e2 = -1, index -1 past the last candidate).  Taken candidates are
// cleared from the lanes' registers.  Every lane of the wave takes part.
template <int KPL>
__device__ __forceinline__ void wave_top(double (&e)[KPL], const int32_t (&o)[KPL], const int32_t (&ix)[KPL], int np,
                                         double* __restrict__ out_e, int32_t* __restrict__ out_o,
                                         int32_t* __restrict__ out_ix) {
    const int lane = threadIdx.x & 63;
    for (int r = 0; r < np; ++r) {
        double be = -1.0;
        int32_t bo = 0x7fffffff, bi = -1;
#pragma unroll
        for (int k = 0; k < KPL; ++k)
            if (e[k] >= 0.0 && better(e[k], o[k], be, bo)) { be = e[k]; bo = o[k]; bi = ix[k]; }
        const Best b = wave_best(Best{be, bo, lane});
        const bool have = b.v >= 0.0;
        if (have && lane == b.aux) {
            out_e[r] = be;
            out_o[r] = bo;
            out_ix[r] = bi;
#pragma unroll
            for (int k = 0; k < KPL; ++k)
                if (e[k] >= 0.0 && o[k] == bo) e[k] = -1.0;
        }
        if (!have && lane == 0) {
            out_e[r] = -1.0;
            out_o[r] = 0x7fffffff;
            out_ix[r] = -1;
        }
    }
}

constexpr int kSelRec = 8;                         // records per thread per tile of the selection kernel
constexpr int kSelLists = kBigBlock / 64 + 1;      // the 16 wave lists and the running list

// Offset in a chunk's kBlkPart partials of needed value v < 3 q + q^2 (b_t.W first, then lambda_t.lambda_u).
__device__ __forceinline__ int blk_part_offset(int v, int q) {
    if (v < 3 * q) return v;
    const int y = v - 3 * q, t = y / q;
    return 3 * kMaxPerIter + t * kMaxPerIter + (y - t * q);
}

// Every block of k_factor_l_blk ranks the group's records itself (tiles of kBigBlock * kSelRec records:
// per wave, then merged by wave 0 into a running list) and takes Algorithm 1's decision in block form, so all
// blocks agree with no grid-wide step; block 0 logs it and writes the decision record.  Returns q (0: no
// append), leaves the nodes' coordinates in nd[3][Q] and |S| in *n.
template <int Q>
__device__ int block_select(const FactorBlkArgs& A, const GState& st, double (&nd)[3][Q], int* n_out) {
    constexpr int kSelMerge = (kSelLists * Q + 63) / 64;
    __shared__ double w_e[kSelLists][Q];
    __shared__ int32_t w_o[kSelLists][Q], w_i[kSelLists][Q];
    __shared__ int32_t s_cnt[kBigBlock / 64];
    __shared__ int32_t s_q;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int np = A.ptop;
    constexpr int run = kSelLists - 1;   // the running list
    if (threadIdx.x < Q) {
        w_e[run][threadIdx.x] = -1.0;
        w_o[run][threadIdx.x] = 0x7fffffff;
        w_i[run][threadIdx.x] = -1;
    }
    int32_t cnt = 0;
    for (int base = 0; base < A.nrec; base += kBigBlock * kSelRec) {
        double e[kSelRec];
        int32_t o[kSelRec], ix[kSelRec];
#pragma unroll
        for (int k = 0; k < kSelRec; ++k) {
            const int i = base + (int)threadIdx.x + kBigBlock * k;
            const bool ok = i < A.nrec;
            const int ii = ok ? i : 0;
            const double ev = A.srec[ii].e2;
            const int32_t ov = A.srec[ii].orig, cv = A.srec[ii].count;
            e[k] = ok ? ev : -1.0;
            o[k] = ok ? ov : 0x7fffffff;
            ix[k] = i;
            cnt += ok ? cv : 0;
        }
        wave_top<kSelRec>(e, o, ix, np, w_e[wave], w_o[wave], w_i[wave]);
        __syncthreads();
        if (wave == 0) {
            double me[kSelMerge];
            int32_t mo[kSelMerge], mi[kSelMerge];
#pragma unroll
            for (int k = 0; k < kSelMerge; ++k) {
                const int x = lane + 64 * k;
                const int li = x / Q, r = x - li * Q;
                const bool ok = li < kSelLists && r < np;
                me[k] = ok ? w_e[ok ? li : 0][r] : -1.0;
                mo[k] = ok ? w_o[ok ? li : 0][r] : 0x7fffffff;
                mi[k] = ok ? w_i[ok ? li : 0][r] : -1;
            }
            wave_lds_sync();
            wave_top<kSelMerge>(me, mo, mi, np, w_e[run], w_o[run], w_i[run]);
        }
        __syncthreads();
    }
    cnt = wave_isum(cnt);
    if (lane == 0) s_cnt[wave] = cnt;
    __syncthreads();
    const int n = st.n;
    if (threadIdx.x == 0) {
        int have = 0;
        while (have < np && w_e[run][have] >= 0.0) ++have;
        const double E = have > 0 ? sqrt(w_e[run][0]) : 0.0;
        int over = 0;
        while (over < have && sqrt(w_e[run][over]) > A.tol_abs) ++over;
        int q = 0;
        int32_t done = 0, quiet = st.quiet;
        if (over > 0) {
            if (n < A.nc_max) {
                q = (int)min((int64_t)over, A.nc_max - n);
                if (n + q > A.cap) {
                    done = 4;   // factor capacity exhausted: the host reports an internal error
                    q = 0;
                } else {
                    quiet = 0;
                }
            } else {
                done = 2;
            }
        } else {
            quiet += 1;
        }
        if (done == 0 && q == 0 && quiet >= A.m) done = 1;
        if (blockIdx.x == 0) {
            if (done != 4) {
                uint64_t total = 0;
                for (int w = 0; w < kBigBlock / 64; ++w) total += (uint64_t)s_cnt[w];
                const int64_t it = st.log_len;
                if (it < A.log_cap) {
                    A.log_group[it] = A.g;
                    A.log_node[it] = have > 0 ? w_o[run][0] : -1;
                    A.log_err[it] = E;
                    A.log_app[it] = (int8_t)q;
                }
                A.st->log_len = it + 1;
                A.st->pairs_group = st.pairs_group + total * (uint64_t)n;
            }
            A.st->quiet = quiet;
            A.st->done = done;
            A.brec->n = n;
            A.brec->q = q;
        }
        s_q = q;
    }
    __syncthreads();
    const int q = s_q;
    if ((int)threadIdx.x < q) {
        const int t = threadIdx.x;
        const ArgRec r = A.srec[w_i[run][t]];
        nd[0][t] = r.x;
        nd[1][t] = r.y;
        nd[2][t] = r.z;
        if (blockIdx.x == 0) {
            A.brec->pos[t] = r.pos;
            A.brec->orig[t] = r.orig;
            A.brec->x[t] = r.x;
            A.brec->y[t] = r.y;
            A.brec->z[t] = r.z;
            A.brec->dx[t] = r.dx;
            A.brec->dy[t] = r.dy;
            A.brec->dz[t] = r.dz;
        }
    }
    __syncthreads();
    *n_out = n;
    return q;
}

// The selection (block_select), then Lambda = M B: one wave per row of M (kRowsL rows per block, one chunk),
// B staged in LDS windows of kBWindow / Q supports x q nodes; then this chunk's partials of B^T W (rows of B in
// the chunk) and Lambda^T Lambda, each summed over the chunk's rows in order.
template <int Q>
__global__ __launch_bounds__(kBigBlock) void k_factor_l_blk(FactorBlkArgs A) {
    __shared__ double bw[kBWindow];
    __shared__ double s_nd[3][Q];
    __shared__ double s_lam[kRowsL][Q];
    __shared__ double s_bw[kRowsL][Q][3];
    const GState st = *A.st;
    if (st.done) {
        if (blockIdx.x == 0 && threadIdx.x == 0) A.brec->q = 0;
        return;
    }
    if (blockIdx.x > 0 && (int)blockIdx.x * kRowsL >= st.n) return;   // no rows of M here (block 0 decides)
    int n = 0;
    const int q = block_select<Q>(A, st, s_nd, &n);
    if (q <= 0) return;
    const int i0 = blockIdx.x * kRowsL;
    if (i0 >= n) return;
    const int i1 = min(n, i0 + kRowsL);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const SupportMut sm = A.sm;
    const int i = i0 + wave;
    constexpr int wj = kBWindow / Q;   // B window stored node-major: bw[t * wj + (j - w0)]
    const double* Mi = sm.M + (size_t)i * (i + 1) / 2;
    double acc[Q];
#pragma unroll
    for (int t = 0; t < Q; ++t) acc[t] = 0.0;
    for (int w0 = 0; w0 < i1; w0 += wj) {
        const int w1 = min(i1, w0 + wj);
        __syncthreads();
        for (int x = threadIdx.x; x < (w1 - w0) * q; x += kBigBlock) {
            const int t = x / (w1 - w0), jj = x - t * (w1 - w0), j = w0 + jj;
            bw[t * wj + jj] = wendland_r2(dist2(s_nd[0][t], s_nd[1][t], s_nd[2][t], sm.sx[j], sm.sy[j], sm.sz[j]));
        }
        __syncthreads();
        if (i < i1) {
            const int je = min(w1, i + 1);
            for (int j = w0 + lane; j < je; j += 64) {
                const double m = Mi[j];
#pragma unroll
                for (int t = 0; t < Q; ++t)
                    if (t < q) acc[t] = fma(m, bw[t * wj + (j - w0)], acc[t]);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < Q; ++t) {
        if (t < q) {
            const double lt = wave_sum(acc[t]);
            if (lane == 0 && i < i1) {
                A.lam[(size_t)t * A.cap + i] = lt;   // column-major: the column kernel reads it coalesced
                s_lam[wave][t] = lt;
            }
        }
    }
    for (int x = threadIdx.x; x < (i1 - i0) * q; x += kBigBlock) {
        const int jj = x / q, t = x - jj * q, j = i0 + jj;
        const double b = wendland_r2(dist2(s_nd[0][t], s_nd[1][t], s_nd[2][t], sm.sx[j], sm.sy[j], sm.sz[j]));
        s_bw[jj][t][0] = b * sm.wx[j];
        s_bw[jj][t][1] = b * sm.wy[j];
        s_bw[jj][t][2] = b * sm.wz[j];
    }
    __syncthreads();
    double* P = A.Pb + (size_t)blockIdx.x * kBlkPart;
    for (int x = threadIdx.x; x < 3 * q + q * q; x += kBigBlock) {
        double v = 0.0;
        if (x < 3 * q) {
            const int t = x / 3, c = x - 3 * t;
            for (int jj = 0; jj < i1 - i0; ++jj) v += s_bw[jj][t][c];
        } else {
            const int y = x - 3 * q, t = y / q, u = y - t * q;
            for (int r = 0; r < i1 - i0; ++r) v = fma(s_lam[r][t], s_lam[r][u], v);
        }
        P[blk_part_offset(x, q)] = v;
    }
}

// Every block sums the partials over the chunks in chunk order; wave 0 forms C - Lambda^T Lambda, its Cholesky
// factor L22 (pivots checked), L22^-1 and Z; then one wave per column j of M: u = (M^T Lambda)_j from the
// column-major copy, the new entries of rows n..n+q-1, and the W update.  Block 0 writes the diagonal block,
// the new supports and their weights, and commits |S| = n + q.
template <int Q>
__global__ __launch_bounds__(kBigBlock) void k_factor_u_blk(FactorBlkArgs A) {
    __shared__ double s_red[kBlkPart];
    __shared__ double s_part[kBigBlock];
    __shared__ double L[Q][Q], Li[Q][Q];
    __shared__ double s_e[Q][3], s_y[Q][3], s_z[Q][3];
    __shared__ double s_nd[6][Q];
    __shared__ double s_dinv[Q];
    __shared__ int32_t s_bad;
    const int q = A.brec->q, n = A.brec->n;
    if (q <= 0) return;
    if (blockIdx.x > 0 && (int)blockIdx.x * kRowsL >= n) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const SupportMut sm = A.sm;
    const int ncb = (n + kRowsL - 1) / kRowsL;
    {
        // the 3 q + q^2 needed sums over the chunks: thread (part, v) adds chunks part, part + parts, ... in order,
        // then one thread per value adds the parts in order (a fixed order whatever the scheduling)
        const int nval = 3 * q + q * q;
        const int parts = kBigBlock / nval;
        const int part = threadIdx.x / nval, v = threadIdx.x - part * nval;
        if (part < parts) {
            const int off = blk_part_offset(v, q);
            double a = 0.0;
#pragma unroll 4
            for (int c = part; c < ncb; c += parts) a += A.Pb[(size_t)c * kBlkPart + off];
            s_part[threadIdx.x] = a;
        }
        __syncthreads();
        if ((int)threadIdx.x < nval) {
            double r = 0.0;
            for (int pp = 0; pp < parts; ++pp) r += s_part[pp * nval + threadIdx.x];
            s_red[blk_part_offset(threadIdx.x, q)] = r;
        }
    }
    if ((int)threadIdx.x < q) {
        const int t = threadIdx.x;
        s_nd[0][t] = A.brec->x[t];
        s_nd[1][t] = A.brec->y[t];
        s_nd[2][t] = A.brec->z[t];
        s_nd[3][t] = A.brec->dx[t];
        s_nd[4][t] = A.brec->dy[t];
        s_nd[5][t] = A.brec->dz[t];
    }
    if (threadIdx.x == 0) s_bad = -1;
    __syncthreads();
    if (wave == 0) {
        for (int x = lane; x < q * q; x += 64) {
            const int t = x / q, u = x - t * q;
            const double c = wendland_r2(dist2(s_nd[0][t], s_nd[1][t], s_nd[2][t], s_nd[0][u], s_nd[1][u], s_nd[2][u]));
            L[t][u] = c - s_red[3 * kMaxPerIter + t * kMaxPerIter + u];
        }
        for (int x = lane; x < 3 * q; x += 64) {
            const int t = x / 3, c = x - 3 * t;
            s_e[t][c] = s_nd[3 + c][t] - s_red[3 * t + c];
        }
        wave_lds_sync();
        // right-looking Cholesky of the Schur complement
        int bad = -1;
        for (int k = 0; k < q; ++k) {
            const double piv = L[k][k];
            if (!(piv > kSingularTol)) {
                bad = k;
                break;
            }
            const double rk = sqrt(piv), inv = 1.0 / rk;
            wave_lds_sync();
            if (lane > k && lane < q) L[lane][k] *= inv;
            if (lane == k) L[k][k] = rk;
            wave_lds_sync();
            const int rem = q - k - 1;
            for (int x = lane; x < rem * rem; x += 64) {
                const int a = k + 1 + x / rem, b = k + 1 + x % rem;
                if (b <= a) L[a][b] = fma(-L[a][k], L[b][k], L[a][b]);
            }
            wave_lds_sync();
        }
        if (bad >= 0) {
            if (lane == 0) s_bad = bad;
        } else {
            if (lane < q) s_dinv[lane] = 1.0 / L[lane][lane];
            wave_lds_sync();
            // L22^-1 by forward substitution, lane c holding column c in registers
            double col[Q];
#pragma unroll
            for (int r = 0; r < Q; ++r) {
                double sacc = 0.0;
#pragma unroll
                for (int k = 0; k < r; ++k) sacc = fma(L[r][k], col[k], sacc);
                col[r] = r < q ? ((r == lane ? 1.0 : 0.0) - sacc) * s_dinv[r < q ? r : 0] : 0.0;
            }
            if (lane < q) {
#pragma unroll
                for (int r = 0; r < Q; ++r)
                    if (r < q) Li[r][lane] = col[r];
            }
            wave_lds_sync();
            // Z = L22^-T (L22^-1 E)
            if (lane < 3 * q) {
                const int t = lane / 3, c = lane - 3 * t;
                double y = 0.0;
#pragma unroll
                for (int k = 0; k < Q; ++k)
                    if (k <= t) y = fma(Li[t][k], s_e[k][c], y);
                s_y[t][c] = y;
            }
            wave_lds_sync();
            if (lane < 3 * q) {
                const int t = lane / 3, c = lane - 3 * t;
                double z = 0.0;
#pragma unroll
                for (int k = 0; k < Q; ++k)
                    if (k >= t && k < q) z = fma(Li[k][t], s_y[k][c], z);
                s_z[t][c] = z;
            }
        }
    }
    __syncthreads();
    if (s_bad >= 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            A.st->done = 3;
            A.st->singular_node = A.brec->orig[s_bad];
        }
        return;
    }
    const int j = blockIdx.x * kRowsL + wave;
    if (j < n) {
        double* col = A.Mc + (size_t)j * A.cap - (size_t)j * (j - 1) / 2;   // rows j.. of column j
        double u[Q];
#pragma unroll
        for (int t = 0; t < Q; ++t) u[t] = 0.0;
        for (int i = j + lane; i < n; i += 64) {
            const double m = col[i - j];
#pragma unroll
            for (int t = 0; t < Q; ++t)
                if (t < q) u[t] = fma(m, A.lam[(size_t)t * A.cap + i], u[t]);
        }
#pragma unroll
        for (int t = 0; t < Q; ++t)
            if (t < q) u[t] = wave_sum(u[t]);
        if (lane < q) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < Q; ++k)
                if (k <= lane) v = fma(Li[lane][k], u[k], v);
            const int r = n + lane;
            sm.M[(size_t)r * (r + 1) / 2 + j] = -v;
            col[r - j] = -v;
        }
        if (lane == 0) {
            double wx = sm.wx[j], wy = sm.wy[j], wz = sm.wz[j];
#pragma unroll
            for (int t = 0; t < Q; ++t) {
                if (t < q) {
                    wx = fma(-u[t], s_z[t][0], wx);
                    wy = fma(-u[t], s_z[t][1], wy);
                    wz = fma(-u[t], s_z[t][2], wz);
                }
            }
            sm.wx[j] = wx;
            sm.wy[j] = wy;
            sm.wz[j] = wz;
        }
    }
    if (blockIdx.x == 0) {
        for (int x = threadIdx.x; x < q * q; x += kBigBlock) {
            const int t = x / q, u = x - t * q;
            if (u <= t) {
                const int r = n + t, c = n + u;
                sm.M[(size_t)r * (r + 1) / 2 + c] = Li[t][u];
                A.Mc[(size_t)c * A.cap - (size_t)c * (c - 1) / 2 + (r - c)] = Li[t][u];
            }
        }
        if ((int)threadIdx.x < q) {
            const int t = threadIdx.x;
            sm.sx[n + t] = s_nd[0][t];
            sm.sy[n + t] = s_nd[1][t];
            sm.sz[n + t] = s_nd[2][t];
            sm.wx[n + t] = s_z[t][0];
            sm.wy[n + t] = s_z[t][1];
            sm.wz[n + t] = s_z[t][2];
            sm.orig[n + t] = A.brec->orig[t];
            A.inS[A.brec->pos[t]] = 1;
        }
        if (threadIdx.x == 0) {
            A.st->n = n + q;
            A.st->pairs_append += (uint64_t)q * (uint64_t)n + (uint64_t)q * (uint64_t)(q - 1) / 2;
        }
    }
}

// ---------------------------------------------------------------- batched iteration kernels (a10)
// One launch advances every surface of a batch: block b belongs to surface s
// with map.off[s] <= b < map.off[s+1]; the surface's arguments for this
// iteration are read from a table the host fills before each chunk.
__device__ __forceinline__ int batch_surface(const BlockMap& map, int b) {
    int s = 0;
    while (s + 1 < map.count && map.off[s + 1] <= b) ++s;
    return s;
}

__global__ __launch_bounds__(kBlock) void k_sweep_batch(const SweepArgs* __restrict__ tab, BlockMap map) {
    const int s = batch_surface(map, blockIdx.x);
    const SweepArgs A = tab[s];
    const int local = blockIdx.x - map.off[s];
    if (A.T <= 0 || local >= sweep_nblocks_dev(A.T, A.lpt, A.tpl)) return;
    sweep_body<kStageBatch>(A, local);
}

template <int RPW>
__global__ __launch_bounds__(kBigBlock) void k_factor_l_batch(const FactorLArgs* __restrict__ tab, BlockMap map) {
    const int s = batch_surface(map, blockIdx.x);
    const FactorLArgs A = tab[s];
    if (!A.active) return;
    factor_l_body<RPW>(A, blockIdx.x - map.off[s]);
}

template <int RPW>
__global__ __launch_bounds__(kBigBlock) void k_factor_u_batch(const FactorUArgs* __restrict__ tab, BlockMap map) {
    const int s = batch_surface(map, blockIdx.x);
    const FactorUArgs A = tab[s];
    if (!A.active) return;
    factor_u_body<RPW>(A, blockIdx.x - map.off[s]);
}

// Column-major copy of the first n rows of the packed row-major factor for
// capacity cap (after the support arrays grow).
__global__ __launch_bounds__(kBlock) void k_transpose_factor(const double* __restrict__ Mr, double* __restrict__ Mc,
                                                             int n, int64_t cap) {
    const int64_t x = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (x >= (int64_t)n * (n + 1) / 2) return;
    int i = (int)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
    while ((int64_t)(i + 1) * (i + 2) / 2 <= x) ++i;
    while ((int64_t)i * (i + 1) / 2 > x) --i;
    const int j = (int)(x - (int64_t)i * (i + 1) / 2);
    Mc[(size_t)j * cap - (size_t)j * (j - 1) / 2 + (i - j)] = Mr[x];
}

// ---------------------------------------------------------------- starting nodes
// mode 0: |d_j|^2; mode 1: |r_j - r_a|^2; mode 2: min(|r_j - r_a|^2, |r_j - r_b|^2),
// original order, ties to the lowest index; one record per block.
__global__ __launch_bounds__(kBlock) void k_init_argmax(int mode, int64_t nb, const double* __restrict__ xyz,
                                                        const double* __restrict__ disp,
                                                        const int32_t* __restrict__ init, ArgRec* __restrict__ rec) {
    Best b{-1.0, 0x7fffffff, -1};
    const int a = mode >= 1 ? init[0] : 0;
    const int c = mode >= 2 ? init[1] : 0;
    for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < nb; j += (int64_t)gridDim.x * kBlock) {
        double v;
        if (mode == 0) {
            v = sq3_exact(disp[3 * j], disp[3 * j + 1], disp[3 * j + 2]);
        } else {
            v = sq3_exact(xyz[3 * j] - xyz[3 * a], xyz[3 * j + 1] - xyz[3 * a + 1], xyz[3 * j + 2] - xyz[3 * a + 2]);
            if (mode == 2) {
                const double w = sq3_exact(xyz[3 * j] - xyz[3 * c], xyz[3 * j + 1] - xyz[3 * c + 1],
                                           xyz[3 * j + 2] - xyz[3 * c + 2]);
                v = v < w ? v : w;
            }
        }
        if (better(v, (int32_t)j, b.v, b.idx)) { b.v = v; b.idx = (int32_t)j; }
    }
    b = block_best(b);
    if (threadIdx.x == 0) rec[blockIdx.x] = ArgRec{b.v, b.idx, b.idx, 0, 0};
}

__global__ __launch_bounds__(kBlock) void k_init_final(int mode, int nrec, const ArgRec* __restrict__ rec,
                                                       int32_t* __restrict__ init) {
    Best b{-1.0, 0x7fffffff, -1};
    for (int i = threadIdx.x; i < nrec; i += kBlock)
        if (better(rec[i].e2, rec[i].orig, b.v, b.idx)) { b.v = rec[i].e2; b.idx = rec[i].orig; }
    b = block_best(b);
    if (threadIdx.x == 0) init[mode] = b.idx;
}

// ---------------------------------------------------------------- certificate (a6)
// e_j^2 over all boundary nodes; per block: max and sum.
// All-node error sweep (a6): kCertTargets targets per block, the supports
// split into four contiguous quarters over the block's four waves (four times
// the waves of one target per thread, for occupancy), the quarter sums added
// in a fixed order; one (max e^2, sum e^2) pair per block into red.
constexpr int kCertTargets = kBlock / 4;

int64_t certify_blocks(int64_t nb) { return (nb + kCertTargets - 1) / kCertTargets; }

__device__ __forceinline__ void all_node_block(int64_t nb, const double* __restrict__ px,
                                               const double* __restrict__ py, const double* __restrict__ pz,
                                               const double* __restrict__ pdx, const double* __restrict__ pdy,
                                               const double* __restrict__ pdz, const SupportView& sv, int n,
                                               double* __restrict__ red) {
    __shared__ double part[3][4][kCertTargets];
    // the quarter of the supports is wave-uniform; readfirstlane says so to the compiler, so the support loads
    // become scalar loads (SGPR operands) rather than one vector load per lane of the same address
    const int q = __builtin_amdgcn_readfirstlane(threadIdx.x / kCertTargets), tl = threadIdx.x % kCertTargets;
    const int64_t t = blockIdx.x * (int64_t)kCertTargets + tl;
    const bool live = t < nb;
    const int64_t tt = live ? t : nb - 1;
    const int s0 = (int)((int64_t)n * q / 4), s1 = (int)((int64_t)n * (q + 1) / 4);
    double ax = 0.0, ay = 0.0, az = 0.0;
    accumulate64(px[tt], py[tt], pz[tt], s0, s1, sv.sx, sv.sy, sv.sz, sv.wx, sv.wy, sv.wz, ax, ay, az);
    part[0][q][tl] = ax;
    part[1][q][tl] = ay;
    part[2][q][tl] = az;
    __syncthreads();
    const bool mine = q == 0 && live;
    double e2 = 0.0;
    if (mine) {
        const double fx = (part[0][0][tl] + part[0][1][tl]) + (part[0][2][tl] + part[0][3][tl]);
        const double fy = (part[1][0][tl] + part[1][1][tl]) + (part[1][2][tl] + part[1][3][tl]);
        const double fz = (part[2][0][tl] + part[2][1][tl]) + (part[2][2][tl] + part[2][3][tl]);
        const double ex = fx - pdx[t], ey = fy - pdy[t], ez = fz - pdz[t];
        e2 = fma(ez, ez, fma(ey, ey, ex * ex));
    }
    Best b{mine ? e2 : -1.0, (int32_t)t, 0};
    b = block_best(b);
    const double sum = block_sum<kBlock>(e2);
    if (threadIdx.x == 0) {
        red[2 * blockIdx.x] = b.v;
        red[2 * blockIdx.x + 1] = sum;
    }
}

__global__ __launch_bounds__(kBlock) void k_certify(int64_t nb, const double* __restrict__ px,
                                                    const double* __restrict__ py, const double* __restrict__ pz,
                                                    const double* __restrict__ pdx, const double* __restrict__ pdy,
                                                    const double* __restrict__ pdz, SupportView sv, int n,
                                                    double* __restrict__ red) {
    all_node_block(nb, px, py, pz, pdx, pdy, pdz, sv, n, red);
}

// Convergence probe: the FP64 error of every boundary node with the current W (the certificate's layout: one
// target per lane, the supports split over the block's four waves), one value per node.
__global__ __launch_bounds__(kBlock) void k_probe_err(int64_t nb, const double* __restrict__ px,
                                                      const double* __restrict__ py, const double* __restrict__ pz,
                                                      const double* __restrict__ pdx, const double* __restrict__ pdy,
                                                      const double* __restrict__ pdz, SupportView sv, int n,
                                                      double* __restrict__ perr) {
    __shared__ double part[3][4][kCertTargets];
    // the quarter of the supports is wave-uniform; readfirstlane says so to the compiler, so the support loads
    // become scalar loads (SGPR operands) rather than one vector load per lane of the same address
    const int q = __builtin_amdgcn_readfirstlane(threadIdx.x / kCertTargets), tl = threadIdx.x % kCertTargets;
    const int64_t t = blockIdx.x * (int64_t)kCertTargets + tl;
    const bool live = t < nb;
    const int64_t tt = live ? t : nb - 1;
    const int s0 = (int)((int64_t)n * q / 4), s1 = (int)((int64_t)n * (q + 1) / 4);
    double ax = 0.0, ay = 0.0, az = 0.0;
    accumulate64(px[tt], py[tt], pz[tt], s0, s1, sv.sx, sv.sy, sv.sz, sv.wx, sv.wy, sv.wz, ax, ay, az);
    part[0][q][tl] = ax;
    part[1][q][tl] = ay;
    part[2][q][tl] = az;
    __syncthreads();
    if (q == 0 && live) {
        const double fx = (part[0][0][tl] + part[0][1][tl]) + (part[0][2][tl] + part[0][3][tl]);
        const double fy = (part[1][0][tl] + part[1][1][tl]) + (part[1][2][tl] + part[1][3][tl]);
        const double fz = (part[2][0][tl] + part[2][1][tl]) + (part[2][2][tl] + part[2][3][tl]);
        const double ex = fx - pdx[t], ey = fy - pdy[t], ez = fz - pdz[t];
        perr[t] = fma(ez, ez, fma(ey, ey, ex * ex));
    }
}

// Per group (one block each, groups contiguous in the permuted order): the largest squared error over the nodes
// not in S, ties to the lowest original index, and the count of those nodes.
__global__ __launch_bounds__(kBlock) void k_probe_groups(const int32_t* __restrict__ goff,
                                                         const int32_t* __restrict__ perm,
                                                         const uint8_t* __restrict__ inS,
                                                         const double* __restrict__ perr, GroupMax* __restrict__ out) {
    __shared__ int32_t s_cnt[kBlock / 64];
    __shared__ double s_max[kBlock / 64];
    const int g = blockIdx.x;
    const int a = goff[g], b = goff[g + 1];
    Best best{-1.0, 0x7fffffff, 0};
    int32_t cnt = 0;
    double amax = 0.0, asum = 0.0;
    for (int p = a + (int)threadIdx.x; p < b; p += kBlock) {
        const double e = perr[p];
        amax = fmax(amax, e);
        asum += e;
        if (inS[p]) continue;
        ++cnt;
        const int32_t o = perm[p];
        if (better(e, o, best.v, best.idx)) {
            best.v = e;
            best.idx = o;
        }
    }
    best = block_best(best);
    const double gsum = block_sum<kBlock>(asum);
    cnt = wave_isum(cnt);
    amax = wave_max(amax);
    if ((threadIdx.x & 63) == 0) {
        s_cnt[threadIdx.x >> 6] = cnt;
        s_max[threadIdx.x >> 6] = amax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t total = 0;
        double gmx = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) {
            total += s_cnt[w];
            gmx = fmax(gmx, s_max[w]);
        }
        out[g] = GroupMax{best.v, best.idx, total, gmx, gsum};
    }
}

void launch_probe(hipStream_t s, const Boundary& bd, const Support& sp, int n, double* perr, GroupMax* out) {
    const unsigned g = (unsigned)certify_blocks(bd.nb);
    GCB_LAUNCH(k_probe_err, dim3(g), dim3(kBlock), s, bd.nb, bd.px, bd.py, bd.pz, bd.pdx, bd.pdy, bd.pdz, view(sp), n,
               perr);
    GCB_LAUNCH(k_probe_groups, dim3((unsigned)bd.m), dim3(kBlock), s, bd.goff, bd.perm, bd.inS, perr, out);
}

__global__ __launch_bounds__(kBlock) void k_certify_final(int nblk, const double* __restrict__ red,
                                                          double* __restrict__ out) {
    // fixed order: each thread sums a contiguous stretch, then the block in thread order
    double mx = 0.0, s = 0.0;
    const int per = (nblk + kBlock - 1) / kBlock;
    const int i0 = threadIdx.x * per, i1 = min(nblk, i0 + per);
    for (int i = i0; i < i1; ++i) {
        mx = fmax(mx, red[2 * i]);
        s += red[2 * i + 1];
    }
    __shared__ double smx[kBlock], ss[kBlock];
    smx[threadIdx.x] = mx;
    ss[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double M = 0.0, S = 0.0;
        for (int i = 0; i < kBlock; ++i) {
            M = fmax(M, smx[i]);
            S += ss[i];
        }
        out[0] = M;
        out[1] = S;
    }
}

// Monitor sample (never alters the selection): the all-node error with the
// current W after the loop iteration that brings the log to `need` entries;
// nothing is written if the selection stopped before that iteration ran.
__global__ __launch_bounds__(kBlock) void k_monitor(int64_t nb, const double* __restrict__ px,
                                                    const double* __restrict__ py, const double* __restrict__ pz,
                                                    const double* __restrict__ pdx, const double* __restrict__ pdy,
                                                    const double* __restrict__ pdz, SupportView sv,
                                                    const GState* __restrict__ st, int64_t need,
                                                    double* __restrict__ red) {
    const GState s = *st;
    if (s.log_len < need) return;
    all_node_block(nb, px, py, pz, pdx, pdy, pdz, sv, s.n, red);
}

__global__ __launch_bounds__(kBlock) void k_monitor_final(int nblk, const double* __restrict__ red,
                                                          const GState* __restrict__ st, int64_t need,
                                                          double* __restrict__ out) {
    if (st->log_len < need) return;
    double mx = 0.0, s = 0.0;
    const int per = (nblk + kBlock - 1) / kBlock;
    const int i0 = threadIdx.x * per, i1 = min(nblk, i0 + per);
    for (int i = i0; i < i1; ++i) {
        mx = fmax(mx, red[2 * i]);
        s += red[2 * i + 1];
    }
    __shared__ double smx[kBlock], ss[kBlock];
    smx[threadIdx.x] = mx;
    ss[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double M = 0.0, S = 0.0;
        for (int i = 0; i < kBlock; ++i) {
            M = fmax(M, smx[i]);
            S += ss[i];
        }
        out[0] = M;
        out[1] = S;
    }
}

// ---------------------------------------------------------------- volume (a7)
// Half-scaled supports centred at the first one, and their squared norms.
__global__ __launch_bounds__(kBlock) void k_volume_table(int n, SupportView sv, VolTable vt) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const double x = fma(sv.sx[j], 0.5, -0.5 * sv.sx[0]);
    const double y = fma(sv.sy[j], 0.5, -0.5 * sv.sy[0]);
    const double z = fma(sv.sz[j], 0.5, -0.5 * sv.sz[0]);
    vt.qx[j] = x;
    vt.qy[j] = y;
    vt.qz[j] = z;
    vt.qq[j] = fma(z, z, fma(y, y, x * x));
}

template <typename TIn, typename TOut>
__global__ __launch_bounds__(kBlock) void k_volume64(int64_t nv, const TIn* __restrict__ xyz, double inv_r,
                                                     SupportView sv, VolTable vt, int n, TOut* __restrict__ out) {
    const int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    const bool live = t < nv;
    const int64_t tt = live ? t : nv - 1;
    const VolTarget u = vol_target((double)xyz[3 * tt], (double)xyz[3 * tt + 1], (double)xyz[3 * tt + 2], inv_r, sv);
    double ax = 0.0, ay = 0.0, az = 0.0;
    accumulate_vol(u.mx, u.my, u.mz, u.uu, n, vt, sv.wx, sv.wy, sv.wz, ax, ay, az);
    if (live) {
        out[3 * t] = (TOut)ax;
        out[3 * t + 1] = (TOut)ay;
        out[3 * t + 2] = (TOut)az;
    }
}

// FP32 evaluation of Eq. (6): coordinates (scaled), weights and phi in FP32,
// each chunk of kChunk32 supports summed in FP32 and the chunk sums carried
// in FP64 (blocked compensation), so the summation adds little to the FP32
// error of phi itself.
constexpr int kChunk32 = 32;

// phi in FP32 from r2 >= 0: the hardware square root (about 1 ulp) needs no
// guard at r2 = 0, unlike r2 * rsq(r2).
__device__ __forceinline__ float wendland_r2_f32(float r2) {
    const float eta = __builtin_amdgcn_sqrtf(r2);
    const float t = fminf(fmaxf(1.0f - eta, 0.0f), 1.0f);
    const float t2 = t * t;
    return (t2 * t2) * fmaf(-4.0f, t, 5.0f);
}

template <typename TIn, typename TOut>
__global__ __launch_bounds__(kBlock) void k_volume32(int64_t nv, const TIn* __restrict__ xyz, double inv_r, int n,
                                                     const float* __restrict__ fsx, const float* __restrict__ fsy,
                                                     const float* __restrict__ fsz, const float* __restrict__ fwx,
                                                     const float* __restrict__ fwy, const float* __restrict__ fwz,
                                                     TOut* __restrict__ out) {
    const int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    const bool live = t < nv;
    const int64_t tt = live ? t : nv - 1;
    const float tx = (float)((double)xyz[3 * tt] * inv_r);
    const float ty = (float)((double)xyz[3 * tt + 1] * inv_r);
    const float tz = (float)((double)xyz[3 * tt + 2] * inv_r);
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int j0 = 0; j0 < n; j0 += kChunk32) {
        const int j1 = min(n, j0 + kChunk32);
        float bx = 0.0f, by = 0.0f, bz = 0.0f;
        int j = j0;
        for (; j + 4 <= j1; j += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float dx = tx - fsx[j + u], dy = ty - fsy[j + u], dz = tz - fsz[j + u];
                const float phi = wendland_r2_f32(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
                bx = fmaf(fwx[j + u], phi, bx);
                by = fmaf(fwy[j + u], phi, by);
                bz = fmaf(fwz[j + u], phi, bz);
            }
        }
        for (; j < j1; ++j) {
            const float dx = tx - fsx[j], dy = ty - fsy[j], dz = tz - fsz[j];
            const float phi = wendland_r2_f32(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
            bx = fmaf(fwx[j], phi, bx);
            by = fmaf(fwy[j], phi, by);
            bz = fmaf(fwz[j], phi, bz);
        }
        ax += (double)bx;
        ay += (double)by;
        az += (double)bz;
    }
    if (live) {
        out[3 * t] = (TOut)ax;
        out[3 * t + 1] = (TOut)ay;
        out[3 * t + 2] = (TOut)az;
    }
}

__global__ __launch_bounds__(kBlock) void k_support_f32(int n, SupportView sv, float* __restrict__ fsx,
                                                        float* __restrict__ fsy, float* __restrict__ fsz,
                                                        float* __restrict__ fwx, float* __restrict__ fwy,
                                                        float* __restrict__ fwz) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    fsx[j] = (float)sv.sx[j];
    fsy[j] = (float)sv.sy[j];
    fsz[j] = (float)sv.sz[j];
    fwx[j] = (float)sv.wx[j];
    fwy[j] = (float)sv.wy[j];
    fwz[j] = (float)sv.wz[j];
}

// Eq. (6) for several surfaces in one launch: block b belongs to surface s
// with map.off[s] <= b < map.off[s+1].
__global__ __launch_bounds__(kBlock) void k_volume_table_batch(const VolDesc* __restrict__ tab, BlockMap map) {
    const int s = batch_surface(map, blockIdx.x);
    const VolDesc& d = tab[s];
    const int j = (blockIdx.x - map.off[s]) * kBlock + threadIdx.x;
    if (j >= d.n) return;
    const double x = fma(d.sv.sx[j], 0.5, -0.5 * d.sv.sx[0]);
    const double y = fma(d.sv.sy[j], 0.5, -0.5 * d.sv.sy[0]);
    const double z = fma(d.sv.sz[j], 0.5, -0.5 * d.sv.sz[0]);
    d.vt.qx[j] = x;
    d.vt.qy[j] = y;
    d.vt.qz[j] = z;
    d.vt.qq[j] = fma(z, z, fma(y, y, x * x));
}

template <typename TIn, typename TOut>
__global__ __launch_bounds__(kBlock) void k_volume_batch(const VolDesc* __restrict__ tab, BlockMap map) {
    const int s = batch_surface(map, blockIdx.x);
    const VolDesc d = tab[s];
    const int64_t t = (int64_t)(blockIdx.x - map.off[s]) * kBlock + threadIdx.x;
    const bool live = t < d.nv;
    const int64_t tt = live ? t : d.nv - 1;
    const TIn* xyz = static_cast<const TIn*>(d.xyz);
    const VolTarget u =
        vol_target((double)xyz[3 * tt], (double)xyz[3 * tt + 1], (double)xyz[3 * tt + 2], d.inv_r, d.sv);
    double ax = 0.0, ay = 0.0, az = 0.0;
    accumulate_vol(u.mx, u.my, u.mz, u.uu, d.n, d.vt, d.sv.wx, d.sv.wy, d.sv.wz, ax, ay, az);
    if (live) {
        TOut* out = static_cast<TOut*>(d.out);
        out[3 * t] = (TOut)ax;
        out[3 * t + 1] = (TOut)ay;
        out[3 * t + 2] = (TOut)az;
    }
}

void launch_volume_batch(hipStream_t s, const VolDesc* tab, const BlockMap& map, const BlockMap& table_map,
                         int in_f64, int out_f64) {
    if (table_map.off[table_map.count] > 0)
        GCB_LAUNCH(k_volume_table_batch, dim3((unsigned)table_map.off[table_map.count]), dim3(kBlock), s, tab,
                   table_map);
    const dim3 g((unsigned)map.off[map.count]);
    if (in_f64 && out_f64) GCB_LAUNCH((k_volume_batch<double, double>), g, dim3(kBlock), s, tab, map);
    else if (in_f64) GCB_LAUNCH((k_volume_batch<double, float>), g, dim3(kBlock), s, tab, map);
    else if (out_f64) GCB_LAUNCH((k_volume_batch<float, double>), g, dim3(kBlock), s, tab, map);
    else GCB_LAUNCH((k_volume_batch<float, float>), g, dim3(kBlock), s, tab, map);
}

// ---------------------------------------------------------------- staging (a1)
// Gather the caller's AoS boundary into the permuted, group-contiguous SoA
// layout, coordinates scaled by 1/R.
__global__ __launch_bounds__(kBlock) void k_stage(int64_t nb, const double* __restrict__ xyz,
                                                  const double* __restrict__ disp, const int32_t* __restrict__ perm,
                                                  double inv_r, double* __restrict__ px, double* __restrict__ py,
                                                  double* __restrict__ pz, double* __restrict__ pdx,
                                                  double* __restrict__ pdy, double* __restrict__ pdz,
                                                  int32_t* __restrict__ pos_of, uint8_t* __restrict__ inS) {
    const int64_t p = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (p >= nb) return;
    const int o = perm[p];
    px[p] = xyz[3 * o] * inv_r;
    py[p] = xyz[3 * o + 1] * inv_r;
    pz[p] = xyz[3 * o + 2] * inv_r;
    pdx[p] = disp[3 * o];
    pdy[p] = disp[3 * o + 1];
    pdz[p] = disp[3 * o + 2];
    pos_of[o] = (int32_t)p;
    inS[p] = 0;
}

// Non-finite check: flag[0] = 1 if any of the 3*nb values of a or b is not finite.
__global__ __launch_bounds__(kBlock) void k_check_finite(int64_t count, const double* __restrict__ a,
                                                         const double* __restrict__ b, int32_t* __restrict__ flag) {
    int bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < count; i += (int64_t)gridDim.x * kBlock) {
        if (!isfinite(a[i])) bad = 1;
        if (b && !isfinite(b[i])) bad = 1;
    }
    if (bad) flag[0] = 1;
}

// Nodes of a kept support set are in S again after the boundary is re-staged.
__global__ __launch_bounds__(kBlock) void k_mark_support(int n, const int32_t* __restrict__ orig,
                                                         const int32_t* __restrict__ pos_of, uint8_t* __restrict__ inS) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j < n) inS[pos_of[orig[j]]] = 1;
}

// ---------------------------------------------------------------- launchers

void launch_mark_support(hipStream_t s, const Boundary& bd, const Support& sp, int n) {
    if (n <= 0) return;
    GCB_LAUNCH(k_mark_support, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), s, n, sp.orig, bd.pos_of,
               bd.inS);
}

void launch_stage(hipStream_t s, int64_t nb, const double* xyz, const double* disp, const int32_t* perm,
                  double inv_r, Boundary& bd) {
    const unsigned g = (unsigned)((nb + kBlock - 1) / kBlock);
    GCB_LAUNCH(k_stage, dim3(g), dim3(kBlock), s, nb, xyz, disp, perm, inv_r, bd.px, bd.py, bd.pz, bd.pdx, bd.pdy,
               bd.pdz, bd.pos_of, bd.inS);
}

void launch_check_finite(hipStream_t s, int64_t count, const double* a, const double* b, int32_t* flag) {
    GCB_LAUNCH(k_check_finite, dim3(1024), dim3(kBlock), s, count, a, b, flag);
}

void launch_init_nodes(hipStream_t s, const Boundary& bd, int32_t* init, ArgRec* rec) {
    const int nblk = 512;
    for (int mode = 0; mode < 3; ++mode) {
        GCB_LAUNCH(k_init_argmax, dim3(nblk), dim3(kBlock), s, mode, bd.nb, bd.xyz0, bd.disp0, init, rec);
        GCB_LAUNCH(k_init_final, dim3(1), dim3(kBlock), s, mode, nblk, rec, init);
    }
}

SweepArgs make_sweep_args(const IterCtx& ic, int g) {
    const Boundary& bd = *ic.bd;
    SweepArgs A;
    A.st = ic.st;
    A.t0 = bd.goff_h[g];
    A.T = bd.goff_h[g + 1] - A.t0;
    sweep_layout(A.T, A.lpt, A.tpl);
    A.px = bd.px; A.py = bd.py; A.pz = bd.pz;
    A.pdx = bd.pdx; A.pdy = bd.pdy; A.pdz = bd.pdz;
    A.inS = bd.inS;
    A.perm = bd.perm;
    A.sv = view(*ic.sp);
    A.nub = ic.sp->cap;
    A.rec = ic.srec;
    A.ptop = 0;
    return A;
}

FactorLArgs make_factor_l_args(const IterCtx& ic, int g, int nrec, int init_t) {
    const Boundary& bd = *ic.bd;
    Support& sp = *ic.sp;
    FactorLArgs A;
    A.st = ic.st; A.irec = ic.irec; A.srec = ic.srec; A.nrec = nrec; A.m = bd.m; A.g = g; A.init_t = init_t;
    A.init = ic.init; A.pos_of = bd.pos_of;
    A.px = bd.px; A.py = bd.py; A.pz = bd.pz; A.pdx = bd.pdx; A.pdy = bd.pdy; A.pdz = bd.pdz;
    A.sv = view(sp); A.Mr = sp.M; A.l = sp.l; A.Pb = ic.Pb;
    A.tol_abs = ic.tol_abs; A.nc_max = ic.nc_max; A.cap = sp.cap;
    A.log_group = ic.log_group; A.log_node = ic.log_node; A.log_err = ic.log_err; A.log_app = ic.log_app;
    A.log_cap = ic.log_cap;
    A.active = 1;
    return A;
}

FactorUArgs make_factor_u_args(const IterCtx& ic) {
    const Boundary& bd = *ic.bd;
    Support& sp = *ic.sp;
    FactorUArgs A;
    A.st = ic.st; A.irec = ic.irec; A.inS = bd.inS; A.sm = mut(sp); A.Mc = sp.Mc; A.cap = sp.cap; A.l = sp.l;
    A.Pb = ic.Pb;
    A.active = 1;
    return A;
}

int sweep_records(const SweepArgs& A) { return A.T > 0 ? sweep_nblocks_dev(A.T, A.lpt, A.tpl) : 0; }

int factor_blocks(int64_t n_ub, int rpw) {
    const int64_t rpb = (int64_t)kRowsL * rpw;
    return (int)std::max<int64_t>(1, (n_ub + rpb - 1) / rpb);
}

// Group sweep layout of a batched launch: the batch supplies the parallelism,
// so blocks hold more targets (fewer blocks, each staging the supports once).
void sweep_layout_batch(int T, int& lpt, int& tpl) {
    // measured on 32 uneven surfaces: four targets per lane beats one or two at every support count
    lpt = 64;
    tpl = T <= 64 ? 1 : 4;
}

static void launch_factor(hipStream_t s, const IterCtx& ic, int grid, int init_t, int g, int nrec) {
    GCB_LAUNCH(k_factor_l, dim3(grid), dim3(kBigBlock), s, make_factor_l_args(ic, g, nrec, init_t));
    GCB_LAUNCH(k_factor_u, dim3(grid), dim3(kBigBlock), s, make_factor_u_args(ic));
}

void launch_init_append(hipStream_t s, const IterCtx& ic, int t) { launch_factor(s, ic, 1, t, 0, 0); }

int sweep_blocks(int gmax) {
    int best = 1;
    for (int T : {std::min(gmax, 512), std::min(gmax, 4096), std::min(gmax, 8192), gmax})
        if (T > 0) best = std::max(best, sweep_nblocks(T));
    return best;
}

int launch_iteration(hipStream_t s, const IterCtx& ic, int g, int n_ub, const hipEvent_t* marks) {
    const SweepArgs A = make_sweep_args(ic, g);
    // above 8,192 targets the lanes form has at least 129 blocks of 64 targets; below, too few to fill the chip
    const bool lanes = A.T > 8192;
    const int nrec = A.T > 0 ? (lanes ? sweep_lanes_blocks(A.T) : sweep_nblocks(A.T)) : 0;
    if (marks) (void)hipEventRecord(marks[0], s);
    if (A.T > 0) {
        if (lanes) GCB_LAUNCH(k_sweep_lanes, dim3(nrec), dim3(kBlock), s, A);
        else if (A.tpl > 1) GCB_LAUNCH(k_sweep_wide, dim3(nrec), dim3(kBlock), s, A);
        else GCB_LAUNCH(k_sweep, dim3(nrec), dim3(kBlock), s, A);
    }
    const int grid = factor_blocks(n_ub);
    if (marks) (void)hipEventRecord(marks[1], s);
    GCB_LAUNCH(k_factor_l, dim3(grid), dim3(kBigBlock), s, make_factor_l_args(ic, g, nrec, -1));
    if (marks) (void)hipEventRecord(marks[2], s);
    GCB_LAUNCH(k_factor_u, dim3(grid), dim3(kBigBlock), s, make_factor_u_args(ic));
    if (marks) (void)hipEventRecord(marks[3], s);
    return A.T > 0;
}

template <int Q>
static void launch_block_kernels(hipStream_t s, const FactorBlkArgs& F, dim3 grid) {
    GCB_LAUNCH(k_factor_l_blk<Q>, grid, dim3(kBigBlock), s, F);
    GCB_LAUNCH(k_factor_u_blk<Q>, grid, dim3(kBigBlock), s, F);
}

void launch_iteration_block(hipStream_t s, const IterCtx& ic, int g, int n_ub, int p) {
    SweepArgs A = make_sweep_args(ic, g);
    const bool lanes = A.T > 8192;
    const int nblk = A.T > 0 ? (lanes ? sweep_lanes_blocks(A.T) : sweep_nblocks(A.T)) : 0;
    const int cand = lanes ? kLaneTargets : (kBlock / A.lpt) * A.tpl;   // candidates one block holds
    A.ptop = std::min(p, cand);
    if (A.T > 0) {
        if (lanes) GCB_LAUNCH(k_sweep_lanes_top, dim3(nblk), dim3(kBlock), s, A);
        else if (A.tpl > 1) GCB_LAUNCH(k_sweep_wide_top, dim3(nblk), dim3(kBlock), s, A);
        else GCB_LAUNCH(k_sweep_top, dim3(nblk), dim3(kBlock), s, A);
    }
    const Support& sp = *ic.sp;
    FactorBlkArgs F;
    F.st = ic.st; F.brec = ic.brec; F.sm = mut(*ic.sp); F.Mc = sp.Mc; F.cap = sp.cap; F.lam = ic.lam; F.Pb = ic.Pb;
    F.inS = ic.bd->inS;
    F.srec = ic.srec; F.nrec = nblk * A.ptop; F.ptop = p; F.m = ic.bd->m; F.g = g;
    F.tol_abs = ic.tol_abs; F.nc_max = ic.nc_max;
    F.log_group = ic.log_group; F.log_node = ic.log_node; F.log_err = ic.log_err; F.log_app = ic.log_app;
    F.log_cap = ic.log_cap;
    const dim3 grid((unsigned)factor_blocks(n_ub));
    // kernels compiled for up to Q = 2, 4, 8, 16 nodes per iteration
    if (p <= 2) launch_block_kernels<2>(s, F, grid);
    else if (p <= 4) launch_block_kernels<4>(s, F, grid);
    else if (p <= 8) launch_block_kernels<8>(s, F, grid);
    else launch_block_kernels<16>(s, F, grid);
}

void launch_iteration_batch(hipStream_t s, const SweepArgs* sweep_tab, const FactorLArgs* fl_tab,
                            const FactorUArgs* fu_tab, const BlockMap& sweep_map, const BlockMap& factor_map, int rpw) {
    if (sweep_map.off[sweep_map.count] > 0)   // every group of the step may be empty
        GCB_LAUNCH(k_sweep_batch, dim3(sweep_map.off[sweep_map.count]), dim3(kBlock), s, sweep_tab, sweep_map);
    const dim3 fg((unsigned)factor_map.off[factor_map.count]);
    if (rpw == kMaxRowsPerWave) {
        GCB_LAUNCH(k_factor_l_batch<kMaxRowsPerWave>, fg, dim3(kBigBlock), s, fl_tab, factor_map);
        GCB_LAUNCH(k_factor_u_batch<kMaxRowsPerWave>, fg, dim3(kBigBlock), s, fu_tab, factor_map);
    } else {
        GCB_LAUNCH(k_factor_l_batch<1>, fg, dim3(kBigBlock), s, fl_tab, factor_map);
        GCB_LAUNCH(k_factor_u_batch<1>, fg, dim3(kBigBlock), s, fu_tab, factor_map);
    }
}

void launch_transpose_factor(hipStream_t s, const double* Mr, double* Mc, int n, int64_t cap) {
    const int64_t cnt = (int64_t)n * (n + 1) / 2;
    if (cnt == 0) return;
    GCB_LAUNCH(k_transpose_factor, dim3((unsigned)((cnt + kBlock - 1) / kBlock)), dim3(kBlock), s, Mr, Mc, n, cap);
}

void launch_monitor(hipStream_t s, const Boundary& bd, const Support& sp, const GState* st, int64_t need,
                    double* red, double* out) {
    const unsigned g = (unsigned)certify_blocks(bd.nb);
    GCB_LAUNCH(k_monitor, dim3(g), dim3(kBlock), s, bd.nb, bd.px, bd.py, bd.pz, bd.pdx, bd.pdy, bd.pdz, view(sp), st,
               need, red);
    GCB_LAUNCH(k_monitor_final, dim3(1), dim3(kBlock), s, (int)g, red, st, need, out);
}

void launch_certify(hipStream_t s, const Boundary& bd, const Support& sp, int n, double* red, double* out) {
    const unsigned g = (unsigned)certify_blocks(bd.nb);
    GCB_LAUNCH(k_certify, dim3(g), dim3(kBlock), s, bd.nb, bd.px, bd.py, bd.pz, bd.pdx, bd.pdy, bd.pdz, view(sp), n, red);
    GCB_LAUNCH(k_certify_final, dim3(1), dim3(kBlock), s, (int)g, red, out);
}

template <typename TIn, typename TOut>
static void vol(hipStream_t s, int64_t nv, const void* xyz, double inv_r, SupportView sv, VolTable vt, int n,
                void* out) {
    const unsigned g = (unsigned)((nv + kBlock - 1) / kBlock);
    GCB_LAUNCH((k_volume64<TIn, TOut>), dim3(g), dim3(kBlock), s, nv, (const TIn*)xyz, inv_r, sv, vt, n, (TOut*)out);
}

template <typename TIn, typename TOut>
static void vol32(hipStream_t s, int64_t nv, const void* xyz, double inv_r, float* const f[6], int n, void* out) {
    const unsigned g = (unsigned)((nv + kBlock - 1) / kBlock);
    GCB_LAUNCH((k_volume32<TIn, TOut>), dim3(g), dim3(kBlock), s, nv, (const TIn*)xyz, inv_r, n, f[0], f[1], f[2],
               f[3], f[4], f[5], (TOut*)out);
}

// FP32 evaluation with the FP32 copies of the supports in f[0..5] (x, y, z, wx, wy, wz; n floats each).
static void volume32_into(hipStream_t s, int64_t nv, const void* xyz, int in_f64, double inv_r, SupportView sv,
                          float* const f[6], int n, void* out, int out_f64) {
    if (n > 0)
        GCB_LAUNCH(k_support_f32, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), s, n, sv, f[0], f[1],
                   f[2], f[3], f[4], f[5]);
    if (in_f64 && out_f64) vol32<double, double>(s, nv, xyz, inv_r, f, n, out);
    else if (in_f64) vol32<double, float>(s, nv, xyz, inv_r, f, n, out);
    else if (out_f64) vol32<float, double>(s, nv, xyz, inv_r, f, n, out);
    else vol32<float, float>(s, nv, xyz, inv_r, f, n, out);
}

// FP64 evaluation with the support table in vt (four arrays of at least n doubles).
static void volume64_into(hipStream_t s, int64_t nv, const void* xyz, int in_f64, double inv_r, SupportView sv,
                          VolTable vt, int n, void* out, int out_f64) {
    if (n > 0) GCB_LAUNCH(k_volume_table, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), s, n, sv, vt);
    if (in_f64 && out_f64) vol<double, double>(s, nv, xyz, inv_r, sv, vt, n, out);
    else if (in_f64) vol<double, float>(s, nv, xyz, inv_r, sv, vt, n, out);
    else if (out_f64) vol<float, double>(s, nv, xyz, inv_r, sv, vt, n, out);
    else vol<float, float>(s, nv, xyz, inv_r, sv, vt, n, out);
}

void launch_volume32(hipStream_t s, int64_t nv, const void* xyz, int in_f64, double inv_r, const Support& sp, int n,
                     void* out, int out_f64) {
    float* const f[6] = {sp.fsx, sp.fsy, sp.fsz, sp.fwx, sp.fwy, sp.fwz};
    volume32_into(s, nv, xyz, in_f64, inv_r, view(sp), f, n, out, out_f64);
}

void launch_volume(hipStream_t s, int64_t nv, const void* xyz, int in_f64, double inv_r, const Support& sp, int n,
                   void* out, int out_f64) {
    volume64_into(s, nv, xyz, in_f64, inv_r, view(sp), vtable(sp), n, out, out_f64);
}

// ---------------------------------------------------------------- compact-support culling of Eq. (6)
// phi is exactly zero beyond R (Eq. 2), so a (target, support) pair farther apart adds nothing.  Points are
// evaluated in Morton order of their cells (a sorted index list), supports in Morton order in tiles of
// kCullTile with bounding boxes; a wave skips every tile whose box lies farther than R from the box of its 64
// points.  Distances are in the volume table's units (1/(2R)), so R is 0.5; the test keeps a relative margin of
// 1e-9, far above the rounding of the evaluated distance, so every skipped pair would have evaluated to zero.
constexpr int kCullTile = 32;
constexpr double kCullGap2 = 0.25 * (1.0 + 1e-9);

__device__ __forceinline__ uint32_t spread10(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// Morton key of a point in the culling frame: 10 bits per axis over [lo, lo + 1023 / sc]; points outside the
// frame (farther than R from every support along some axis) are clamped to it and get bit 30, so they sort after
// the others, still in spatial order.
__device__ __forceinline__ uint32_t cull_key(double ux, double uy, double uz, const CullFrame& f) {
    const double qx = (ux - f.lox) * f.sc, qy = (uy - f.loy) * f.sc, qz = (uz - f.loz) * f.sc;
    const bool in = qx >= 0.0 && qy >= 0.0 && qz >= 0.0 && qx <= 1023.0 && qy <= 1023.0 && qz <= 1023.0;
    const uint32_t ix = (uint32_t)fmin(fmax(qx, 0.0), 1023.0), iy = (uint32_t)fmin(fmax(qy, 0.0), 1023.0),
                   iz = (uint32_t)fmin(fmax(qz, 0.0), 1023.0);
    return (in ? 0u : (1u << 30)) | spread10(ix) | (spread10(iy) << 1) | (spread10(iz) << 2);
}

template <typename TIn>
__global__ __launch_bounds__(kBlock) void k_cull_keys(int64_t nv, const TIn* __restrict__ xyz, double h, double c0x,
                                                      double c0y, double c0z, CullFrame f, uint32_t* __restrict__ keys,
                                                      int32_t* __restrict__ idx) {
    const int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    if (t >= nv) return;
    const double ux = fma((double)xyz[3 * t], h, -c0x), uy = fma((double)xyz[3 * t + 1], h, -c0y),
                 uz = fma((double)xyz[3 * t + 2], h, -c0z);
    keys[t] = cull_key(ux, uy, uz, f);
    idx[t] = (int32_t)t;
}

template <typename TIn, typename TOut>
__global__ __launch_bounds__(kBlock) void k_volume64_cull(int64_t nv, const TIn* __restrict__ xyz,
                                                          const int32_t* __restrict__ order, double h, double c0x,
                                                          double c0y, double c0z, CullSupports cs, int n,
                                                          TOut* __restrict__ out, uint64_t* __restrict__ evaluated) {
    __shared__ uint64_t s_ev[kBlock / 64];
    const int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    const bool live = t < nv;
    const int64_t src = order[live ? t : nv - 1];
    const double ux = fma((double)xyz[3 * src], h, -c0x), uy = fma((double)xyz[3 * src + 1], h, -c0y),
                 uz = fma((double)xyz[3 * src + 2], h, -c0z);
    const double mx = -2.0 * ux, my = -2.0 * uy, mz = -2.0 * uz, uu = fma(uz, uz, fma(uy, uy, ux * ux));
    const double lox = wave_min(ux), loy = wave_min(uy), loz = wave_min(uz);
    const double hix = wave_max(ux), hiy = wave_max(uy), hiz = wave_max(uz);
    const double* __restrict__ qx = cs.qx;
    const double* __restrict__ qy = cs.qy;
    const double* __restrict__ qz = cs.qz;
    const double* __restrict__ qq = cs.qq;
    const double* __restrict__ wx = cs.wx;
    const double* __restrict__ wy = cs.wy;
    const double* __restrict__ wz = cs.wz;
    double ax = 0.0, ay = 0.0, az = 0.0;
    uint32_t evals = 0;
    const int ntiles = (n + kCullTile - 1) / kCullTile;
#pragma unroll 1
    for (int k = 0; k < ntiles; ++k) {
        const double* b = cs.box + 6 * k;   // min x, y, z, max x, y, z of the tile's supports
        const double gx = fmax(0.0, fmax(b[0] - hix, lox - b[3]));
        const double gy = fmax(0.0, fmax(b[1] - hiy, loy - b[4]));
        const double gz = fmax(0.0, fmax(b[2] - hiz, loz - b[5]));
        if (fma(gz, gz, fma(gy, gy, gx * gx)) > kCullGap2) continue;
        const int j0 = k * kCullTile, j1 = min(n, j0 + kCullTile);
        int j = j0;
#pragma unroll 1
        for (; j + 8 <= j1; j += 8) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double d = fma(mx, qx[j + u], fma(my, qy[j + u], fma(mz, qz[j + u], uu + qq[j + u])));
                const double phi = wendland_quarter(d);
                ax = fma(wx[j + u], phi, ax);
                ay = fma(wy[j + u], phi, ay);
                az = fma(wz[j + u], phi, az);
            }
        }
#pragma unroll 1
        for (; j < j1; ++j) {
            const double d = fma(mx, qx[j], fma(my, qy[j], fma(mz, qz[j], uu + qq[j])));
            const double phi = wendland_quarter(d);
            ax = fma(wx[j], phi, ax);
            ay = fma(wy[j], phi, ay);
            az = fma(wz[j], phi, az);
        }
        evals += (uint32_t)(j1 - j0);
    }
    if (live) {
        out[3 * src] = (TOut)ax;
        out[3 * src + 1] = (TOut)ay;
        out[3 * src + 2] = (TOut)az;
    }
    // pairs evaluated: the wave's evaluated supports times its live points
    const int32_t nlive = wave_isum(live ? 1 : 0);
    if ((threadIdx.x & 63) == 0) s_ev[threadIdx.x >> 6] = (uint64_t)evals * (uint64_t)nlive;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t sum = 0;
        for (int w = 0; w < kBlock / 64; ++w) sum += s_ev[w];
        evaluated[blockIdx.x] = sum;
    }
}

void launch_cull_keys(hipStream_t s, int64_t nv, const void* xyz, int in_f64, double inv_r, const double c0[3],
                      const CullFrame& f, uint32_t* keys, int32_t* idx) {
    const unsigned g = (unsigned)((nv + kBlock - 1) / kBlock);
    const double h = 0.5 * inv_r;
    if (in_f64) GCB_LAUNCH(k_cull_keys<double>, dim3(g), dim3(kBlock), s, nv, (const double*)xyz, h, c0[0], c0[1],
                           c0[2], f, keys, idx);
    else GCB_LAUNCH(k_cull_keys<float>, dim3(g), dim3(kBlock), s, nv, (const float*)xyz, h, c0[0], c0[1], c0[2], f,
                    keys, idx);
}

template <typename TIn, typename TOut>
static void vol_cull(hipStream_t s, int64_t nv, const void* xyz, const int32_t* order, double h, const double c0[3],
                     const CullSupports& cs, int n, void* out, uint64_t* evaluated) {
    const unsigned g = (unsigned)((nv + kBlock - 1) / kBlock);
    GCB_LAUNCH((k_volume64_cull<TIn, TOut>), dim3(g), dim3(kBlock), s, nv, (const TIn*)xyz, order, h, c0[0], c0[1],
               c0[2], cs, n, (TOut*)out, evaluated);
}

void launch_volume_cull(hipStream_t s, int64_t nv, const void* xyz, int in_f64, const int32_t* order, double inv_r,
                        const double c0[3], const CullSupports& cs, int n, void* out, int out_f64,
                        uint64_t* evaluated) {
    const double h = 0.5 * inv_r;
    if (in_f64 && out_f64) vol_cull<double, double>(s, nv, xyz, order, h, c0, cs, n, out, evaluated);
    else if (in_f64) vol_cull<double, float>(s, nv, xyz, order, h, c0, cs, n, out, evaluated);
    else if (out_f64) vol_cull<float, double>(s, nv, xyz, order, h, c0, cs, n, out, evaluated);
    else vol_cull<float, float>(s, nv, xyz, order, h, c0, cs, n, out, evaluated);
}

int cull_blocks(int64_t nv) { return (int)((nv + kBlock - 1) / kBlock); }

void launch_volume_table(hipStream_t s, const Support& sp, int n) {
    if (n > 0) GCB_LAUNCH(k_volume_table, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), s, n, view(sp),
                          vtable(sp));
}

// ---------------------------------------------------------------- allocation-free deformation
// The support table of the FP64 sweep (four arrays of kNoAllocSupports doubles) or the FP32 copies
// of the supports (six arrays of kNoAllocSupports floats) live in this static array instead of in
// context buffers.  Every GPU holds one copy until the process ends; every call on that GPU shares
// it, so calls that overlap on one GPU race.  Both tables are written in full (entries 0..n-1)
// before the sweep reads them, so nothing needs clearing between calls.
constexpr int kNoAllocSupports = GCB_NOALLOC_MAX_SUPPORTS;
static __device__ __align__(256) double scratch[4 * kNoAllocSupports];

static std::mutex g_scratch_mu;
static std::vector<void*> g_scratch_ptr;   // device address of `scratch`, per device

hipError_t noalloc_setup(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize((size_t)device + 1, nullptr);
    if (g_scratch_ptr[(size_t)device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));   // `device` is current
    if (e != hipSuccess) return e;
    g_scratch_ptr[(size_t)device] = ptr;
    return hipSuccess;
}

void* noalloc_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return device >= 0 && device < (int)g_scratch_ptr.size() ? g_scratch_ptr[(size_t)device] : nullptr;
}

void launch_volume_noalloc(hipStream_t s, int64_t nv, const void* xyz, int in_f64, double inv_r, const Support& sp,
                           int n, void* out, int out_f64, int fp32_eval, void* scratch_ptr) {
    if (fp32_eval) {
        float* base = static_cast<float*>(scratch_ptr);
        float* const f[6] = {base, base + kNoAllocSupports, base + 2 * kNoAllocSupports,
                             base + 3 * kNoAllocSupports, base + 4 * kNoAllocSupports, base + 5 * kNoAllocSupports};
        volume32_into(s, nv, xyz, in_f64, inv_r, view(sp), f, n, out, out_f64);
    } else {
        double* base = static_cast<double*>(scratch_ptr);
        const VolTable vt{base, base + kNoAllocSupports, base + 2 * kNoAllocSupports, base + 3 * kNoAllocSupports};
        volume64_into(s, nv, xyz, in_f64, inv_r, view(sp), vt, n, out, out_f64);
    }
}

}  // namespace gcb
