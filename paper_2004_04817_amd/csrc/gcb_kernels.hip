// HIP kernels for gfx950: RBF interpolant sweeps (Eq. 1 / Eq. 6), group
// argmax (Algorithm 1), starting-node rule, inverse-factor append and the
// FP64 certificate.  Every lane owns one target point; support data is
// wave-uniform, so the pair loops read it through the scalar cache (SGPR
// operands of the VALU ops) and need neither LDS staging nor barriers.
#include "gcb_internal.h"
#include "gcb_kernels.h"

namespace gcb {

// ---------------------------------------------------------------- Eq. (2)
// Wendland C2 from the squared scaled distance r2 = (|r - r_i| / R)^2:
// eta = sqrt(r2) by one Newton step on the hardware reciprocal square root
// and one on the square root itself; t = clamp(1 - eta, 0, 1);
// phi = (1 - eta)^4 (4 eta + 1) = t^4 (5 - 4 t).  Exactly 0 for eta >= 1.
__device__ __forceinline__ double wendland_r2(double r2) {
    const double x = fmax(r2, 1e-200);
    double r = __builtin_amdgcn_rsq(x);
    double y = x * r;
    const double e = fma(-y, r, 1.0);
    r = fma(0.5 * r, e, r);
    y = x * r;
    const double d = fma(-y, y, x);
    y = fma(0.5 * r, d, y);
    const double t = fmin(fmax(1.0 - y, 0.0), 1.0);
    const double t2 = t * t;
    return (t2 * t2) * fma(-4.0, t, 5.0);
}

__device__ __forceinline__ double dist2(double ax, double ay, double az, double bx, double by, double bz) {
    const double dx = ax - bx, dy = ay - by, dz = az - bz;
    return fma(dz, dz, fma(dy, dy, dx * dx));
}

// Squared norm summed as (x^2 + y^2) + z^2 with no fused multiply-add, for
// the integer decisions of the starting-node rule.
__device__ __forceinline__ double sq3_exact(double x, double y, double z) {
#pragma clang fp contract(off)
    const double s = x * x + y * y;
    return s + z * z;
}

// Accumulate sum_{j in [s0, s1)} w_j phi(|t - s_j|) for one target per lane.
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

// ---------------------------------------------------------------- reductions
struct Best {
    double v;
    int32_t idx;   // decides ties (lowest wins)
    int32_t aux;
};

__device__ __forceinline__ bool better(double v, int32_t i, double bv, int32_t bi) {
    return v > bv || (v == bv && i < bi);
}

__device__ __forceinline__ Best wave_best(Best b) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double v = __shfl_xor(b.v, off, 64);
        const int32_t i = __shfl_xor(b.idx, off, 64);
        const int32_t a = __shfl_xor(b.aux, off, 64);
        if (better(v, i, b.v, b.idx)) { b.v = v; b.idx = i; b.aux = a; }
    }
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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

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
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---------------------------------------------------------------- sweep chunking
// Split-K layout of a group sweep: T targets in wave tiles of 64, n supports
// in `nch` chunks of `cs` supports.  A function of (T, n) only, so the
// summation order never depends on scheduling.
__host__ __device__ inline void sweep_split(int T, int n, int& ntile, int& nch, int& cs) {
    ntile = (T + 63) / 64;
    int want = (2048 + ntile - 1) / (ntile > 0 ? ntile : 1);
    int lim = (n + 7) / 8;
    nch = want < kMaxChunks ? want : kMaxChunks;
    if (nch > lim) nch = lim;
    if (nch < 1) nch = 1;
    cs = (n + nch - 1) / nch;
    if (cs < 1) cs = 1;
    nch = (n + cs - 1) / cs;
    if (nch < 1) nch = 1;
}

// ---------------------------------------------------------------- group sweep (a3)
// Wave w of the grid takes (target tile w % ntile, support chunk w / ntile)
// and writes its partial sums to P[chunk][c][t] (c = x, y, z; stride Tmax).
__global__ __launch_bounds__(kBlock) void k_group_sweep64(const GState* __restrict__ st, int32_t m,
                                                          const int32_t* __restrict__ goff,
                                                          const double* __restrict__ px,
                                                          const double* __restrict__ py,
                                                          const double* __restrict__ pz, SupportView sv,
                                                          double* __restrict__ P, int32_t Tmax) {
    if (st->done) return;
    const int g = (int)(st->k % m);
    const int t0 = goff[g];
    const int T = goff[g + 1] - t0;
    const int n = st->n;
    if (T <= 0 || n <= 0) return;   // empty group (possible with an explicit partition)
    int ntile, nch, cs;
    sweep_split(T, n, ntile, nch, cs);
    const int gw = (int)((blockIdx.x * (size_t)kBlock + threadIdx.x) >> 6);
    const int tile = gw % ntile;
    const int ch = gw / ntile;
    if (ch >= nch) return;
    const int lane = threadIdx.x & 63;
    const int t = tile * 64 + lane;
    const bool live = t < T;
    const int tt = live ? t : T - 1;
    const double tx = px[t0 + tt], ty = py[t0 + tt], tz = pz[t0 + tt];
    double ax = 0.0, ay = 0.0, az = 0.0;
    const int s0 = ch * cs;
    const int s1 = min(n, s0 + cs);
    accumulate64(tx, ty, tz, s0, s1, sv.sx, sv.sy, sv.sz, sv.wx, sv.wy, sv.wz, ax, ay, az);
    if (live) {
        double* Pc = P + (size_t)ch * 3 * Tmax;
        Pc[t] = ax;
        Pc[Tmax + t] = ay;
        Pc[2 * (size_t)Tmax + t] = az;
    }
}

// Sum the chunk partials in chunk order, form e^2 = |F - d|^2 for the
// targets not in S, and reduce each block to its best (e^2, lowest index).
__global__ __launch_bounds__(kBlock) void k_group_reduce(const GState* __restrict__ st, int32_t m,
                                                         const int32_t* __restrict__ goff,
                                                         const double* __restrict__ pdx,
                                                         const double* __restrict__ pdy,
                                                         const double* __restrict__ pdz,
                                                         const uint8_t* __restrict__ inS,
                                                         const int32_t* __restrict__ perm,
                                                         const double* __restrict__ P, int32_t Tmax,
                                                         ArgRec* __restrict__ rec) {
    if (st->done) return;
    const int g = (int)(st->k % m);
    const int t0 = goff[g];
    const int T = goff[g + 1] - t0;
    const int n = st->n;
    int ntile, nch, cs;
    sweep_split(T, n, ntile, nch, cs);
    const int t = blockIdx.x * kBlock + threadIdx.x;
    Best b{-1.0, 0x7fffffff, -1};
    int32_t cnt = 0;
    if (t < T && !inS[t0 + t]) {
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int c = 0; c < nch; ++c) {
            const double* Pc = P + (size_t)c * 3 * Tmax;
            fx += Pc[t];
            fy += Pc[Tmax + t];
            fz += Pc[2 * (size_t)Tmax + t];
        }
        const double ex = fx - pdx[t0 + t], ey = fy - pdy[t0 + t], ez = fz - pdz[t0 + t];
        b.v = fma(ez, ez, fma(ey, ey, ex * ex));
        b.idx = perm[t0 + t];
        b.aux = t0 + t;
        cnt = 1;
    }
    cnt = wave_isum(cnt);
    __shared__ int32_t scnt[kBlock / 64];
    if ((threadIdx.x & 63) == 0) scnt[threadIdx.x >> 6] = cnt;
    b = block_best(b);
    if (threadIdx.x == 0) {
        int32_t c = 0;
        for (int i = 0; i < kBlock / 64; ++i) c += scnt[i];
        rec[blockIdx.x] = ArgRec{b.v, b.idx, b.aux, c, 0};
    }
}

// One block: reduce the per-block records in block order, log the
// iteration and take Algorithm 1's decision (append iff E > E* and |S| < cap).
__global__ __launch_bounds__(kBlock) void k_group_decide(GState* __restrict__ st, int32_t m,
                                                         const int32_t* __restrict__ goff,
                                                         const ArgRec* __restrict__ rec, double tol_abs,
                                                         int64_t nc_max, int64_t cap, int32_t* __restrict__ log_group,
                                                         int32_t* __restrict__ log_node, double* __restrict__ log_err,
                                                         int8_t* __restrict__ log_app, int64_t log_cap) {
    if (st->done) return;
    const int g = (int)(st->k % m);
    const int T = goff[g + 1] - goff[g];
    const int nrec = (T + kBlock - 1) / kBlock;
    Best b{-1.0, 0x7fffffff, -1};
    int32_t cnt = 0;
    for (int i = threadIdx.x; i < nrec; i += kBlock) {
        const ArgRec r = rec[i];
        if (better(r.e2, r.orig, b.v, b.idx)) { b.v = r.e2; b.idx = r.orig; b.aux = r.pos; }
        cnt += r.count;
    }
    __shared__ int32_t scnt[kBlock / 64];
    cnt = wave_isum(cnt);
    if ((threadIdx.x & 63) == 0) scnt[threadIdx.x >> 6] = cnt;
    b = block_best(b);
    if (threadIdx.x != 0) return;
    int32_t total = 0;
    for (int i = 0; i < kBlock / 64; ++i) total += scnt[i];
    const bool have = b.v >= 0.0;
    const double E = have ? sqrt(b.v) : 0.0;
    const int n = st->n;
    st->pairs_group += (uint64_t)total * (uint64_t)n;
    int32_t app = 0;
    if (have && E > tol_abs) {
        if (n < nc_max && n < cap) {
            app = 1;
            st->quiet = 0;
        } else if (n >= nc_max) {
            st->done = 2;
        } else {
            st->done = 4;   // factor capacity: the host grows the arrays and resumes
        }
    } else {
        st->quiet += 1;
    }
    if (st->done != 4) {
        const int64_t it = st->log_len;
        if (it < log_cap) {
            log_group[it] = g;
            log_node[it] = have ? b.idx : -1;
            log_err[it] = E;
            log_app[it] = (int8_t)app;
        }
        st->log_len = it + 1;
    }
    st->E = E;
    st->app = app;
    st->node_pos = app ? b.aux : -1;
    st->node_orig = app ? b.idx : -1;
    if (st->done == 0 && !app && st->quiet >= m) st->done = 1;
    if (st->done != 4) st->k += 1;   // the append kernels that follow do not read k
}

// ---------------------------------------------------------------- append (a5)
// b_j = phi(|r_new - s_j| / R), j < n, in FP64.
__global__ __launch_bounds__(kBlock) void k_append_b(const GState* __restrict__ st, const double* __restrict__ px,
                                                     const double* __restrict__ py, const double* __restrict__ pz,
                                                     SupportView sv, double* __restrict__ b) {
    if (!st->app) return;
    const int n = st->n;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const int p = st->node_pos;
    b[j] = wendland_r2(dist2(px[p], py[p], pz[p], sv.sx[j], sv.sy[j], sv.sz[j]));
}

// l = M b over the packed lower triangle: one wave per row i < n.
__global__ __launch_bounds__(kBlock) void k_append_l(const GState* __restrict__ st, const double* __restrict__ M,
                                                     const double* __restrict__ b, double* __restrict__ l) {
    if (!st->app) return;
    const int n = st->n;
    const int i = (int)((blockIdx.x * (size_t)kBlock + threadIdx.x) >> 6);
    if (i >= n) return;
    const int lane = threadIdx.x & 63;
    const double* Mi = M + (size_t)i * (i + 1) / 2;
    double acc = 0.0;
    for (int j = lane; j <= i; j += 64) acc = fma(Mi[j], b[j], acc);
    acc = wave_sum(acc);
    if (lane == 0) l[i] = acc;
}

// Partial column sums of u = M^T l: block (column tile x, row chunk y)
// covers columns [x*kBlock, +kBlock) and rows [y*kBlock, +kBlock).
__global__ __launch_bounds__(kBlock) void k_append_u(const GState* __restrict__ st, const double* __restrict__ M,
                                                     const double* __restrict__ l, double* __restrict__ Pu,
                                                     int64_t pu_stride) {
    if (!st->app) return;
    const int n = st->n;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    const int r0 = blockIdx.y * kBlock;
    if (r0 >= n || (int)(blockIdx.x * kBlock) >= n) return;
    if (r0 + kBlock - 1 < (int)(blockIdx.x * kBlock)) return;   // block entirely above the diagonal
    const int r1 = min(n, r0 + kBlock);
    double acc = 0.0;
    if (j < n) {
        for (int i = max(r0, j); i < r1; ++i) acc = fma(M[(size_t)i * (i + 1) / 2 + j], l[i], acc);
        Pu[(size_t)blockIdx.y * pu_stride + j] = acc;
    }
}

// Finish the append in one block: s = 1 - l.l, residual e = d_new - b.W,
// new row of M = [-u^T / sqrt(s), 1 / sqrt(s)], W <- [W - u e / s; e / s].
__global__ __launch_bounds__(1024) void k_append_finish(GState* __restrict__ st, const double* __restrict__ px,
                                                        const double* __restrict__ py, const double* __restrict__ pz,
                                                        const double* __restrict__ pdx, const double* __restrict__ pdy,
                                                        const double* __restrict__ pdz, const int32_t* __restrict__ perm,
                                                        uint8_t* __restrict__ inS, SupportMut sm,
                                                        const double* __restrict__ b, const double* __restrict__ l,
                                                        const double* __restrict__ Pu, int64_t pu_stride) {
    if (!st->app) return;
    const int n = st->n;
    const int p = st->node_pos;
    double ll = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    for (int j = threadIdx.x; j < n; j += 1024) {
        ll = fma(l[j], l[j], ll);
        fx = fma(b[j], sm.wx[j], fx);
        fy = fma(b[j], sm.wy[j], fy);
        fz = fma(b[j], sm.wz[j], fz);
    }
    ll = block_sum<1024>(ll);
    fx = block_sum<1024>(fx);
    fy = block_sum<1024>(fy);
    fz = block_sum<1024>(fz);
    __shared__ double sh[5];
    __shared__ int bad;
    if (threadIdx.x == 0) {
        const double s = 1.0 - ll;
        bad = !(s > kSingularTol);
        sh[0] = s;
        sh[1] = pdx[p] - fx;
        sh[2] = pdy[p] - fy;
        sh[3] = pdz[p] - fz;
        sh[4] = 1.0 / sqrt(s);
    }
    __syncthreads();
    if (bad) {
        if (threadIdx.x == 0) {
            st->done = 3;
            st->singular_node = st->node_orig;
            st->app = 0;
        }
        return;
    }
    const double s = sh[0], ex = sh[1], ey = sh[2], ez = sh[3], rs = sh[4];
    const double cx = ex / s, cy = ey / s, cz = ez / s;
    double* Mn = sm.M + (size_t)n * (n + 1) / 2;
    const int nrow = (n + kBlock - 1) / kBlock;
    for (int j = threadIdx.x; j < n; j += 1024) {
        double u = 0.0;
        for (int r = j / kBlock; r < nrow; ++r) u += Pu[(size_t)r * pu_stride + j];
        Mn[j] = -u * rs;
        sm.wx[j] = fma(-u, cx, sm.wx[j]);
        sm.wy[j] = fma(-u, cy, sm.wy[j]);
        sm.wz[j] = fma(-u, cz, sm.wz[j]);
    }
    if (threadIdx.x == 0) {
        Mn[n] = rs;
        sm.wx[n] = cx;
        sm.wy[n] = cy;
        sm.wz[n] = cz;
        sm.sx[n] = px[p];
        sm.sy[n] = py[p];
        sm.sz[n] = pz[p];
        sm.orig[n] = perm[p];
        inS[p] = 1;
        st->n = n + 1;
        st->app = 0;
        if (st->init_left > 0) st->init_left -= 1;   // starting nodes are not loop appends
        else st->pairs_append += (uint64_t)n;
    }
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

// Stage the t-th starting node as the node to append.
__global__ void k_init_stage(GState* __restrict__ st, const int32_t* __restrict__ init, int t,
                             const int32_t* __restrict__ pos_of) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int o = init[t];
    st->app = 1;
    st->node_orig = o;
    st->node_pos = pos_of[o];
}

// ---------------------------------------------------------------- certificate (a6)
// e_j^2 over all boundary nodes; per block: max and sum.
__global__ __launch_bounds__(kBlock) void k_certify(int64_t nb, const double* __restrict__ px,
                                                    const double* __restrict__ py, const double* __restrict__ pz,
                                                    const double* __restrict__ pdx, const double* __restrict__ pdy,
                                                    const double* __restrict__ pdz, SupportView sv, int n,
                                                    double* __restrict__ red) {
    const int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    const bool live = t < nb;
    const int64_t tt = live ? t : nb - 1;
    double ax = 0.0, ay = 0.0, az = 0.0;
    accumulate64(px[tt], py[tt], pz[tt], 0, n, sv.sx, sv.sy, sv.sz, sv.wx, sv.wy, sv.wz, ax, ay, az);
    double e2 = 0.0;
    if (live) {
        const double ex = ax - pdx[t], ey = ay - pdy[t], ez = az - pdz[t];
        e2 = fma(ez, ez, fma(ey, ey, ex * ex));
    }
    Best b{live ? e2 : -1.0, (int32_t)t, 0};
    b = block_best(b);
    const double s = block_sum<kBlock>(e2);
    if (threadIdx.x == 0) {
        red[2 * blockIdx.x] = b.v;
        red[2 * blockIdx.x + 1] = s;
    }
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

// ---------------------------------------------------------------- volume (a7)
template <typename TIn, typename TOut>
__global__ __launch_bounds__(kBlock) void k_volume64(int64_t nv, const TIn* __restrict__ xyz, double inv_r,
                                                     SupportView sv, int n, TOut* __restrict__ out) {
    const int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x;
    const bool live = t < nv;
    const int64_t tt = live ? t : nv - 1;
    const double tx = (double)xyz[3 * tt] * inv_r;
    const double ty = (double)xyz[3 * tt + 1] * inv_r;
    const double tz = (double)xyz[3 * tt + 2] * inv_r;
    double ax = 0.0, ay = 0.0, az = 0.0;
    accumulate64(tx, ty, tz, 0, n, sv.sx, sv.sy, sv.sz, sv.wx, sv.wy, sv.wz, ax, ay, az);
    if (live) {
        out[3 * t] = (TOut)ax;
        out[3 * t + 1] = (TOut)ay;
        out[3 * t + 2] = (TOut)az;
    }
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

// ---------------------------------------------------------------- launchers
#define GCB_LAUNCH(kern, grid, block, stream, ...) hipLaunchKernelGGL(kern, grid, block, 0, stream, __VA_ARGS__)

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

void launch_append(hipStream_t s, GState* st, const Boundary& bd, Support& sp, int n_ub) {
    SupportView sv = view(sp);
    SupportMut sm = mut(sp);
    const unsigned nb_b = (unsigned)((n_ub + kBlock - 1) / kBlock);
    GCB_LAUNCH(k_append_b, dim3(nb_b > 0 ? nb_b : 1), dim3(kBlock), s, st, bd.px, bd.py, bd.pz, sv, sp.b);
    const unsigned nw = (unsigned)((n_ub + 3) / 4);
    GCB_LAUNCH(k_append_l, dim3(nw > 0 ? nw : 1), dim3(kBlock), s, st, sp.M, sp.b, sp.l);
    GCB_LAUNCH(k_append_u, dim3(nb_b > 0 ? nb_b : 1, nb_b > 0 ? nb_b : 1), dim3(kBlock), s, st, sp.M, sp.l, sp.Pu,
               (int64_t)sp.cap);
    GCB_LAUNCH(k_append_finish, dim3(1), dim3(1024), s, st, bd.px, bd.py, bd.pz, bd.pdx, bd.pdy, bd.pdz, bd.perm,
               bd.inS, sm, sp.b, sp.l, sp.Pu, (int64_t)sp.cap);
}

void launch_init_stage(hipStream_t s, GState* st, const int32_t* init, int t, const int32_t* pos_of) {
    GCB_LAUNCH(k_init_stage, dim3(1), dim3(64), s, st, init, t, pos_of);
}

void launch_iteration(hipStream_t s, GState* st, const Boundary& bd, Support& sp, double* P, int32_t Tmax,
                      ArgRec* rec, double tol_abs, int64_t nc_max, int64_t log_cap, int32_t* lg, int32_t* ln,
                      double* le, int8_t* la, int n_ub) {
    SupportView sv = view(sp);
    // upper bound of waves over any group and any n <= n_ub: tiles of the largest group x kMaxChunks
    const int64_t waves = (int64_t)((bd.gmax + 63) / 64) * kMaxChunks;
    const unsigned gs = (unsigned)((waves * 64 + kBlock - 1) / kBlock);
    GCB_LAUNCH(k_group_sweep64, dim3(gs), dim3(kBlock), s, st, bd.m, bd.goff, bd.px, bd.py, bd.pz, sv, P, Tmax);
    const unsigned gr = (unsigned)((bd.gmax + kBlock - 1) / kBlock);
    GCB_LAUNCH(k_group_reduce, dim3(gr), dim3(kBlock), s, st, bd.m, bd.goff, bd.pdx, bd.pdy, bd.pdz, bd.inS, bd.perm,
               P, Tmax, rec);
    GCB_LAUNCH(k_group_decide, dim3(1), dim3(kBlock), s, st, bd.m, bd.goff, rec, tol_abs, nc_max, sp.cap, lg, ln, le, la,
               log_cap);
    launch_append(s, st, bd, sp, n_ub);
}

void launch_certify(hipStream_t s, const Boundary& bd, const Support& sp, int n, double* red, double* out) {
    const unsigned g = (unsigned)((bd.nb + kBlock - 1) / kBlock);
    GCB_LAUNCH(k_certify, dim3(g), dim3(kBlock), s, bd.nb, bd.px, bd.py, bd.pz, bd.pdx, bd.pdy, bd.pdz, view(sp), n, red);
    GCB_LAUNCH(k_certify_final, dim3(1), dim3(kBlock), s, (int)g, red, out);
}

template <typename TIn, typename TOut>
static void vol(hipStream_t s, int64_t nv, const void* xyz, double inv_r, SupportView sv, int n, void* out) {
    const unsigned g = (unsigned)((nv + kBlock - 1) / kBlock);
    GCB_LAUNCH((k_volume64<TIn, TOut>), dim3(g), dim3(kBlock), s, nv, (const TIn*)xyz, inv_r, sv, n, (TOut*)out);
}

void launch_volume(hipStream_t s, int64_t nv, const void* xyz, int in_f64, double inv_r, const Support& sp, int n,
                   void* out, int out_f64) {
    SupportView sv = view(sp);
    if (in_f64 && out_f64) vol<double, double>(s, nv, xyz, inv_r, sv, n, out);
    else if (in_f64) vol<double, float>(s, nv, xyz, inv_r, sv, n, out);
    else if (out_f64) vol<float, double>(s, nv, xyz, inv_r, sv, n, out);
    else vol<float, float>(s, nv, xyz, inv_r, sv, n, out);
}

}  // namespace gcb
