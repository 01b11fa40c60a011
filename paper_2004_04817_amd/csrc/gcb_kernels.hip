// HIP kernels for gfx950: RBF interpolant sweeps (Eq. 1 / Eq. 6), group
// argmax (Algorithm 1), starting-node rule, inverse-factor append and the
// FP64 certificate.  Every lane owns one target point; support data is
// wave-uniform, so the pair loops read it through the scalar cache (SGPR
// operands of the VALU ops) and need neither LDS staging nor barriers.
#include "gcb_internal.h"
#include "gcb_kernels.h"

#include <algorithm>

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
//   k_sweep   group sweep (a3): a wave owns `tw` targets of the active group
//             and its 64 lanes split the n supports; per-block best record.
//   k_factor_l decision (a4) from the block records, then b and l = M b (a5).
//   k_factor_u u = M^T l, new row of M, W update, commit of the iteration.

__host__ __device__ inline int sweep_tw(int T) { return T >= 4096 ? 4 : (T >= 1024 ? 2 : 1); }

// Algorithm 1's decision for iteration k from the group's best candidate.
// Computed identically by every block of k_factor_l; only block 0 stores it.
struct Decision {
    int32_t app, done, quiet;
    double E;
};

__device__ __forceinline__ Decision decide_local(const GState& st, int n, int32_t m, double e2, double tol_abs,
                                                 int64_t nc_max, int64_t cap) {
    Decision d;
    const bool have = e2 >= 0.0;
    d.E = have ? sqrt(e2) : 0.0;
    d.app = 0;
    d.done = st.done;
    d.quiet = st.quiet;
    if (have && d.E > tol_abs) {
        if (n < nc_max && n < cap) {
            d.app = 1;
            d.quiet = 0;
        } else if (n >= nc_max) {
            d.done = 2;
        } else {
            d.done = 4;   // factor capacity: the host grows the arrays and this iteration runs again
        }
    } else {
        d.quiet += 1;
    }
    if (d.done == 0 && !d.app && d.quiet >= m) d.done = 1;
    return d;
}

__global__ __launch_bounds__(kBlock) void k_sweep(const GState* __restrict__ st, int32_t m,
                                                  const int32_t* __restrict__ goff, const double* __restrict__ px,
                                                  const double* __restrict__ py, const double* __restrict__ pz,
                                                  const double* __restrict__ pdx, const double* __restrict__ pdy,
                                                  const double* __restrict__ pdz, const uint8_t* __restrict__ inS,
                                                  const int32_t* __restrict__ perm, SupportView sv,
                                                  ArgRec* __restrict__ rec) {
    __shared__ Best sb[kWavesPerBlock];
    __shared__ int32_t sc[kWavesPerBlock];
    if (st->done) return;
    const int n = st->n;
    const int g = (int)(st->k % m);
    const int t0 = goff[g];
    const int T = goff[g + 1] - t0;
    const int tw = sweep_tw(T);
    const int per_block = kWavesPerBlock * tw;
    if ((int)blockIdx.x * per_block >= T) return;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int tbase = blockIdx.x * per_block + wave * tw;
    double tx[4], ty[4], tz[4], ax[4], ay[4], az[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int t = min(tbase + q, T - 1);
        tx[q] = px[t0 + t];
        ty[q] = py[t0 + t];
        tz[q] = pz[t0 + t];
        ax[q] = ay[q] = az[q] = 0.0;
    }
    // lane handles supports lane, lane+64, ...; four supports' loads are issued before their use
    int j = lane;
    for (; j + 192 < n; j += 256) {
        double sx[4], sy[4], sz[4], wx[4], wy[4], wz[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            sx[u] = sv.sx[j + 64 * u];
            sy[u] = sv.sy[j + 64 * u];
            sz[u] = sv.sz[j + 64 * u];
            wx[u] = sv.wx[j + 64 * u];
            wy[u] = sv.wy[j + 64 * u];
            wz[u] = sv.wz[j + 64 * u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q < tw) {
                    const double phi = wendland_r2(dist2(tx[q], ty[q], tz[q], sx[u], sy[u], sz[u]));
                    ax[q] = fma(wx[u], phi, ax[q]);
                    ay[q] = fma(wy[u], phi, ay[q]);
                    az[q] = fma(wz[u], phi, az[q]);
                }
            }
        }
    }
    for (; j < n; j += 64) {
        const double sx = sv.sx[j], sy = sv.sy[j], sz = sv.sz[j];
        const double wx = sv.wx[j], wy = sv.wy[j], wz = sv.wz[j];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q < tw) {
                const double phi = wendland_r2(dist2(tx[q], ty[q], tz[q], sx, sy, sz));
                ax[q] = fma(wx, phi, ax[q]);
                ay[q] = fma(wy, phi, ay[q]);
                az[q] = fma(wz, phi, az[q]);
            }
        }
    }
    Best b{-1.0, 0x7fffffff, -1};
    int32_t cnt = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q < tw) {
            const double fx = wave_sum(ax[q]), fy = wave_sum(ay[q]), fz = wave_sum(az[q]);
            const int t = tbase + q;
            if (t < T && !inS[t0 + t]) {
                const double ex = fx - pdx[t0 + t], ey = fy - pdy[t0 + t], ez = fz - pdz[t0 + t];
                const double e2 = fma(ez, ez, fma(ey, ey, ex * ex));
                const int32_t o = perm[t0 + t];
                if (better(e2, o, b.v, b.idx)) { b.v = e2; b.idx = o; b.aux = t0 + t; }
                cnt += 1;
            }
        }
    }
    if (lane == 0) {
        sb[wave] = b;
        sc[wave] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Best r = sb[0];
        int32_t c = sc[0];
        for (int w = 1; w < kWavesPerBlock; ++w) {
            if (better(sb[w].v, sb[w].idx, r.v, r.idx)) r = sb[w];
            c += sc[w];
        }
        rec[blockIdx.x] = ArgRec{r.v, r.idx, r.aux, c, 0};
    }
}

// l = M b, one wave per row of M (16 rows per block).  b_j = phi(|r_new -
// s_j| / R) is staged in LDS windows.  Block partials Pb[blk] = (b.W over
// columns [i0, i0+16), l.l over rows [i0, i0+16)).  Before that, every block
// reduces the sweep's block records to the group maximum and takes the
// decision; block 0 stores it (log, state, iteration record).  With
// init_t >= 0 the node is the starting node init[init_t] instead.
__global__ __launch_bounds__(kBigBlock) void k_factor_l(
    GState* __restrict__ st, IterRec* __restrict__ irec, const ArgRec* __restrict__ srec, int32_t m,
    const int32_t* __restrict__ goff, int init_t, const int32_t* __restrict__ init, const int32_t* __restrict__ pos_of,
    const double* __restrict__ px, const double* __restrict__ py, const double* __restrict__ pz, SupportView sv,
    const double* __restrict__ Mr, double* __restrict__ l, double* __restrict__ Pb, double tol_abs, int64_t nc_max,
    int64_t cap, int32_t* __restrict__ log_group, int32_t* __restrict__ log_node, double* __restrict__ log_err,
    int8_t* __restrict__ log_app, int64_t log_cap) {
    __shared__ double bw[kBWindow];
    __shared__ double sl[kRowsL];
    __shared__ int32_t s_app, s_pos, s_orig, s_n;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    if (init_t >= 0) {
        if (threadIdx.x == 0) {
            s_app = 1;
            s_orig = init[init_t];
            s_pos = pos_of[s_orig];
            s_n = init_t;
            if (blockIdx.x == 0) {
                irec->k = 0;
                irec->n = init_t;
                irec->app = 1;
                irec->init = 1;
                irec->ran = 0;
                irec->node_pos = s_pos;
                irec->node_orig = s_orig;
                irec->singular = 0;
                irec->E = 0.0;
            }
        }
    } else {
        // one snapshot of the state per block: block 0 updates it below, and
        // every thread of a block must take the same branches
        __shared__ GState s_st;
        if (threadIdx.x == 0) s_st = *st;
        __syncthreads();
        const GState sg = s_st;
        if (sg.done) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                irec->app = 0;
                irec->ran = 0;
            }
            return;
        }
        const int n = sg.n;
        const int g = (int)(sg.k % m);
        const int T = goff[g + 1] - goff[g];
        const int per_block = kWavesPerBlock * sweep_tw(T);
        const int nrec = (T + per_block - 1) / per_block;
        Best b{-1.0, 0x7fffffff, -1};
        int32_t c = 0;
        for (int i = threadIdx.x; i < nrec; i += kBigBlock) {
            const ArgRec r = srec[i];
            if (better(r.e2, r.orig, b.v, b.idx)) { b.v = r.e2; b.idx = r.orig; b.aux = r.pos; }
            c += r.count;
        }
        b = big_block_best(b);
        c = big_block_isum(c);
        if (threadIdx.x == 0) {
            const Decision d = decide_local(sg, n, m, b.v, tol_abs, nc_max, cap);
            s_app = d.app;
            s_pos = b.aux;
            s_orig = b.idx;
            s_n = n;
            if (blockIdx.x == 0) {
                if (d.done != 4) {
                    const int64_t it = sg.log_len;
                    if (it < log_cap) {
                        log_group[it] = g;
                        log_node[it] = b.v >= 0.0 ? b.idx : -1;
                        log_err[it] = d.E;
                        log_app[it] = (int8_t)d.app;
                    }
                    st->log_len = it + 1;
                    st->pairs_group = sg.pairs_group + (uint64_t)c * (uint64_t)n;
                }
                st->quiet = d.quiet;
                st->done = d.done;
                irec->k = sg.k;
                irec->n = n;
                irec->app = d.app;
                irec->init = 0;
                irec->ran = d.done != 4;
                irec->node_pos = d.app ? b.aux : -1;
                irec->node_orig = d.app ? b.idx : -1;
                irec->singular = 0;
                irec->E = d.E;
            }
        }
    }
    __syncthreads();
    if (!s_app) return;
    const int n = s_n;
    const int p = s_pos;
    const int nblk = max(1, (n + kRowsL - 1) / kRowsL);
    if ((int)blockIdx.x >= nblk) return;
    const int i0 = blockIdx.x * kRowsL;
    const int i1 = min(n, i0 + kRowsL);
    const int i = i0 + wave;
    const double qx = px[p], qy = py[p], qz = pz[p];
    double acc = 0.0;
    for (int w0 = 0; w0 < i1; w0 += kBWindow) {
        const int w1 = min(i1, w0 + kBWindow);
        __syncthreads();
        for (int j = w0 + threadIdx.x; j < w1; j += kBigBlock)
            bw[j - w0] = wendland_r2(dist2(qx, qy, qz, sv.sx[j], sv.sy[j], sv.sz[j]));
        __syncthreads();
        if (i < i1) {
            const double* Mi = Mr + (size_t)i * (i + 1) / 2;
            const int je = min(w1, i + 1);
            double a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int j = w0 + lane;
            for (; j + 192 < je; j += 256) {
                const double m0 = Mi[j], m1 = Mi[j + 64], m2 = Mi[j + 128], m3 = Mi[j + 192];
                acc = fma(m0, bw[j - w0], acc);
                a1 = fma(m1, bw[j + 64 - w0], a1);
                a2 = fma(m2, bw[j + 128 - w0], a2);
                a3 = fma(m3, bw[j + 192 - w0], a3);
            }
            for (; j < je; j += 64) acc = fma(Mi[j], bw[j - w0], acc);
            acc = (acc + a1) + (a2 + a3);
        }
    }
    const double li = wave_sum(acc);
    if (lane == 0 && i < i1) {
        l[i] = li;
        sl[wave] = li;
    }
    __syncthreads();
    if (wave == 0) {
        // this block's share of b.W (columns i0..i1-1) and of l.l (rows i0..i1-1), xor-tree order
        double fx = 0.0, fy = 0.0, fz = 0.0, ll = 0.0;
        const int j = i0 + lane;
        if (lane < kRowsL && j < i1) {
            const double bj = wendland_r2(dist2(qx, qy, qz, sv.sx[j], sv.sy[j], sv.sz[j]));
            fx = bj * sv.wx[j];
            fy = bj * sv.wy[j];
            fz = bj * sv.wz[j];
            ll = sl[lane] * sl[lane];
        }
        fx = wave_sum(fx);
        fy = wave_sum(fy);
        fz = wave_sum(fz);
        ll = wave_sum(ll);
        if (lane == 0) {
            Pb[4 * blockIdx.x + 0] = fx;
            Pb[4 * blockIdx.x + 1] = fy;
            Pb[4 * blockIdx.x + 2] = fz;
            Pb[4 * blockIdx.x + 3] = ll;
        }
    }
}

// u = M^T l, one wave per column j of M read from the column-major copy Mc
// (column j holds rows j.. at offset j*cap - j(j-1)/2).  Every block first
// sums the k_factor_l partials in block order to s = 1 - l.l and
// e = d_new - b.W.  Writes the new row [-u^T/sqrt(s), 1/sqrt(s)] into both
// copies of M and W <- [W - u e/s; e/s]; block 0 commits the iteration.
__global__ __launch_bounds__(kBigBlock) void k_factor_u(
    GState* __restrict__ st, IterRec* __restrict__ irec, const double* __restrict__ px, const double* __restrict__ py,
    const double* __restrict__ pz, const double* __restrict__ pdx, const double* __restrict__ pdy,
    const double* __restrict__ pdz, const int32_t* __restrict__ perm, uint8_t* __restrict__ inS, SupportMut sm,
    double* __restrict__ Mc, int64_t cap, const double* __restrict__ l, const double* __restrict__ Pb) {
    __shared__ double part[4][kBigBlock / 64];
    __shared__ double sh[5];
    __shared__ int32_t s_bad;
    // the iteration record is only read here (k_factor_l wrote it), so every
    // block sees the same values
    const IterRec r = *irec;
    if (!r.app) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && r.ran) st->k = r.k + 1;
        return;
    }
    const int n = r.n;
    const int p = r.node_pos;
    const int nbl = max(1, (n + kRowsL - 1) / kRowsL);
    const int ncb = max(1, (n + kRowsL - 1) / kRowsL);
    if ((int)blockIdx.x >= ncb) return;
    {
        // fixed-order reduction: per thread in block order, xor tree per wave, waves in order
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int b = threadIdx.x; b < nbl; b += kBigBlock)
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] += Pb[4 * b + c];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            v[c] = wave_sum(v[c]);
            if ((threadIdx.x & 63) == 0) part[c][threadIdx.x >> 6] = v[c];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double f[4] = {0.0, 0.0, 0.0, 0.0};
            for (int t = 0; t < kBigBlock / 64; ++t)
#pragma unroll
                for (int c = 0; c < 4; ++c) f[c] += part[c][t];
            const double s = 1.0 - f[3];
            s_bad = !(s > kSingularTol);
            sh[0] = 1.0 / sqrt(s);
            sh[1] = (pdx[p] - f[0]) / s;
            sh[2] = (pdy[p] - f[1]) / s;
            sh[3] = (pdz[p] - f[2]) / s;
        }
        __syncthreads();
    }
    if (s_bad) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->done = 3;
            st->singular_node = r.node_orig;
        }
        return;
    }
    const double rs = sh[0], cx = sh[1], cy = sh[2], cz = sh[3];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * kRowsL + wave;
    if (j < n) {
        const double* col = Mc + (size_t)j * cap - (size_t)j * (j - 1) / 2;   // rows j.. of column j
        double a0 = 0.0, a1 = 0.0;
        int i = j + lane;
        for (; i + 64 < n; i += 128) {
            a0 = fma(col[i - j], l[i], a0);
            a1 = fma(col[i + 64 - j], l[i + 64], a1);
        }
        if (i < n) a0 = fma(col[i - j], l[i], a0);
        const double u = wave_sum(a0 + a1);
        if (lane == 0) {
            const double v = -u * rs;
            sm.M[(size_t)n * (n + 1) / 2 + j] = v;
            Mc[(size_t)j * cap - (size_t)j * (j - 1) / 2 + (n - j)] = v;
            sm.wx[j] = fma(-u, cx, sm.wx[j]);
            sm.wy[j] = fma(-u, cy, sm.wy[j]);
            sm.wz[j] = fma(-u, cz, sm.wz[j]);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sm.M[(size_t)n * (n + 1) / 2 + n] = rs;
        Mc[(size_t)n * cap - (size_t)n * (n - 1) / 2] = rs;
        sm.wx[n] = cx;
        sm.wy[n] = cy;
        sm.wz[n] = cz;
        sm.sx[n] = px[p];
        sm.sy[n] = py[p];
        sm.sz[n] = pz[p];
        sm.orig[n] = perm[p];
        inS[p] = 1;
        st->n = n + 1;
        if (r.init) {
            st->init_left -= 1;   // starting nodes are not loop appends
        } else {
            st->pairs_append += (uint64_t)n;
            st->k = r.k + 1;
        }
    }
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

static void launch_factor(hipStream_t s, const IterCtx& ic, int n_ub, int init_t) {
    const Boundary& bd = *ic.bd;
    Support& sp = *ic.sp;
    const unsigned g = (unsigned)std::max(1, (n_ub + kRowsL - 1) / kRowsL);
    GCB_LAUNCH(k_factor_l, dim3(g), dim3(kBigBlock), s, ic.st, ic.irec, ic.srec, bd.m, bd.goff, init_t, ic.init,
               bd.pos_of, bd.px, bd.py, bd.pz, view(sp), sp.M, sp.l, ic.Pb, ic.tol_abs, ic.nc_max, sp.cap,
               ic.log_group, ic.log_node, ic.log_err, ic.log_app, ic.log_cap);
    GCB_LAUNCH(k_factor_u, dim3(g), dim3(kBigBlock), s, ic.st, ic.irec, bd.px, bd.py, bd.pz, bd.pdx, bd.pdy, bd.pdz,
               bd.perm, bd.inS, mut(sp), sp.Mc, sp.cap, sp.l, ic.Pb);
}

void launch_init_append(hipStream_t s, const IterCtx& ic, int t) { launch_factor(s, ic, t, t); }

// Blocks of k_sweep that cover every group size T <= gmax (the targets per
// wave, and so the targets per block, grow with T).
int sweep_blocks(int gmax) {
    int best = 1;
    for (int T : {std::min(gmax, 1023), std::min(gmax, 4095), gmax}) {
        const int per_block = kWavesPerBlock * sweep_tw(T);
        best = std::max(best, (T + per_block - 1) / per_block);
    }
    return best;
}

void launch_iteration(hipStream_t s, const IterCtx& ic, int n_ub) {
    const Boundary& bd = *ic.bd;
    const unsigned gs = (unsigned)sweep_blocks(bd.gmax);
    GCB_LAUNCH(k_sweep, dim3(gs), dim3(kBlock), s, ic.st, bd.m, bd.goff, bd.px, bd.py, bd.pz, bd.pdx, bd.pdy, bd.pdz,
               bd.inS, bd.perm, view(*ic.sp), ic.srec);
    launch_factor(s, ic, n_ub, -1);
}

void launch_transpose_factor(hipStream_t s, const double* Mr, double* Mc, int n, int64_t cap) {
    const int64_t cnt = (int64_t)n * (n + 1) / 2;
    if (cnt == 0) return;
    GCB_LAUNCH(k_transpose_factor, dim3((unsigned)((cnt + kBlock - 1) / kBlock)), dim3(kBlock), s, Mr, Mc, n, cap);
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
