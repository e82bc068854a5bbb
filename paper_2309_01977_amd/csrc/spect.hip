// spect.hip - gfx950 kernels and C ABI of the SPECT projector library.
//
// The operator is the parallel-hole SPECT system matrix of the paper (Section
// 2.1.1, Eq. 1): per angle, rotate the object (bilinear, per axial slice),
// attenuate along the rotated depth axis, blur every depth plane with its own
// separable Gaussian collimator-detector kernel, and sum over depth.  The
// transpose runs the same steps backwards.  include/spect.h states the
// discretisation and the array layouts.
//
// Parallel decomposition (one launch covers a list of angles):
//   workgroup = (angle, axial slab of 16 slices, depth chunk); thread (j', h)
//   owns detector bin j' and axial rows 8h..8h+7 of the slab and walks the
//   depth axis of its chunk from the detector side.  Per depth it samples the
//   object (four bilinear corners, each a contiguous z-run), updates its
//   running attenuation sum, blurs along the bin axis through LDS (the
//   neighbouring bins belong to other threads), and scatters the axial blur
//   of its own eight rows into registers that hold the slab's partial
//   projection rows.  A reduction kernel adds the partial rows of
//   neighbouring slabs and of the depth chunks.
//   Depth chunks raise parallelism for small angle subsets; their
//   attenuation offsets come from a pre-pass that walks each ray once.
// Back projection:
//   back_rot  : same workgroups; per depth, axial blur of the projection in
//               registers, bin-axis blur through LDS, times exp(-tau); writes
//               the rotated-frame volume Z of each angle to the workspace;
//   back_gather: thread per (x, y, slab) gathers from the <= 3x3 rotated
//               samples whose bilinear footprint covers the voxel, with the
//               forward's own FP32 weights, so the pair is an exact transpose
//               up to summation order; the OSEM update is fused here.
// No MFMA: nothing on this path is a dense contraction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "spect.h"

namespace {

constexpr int SLAB = 16;   // axial rows per workgroup
constexpr int ROWS = 8;    // axial rows per thread
constexpr int MAXL = 128;  // angles per launch

struct AngleList {
    int n;
    int idx[MAXL];
};

// Device view of the plan tables.
struct DevGeom {
    const float2 *cs;   // [A] (cos, sin)
    const float2 *xy0;  // [A][N] rotated-frame origin of ray j': X = X0 + i' cos, Y = Y0 + i' sin
    const int *kdep;    // [A][N] blur radius per depth
    const float *taps;  // [A][N][TS] one-sided taps g[0..K]
    int N, Nz, A, TS;
    float tau_scale;    // dx * log2(e): exp(-tau) = exp2(-tau_scale * (sum mu))
};

// --------------------------------------------------------------- helpers --

struct Corners {
    int o00, o10, o01, o11;      // element offsets of (x0,y0), (x0+1,y0), (x0,y0+1), (x0+1,y0+1)
    float w00, w10, w01, w11;    // bilinear weights, 0 for corners outside the grid
};

// Bilinear footprint of point (X, Y) in an N x N slice with z-runs of length Nz.
__device__ __forceinline__ Corners corners(float X, float Y, int N, int Nz)
{
    const float xf = floorf(X), yf = floorf(Y);
    const int x0 = (int)xf, y0 = (int)yf;
    const float fx = X - xf, fy = Y - yf;
    const float gx = 1.f - fx, gy = 1.f - fy;
    const bool vx0 = (unsigned)x0 < (unsigned)N, vx1 = (unsigned)(x0 + 1) < (unsigned)N;
    const bool vy0 = (unsigned)y0 < (unsigned)N, vy1 = (unsigned)(y0 + 1) < (unsigned)N;
    Corners c;
    c.w00 = (vx0 && vy0) ? gx * gy : 0.f;
    c.w10 = (vx1 && vy0) ? fx * gy : 0.f;
    c.w01 = (vx0 && vy1) ? gx * fy : 0.f;
    c.w11 = (vx1 && vy1) ? fx * fy : 0.f;
    const int xa = min(max(x0, 0), N - 1), xb = min(max(x0 + 1, 0), N - 1);
    const int ya = min(max(y0, 0), N - 1), yb = min(max(y0 + 1, 0), N - 1);
    c.o00 = (xa * N + ya) * Nz;
    c.o10 = (xb * N + ya) * Nz;
    c.o01 = (xa * N + yb) * Nz;
    c.o11 = (xb * N + yb) * Nz;
    return c;
}

// Raw corner values of ROWS axial rows starting at kb: v[corner][row] for the
// corners (x0,y0), (x0+1,y0), (x0,y0+1), (x0+1,y0+1).  Every load is issued
// unconditionally (rows past Nz read a clamped, valid address and are zeroed
// when combined), so all of them are in flight together.  Vector path:
// Nz % 4 == 0 and a 16-byte aligned volume.
struct Raw {
    float v[4][ROWS];
};

template <bool VEC>
__device__ __forceinline__ void load_raw(const float *__restrict__ vol, const Corners &c, int kb, int Nz, Raw &r)
{
    const int o[4] = {c.o00, c.o10, c.o01, c.o11};
    if constexpr (VEC) {
#pragma unroll
        for (int q = 0; q < ROWS / 4; ++q) {
            const int k = min(kb + 4 * q, Nz - 4);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float4 t = *reinterpret_cast<const float4 *>(vol + o[j] + k);
                r.v[j][4 * q + 0] = t.x;
                r.v[j][4 * q + 1] = t.y;
                r.v[j][4 * q + 2] = t.z;
                r.v[j][4 * q + 3] = t.w;
            }
        }
    } else {
#pragma unroll
        for (int rr = 0; rr < ROWS; ++rr) {
            const int k = min(kb + rr, Nz - 1);
#pragma unroll
            for (int j = 0; j < 4; ++j) r.v[j][rr] = vol[o[j] + k];
        }
    }
}

// Bilinear combination of raw corner values; rows >= Nz give 0.
__device__ __forceinline__ void combine(const Raw &r, const Corners &c, int kb, int Nz, float (&v)[ROWS])
{
#pragma unroll
    for (int rr = 0; rr < ROWS; ++rr) {
        const float z = (kb + rr < Nz) ? 1.f : 0.f;
        v[rr] = z * fmaf(c.w11, r.v[3][rr], fmaf(c.w01, r.v[2][rr], fmaf(c.w10, r.v[1][rr], c.w00 * r.v[0][rr])));
    }
}

template <bool VEC>
__device__ __forceinline__ void sample_rows(const float *__restrict__ vol, const Corners &c, int kb, int Nz,
                                            float (&v)[ROWS])
{
    Raw r;
    load_raw<VEC>(vol, c, kb, Nz, r);
    combine(r, c, kb, Nz, v);
}

// Attenuation factors for one depth: exp(-dx (mu/2 + sum beyond)), then add
// this depth's samples to the running sum.
__device__ __forceinline__ void attenuate(const float (&m)[ROWS], float (&S)[ROWS], float scale,
                                          float (&att)[ROWS])
{
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        att[r] = __builtin_amdgcn_exp2f(-scale * fmaf(0.5f, m[r], S[r]));
        S[r] += m[r];
    }
}

// LDS row buffers for the bin-axis blur: [buf][q][row][h] float4, row = j' + KMC,
// KMC zero rows on each side.
__device__ __forceinline__ int wb_index(int buf, int q, int row, int h, int nrows)
{
    return ((buf * 2 + q) * nrows + row) * 2 + h;
}

// Zero the KMC padding rows on both sides of both row buffers.
template <int KMC>
__device__ __forceinline__ void zero_padding(float4 *smem, int N, int nrows)
{
    if constexpr (KMC > 0) {
        for (int i = threadIdx.x; i < 2 * 2 * 2 * KMC * 2; i += blockDim.x) {
            const int hh = i & 1, rest = i >> 1;
            const int prow = rest % (2 * KMC), bq = rest / (2 * KMC);
            const int row = prow < KMC ? prow : prow + N;
            smem[wb_index(bq >> 1, bq & 1, row, hh, nrows)] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
}

// Bin-axis blur of the thread's 8 rows: U = g0 W(j') + sum_m g_m (W(j'-m) + W(j'+m)).
__device__ __forceinline__ void blur_bins(const float4 *__restrict__ wb, int buf, int row, int h,
                                          int nrows, int K, const float *__restrict__ g,
                                          const float (&self)[ROWS], float (&u)[ROWS])
{
    const float g0 = g[0];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) u[r] = g0 * self[r];
    for (int m = 1; m <= K; ++m) {
        const float gm = g[m];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const float4 a = wb[wb_index(buf, q, row - m, h, nrows)];
            const float4 b = wb[wb_index(buf, q, row + m, h, nrows)];
            u[4 * q + 0] = fmaf(gm, a.x + b.x, u[4 * q + 0]);
            u[4 * q + 1] = fmaf(gm, a.y + b.y, u[4 * q + 1]);
            u[4 * q + 2] = fmaf(gm, a.z + b.z, u[4 * q + 2]);
            u[4 * q + 3] = fmaf(gm, a.w + b.w, u[4 * q + 3]);
        }
    }
}

// Axial blur as a scatter: input row s (0..7) adds g(|l|) u[s] to output row
// s + l, l in [-K, K]; acc[t] holds output row kb - KMC + t.
template <int K, int KMC>
__device__ __forceinline__ void zscatter(float (&acc)[ROWS + 2 * KMC], const float (&u)[ROWS],
                                         const float *__restrict__ g)
{
    float gk[K + 1];
#pragma unroll
    for (int l = 0; l <= K; ++l) gk[l] = g[l];
#pragma unroll
    for (int s = 0; s < ROWS; ++s)
#pragma unroll
        for (int l = -K; l <= K; ++l) acc[s + l + KMC] = fmaf(gk[l < 0 ? -l : l], u[s], acc[s + l + KMC]);
}

template <int K, int KMC>
struct ZScatter {
    static __device__ __forceinline__ void run(int k, float (&acc)[ROWS + 2 * KMC], const float (&u)[ROWS],
                                               const float *__restrict__ g)
    {
        if (k == K)
            zscatter<K, KMC>(acc, u, g);
        else
            ZScatter<K - 1, KMC>::run(k, acc, u, g);
    }
};
template <int KMC>
struct ZScatter<-1, KMC> {
    static __device__ __forceinline__ void run(int, float (&)[ROWS + 2 * KMC], const float (&)[ROWS],
                                               const float *__restrict__)
    {
    }
};

// Axial blur as a gather from a column of LDS values: win[t] is axial row
// kb - K + t; out[s] = sum_l g(|l|) win[s + K - l].
template <int K>
__device__ __forceinline__ void zgather(const float *__restrict__ win, const float *__restrict__ g,
                                        float (&out)[ROWS])
{
    float v[ROWS + 2 * K];
#pragma unroll
    for (int t = 0; t < ROWS + 2 * K; ++t) v[t] = win[t];
    float gk[K + 1];
#pragma unroll
    for (int l = 0; l <= K; ++l) gk[l] = g[l];
#pragma unroll
    for (int s = 0; s < ROWS; ++s) {
        float a = gk[0] * v[s + K];
#pragma unroll
        for (int l = 1; l <= K; ++l) a = fmaf(gk[l], v[s + K - l] + v[s + K + l], a);
        out[s] = a;
    }
}

template <int K>
struct ZGather {
    static __device__ __forceinline__ void run(int k, const float *__restrict__ col, int base,
                                               const float *__restrict__ g, float (&out)[ROWS])
    {
        if (k == K)
            zgather<K>(col + base - K, g, out);
        else
            ZGather<K - 1>::run(k, col, base, g, out);
    }
};
template <>
struct ZGather<-1> {
    static __device__ __forceinline__ void run(int, const float *__restrict__, int, const float *__restrict__,
                                               float (&)[ROWS])
    {
    }
};

// ----------------------------------------------------------- attenuation --

struct TauArgs {
    DevGeom g;
    AngleList L;
    const float *mu;
    float *tau;      // [L][nchunk][N][Nz]: sum of mu samples over the depths of chunk c
    int nchunk, dchunk;
    int vec;
};

// One thread per (angle, chunk, bin, 8 axial rows): sum the attenuation
// samples of the chunk's depths.  Chunk c covers depths
// [N - (c+1) D, N - c D); chunk 0 touches the detector.  A chunk's starting
// attenuation is the sum of the partial sums of the chunks nearer the
// detector (the last chunk's own sum is never needed).
template <bool VEC>
__global__ __launch_bounds__(256) void tau_prepass(TauArgs a)
{
    const int N = a.g.N, Nz = a.g.Nz;
    const int ngrp = (Nz + ROWS - 1) / ROWS;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * ngrp) return;
    const int ch = blockIdx.y, al = blockIdx.z;
    const int ang = a.L.idx[al];
    const int jp = t / ngrp, kb = (t % ngrp) * ROWS;
    const float2 cs = a.g.cs[ang];
    const float2 o = a.g.xy0[(size_t)ang * N + jp];
    float S[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) S[r] = 0.f;
    const int ihi = N - ch * a.dchunk - 1;
    const int ilo = max(0, N - (ch + 1) * a.dchunk);
#pragma unroll 2
    for (int ip = ihi; ip >= ilo; --ip) {
        const Corners c = corners(fmaf((float)ip, cs.x, o.x), fmaf((float)ip, cs.y, o.y), N, Nz);
        float m[ROWS];
        sample_rows<VEC>(a.mu, c, kb, Nz, m);
#pragma unroll
        for (int r = 0; r < ROWS; ++r) S[r] += m[r];
    }
    float *dst = a.tau + (((size_t)al * a.nchunk + ch) * N + jp) * Nz;
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
        if (kb + r < Nz) dst[kb + r] = S[r];
}

// Attenuation sum at the detector side of chunk `chunk`: the partial sums of
// chunks 0 .. chunk-1.
__device__ __forceinline__ void chunk_start(const float *__restrict__ tau, int al, int nchunk, int chunk, int N,
                                            int Nz, int jp, int kb, float (&S)[ROWS])
{
#pragma unroll
    for (int r = 0; r < ROWS; ++r) S[r] = 0.f;
    for (int c = 0; c < chunk; ++c) {
        const float *src = tau + (((size_t)al * nchunk + c) * N + jp) * Nz;
#pragma unroll
        for (int r = 0; r < ROWS; ++r) S[r] += (kb + r < Nz) ? src[kb + r] : 0.f;
    }
}

// ------------------------------------------------------------- forward ----

struct FwdArgs {
    DevGeom g;
    AngleList L;
    const float *f;
    const float *mu;
    const float *tau;   // chunk offsets or nullptr when nchunk == 1
    float *part;        // [L][nslab][nchunk][N][SLAB + 2 KMC]
    int nslab, nchunk, dchunk;
    int vec;
};

template <bool MU, int KMC, bool VEC>
__global__ __launch_bounds__(512) void fwd_main(FwdArgs a)
{
    extern __shared__ float4 smem[];
    const int N = a.g.N, Nz = a.g.Nz;
    const int slab = blockIdx.x, chunk = blockIdx.y, al = blockIdx.z;
    const int ang = a.L.idx[al];
    const int jp = threadIdx.x >> 1, h = threadIdx.x & 1;
    const bool active = jp < N;
    const int nrows = N + 2 * KMC;
    const int kb = slab * SLAB + h * ROWS;

    zero_padding<KMC>(smem, N, nrows);

    const float2 cs = a.g.cs[ang];
    const float2 o = active ? a.g.xy0[(size_t)ang * N + jp] : make_float2(0.f, 0.f);
    float S[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) S[r] = 0.f;
    if (MU && chunk > 0 && active) chunk_start(a.tau, al, a.nchunk, chunk, N, Nz, jp, kb, S);
    float acc[ROWS + 2 * KMC];
#pragma unroll
    for (int t = 0; t < ROWS + 2 * KMC; ++t) acc[t] = 0.f;

    const int ihi = N - chunk * a.dchunk - 1;
    const int ilo = max(0, N - (chunk + 1) * a.dchunk);
    const int *kd = a.g.kdep + (size_t)ang * N;
    int buf = 0;
    __syncthreads();
    for (int ip = ihi; ip >= ilo; --ip) {
        const int K = kd[ip];
        const float *gt = a.g.taps + ((size_t)ang * N + ip) * a.g.TS;
        float w[ROWS];
        if (active) {
            const Corners cn = corners(fmaf((float)ip, cs.x, o.x), fmaf((float)ip, cs.y, o.y), N, Nz);
            Raw rf, rm;
            load_raw<VEC>(a.f, cn, kb, Nz, rf);
            if (MU) load_raw<VEC>(a.mu, cn, kb, Nz, rm);
            combine(rf, cn, kb, Nz, w);
            if (MU) {
                float m[ROWS], att[ROWS];
                combine(rm, cn, kb, Nz, m);
                attenuate(m, S, a.g.tau_scale, att);
#pragma unroll
                for (int r = 0; r < ROWS; ++r) w[r] *= att[r];
            }
            smem[wb_index(buf, 0, jp + KMC, h, nrows)] = make_float4(w[0], w[1], w[2], w[3]);
            smem[wb_index(buf, 1, jp + KMC, h, nrows)] = make_float4(w[4], w[5], w[6], w[7]);
        }
        __syncthreads();
        if (active) {
            float u[ROWS];
            blur_bins(smem, buf, jp + KMC, h, nrows, K, gt, w, u);
            ZScatter<KMC, KMC>::run(K, acc, u, gt);
        }
        buf ^= 1;
    }

    // merge the two half-slabs of each bin and write the partial rows
    __syncthreads();
    float *mb = reinterpret_cast<float *>(smem);
    constexpr int AC = ROWS + 2 * KMC;
    constexpr int R = SLAB + 2 * KMC;
    if (active && h == 1) {
#pragma unroll
        for (int t = 0; t < AC; ++t) mb[jp * (AC + 1) + t] = acc[t];
    }
    __syncthreads();
    if (active && h == 0) {
        float *dst = a.part + ((((size_t)al * a.nslab + slab) * a.nchunk + chunk) * N + jp) * R;
#pragma unroll
        for (int t = 0; t < R; t += 4) {
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int tt = t + e;
                float x = (tt < AC) ? acc[tt < AC ? tt : 0] : 0.f;
                if (tt >= ROWS) x += mb[jp * (AC + 1) + tt - ROWS];
                v[e] = x;
            }
            *reinterpret_cast<float4 *>(dst + t) = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
}

struct ReduceArgs {
    AngleList L;
    const float *part;
    int N, Nz, nslab, nchunk, kmc;
    int mode;           // 0: write projection rows; 1: OSEM ratio into q
    float *proj;        // mode 0: (A, N, Nz)
    const float *g;     // mode 1: measured data (A, N, Nz)
    const float *s_add; // mode 1: additive term or nullptr
    float *q;           // mode 1: [L][N][Nz]
};

// Sum the partial rows of all chunks and overlapping slabs for one output
// element (angle, bin, row).
__global__ __launch_bounds__(256) void fwd_reduce(ReduceArgs a)
{
    const int N = a.N, Nz = a.Nz;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * Nz) return;
    const int al = blockIdx.y;
    const int ang = a.L.idx[al];
    const int r = t / Nz, k = t % Nz;
    const int R = SLAB + 2 * a.kmc;
    const int slo = max(0, (k + a.kmc - R) / SLAB);  // loose bound; rows are checked below
    const int shi = min(a.nslab - 1, (k + a.kmc) / SLAB);
    float sum = 0.f;
    for (int c = 0; c < a.nchunk; ++c)
        for (int s = slo; s <= shi; ++s) {
            const int row = k - s * SLAB + a.kmc;
            if (row < 0 || row >= R) continue;
            sum += a.part[((((size_t)al * a.nslab + s) * a.nchunk + c) * N + r) * R + row];
        }
    const size_t o = ((size_t)ang * N + r) * Nz + k;
    if (a.mode == 0) {
        a.proj[o] = sum;
    } else {
        const float e = a.s_add ? sum + a.s_add[o] : sum;
        a.q[((size_t)al * N + r) * Nz + k] = e > 0.f ? a.g[o] / e : 0.f;
    }
}

// ---------------------------------------------------------- back project --

struct BackRotArgs {
    DevGeom g;
    AngleList L;
    const float *y;     // projections; row of list entry al at y + row_index * N * Nz
    int y_compact;      // 1: row_index = al (compact list buffer); 0: row_index = angle
    int ones;           // 1: y is all ones (sensitivity)
    const float *mu;
    const float *tau;
    float *z;           // [L][nslab][N][N][SLAB] rotated-frame values
    int nslab, nchunk, dchunk;
    int vec;
};

template <bool MU, int KMC, bool VEC>
__global__ __launch_bounds__(512) void back_rot(BackRotArgs a)
{
    extern __shared__ float4 smem[];
    const int N = a.g.N, Nz = a.g.Nz;
    const int slab = blockIdx.x, chunk = blockIdx.y, al = blockIdx.z;
    const int ang = a.L.idx[al];
    const int jp = threadIdx.x >> 1, h = threadIdx.x & 1;
    const bool active = jp < N;
    const int nrows = N + 2 * KMC;
    const int k0 = slab * SLAB;
    const int kb = k0 + h * ROWS;
    constexpr int R = SLAB + 2 * KMC;
    constexpr int YP = R + 1;
    float *ybuf = reinterpret_cast<float *>(smem + 2 * 2 * nrows * 2);

    zero_padding<KMC>(smem, N, nrows);
    // axial rows k0 - KMC .. k0 + SLAB + KMC - 1 of the projection, per bin
    if (active) {
        const float *yr = a.y + ((size_t)(a.y_compact ? al : ang) * N + jp) * Nz;
        for (int t = h; t < R; t += 2) {
            const int k = k0 - KMC + t;
            float v = 0.f;
            if (k >= 0 && k < Nz) v = a.ones ? 1.f : yr[k];
            ybuf[jp * YP + t] = v;
        }
    }

    const float2 cs = a.g.cs[ang];
    const float2 o = active ? a.g.xy0[(size_t)ang * N + jp] : make_float2(0.f, 0.f);
    float S[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) S[r] = 0.f;
    if (MU && chunk > 0 && active) chunk_start(a.tau, al, a.nchunk, chunk, N, Nz, jp, kb, S);
    const int ihi = N - chunk * a.dchunk - 1;
    const int ilo = max(0, N - (chunk + 1) * a.dchunk);
    const int *kd = a.g.kdep + (size_t)ang * N;
    int buf = 0;
    __syncthreads();
    for (int ip = ihi; ip >= ilo; --ip) {
        const int K = kd[ip];
        const float *gt = a.g.taps + ((size_t)ang * N + ip) * a.g.TS;
        float v[ROWS];
        Corners cn;
        Raw rm;
        if (active) {
            if (MU) {
                // attenuation samples of this depth, in flight during the blur
                cn = corners(fmaf((float)ip, cs.x, o.x), fmaf((float)ip, cs.y, o.y), N, Nz);
                load_raw<VEC>(a.mu, cn, kb, Nz, rm);
            }
            ZGather<KMC>::run(K, ybuf + jp * YP, h * ROWS + KMC, gt, v);
            smem[wb_index(buf, 0, jp + KMC, h, nrows)] = make_float4(v[0], v[1], v[2], v[3]);
            smem[wb_index(buf, 1, jp + KMC, h, nrows)] = make_float4(v[4], v[5], v[6], v[7]);
        }
        __syncthreads();
        if (active) {
            float u[ROWS];
            blur_bins(smem, buf, jp + KMC, h, nrows, K, gt, v, u);
            if (MU) {
                float m[ROWS], att[ROWS];
                combine(rm, cn, kb, Nz, m);
                attenuate(m, S, a.g.tau_scale, att);
#pragma unroll
                for (int r = 0; r < ROWS; ++r) u[r] *= att[r];
            }
            float *dst = a.z + ((((size_t)al * a.nslab + slab) * N + ip) * N + jp) * SLAB + h * ROWS;
            reinterpret_cast<float4 *>(dst)[0] = make_float4(u[0], u[1], u[2], u[3]);
            reinterpret_cast<float4 *>(dst)[1] = make_float4(u[4], u[5], u[6], u[7]);
        }
        buf ^= 1;
    }
}

struct GatherArgs {
    DevGeom g;
    AngleList L;
    const float *z;
    int nslab;
    int mode;            // 0: out = sum; 1: out += sum; 2: OSEM update of out with sens
    float *out;
    const float *sens;
};

// Transpose of the bilinear rotation, as a gather.  Workgroup = 8 x 8 object
// columns x one slab; a wave covers 16 columns and four lanes share a column,
// one per 16-byte quad of its 16 axial rows, so that every candidate brick
// (64 bytes) is read by four adjacent lanes.  For each angle a column takes
// the <= 3 x 3 rotated samples around its rotated position; the weight of
// sample P is the bilinear hat max(0, 1 - |X_P - x|) max(0, 1 - |Y_P - y|),
// with X_P, Y_P computed by the forward's own FP32 expression, so the weights
// equal the forward's to within one rounding.
constexpr int GT = 8;  // gather tile edge

__global__ __launch_bounds__(256) void back_gather(GatherArgs a)
{
    const int N = a.g.N, Nz = a.g.Nz;
    const int tiles = (N + GT - 1) / GT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane >> 2, q = lane & 3;
    const int x = (blockIdx.x / tiles) * GT + wave * 2 + (col >> 3);
    const int y = (blockIdx.x % tiles) * GT + (col & 7);
    const int slab = blockIdx.y;
    if (x >= N || y >= N) return;
    const float c = 0.5f * (float)(N - 1);
    const float xx = (float)x - c, yy = (float)y - c;
    const float fxv = (float)x, fyv = (float)y;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    const size_t zstride = (size_t)a.nslab * N * N * SLAB;
    const float *zq = a.z + (size_t)slab * N * N * SLAB + 4 * q;
    for (int al = 0; al < a.L.n; ++al) {
        const int ang = a.L.idx[al];
        const float2 cs = a.g.cs[ang];
        const float2 *xy0 = a.g.xy0 + (size_t)ang * N;
        const float wdw = fabsf(cs.x) + fabsf(cs.y) + 1e-3f;
        const float ic = c + cs.x * xx + cs.y * yy;
        const float jc = c - cs.y * xx + cs.x * yy;
        const int ilo = (int)ceilf(ic - wdw), jlo = (int)ceilf(jc - wdw);
        const float *zb = zq + (size_t)al * zstride;
        float2 o[3];
        float4 v[9];
#pragma unroll
        for (int dj = 0; dj < 3; ++dj) o[dj] = xy0[min(max(jlo + dj, 0), N - 1)];
#pragma unroll
        for (int d = 0; d < 9; ++d) {
            const int ipc = min(max(ilo + d / 3, 0), N - 1), jpc = min(max(jlo + d % 3, 0), N - 1);
            v[d] = *reinterpret_cast<const float4 *>(zb + ((size_t)ipc * N + jpc) * SLAB);
        }
#pragma unroll
        for (int d = 0; d < 9; ++d) {
            const int ip = ilo + d / 3, jp = jlo + d % 3;
            const bool inr = (unsigned)ip < (unsigned)N && (unsigned)jp < (unsigned)N;
            const float X = fmaf((float)ip, cs.x, o[d % 3].x), Y = fmaf((float)ip, cs.y, o[d % 3].y);
            const float wx = fmaxf(0.f, 1.f - fabsf(X - fxv)), wy = fmaxf(0.f, 1.f - fabsf(Y - fyv));
            const float w = inr ? wx * wy : 0.f;
            acc[0] = fmaf(w, v[d].x, acc[0]);
            acc[1] = fmaf(w, v[d].y, acc[1]);
            acc[2] = fmaf(w, v[d].z, acc[2]);
            acc[3] = fmaf(w, v[d].w, acc[3]);
        }
    }
    const size_t base = ((size_t)x * N + y) * Nz;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int k = slab * SLAB + 4 * q + r;
        if (k >= Nz) break;
        float *p = a.out + base + k;
        if (a.mode == 0) {
            *p = acc[r];
        } else if (a.mode == 1) {
            *p += acc[r];
        } else {
            const float sv = a.sens[base + k];
            if (sv > 0.f) *p = *p * acc[r] / sv;
        }
    }
}

__global__ __launch_bounds__(256) void fill_zero(float *p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

}  // namespace

// ================================================================= host ===

struct spect_plan {
    int N, Nz, A;
    double voxel_cm;
    int kmax;   // largest blur radius
    int kmc;    // compile-time radius class (multiple of 4, <= 32)
    int TS;     // tap row stride
    int device;
    int fwd_slots[2];   // resident forward workgroups on the device, without / with attenuation
    int back_slots[2];  // same for the rotated-frame back-projection kernel
    void *dmem;
    DevGeom g;
};

namespace {

// ------------------------------------------------------------- timing ----
// Optional per-kernel timing: while enabled, every launch is bracketed by two
// HIP events recorded on the launch's own stream.

enum KernelId { K_TAU = 0, K_FWD, K_REDUCE, K_BACK_ROT, K_GATHER, K_FILL, K_COUNT };
const char *const kKernelNames[K_COUNT] = {"tau_prepass", "fwd_main", "fwd_reduce", "back_rot",
                                           "back_gather", "fill_zero"};

struct ProfRec {
    int kernel;
    hipEvent_t a, b;
};

std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;

struct ProfScope {
    int kernel;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    bool on;
    ProfScope(int k, hipStream_t s) : kernel(k), st(s)
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        on = g_prof_on;
        if (on && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, st);
        else
            on = false;
    }
    ~ProfScope()
    {
        if (!on) return;
        (void)hipEventRecord(b, st);
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof.push_back({kernel, a, b});
    }
};

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok()
{
    g_err.clear();
    return SPECT_OK;
}

void trig_deg(double deg, double *c, double *s)
{
    double r = std::fmod(deg, 360.0);
    if (r < 0) r += 360.0;
    const double t = r * (M_PI / 180.0);
    double cc = std::cos(t), ss = std::sin(t);
    if (std::fabs(cc) < 1e-15) cc = 0.0;
    if (std::fabs(ss) < 1e-15) ss = 0.0;
    *c = cc;
    *s = ss;
}

// Blur radius and one-sided taps at depth ip for detector distance R.
int depth_kernel(const spect_geometry &g, double R, int ip, std::vector<double> *taps)
{
    const double c = 0.5 * (g.n - 1);
    double d = R - (ip - c) * g.voxel_cm;
    if (d < 0) d = 0;
    const double sigma = g.psf_a * d + g.psf_b;
    if (!(sigma > 0)) {
        if (taps) taps->assign(1, 1.0);
        return 0;
    }
    const double s = sigma / g.voxel_cm;
    const double nsig = g.psf_nsigma > 0 ? g.psf_nsigma : 4.0;
    const double kr = std::ceil(nsig * s - 1e-9);
    if (kr > 1e6) return 1 << 30;
    const int K = kr < 0 ? 0 : (int)kr;
    if (taps && K <= SPECT_MAX_K) {
        double sum = 0;
        for (int m = -K; m <= K; ++m) sum += std::exp(-(double)m * m / (2 * s * s));
        taps->resize(K + 1);
        for (int m = 0; m <= K; ++m) (*taps)[m] = std::exp(-(double)m * m / (2 * s * s)) / sum;
    }
    return K;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(SPECT_EHIP, "%s: %s", what, hipGetErrorString(e));
}

struct Tuning {
    int nslab, nchunk, dchunk;
};

enum { T_FWD = 1, T_BACK = 2, T_BOTH = 3 };

// Depth chunking of a launch over n_list angles: pick the chunk count that
// minimises (waves of resident workgroups) x (depths per workgroup + a fixed
// per-workgroup cost), summed over the kernels that share the split (both
// passes of an OSEM step share the attenuation offsets).  Splitting adds an
// attenuation pre-pass when a map is given.
Tuning tune(const spect_plan *p, int n_list, bool mu, int which)
{
    Tuning t;
    t.nslab = (p->Nz + SLAB - 1) / SLAB;
    const long base = (long)std::max(1, n_list) * t.nslab;
    const int cap = std::max(1, p->N / 8);  // at least 8 depths per chunk
    double best = 1e300;
    t.nchunk = 1;
    t.dchunk = p->N;
    for (int nc = 1; nc <= cap; ++nc) {
        const int D = (p->N + nc - 1) / nc;
        const int ncc = (p->N + D - 1) / D;
        if (ncc != nc) continue;
        const long wgs = base * ncc;
        double cost = 0;
        if (which & T_FWD) cost += (double)((wgs + p->fwd_slots[mu] - 1) / p->fwd_slots[mu]) * (D + 6);
        if (which & T_BACK) cost += (double)((wgs + p->back_slots[mu] - 1) / p->back_slots[mu]) * (D + 6);
        if (mu && ncc > 1) cost += 2 + D / 4.0;
        if (cost < best - 1e-9) {
            best = cost;
            t.nchunk = ncc;
            t.dchunk = D;
        }
    }
    return t;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t tau_bytes(const spect_plan *p, const Tuning &t, int n_list, bool mu)
{
    if (!mu || t.nchunk <= 1) return 0;
    return align256(sizeof(float) * (size_t)n_list * t.nchunk * p->N * p->Nz);
}

size_t part_bytes(const spect_plan *p, const Tuning &t, int n_list)
{
    return align256(sizeof(float) * (size_t)n_list * t.nslab * t.nchunk * p->N * (SLAB + 2 * p->kmc));
}

size_t z_bytes(const spect_plan *p, const Tuning &t, int n_list)
{
    return align256(sizeof(float) * (size_t)n_list * t.nslab * p->N * p->N * SLAB);
}

// Angles per back-projection group: bounded by the launch list and by a
// 512 MiB rotated-frame buffer.
int back_group(const spect_plan *p, int n_idx)
{
    const size_t per = sizeof(float) * (size_t)((p->Nz + SLAB - 1) / SLAB) * SLAB * p->N * p->N;
    size_t g = (size_t(512) << 20) / std::max<size_t>(per, 1);
    g = std::max<size_t>(1, std::min<size_t>(g, MAXL));
    return (int)std::min<size_t>(g, std::max(1, n_idx));
}

// Launch lists of a call: batches of B angles and a smaller last batch.
std::vector<int> batch_sizes(int n, int B)
{
    std::vector<int> v;
    if (n >= B) v.push_back(B);
    if (n % B) v.push_back(n % B);
    return v;
}

size_t fwd_need(const spect_plan *p, int nl, bool mu, int which = T_FWD)
{
    const Tuning t = tune(p, nl, mu, which);
    return tau_bytes(p, t, nl, mu) + part_bytes(p, t, nl);
}

size_t back_need(const spect_plan *p, int nl, bool mu, int which = T_BACK)
{
    const Tuning t = tune(p, nl, mu, which);
    return tau_bytes(p, t, nl, mu) + z_bytes(p, t, nl);
}

size_t fwd_ws(const spect_plan *p, int n_idx, bool mu)
{
    size_t b = 0;
    for (int nl : batch_sizes(std::max(n_idx, 1), MAXL)) b = std::max(b, fwd_need(p, nl, mu));
    return b;
}

size_t back_ws(const spect_plan *p, int n_idx, bool mu)
{
    size_t b = 0;
    const int G = back_group(p, n_idx);
    for (int nl : batch_sizes(std::max(n_idx, 1), G)) b = std::max(b, back_need(p, nl, mu));
    return b;
}

// OSEM workspace: [q][tau][partial | z]; the back pass reuses the forward's
// attenuation offsets and overwrites the partial rows.  Interleaved subsets
// have at most two sizes, floor(A/M) and ceil(A/M).
size_t osem_q_bytes(const spect_plan *p, int M)
{
    const int nl_max = (p->A + M - 1) / M;
    return align256(sizeof(float) * (size_t)nl_max * p->N * p->Nz);
}

size_t osem_ws(const spect_plan *p, int M, bool mu)
{
    size_t b = 0;
    for (int nl : {p->A / M, (p->A + M - 1) / M}) {
        if (nl < 1) continue;
        const Tuning t = tune(p, nl, mu, T_BOTH);
        b = std::max(b, tau_bytes(p, t, nl, mu) + std::max(part_bytes(p, t, nl), z_bytes(p, t, nl)));
    }
    return osem_q_bytes(p, M) + b;
}

typedef void (*KernelFn)(FwdArgs);
typedef void (*BackFn)(BackRotArgs);

template <bool MU, bool VEC>
KernelFn fwd_kernel_k(int kmc)
{
    switch (kmc) {
    case 0: return fwd_main<MU, 0, VEC>;
    case 4: return fwd_main<MU, 4, VEC>;
    case 8: return fwd_main<MU, 8, VEC>;
    case 12: return fwd_main<MU, 12, VEC>;
    case 16: return fwd_main<MU, 16, VEC>;
    case 20: return fwd_main<MU, 20, VEC>;
    case 24: return fwd_main<MU, 24, VEC>;
    case 28: return fwd_main<MU, 28, VEC>;
    default: return fwd_main<MU, 32, VEC>;
    }
}

KernelFn fwd_kernel(bool mu, int kmc, bool vec)
{
    if (mu) return vec ? fwd_kernel_k<true, true>(kmc) : fwd_kernel_k<true, false>(kmc);
    return vec ? fwd_kernel_k<false, true>(kmc) : fwd_kernel_k<false, false>(kmc);
}

template <bool MU, bool VEC>
BackFn back_kernel_k(int kmc)
{
    switch (kmc) {
    case 0: return back_rot<MU, 0, VEC>;
    case 4: return back_rot<MU, 4, VEC>;
    case 8: return back_rot<MU, 8, VEC>;
    case 12: return back_rot<MU, 12, VEC>;
    case 16: return back_rot<MU, 16, VEC>;
    case 20: return back_rot<MU, 20, VEC>;
    case 24: return back_rot<MU, 24, VEC>;
    case 28: return back_rot<MU, 28, VEC>;
    default: return back_rot<MU, 32, VEC>;
    }
}

BackFn back_kernel(bool mu, int kmc, bool vec)
{
    if (mu) return vec ? back_kernel_k<true, true>(kmc) : back_kernel_k<true, false>(kmc);
    return vec ? back_kernel_k<false, true>(kmc) : back_kernel_k<false, false>(kmc);
}

int block_threads(int N) { return std::min(512, ((2 * N + 63) / 64) * 64); }

size_t wb_bytes(const spect_plan *p) { return sizeof(float4) * 2 * 2 * 2 * (size_t)(p->N + 2 * p->kmc); }

size_t fwd_smem(const spect_plan *p)
{
    const size_t merge = sizeof(float) * (size_t)p->N * (ROWS + 2 * p->kmc + 1);
    return std::max(wb_bytes(p), merge);
}

size_t back_smem(const spect_plan *p)
{
    return wb_bytes(p) + sizeof(float) * (size_t)p->N * (SLAB + 2 * p->kmc + 1);
}

// Kernels that need more than 64 KiB of dynamic LDS must say so first.
void allow_smem(const void *fn, size_t bytes)
{
    if (bytes > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

bool aligned16(const void *q) { return ((uintptr_t)q & 15) == 0; }

int check_plan(const spect_plan *p)
{
    if (!p) return fail(SPECT_EINVAL, "plan is NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != p->device)
        return fail(SPECT_EINVAL, "current HIP device %d is not the plan's device %d", dev, p->device);
    return SPECT_OK;
}

int check_ptr(const void *q, const char *name, bool nullable)
{
    if (!q) return nullable ? SPECT_OK : fail(SPECT_EINVAL, "%s is NULL", name);
    if ((uintptr_t)q & 3) return fail(SPECT_EINVAL, "%s is not 4-byte aligned", name);
    return SPECT_OK;
}

int make_list(const spect_plan *p, const int32_t *idx, int32_t n_idx, std::vector<int> *out)
{
    out->clear();
    if (!idx) {
        for (int i = 0; i < p->A; ++i) out->push_back(i);
        return SPECT_OK;
    }
    if (n_idx < 0) return fail(SPECT_EINVAL, "n_idx = %d is negative", n_idx);
    for (int i = 0; i < n_idx; ++i) {
        if (idx[i] < 0 || idx[i] >= p->A)
            return fail(SPECT_EINVAL, "angle_idx[%d] = %d outside [0, %d)", i, idx[i], p->A);
        out->push_back(idx[i]);
    }
    return SPECT_OK;
}

int check_ws(void *ws, size_t have, size_t need)
{
    if (need == 0) return SPECT_OK;
    if (!ws) return fail(SPECT_EINVAL, "workspace is NULL but %zu bytes are needed", need);
    if ((uintptr_t)ws & 255) return fail(SPECT_EINVAL, "workspace is not 256-byte aligned");
    if (have < need) return fail(SPECT_EINVAL, "workspace has %zu bytes, %zu needed", have, need);
    return SPECT_OK;
}

AngleList to_list(const int *a, int n)
{
    AngleList L;
    L.n = n;
    for (int i = 0; i < n; ++i) L.idx[i] = a[i];
    for (int i = n; i < MAXL; ++i) L.idx[i] = 0;
    return L;
}

// Attenuation offsets for chunked launches.
void launch_tau(const spect_plan *p, const AngleList &L, const Tuning &t, const float *mu, float *tau,
                bool vec, hipStream_t st)
{
    TauArgs a;
    a.g = p->g;
    a.L = L;
    a.mu = mu;
    a.tau = tau;
    a.nchunk = t.nchunk;
    a.dchunk = t.dchunk;
    a.vec = vec;
    const int ngrp = (p->Nz + ROWS - 1) / ROWS;
    dim3 grid((p->N * ngrp + 255) / 256, t.nchunk - 1, L.n);
    ProfScope ps(K_TAU, st);
    hipLaunchKernelGGL(vec ? tau_prepass<true> : tau_prepass<false>, grid, dim3(256), 0, st, a);
}

// Forward projection of one list into partial rows, then the reduction.
// ws holds [tau][partial]; tau_given != nullptr reuses attenuation offsets
// already computed for the same list (the tau region is then skipped).
int run_forward(const spect_plan *p, const float *f, const float *mu, const AngleList &L, char *ws,
                size_t ws_avail, const float *tau_given, int mode, float *proj, const float *g,
                const float *s_add, float *q, bool vec, int which, hipStream_t st)
{
    const Tuning t = tune(p, L.n, mu != nullptr, which);
    if (fwd_need(p, L.n, mu != nullptr, which) > ws_avail)
        return fail(SPECT_EINVAL, "workspace too small for a %d-angle forward launch", L.n);
    const float *tau = nullptr;
    size_t off = 0;
    const size_t tb = tau_bytes(p, t, L.n, mu != nullptr);
    if (tb) {
        off += tb;
        if (tau_given) {
            tau = tau_given;
        } else {
            launch_tau(p, L, t, mu, reinterpret_cast<float *>(ws), vec, st);
            tau = reinterpret_cast<const float *>(ws);
        }
    }
    float *part = reinterpret_cast<float *>(ws + off);
    FwdArgs a;
    a.g = p->g;
    a.L = L;
    a.f = f;
    a.mu = mu;
    a.tau = tau;
    a.part = part;
    a.nslab = t.nslab;
    a.nchunk = t.nchunk;
    a.dchunk = t.dchunk;
    a.vec = vec;
    KernelFn fk = fwd_kernel(mu != nullptr, p->kmc, vec);
    allow_smem(reinterpret_cast<const void *>(fk), fwd_smem(p));
    {
        ProfScope ps(K_FWD, st);
        hipLaunchKernelGGL(fk, dim3(t.nslab, t.nchunk, L.n), dim3(block_threads(p->N)), fwd_smem(p), st, a);
    }
    ReduceArgs r;
    r.L = L;
    r.part = part;
    r.N = p->N;
    r.Nz = p->Nz;
    r.nslab = t.nslab;
    r.nchunk = t.nchunk;
    r.kmc = p->kmc;
    r.mode = mode;
    r.proj = proj;
    r.g = g;
    r.s_add = s_add;
    r.q = q;
    {
        ProfScope ps(K_REDUCE, st);
        hipLaunchKernelGGL(fwd_reduce, dim3((p->N * p->Nz + 255) / 256, L.n), dim3(256), 0, st, r);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    return SPECT_OK;
}

// Back projection of one list: rotated-frame pass, then the gather.
// ws holds [tau][z]; tau_given as in run_forward.
int run_back(const spect_plan *p, const float *y, int y_compact, int ones, const float *mu,
             const AngleList &L, char *ws, size_t ws_avail, const float *tau_given, int mode, float *out,
             const float *sens, bool vec, int which, hipStream_t st)
{
    const Tuning t = tune(p, L.n, mu != nullptr, which);
    if (back_need(p, L.n, mu != nullptr, which) > ws_avail)
        return fail(SPECT_EINVAL, "workspace too small for a %d-angle back-projection launch", L.n);
    const float *tau = nullptr;
    size_t off = 0;
    const size_t tb = tau_bytes(p, t, L.n, mu != nullptr);
    if (tb) {
        off += tb;
        if (tau_given) {
            tau = tau_given;
        } else {
            launch_tau(p, L, t, mu, reinterpret_cast<float *>(ws), vec, st);
            tau = reinterpret_cast<const float *>(ws);
        }
    }
    float *z = reinterpret_cast<float *>(ws + off);
    BackRotArgs b;
    b.g = p->g;
    b.L = L;
    b.y = y;
    b.y_compact = y_compact;
    b.ones = ones;
    b.mu = mu;
    b.tau = tau;
    b.z = z;
    b.nslab = t.nslab;
    b.nchunk = t.nchunk;
    b.dchunk = t.dchunk;
    b.vec = vec;
    BackFn bk = back_kernel(mu != nullptr, p->kmc, vec);
    allow_smem(reinterpret_cast<const void *>(bk), back_smem(p));
    {
        ProfScope ps(K_BACK_ROT, st);
        hipLaunchKernelGGL(bk, dim3(t.nslab, t.nchunk, L.n), dim3(block_threads(p->N)), back_smem(p), st, b);
    }
    GatherArgs gg;
    gg.g = p->g;
    gg.L = L;
    gg.z = z;
    gg.nslab = t.nslab;
    gg.mode = mode;
    gg.out = out;
    gg.sens = sens;
    const int tiles = (p->N + GT - 1) / GT;
    {
        ProfScope ps(K_GATHER, st);
        hipLaunchKernelGGL(back_gather, dim3(tiles * tiles, t.nslab), dim3(256), 0, st, gg);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "back projection launch");
    return SPECT_OK;
}

int clear(float *p, size_t n, hipStream_t st)
{
    ProfScope ps(K_FILL, st);
    hipLaunchKernelGGL(fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPECT_OK : hip_fail(e, "clear launch");
}

bool want_vec(const spect_plan *p, std::initializer_list<const void *> ptrs)
{
    if (p->Nz % 4) return false;
    for (const void *q : ptrs)
        if (q && !aligned16(q)) return false;
    return true;
}

}  // namespace

// ============================================================== C ABI ====

extern "C" {

const char *spect_last_error(void) { return g_err.c_str(); }

int spect_profile_enable(int enable)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = enable != 0;
    return ok();
}

int spect_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto &r : g_prof) {
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(SPECT_EHIP, "waiting for a timing event failed");
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof.clear();
    return ok();
}

int spect_profile_query(const char *kernel, int32_t *launches, double *total_ms)
{
    if (!kernel || !launches || !total_ms) return fail(SPECT_EINVAL, "NULL argument");
    int id = -1;
    for (int k = 0; k < K_COUNT; ++k)
        if (std::strcmp(kernel, kKernelNames[k]) == 0) id = k;
    if (id < 0) return fail(SPECT_EINVAL, "unknown kernel name '%s'", kernel);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    int n = 0;
    double ms = 0;
    for (auto &r : g_prof) {
        if (r.kernel != id) continue;
        float e = 0;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&e, r.a, r.b) != hipSuccess)
            return fail(SPECT_EHIP, "reading a timing event failed");
        ++n;
        ms += e;
    }
    *launches = n;
    *total_ms = ms;
    return ok();
}

int spect_plan_create(const spect_geometry *geom, spect_plan **out)
{
    if (!out) return fail(SPECT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!geom) return fail(SPECT_EINVAL, "geometry is NULL");
    const spect_geometry &g = *geom;
    if (g.flags != 0) return fail(SPECT_EINVAL, "flags must be 0");
    if (g.n < 1 || g.nz < 1 || g.n_angles < 1)
        return fail(SPECT_EINVAL, "sizes must be >= 1 (n=%d nz=%d n_angles=%d)", g.n, g.nz, g.n_angles);
    if (!(std::isfinite(g.voxel_cm) && g.voxel_cm > 0)) return fail(SPECT_EINVAL, "voxel_cm must be > 0");
    if (!(std::isfinite(g.psf_a) && std::isfinite(g.psf_b) && g.psf_a >= 0 && g.psf_b >= 0))
        return fail(SPECT_EINVAL, "psf_a and psf_b must be finite and >= 0");
    if (!std::isfinite(g.psf_nsigma)) return fail(SPECT_EINVAL, "psf_nsigma must be finite");
    if (g.n > SPECT_MAX_N) return fail(SPECT_EUNSUPPORTED, "n = %d exceeds %d", g.n, SPECT_MAX_N);
    const double vol = (double)g.n * g.n * g.nz, prj = (double)g.n_angles * g.n * g.nz;
    if (vol >= 2147483647.0 || prj >= 2147483647.0)
        return fail(SPECT_EUNSUPPORTED, "object or projection element count exceeds 2^31");
    std::vector<double> ang(g.n_angles), rad(g.n_angles);
    for (int i = 0; i < g.n_angles; ++i) {
        ang[i] = g.angles_deg ? g.angles_deg[i] : i * 360.0 / g.n_angles;
        rad[i] = g.radius_cm ? g.radius_cm[i] : 0.5 * g.n * g.voxel_cm;
        if (!std::isfinite(ang[i])) return fail(SPECT_EINVAL, "angles_deg[%d] is not finite", i);
        if (!(std::isfinite(rad[i]) && rad[i] >= 0)) return fail(SPECT_EINVAL, "radius_cm[%d] must be >= 0", i);
    }
    int kmax = 0;
    for (int i = 0; i < g.n_angles; ++i)
        for (int ip = 0; ip < g.n; ++ip) kmax = std::max(kmax, depth_kernel(g, rad[i], ip, nullptr));
    if (kmax > SPECT_MAX_K)
        return fail(SPECT_EUNSUPPORTED, "collimator blur radius %d pixels exceeds %d", kmax, SPECT_MAX_K);

    spect_plan *p = new spect_plan();
    p->N = g.n;
    p->Nz = g.nz;
    p->A = g.n_angles;
    p->voxel_cm = g.voxel_cm;
    p->kmax = kmax;
    p->kmc = ((kmax + 3) / 4) * 4;
    p->TS = p->kmc + 1;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return fail(SPECT_EHIP, "no HIP device");
    }
    const int N = g.n, A = g.n_angles;
    std::vector<float2> cs(A), xy0((size_t)A * N);
    std::vector<int> kd((size_t)A * N);
    std::vector<float> taps((size_t)A * N * p->TS, 0.f);
    const double c = 0.5 * (N - 1);
    std::vector<double> t;
    for (int i = 0; i < A; ++i) {
        double cc, ss;
        trig_deg(ang[i], &cc, &ss);
        cs[i] = make_float2((float)cc, (float)ss);
        for (int jp = 0; jp < N; ++jp)
            xy0[(size_t)i * N + jp] = make_float2((float)(c - cc * c - ss * (jp - c)),
                                                  (float)(c - ss * c + cc * (jp - c)));
        for (int ip = 0; ip < N; ++ip) {
            const int K = depth_kernel(g, rad[i], ip, &t);
            kd[(size_t)i * N + ip] = K;
            for (int m = 0; m <= K; ++m) taps[((size_t)i * N + ip) * p->TS + m] = (float)t[m];
        }
    }
    const size_t b_cs = align256(sizeof(float2) * A), b_xy = align256(sizeof(float2) * (size_t)A * N);
    const size_t b_kd = align256(sizeof(int) * (size_t)A * N), b_tp = align256(sizeof(float) * taps.size());
    hipError_t e = hipMalloc(&p->dmem, b_cs + b_xy + b_kd + b_tp);
    if (e != hipSuccess) {
        delete p;
        return fail(SPECT_ENOMEM, "hipMalloc of plan tables failed: %s", hipGetErrorString(e));
    }
    char *base = static_cast<char *>(p->dmem);
    e = hipMemcpy(base, cs.data(), sizeof(float2) * A, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + b_cs, xy0.data(), sizeof(float2) * xy0.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + b_cs + b_xy, kd.data(), sizeof(int) * kd.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(base + b_cs + b_xy + b_kd, taps.data(), sizeof(float) * taps.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p->dmem);
        delete p;
        return hip_fail(e, "upload of plan tables");
    }
    p->g.cs = reinterpret_cast<const float2 *>(base);
    p->g.xy0 = reinterpret_cast<const float2 *>(base + b_cs);
    p->g.kdep = reinterpret_cast<const int *>(base + b_cs + b_xy);
    p->g.taps = reinterpret_cast<const float *>(base + b_cs + b_xy + b_kd);
    p->g.N = N;
    p->g.Nz = g.nz;
    p->g.A = A;
    p->g.TS = p->TS;
    p->g.tau_scale = (float)(g.voxel_cm / std::log(2.0));
    // resident workgroups per device for the chunk tuning
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || cus < 1)
        cus = 256;
    for (int mu = 0; mu < 2; ++mu) {
        int nb = 0;
        const void *fk = reinterpret_cast<const void *>(fwd_kernel(mu != 0, p->kmc, true));
        allow_smem(fk, fwd_smem(p));
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fk, block_threads(N), fwd_smem(p)) != hipSuccess)
            nb = 1;
        p->fwd_slots[mu] = std::max(1, nb) * cus;
        const void *bk = reinterpret_cast<const void *>(back_kernel(mu != 0, p->kmc, true));
        allow_smem(bk, back_smem(p));
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bk, block_threads(N), back_smem(p)) != hipSuccess)
            nb = 1;
        p->back_slots[mu] = std::max(1, nb) * cus;
    }
    (void)hipGetLastError();
    *out = p;
    return ok();
}

int spect_plan_destroy(spect_plan *plan)
{
    if (!plan) return ok();
    if (plan->dmem) (void)hipFree(plan->dmem);
    delete plan;
    return ok();
}

int spect_workspace_size(const spect_plan *plan, int op, int32_t n_idx, int with_mu, size_t *bytes)
{
    if (!plan) return fail(SPECT_EINVAL, "plan is NULL");
    if (!bytes) return fail(SPECT_EINVAL, "bytes is NULL");
    if (n_idx < 1) return fail(SPECT_EINVAL, "n_idx must be >= 1");
    const bool mu = with_mu != 0;
    switch (op) {
    case SPECT_OP_FWD: *bytes = fwd_ws(plan, n_idx, mu); break;
    case SPECT_OP_BACK:
    case SPECT_OP_SENS: *bytes = back_ws(plan, n_idx, mu); break;
    case SPECT_OP_OSEM:
        if (n_idx > plan->A) return fail(SPECT_EINVAL, "n_subsets %d exceeds n_angles %d", n_idx, plan->A);
        *bytes = osem_ws(plan, n_idx, mu);
        break;
    default: return fail(SPECT_EINVAL, "unknown op %d", op);
    }
    return ok();
}

int spect_fwd(const spect_plan *plan, const float *f, const float *mu, float *proj,
              const int32_t *angle_idx, int32_t n_idx, void *ws, size_t ws_bytes, void *stream)
{
    int st;
    if ((st = check_plan(plan))) return st;
    if ((st = check_ptr(f, "f", false)) || (st = check_ptr(mu, "mu", true)) ||
        (st = check_ptr(proj, "proj", false)))
        return st;
    std::vector<int> list;
    if ((st = make_list(plan, angle_idx, n_idx, &list))) return st;
    if (list.empty()) return ok();
    if ((st = check_ws(ws, ws_bytes, fwd_ws(plan, (int)list.size(), mu != nullptr)))) return st;
    const bool vec = want_vec(plan, {f, mu});
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (size_t b = 0; b < list.size(); b += MAXL) {
        const int n = (int)std::min<size_t>(MAXL, list.size() - b);
        const AngleList L = to_list(list.data() + b, n);
        if ((st = run_forward(plan, f, mu, L, static_cast<char *>(ws), ws_bytes, nullptr, 0, proj, nullptr, nullptr,
                              nullptr, vec, T_FWD, s)))
            return st;
    }
    return ok();
}

int spect_back(const spect_plan *plan, const float *proj, const float *mu, float *f_out,
               const int32_t *angle_idx, int32_t n_idx, int accumulate, void *ws, size_t ws_bytes,
               void *stream)
{
    int st;
    if ((st = check_plan(plan))) return st;
    if ((st = check_ptr(proj, "proj", false)) || (st = check_ptr(mu, "mu", true)) ||
        (st = check_ptr(f_out, "f_out", false)))
        return st;
    std::vector<int> list;
    if ((st = make_list(plan, angle_idx, n_idx, &list))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (list.empty()) {
        if (accumulate) return ok();
        return (st = clear(f_out, (size_t)plan->N * plan->N * plan->Nz, s)) ? st : ok();
    }
    if ((st = check_ws(ws, ws_bytes, back_ws(plan, (int)list.size(), mu != nullptr)))) return st;
    const bool vec = want_vec(plan, {mu});
    const int G = back_group(plan, (int)list.size());
    for (size_t b = 0; b < list.size(); b += G) {
        const int n = (int)std::min<size_t>(G, list.size() - b);
        const AngleList L = to_list(list.data() + b, n);
        const int mode = (b == 0 && !accumulate) ? 0 : 1;
        if ((st = run_back(plan, proj, 0, 0, mu, L, static_cast<char *>(ws), ws_bytes, nullptr, mode, f_out, nullptr, vec,
                            T_BACK, s)))
            return st;
    }
    return ok();
}

int spect_sensitivity(const spect_plan *plan, const float *mu, float *sens, const int32_t *angle_idx,
                      int32_t n_idx, void *ws, size_t ws_bytes, void *stream)
{
    int st;
    if ((st = check_plan(plan))) return st;
    if ((st = check_ptr(mu, "mu", true)) || (st = check_ptr(sens, "sens", false))) return st;
    std::vector<int> list;
    if ((st = make_list(plan, angle_idx, n_idx, &list))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (list.empty()) {
        return (st = clear(sens, (size_t)plan->N * plan->N * plan->Nz, s)) ? st : ok();
    }
    if ((st = check_ws(ws, ws_bytes, back_ws(plan, (int)list.size(), mu != nullptr)))) return st;
    const bool vec = want_vec(plan, {mu});
    const int G = back_group(plan, (int)list.size());
    for (size_t b = 0; b < list.size(); b += G) {
        const int n = (int)std::min<size_t>(G, list.size() - b);
        const AngleList L = to_list(list.data() + b, n);
        if ((st = run_back(plan, nullptr, 0, 1, mu, L, static_cast<char *>(ws), ws_bytes, nullptr, b == 0 ? 0 : 1, sens,
                           nullptr, vec, T_BACK, s)))
            return st;
    }
    return ok();
}

int osem_subset_step(const spect_plan *plan, float *f, const float *mu, const float *g, const float *s_add,
                     const float *sens_m, int32_t m, int32_t n_subsets, void *ws, size_t ws_bytes, void *stream)
{
    int st;
    if ((st = check_plan(plan))) return st;
    if ((st = check_ptr(f, "f", false)) || (st = check_ptr(mu, "mu", true)) || (st = check_ptr(g, "g", false)) ||
        (st = check_ptr(s_add, "s_add", true)) || (st = check_ptr(sens_m, "sens_m", false)))
        return st;
    if (n_subsets < 1 || n_subsets > plan->A)
        return fail(SPECT_EINVAL, "n_subsets = %d outside [1, %d]", n_subsets, plan->A);
    if (m < 0 || m >= n_subsets) return fail(SPECT_EINVAL, "m = %d outside [0, %d)", m, n_subsets);
    const int nl_max = (plan->A + n_subsets - 1) / n_subsets;
    if (nl_max > MAXL) return fail(SPECT_EUNSUPPORTED, "subsets of more than %d angles", MAXL);
    if ((st = check_ws(ws, ws_bytes, osem_ws(plan, n_subsets, mu != nullptr)))) return st;
    std::vector<int> list;
    for (int n = m; n < plan->A; n += n_subsets) list.push_back(n);
    const AngleList L = to_list(list.data(), (int)list.size());
    const bool vec = want_vec(plan, {f, mu});
    hipStream_t s = static_cast<hipStream_t>(stream);
    // workspace [q][tau][partial | z] (see osem_ws)
    char *w = static_cast<char *>(ws);
    float *q = reinterpret_cast<float *>(w);
    const size_t qb = osem_q_bytes(plan, n_subsets);
    char *rest = w + qb;
    const size_t avail = ws_bytes - qb;
    if ((st = run_forward(plan, f, mu, L, rest, avail, nullptr, 1, nullptr, g, s_add, q, vec, T_BOTH, s)))
        return st;
    // same list, same tuning: the attenuation offsets at the start of rest are reused
    if ((st = run_back(plan, q, 1, 0, mu, L, rest, avail, reinterpret_cast<const float *>(rest), 2, f, sens_m,
                       vec, T_BOTH, s)))
        return st;
    return ok();
}

}  // extern "C"
