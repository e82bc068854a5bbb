// spect_device.h - device code of the SPECT projector library (gfx950).
//
// The operator is the parallel-hole SPECT system matrix of the paper (Section
// 2.1.1, Eq. 1): per angle, rotate the object (bilinear, per axial slice),
// attenuate along the rotated depth axis, blur every depth plane with its own
// separable Gaussian collimator-detector kernel, and sum over depth.  The
// transpose runs the same steps backwards.  include/spect.h states the
// discretisation and the array layouts.
//
// Parallel decomposition (one launch covers a list of angles):
//   workgroup = (angle, axial slab of 16 slices, depth chunk); in the forward
//   four lanes share detector bin j', lane q owning axial rows 4q..4q+3 of
//   the slab, and walk the depth axis of their chunk from the detector side.
//   Per depth a lane samples the object (four bilinear corners, each a
//   contiguous z-run), applies the attenuation factors, blurs along the bin
//   axis through LDS (the neighbouring bins belong to other lanes), and
//   scatters the axial blur of its rows into registers that hold the slab's
//   partial projection rows.  A reduction kernel adds the partial rows of
//   neighbouring slabs and of the depth chunks.
//   Depth chunks raise parallelism for small angle subsets; their
//   attenuation offsets come from a pre-pass that walks each ray once.
// Attenuation modes (template parameter ATT): none; sample mu and form
// exp(-tau) in the kernel; the same and also store the factors in a table
// laid out like the rotated-frame volume, [angle][slab][i'][j'][16]; read
// the factors from that table.  A whole reconstruction writes the table once
// per subset (its sensitivity pass) and every later pass streams it.
// Back projection:
//   back_rot  : same workgroups; per depth, axial blur of the projection in
//               registers, bin-axis blur through LDS, times exp(-tau); writes
//               the rotated-frame volume Z of each angle to the workspace;
//   back_gather: thread per (x, y, slab) gathers from the <= 3x3 rotated
//               samples whose bilinear footprint covers the voxel, with the
//               forward's own FP32 weights, so the pair is an exact transpose
//               up to summation order; the OSEM update is fused here.
// No MFMA: nothing on this path is a dense contraction.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace spectk {

constexpr int SLAB = 16;   // axial rows per workgroup
constexpr int ROWS = 8;    // axial rows per thread
constexpr int MAXL = 128;  // angles per launch

enum AttMode { ATT_NONE = 0, ATT_SAMPLE = 1, ATT_WRITE = 2, ATT_READ = 3 };

// Work-list of a batched launch: task = (reconstruction r, x, y, z), where
// (x, y, z) are the block coordinates the single-reconstruction launch would
// use; args[r] are reconstruction r's launch arguments.  A persistent batched
// kernel (PERSIST) has workgroup b take tasks b, b + gridDim.x, ...; the
// other form runs one task per workgroup (grid = task count), which keeps
// the register count of the single-reconstruction kernel.
struct Task {
    int r, x, y, z;
};

template <class Args>
struct BatchList {
    const Args *args;
    const Task *tasks;
    int ntasks;
};

// The argument and task arrays of a batched launch are written by the host
// before the launch and only read by it, so the kernels read them through
// the constant address space: uniform fields then come in with scalar loads.
template <class T>
using ConstMem = const __attribute__((address_space(4))) T;

template <class T>
__device__ __forceinline__ ConstMem<T> *as_const(const T *p)
{
    return (ConstMem<T> *)p;
}

// Element offset of the 16 axial rows of (angle al, slab, depth i', bin j')
// in a rotated-frame brick volume [L][nslab][N][N][16] (the back-projection
// workspace and the attenuation table share this layout).
__device__ __forceinline__ size_t brick_offset(int al, int nslab, int slab, int N, int ip, int jp)
{
    return ((((size_t)al * nslab + slab) * N + ip) * N + jp) * SLAB;
}

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
    const float *ctaps; // [A][N][TS] their running sums C[m] = g[0] + ... + g[m]
    const int *cbnd;    // [2][cap][A][cap + 1] depth-chunk boundaries (see chunk_range)
    int N, Nz, A, TS;
    int cap;            // largest depth-chunk count
    float tau_scale;    // dx * log2(e): exp(-tau) = exp2(-tau_scale * (sum mu))
};

// Depths of chunk `chunk` of a launch split into nchunk chunks, for angle
// ang: ihi down to ilo (chunk 0 touches the detector).  The boundaries come
// from the plan: set 0 gives the chunks equal depth counts (the forward,
// whose time hardly depends on the blur radius, and the passes that share
// attenuation offsets), set 1 balances the blur work of the rotated-frame
// pass (about 10 + K per depth).
// A value every lane of the wave holds (workgroup coordinates, plan table
// entries they select), moved to a scalar register: loops and radius
// dispatch that depend on it then run as scalar branches, and the loads it
// addresses (radii, taps) as scalar loads, instead of being treated as
// per-lane values.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <class G>
__device__ __forceinline__ void chunk_range(const G &g, int set, int nchunk, int ang, int chunk, int &ihi, int &ilo)
{
    ConstMem<int> *cb = as_const(g.cbnd + (((size_t)set * g.cap + nchunk - 1) * g.A + ang) * (g.cap + 1));
    ihi = uniform(cb[chunk] - 1);
    ilo = uniform(cb[chunk + 1]);
}

// --------------------------------------------------------------- helpers --

struct Corners {
    uint32_t b00, b10, b01, b11;  // byte offsets of the z-runs of (x0,y0), (x0+1,y0), (x0,y0+1), (x0+1,y0+1)
    float w00, w10, w01, w11;     // bilinear weights, 0 for corners outside the grid
};

// Bilinear footprint of point (X, Y) in an N x N slice of z-runs.
__device__ __forceinline__ Corners corners(float X, float Y, int N, uint32_t rowb)
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
    // (xb, yb) differ from (xa, ya) by 0 or 1 after clamping
    c.b00 = __umul24(__umul24((uint32_t)xa, (uint32_t)N) + (uint32_t)ya, rowb);
    const uint32_t dx = (xb != xa) ? __umul24((uint32_t)N, rowb) : 0u;
    const uint32_t dy = (yb != ya) ? rowb : 0u;
    c.b10 = c.b00 + dx;
    c.b01 = c.b00 + dy;
    c.b11 = c.b10 + dy;
    return c;
}

template <typename T>
__device__ __forceinline__ const T &at_byte(const float *base, uint32_t off)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off);
}

// Third descriptor word of a raw (unswizzled, unformatted) buffer resource on
// gfx9-family GPUs.
constexpr int kBufferDword3 = 0x00020000;
// A byte offset past the end of every object volume a plan accepts (below
// 2^29 voxels, 2 GiB): a raw buffer load there returns zeros.
constexpr int kVolPastEnd = (int)0x80000000u;
// Cache-policy bits of a buffer load: non-temporal (the line is not kept).
constexpr int kNonTemporal = 2;

// Bilinear corners of one sample: weights and byte offsets of the corners'
// z-runs (plus the lane's row offset dk), for raw buffer loads over the
// volume.  Such a load returns zeros past the end of the volume, and at
// "negative" offsets, which are above 2^31 as unsigned; so a corner with x
// outside [0, N) needs no test (its offset falls outside the volume for every
// sample of a rotated grid, |X - c| <= sqrt(2) c), while a corner with y
// outside [0, N) would alias a neighbouring column and gets the
// past-the-end offset.  Corners outside the grid thus read zeros and keep
// their weights.
struct FCorner {
    float w[4];
    int o[4];
};

__device__ __forceinline__ FCorner fcorners(float X, float Y, int N, uint32_t rowb, uint32_t colb, uint32_t dk)
{
    const float xf = floorf(X), yf = floorf(Y);
    const int x0 = (int)xf, y0 = (int)yf;
    const float fx = X - xf, fy = Y - yf;
    const float gx = 1.f - fx, gy = 1.f - fy;
    FCorner r;
    r.w[0] = gx * gy;
    r.w[1] = fx * gy;
    r.w[2] = gx * fy;
    r.w[3] = fx * fy;
    const uint32_t base = (uint32_t)(x0 * N + y0) * rowb + dk;
    const bool vy0 = (unsigned)y0 < (unsigned)N, vy1 = (unsigned)(y0 + 1) < (unsigned)N;
    r.o[0] = vy0 ? (int)base : kVolPastEnd;
    r.o[1] = vy0 ? (int)(base + colb) : kVolPastEnd;
    r.o[2] = vy1 ? (int)(base + rowb) : kVolPastEnd;
    r.o[3] = vy1 ? (int)(base + colb + rowb) : kVolPastEnd;
    return r;
}

// The lane's rows kb .. kb+7 of the four corners: two 16-byte loads per
// corner (vector path, row offset in the corner offsets; rows past Nz read
// the next column or zeros) or one load per row at the clamped offsets dks.
template <bool VEC>
__device__ __forceinline__ void fload8(__amdgpu_buffer_rsrc_t rs, const FCorner &c, const int (&dks)[8],
                                       float4 (&v)[4][2])
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if constexpr (VEC) {
            v[j][0] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, c.o[j], 0, 0));
            v[j][1] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(
                                                     rs, (int)((uint32_t)c.o[j] + 16u), 0, 0));
        } else {
            float t[8];
#pragma unroll
            for (int r = 0; r < 8; ++r)
                t[r] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                     rs, (int)((uint32_t)c.o[j] + (uint32_t)dks[r]), 0, 0));
            v[j][0] = make_float4(t[0], t[1], t[2], t[3]);
            v[j][1] = make_float4(t[4], t[5], t[6], t[7]);
        }
    }
}

// Bilinear combination of 8 rows; rows at or past Nz give 0.
__device__ __forceinline__ void fcombine8(const FCorner &c, const float4 (&v)[4][2], int kb, int Nz, float (&m)[8])
{
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        m[4 * hh + 0] = fmaf(c.w[3], v[3][hh].x, fmaf(c.w[2], v[2][hh].x, fmaf(c.w[1], v[1][hh].x, c.w[0] * v[0][hh].x)));
        m[4 * hh + 1] = fmaf(c.w[3], v[3][hh].y, fmaf(c.w[2], v[2][hh].y, fmaf(c.w[1], v[1][hh].y, c.w[0] * v[0][hh].y)));
        m[4 * hh + 2] = fmaf(c.w[3], v[3][hh].z, fmaf(c.w[2], v[2][hh].z, fmaf(c.w[1], v[1][hh].z, c.w[0] * v[0][hh].z)));
        m[4 * hh + 3] = fmaf(c.w[3], v[3][hh].w, fmaf(c.w[2], v[2][hh].w, fmaf(c.w[1], v[1][hh].w, c.w[0] * v[0][hh].w)));
    }
#pragma unroll
    for (int r = 0; r < 8; ++r)
        if (kb + r >= Nz) m[r] = 0.f;
}


// The attenuation table is streamed: a pass reads (or the sensitivity pass
// writes) every entry once, and the next pass to touch it comes after other
// kernels.  The forward's reads and the sensitivity pass's writes are
// non-temporal, so they do not push the reused corner lines of the activity
// volume out of the caches (measured: forward 103 -> 102 us, sensitivity
// pass 78 -> 72-77 us, the gather that follows the passes 45 -> 42-43 us);
// in the rotated-frame pass non-temporal reads were slower (64 -> 71 us)
// and it keeps ordinary loads.
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef float f2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float4 stream_f4(const float *base, uint32_t off)
{
    const f4_t v = __builtin_nontemporal_load(
        reinterpret_cast<const f4_t *>(reinterpret_cast<const char *>(base) + off));
    return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ void stream_store_f4(float *p, float a, float b, float c, float d)
{
    __builtin_nontemporal_store(f4_t{a, b, c, d}, reinterpret_cast<f4_t *>(p));
}

__device__ __forceinline__ void stream_store_f2(float *p, float a, float b)
{
    __builtin_nontemporal_store(f2_t{a, b}, reinterpret_cast<f2_t *>(p));
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

// Binary dispatch of a run-time blur radius k in [LO, HI] to f.template
// go<k>(): about log2(HI - LO + 1) scalar branches per call.
template <int LO, int HI>
struct KSwitch {
    template <class F>
    static __device__ __forceinline__ void run(int k, F &f)
    {
        if constexpr (LO == HI) {
            f.template go<LO>();
        } else {
            constexpr int MID = (LO + HI) / 2;
            if (k <= MID)
                KSwitch<LO, MID>::run(k, f);
            else
                KSwitch<MID + 1, HI>::run(k, f);
        }
    }
};

// Bin-axis blur of the thread's 8 rows with a compile-time radius:
// U = g0 W(j') + sum_m g_m (W(j'-m) + W(j'+m)); i0/i1 index the thread's two
// float4 of row j' in the row buffer (row stride 2 float4), so every read
// uses an immediate offset.
template <int K, int G>
__device__ __forceinline__ void blur_bins(const float4 *__restrict__ wb, int i0, int i1, const float (&gk)[G],
                                          const float (&self)[ROWS], float (&u)[ROWS])
{
    static_assert(K < G, "taps past the radius");
#pragma unroll
    for (int r = 0; r < ROWS; ++r) u[r] = gk[0] * self[r];
#pragma unroll
    for (int m = 1; m <= K; ++m) {
        const float4 a = wb[i0 - 2 * m], b = wb[i0 + 2 * m];
        const float4 c = wb[i1 - 2 * m], d = wb[i1 + 2 * m];
        u[0] = fmaf(gk[m], a.x + b.x, u[0]);
        u[1] = fmaf(gk[m], a.y + b.y, u[1]);
        u[2] = fmaf(gk[m], a.z + b.z, u[2]);
        u[3] = fmaf(gk[m], a.w + b.w, u[3]);
        u[4] = fmaf(gk[m], c.x + d.x, u[4]);
        u[5] = fmaf(gk[m], c.y + d.y, u[5]);
        u[6] = fmaf(gk[m], c.z + d.z, u[6]);
        u[7] = fmaf(gk[m], c.w + d.w, u[7]);
    }
}

// The plan's tables (radii, taps, tap sums) never change once built, so the
// kernels read them through the constant address space: uniform reads are
// then scalar loads even in loops that also store to global memory.
template <int KMC>
__device__ __forceinline__ void load_taps_all(const float *__restrict__ g, float (&gz)[KMC + 1])
{
    ConstMem<float> *cg = as_const(g);
#pragma unroll
    for (int m = 0; m <= KMC; ++m) gz[m] = cg[m];
}

// Adjoint, bin-axis blur of the row buffer (taps gz in registers).
template <int KMC>
struct BackBlur {
    const float (&v)[ROWS];
    float (&u)[ROWS];
    const float4 *wb;
    int i0, i1;
    const float (&gz)[KMC + 1];
    template <int K>
    __device__ __forceinline__ void go()
    {
        blur_bins<K>(wb, i0, i1, gz, v, u);
    }
};

// Axial blur as a gather from a column of LDS values: col[base - K + t] is
// axial row kb - K + t; out[s] = sum_l g(|l|) win[s + K - l] (taps gz in
// registers).
template <int KMC>
struct ZGather {
    const float *col;
    int base;
    const float (&gz)[KMC + 1];
    float (&out)[ROWS];
    template <int K>
    __device__ __forceinline__ void go()
    {
        const float *win = col + base - K;
        float v[ROWS + 2 * K];
#pragma unroll
        for (int t = 0; t < ROWS + 2 * K; ++t) v[t] = win[t];
#pragma unroll
        for (int s = 0; s < ROWS; ++s) {
            float a = gz[0] * v[s + K];
#pragma unroll
            for (int l = 1; l <= K; ++l) a = fmaf(gz[l], v[s + K - l] + v[s + K + l], a);
            out[s] = a;
        }
    }
};

// ----------------------------------------------------------- attenuation --

struct TauArgs {
    DevGeom g;
    AngleList L;
    const float *mu;
    float *tau;      // [L][nchunk][N][Nz]: sum of mu samples over the depths of chunk c
    int nchunk, cbset;
    int vec;
};

// One thread per (angle, chunk, bin, 8 axial rows): sum the attenuation
// samples of the chunk's depths (chunk_range; chunk 0 touches the detector).
// A chunk's starting attenuation is the sum of the partial sums of the
// chunks nearer the detector (the last chunk's own sum is never needed).
template <bool VEC>
__global__ __launch_bounds__(256) void tau_prepass(TauArgs a)
{
    const int N = a.g.N, Nz = a.g.Nz;
    const int ngrp = (Nz + ROWS - 1) / ROWS;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * ngrp) return;
    const int ch = blockIdx.y, al = blockIdx.z;
    const int ang = uniform(a.L.idx[al]);
    const int jp = t / ngrp, kb = (t % ngrp) * ROWS;
    const float2 cs = a.g.cs[ang];
    const float2 o = a.g.xy0[(size_t)ang * N + jp];
    float S[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) S[r] = 0.f;
    int ihi, ilo;
    chunk_range(a.g, a.cbset, a.nchunk, ang, ch, ihi, ilo);
    const uint32_t rowb = 4u * (uint32_t)Nz, colb = rowb * (uint32_t)N;
    int dks[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) dks[r] = 4 * min(kb + r, Nz - 1);
    const __amdgpu_buffer_rsrc_t rm = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(a.mu), (short)0,
                                                                        (int)(colb * (uint32_t)N), kBufferDword3);
#pragma unroll 2
    for (int ip = ihi; ip >= ilo; --ip) {
        const FCorner c = fcorners(fmaf((float)ip, cs.x, o.x), fmaf((float)ip, cs.y, o.y), N, rowb, colb,
                                   VEC ? 4u * (uint32_t)kb : 0u);
        float4 v[4][2];
        fload8<VEC>(rm, c, dks, v);
        float m[ROWS];
        fcombine8(c, v, kb, Nz, m);
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
//
// Forward lanes: FQ = 4 lanes per detector bin, lane q owning the FR = 4
// axial rows 4q .. 4q+3 of the 16-row slab, so that a bilinear corner is one
// 16-byte load per lane and the four lanes of a bin read its whole 64-byte
// z-run.  Per depth a lane samples its rows (four corner loads), multiplies
// by the attenuation factors (read one depth ahead from the table, or
// formed from mu samples and a running sum), writes them to the row buffer,
// and after one workgroup barrier blurs along the bins from LDS and scatters
// the axial blur into its partial rows.

constexpr int FQ = 4;
constexpr int FR = SLAB / FQ;

struct FwdArgs {
    DevGeom g;
    AngleList L;
    const float *f;
    const float *mu;
    const float *tau;   // chunk offsets or nullptr when nchunk == 1
    const float *att;   // ATT_READ: attenuation table [L][nslab][N][N][16]
    float *part;        // [L][nslab][nchunk][N][SLAB + 2 KMC]
    int nslab, nchunk, cbset;
    int vec;
    int zs;             // column stride of f in floats (0: Nz); mu, when sampled, is never padded
    int cus;            // compute units (0: chunks in grid order; see fwd_main)
};

// LDS row buffers of the forward: [buf][row j' + KMC][q] float4, two buffers
// of nrows = N + 2 KMC rows (KMC zero rows on each side).
__device__ __forceinline__ int fwb_index(int buf, int row, int q, int nrows) { return (buf * nrows + row) * FQ + q; }

// Value of lane `src` of this lane's quad (all four lanes active).
template <int SRC>
__device__ __forceinline__ int quad_bcast(int v)
{
    return __builtin_amdgcn_mov_dpp(v, SRC * 0x55, 0xF, 0xF, false);
}

template <int SRC>
__device__ __forceinline__ float quad_bcast(float v)
{
    return __int_as_float(quad_bcast<SRC>(__float_as_int(v)));
}

// Workgroup barrier that orders LDS accesses only: global loads in flight
// stay in flight across it (__syncthreads() would also wait for them).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The lane's 4 rows of each corner.  Vector path: one 16-byte load per
// corner (the row offset is in the corner offsets); scalar path: one load per
// row at the clamped row offsets dks[r].
template <bool VEC>
__device__ __forceinline__ void fload(__amdgpu_buffer_rsrc_t rs, const FCorner &c, const int (&dks)[FR],
                                      float4 (&v)[4])
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if constexpr (VEC) {
            v[j] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, c.o[j], 0, 0));
        } else {
            float t[FR];
#pragma unroll
            for (int r = 0; r < FR; ++r)
                t[r] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                     rs, (int)((uint32_t)c.o[j] + (uint32_t)dks[r]), 0, 0));
            v[j] = make_float4(t[0], t[1], t[2], t[3]);
        }
    }
}

// Bilinear combination of the corners' rows.
__device__ __forceinline__ float4 fcombine(const FCorner &c, const float4 (&v)[4])
{
    float4 r;
    r.x = fmaf(c.w[3], v[3].x, fmaf(c.w[2], v[2].x, fmaf(c.w[1], v[1].x, c.w[0] * v[0].x)));
    r.y = fmaf(c.w[3], v[3].y, fmaf(c.w[2], v[2].y, fmaf(c.w[1], v[1].y, c.w[0] * v[0].y)));
    r.z = fmaf(c.w[3], v[3].z, fmaf(c.w[2], v[2].z, fmaf(c.w[1], v[1].z, c.w[0] * v[0].z)));
    r.w = fmaf(c.w[3], v[3].w, fmaf(c.w[2], v[2].w, fmaf(c.w[1], v[1].w, c.w[0] * v[0].w)));
    return r;
}

// Bin-axis blur of the lane's rows with a compile-time radius K (KSwitch
// picks the code path per depth; the taps gz are already in registers), so
// that every LDS read of the depth can be issued before the arithmetic:
// U = g0 W(j') + sum_m g_m (W(j'-m) + W(j'+m)), i0 the lane's float4 of row
// j' (bin stride FQ float4).
template <int KMC>
struct FBinBlur {
    const float4 *wb;
    int i0;
    const float (&gz)[KMC + 1];
    const float4 &self;
    float (&u)[FR];
    template <int K>
    __device__ __forceinline__ void go()
    {
        u[0] = gz[0] * self.x;
        u[1] = gz[0] * self.y;
        u[2] = gz[0] * self.z;
        u[3] = gz[0] * self.w;
#pragma unroll
        for (int m = 1; m <= K; ++m) {
            const float4 a = wb[i0 - FQ * m], b = wb[i0 + FQ * m];
            u[0] = fmaf(gz[m], a.x + b.x, u[0]);
            u[1] = fmaf(gz[m], a.y + b.y, u[1]);
            u[2] = fmaf(gz[m], a.z + b.z, u[2]);
            u[3] = fmaf(gz[m], a.w + b.w, u[3]);
        }
    }
};

// Axial blur as a scatter, with the depth's radius K <= KMC at run time:
// input row s (0..3) adds g(|l|) U[s] to output row s + l, |l| <= K;
// acc[t] holds output row kb - KMC + t.  The guards are scalar branches (K
// is uniform) and every accumulator is updated in place along one chain of
// guarded blocks, with no code path per radius.
template <int KMC>
__device__ __forceinline__ void fzscatter(float (&acc)[FR + 2 * KMC], const float (&u)[FR], const float (&gz)[KMC + 1],
                                          int K)
{
#pragma unroll
    for (int s = 0; s < FR; ++s) acc[s + KMC] = fmaf(gz[0], u[s], acc[s + KMC]);
#pragma unroll
    for (int l = 1; l <= KMC; ++l) {
        if (l > K) continue;
#pragma unroll
        for (int s = 0; s < FR; ++s) {
            acc[s + KMC + l] = fmaf(gz[l], u[s], acc[s + KMC + l]);
            acc[s + KMC - l] = fmaf(gz[l], u[s], acc[s + KMC - l]);
        }
    }
}

// The forward of one workgroup (angle, slab, depth chunk): the state that
// lives across depths, and one depth.
template <int ATT, int KMC, bool VEC>
struct FwdWalk {
    static constexpr bool MU = ATT == ATT_SAMPLE;
    // the next depth's corner loads are issued before the current depth's
    // blur; the widest blur classes keep their registers for the partial
    // rows instead (the prefetch would make them spill)
    static constexpr bool PREFETCH = KMC <= (MU ? 20 : 24);
    float4 *smem;
    const float *taps;  // this angle's taps, TS per depth
    int TS, N, Nz, jp, q, kb, nrows, ilo;
    int dks[FR];
    bool active, live, full;  // live: the lane has rows below Nz
    float2 cs, o;
    uint32_t rowb, colb, dk;
    float tau_scale;
    __amdgpu_buffer_rsrc_t rf, rm;
    // ATT_READ: the (angle, slab) brick run of the table; the lane's 4
    // factors of depth 0 at byte offset toff (past the brick run when the
    // lane has no rows, so the load returns zeros), tstep bytes per depth
    __amdgpu_buffer_rsrc_t rt;
    uint32_t toff, tstep;
    float acc[FR + 2 * KMC];
    float S[FR];       // running attenuation sums (mu sampled)
    float4 vt;         // attenuation factors of the current depth (table)
    int buf;
    FCorner cn;        // bilinear corners of the depth whose loads are in flight
    float4 vf[4], vm[4];

    // the factors of depth ip: one unconditional non-temporal buffer load
    // (no branch on the lane, so the load stays in flight across the blur)
    __device__ __forceinline__ void tload(int ip)
    {
        vt = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rt, toff + (uint32_t)ip * tstep, 0, kNonTemporal));
    }

    // issue the corner loads of depth ip (activity, and mu when sampled);
    // they are consumed one depth later
    __device__ __forceinline__ void cload(int ip)
    {
        cn = fcorners(fmaf((float)ip, cs.x, o.x), fmaf((float)ip, cs.y, o.y), N, rowb, colb, VEC ? dk : 0u);
        fload<VEC>(rf, cn, dks, vf);
        if (MU) fload<VEC>(rm, cn, dks, vm);
    }

    __device__ __forceinline__ float4 zero_past_nz(float4 v) const
    {
        if (!full) {
            if (kb + 0 >= Nz) v.x = 0.f;
            if (kb + 1 >= Nz) v.y = 0.f;
            if (kb + 2 >= Nz) v.z = 0.f;
            if (kb + 3 >= Nz) v.w = 0.f;
        }
        return v;
    }

    // depth ip of radius K (with PREFETCH its corner loads were issued one
    // depth earlier)
    __device__ __forceinline__ void depth(int ip, int K)
    {
        float4 w = make_float4(0.f, 0.f, 0.f, 0.f);
        if (active) {
            if (!PREFETCH) cload(ip);
            w = zero_past_nz(fcombine(cn, vf));
            const float4 m = MU ? zero_past_nz(fcombine(cn, vm)) : w;
            // the next depth's corners (and factors), in flight during this blur
            if (PREFETCH && ip > ilo) cload(ip - 1);
            if (ATT == ATT_READ) {
                w.x *= vt.x;
                w.y *= vt.y;
                w.z *= vt.z;
                w.w *= vt.w;
                // unconditional (the last depth reloads its own factors): a
                // skipped load would leave two values of vt to merge, and the
                // merge waits for every load in flight
                tload(max(ip - 1, ilo));
            }
            if (MU) {
                const float mm[FR] = {m.x, m.y, m.z, m.w};
                float at[FR];
#pragma unroll
                for (int r = 0; r < FR; ++r) {
                    at[r] = __builtin_amdgcn_exp2f(-tau_scale * fmaf(0.5f, mm[r], S[r]));
                    S[r] += mm[r];
                }
                w.x *= at[0];
                w.y *= at[1];
                w.z *= at[2];
                w.w *= at[3];
            }
            smem[fwb_index(buf, jp + KMC, q, nrows)] = w;
        }
        // the depth's taps, loaded while the workgroup gathers at the barrier
        // (indices past the plan's radius read zeros, or the next depth's taps
        // when a batched member's radius class is below KMC; the guards never
        // use them)
        float gz[KMC + 1];
        load_taps_all<KMC>(taps + (size_t)ip * TS, gz);
        lds_barrier();
        if (active) {
            float u[FR];
            FBinBlur<KMC> bb{smem, fwb_index(buf, jp + KMC, q, nrows), gz, w, u};
            KSwitch<0, KMC>::run(K, bb);
            fzscatter<KMC>(acc, u, gz, K);
        }
        buf ^= 1;
    }
};

template <int ATT, int KMC, bool VEC, class Args>
__device__ __forceinline__ void fwd_body(const Args &a, int slab, int chunk, int al)
{
    static_assert(ATT != ATT_WRITE, "the forward kernel does not write the table");
    constexpr bool MU = ATT == ATT_SAMPLE;
    constexpr int R = SLAB + 2 * KMC;  // the slab's partial rows
    extern __shared__ float4 smem[];
    FwdWalk<ATT, KMC, VEC> w;
    const int N = a.g.N, Nz = a.g.Nz;
    const int ang = uniform(a.L.idx[al]);
    w.smem = smem;
    w.N = N;
    w.Nz = Nz;
    w.TS = a.g.TS;
    w.taps = a.g.taps + (size_t)ang * N * a.g.TS;
    w.jp = threadIdx.x / FQ;
    w.q = threadIdx.x % FQ;
    w.active = w.jp < N;
    w.nrows = N + 2 * KMC;
    w.kb = slab * SLAB + w.q * FR;
    w.live = w.active && w.kb < Nz;
    w.full = slab * SLAB + SLAB <= Nz;  // no rows past Nz in this slab
    w.tau_scale = a.g.tau_scale;

    // zero the KMC padding rows of both buffers
    if constexpr (KMC > 0) {
        for (int i = threadIdx.x; i < 2 * 2 * KMC * FQ; i += blockDim.x) {
            const int qq = i % FQ, rest = i / FQ;
            const int prow = rest % (2 * KMC), bb = rest / (2 * KMC);
            smem[fwb_index(bb, prow < KMC ? prow : prow + N, qq, w.nrows)] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }

    w.cs = a.g.cs[ang];
    w.o = w.active ? a.g.xy0[(size_t)ang * N + w.jp] : make_float2(0.f, 0.f);
#pragma unroll
    for (int r = 0; r < FR; ++r) w.S[r] = 0.f;
    if (MU && chunk > 0 && w.active) {
        for (int c = 0; c < chunk; ++c) {
            const float *src = a.tau + (((size_t)al * a.nchunk + c) * N + w.jp) * Nz;
#pragma unroll
            for (int r = 0; r < FR; ++r) w.S[r] += (w.kb + r < Nz) ? src[w.kb + r] : 0.f;
        }
    }
#pragma unroll
    for (int t = 0; t < FR + 2 * KMC; ++t) w.acc[t] = 0.f;

    int ihi, ilo;
    chunk_range(a.g, a.cbset, a.nchunk, ang, chunk, ihi, ilo);
    ConstMem<int> *kd = as_const(a.g.kdep + (size_t)ang * N);
    w.ilo = ilo;
    w.rowb = 4u * (uint32_t)(a.zs > 0 && !MU ? a.zs : Nz);
    w.colb = w.rowb * (uint32_t)N;
    // row offsets in a z-run (clamped to valid rows; rows past Nz are zeroed)
    w.dk = 4u * (uint32_t)max(min(w.kb, Nz - 4), 0);
#pragma unroll
    for (int r = 0; r < FR; ++r) w.dks[r] = 4 * min(w.kb + r, Nz - 1);
    const int vbytes = (int)(w.colb * (uint32_t)N);
    w.rf = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(a.f), (short)0, vbytes, kBufferDword3);
    w.rm = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(MU ? a.mu : a.f), (short)0, vbytes, kBufferDword3);
    // attenuation table: the lane's rows in the 16-row brick of (angle, slab,
    // depth 0, bin j')
    if constexpr (ATT == ATT_READ) {
        w.tstep = 4u * (uint32_t)(N * SLAB);
        w.rt = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(a.att + brick_offset(al, a.nslab, slab, N, 0, 0)),
                                                 (short)0, (int)(w.tstep * (uint32_t)N), kBufferDword3);
        w.toff = w.live ? 4u * (uint32_t)(w.jp * SLAB + w.q * FR) : (uint32_t)kVolPastEnd;
    }
    w.buf = 0;
    if (ATT == ATT_READ && w.active && ihi >= ilo) w.tload(ihi);
    if (w.PREFETCH && w.active && ihi >= ilo) w.cload(ihi);
    __syncthreads();
    for (int ip = ihi; ip >= ilo; --ip) w.depth(ip, uniform(kd[ip]));

    // merge the four lanes of each bin (lane q's row t is the slab's partial
    // row 4q + t) in registers: lane 0 of the quad reads the other lanes'
    // rows through DPP and adds them in the order q = 0..3, then stores the
    // bin's R partial rows as 16-byte stores.  Every lane takes part in the
    // DPP moves (the four lanes of a quad are always active here).
    static_assert(R % 4 == 0, "partial rows in whole 16-byte groups");
    constexpr int T = FR + 2 * KMC;
    float *dst = a.part + (((size_t)al * a.nslab + slab) * a.nchunk + chunk) * N * R + (size_t)w.jp * R;
    const bool store = w.active && w.q == 0;
#pragma unroll
    for (int t0 = 0; t0 < R; t0 += 4) {
        float o[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + u;
            float v = t < T ? w.acc[t] : 0.f;
            if (t >= 4 && t - 4 < T) v += quad_bcast<1>(w.acc[t - 4]);
            if (t >= 8 && t - 8 < T) v += quad_bcast<2>(w.acc[t - 8]);
            if (t >= 12 && t - 12 < T) v += quad_bcast<3>(w.acc[t - 12]);
            o[u] = v;
        }
        if (store) *reinterpret_cast<float4 *>(dst + t0) = make_float4(o[0], o[1], o[2], o[3]);
    }
}

// Largest forward workgroup: FQ lanes per bin, N <= 256.
constexpr int FWD_MAX_THREADS = FQ * 256;

// Workgroups are dispatched in linear order, and a CU receives a second
// workgroup one device-full of workgroups after its first; with the chunk as
// the fast index after the slab, a CU's two workgroups would hold the same
// chunk of two angles (two of the heaviest, or two of the lightest).  The
// angles whose workgroups start in an odd device-full take their chunks in
// reverse order instead, so that heavy and light chunks share CUs.  The
// reversal is per angle, so every (slab, chunk, angle) is still covered once.
template <int ATT, int KMC, bool VEC>
__global__ __launch_bounds__(FWD_MAX_THREADS) void fwd_main(FwdArgs a)
{
    const int z = blockIdx.z;
    const int round = a.cus > 0 ? (int)(((long)a.nslab * a.nchunk * z) / a.cus) : 0;
    const int chunk = (round & 1) ? a.nchunk - 1 - (int)blockIdx.y : (int)blockIdx.y;
    fwd_body<ATT, KMC, VEC>(a, blockIdx.x, chunk, z);
}

template <int ATT, int KMC, bool VEC, bool PERSIST>
__global__ __launch_bounds__(FWD_MAX_THREADS) void fwd_batch(BatchList<FwdArgs> b)
{
    ConstMem<FwdArgs> *args = as_const(b.args);
    ConstMem<Task> *tasks = as_const(b.tasks);
    if (!PERSIST) {
        const int t = blockIdx.x;
        if (t < b.ntasks) fwd_body<ATT, KMC, VEC>(args[tasks[t].r], tasks[t].x, tasks[t].y, tasks[t].z);
        return;
    }
    for (int t = blockIdx.x; t < b.ntasks; t += gridDim.x) {
        const int r = tasks[t].r, x = tasks[t].x, y = tasks[t].y, z = tasks[t].z;
        fwd_body<ATT, KMC, VEC>(args[r], x, y, z);
        __syncthreads();  // the next task rewrites the row buffers
    }
}

struct ReduceArgs {
    AngleList L;
    const float *part;
    int N, Nz, nslab, nchunk, kmc;
    int mode;           // 0: write projection rows; 1: OSEM ratio into q; 2: ratio into q and
                        // e = Hf + s into e; 3: ratio derivative into q (see reduce_body)
    float *proj;        // mode 0: (A, N, Nz)
    const float *g;     // modes 1-3: measured data (A, N, Nz)
    const float *s_add; // modes 1, 2: additive term or nullptr
    float *q;           // modes 1-3: [L][N][Nz]
    float *e;           // mode 2 writes, mode 3 reads: [L][N][Nz]
};

#ifdef SPECT_HOST_TU
// Sum the partial rows of all chunks and overlapping slabs for one output
// element (angle, bin, row), chunks outer and slabs ascending.  The slabs
// whose partial rows hold row k are s with k + kmc - R < 16 s <= k + kmc, a
// half-open range of R = 16 + 2 kmc rows: at most ceil(R / 16) slabs (NSL;
// five for kmc <= 32), so their offsets are fixed before the chunk loop.
// The measured row (and the additive term) is loaded first and up to eight
// chunks' loads are issued together: the kernel is one short dependency
// chain per thread, so every load it can start at once is a round trip saved.
constexpr int RED_SLABS = 5;

// G chunks' partial rows, loaded together and added in chunk order.
template <int G, int NSL>
__device__ __forceinline__ float reduce_group(const float *pc, size_t cstride, int c, const size_t (&off)[NSL],
                                              const bool (&ok)[NSL], float sum)
{
    float v[G][NSL];
#pragma unroll
    for (int u = 0; u < G; ++u) {
        const float *p = pc + (size_t)(c + u) * cstride;
#pragma unroll
        for (int i = 0; i < NSL; ++i) v[u][i] = p[off[i]];
    }
#pragma unroll
    for (int u = 0; u < G; ++u)
#pragma unroll
        for (int i = 0; i < NSL; ++i)
            if (ok[i]) sum += v[u][i];
    return sum;
}

template <int NSL, class Args>
__device__ __forceinline__ void reduce_body(const Args &a, int blk, int al)
{
    const int N = a.N, Nz = a.Nz;
    const int t = blk * blockDim.x + threadIdx.x;
    if (t >= N * Nz) return;
    const int ang = uniform(a.L.idx[al]);
    const int r = t / Nz, k = t % Nz;
    const size_t o = ((size_t)ang * N + r) * Nz + k;
    const size_t oc = ((size_t)al * N + r) * Nz + k;
    const int mode = a.mode;
    const float *const gd = a.g, *const sa = a.s_add;
    float *const ev = a.e;
    float gv = 0.f, sv = 0.f, ev3 = 0.f;
    if (mode != 0) {
        gv = gd[o];
        if (mode == 3) ev3 = ev[oc];
        else if (sa) sv = sa[o];
    }
    const int R = SLAB + 2 * a.kmc;
    const int slo = max(0, (k + a.kmc - R + 4 * SLAB) / SLAB - 3);  // floor((k + kmc - R) / 16) + 1
    const int shi = min(a.nslab - 1, (k + a.kmc) / SLAB);
    const size_t cstride = (size_t)N * R;  // one chunk
    const float *pc = a.part + (size_t)al * a.nslab * a.nchunk * cstride + (size_t)r * R;
    size_t off[NSL];
    bool ok[NSL];
#pragma unroll
    for (int i = 0; i < NSL; ++i) {
        const int s = slo + i;
        ok[i] = s <= shi;
        off[i] = ok[i] ? (size_t)s * a.nchunk * cstride + (size_t)(k - s * SLAB + a.kmc) : 0;
    }
    float sum = 0.f;
    const int nch = a.nchunk;
    int c = 0;
    for (; c + 8 <= nch; c += 8) sum = reduce_group<8, NSL>(pc, cstride, c, off, ok, sum);
    if (c + 4 <= nch) {
        sum = reduce_group<4, NSL>(pc, cstride, c, off, ok, sum);
        c += 4;
    }
    for (; c < nch; ++c) sum = reduce_group<1, NSL>(pc, cstride, c, off, ok, sum);
    float *const q = a.q;
    if (mode == 0) {
        a.proj[o] = sum;
    } else if (mode != 3) {
        const float e = sa ? sum + sv : sum;
        q[oc] = e > 0.f ? gv / e : 0.f;
        if (mode == 2) ev[oc] = e;
    } else {
        // sum = (H v)_o for the gradient v of the ratio q = g / e; its
        // derivative in e is -g / e^2 where e > 0 and 0 elsewhere
        q[oc] = ev3 > 0.f ? -sum * gv / (ev3 * ev3) : 0.f;
    }
}

template <int NSL>
__global__ __launch_bounds__(256) void fwd_reduce(ReduceArgs a) { reduce_body<NSL>(a, blockIdx.x, blockIdx.y); }

__global__ __launch_bounds__(256) void reduce_batch(BatchList<ReduceArgs> b)
{
    ConstMem<ReduceArgs> *args = as_const(b.args);
    ConstMem<Task> *tasks = as_const(b.tasks);
    for (int t = blockIdx.x; t < b.ntasks; t += gridDim.x) {
        const int r = tasks[t].r, x = tasks[t].x, z = tasks[t].z;
        reduce_body<RED_SLABS>(args[r], x, z);
    }
}

#endif  // SPECT_HOST_TU

// ---------------------------------------------------------- back project --

struct BackRotArgs {
    DevGeom g;
    AngleList L;
    const float *y;     // projections; row of list entry al at y + row_index * N * Nz
    int y_compact;      // 1: row_index = al (compact list buffer); 0: row_index = angle
    int ones;           // 1: y is all ones (sensitivity)
    const float *mu;
    const float *tau;
    float *att;         // ATT_WRITE / ATT_READ: attenuation table [L][nslab][N][N][16]
    float *z;           // [L][nslab][N][N][SLAB] rotated-frame values
    int nslab, nchunk, cbset;
    int vec;
    float *fill;        // sensitivity pass: also set fill[0 .. fill_n) to 1 (or nullptr)
    size_t fill_n;
};

template <int ATT, int KMC, bool VEC, class Args>
__device__ __forceinline__ void back_body(const Args &a, int slab, int chunk, int al)
{
    constexpr bool MU = ATT == ATT_SAMPLE || ATT == ATT_WRITE;
    extern __shared__ float4 smem[];
    const int N = a.g.N, Nz = a.g.Nz;
    const int ang = uniform(a.L.idx[al]);
    const int jp = threadIdx.x >> 1, h = threadIdx.x & 1;
    const bool active = jp < N;
    const int nrows = N + 2 * KMC;
    const int k0 = slab * SLAB;
    const int kb = k0 + h * ROWS;
    constexpr int R = SLAB + 2 * KMC;
    constexpr int YP = R + 1;
    float *ybuf = reinterpret_cast<float *>(smem + 2 * 2 * nrows * 2);

    zero_padding<KMC>(smem, N, nrows);
    // axial rows k0 - KMC .. k0 + SLAB + KMC - 1 of the projection, per bin;
    // bin jp's column starts at jp * YP + 8 (jp / 8), which puts the 64 lanes
    // of a column read (bins jp, halves h reading rows 8 h + c) in distinct
    // banks of a 32- or 64-bank LDS
    float *ycol = ybuf + jp * YP + 8 * (jp >> 3);
    if (active) {
        const float *yr = a.y + ((size_t)(a.y_compact ? al : ang) * N + jp) * Nz;
        for (int t = h; t < R; t += 2) {
            const int k = k0 - KMC + t;
            float v = 0.f;
            if (k >= 0 && k < Nz) v = a.ones ? 1.f : yr[k];
            ycol[t] = v;
        }
    }

    const float2 cs = a.g.cs[ang];
    const float2 o = active ? a.g.xy0[(size_t)ang * N + jp] : make_float2(0.f, 0.f);
    float S[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) S[r] = 0.f;
    if (MU && chunk > 0 && active) chunk_start(a.tau, al, a.nchunk, chunk, N, Nz, jp, kb, S);
    int ihi, ilo;
    chunk_range(a.g, a.cbset, a.nchunk, ang, chunk, ihi, ilo);
    ConstMem<int> *kd = as_const(a.g.kdep + (size_t)ang * N);
    const float *taps = a.g.taps + (size_t)ang * N * a.g.TS;
    // mu corners: raw buffer loads over the map (see fcorners); the vector
    // path reads the lane's 8 rows as two 16-byte loads per corner (rows past
    // Nz read the next column or zeros, and are zeroed below)
    const uint32_t rowb = 4u * (uint32_t)Nz, colb = rowb * (uint32_t)N;
    const uint32_t dk8 = 4u * (uint32_t)kb;
    int dks[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) dks[r] = 4 * min(kb + r, Nz - 1);
    const __amdgpu_buffer_rsrc_t rm = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float *>(MU ? a.mu : a.y), (short)0, MU ? (int)(colb * (uint32_t)N) : 0, kBufferDword3);
    // table and rotated-frame bricks: uniform base of this (angle, slab) + per-thread offset
    const size_t wg0 = brick_offset(al, a.nslab, slab, N, 0, 0);
    const uint32_t toff = 4u * (uint32_t)(jp * SLAB + h * ROWS);
    int buf = 0;
    __syncthreads();
    for (int ip = ihi; ip >= ilo; --ip) {
        const int K = uniform(kd[ip]);
        float gz[KMC + 1];
        load_taps_all<KMC>(taps + (size_t)ip * a.g.TS, gz);
        float v[ROWS];
        FCorner cn;
        float4 mc[4][2];
        float4 t0, t1;
        const size_t row0 = wg0 + (size_t)ip * N * SLAB;
        if (active) {
            // attenuation factors of this depth, in flight during the blur
            if (ATT == ATT_READ) {
                t0 = at_byte<float4>(a.att + row0, toff);
                t1 = at_byte<float4>(a.att + row0, toff + 16);
            }
            ZGather<KMC> zg{ycol, h * ROWS + KMC, gz, v};
            KSwitch<0, KMC>::run(K, zg);
            smem[wb_index(buf, 0, jp + KMC, h, nrows)] = make_float4(v[0], v[1], v[2], v[3]);
            smem[wb_index(buf, 1, jp + KMC, h, nrows)] = make_float4(v[4], v[5], v[6], v[7]);
            // attenuation samples of this depth, in flight during the bin blur
            if (MU) {
                cn = fcorners(fmaf((float)ip, cs.x, o.x), fmaf((float)ip, cs.y, o.y), N, rowb, colb,
                              VEC ? dk8 : 0u);
                fload8<VEC>(rm, cn, dks, mc);
            }
        }
        lds_barrier();
        if (active) {
            float u[ROWS];
            BackBlur<KMC> bb{v, u, smem, wb_index(buf, 0, jp + KMC, h, nrows), wb_index(buf, 1, jp + KMC, h, nrows),
                             gz};
            KSwitch<0, KMC>::run(K, bb);
            if (MU) {
                float m[ROWS], att[ROWS];
                fcombine8(cn, mc, kb, Nz, m);
                attenuate(m, S, a.g.tau_scale, att);
#pragma unroll
                for (int r = 0; r < ROWS; ++r) u[r] *= att[r];
                if (ATT == ATT_WRITE) {
                    float *tb = reinterpret_cast<float *>(reinterpret_cast<char *>(a.att + row0) + toff);
                    stream_store_f4(tb, att[0], att[1], att[2], att[3]);
                    stream_store_f4(tb + 4, att[4], att[5], att[6], att[7]);
                }
            }
            if (ATT == ATT_READ) {
                u[0] *= t0.x;
                u[1] *= t0.y;
                u[2] *= t0.z;
                u[3] *= t0.w;
                u[4] *= t1.x;
                u[5] *= t1.y;
                u[6] *= t1.z;
                u[7] *= t1.w;
            }
            float4 *dst = reinterpret_cast<float4 *>(reinterpret_cast<char *>(a.z + row0) + toff);
            dst[0] = make_float4(u[0], u[1], u[2], u[3]);
            dst[1] = make_float4(u[4], u[5], u[6], u[7]);
        }
        buf ^= 1;
    }
}

template <int ATT, int KMC, bool VEC>
__global__ __launch_bounds__(512) void back_rot(BackRotArgs a)
{
    back_body<ATT, KMC, VEC>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <int ATT, int KMC, bool VEC, bool PERSIST>
__global__ __launch_bounds__(512) void back_batch(BatchList<BackRotArgs> b)
{
    ConstMem<BackRotArgs> *args = as_const(b.args);
    ConstMem<Task> *tasks = as_const(b.tasks);
    if (!PERSIST) {
        const int t = blockIdx.x;
        if (t < b.ntasks) back_body<ATT, KMC, VEC>(args[tasks[t].r], tasks[t].x, tasks[t].y, tasks[t].z);
        return;
    }
    for (int t = blockIdx.x; t < b.ntasks; t += gridDim.x) {
        const int r = tasks[t].r, x = tasks[t].x, y = tasks[t].y, z = tasks[t].z;
        back_body<ATT, KMC, VEC>(args[r], x, y, z);
        __syncthreads();  // the next task rewrites the row and projection buffers
    }
}

#ifdef SPECT_HOST_TU
// Rotated-frame pass of the sensitivity H^T 1.  The projection is all ones,
// so the separable blur of depth i' reduces to the product of the in-range
// tap sums along the bin axis and the axial axis:
//     (G_r G_z 1)(j', k) = e_r(j') e_z(k),  e_r(j') = sum_{|m|<=K, 0<=j'+m<N} g_|m|
//                                                  = C[min(K, j')] + C[min(K, N-1-j')] - g_0
// with the running tap sums C (e_z likewise over 0 <= k+l < Nz); the value is
// that product times the attenuation factor, written to the rotated-frame
// bricks like back_rot (ATT_WRITE also stores the factors).  No neighbours
// are needed, so one thread per (angle, slab, bin, pair of axial rows) walks
// every depth from the detector side with no LDS and no depth split: the
// attenuation sum is one running sum per row and mu is sampled once per
// depth.  V2: Nz even and an 8-byte aligned mu, so a pair of rows loads as
// one float2.
constexpr int SL_THREADS = 256;

template <int ATT, bool V2, class Args>
__device__ __forceinline__ void sensl_walk(const Args &a, int jp, int rp, int slab, int al, int ang,
                                           const float *ctl, int chunk);

// blk: thread block within the (slab, angle) and, without attenuation (no
// running sum), depth chunk: blocks of chunk c are c * nblk .. c * nblk +
// nblk - 1 for the nchunk equal depth chunks of the launch.
template <int ATT, bool V2, class Args>
__device__ __forceinline__ void sensl_body(const Args &a, int blk, int slab, int al)
{
    const int N = a.g.N;
    const int nblk = (N * (SLAB / 2) + SL_THREADS - 1) / SL_THREADS;
    const int chunk = blk / nblk;
    blk -= chunk * nblk;
    const int t = blk * SL_THREADS + threadIdx.x;
    const int jp = t >> 3, rp = t & 7;
    const int ang = uniform(a.L.idx[al]);
    // this angle's running tap sums C[i'][m] in LDS: the per-lane lookups of
    // the in-range sums then use the LDS pipe, not the vector-memory return
    // path that the mu samples need (dynamic LDS of N * TS floats)
    extern __shared__ float4 smem[];
    float *ctl = reinterpret_cast<float *>(smem);
    const int TS = a.g.TS;
    {
        ConstMem<float> *cta = as_const(a.g.ctaps + (size_t)ang * N * TS);
        for (int i = threadIdx.x; i < N * TS; i += SL_THREADS) ctl[i] = cta[i];
    }
    __syncthreads();
    if (jp < N) sensl_walk<ATT, V2>(a, jp, rp, slab, al, ang, ctl, chunk);
    __syncthreads();  // a batch's next task rewrites the sums
}

// The depth walk of one (bin, pair of rows) thread of the sensitivity pass;
// ctl holds the angle's running tap sums, TS per depth.
template <int ATT, bool V2, class Args>
__device__ __forceinline__ void sensl_walk(const Args &a, int jp, int rp, int slab, int al, int ang,
                                           const float *ctl, int chunk)
{
    constexpr bool MU = ATT == ATT_SAMPLE || ATT == ATT_WRITE;
    const int N = a.g.N, Nz = a.g.Nz;
    const int TS = a.g.TS;
    const int k0 = slab * SLAB;
    const int k = k0 + 2 * rp;  // rows k and k + 1; rows past Nz get values the gather never reads
    const bool in0 = k < Nz, in1 = k + 1 < Nz;
    const float2 cs = a.g.cs[ang];
    const float2 o = a.g.xy0[(size_t)ang * N + jp];
    ConstMem<int> *kd = as_const(a.g.kdep + (size_t)ang * N);
    // mu is only read here, so its loads may move ahead of this thread's
    // stores (next depth's corners are loaded before this depth is stored)
    ConstMem<float> *mu = as_const(a.mu);
    const uint32_t rowb = 4u * (uint32_t)Nz;
    // byte offsets of the two rows in a z-run, clamped to valid rows (V2: k
    // and Nz even, so both rows are in range or both past Nz)
    const uint32_t dk0 = 4u * (uint32_t)min(k, Nz - 1), dk1 = 4u * (uint32_t)min(k + 1, Nz - 1);
    const uint32_t dkp = 4u * (uint32_t)max(0, min(k, Nz - 2));
    const size_t e0 = brick_offset(al, a.nslab, slab, N, 0, 0) + (size_t)jp * SLAB + 2 * rp;
    struct Samp {
        Corners cn;
        float v0[4], v1[4];
    };
    auto sample = [&](int ip, Samp &sp) {
        sp.cn = corners(fmaf((float)ip, cs.x, o.x), fmaf((float)ip, cs.y, o.y), N, rowb);
        const uint32_t oc[4] = {sp.cn.b00, sp.cn.b10, sp.cn.b01, sp.cn.b11};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if constexpr (V2) {
                typedef float pair_t __attribute__((ext_vector_type(2)));
                const pair_t pr = *reinterpret_cast<ConstMem<pair_t> *>(reinterpret_cast<ConstMem<char> *>(mu) + oc[j] + dkp);
                sp.v0[j] = pr.x;
                sp.v1[j] = pr.y;
            } else {
                sp.v0[j] = *reinterpret_cast<ConstMem<float> *>(reinterpret_cast<ConstMem<char> *>(mu) + oc[j] + dk0);
                sp.v1[j] = *reinterpret_cast<ConstMem<float> *>(reinterpret_cast<ConstMem<char> *>(mu) + oc[j] + dk1);
            }
        }
    };
    float S0 = 0.f, S1 = 0.f;
    // one depth from the samples in sp (loaded one depth earlier)
    auto step = [&](int ip, const Samp &sp) {
        const int K = uniform(kd[ip]);
        const float *ct = ctl + ip * TS;
        const float g0 = ct[0], cK = ct[K];
        // in-range tap sums across bins and rows; an interior slab (both
        // sides reach K inside the detector) takes 2 C[K] - g0
        const float cr0 = ct[min(K, jp)], cr1 = ct[min(K, N - 1 - jp)];
        const bool zin = k0 - K >= 0 && k0 + SLAB - 1 + K < Nz;
        const float cz0 = ct[min(K, max(k, 0))], cz1 = ct[max(0, min(K, Nz - 1 - k))];
        const float cz2 = ct[min(K, max(k + 1, 0))], cz3 = ct[max(0, min(K, Nz - 2 - k))];
        const float er = cr0 + cr1 - g0;
        const float ezi = 2.f * cK - g0;
        float u0 = er * (zin ? ezi : cz0 + cz1 - g0);
        float u1 = er * (zin ? ezi : cz2 + cz3 - g0);
        const size_t e = e0 + (size_t)ip * N * SLAB;
        if (MU) {
            const Corners &cn = sp.cn;
            float m0 = fmaf(cn.w11, sp.v0[3], fmaf(cn.w01, sp.v0[2], fmaf(cn.w10, sp.v0[1], cn.w00 * sp.v0[0])));
            float m1 = fmaf(cn.w11, sp.v1[3], fmaf(cn.w01, sp.v1[2], fmaf(cn.w10, sp.v1[1], cn.w00 * sp.v1[0])));
            if (!in0) m0 = 0.f;
            if (!in1) m1 = 0.f;
            const float a0 = __builtin_amdgcn_exp2f(-a.g.tau_scale * fmaf(0.5f, m0, S0));
            const float a1 = __builtin_amdgcn_exp2f(-a.g.tau_scale * fmaf(0.5f, m1, S1));
            S0 += m0;
            S1 += m1;
            u0 *= a0;
            u1 *= a1;
            if (ATT == ATT_WRITE) stream_store_f2(a.att + e, a0, a1);
        }
        *reinterpret_cast<float2 *>(a.z + e) = make_float2(u0, u1);
    };
    Samp s0, s1, s2, s3;
    if (!MU) {
        // no attenuation: the depths are independent; this chunk's only
        const int len = (N + a.nchunk - 1) / a.nchunk;
        const int ihi = N - 1 - chunk * len, ilo = max(0, ihi - len + 1);
        for (int ip = ihi; ip >= ilo; --ip) step(ip, s0);
        return;
    }
    // four sample buffers used in turn: the corners of the depth three
    // steps ahead are loaded before this depth is computed and stored, and
    // every load is waited for only where it is used (no register copies)
    if (MU) {
        sample(N - 1, s0);
        sample(max(N - 2, 0), s1);
        sample(max(N - 3, 0), s2);
    }
    for (int ip = N - 1; ip >= 0; ip -= 4) {
        if (MU) sample(max(ip - 3, 0), s3);
        step(ip, s0);
        if (ip - 1 < 0) break;
        if (MU) sample(max(ip - 4, 0), s0);
        step(ip - 1, s1);
        if (ip - 2 < 0) break;
        if (MU) sample(max(ip - 5, 0), s1);
        step(ip - 2, s2);
        if (ip - 3 < 0) break;
        if (MU) sample(max(ip - 6, 0), s2);
        step(ip - 3, s3);
    }
}

template <int ATT, bool V2>
__global__ __launch_bounds__(SL_THREADS) void sens_line(BackRotArgs a)
{
    if (a.fill) {
        // a reconstruction's start image, 1 everywhere, written by the
        // launch that precedes its first read
        const size_t nt = (size_t)gridDim.x * gridDim.y * gridDim.z * SL_THREADS;
        const size_t t0 = (((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * SL_THREADS +
                          threadIdx.x;
        for (size_t i = t0; i < a.fill_n; i += nt) a.fill[i] = 1.f;
    }
    sensl_body<ATT, V2>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

// The same over a batch work-list: task (member, thread block, slab, angle).
template <int ATT, bool V2>
__global__ __launch_bounds__(SL_THREADS) void sensl_batch(BatchList<BackRotArgs> b)
{
    ConstMem<BackRotArgs> *args = as_const(b.args);
    ConstMem<Task> *tasks = as_const(b.tasks);
    for (int t = blockIdx.x; t < b.ntasks; t += gridDim.x)
        sensl_body<ATT, V2>(args[tasks[t].r], tasks[t].x, tasks[t].y, tasks[t].z);
}

#endif  // SPECT_HOST_TU

// Terms of the BSREM update (gather mode 3): where sens_all > 0,
// out <- max(0, out + out * a_over_c / sens_all * (sum - sens - c_beta * prior)).
struct BsremTerms {
    const float *sens_all;  // H^T 1 over all angles
    const float *prior;     // gradient of the prior at out
    float a_over_c;         // relaxation / subset share
    float c_beta;           // subset share * prior weight
};

// Terms of the OSEM update and of its vector-Jacobian product (gather modes 2
// and 4).  Mode 2 reads the image from fin when it is given (out-of-place
// update) and from out otherwise.  Mode 4, with b the gathered sum:
//     out = gout * b / sens,  gb = gout * fin / sens   where sens > 0,
//     out = gout,             gb = 0                   elsewhere,
// the derivatives of f' = f b / sens (f' = f where sens = 0) in f and in b.
struct StepTerms {
    const float *fin;
    const float *gout;
    float *gb;
};

struct GatherArgs {
    DevGeom g;
    AngleList L;
    const float *z;
    int nslab;
    int mode;            // 0: out = sum; 1: out += sum; 2: OSEM update of out with sens; 3: BSREM update;
                         // 4: OSEM update derivative (StepTerms)
    float *out;
    const float *sens;   // modes 2-4: subset sensitivity H_m^T 1
    BsremTerms bt;       // mode 3
    StepTerms st;        // modes 2, 4
    float *fpad;         // modes 2, 3: also store the updated image here, columns zs floats apart
    int zs;
    int v4;              // Nz % 4 == 0 and every array 16-byte aligned: modes 0, 2, 3 use 16-byte accesses
    int zshare;          // 1: every angle reads the one brick volume at z
};

// Transpose of the bilinear rotation, as a gather.  Workgroup = 8 x 8 object
// columns x two slabs; a wave covers 16 columns and four lanes share a
// column, lane q taking the 16-byte quad q of the column's 16 axial rows in
// both slabs, so that every candidate brick (64 bytes) is read by four
// adjacent lanes.  For each angle a column takes the <= 3 x 3 rotated samples
// around its rotated position; the weight of sample P is the bilinear hat
// max(0, 1 - |X_P - x|) max(0, 1 - |Y_P - y|), with X_P, Y_P computed by the
// forward's own FP32 expression, so the weights equal the forward's to within
// one rounding.  Lane q of a column evaluates the three candidates of window
// column q (lane 3 none) and writes their weights and brick offsets to the
// quad's nine-entry table in LDS; the quad then loads only the candidates of
// non-zero weight, in window order, through at most GC slots (a rotated unit
// lattice puts at most five samples strictly inside the 2 x 2 box around a
// column; a general loop takes any further ones).  The data-return path,
// which spends the same cycles on a wave load whatever its lane mask, bounds
// this kernel, so the load count is what matters; the two slabs use the same
// weights.
constexpr int GT = 8;  // gather tile edge
constexpr int GS = 2;  // slabs per gather workgroup
constexpr int GC = 5;  // candidate load slots per angle

#ifdef SPECT_HOST_TU
// NS slabs per workgroup: GS, or 1 for launches too small to fill the
// device (the sums are formed in the same order either way).
template <int NS, class Args>
__device__ __forceinline__ void gather_body(const Args &a, int tile, int pair, int ao = 0, int na = -1,
                                            const float *zb = nullptr, float *outp = nullptr)
{
    // angles ao .. ao + na - 1 of the list, their bricks from zb and the
    // result into outp (by default the whole list, the bricks and the output
    // of the arguments)
    if (na < 0) na = a.L.n;
    if (!zb) zb = a.z;
    if (!outp) outp = a.out;
    const int N = a.g.N, Nz = a.g.Nz;
    const int tiles = (N + GT - 1) / GT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane >> 2, q = lane & 3;
    const int x = (tile / tiles) * GT + wave * 2 + (col >> 3);
    const int y = (tile % tiles) * GT + (col & 7);
    if (x >= N || y >= N) return;  // whole quads leave together
    const int slab0 = pair * NS;
    const int nsl = min(NS, a.nslab - slab0);  // slabs present in this pair
    const float c = 0.5f * (float)(N - 1);
    const float xx = (float)x - c, yy = (float)y - c;
    const float fxv = (float)x, fyv = (float)y;
    float acc[NS][4] = {};
    const size_t zstride = a.zshare ? 0 : (size_t)a.nslab * N * N * SLAB;
    const float *zs = zb + (size_t)slab0 * N * N * SLAB;
    const int qoff = 16 * q;
    const uint32_t rowb = (uint32_t)N * SLAB * 4;  // bytes per rotated row i' (N <= 256: < 2^22)
    const int planeb = (int)(N * rowb);             // bytes per slab plane (<= 4 MiB)
    // Candidate window of angle al and the ray origin of this lane's window
    // column; fetched one angle ahead so that the weights are known before
    // the brick loads are issued.
    struct Win {
        float2 cs, o;
        int ilo, jlo;
    };
    auto window = [&](int al) {
        Win w;
        const int ang = uniform(a.L.idx[ao + al]);
        w.cs = a.g.cs[ang];
        const float wdw = fabsf(w.cs.x) + fabsf(w.cs.y) + 1e-3f;
        const float ic = c + w.cs.x * xx + w.cs.y * yy;
        const float jc = c - w.cs.y * xx + w.cs.x * yy;
        w.ilo = (int)ceilf(ic - wdw);
        w.jlo = (int)ceilf(jc - wdw);
        w.o = a.g.xy0[(size_t)ang * N + min(max(w.jlo + q, 0), N - 1)];
        return w;
    };
    if constexpr (NS == 1) {
        // One slab per workgroup: small launches, bound by the latency of
        // each angle's candidate loads.  The loads of angle al + 1 are issued
        // before the sums of angle al (two register sets, two candidate
        // tables), every slot unconditionally (an empty slot reads zeros past
        // the end of the angle's plane), so that no branch makes the compiler
        // wait for them early.  The sums are formed in the same order as in
        // the loop below.
        __shared__ float2 ctab2[2][256 / 4][9];
        struct Stage {
            float4 v[GC];
            float w[GC];
            int m;  // the quad's candidates beyond the slots
            __amdgpu_buffer_rsrc_t zr;
        };
        // the window (and its ray-origin load) one stage ahead, as below.
        // Stages run in pairs without branches around their loads: a stage
        // past the last angle (al == L) has no candidates and adds zeros.
        const int L = max(na, 1);  // an empty list runs one stage of zeros
        Win wn = window(0);
        auto stage = [&](int al, Stage &S, int buf) {
            const bool live = al < na;
            const Win cur = wn;
            wn = window(min(al + 1, L - 1));
            S.zr = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(zs + (size_t)min(al, L - 1) * zstride),
                                                     (short)0, nsl * planeb, kBufferDword3);
            float2 *qt = ctab2[buf][threadIdx.x >> 2];
            const int jp = cur.jlo + q;
            const bool jin = live && q < 3 && (unsigned)jp < (unsigned)N;
            const uint32_t jb = (uint32_t)jp * (SLAB * 4);
            int mq = 0;
#pragma unroll
            for (int di = 0; di < 3; ++di) {
                const int ip = cur.ilo + di;
                const bool inr = jin && (unsigned)ip < (unsigned)N;
                const float X = fmaf((float)ip, cur.cs.x, cur.o.x), Y = fmaf((float)ip, cur.cs.y, cur.o.y);
                const float wx = fmaxf(0.f, 1.f - fabsf(X - fxv)), wy = fmaxf(0.f, 1.f - fabsf(Y - fyv));
                const float wt = inr ? wx * wy : 0.f;
                if (q < 3) qt[3 * q + di] = make_float2(wt, __int_as_float((int)((uint32_t)ip * rowb + jb)));
                mq |= (wt > 0.f ? 1 : 0) << di;
            }
            int m = quad_bcast<0>(mq) | (quad_bcast<1>(mq) << 3) | (quad_bcast<2>(mq) << 6);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
            bool hk[GC];
            float2 ek[GC];
#pragma unroll
            for (int k = 0; k < GC; ++k) {
                hk[k] = m != 0;
                ek[k] = qt[hk[k] ? __builtin_ctz(m) : 0];
                m &= m - 1;
            }
#pragma unroll
            for (int k = 0; k < GC; ++k) {
                S.w[k] = hk[k] ? ek[k].x : 0.f;
                const int off = hk[k] ? __float_as_int(ek[k].y) + qoff : kVolPastEnd;
                S.v[k] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(S.zr, off, 0, 0));
            }
            S.m = m;
        };
        auto accum = [&](const Stage &S, int buf) {
#pragma unroll
            for (int k = 0; k < GC; ++k) {
                acc[0][0] = fmaf(S.w[k], S.v[k].x, acc[0][0]);
                acc[0][1] = fmaf(S.w[k], S.v[k].y, acc[0][1]);
                acc[0][2] = fmaf(S.w[k], S.v[k].z, acc[0][2]);
                acc[0][3] = fmaf(S.w[k], S.v[k].w, acc[0][3]);
            }
            const float2 *qt = ctab2[buf][threadIdx.x >> 2];
            int m = S.m;
            while (m != 0) {
                const float2 e = qt[__builtin_ctz(m)];
                m &= m - 1;
                const float4 v = __builtin_bit_cast(
                    float4, __builtin_amdgcn_raw_buffer_load_b128(S.zr, __float_as_int(e.y) + qoff, 0, 0));
                acc[0][0] = fmaf(e.x, v.x, acc[0][0]);
                acc[0][1] = fmaf(e.x, v.y, acc[0][1]);
                acc[0][2] = fmaf(e.x, v.z, acc[0][2]);
                acc[0][3] = fmaf(e.x, v.w, acc[0][3]);
            }
        };
        Stage sa, sb;
        stage(0, sa, 0);
        for (int al = 0; al < L; al += 2) {
            stage(al + 1, sb, 1);
            accum(sa, 0);
            stage(al + 2, sa, 0);
            accum(sb, 1);
        }
    } else {
        Win nxt;
        if (na > 0) nxt = window(0);
        // the quad's candidate table: entry 3 q + di = (weight, byte offset) of
        // window row di, column q
        __shared__ float2 ctab[256 / 4][9];
        float2 *qt = ctab[threadIdx.x >> 2];
        // loaded candidate bricks, kept across angles (see below)
        float4 vv[NS][GC];
#pragma unroll
        for (int sl = 0; sl < NS; ++sl)
#pragma unroll
            for (int k = 0; k < GC; ++k) vv[sl][k] = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int al = 0; al < na; ++al) {
            const Win cur = nxt;
            if (al + 1 < na) nxt = window(al + 1);
            // raw buffer over the angle's planes of this slab pair: an offset
            // past its end reads zeros (the second plane of a lone last slab)
            const __amdgpu_buffer_rsrc_t zr = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<float *>(zs + (size_t)al * zstride), (short)0, nsl * planeb, kBufferDword3);
            // this lane's window column jlo + q: weights and brick offsets of its
            // three rows (lane 3 has none)
            const int jp = cur.jlo + q;
            const bool jin = q < 3 && (unsigned)jp < (unsigned)N;
            const uint32_t jb = (uint32_t)jp * (SLAB * 4);
            int mq = 0;  // bit di: row di of this window column has a non-zero weight
#pragma unroll
            for (int di = 0; di < 3; ++di) {
                const int ip = cur.ilo + di;
                const bool inr = jin && (unsigned)ip < (unsigned)N;
                const float X = fmaf((float)ip, cur.cs.x, cur.o.x), Y = fmaf((float)ip, cur.cs.y, cur.o.y);
                const float wx = fmaxf(0.f, 1.f - fabsf(X - fxv)), wy = fmaxf(0.f, 1.f - fabsf(Y - fyv));
                const float wt = inr ? wx * wy : 0.f;
                if (q < 3) qt[3 * q + di] = make_float2(wt, __int_as_float((int)((uint32_t)ip * rowb + jb)));
                mq |= (wt > 0.f ? 1 : 0) << di;
            }
            // the quad's non-zero candidates, bit 3 q + di
            int m = quad_bcast<0>(mq) | (quad_bcast<1>(mq) << 3) | (quad_bcast<2>(mq) << 6);
            // the table entries are written and read by lanes of this wave only
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
            // slot k takes the k-th non-zero candidate.  A quad with fewer
            // candidates leaves the slot's registers as they are and gives it
            // weight 0: they hold zero or a value this lane loaded earlier with a
            // positive weight into the same row sums, so the product is 0 unless
            // that row's sum is already non-finite.
            // the slots' table reads are issued together, then their loads
            bool hk[GC];
            float2 ek[GC];
#pragma unroll
            for (int k = 0; k < GC; ++k) {
                hk[k] = m != 0;
                ek[k] = qt[hk[k] ? __builtin_ctz(m) : 0];
                m &= m - 1;
            }
            float wk[GC];
#pragma unroll
            for (int k = 0; k < GC; ++k) {
                wk[k] = hk[k] ? ek[k].x : 0.f;
                if (hk[k]) {
                    const int off = __float_as_int(ek[k].y) + qoff;
#pragma unroll
                    for (int sl = 0; sl < NS; ++sl)
                        vv[sl][k] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(zr, off + sl * planeb, 0, 0));
                }
            }
#pragma unroll
            for (int k = 0; k < GC; ++k) {
#pragma unroll
                for (int sl = 0; sl < NS; ++sl) {
                    acc[sl][0] = fmaf(wk[k], vv[sl][k].x, acc[sl][0]);
                    acc[sl][1] = fmaf(wk[k], vv[sl][k].y, acc[sl][1]);
                    acc[sl][2] = fmaf(wk[k], vv[sl][k].z, acc[sl][2]);
                    acc[sl][3] = fmaf(wk[k], vv[sl][k].w, acc[sl][3]);
                }
            }
            // candidates beyond the slots (not expected; kept for any geometry)
            while (m != 0) {
                const float2 e = qt[__builtin_ctz(m)];
                m &= m - 1;
                const int off = __float_as_int(e.y) + qoff;
#pragma unroll
                for (int sl = 0; sl < NS; ++sl) {
                    const float4 v = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(zr, off + sl * planeb, 0, 0));
                    acc[sl][0] = fmaf(e.x, v.x, acc[sl][0]);
                    acc[sl][1] = fmaf(e.x, v.y, acc[sl][1]);
                    acc[sl][2] = fmaf(e.x, v.z, acc[sl][2]);
                    acc[sl][3] = fmaf(e.x, v.w, acc[sl][3]);
                }
            }
        }
    }
    const size_t base = ((size_t)x * N + y) * Nz;
    if (a.v4 && (a.mode == 0 || (a.mode == 2 && !a.st.fin) || a.mode == 3)) {
        // the lane's 4 rows of each slab as one 16-byte access per array
        // (the same arithmetic per element as the general path below)
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
            const int k = (slab0 + sl) * SLAB + 4 * q;
            if (k >= Nz) break;
            float4 *p = reinterpret_cast<float4 *>(outp + base + k);
            float4 v;
            if (a.mode == 0) {
                v = make_float4(acc[sl][0], acc[sl][1], acc[sl][2], acc[sl][3]);
            } else if (a.mode == 2) {
                const float4 sv = *reinterpret_cast<const float4 *>(a.sens + base + k), fv = *p;
                v.x = sv.x > 0.f ? fv.x * acc[sl][0] / sv.x : fv.x;
                v.y = sv.y > 0.f ? fv.y * acc[sl][1] / sv.y : fv.y;
                v.z = sv.z > 0.f ? fv.z * acc[sl][2] / sv.z : fv.z;
                v.w = sv.w > 0.f ? fv.w * acc[sl][3] / sv.w : fv.w;
            } else {
                const float4 sa = *reinterpret_cast<const float4 *>(a.bt.sens_all + base + k), fv = *p;
                const float4 sm = *reinterpret_cast<const float4 *>(a.sens + base + k);
                const float4 pr = *reinterpret_cast<const float4 *>(a.bt.prior + base + k);
                const float sav[4] = {sa.x, sa.y, sa.z, sa.w}, fvv[4] = {fv.x, fv.y, fv.z, fv.w};
                const float smv[4] = {sm.x, sm.y, sm.z, sm.w}, prv[4] = {pr.x, pr.y, pr.z, pr.w};
                float o[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float step = acc[sl][r] - smv[r] - a.bt.c_beta * prv[r];
                    o[r] = sav[r] > 0.f ? fmaxf(0.f, fvv[r] + fvv[r] * a.bt.a_over_c / sav[r] * step) : fvv[r];
                }
                v = make_float4(o[0], o[1], o[2], o[3]);
            }
            *p = v;
            if (a.mode != 0 && a.fpad) *reinterpret_cast<float4 *>(a.fpad + ((size_t)x * N + y) * a.zs + k) = v;
        }
        return;
    }
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = (slab0 + sl) * SLAB + 4 * q + r;
            if (k >= Nz) break;
            float *p = outp + base + k;
            if (a.mode == 0) {
                *p = acc[sl][r];
            } else if (a.mode == 1) {
                *p += acc[sl][r];
            } else if (a.mode == 2) {
                const float sv = a.sens[base + k];
                if (a.st.fin) {
                    const float fv = a.st.fin[base + k];
                    *p = sv > 0.f ? fv * acc[sl][r] / sv : fv;
                } else if (sv > 0.f) {
                    *p = *p * acc[sl][r] / sv;
                }
            } else if (a.mode == 4) {
                const float sv = a.sens[base + k], go = a.st.gout[base + k];
                *p = sv > 0.f ? go * acc[sl][r] / sv : go;
                a.st.gb[base + k] = sv > 0.f ? go * a.st.fin[base + k] / sv : 0.f;
            } else {
                const float sa = a.bt.sens_all[base + k];
                if (sa > 0.f) {
                    const float fv = *p;
                    const float step = acc[sl][r] - a.sens[base + k] - a.bt.c_beta * a.bt.prior[base + k];
                    *p = fmaxf(0.f, fv + fv * a.bt.a_over_c / sa * step);
                }
            }
            if ((a.mode == 2 || a.mode == 3) && a.fpad) a.fpad[((size_t)x * N + y) * a.zs + k] = *p;
        }
    }
}

#endif  // SPECT_HOST_TU

#ifdef SPECT_HOST_TU
template <int NS>
__global__ __launch_bounds__(256) void back_gather(GatherArgs a)
{
    gather_body<NS>(a, blockIdx.x, blockIdx.y);
}

// The gathers of M interleaved subsets in one launch (blockIdx.z = subset):
// a.L lists every angle, subset after subset (subset m holds the angles
// m, m + M, ..., so its count is ceil((A - m) / M)); subset m's bricks follow
// those of the subsets before it in a.z, and its result goes to
// a.out + m * out_stride (with a.zshare, every angle's brick is the one at
// a.z).
template <int NS>
__global__ __launch_bounds__(256) void back_gather_subsets(GatherArgs a, int M, size_t out_stride)
{
    const int m = blockIdx.z, A = a.L.n;
    const int first = m * (A / M) + min(m, A % M), count = A / M + (m < A % M ? 1 : 0);
    const size_t per = a.zshare ? 0 : (size_t)a.nslab * a.g.N * a.g.N * SLAB;
    gather_body<NS>(a, blockIdx.x, blockIdx.y, first, count, a.z + (size_t)first * per,
                    a.out + (size_t)m * out_stride);
}

__global__ __launch_bounds__(256) void gather_batch(BatchList<GatherArgs> b)
{
    ConstMem<GatherArgs> *args = as_const(b.args);
    ConstMem<Task> *tasks = as_const(b.tasks);
    for (int t = blockIdx.x; t < b.ntasks; t += gridDim.x) {
        const int r = tasks[t].r, x = tasks[t].x, y = tasks[t].y;
        gather_body<GS>(args[r], x, y);
    }
}

__global__ __launch_bounds__(256) void fill_zero(float *p, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// dst = src with columns zs floats apart instead of Nz (Nz a multiple of 4;
// the rows past Nz are not written).
__global__ __launch_bounds__(256) void pad_columns(const float4 *src, float4 *dst, size_t ncol, int nz4, int zs4)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncol * nz4) return;
    const size_t c = i / nz4, k = i % nz4;
    dst[c * zs4 + k] = src[i];
}

// out = sum of n volumes spaced `stride` floats apart from `first`.
__global__ __launch_bounds__(256) void vol_sum(const float *first, size_t stride, int n, float *out, size_t count)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float acc = 0.f;
    for (int m = 0; m < n; ++m) acc += first[m * stride + i];
    out[i] = acc;
}

// ------------------------------------------------ relative difference prior --
//
// Gradient of V(f) = sum_r sum_{s in N(r)} w_rs phi(f_r, f_s) with the
// relative difference weighting phi(a, b) = (a - b)^2 / (a + b + gamma |a - b|)
// (Table 1): dV/df_r = 2 sum_s w_rs (f_r - f_s)(f_r + 3 f_s + gamma |f_r - f_s|)
// / (f_r + f_s + gamma |f_r - f_s|)^2 over the 26 neighbours inside the grid,
// w = 1 / distance; a pair with a zero denominator contributes 0.  One thread
// per voxel, z fastest so that a wave reads contiguous z-runs of each of the
// 27 columns it touches.
__device__ __forceinline__ float rdp_pair(float a, float b, float gamma)
{
    const float d = a - b, ad = fabsf(d);
    const float den = fmaf(gamma, ad, a + b);
    const float num = d * fmaf(gamma, ad, fmaf(3.f, b, a));
    return den > 0.f ? num * __builtin_amdgcn_rcpf(den * den) : 0.f;
}

struct RdpArgs {
    const float *f;
    float *grad;
    int N, Nz;
    float gamma;
};

// A workgroup covers a 2 x 4 x 32 (x, y, z) block of voxels; the block and
// its one-voxel halo are staged in LDS with coalesced z-runs (3.2 global
// loads per voxel instead of 27), and each voxel reads its 26 neighbours
// from there in the same order as a direct gather.
constexpr int RDP_TX = 2, RDP_TY = 4, RDP_TZ = 32;
constexpr int RDP_HX = RDP_TX + 2, RDP_HY = RDP_TY + 2, RDP_HZ = RDP_TZ + 2;

__global__ __launch_bounds__(256) void rdp_grad(RdpArgs a)
{
    __shared__ float tile[RDP_HX * RDP_HY * RDP_HZ];
    const int N = a.N, Nz = a.Nz;
    const int nzt = (Nz + RDP_TZ - 1) / RDP_TZ, nyt = (N + RDP_TY - 1) / RDP_TY;
    int blk = blockIdx.x;
    const int z0 = (blk % nzt) * RDP_TZ;
    blk /= nzt;
    const int y0 = (blk % nyt) * RDP_TY;
    const int x0 = (blk / nyt) * RDP_TX;
    for (int t = threadIdx.x; t < RDP_HX * RDP_HY * RDP_HZ; t += blockDim.x) {
        const int hz = t % RDP_HZ, hy = (t / RDP_HZ) % RDP_HY, hx = t / (RDP_HZ * RDP_HY);
        const int x = x0 + hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
        float v = 0.f;
        if ((unsigned)x < (unsigned)N && (unsigned)y < (unsigned)N && (unsigned)z < (unsigned)Nz)
            v = a.f[((size_t)x * N + y) * Nz + z];
        tile[t] = v;
    }
    __syncthreads();
    const int tz = threadIdx.x % RDP_TZ, ty = (threadIdx.x / RDP_TZ) % RDP_TY, tx = threadIdx.x / (RDP_TZ * RDP_TY);
    const int x = x0 + tx, y = y0 + ty, k = z0 + tz;
    if (x >= N || y >= N || k >= Nz) return;
    const float *c0 = tile + ((tx + 1) * RDP_HY + (ty + 1)) * RDP_HZ + tz + 1;
    const float fr = c0[0];
    const float w2 = 1.41421356237309515f / 2.f, w3 = 1.73205080756887719f / 3.f;
    float acc1 = 0.f, acc2 = 0.f, acc3 = 0.f;  // face, edge and corner neighbours
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) {
        if ((unsigned)(x + dx) >= (unsigned)N) continue;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            if ((unsigned)(y + dy) >= (unsigned)N) continue;
            const float *col = c0 + (dx * RDP_HY + dy) * RDP_HZ;
#pragma unroll
            for (int dz = -1; dz <= 1; ++dz) {
                const int nd = (dx != 0) + (dy != 0) + (dz != 0);
                if (nd == 0 || (unsigned)(k + dz) >= (unsigned)Nz) continue;
                const float t = rdp_pair(fr, col[dz], a.gamma);
                if (nd == 1) acc1 += t;
                else if (nd == 2) acc2 += t;
                else acc3 += t;
            }
        }
    }
    a.grad[((size_t)x * N + y) * Nz + k] = 2.f * (acc1 + w2 * acc2 + w3 * acc3);
}

#endif  // SPECT_HOST_TU

// Blur-class kernels: each class (KMC = 0, 4, ..., 32) is instantiated in its
// own translation unit (spect_kmc.hip compiled with -DSPECT_KMC=<class>).
typedef void (*KernelFn)(FwdArgs);
typedef void (*BackFn)(BackRotArgs);
typedef void (*FwdBatchFn)(BatchList<FwdArgs>);
typedef void (*BackBatchFn)(BatchList<BackRotArgs>);
// att is an AttMode (the forward kernel has no ATT_WRITE variant; the batched
// kernels exist for ATT_NONE and ATT_READ).
#define SPECT_DECLARE_CLASS(K)                                 \
    KernelFn fwd_kernel_kmc##K(int att, bool vec);           \
    BackFn back_kernel_kmc##K(int att, bool vec);            \
    FwdBatchFn fwd_batch_kmc##K(int att, bool vec, bool persist); \
    BackBatchFn back_batch_kmc##K(int att, bool vec, bool persist);
SPECT_DECLARE_CLASS(0)
SPECT_DECLARE_CLASS(4)
SPECT_DECLARE_CLASS(8)
SPECT_DECLARE_CLASS(12)
SPECT_DECLARE_CLASS(16)
SPECT_DECLARE_CLASS(20)
SPECT_DECLARE_CLASS(24)
SPECT_DECLARE_CLASS(28)
SPECT_DECLARE_CLASS(32)
#undef SPECT_DECLARE_CLASS

}  // namespace spectk
