// spect.hip - host side and C ABI of the SPECT projector library, plus the
// kernels that do not depend on the blur-radius class (the blur-class kernels
// are instantiated in spect_kmc.hip, compiled once per class).
#define SPECT_HOST_TU
#include "spect_device.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "spect.h"
#include "spect_internal.h"

using namespace spectk;

// ======================================================= static scratch ===
// Scratch of the allocation-free forward projection (spect_fwd_static): a
// device array of fixed size; every device holds its own copy.  Host code
// never uses the array's name as an address: the device address is looked up
// once per device (bind_static_scratch, run when a plan is created on that
// device) and kept in g_scratch_dev.
static __device__ __align__(256) char scratch[SPECT_STATIC_SCRATCH_BYTES];

// ================================================================= host ===

struct spect_plan {
    int N, Nz, A;
    double voxel_cm;
    int kmax;   // largest blur radius
    int kmc;    // compile-time radius class (multiple of 4, <= 32)
    bool one_psf;  // every angle at one detector distance: the same taps per depth
    int TS;     // tap row stride
    int device;
    int cus;            // compute units of the device
    int fwd_slots[4];   // resident forward workgroups on the device, per attenuation mode
    int back_slots[4];  // same for the rotated-frame back-projection kernel
    void *dmem;
    DevGeom g;
    // depth chunking: per boundary set (0: equal depth counts, 1: equal
    // blur work 10 + K per depth) and angle, the prefix sums wpre[set][a][i]
    // of the per-depth work over depths < i; the boundaries are uploaded to
    // g.cbnd; chunk_cost[set][nc] is the largest chunk's work over all
    // angles, in depths of average work
    int cap = 1;
    std::vector<double> wpre[2];       // [A][N + 1]
    std::vector<double> chunk_cost[2]; // [cap + 1]
    // whole reconstructions replayed as HIP graphs (see recon_graph)
    struct GraphKey {
        const void *f, *mu, *g, *s_add, *ws;
        size_t ws_bytes;
        int iters, subsets, bsrem;
        float beta, gamma;
        std::vector<float> relax;
        bool ones;  // the start image is written (1 everywhere), not read
        bool operator==(const GraphKey &o) const
        {
            return f == o.f && mu == o.mu && g == o.g && s_add == o.s_add && ws == o.ws && ws_bytes == o.ws_bytes &&
                   iters == o.iters && subsets == o.subsets && bsrem == o.bsrem && beta == o.beta &&
                   gamma == o.gamma && relax == o.relax && ones == o.ones;
        }
    };
    struct CachedGraph {
        GraphKey key;
        hipGraphExec_t exec;
    };
    mutable std::mutex graph_mu;
    mutable std::vector<CachedGraph> graphs;  // most recently used last
    mutable std::vector<GraphKey> seen;       // keys run eagerly once
    mutable hipStream_t capture_stream = nullptr;
};

namespace {

// ------------------------------------------------------------- timing ----
// Optional per-kernel timing: while enabled, every launch is bracketed by two
// HIP events recorded on the launch's own stream.

enum KernelId {
    K_TAU = 0, K_FWD, K_REDUCE, K_BACK_ROT, K_GATHER, K_FILL, K_RDP, K_SUM,
    K_FWD_B, K_REDUCE_B, K_BACK_B, K_GATHER_B, K_SENS, K_PAD, K_COUNT
};
const char *const kKernelNames[K_COUNT] = {"tau_prepass", "fwd_main", "fwd_reduce", "back_rot",
                                           "back_gather", "fill_zero", "rdp_grad", "vol_sum",
                                           "fwd_batch", "reduce_batch", "back_batch", "gather_batch",
                                           "sens_line", "pad_columns"};

struct ProfRec {
    int kernel;
    hipEvent_t a, b;
};

std::mutex g_prof_mu;
bool g_prof_on = false;
thread_local bool t_capturing = false;  // this thread is capturing a graph
std::vector<ProfRec> g_prof;

struct ProfScope {
    int kernel;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    bool on;
    // allowed = false while a stream is being captured into a graph
    ProfScope(int k, hipStream_t s, bool allowed = true) : kernel(k), st(s)
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        on = g_prof_on && allowed && !t_capturing;
        if (!on) return;
        if (hipEventCreate(&a) != hipSuccess) {
            on = false;
        } else if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            on = false;
        } else {
            (void)hipEventRecord(a, st);
        }
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
    int nslab, nchunk;
    int nchunk_b;  // depth chunks of the rotated-frame pass
};

enum { T_FWD = 1, T_BACK = 2, T_BOTH = 3 };

// Depth chunking of a launch over n_list angles: pick the chunk count that
// minimises (rounds of resident workgroups) x (depths per workgroup + a fixed
// per-workgroup cost), summed over the kernels that share the split; a last,
// partly filled round counts in proportion to its fill, up to a whole round
// at half fill (its workgroups share their CUs with fewer others and run
// faster).  The two
// passes of an OSEM step share one split when they sample the attenuation
// map (they share its chunk offsets, and splitting adds a pre-pass that
// forms them); otherwise each pass takes its own (nchunk for the forward,
// nchunk_b for the rotated-frame pass).  Only the forward's split changes
// rounding (its chunks' partial rows are summed); every depth of the
// rotated-frame pass is written by exactly one chunk.
bool samples_mu(int att) { return att == ATT_SAMPLE || att == ATT_WRITE; }
int att_of(bool mu) { return mu ? ATT_SAMPLE : ATT_NONE; }

// Chunk boundary set of the forward and rotated-frame passes: chunks of
// equal blur work (the far depths blur widest, so their chunks hold fewer
// depths), or of equal depth counts when both passes of a step sample mu and
// share the chunks' attenuation offsets (which = T_BOTH).
int chunk_set(int att, int which) { return samples_mu(att) && which == T_BOTH ? 0 : 1; }

double rounds(long wgs, int slots)
{
    const double x = (double)wgs / std::max(1, slots), whole = std::floor(x);
    return std::max(1.0, whole + std::min(1.0, 2.0 * (x - whole)));
}

Tuning tune(const spect_plan *p, int n_list, int att, int which)
{
    Tuning t;
    t.nslab = (p->Nz + SLAB - 1) / SLAB;
    const long base = (long)std::max(1, n_list) * t.nslab;
    auto best_split = [&](int passes) {
        double best = 1e300;
        int bn = 1;
        // chunks of 4 depths at the least, on average
        const int ncmax = p->cap;
        for (int nc = 1; nc <= ncmax; ++nc) {
            // the largest chunk, in depths of average work, of each pass
            const double Df = p->chunk_cost[chunk_set(att, which)][nc], Db = Df;
            const long wgs = base * nc;
            double cost = 0;
            if (passes & T_FWD) cost += rounds(wgs, p->fwd_slots[att]) * (Df + 6);
            if (passes & T_BACK) cost += rounds(wgs, p->back_slots[att]) * (Db + 6);
            // the offsets pre-pass samples mu over (nc - 1) / nc of the
            // depths, at about 0.3 of a projection's cost per depth
            if (samples_mu(att) && nc > 1)
                cost += 2 + 0.3 * (nc - 1) / nc * ((double)base / p->back_slots[att]) * p->N;
            if (cost < best - 1e-9) {
                best = cost;
                bn = nc;
            }
        }
        return bn;
    };
    if (which == T_BOTH && !samples_mu(att)) {
        t.nchunk = best_split(T_FWD);
        t.nchunk_b = best_split(T_BACK);
    } else {
        t.nchunk = t.nchunk_b = best_split(which);
    }
    return t;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Per-depth blur work (fixed part + radius) used to balance depth chunks.
constexpr double kChunkW0 = 10.0;

// Depth-chunk boundaries of one angle for nc chunks from the prefix sums
// pre[i] of its per-depth work (depths < i): b[0] = N > b[1] > ... > b[nc] =
// 0, chunk c covering depths b[c+1] .. b[c]-1 (chunk 0 touches the
// detector), each chunk's work as close to 1/nc of the angle's as whole
// depths allow.
void chunk_bounds(const double *pre, int N, int nc, int *b)
{
    const double tot = pre[N];
    b[0] = N;
    b[nc] = 0;
    for (int c = 1; c < nc; ++c) {
        // work nearer the detector than boundary i is tot - pre[i]
        const double target = tot * c / nc;
        int best = b[c - 1] - 1;
        double bd = 1e300;
        for (int i = b[c - 1] - 1; i >= nc - c; --i) {
            const double d = std::fabs((tot - pre[i]) - target);
            if (d < bd) {
                bd = d;
                best = i;
            }
        }
        b[c] = best;
    }
}

// Work of chunk c of nc chunks at angle a in boundary set `set`.
double chunk_work(const spect_plan *p, int set, int nc, int a, int c)
{
    const double *pre = p->wpre[set].data() + (size_t)a * (p->N + 1);
    std::vector<int> b(nc + 1);
    chunk_bounds(pre, p->N, nc, b.data());
    return pre[b[c]] - pre[b[c + 1]];
}

size_t tau_bytes(const spect_plan *p, const Tuning &t, int n_list, int att)
{
    if (!samples_mu(att) || t.nchunk <= 1) return 0;
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
// 4 GiB rotated-frame buffer (a whole 128^3 x 120 adjoint is one group: one
// rotated-frame launch, which then needs no depth chunks, and one gather).
int back_group(const spect_plan *p, int n_idx)
{
    const size_t per = sizeof(float) * (size_t)((p->Nz + SLAB - 1) / SLAB) * SLAB * p->N * p->N;
    size_t g = (size_t(4) << 30) / std::max<size_t>(per, 1);
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

size_t fwd_need(const spect_plan *p, int nl, int att, int which = T_FWD)
{
    const Tuning t = tune(p, nl, att, which);
    return tau_bytes(p, t, nl, att) + part_bytes(p, t, nl);
}

size_t back_need(const spect_plan *p, int nl, int att, int which = T_BACK)
{
    const Tuning t = tune(p, nl, att, which);
    return tau_bytes(p, t, nl, att) + z_bytes(p, t, nl);
}

size_t fwd_ws(const spect_plan *p, int n_idx, int att)
{
    size_t b = 0;
    for (int nl : batch_sizes(std::max(n_idx, 1), MAXL)) b = std::max(b, fwd_need(p, nl, att));
    return b;
}

size_t back_ws(const spect_plan *p, int n_idx, int att)
{
    size_t b = 0;
    const int G = back_group(p, n_idx);
    for (int nl : batch_sizes(std::max(n_idx, 1), G)) b = std::max(b, back_need(p, nl, att));
    return b;
}

// Floats of the attenuation-factor table per listed angle: [slab][i'][j'][16].
size_t table_angle_floats(const spect_plan *p)
{
    return (size_t)((p->Nz + SLAB - 1) / SLAB) * p->N * p->N * SLAB;
}

// OSEM workspace: [q][tau][partial | z]; the back pass reuses the forward's
// attenuation offsets and overwrites the partial rows.  Interleaved subsets
// have at most two sizes, floor(A/M) and ceil(A/M).
size_t osem_q_bytes(const spect_plan *p, int M)
{
    const int nl_max = (p->A + M - 1) / M;
    return align256(sizeof(float) * (size_t)nl_max * p->N * p->Nz);
}

// Whole-reconstruction workspace.  With an attenuation map the sensitivity
// pass of each subset stores its attenuation factors in a table (the
// rotated-frame brick layout, 64 bytes per angle, slab, depth and bin) and
// every later pass reads it: [sens: M volumes][table of each subset][q]
// [scratch].  Tables larger than kMaxTableBytes in total fall back to
// sampling mu in every pass, keeping each subset's chunk offsets instead:
// [sens][tau offsets of each subset][q][scratch].
constexpr size_t kMaxTableBytes = size_t(32) << 30;

size_t vol_bytes(const spect_plan *p) { return align256(sizeof(float) * (size_t)p->N * p->N * p->Nz); }

// Column stride (floats) of the reconstruction's padded copy of f, or 0 for
// none.  With columns a multiple of 512 bytes apart, the forward's
// workgroups of one slab read a fixed 64-byte slice of every column, and the
// slabs whose slice falls in the last quarter of each 512 bytes were measured
// about 10 % slower than the rest (128^3: 84-90 us per 15-angle launch
// against 73-76 us with 640-byte columns).  Only for the passes that do not
// sample mu (mu would need the same stride).
int pad_stride(const spect_plan *p, int att)
{
    if (att == ATT_SAMPLE || att == ATT_WRITE) return 0;
    return (p->Nz % 128 == 0) ? p->Nz + 32 : 0;
}

size_t pad_bytes(const spect_plan *p, int att)
{
    const int zs = pad_stride(p, att);
    return zs ? align256(sizeof(float) * (size_t)p->N * p->N * zs) : 0;
}

int subset_size(const spect_plan *p, int M, int m) { return (p->A - m + M - 1) / M; }

size_t table_bytes(const spect_plan *p, int nl)
{
    return align256(sizeof(float) * (size_t)nl * table_angle_floats(p));
}

bool use_table(const spect_plan *p, int M, bool mu)
{
    if (!mu) return false;
    size_t b = 0;
    for (int m = 0; m < M; ++m) b += table_bytes(p, subset_size(p, M, m));
    return b <= kMaxTableBytes;
}

size_t recon_tau_bytes(const spect_plan *p, int M, int m, bool mu)
{
    const int nl = subset_size(p, M, m);
    if (use_table(p, M, mu)) return table_bytes(p, nl);
    return tau_bytes(p, tune(p, nl, att_of(mu), T_BOTH), nl, att_of(mu));
}

size_t osem_ws(const spect_plan *p, int M, bool mu);

// Without attenuation the reconstruction runs the sensitivity passes of all
// subsets as one launch over every angle (subset after subset), then the
// subsets' gathers as one launch: the per-subset passes of a small object
// are too short to fill the device.  A brick of the constant projection then
// holds in-range tap sums of its depth only, so when every angle has the
// same taps the pass forms one angle's brick and the gathers read it for
// every angle; otherwise it forms a brick per angle, and only for small
// objects (the bricks of every angle within 512 MiB of workspace; larger ones
// fill the device subset by subset).
bool combined_sens(const spect_plan *p, int M, bool mu)
{
    return !mu && M > 1 && p->A <= MAXL &&
           (p->one_psf || (size_t)p->A * vol_bytes(p) <= (size_t(512) << 20));
}

// Brick volumes the combined sensitivity pass forms.
int sens_bricks(const spect_plan *p) { return p->one_psf ? 1 : p->A; }

size_t recon_ws(const spect_plan *p, int M, bool mu)
{
    size_t b = (size_t)M * vol_bytes(p);
    for (int m = 0; m < M; ++m) b += recon_tau_bytes(p, M, m, mu);
    const int att = use_table(p, M, mu) ? ATT_READ : att_of(mu);
    b += pad_bytes(p, att);
    if (!use_table(p, M, mu)) {
        size_t rest = osem_ws(p, M, mu);
        if (combined_sens(p, M, mu))
            rest = std::max(rest, osem_q_bytes(p, M) + back_need(p, sens_bricks(p), ATT_NONE, T_BACK));
        return b + rest;
    }
    size_t scratch = 0;
    for (int nl : {p->A / M, (p->A + M - 1) / M}) {
        if (nl < 1) continue;
        scratch = std::max(scratch, back_need(p, nl, ATT_WRITE, T_BACK));
        scratch = std::max(scratch, fwd_need(p, nl, ATT_READ, T_BOTH));
        scratch = std::max(scratch, back_need(p, nl, ATT_READ, T_BOTH));
    }
    return b + osem_q_bytes(p, M) + scratch;
}

size_t osem_ws(const spect_plan *p, int M, bool mu)
{
    size_t b = 0;
    for (int nl : {p->A / M, (p->A + M - 1) / M}) {
        if (nl < 1) continue;
        const Tuning t = tune(p, nl, att_of(mu), T_BOTH);
        b = std::max(b, tau_bytes(p, t, nl, att_of(mu)) + std::max(part_bytes(p, t, nl), z_bytes(p, t, nl)));
    }
    return osem_q_bytes(p, M) + b;
}

// ---------------------------------------- subiteration over an angle list --
// Workspace of osem_list_step: [q: projection rows of the list][scratch of
// one forward and one back projection of the list sharing a tuning (and the
// attenuation offsets, when mu is sampled)]; osem_list_step_vjp adds the
// rows of Hf + s and one volume in front: [e][q][volume][scratch].
size_t list_rows_bytes(const spect_plan *p, int nl) { return align256(sizeof(float) * (size_t)nl * p->N * p->Nz); }

size_t list_scratch(const spect_plan *p, int nl, int att)
{
    const Tuning t = tune(p, nl, att, T_BOTH);
    return tau_bytes(p, t, nl, att) + std::max(part_bytes(p, t, nl), z_bytes(p, t, nl));
}

size_t step_ws(const spect_plan *p, int nl, int att) { return list_rows_bytes(p, nl) + list_scratch(p, nl, att); }

size_t step_vjp_ws(const spect_plan *p, int nl, int att)
{
    return 2 * list_rows_bytes(p, nl) + vol_bytes(p) + list_scratch(p, nl, att);
}

KernelFn fwd_kernel(int att, int kmc, bool vec)
{
    switch (kmc) {
    case 0: return fwd_kernel_kmc0(att, vec);
    case 4: return fwd_kernel_kmc4(att, vec);
    case 8: return fwd_kernel_kmc8(att, vec);
    case 12: return fwd_kernel_kmc12(att, vec);
    case 16: return fwd_kernel_kmc16(att, vec);
    case 20: return fwd_kernel_kmc20(att, vec);
    case 24: return fwd_kernel_kmc24(att, vec);
    case 28: return fwd_kernel_kmc28(att, vec);
    default: return fwd_kernel_kmc32(att, vec);
    }
}

BackFn back_kernel(int att, int kmc, bool vec)
{
    switch (kmc) {
    case 0: return back_kernel_kmc0(att, vec);
    case 4: return back_kernel_kmc4(att, vec);
    case 8: return back_kernel_kmc8(att, vec);
    case 12: return back_kernel_kmc12(att, vec);
    case 16: return back_kernel_kmc16(att, vec);
    case 20: return back_kernel_kmc20(att, vec);
    case 24: return back_kernel_kmc24(att, vec);
    case 28: return back_kernel_kmc28(att, vec);
    default: return back_kernel_kmc32(att, vec);
    }
}

FwdBatchFn fwd_batch_kernel(int att, int kmc, bool vec, bool persist)
{
    switch (kmc) {
    case 0: return fwd_batch_kmc0(att, vec, persist);
    case 4: return fwd_batch_kmc4(att, vec, persist);
    case 8: return fwd_batch_kmc8(att, vec, persist);
    case 12: return fwd_batch_kmc12(att, vec, persist);
    case 16: return fwd_batch_kmc16(att, vec, persist);
    case 20: return fwd_batch_kmc20(att, vec, persist);
    case 24: return fwd_batch_kmc24(att, vec, persist);
    case 28: return fwd_batch_kmc28(att, vec, persist);
    default: return fwd_batch_kmc32(att, vec, persist);
    }
}

BackBatchFn back_batch_kernel(int att, int kmc, bool vec, bool persist)
{
    switch (kmc) {
    case 0: return back_batch_kmc0(att, vec, persist);
    case 4: return back_batch_kmc4(att, vec, persist);
    case 8: return back_batch_kmc8(att, vec, persist);
    case 12: return back_batch_kmc12(att, vec, persist);
    case 16: return back_batch_kmc16(att, vec, persist);
    case 20: return back_batch_kmc20(att, vec, persist);
    case 24: return back_batch_kmc24(att, vec, persist);
    case 28: return back_batch_kmc28(att, vec, persist);
    default: return back_batch_kmc32(att, vec, persist);
    }
}

// Threads of a forward workgroup (FQ lanes per bin) and of a rotated-frame
// back-projection workgroup (2 lanes per bin), whole waves.
int fwd_threads(int N) { return std::min(FWD_MAX_THREADS, ((FQ * N + 63) / 64) * 64); }
int block_threads(int N) { return std::min(512, ((2 * N + 63) / 64) * 64); }

size_t wb_bytes(int N, int kmc) { return sizeof(float4) * 2 * 2 * 2 * (size_t)(N + 2 * kmc); }

// Forward: the two row buffers ([2][N + 2 kmc][FQ] float4).
size_t fwd_smem(int N, int kmc) { return sizeof(float4) * 2 * FQ * (size_t)(N + 2 * kmc); }

// Row buffers plus the projection columns: N columns of SLAB + 2 kmc + 1
// floats, skewed by 8 floats per group of 8 bins.
size_t back_smem(int N, int kmc) { return wb_bytes(N, kmc) + sizeof(float) * (size_t)N * (SLAB + 2 * kmc + 2); }

// Sensitivity pass: one angle's running tap sums, N depths of TS floats.
size_t sens_smem(int N, int TS) { return sizeof(float) * (size_t)N * TS; }

size_t fwd_smem(const spect_plan *p) { return fwd_smem(p->N, p->kmc); }
size_t back_smem(const spect_plan *p) { return back_smem(p->N, p->kmc); }

// Kernels that need more than 64 KiB of dynamic LDS must say so first.
void allow_smem(const void *fn, size_t bytes)
{
    if (bytes > 65536) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

bool aligned16(const void *q) { return ((uintptr_t)q & 15) == 0; }
bool aligned8(const void *q) { return ((uintptr_t)q & 7) == 0; }

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
                bool vec, hipStream_t st, int set)
{
    TauArgs a;
    a.g = p->g;
    a.L = L;
    a.mu = mu;
    a.tau = tau;
    a.nchunk = t.nchunk;
    a.cbset = set;
    a.vec = vec;
    const int ngrp = (p->Nz + ROWS - 1) / ROWS;
    dim3 grid((p->N * ngrp + 255) / 256, t.nchunk - 1, L.n);
    ProfScope ps(K_TAU, st);
    hipLaunchKernelGGL(vec ? tau_prepass<true> : tau_prepass<false>, grid, dim3(256), 0, st, a);
}

// Forward projection of one list into partial rows, then the reduction.
// att: ATT_NONE / ATT_SAMPLE (from mu) / ATT_READ (from table).
// ws holds [tau][partial]; tau_given != nullptr reuses attenuation offsets
// already computed for the same list (the tau region is then skipped).
int run_forward(const spect_plan *p, const float *f, const float *mu, int att, const float *table,
                const AngleList &L, char *ws, size_t ws_avail, const float *tau_given, int mode, float *proj,
                const float *g, const float *s_add, float *q, bool vec, int which, hipStream_t st,
                float *e_rows = nullptr, int zs = 0)
{
    const Tuning t = tune(p, L.n, att, which);
    if (fwd_need(p, L.n, att, which) > ws_avail)
        return fail(SPECT_EINVAL, "workspace too small for a %d-angle forward launch", L.n);
    const float *tau = nullptr;
    size_t off = 0;
    const size_t tb = tau_bytes(p, t, L.n, att);
    if (tb) {
        off += tb;
        if (tau_given) {
            tau = tau_given;
        } else {
            launch_tau(p, L, t, mu, reinterpret_cast<float *>(ws), vec, st, chunk_set(att, which));
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
    a.att = table;
    a.part = part;
    a.nslab = t.nslab;
    a.nchunk = t.nchunk;
    a.cbset = chunk_set(att, which);
    a.vec = vec;
    a.zs = zs;
    a.cus = p->cus;
    KernelFn fk = fwd_kernel(att, p->kmc, vec);
    allow_smem(reinterpret_cast<const void *>(fk), fwd_smem(p));
    {
        ProfScope ps(K_FWD, st);
        hipLaunchKernelGGL(fk, dim3(t.nslab, t.nchunk, L.n), dim3(fwd_threads(p->N)), fwd_smem(p), st, a);
    }
    ReduceArgs r{};
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
    r.e = e_rows;
    {
        ProfScope ps(K_REDUCE, st);
        // slabs whose partial rows overlap one output row: at most
        // ceil((16 + 2 kmc) / 16)
        const dim3 grid((p->N * p->Nz + 255) / 256, L.n);
        if (p->kmc <= 16) hipLaunchKernelGGL(fwd_reduce<3>, grid, dim3(256), 0, st, r);
        else if (p->kmc <= 24) hipLaunchKernelGGL(fwd_reduce<4>, grid, dim3(256), 0, st, r);
        else hipLaunchKernelGGL(fwd_reduce<RED_SLABS>, grid, dim3(256), 0, st, r);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    return SPECT_OK;
}

// The gather's 16-byte output path: Nz a multiple of 4 and every array it
// touches 16-byte aligned.
bool gather_v4(const spect_plan *p, std::initializer_list<const void *> ptrs)
{
    if (p->Nz % 4) return false;
    for (const void *q : ptrs)
        if (q && reinterpret_cast<uintptr_t>(q) % 16) return false;
    return true;
}

// The gather of a back projection: the object-space sums over the list's
// angles of the rotated-frame bricks z ([L][nslab][N][N][16]), combined into
// out by `mode` (see GatherArgs).
int launch_gather(const spect_plan *p, const AngleList &L, const float *z, int nslab, int mode, float *out,
                  const float *sens, float *fpad, int zs, const BsremTerms *bt, const StepTerms *stt, hipStream_t st,
                  bool zshare = false)
{
    GatherArgs gg{};
    gg.g = p->g;
    gg.L = L;
    gg.z = z;
    gg.nslab = nslab;
    gg.mode = mode;
    gg.out = out;
    gg.sens = sens;
    gg.fpad = fpad;
    gg.zs = zs;
    gg.v4 = gather_v4(p, {out, sens, fpad, bt ? bt->sens_all : nullptr, bt ? bt->prior : nullptr});
    gg.bt = bt ? *bt : BsremTerms{nullptr, nullptr, 0.f, 0.f};
    gg.st = stt ? *stt : StepTerms{nullptr, nullptr, nullptr};
    gg.zshare = zshare ? 1 : 0;
    const int tiles = (p->N + GT - 1) / GT;
    {
        // one slab per workgroup when two would leave the device under-filled
        const bool one = (long)tiles * tiles * ((nslab + GS - 1) / GS) < 2L * p->cus;
        ProfScope ps(K_GATHER, st);
        if (one)
            hipLaunchKernelGGL(back_gather<1>, dim3(tiles * tiles, nslab), dim3(256), 0, st, gg);
        else
            hipLaunchKernelGGL(back_gather<GS>, dim3(tiles * tiles, (nslab + GS - 1) / GS), dim3(256), 0, st, gg);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "back projection launch");
    return SPECT_OK;
}

// Sensitivity gathers of the M interleaved subsets of La (every angle,
// subset after subset) in one launch: subset m's sum into
// sens0 + m * out_stride (see back_gather_subsets); zshare: one brick volume
// at z serves every angle.
int launch_gather_subsets(const spect_plan *p, const AngleList &La, const float *z, int nslab, int M, float *sens0,
                          size_t out_stride, bool zshare, hipStream_t st)
{
    GatherArgs gg{};
    gg.g = p->g;
    gg.L = La;
    gg.z = z;
    gg.nslab = nslab;
    gg.mode = 0;
    gg.out = sens0;
    gg.zshare = zshare ? 1 : 0;
    gg.v4 = gather_v4(p, {sens0}) && (out_stride % 4 == 0);
    const int tiles = (p->N + GT - 1) / GT;
    {
        const bool one = (long)tiles * tiles * ((nslab + GS - 1) / GS) * M < 2L * p->cus;
        ProfScope ps(K_GATHER, st);
        if (one)
            hipLaunchKernelGGL(back_gather_subsets<1>, dim3(tiles * tiles, nslab, M), dim3(256), 0, st, gg, M,
                               out_stride);
        else
            hipLaunchKernelGGL(back_gather_subsets<GS>, dim3(tiles * tiles, (nslab + GS - 1) / GS, M), dim3(256), 0,
                               st, gg, M, out_stride);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPECT_OK : hip_fail(e, "sensitivity gather launch");
}

// Back projection of one list: rotated-frame pass, then the gather.
// att: ATT_NONE / ATT_SAMPLE / ATT_WRITE (sample mu and fill table) /
// ATT_READ (from table).  ws holds [tau][z]; tau_given as in run_forward.
int run_back(const spect_plan *p, const float *y, int y_compact, int ones, const float *mu, int att,
             float *table, const AngleList &L, char *ws, size_t ws_avail, const float *tau_given, int mode,
             float *out, const float *sens, bool vec, int which, hipStream_t st, const BsremTerms *bt = nullptr,
             const StepTerms *stt = nullptr, float *fpad = nullptr, int zs = 0, bool do_gather = true,
             float *fill = nullptr)
{
    const Tuning t = tune(p, L.n, att, which);
    if (back_need(p, L.n, att, which) > ws_avail)
        return fail(SPECT_EINVAL, "workspace too small for a %d-angle back-projection launch", L.n);
    const float *tau = nullptr;
    size_t off = 0;
    // the sensitivity pass (ones) keeps one running attenuation sum per
    // thread and needs no chunk offsets
    const size_t tb = ones ? 0 : tau_bytes(p, t, L.n, att);
    if (tb) {
        off += tb;
        if (tau_given) {
            tau = tau_given;
        } else {
            launch_tau(p, L, t, mu, reinterpret_cast<float *>(ws), vec, st, chunk_set(att, which));
            tau = reinterpret_cast<const float *>(ws);
        }
    }
    float *z = reinterpret_cast<float *>(ws + off);
    BackRotArgs b{};
    b.g = p->g;
    b.L = L;
    b.y = y;
    b.y_compact = y_compact;
    b.ones = ones;
    b.mu = mu;
    b.tau = tau;
    b.att = table;
    b.z = z;
    b.nslab = t.nslab;
    b.nchunk = t.nchunk_b;
    b.cbset = chunk_set(att, which);
    b.vec = vec;
    if (ones) {
        // constant projection: the blur reduces to in-range tap sums, and the
        // pass walks every depth in one thread (no chunk offsets)
        const bool v2 = p->Nz % 2 == 0 && (mu == nullptr || aligned8(mu));
        // the sensitivity launch may also write a start image of ones
        b.fill = fill;
        b.fill_n = fill ? (size_t)p->N * p->N * p->Nz : 0;
        BackFn sk = nullptr;
        if (att == ATT_WRITE) sk = v2 ? sens_line<ATT_WRITE, true> : sens_line<ATT_WRITE, false>;
        else if (att == ATT_SAMPLE) sk = v2 ? sens_line<ATT_SAMPLE, true> : sens_line<ATT_SAMPLE, false>;
        else if (att == ATT_NONE) sk = sens_line<ATT_NONE, false>;
        if (!sk) return fail(SPECT_EINVAL, "no sensitivity pass for attenuation mode %d", att);
        const int nblk = (p->N * (SLAB / 2) + SL_THREADS - 1) / SL_THREADS;
        // without attenuation the depths are independent: split them into
        // chunks until the launch fills the device (2 blocks per CU)
        b.nchunk = 1;
        if (att == ATT_NONE) {
            const long blocks = (long)nblk * t.nslab * L.n;
            b.nchunk = (int)std::min<long>(std::max(1, p->N / 2), (2L * p->cus + blocks - 1) / blocks);
            b.nchunk = std::max(1, b.nchunk);
        }
        b.cbset = 0;
        const size_t smem = sens_smem(p->N, p->TS);
        allow_smem(reinterpret_cast<const void *>(sk), smem);
        ProfScope ps(K_SENS, st);
        hipLaunchKernelGGL(sk, dim3(nblk * b.nchunk, t.nslab, L.n), dim3(SL_THREADS), smem, st, b);
    } else {
        BackFn bk = back_kernel(att, p->kmc, vec);
        allow_smem(reinterpret_cast<const void *>(bk), back_smem(p));
        ProfScope ps(K_BACK_ROT, st);
        hipLaunchKernelGGL(bk, dim3(t.nslab, t.nchunk_b, L.n), dim3(block_threads(p->N)), back_smem(p), st, b);
    }
    if (!do_gather) {
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? SPECT_OK : hip_fail(e, "back projection launch");
    }
    return launch_gather(p, L, z, t.nslab, mode, out, sens, fpad, zs, bt, stt, st);
}

// grad = gradient of the relative difference prior at f (weight gamma).
int launch_rdp(const spect_plan *p, const float *f, float *grad, float gamma, hipStream_t st)
{
    RdpArgs a{f, grad, p->N, p->Nz, gamma};
    // one workgroup per 2 x 4 x 32 block of voxels (x, y, z)
    const size_t nblk = (size_t)((p->N + RDP_TX - 1) / RDP_TX) * ((p->N + RDP_TY - 1) / RDP_TY) *
                        ((p->Nz + RDP_TZ - 1) / RDP_TZ);
    {
        ProfScope ps(K_RDP, st);
        hipLaunchKernelGGL(rdp_grad, dim3((unsigned)nblk), dim3(256), 0, st, a);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPECT_OK : hip_fail(e, "prior gradient launch");
}

// out = sum of n volumes of the plan's size spaced `stride` floats apart.
int launch_sum(const spect_plan *p, const float *first, size_t stride, int n, float *out, hipStream_t st)
{
    const size_t count = (size_t)p->N * p->N * p->Nz;
    {
        ProfScope ps(K_SUM, st);
        hipLaunchKernelGGL(vol_sum, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, first, stride, n, out,
                           count);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPECT_OK : hip_fail(e, "volume sum launch");
}

// dst = src with columns zs floats apart (the reconstruction's padded f).
int launch_pad(const spect_plan *p, const float *src, float *dst, int zs, hipStream_t st)
{
    const size_t ncol = (size_t)p->N * p->N, n4 = ncol * (p->Nz / 4);
    {
        ProfScope ps(K_PAD, st);
        hipLaunchKernelGGL(pad_columns, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, st,
                           reinterpret_cast<const float4 *>(src), reinterpret_cast<float4 *>(dst), ncol, p->Nz / 4,
                           zs / 4);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPECT_OK : hip_fail(e, "padded copy launch");
}

int clear(float *p, size_t n, hipStream_t st)
{
    ProfScope ps(K_FILL, st);
    hipLaunchKernelGGL(fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPECT_OK : hip_fail(e, "clear launch");
}

std::mutex g_scratch_mu;
std::vector<char *> g_scratch_dev;  // device address of `scratch`, per device id

// Look up this device's copy of the static scratch array (the device must be
// current); done once per device.
int bind_static_scratch(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < 0) return fail(SPECT_EHIP, "invalid device %d", device);
    if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize(device + 1, nullptr);
    if (g_scratch_dev[device]) return SPECT_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "device address of the static scratch array");
    if (!ptr || ((uintptr_t)ptr & 255)) return fail(SPECT_EHIP, "static scratch array has no usable address");
    g_scratch_dev[device] = static_cast<char *>(ptr);
    return SPECT_OK;
}

char *static_scratch(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return device >= 0 && device < (int)g_scratch_dev.size() ? g_scratch_dev[device] : nullptr;
}

bool want_vec(const spect_plan *p, std::initializer_list<const void *> ptrs)
{
    if (p->Nz % 4) return false;
    for (const void *q : ptrs)
        if (q && !aligned16(q)) return false;
    return true;
}

}  // namespace

// Error reporting for the other host translation units (spect_internal.h).
namespace spect_internal {
int set_error(int code, const char *msg) { return fail(code, "%s", msg); }
int clear_error() { return ok(); }
}  // namespace spect_internal

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
    // kernels address a volume with 32-bit byte offsets and 24-bit row products
    if (vol >= 536870912.0) return fail(SPECT_EUNSUPPORTED, "object of 2^29 voxels or more");
    if (prj >= 2147483647.0) return fail(SPECT_EUNSUPPORTED, "projection element count exceeds 2^31");
    if (g.nz >= (1 << 22)) return fail(SPECT_EUNSUPPORTED, "nz = %d is 2^22 or more", g.nz);
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
    p->one_psf = std::all_of(rad.begin(), rad.end(), [&](double r) { return r == rad[0]; });
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
    std::vector<float> taps((size_t)A * N * p->TS, 0.f), ctaps((size_t)A * N * p->TS, 0.f);
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
            double run = 0.0;
            for (int m = 0; m < p->TS; ++m) {
                if (m <= K) {
                    taps[((size_t)i * N + ip) * p->TS + m] = (float)t[m];
                    run += t[m];
                }
                ctaps[((size_t)i * N + ip) * p->TS + m] = (float)run;
            }
        }
    }
    // depth chunking: per-depth work 10 + K, boundaries per chunk count and
    // angle (at least 4 depths per chunk on average)
    p->cap = std::max(1, N / 4);
    const int cap = p->cap;
    std::vector<int> cb((size_t)2 * cap * A * (cap + 1), 0);
    for (int set = 0; set < 2; ++set) {
        std::vector<double> &wp = p->wpre[set];
        wp.assign((size_t)A * (N + 1), 0.0);
        for (int i = 0; i < A; ++i)
            for (int ip = 0; ip < N; ++ip)
                wp[(size_t)i * (N + 1) + ip + 1] =
                    wp[(size_t)i * (N + 1) + ip] + (set == 0 ? 1.0 : kChunkW0 + kd[(size_t)i * N + ip]);
        p->chunk_cost[set].assign(cap + 1, 0.0);
        for (int nc = 1; nc <= cap; ++nc)
            for (int i = 0; i < A; ++i) {
                int *b = cb.data() + (((size_t)set * cap + nc - 1) * A + i) * (cap + 1);
                const double *pre = wp.data() + (size_t)i * (N + 1);
                chunk_bounds(pre, N, nc, b);
                const double avg = pre[N] / N;
                for (int c = 0; c < nc; ++c)
                    p->chunk_cost[set][nc] = std::max(p->chunk_cost[set][nc], (pre[b[c]] - pre[b[c + 1]]) / avg);
            }
    }
    const size_t b_cs = align256(sizeof(float2) * A), b_xy = align256(sizeof(float2) * (size_t)A * N);
    const size_t b_kd = align256(sizeof(int) * (size_t)A * N), b_tp = align256(sizeof(float) * taps.size());
    const size_t b_cb = align256(sizeof(int) * cb.size());
    hipError_t e = hipMalloc(&p->dmem, b_cs + b_xy + b_kd + 2 * b_tp + b_cb);
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
    if (e == hipSuccess)
        e = hipMemcpy(base + b_cs + b_xy + b_kd + b_tp, ctaps.data(), sizeof(float) * ctaps.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(base + b_cs + b_xy + b_kd + 2 * b_tp, cb.data(), sizeof(int) * cb.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p->dmem);
        delete p;
        return hip_fail(e, "upload of plan tables");
    }
    p->g.cs = reinterpret_cast<const float2 *>(base);
    p->g.xy0 = reinterpret_cast<const float2 *>(base + b_cs);
    p->g.kdep = reinterpret_cast<const int *>(base + b_cs + b_xy);
    p->g.taps = reinterpret_cast<const float *>(base + b_cs + b_xy + b_kd);
    p->g.ctaps = reinterpret_cast<const float *>(base + b_cs + b_xy + b_kd + b_tp);
    p->g.cbnd = reinterpret_cast<const int *>(base + b_cs + b_xy + b_kd + 2 * b_tp);
    p->g.cap = cap;
    p->g.N = N;
    p->g.Nz = g.nz;
    p->g.A = A;
    p->g.TS = p->TS;
    p->g.tau_scale = (float)(g.voxel_cm / std::log(2.0));
    // resident workgroups per device for the chunk tuning
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || cus < 1)
        cus = 256;
    p->cus = cus;
    for (int att = ATT_NONE; att <= ATT_READ; ++att) {
        int nb = 0;
        const void *fk = reinterpret_cast<const void *>(fwd_kernel(att == ATT_WRITE ? ATT_SAMPLE : att, p->kmc, true));
        allow_smem(fk, fwd_smem(p));
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fk, fwd_threads(N), fwd_smem(p)) != hipSuccess)
            nb = 1;
        p->fwd_slots[att] = std::max(1, nb) * cus;
        const void *bk = reinterpret_cast<const void *>(back_kernel(att, p->kmc, true));
        allow_smem(bk, back_smem(p));
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bk, block_threads(N), back_smem(p)) != hipSuccess)
            nb = 1;
        p->back_slots[att] = std::max(1, nb) * cus;
    }
    (void)hipGetLastError();
    // the library's per-device set-up: the static scratch array's address
    if (const int st = bind_static_scratch(p->device)) {
        spect_plan_destroy(p);
        return st;
    }
    *out = p;
    return ok();
}

int spect_plan_destroy(spect_plan *plan)
{
    if (!plan) return ok();
    if (plan->dmem) (void)hipFree(plan->dmem);
    for (auto &c : plan->graphs) (void)hipGraphExecDestroy(c.exec);
    if (plan->capture_stream) (void)hipStreamDestroy(plan->capture_stream);
    delete plan;
    return ok();
}

int spect_workspace_size(const spect_plan *plan, int op, int32_t n_idx, int with_mu, size_t *bytes)
{
    if (!plan) return fail(SPECT_EINVAL, "plan is NULL");
    if (!bytes) return fail(SPECT_EINVAL, "bytes is NULL");
    if (n_idx < 1) return fail(SPECT_EINVAL, "n_idx must be >= 1");
    if (with_mu < 0 || with_mu > SPECT_ATT_TABLE) return fail(SPECT_EINVAL, "with_mu = %d outside [0, 2]", with_mu);
    const bool mu = with_mu != 0;
    const bool tab = with_mu == SPECT_ATT_TABLE;
    if (tab && op != SPECT_OP_FWD && op != SPECT_OP_BACK && op != SPECT_OP_SENS && op != SPECT_OP_STEP &&
        op != SPECT_OP_STEP_VJP)
        return fail(SPECT_EINVAL,
                    "with_mu = SPECT_ATT_TABLE applies to SPECT_OP_FWD, _BACK, _SENS, _STEP and _STEP_VJP only");
    switch (op) {
    case SPECT_OP_FWD: *bytes = fwd_ws(plan, n_idx, tab ? ATT_READ : att_of(mu)); break;
    case SPECT_OP_BACK: *bytes = back_ws(plan, n_idx, tab ? ATT_READ : att_of(mu)); break;
    case SPECT_OP_SENS: *bytes = back_ws(plan, n_idx, tab ? ATT_WRITE : att_of(mu)); break;
    case SPECT_OP_OSEM:
        if (n_idx > plan->A) return fail(SPECT_EINVAL, "n_subsets %d exceeds n_angles %d", n_idx, plan->A);
        *bytes = osem_ws(plan, n_idx, mu);
        break;
    case SPECT_OP_RECON:
        if (n_idx > plan->A) return fail(SPECT_EINVAL, "n_subsets %d exceeds n_angles %d", n_idx, plan->A);
        *bytes = recon_ws(plan, n_idx, mu);
        break;
    case SPECT_OP_BSREM_STEP:
        if (n_idx > plan->A) return fail(SPECT_EINVAL, "n_subsets %d exceeds n_angles %d", n_idx, plan->A);
        *bytes = vol_bytes(plan) + osem_ws(plan, n_idx, mu);
        break;
    case SPECT_OP_BSREM:
        if (n_idx > plan->A) return fail(SPECT_EINVAL, "n_subsets %d exceeds n_angles %d", n_idx, plan->A);
        *bytes = recon_ws(plan, n_idx, mu) + 2 * vol_bytes(plan);
        break;
    case SPECT_OP_STEP:
    case SPECT_OP_STEP_VJP: {
        if (n_idx > MAXL) return fail(SPECT_EUNSUPPORTED, "a subiteration over more than %d angles", MAXL);
        const int att = tab ? ATT_READ : att_of(mu);
        *bytes = op == SPECT_OP_STEP ? step_ws(plan, n_idx, att) : step_vjp_ws(plan, n_idx, att);
        break;
    }
    default: return fail(SPECT_EINVAL, "unknown op %d", op);
    }
    return ok();
}

}  // extern "C"

namespace {

// Shared bodies of the projector calls.  table == nullptr: attenuation from
// mu (or none); otherwise the factors of the listed angles are read from
// (forward, adjoint) or written to (sensitivity) the table, whose list
// position i starts at table + i * table_angle_floats.
int do_fwd(const spect_plan *plan, const float *f, const float *mu, const float *table, float *proj,
           const int32_t *angle_idx, int32_t n_idx, void *ws, size_t ws_bytes, void *stream)
{
    int st;
    if ((st = check_plan(plan))) return st;
    if ((st = check_ptr(f, "f", false)) || (st = check_ptr(proj, "proj", false))) return st;
    std::vector<int> list;
    if ((st = make_list(plan, angle_idx, n_idx, &list))) return st;
    if (list.empty()) return ok();
    const int att = table ? ATT_READ : att_of(mu != nullptr);
    if ((st = check_ws(ws, ws_bytes, fwd_ws(plan, (int)list.size(), att)))) return st;
    const bool vec = want_vec(plan, {f, mu});
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (size_t b = 0; b < list.size(); b += MAXL) {
        const int n = (int)std::min<size_t>(MAXL, list.size() - b);
        const AngleList L = to_list(list.data() + b, n);
        const float *tb = table ? table + b * table_angle_floats(plan) : nullptr;
        if ((st = run_forward(plan, f, mu, att, tb, L, static_cast<char *>(ws), ws_bytes, nullptr, 0, proj,
                              nullptr, nullptr, nullptr, vec, T_FWD, s)))
            return st;
    }
    return ok();
}

int do_back(const spect_plan *plan, const float *proj, const float *mu, const float *table, float *f_out,
            const int32_t *angle_idx, int32_t n_idx, int accumulate, void *ws, size_t ws_bytes, void *stream)
{
    int st;
    if ((st = check_plan(plan))) return st;
    if ((st = check_ptr(proj, "proj", false)) || (st = check_ptr(f_out, "f_out", false))) return st;
    std::vector<int> list;
    if ((st = make_list(plan, angle_idx, n_idx, &list))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (list.empty()) {
        if (accumulate) return ok();
        return (st = clear(f_out, (size_t)plan->N * plan->N * plan->Nz, s)) ? st : ok();
    }
    const int att = table ? ATT_READ : att_of(mu != nullptr);
    if ((st = check_ws(ws, ws_bytes, back_ws(plan, (int)list.size(), att)))) return st;
    const bool vec = want_vec(plan, {mu});
    const int G = back_group(plan, (int)list.size());
    for (size_t b = 0; b < list.size(); b += G) {
        const int n = (int)std::min<size_t>(G, list.size() - b);
        const AngleList L = to_list(list.data() + b, n);
        const int mode = (b == 0 && !accumulate) ? 0 : 1;
        float *tb = table ? const_cast<float *>(table) + b * table_angle_floats(plan) : nullptr;
        if ((st = run_back(plan, proj, 0, 0, mu, att, tb, L, static_cast<char *>(ws), ws_bytes, nullptr, mode,
                           f_out, nullptr, vec, T_BACK, s)))
            return st;
    }
    return ok();
}

int do_sens(const spect_plan *plan, const float *mu, float *sens, float *table, const int32_t *angle_idx,
            int32_t n_idx, void *ws, size_t ws_bytes, void *stream)
{
    int st;
    if ((st = check_plan(plan))) return st;
    if ((st = check_ptr(sens, "sens", false))) return st;
    std::vector<int> list;
    if ((st = make_list(plan, angle_idx, n_idx, &list))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (list.empty()) return (st = clear(sens, (size_t)plan->N * plan->N * plan->Nz, s)) ? st : ok();
    const int att = table ? ATT_WRITE : att_of(mu != nullptr);
    if ((st = check_ws(ws, ws_bytes, back_ws(plan, (int)list.size(), att)))) return st;
    const bool vec = want_vec(plan, {mu});
    const int G = back_group(plan, (int)list.size());
    if (att == ATT_NONE && plan->one_psf) {
        // no attenuation and the same taps for every angle: one angle's brick
        // of the constant projection serves every angle's gather
        char *w = static_cast<char *>(ws);
        const AngleList L1 = to_list(list.data(), 1);
        if ((st = run_back(plan, nullptr, 0, 1, nullptr, ATT_NONE, nullptr, L1, w, ws_bytes, nullptr, 0, nullptr,
                           nullptr, vec, T_BACK, s, nullptr, nullptr, nullptr, 0, false)))
            return st;
        const int nslab = tune(plan, 1, ATT_NONE, T_BACK).nslab;
        for (size_t b = 0; b < list.size(); b += G) {
            const int n = (int)std::min<size_t>(G, list.size() - b);
            if ((st = launch_gather(plan, to_list(list.data() + b, n), reinterpret_cast<const float *>(w), nslab,
                                    b == 0 ? 0 : 1, sens, nullptr, nullptr, 0, nullptr, nullptr, s, true)))
                return st;
        }
        return ok();
    }
    for (size_t b = 0; b < list.size(); b += G) {
        const int n = (int)std::min<size_t>(G, list.size() - b);
        const AngleList L = to_list(list.data() + b, n);
        float *tb = table ? table + b * table_angle_floats(plan) : nullptr;
        if ((st = run_back(plan, nullptr, 0, 1, mu, att, tb, L, static_cast<char *>(ws), ws_bytes, nullptr,
                           b == 0 ? 0 : 1, sens, nullptr, vec, T_BACK, s)))
            return st;
    }
    return ok();
}

int check_table(const float *table)
{
    if (!table) return fail(SPECT_EINVAL, "table is NULL");
    if ((uintptr_t)table & 15) return fail(SPECT_EINVAL, "table is not 16-byte aligned");
    return SPECT_OK;
}

// The angle list of a subiteration: 1 to MAXL distinct angles.
int step_list(const spect_plan *p, const int32_t *idx, int32_t n_idx, std::vector<int> *list)
{
    int st;
    if ((st = make_list(p, idx, n_idx, list))) return st;
    if (list->empty()) return fail(SPECT_EINVAL, "the angle list is empty");
    if ((int)list->size() > MAXL) return fail(SPECT_EUNSUPPORTED, "a subiteration over more than %d angles", MAXL);
    std::vector<char> seen(p->A, 0);
    for (int n : *list)
        if (seen[n]++) return fail(SPECT_EINVAL, "angle %d is listed twice", n);
    return SPECT_OK;
}

// Attenuation of a subiteration call: at most one of mu and table.
int step_att(const float *mu, const float *table, int *att)
{
    if (mu && table) return fail(SPECT_EINVAL, "pass an attenuation map or a table, not both");
    if (table) {
        const int st = check_table(table);
        if (st) return st;
    }
    *att = table ? ATT_READ : att_of(mu != nullptr);
    return SPECT_OK;
}

}  // namespace

extern "C" {

int spect_fwd(const spect_plan *plan, const float *f, const float *mu, float *proj,
              const int32_t *angle_idx, int32_t n_idx, void *ws, size_t ws_bytes, void *stream)
{
    const int st = check_ptr(mu, "mu", true);
    return st ? st : do_fwd(plan, f, mu, nullptr, proj, angle_idx, n_idx, ws, ws_bytes, stream);
}

int spect_fwd_static(const spect_plan *plan, const float *f, const float *mu, float *proj,
                     const int32_t *angle_idx, int32_t n_idx, void *stream)
{
    int st;
    if ((st = check_plan(plan))) return st;
    if ((st = check_ptr(mu, "mu", true))) return st;
    std::vector<int> list;
    if ((st = make_list(plan, angle_idx, n_idx, &list))) return st;
    if (list.empty()) return ok();
    const size_t need = fwd_ws(plan, (int)list.size(), att_of(mu != nullptr));
    if (need > SPECT_STATIC_SCRATCH_BYTES)
        return fail(SPECT_EINVAL, "%zu angles need %zu scratch bytes; the static scratch holds %zu",
                    list.size(), need, (size_t)SPECT_STATIC_SCRATCH_BYTES);
    char *ws = static_scratch(plan->device);
    if (!ws) return fail(SPECT_EHIP, "static scratch not set up on device %d", plan->device);
    return do_fwd(plan, f, mu, nullptr, proj, angle_idx, n_idx, ws, SPECT_STATIC_SCRATCH_BYTES, stream);
}

int spect_back(const spect_plan *plan, const float *proj, const float *mu, float *f_out,
               const int32_t *angle_idx, int32_t n_idx, int accumulate, void *ws, size_t ws_bytes,
               void *stream)
{
    const int st = check_ptr(mu, "mu", true);
    return st ? st : do_back(plan, proj, mu, nullptr, f_out, angle_idx, n_idx, accumulate, ws, ws_bytes, stream);
}

int spect_sensitivity(const spect_plan *plan, const float *mu, float *sens, const int32_t *angle_idx,
                      int32_t n_idx, void *ws, size_t ws_bytes, void *stream)
{
    const int st = check_ptr(mu, "mu", true);
    return st ? st : do_sens(plan, mu, sens, nullptr, angle_idx, n_idx, ws, ws_bytes, stream);
}

int spect_table_size(const spect_plan *plan, int32_t n_idx, size_t *bytes)
{
    if (!plan) return fail(SPECT_EINVAL, "plan is NULL");
    if (!bytes) return fail(SPECT_EINVAL, "bytes is NULL");
    if (n_idx < 0) return fail(SPECT_EINVAL, "n_idx = %d is negative", n_idx);
    *bytes = sizeof(float) * (size_t)n_idx * table_angle_floats(plan);
    return ok();
}

int spect_sensitivity_table(const spect_plan *plan, const float *mu, float *sens, float *table,
                            const int32_t *angle_idx, int32_t n_idx, void *ws, size_t ws_bytes, void *stream)
{
    int st;
    if ((st = check_ptr(mu, "mu", false)) || (st = check_table(table))) return st;
    return do_sens(plan, mu, sens, table, angle_idx, n_idx, ws, ws_bytes, stream);
}

int spect_fwd_table(const spect_plan *plan, const float *f, const float *table, float *proj,
                    const int32_t *angle_idx, int32_t n_idx, void *ws, size_t ws_bytes, void *stream)
{
    const int st = check_table(table);
    return st ? st : do_fwd(plan, f, nullptr, table, proj, angle_idx, n_idx, ws, ws_bytes, stream);
}

int spect_back_table(const spect_plan *plan, const float *proj, const float *table, float *f_out,
                     const int32_t *angle_idx, int32_t n_idx, int accumulate, void *ws, size_t ws_bytes,
                     void *stream)
{
    const int st = check_table(table);
    return st ? st : do_back(plan, proj, nullptr, table, f_out, angle_idx, n_idx, accumulate, ws, ws_bytes, stream);
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
    if ((st = run_forward(plan, f, mu, att_of(mu), nullptr, L, rest, avail, nullptr, 1, nullptr, g, s_add, q, vec, T_BOTH, s)))
        return st;
    // same list, same tuning: the attenuation offsets at the start of rest are reused
    if ((st = run_back(plan, q, 1, 0, mu, att_of(mu), nullptr, L, rest, avail, reinterpret_cast<const float *>(rest), 2, f, sens_m,
                       vec, T_BOTH, s)))
        return st;
    return ok();
}

}  // extern "C"

namespace {

// Whole reconstructions as HIP graphs.  A reconstruction's launches depend
// only on the plan and on its arguments, so the second call with the same
// arguments (array addresses, workspace, iteration and subset counts, BSREM
// parameters) captures them into a graph on the plan's capture stream, and
// later calls replay it on the caller's stream: one submission instead of
// four or five kernel launches per subiteration.  Calls with new arguments
// launch eagerly, as do all calls while kernel timing is on.  The plan keeps
// the kGraphs most recently used graphs.
constexpr size_t kGraphs = 8;

template <class Launch>
int recon_graph(const spect_plan *plan, const spect_plan::GraphKey &key, Launch &launch_all, hipStream_t s)
{
    bool timing;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        timing = g_prof_on;
    }
    if (timing) return launch_all(s);  // (the launches take g_prof_mu themselves)
    std::lock_guard<std::mutex> lk(plan->graph_mu);
    auto &G = plan->graphs;
    for (size_t i = 0; i < G.size(); ++i) {
        if (!(G[i].key == key)) continue;
        std::rotate(G.begin() + i, G.begin() + i + 1, G.end());
        const hipError_t e = hipGraphLaunch(G.back().exec, s);
        return e == hipSuccess ? ok() : hip_fail(e, "reconstruction graph launch");
    }
    auto &seen = plan->seen;
    const auto it = std::find(seen.begin(), seen.end(), key);
    if (it == seen.end()) {
        if (seen.size() >= kGraphs) seen.erase(seen.begin());
        seen.push_back(key);
        return launch_all(s);
    }
    seen.erase(it);
    if (!plan->capture_stream && hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        plan->capture_stream = nullptr;
        (void)hipGetLastError();
        return launch_all(s);
    }
    if (hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        (void)hipGetLastError();
        return launch_all(s);
    }
    t_capturing = true;
    const int st = launch_all(plan->capture_stream);
    t_capturing = false;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(plan->capture_stream, &graph);
    if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess && graph) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess || !exec) {
        (void)hipGetLastError();
        return launch_all(s);
    }
    if (G.size() >= kGraphs) {
        (void)hipGraphExecDestroy(G.front().exec);
        G.erase(G.begin());
    }
    G.push_back({key, exec});
    e = hipGraphLaunch(exec, s);
    return e == hipSuccess ? ok() : hip_fail(e, "reconstruction graph launch");
}

// BSREM parameters of a whole reconstruction (nullptr: OSEM).
struct BsremSpec {
    float beta, gamma;
    const float *relax;  // host, one relaxation per iteration; nullptr: 1 / (1 + k)
};

bool finite_nonneg(float x) { return std::isfinite(x) && x >= 0.f; }

// Whole reconstruction: subset sensitivities (and attenuation tables), then
// n_iters x M subiterations, each an OSEM update or, with bs, the BSREM
// update with the relative difference prior.  Workspace as recon_ws, plus
// two volumes (all-angle sensitivity, prior gradient) for BSREM right after
// the M sensitivities.
int reconstruct(const spect_plan *plan, float *f, const float *mu, const float *g, const float *s_add,
                int32_t n_iters, int32_t n_subsets, void *ws, size_t ws_bytes, void *stream, const BsremSpec *bs,
                bool from_ones = false)
{
    int st;
    if ((st = check_plan(plan))) return st;
    if ((st = check_ptr(f, "f", false)) || (st = check_ptr(mu, "mu", true)) || (st = check_ptr(g, "g", false)) ||
        (st = check_ptr(s_add, "s_add", true)))
        return st;
    if (n_subsets < 1 || n_subsets > plan->A)
        return fail(SPECT_EINVAL, "n_subsets = %d outside [1, %d]", n_subsets, plan->A);
    if (n_iters < 0) return fail(SPECT_EINVAL, "n_iters = %d is negative", n_iters);
    if (bs) {
        if (!finite_nonneg(bs->beta) || !finite_nonneg(bs->gamma))
            return fail(SPECT_EINVAL, "beta and gamma must be finite and >= 0");
        for (int k = 0; bs->relax && k < n_iters; ++k)
            if (!(std::isfinite(bs->relax[k]) && bs->relax[k] > 0.f))
                return fail(SPECT_EINVAL, "relaxation[%d] must be finite and > 0", k);
    }
    const int M = n_subsets;
    const int nl_max = (plan->A + M - 1) / M;
    if (nl_max > MAXL) return fail(SPECT_EUNSUPPORTED, "subsets of more than %d angles", MAXL);
    const size_t vb = vol_bytes(plan);
    const size_t extra = bs ? 2 * vb : 0;
    if ((st = check_ws(ws, ws_bytes, recon_ws(plan, M, mu != nullptr) + extra))) return st;
    spect_plan::GraphKey key{f, mu, g, s_add, ws, ws_bytes, n_iters, n_subsets, bs ? (bs->relax ? 2 : 1) : 0,
                             bs ? bs->beta : 0.f, bs ? bs->gamma : 0.f, {}, from_ones};
    // from_ones: the first sensitivity launch also writes f = 1 (no launch
    // reads f before it)
    float *const fill = from_ones ? f : nullptr;
    if (bs && bs->relax) key.relax.assign(bs->relax, bs->relax + n_iters);
    auto launch_all = [&](hipStream_t s) -> int {
        const bool vec = want_vec(plan, {f, mu});
        char *w = static_cast<char *>(ws);
        const bool table = use_table(plan, M, mu != nullptr);
        const int att = table ? ATT_READ : att_of(mu != nullptr);
        std::vector<float *> sens(M), per(M, nullptr);  // per subset: attenuation table or chunk offsets
        for (int m = 0; m < M; ++m) sens[m] = reinterpret_cast<float *>(w + (size_t)m * vb);
        float *sens_all = bs ? reinterpret_cast<float *>(w + (size_t)M * vb) : nullptr;
        float *prior = bs ? reinterpret_cast<float *>(w + (size_t)M * vb + vb) : nullptr;
        size_t off = (size_t)M * vb + extra;
        std::vector<AngleList> lists(M);
        for (int m = 0; m < M; ++m) {
            std::vector<int> list;
            for (int n = m; n < plan->A; n += M) list.push_back(n);
            lists[m] = to_list(list.data(), (int)list.size());
            const size_t tb = recon_tau_bytes(plan, M, m, mu != nullptr);
            if (tb) per[m] = reinterpret_cast<float *>(w + off);
            if (tb && !table)
                launch_tau(plan, lists[m], tune(plan, lists[m].n, ATT_SAMPLE, T_BOTH), mu, per[m], vec, s,
                           chunk_set(ATT_SAMPLE, T_BOTH));
            off += tb;
        }
        float *q = reinterpret_cast<float *>(w + off);
        const size_t qb = osem_q_bytes(plan, M);
        // the forward's padded copy of f, kept current by the updates
        const int zs = pad_stride(plan, att);
        const size_t pb = pad_bytes(plan, att);
        float *fpad = zs ? reinterpret_cast<float *>(w + off + qb) : nullptr;
        char *rest = w + off + qb + pb;
        const size_t avail = ws_bytes - off - qb - pb;
        // subset sensitivities H_m^T 1; with a table this pass also fills it
        if (combined_sens(plan, M, mu != nullptr)) {
            std::vector<int> all;
            for (int m = 0; m < M; ++m) all.insert(all.end(), lists[m].idx, lists[m].idx + lists[m].n);
            const AngleList La = to_list(all.data(), (int)all.size());
            const AngleList Lr = to_list(all.data(), sens_bricks(plan));
            if ((st = run_back(plan, nullptr, 0, 1, nullptr, ATT_NONE, nullptr, Lr, rest, avail, nullptr, 0, nullptr,
                               nullptr, vec, T_BACK, s, nullptr, nullptr, nullptr, 0, false, fill)))
                return st;
            // the pass wrote one brick volume per listed angle at the start of
            // the scratch; subset m's are contiguous from its first angle,
            // and the sensitivity volumes are vb bytes apart
            const int nslab = tune(plan, La.n, ATT_NONE, T_BACK).nslab;
            if ((st = launch_gather_subsets(plan, La, reinterpret_cast<const float *>(rest), nslab, M, sens[0],
                                            vb / sizeof(float), plan->one_psf, s)))
                return st;
        }
        for (int m = 0; m < M && !combined_sens(plan, M, mu != nullptr); ++m) {
            float *fl = m == 0 ? fill : nullptr;
            if (table)
                st = run_back(plan, nullptr, 0, 1, mu, ATT_WRITE, per[m], lists[m], rest, avail, nullptr, 0, sens[m],
                              nullptr, vec, T_BACK, s, nullptr, nullptr, nullptr, 0, true, fl);
            else
                st = run_back(plan, nullptr, 0, 1, mu, att, nullptr, lists[m], rest, avail, per[m], 0, sens[m], nullptr,
                              vec, T_BOTH, s, nullptr, nullptr, nullptr, 0, true, fl);
            if (st) return st;
        }
        if (bs && (st = launch_sum(plan, sens[0], vb / sizeof(float), M, sens_all, s))) return st;
        if (zs && n_iters > 0 && (st = launch_pad(plan, f, fpad, zs, s))) return st;
        for (int it = 0; it < n_iters; ++it)
            for (int m = 0; m < M; ++m) {
                float *tab = table ? per[m] : nullptr;
                const float *tau = table ? nullptr : per[m];
                BsremTerms bt{sens_all, prior, 0.f, 0.f};
                if (bs) {
                    const float c = (float)lists[m].n / (float)plan->A;
                    const float alpha = bs->relax ? bs->relax[it] : 1.f / (1.f + (float)it);
                    bt.a_over_c = alpha / c;
                    bt.c_beta = c * bs->beta;
                    if ((st = launch_rdp(plan, f, prior, bs->gamma, s))) return st;
                }
                if ((st = run_forward(plan, zs ? fpad : f, mu, att, tab, lists[m], rest, avail, tau, 1, nullptr, g, s_add,
                                      q, vec, T_BOTH, s, nullptr, zs)))
                    return st;
                if ((st = run_back(plan, q, 1, 0, mu, att, tab, lists[m], rest, avail, tau, bs ? 3 : 2, f, sens[m], vec,
                                   T_BOTH, s, bs ? &bt : nullptr, nullptr, fpad, zs)))
                    return st;
            }
        return ok();
    };
    return recon_graph(plan, key, launch_all, static_cast<hipStream_t>(stream));
}

}  // namespace

extern "C" {

int osem_list_step(const spect_plan *plan, const float *f, float *f_out, const float *mu, const float *table,
                   const float *g, const float *s_add, const float *sens, const int32_t *angle_idx, int32_t n_idx,
                   void *ws, size_t ws_bytes, void *stream)
{
    int st, att;
    if ((st = check_plan(plan))) return st;
    if ((st = check_ptr(f, "f", false)) || (st = check_ptr(f_out, "f_out", false)) || (st = check_ptr(mu, "mu", true)) ||
        (st = check_ptr(g, "g", false)) || (st = check_ptr(s_add, "s_add", true)) ||
        (st = check_ptr(sens, "sens", false)))
        return st;
    if ((st = step_att(mu, table, &att))) return st;
    std::vector<int> list;
    if ((st = step_list(plan, angle_idx, n_idx, &list))) return st;
    const int nl = (int)list.size();
    if ((st = check_ws(ws, ws_bytes, step_ws(plan, nl, att)))) return st;
    const AngleList L = to_list(list.data(), nl);
    const bool vec = want_vec(plan, {f, mu});
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    float *q = reinterpret_cast<float *>(w);
    char *rest = w + list_rows_bytes(plan, nl);
    const size_t avail = ws_bytes - list_rows_bytes(plan, nl);
    if ((st = run_forward(plan, f, mu, att, table, L, rest, avail, nullptr, 1, nullptr, g, s_add, q, vec, T_BOTH, s)))
        return st;
    const StepTerms stt{f_out == f ? nullptr : f, nullptr, nullptr};
    if ((st = run_back(plan, q, 1, 0, mu, att, const_cast<float *>(table), L, rest, avail,
                       reinterpret_cast<const float *>(rest), 2, f_out, sens, vec, T_BOTH, s, nullptr, &stt)))
        return st;
    return ok();
}

int osem_list_step_vjp(const spect_plan *plan, const float *f, const float *mu, const float *table, const float *g,
                       const float *s_add, const float *sens, const int32_t *angle_idx, int32_t n_idx,
                       const float *grad_out, float *grad_f, void *ws, size_t ws_bytes, void *stream)
{
    int st, att;
    if ((st = check_plan(plan))) return st;
    if ((st = check_ptr(f, "f", false)) || (st = check_ptr(mu, "mu", true)) || (st = check_ptr(g, "g", false)) ||
        (st = check_ptr(s_add, "s_add", true)) || (st = check_ptr(sens, "sens", false)) ||
        (st = check_ptr(grad_out, "grad_out", false)) || (st = check_ptr(grad_f, "grad_f", false)))
        return st;
    if (grad_f == f) return fail(SPECT_EINVAL, "grad_f must not be f");
    if ((st = step_att(mu, table, &att))) return st;
    std::vector<int> list;
    if ((st = step_list(plan, angle_idx, n_idx, &list))) return st;
    const int nl = (int)list.size();
    if ((st = check_ws(ws, ws_bytes, step_vjp_ws(plan, nl, att)))) return st;
    const AngleList L = to_list(list.data(), nl);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // workspace [e][q][gb][scratch]
    char *w = static_cast<char *>(ws);
    const size_t rb = list_rows_bytes(plan, nl);
    float *e = reinterpret_cast<float *>(w);
    float *q = reinterpret_cast<float *>(w + rb);
    float *gb = reinterpret_cast<float *>(w + 2 * rb);
    char *rest = w + 2 * rb + vol_bytes(plan);
    const size_t avail = ws_bytes - (2 * rb + vol_bytes(plan));
    const float *tau = reinterpret_cast<const float *>(rest);  // offsets of the first pass, when mu is sampled
    // e = H f + s and q = g / e on the listed rows
    if ((st = run_forward(plan, f, mu, att, table, L, rest, avail, nullptr, 2, nullptr, g, s_add, q,
                          want_vec(plan, {f, mu}), T_BOTH, s, e)))
        return st;
    // b = H^T q; grad_f = direct term of the update, gb = gradient in b
    const StepTerms stt{f, grad_out, gb};
    if ((st = run_back(plan, q, 1, 0, mu, att, const_cast<float *>(table), L, rest, avail, tau, 4, grad_f, sens,
                       want_vec(plan, {mu}), T_BOTH, s, nullptr, &stt)))
        return st;
    // gradient in e: -g / e^2 (H gb) where e > 0
    if ((st = run_forward(plan, gb, mu, att, table, L, rest, avail, tau, 3, nullptr, g, nullptr, q,
                          want_vec(plan, {gb, mu}), T_BOTH, s, e)))
        return st;
    // grad_f += H^T of it
    if ((st = run_back(plan, q, 1, 0, mu, att, const_cast<float *>(table), L, rest, avail, tau, 1, grad_f, nullptr,
                       want_vec(plan, {mu}), T_BOTH, s)))
        return st;
    return ok();
}

int osem_reconstruct(const spect_plan *plan, float *f, const float *mu, const float *g, const float *s_add,
                     int32_t n_iters, int32_t n_subsets, void *ws, size_t ws_bytes, void *stream)
{
    return reconstruct(plan, f, mu, g, s_add, n_iters, n_subsets, ws, ws_bytes, stream, nullptr);
}

int osem_reconstruct_ones(const spect_plan *plan, float *f, const float *mu, const float *g, const float *s_add,
                          int32_t n_iters, int32_t n_subsets, void *ws, size_t ws_bytes, void *stream)
{
    return reconstruct(plan, f, mu, g, s_add, n_iters, n_subsets, ws, ws_bytes, stream, nullptr, true);
}

int bsrem_reconstruct(const spect_plan *plan, float *f, const float *mu, const float *g, const float *s_add,
                      int32_t n_iters, int32_t n_subsets, float beta, float gamma, const float *relaxation,
                      void *ws, size_t ws_bytes, void *stream)
{
    const BsremSpec bs{beta, gamma, relaxation};
    return reconstruct(plan, f, mu, g, s_add, n_iters, n_subsets, ws, ws_bytes, stream, &bs);
}

int spect_rdp_gradient(const spect_plan *plan, const float *f, float *grad, float gamma, void *stream)
{
    int st;
    if ((st = check_plan(plan))) return st;
    if ((st = check_ptr(f, "f", false)) || (st = check_ptr(grad, "grad", false))) return st;
    if (f == grad) return fail(SPECT_EINVAL, "f and grad must not overlap");
    if (!finite_nonneg(gamma)) return fail(SPECT_EINVAL, "gamma must be finite and >= 0");
    if ((st = launch_rdp(plan, f, grad, gamma, static_cast<hipStream_t>(stream)))) return st;
    return ok();
}

int bsrem_subset_step(const spect_plan *plan, float *f, const float *mu, const float *g, const float *s_add,
                      const float *sens_m, const float *sens_all, int32_t m, int32_t n_subsets, float alpha,
                      float beta, float gamma, void *ws, size_t ws_bytes, void *stream)
{
    int st;
    if ((st = check_plan(plan))) return st;
    if ((st = check_ptr(f, "f", false)) || (st = check_ptr(mu, "mu", true)) || (st = check_ptr(g, "g", false)) ||
        (st = check_ptr(s_add, "s_add", true)) || (st = check_ptr(sens_m, "sens_m", false)) ||
        (st = check_ptr(sens_all, "sens_all", false)))
        return st;
    if (n_subsets < 1 || n_subsets > plan->A)
        return fail(SPECT_EINVAL, "n_subsets = %d outside [1, %d]", n_subsets, plan->A);
    if (m < 0 || m >= n_subsets) return fail(SPECT_EINVAL, "m = %d outside [0, %d)", m, n_subsets);
    if (!(std::isfinite(alpha) && alpha > 0.f)) return fail(SPECT_EINVAL, "alpha must be finite and > 0");
    if (!finite_nonneg(beta) || !finite_nonneg(gamma))
        return fail(SPECT_EINVAL, "beta and gamma must be finite and >= 0");
    const int nl_max = (plan->A + n_subsets - 1) / n_subsets;
    if (nl_max > MAXL) return fail(SPECT_EUNSUPPORTED, "subsets of more than %d angles", MAXL);
    const size_t vb = vol_bytes(plan);
    if ((st = check_ws(ws, ws_bytes, vb + osem_ws(plan, n_subsets, mu != nullptr)))) return st;
    std::vector<int> list;
    for (int n = m; n < plan->A; n += n_subsets) list.push_back(n);
    const AngleList L = to_list(list.data(), (int)list.size());
    const bool vec = want_vec(plan, {f, mu});
    hipStream_t s = static_cast<hipStream_t>(stream);
    // workspace [prior][q][tau][partial | z]
    char *w = static_cast<char *>(ws);
    float *prior = reinterpret_cast<float *>(w);
    float *q = reinterpret_cast<float *>(w + vb);
    const size_t qb = osem_q_bytes(plan, n_subsets);
    char *rest = w + vb + qb;
    const size_t avail = ws_bytes - vb - qb;
    const float c = (float)L.n / (float)plan->A;
    const BsremTerms bt{sens_all, prior, alpha / c, c * beta};
    if ((st = launch_rdp(plan, f, prior, gamma, s))) return st;
    if ((st = run_forward(plan, f, mu, att_of(mu), nullptr, L, rest, avail, nullptr, 1, nullptr, g, s_add, q, vec,
                          T_BOTH, s)))
        return st;
    if ((st = run_back(plan, q, 1, 0, mu, att_of(mu), nullptr, L, rest, avail, reinterpret_cast<const float *>(rest),
                       3, f, sens_m, vec, T_BOTH, s, &bt)))
        return st;
    return ok();
}

}  // extern "C"

// ==================================================== batched OSEM ====
//
// Many reconstructions of different geometries advance together: subiteration
// m of every member runs as one batched launch per stage (forward, ratio,
// rotated-frame adjoint, gather with the OSEM update) over a work-list of
// (member, angle, slab, depth-chunk) tasks.  Each member keeps its whole OSEM
// state (sensitivities, attenuation tables, ratio, scratch) in its own region
// of one workspace.  One iteration (M subiterations) is recorded once as a
// HIP graph and replayed.  The schedule (members in one launch per stage or
// one launch per size class; persistent or one-task-per-workgroup grids) is
// chosen by timing the candidates (osem_batch_autotune).

struct BatchLaunch {
    int fthreads = 0, bthreads = 0;  // forward and rotated-frame workgroup sizes
    size_t fsmem = 0, bsmem = 0, ssmem = 0;
    FwdBatchFn fk = nullptr;
    BackBatchFn bk = nullptr;
    BatchList<FwdArgs> fwd{};
    BatchList<ReduceArgs> red{};
    BatchList<BackRotArgs> back{};
    BatchList<GatherArgs> gat{};
    int gf = 0, gr = 0, gb = 0, gg = 0;  // grid sizes
    // sensitivity pass (ones back-projected, attenuation tables written), single depth chunk
    BackBatchFn sk = nullptr;
    BatchList<BackRotArgs> sback{};
    BatchList<GatherArgs> sgat{};
    int gsb = 0, gsg = 0;
};

struct spect_batch {
    int R = 0, M = 0, device = 0, cus = 256;
    bool mu = false;
    std::vector<const spect_plan *> plans;
    std::vector<std::vector<AngleList>> lists;  // [r][m]
    std::vector<std::vector<Tuning>> tun;       // [r][m], passes of the iterations (depth-chunked)
    std::vector<std::vector<Tuning>> tun1;      // [r][m], the same without depth chunks
    int kmc_max = 0;
    std::vector<size_t> base, q_off, scr_off, scr_bytes;
    std::vector<std::vector<size_t>> tab_off;   // [r][m], relative to base[r]
    size_t regions = 0, ws_total = 0;
    int sched = 0;  // bit 0: one launch per size class; bit 1: persistent; bit 2: no depth chunks
    double cand_ms[8] = {-1.0, -1.0, -1.0, -1.0, -1.0, -1.0, -1.0, -1.0};
    std::vector<std::vector<BatchLaunch>> steps;  // [m][group]
    void *dmem = nullptr;
    size_t dmem_bytes = 0;
    std::vector<const void *> key;
    int key_sched = -1;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_sched = -1;
    // vector (16-byte) or scalar kernels in the launch tables, and in the
    // captured graph: arrays that change alignment switch the kernels, so the
    // graph is captured again
    int tables_vec = -1, graph_vec = -1;
};

namespace {

int batch_att(const spect_batch *b) { return b->mu ? ATT_READ : ATT_NONE; }

size_t batch_part_bytes(const spect_plan *p, const Tuning &t, int nl, int kmc)
{
    return align256(sizeof(float) * (size_t)nl * t.nslab * t.nchunk * p->N * (SLAB + 2 * kmc));
}

void drop_graph(spect_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_sched = -1;
    b->graph_vec = -1;
}

struct Ptrs {
    float *const *f;
    const float *const *mu;
    const float *const *g;
    const float *const *s;
    char *ws;
};

template <class T>
size_t put(std::vector<char> &blob, const std::vector<T> &v)
{
    const size_t off = (blob.size() + 255) & ~size_t(255);
    blob.resize(off + sizeof(T) * v.size());
    if (!v.empty()) std::memcpy(blob.data() + off, v.data(), sizeof(T) * v.size());
    return off;
}

// Build the launch tables of schedule `sched` for the given arrays and upload
// them.  Waits for the device first: replays of an earlier build may still
// read the tables.
int build_tables(spect_batch *b, const Ptrs &P, bool vec, int sched)
{
    const int att = batch_att(b);
    const bool grouped = sched & 1, persist = sched & 2;
    const std::vector<std::vector<Tuning>> &tuning = (sched & 4) ? b->tun1 : b->tun;
    // groups: members sharing block size and blur class, or all members
    std::vector<std::vector<int>> groups;
    std::vector<int> gkmc;
    if (grouped) {
        std::vector<std::pair<std::pair<int, int>, int>> keys;
        for (int r = 0; r < b->R; ++r) keys.push_back({{block_threads(b->plans[r]->N), b->plans[r]->kmc}, r});
        std::stable_sort(keys.begin(), keys.end(),
                         [](const auto &x, const auto &y) { return x.first < y.first; });
        for (size_t i = 0; i < keys.size(); ++i) {
            if (i == 0 || keys[i].first != keys[i - 1].first) {
                groups.emplace_back();
                gkmc.push_back(keys[i].first.second);
            }
            groups.back().push_back(keys[i].second);
        }
    } else {
        groups.emplace_back();
        for (int r = 0; r < b->R; ++r) groups.back().push_back(r);
        gkmc.push_back(b->kmc_max);
    }
    struct Offs {
        size_t fa, ft, ra, rt, ba, bt, ga, gt, sa, st, sg;
        int nf, nr, nb, ng, ns;
    };
    std::vector<char> blob;
    std::vector<std::vector<Offs>> offs(b->M);
    for (int m = 0; m < b->M; ++m) {
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const int kmc = gkmc[gi];
            std::vector<FwdArgs> fa;
            std::vector<ReduceArgs> ra;
            std::vector<BackRotArgs> ba;
            std::vector<GatherArgs> ga;
            std::vector<std::pair<long, Task>> ft, bt, stk;
            std::vector<Task> rt, gt;
            std::vector<BackRotArgs> sa;
            std::vector<GatherArgs> sg;
            for (size_t li = 0; li < groups[gi].size(); ++li) {
                const int r = groups[gi][li];
                const spect_plan *p = b->plans[r];
                const AngleList &L = b->lists[r][m];
                const Tuning &t = tuning[r][m];
                char *base = P.ws + b->base[r];
                float *tab = b->mu ? reinterpret_cast<float *>(base + b->tab_off[r][m]) : nullptr;
                float *q = reinterpret_cast<float *>(base + b->q_off[r]);
                float *scr = reinterpret_cast<float *>(base + b->scr_off[r]);
                float *sens = reinterpret_cast<float *>(base + (size_t)m * vol_bytes(p));
                FwdArgs a{};
                a.g = p->g;
                a.L = L;
                a.f = P.f[r];
                a.att = tab;
                a.part = scr;
                a.nslab = t.nslab;
                a.nchunk = t.nchunk;
                a.cbset = 1;
                a.vec = vec;
                fa.push_back(a);
                ReduceArgs rr{};
                rr.L = L;
                rr.part = scr;
                rr.N = p->N;
                rr.Nz = p->Nz;
                rr.nslab = t.nslab;
                rr.nchunk = t.nchunk;
                rr.kmc = kmc;
                rr.mode = 1;
                rr.g = P.g[r];
                rr.s_add = P.s ? P.s[r] : nullptr;
                rr.q = q;
                ra.push_back(rr);
                BackRotArgs bb{};
                bb.g = p->g;
                bb.L = L;
                bb.y = q;
                bb.y_compact = 1;
                bb.att = tab;
                bb.z = scr;
                bb.nslab = t.nslab;
                bb.nchunk = t.nchunk_b;
                bb.cbset = 1;
                bb.vec = vec;
                ba.push_back(bb);
                GatherArgs gg{};
                gg.g = p->g;
                gg.L = L;
                gg.z = scr;
                gg.nslab = t.nslab;
                gg.mode = 2;
                gg.out = P.f[r];
                gg.sens = sens;
                gg.v4 = gather_v4(p, {P.f[r], sens});
                ga.push_back(gg);
                BackRotArgs sb = bb;  // sensitivity: ones, mu sampled, table written, one depth chunk
                sb.y = nullptr;
                sb.y_compact = 0;
                sb.ones = 1;
                sb.mu = b->mu ? P.mu[r] : nullptr;
                sb.nchunk = 1;
                sb.cbset = 0;
                sa.push_back(sb);
                GatherArgs sgg = gg;
                sgg.mode = 0;
                sgg.out = sens;
                sgg.sens = nullptr;
                sgg.v4 = gather_v4(p, {sens});
                sg.push_back(sgg);
                const int sblk = (p->N * (SLAB / 2) + SL_THREADS - 1) / SL_THREADS;
                for (int al = 0; al < L.n; ++al)
                    for (int sl = 0; sl < t.nslab; ++sl)
                        for (int k = 0; k < sblk; ++k)
                            stk.push_back({(long)p->N * p->N, Task{(int)li, k, sl, al}});
                const int li_ = (int)li;
                for (int al = 0; al < L.n; ++al) {
                    // blur work of the chunk's depths x bins
                    for (int c = 0; c < t.nchunk; ++c) {
                        const long fc = (long)(chunk_work(p, 1, t.nchunk, L.idx[al], c) * p->N);
                        for (int sl = 0; sl < t.nslab; ++sl) ft.push_back({fc, Task{li_, sl, c, al}});
                    }
                    for (int c = 0; c < t.nchunk_b; ++c) {
                        const long bc = (long)(chunk_work(p, 1, t.nchunk_b, L.idx[al], c) * p->N);
                        for (int sl = 0; sl < t.nslab; ++sl) bt.push_back({bc, Task{li_, sl, c, al}});
                    }
                }
                const int blocks = (p->N * p->Nz + 255) / 256;
                for (int al = 0; al < L.n; ++al)
                    for (int k = 0; k < blocks; ++k) rt.push_back(Task{li_, k, 0, al});
                const int tiles = (p->N + GT - 1) / GT;
                for (int sp = 0; sp < (t.nslab + GS - 1) / GS; ++sp)
                    for (int k = 0; k < tiles * tiles; ++k) gt.push_back(Task{li_, k, sp, 0});
            }
            // longest tasks first, so that the tail of the launch is short
            auto by_cost = [](const std::pair<long, Task> &x, const std::pair<long, Task> &y) {
                return x.first > y.first;
            };
            std::stable_sort(ft.begin(), ft.end(), by_cost);
            std::stable_sort(bt.begin(), bt.end(), by_cost);
            std::stable_sort(stk.begin(), stk.end(), by_cost);
            std::vector<Task> ftv, btv, stv;
            for (auto &x : ft) ftv.push_back(x.second);
            for (auto &x : bt) btv.push_back(x.second);
            for (auto &x : stk) stv.push_back(x.second);
            Offs o;
            o.fa = put(blob, fa);
            o.ft = put(blob, ftv);
            o.ra = put(blob, ra);
            o.rt = put(blob, rt);
            o.ba = put(blob, ba);
            o.bt = put(blob, btv);
            o.ga = put(blob, ga);
            o.gt = put(blob, gt);
            o.sa = put(blob, sa);
            o.st = put(blob, stv);
            o.sg = put(blob, sg);
            o.ns = (int)stv.size();
            o.nf = (int)ftv.size();
            o.nr = (int)rt.size();
            o.nb = (int)btv.size();
            o.ng = (int)gt.size();
            offs[m].push_back(o);
        }
    }
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "batch table update");
    if (blob.size() > b->dmem_bytes) {
        if (b->dmem) (void)hipFree(b->dmem);
        b->dmem = nullptr;
        b->dmem_bytes = 0;
        if ((e = hipMalloc(&b->dmem, blob.size())) != hipSuccess)
            return fail(SPECT_ENOMEM, "hipMalloc of %zu bytes of batch tables failed", blob.size());
        b->dmem_bytes = blob.size();
        drop_graph(b);  // the graph's kernel arguments point at the old tables
    }
    if ((e = hipMemcpy(b->dmem, blob.data(), blob.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "batch table upload");
    char *d = static_cast<char *>(b->dmem);
    b->steps.assign(b->M, {});
    for (int m = 0; m < b->M; ++m)
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const Offs &o = offs[m][gi];
            BatchLaunch l;
            int Nmax = 0;
            for (int r : groups[gi]) Nmax = std::max(Nmax, b->plans[r]->N);
            l.fthreads = fwd_threads(Nmax);
            l.bthreads = block_threads(Nmax);
            l.fsmem = fwd_smem(Nmax, gkmc[gi]);
            l.bsmem = back_smem(Nmax, gkmc[gi]);
            for (int r : groups[gi]) l.ssmem = std::max(l.ssmem, sens_smem(b->plans[r]->N, b->plans[r]->TS));
            l.fk = fwd_batch_kernel(att, gkmc[gi], vec, persist);
            l.bk = back_batch_kernel(att, gkmc[gi], vec, persist);
            allow_smem(reinterpret_cast<const void *>(l.fk), l.fsmem);
            allow_smem(reinterpret_cast<const void *>(l.bk), l.bsmem);
            l.fwd = {reinterpret_cast<const FwdArgs *>(d + o.fa), reinterpret_cast<const Task *>(d + o.ft), o.nf};
            l.red = {reinterpret_cast<const ReduceArgs *>(d + o.ra), reinterpret_cast<const Task *>(d + o.rt), o.nr};
            l.back = {reinterpret_cast<const BackRotArgs *>(d + o.ba), reinterpret_cast<const Task *>(d + o.bt),
                      o.nb};
            l.gat = {reinterpret_cast<const GatherArgs *>(d + o.ga), reinterpret_cast<const Task *>(d + o.gt), o.ng};
            if (b->mu)
                l.sk = vec ? sensl_batch<ATT_WRITE, true> : sensl_batch<ATT_WRITE, false>;
            else
                l.sk = sensl_batch<ATT_NONE, false>;
            l.sback = {reinterpret_cast<const BackRotArgs *>(d + o.sa), reinterpret_cast<const Task *>(d + o.st),
                       o.ns};
            l.sgat = {reinterpret_cast<const GatherArgs *>(d + o.sg), reinterpret_cast<const Task *>(d + o.gt), o.ng};
            allow_smem(reinterpret_cast<const void *>(l.sk), l.ssmem);
            if (persist) {
                int nb = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(l.fk),
                                                                  l.fthreads, l.fsmem) != hipSuccess || nb < 1)
                    nb = 1;
                l.gf = std::max(1, std::min(o.nf, nb * b->cus));
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(l.bk),
                                                                  l.bthreads, l.bsmem) != hipSuccess || nb < 1)
                    nb = 1;
                l.gb = std::max(1, std::min(o.nb, nb * b->cus));
                l.gr = std::max(1, std::min(o.nr, 8 * b->cus));
                l.gg = std::max(1, std::min(o.ng, 8 * b->cus));
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(l.sk),
                                                                  SL_THREADS, l.ssmem) != hipSuccess || nb < 1)
                    nb = 1;
                l.gsb = std::max(1, std::min(o.ns, nb * b->cus));
            } else {
                l.gf = std::max(1, o.nf);
                l.gb = std::max(1, o.nb);
                l.gr = std::max(1, o.nr);
                l.gg = std::max(1, o.ng);
                l.gsb = std::max(1, o.ns);
            }
            l.gsg = l.gg;
            b->steps[m].push_back(l);
        }
    (void)hipGetLastError();
    return SPECT_OK;
}

// Subiteration m of every member, on stream st (capturing: no event timing).
int launch_step(const spect_batch *b, int m, hipStream_t st, bool capturing)
{
    for (const BatchLaunch &l : b->steps[m]) {
        {
            ProfScope ps(K_FWD_B, st, !capturing);
            hipLaunchKernelGGL(l.fk, dim3(l.gf), dim3(l.fthreads), l.fsmem, st, l.fwd);
        }
        {
            ProfScope ps(K_REDUCE_B, st, !capturing);
            hipLaunchKernelGGL(reduce_batch, dim3(l.gr), dim3(256), 0, st, l.red);
        }
    }
    for (const BatchLaunch &l : b->steps[m]) {
        {
            ProfScope ps(K_BACK_B, st, !capturing);
            hipLaunchKernelGGL(l.bk, dim3(l.gb), dim3(l.bthreads), l.bsmem, st, l.back);
        }
        {
            ProfScope ps(K_GATHER_B, st, !capturing);
            hipLaunchKernelGGL(gather_batch, dim3(l.gg), dim3(256), 0, st, l.gat);
        }
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPECT_OK : hip_fail(e, "batched launch");
}

// Record one iteration (M subiterations) as a graph.
int capture_iteration(spect_batch *b)
{
    drop_graph(b);
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "graph capture begin");
    int st = SPECT_OK;
    for (int m = 0; m < b->M && st == SPECT_OK; ++m) st = launch_step(b, m, b->cap, true);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap, &g);
    if (st != SPECT_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "graph capture end");
    b->graph = g;
    if ((e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
        drop_graph(b);
        return hip_fail(e, "graph instantiation");
    }
    b->graph_sched = b->sched;
    b->graph_vec = b->tables_vec;
    return SPECT_OK;
}

// Sensitivities (and attenuation tables) of every member and subset: per
// subset one batched sensitivity launch per group (constant projection: tap
// sums, mu sampled along whole rays, factors stored) and one gather.
int batch_sensitivities(const spect_batch *b, hipStream_t st)
{
    for (int m = 0; m < b->M; ++m)
        for (const BatchLaunch &l : b->steps[m]) {
            {
                ProfScope ps(K_SENS, st);
                hipLaunchKernelGGL(l.sk, dim3(l.gsb), dim3(SL_THREADS), l.ssmem, st, l.sback);
            }
            {
                ProfScope ps(K_GATHER_B, st);
                hipLaunchKernelGGL(gather_batch, dim3(l.gsg), dim3(256), 0, st, l.sgat);
            }
        }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPECT_OK : hip_fail(e, "batched sensitivity launch");
}

int check_batch_args(const spect_batch *b, const Ptrs &P, size_t ws_bytes, bool *vec)
{
    int st;
    if (!b) return fail(SPECT_EINVAL, "batch is NULL");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
        return fail(SPECT_EINVAL, "current HIP device %d is not the batch's device %d", dev, b->device);
    if (!P.f || !P.g) return fail(SPECT_EINVAL, "f and g arrays must not be NULL");
    if (b->mu && !P.mu) return fail(SPECT_EINVAL, "the batch was created with attenuation: mu array is NULL");
    *vec = true;
    for (int r = 0; r < b->R; ++r) {
        if ((st = check_ptr(P.f[r], "f[r]", false)) || (st = check_ptr(P.g[r], "g[r]", false))) return st;
        if (b->mu && (st = check_ptr(P.mu[r], "mu[r]", false))) return st;
        if (!b->mu && P.mu && P.mu[r]) return fail(SPECT_EINVAL, "the batch was created without attenuation");
        if (P.s && (st = check_ptr(P.s[r], "s_add[r]", true))) return st;
        if (b->plans[r]->Nz % 4 || !aligned16(P.f[r]) || (b->mu && !aligned16(P.mu[r]))) *vec = false;
    }
    return check_ws(P.ws, ws_bytes, b->ws_total);
}

// (Re)build the tables when the arrays or the schedule changed.
int prepare(spect_batch *b, const Ptrs &P, bool vec)
{
    std::vector<const void *> key;
    for (int r = 0; r < b->R; ++r) {
        key.push_back(P.f[r]);
        key.push_back(P.g[r]);
        key.push_back(b->mu ? P.mu[r] : nullptr);
        key.push_back(P.s ? P.s[r] : nullptr);
    }
    key.push_back(P.ws);
    key.push_back(reinterpret_cast<const void *>((uintptr_t)vec));
    if (key == b->key && b->key_sched == b->sched) return SPECT_OK;
    const int st = build_tables(b, P, vec, b->sched);
    if (st) return st;
    b->tables_vec = vec ? 1 : 0;
    b->key = key;
    b->key_sched = b->sched;
    return SPECT_OK;
}

}  // namespace

extern "C" {

int spect_batch_create(const spect_plan *const *plans, int32_t n_members, int32_t n_subsets, int with_mu,
                       spect_batch **out)
{
    if (!out) return fail(SPECT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!plans) return fail(SPECT_EINVAL, "plans is NULL");
    if (n_members < 1) return fail(SPECT_EINVAL, "n_members = %d must be >= 1", n_members);
    if (n_subsets < 1) return fail(SPECT_EINVAL, "n_subsets = %d must be >= 1", n_subsets);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SPECT_EHIP, "no HIP device");
    for (int r = 0; r < n_members; ++r) {
        if (!plans[r]) return fail(SPECT_EINVAL, "plans[%d] is NULL", r);
        if (plans[r]->device != dev) return fail(SPECT_EINVAL, "plans[%d] belongs to another device", r);
        if (n_subsets > plans[r]->A)
            return fail(SPECT_EINVAL, "n_subsets %d exceeds n_angles %d of member %d", n_subsets, plans[r]->A, r);
        if ((plans[r]->A + n_subsets - 1) / n_subsets > MAXL)
            return fail(SPECT_EUNSUPPORTED, "member %d has subsets of more than %d angles", r, MAXL);
    }
    spect_batch *b = new spect_batch();
    b->R = n_members;
    b->M = n_subsets;
    b->device = dev;
    b->mu = with_mu != 0;
    if (hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || b->cus < 1)
        b->cus = 256;
    const int att = batch_att(b);
    size_t off = 0;
    for (int r = 0; r < n_members; ++r) {
        const spect_plan *p = plans[r];
        b->plans.push_back(p);
        b->kmc_max = std::max(b->kmc_max, p->kmc);
    }
    for (int r = 0; r < n_members; ++r) {
        const spect_plan *p = b->plans[r];
        std::vector<AngleList> ls;
        std::vector<Tuning> ts, t1;
        std::vector<size_t> tabs;
        size_t rel = (size_t)n_subsets * vol_bytes(p), scr = 0;
        for (int m = 0; m < n_subsets; ++m) {
            std::vector<int> list;
            for (int n = m; n < p->A; n += n_subsets) list.push_back(n);
            ls.push_back(to_list(list.data(), (int)list.size()));
            const int nl = (int)list.size();
            const Tuning t = tune(p, nl, att, T_BOTH);
            ts.push_back(t);
            t1.push_back(Tuning{t.nslab, 1, 1});
            tabs.push_back(rel);
            if (b->mu) rel += table_bytes(p, nl);
            scr = std::max(scr, batch_part_bytes(p, t, nl, b->kmc_max));
            scr = std::max(scr, z_bytes(p, t, nl));
            scr = std::max(scr, back_need(p, nl, b->mu ? ATT_WRITE : ATT_NONE, T_BACK));
        }
        b->lists.push_back(ls);
        b->tun.push_back(ts);
        b->tun1.push_back(t1);
        b->tab_off.push_back(tabs);
        b->q_off.push_back(rel);
        rel += osem_q_bytes(p, n_subsets);
        b->scr_off.push_back(rel);
        b->scr_bytes.push_back(scr);
        rel += scr;
        b->base.push_back(off);
        off += align256(rel);
    }
    b->regions = off;
    b->ws_total = off;
    for (int r = 0; r < n_members; ++r) b->ws_total += vol_bytes(b->plans[r]);  // image copies for tuning
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return fail(SPECT_EHIP, "stream creation failed");
    }
    *out = b;
    return ok();
}

int spect_batch_destroy(spect_batch *b)
{
    if (!b) return ok();
    (void)hipDeviceSynchronize();
    drop_graph(b);
    if (b->dmem) (void)hipFree(b->dmem);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return ok();
}

int spect_batch_workspace_size(const spect_batch *b, size_t *bytes)
{
    if (!b) return fail(SPECT_EINVAL, "batch is NULL");
    if (!bytes) return fail(SPECT_EINVAL, "bytes is NULL");
    *bytes = b->ws_total;
    return ok();
}

int spect_batch_schedule(const spect_batch *b, int32_t *schedule, double *candidate_ms)
{
    if (!b) return fail(SPECT_EINVAL, "batch is NULL");
    if (schedule) *schedule = b->sched;
    if (candidate_ms)
        for (int c = 0; c < 8; ++c) candidate_ms[c] = b->cand_ms[c];
    return ok();
}

int spect_batch_set_schedule(spect_batch *b, int32_t schedule)
{
    if (!b) return fail(SPECT_EINVAL, "batch is NULL");
    if (schedule < 0 || schedule > 7) return fail(SPECT_EINVAL, "schedule = %d outside [0, 7]", schedule);
    b->sched = schedule;
    return ok();
}

int osem_batch_reconstruct(spect_batch *b, float *const *f, const float *const *mu, const float *const *g,
                           const float *const *s_add, int32_t n_iters, int32_t flags, void *ws, size_t ws_bytes,
                           void *stream)
{
    int st;
    const Ptrs P{f, mu, g, s_add, static_cast<char *>(ws)};
    bool vec = true;
    if ((st = check_batch_args(b, P, ws_bytes, &vec))) return st;
    if (n_iters < 0) return fail(SPECT_EINVAL, "n_iters = %d is negative", n_iters);
    if (flags & ~SPECT_BATCH_EAGER) return fail(SPECT_EINVAL, "unknown flags 0x%x", (unsigned)flags);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = prepare(b, P, vec))) return st;
    if ((st = batch_sensitivities(b, s))) return st;
    if (n_iters == 0) return ok();
    if (flags & SPECT_BATCH_EAGER) {
        for (int it = 0; it < n_iters; ++it)
            for (int m = 0; m < b->M; ++m)
                if ((st = launch_step(b, m, s, false))) return st;
        return ok();
    }
    if (!b->exec || b->graph_sched != b->sched || b->graph_vec != b->tables_vec)
        if ((st = capture_iteration(b))) return st;
    for (int it = 0; it < n_iters; ++it) {
        const hipError_t e = hipGraphLaunch(b->exec, s);
        if (e != hipSuccess) return hip_fail(e, "graph launch");
    }
    return ok();
}

int osem_batch_autotune(spect_batch *b, float *const *f, const float *const *mu, const float *const *g,
                        const float *const *s_add, void *ws, size_t ws_bytes, void *stream)
{
    int st;
    const Ptrs P0{f, mu, g, s_add, static_cast<char *>(ws)};
    bool vec = true;
    if ((st = check_batch_args(b, P0, ws_bytes, &vec))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // work on copies of the images, kept after the member regions
    std::vector<float *> fc(b->R);
    size_t off = b->regions;
    for (int r = 0; r < b->R; ++r) {
        fc[r] = reinterpret_cast<float *>(static_cast<char *>(ws) + off);
        const size_t n = sizeof(float) * (size_t)b->plans[r]->N * b->plans[r]->N * b->plans[r]->Nz;
        const hipError_t e = hipMemcpyAsync(fc[r], f[r], n, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "image copy for tuning");
        off += vol_bytes(b->plans[r]);
    }
    const Ptrs P{fc.data(), mu, g, s_add, static_cast<char *>(ws)};
    bool vec_c = vec;
    for (int r = 0; r < b->R; ++r)
        if (!aligned16(fc[r])) vec_c = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(SPECT_EHIP, "event creation failed");
    int best = 0;
    double best_ms = 1e300;
    for (int c = 0; c < 8 && st == SPECT_OK; ++c) {
        b->sched = c;
        if ((st = prepare(b, P, vec_c))) break;
        if (c == 0 && (st = batch_sensitivities(b, s))) break;
        if ((st = capture_iteration(b))) break;
        hipError_t e = hipGraphLaunch(b->exec, s);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipGraphLaunch(b->exec, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            st = hip_fail(e, "autotune timing");
            break;
        }
        b->cand_ms[c] = ms / 2.0;
        if (ms / 2.0 < best_ms) {
            best_ms = ms / 2.0;
            best = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->sched = best;
    b->key.clear();  // the next reconstruction rebuilds for its own arrays
    drop_graph(b);
    return st ? st : ok();
}

}  // extern "C"

// ============================================= iteration-level batching ===
//
// The engine behind the reconstruction server: every call launches one
// "tick" in which each listed request advances by one step, either one
// subset's sensitivity pass (which also fills that subset's attenuation
// table) or one OSEM subiteration, through the work-list kernels, all
// requests together: one launch per stage (and per blur class for the
// forward and rotated-frame kernels).  A request's state lives in its own
// region laid out as osem_reconstruct's workspace, and its launch arguments
// and tuning are the ones osem_reconstruct uses, so a request advanced tick
// by tick ends with osem_reconstruct's result bitwise, whatever else shares
// its ticks.

namespace spect_internal {

struct TickTables {
    std::vector<char> blob;
    struct Pad {
        const spect_plan *p;
        const float *src;
        float *dst;
        int zs;
    };
    std::vector<Pad> pads;  // padded copies of f made before the tick's kernels
    struct Launch {
        int kind;  // 0 sensitivity, 1 forward, 2 reduce, 3 rotated-frame, 4 gather
        const void *fn;
        int threads;
        size_t smem;
        size_t args, tasks;  // blob offsets
        int ntasks;
    };
    std::vector<Launch> launches;
};

namespace {

struct ItemLayout {
    float *sens, *table, *q;
    float *fpad;  // the forward's padded copy of f (zs floats per column), or nullptr
    int zs;
    char *rest;
};

ItemLayout item_layout(const TickItem &it)
{
    const spect_plan *p = it.plan;
    const int M = it.n_subsets;
    const bool mu = it.mu != nullptr;
    const size_t vb = vol_bytes(p);
    ItemLayout l;
    l.sens = reinterpret_cast<float *>(it.region + (size_t)it.subset * vb);
    size_t off = (size_t)M * vb;
    l.table = nullptr;
    for (int m = 0; m < M; ++m) {
        if (m == it.subset && mu) l.table = reinterpret_cast<float *>(it.region + off);
        off += recon_tau_bytes(p, M, m, mu);
    }
    l.q = reinterpret_cast<float *>(it.region + off);
    off += osem_q_bytes(p, M);
    // as in reconstruct: [q][padded f][scratch]
    const int att = mu ? ATT_READ : ATT_NONE;
    l.zs = pad_stride(p, att);
    l.fpad = l.zs ? reinterpret_cast<float *>(it.region + off) : nullptr;
    l.rest = it.region + off + pad_bytes(p, att);
    return l;
}

AngleList subset_list(const spect_plan *p, int M, int m)
{
    std::vector<int> list;
    for (int n = m; n < p->A; n += M) list.push_back(n);
    return to_list(list.data(), (int)list.size());
}

}  // namespace

int tick_region_bytes(const spect_plan *p, int n_subsets, bool mu, size_t *bytes)
{
    int st;
    if ((st = check_plan(p))) return st;
    if (n_subsets < 1 || n_subsets > p->A)
        return fail(SPECT_EINVAL, "n_subsets = %d outside [1, %d]", n_subsets, p->A);
    if ((p->A + n_subsets - 1) / n_subsets > MAXL)
        return fail(SPECT_EUNSUPPORTED, "subsets of more than %d angles", MAXL);
    if (mu && !use_table(p, n_subsets, true))
        return fail(SPECT_EUNSUPPORTED, "the attenuation tables of this request exceed %zu bytes", kMaxTableBytes);
    *bytes = recon_ws(p, n_subsets, mu);
    return SPECT_OK;
}

double step_work(const spect_plan *p, int n_subsets)
{
    return (double)p->N * p->N * p->Nz * ((p->A + n_subsets - 1) / std::max(1, n_subsets));
}

TickTables *tick_build(const TickItem *items, int n, int *status)
{
    auto *T = new TickTables();
    // launch groups: sensitivity passes by kernel variant; forward and
    // rotated-frame passes by blur class and load width
    struct Group {
        std::vector<FwdArgs> fa;
        std::vector<BackRotArgs> ba;
        std::vector<std::pair<long, Task>> ft, bt;
        int nmax = 0;
    };
    struct SensGroup {
        std::vector<BackRotArgs> sa;
        std::vector<Task> st;
        size_t smem = 0;
    };
    std::vector<std::pair<std::pair<int, int>, Group>> groups;   // (kmc, vec)
    std::vector<std::pair<int, SensGroup>> sgroups;               // variant: 0 none, 1 write, 2 write (pairs)
    std::vector<ReduceArgs> ra;
    std::vector<Task> rt;
    std::vector<GatherArgs> ga;
    std::vector<Task> gt;
    auto group = [&](int kmc, int vec) -> std::pair<int, Group &> {
        for (size_t i = 0; i < groups.size(); ++i)
            if (groups[i].first == std::make_pair(kmc, vec)) return {(int)i, groups[i].second};
        groups.push_back({{kmc, vec}, Group()});
        return {(int)groups.size() - 1, groups.back().second};
    };
    for (int i = 0; i < n; ++i) {
        const TickItem &it = items[i];
        const spect_plan *p = it.plan;
        const int M = it.n_subsets, m = it.subset;
        const bool mu = it.mu != nullptr;
        const ItemLayout lay = item_layout(it);
        const AngleList L = subset_list(p, M, m);
        const bool vec = want_vec(p, {it.f, it.mu});
        const int tiles = (p->N + GT - 1) / GT;
        if (it.sens) {
            // the sensitivity pass of osem_reconstruct (run_back with a
            // constant projection: one depth chunk, tap sums, mu sampled and
            // its factors stored in the subset's table)
            const Tuning t = tune(p, L.n, mu ? ATT_WRITE : ATT_NONE, mu ? T_BACK : T_BOTH);
            const bool v2 = mu && p->Nz % 2 == 0 && aligned8(it.mu);
            const int var = !mu ? 0 : (v2 ? 2 : 1);
            size_t si = 0;
            while (si < sgroups.size() && sgroups[si].first != var) ++si;
            if (si == sgroups.size()) sgroups.push_back({var, SensGroup()});
            SensGroup &sg = sgroups[si].second;
            BackRotArgs sb{};
            sb.g = p->g;
            sb.L = L;
            sb.ones = 1;
            sb.mu = it.mu;
            sb.att = lay.table;
            sb.z = reinterpret_cast<float *>(lay.rest);
            sb.nslab = t.nslab;
            sb.nchunk = 1;
            sb.cbset = 0;
            sb.vec = vec;
            const int li = (int)sg.sa.size();
            sg.sa.push_back(sb);
            sg.smem = std::max(sg.smem, sens_smem(p->N, p->TS));
            const int sblk = (p->N * (SLAB / 2) + SL_THREADS - 1) / SL_THREADS;
            for (int al = 0; al < L.n; ++al)
                for (int sl = 0; sl < t.nslab; ++sl)
                    for (int k = 0; k < sblk; ++k) sg.st.push_back(Task{li, k, sl, al});
            GatherArgs gg{};
            gg.g = p->g;
            gg.L = L;
            gg.z = reinterpret_cast<float *>(lay.rest);
            gg.nslab = t.nslab;
            gg.mode = 0;
            gg.out = lay.sens;
            gg.v4 = gather_v4(p, {lay.sens});
            const int gi = (int)ga.size();
            ga.push_back(gg);
            for (int sp = 0; sp < (t.nslab + GS - 1) / GS; ++sp)
                for (int k = 0; k < tiles * tiles; ++k) gt.push_back(Task{gi, k, sp, 0});
            continue;
        }
        // one subiteration, as osem_reconstruct runs it (run_forward with the
        // fused ratio, run_back with the fused update, shared tuning)
        const int att = mu ? ATT_READ : ATT_NONE;
        const Tuning t = tune(p, L.n, att, T_BOTH);
        auto gr = group(p->kmc, vec ? 1 : 0);
        Group &G = gr.second;
        G.nmax = std::max(G.nmax, p->N);
        float *scr = reinterpret_cast<float *>(lay.rest);
        if (it.first_sub && lay.zs) T->pads.push_back(TickTables::Pad{p, it.f, lay.fpad, lay.zs});
        FwdArgs a{};
        a.g = p->g;
        a.L = L;
        a.f = lay.zs ? lay.fpad : it.f;
        a.zs = lay.zs;
        a.att = lay.table;
        a.part = scr;
        a.nslab = t.nslab;
        a.nchunk = t.nchunk;
        a.cbset = chunk_set(att, T_BOTH);
        a.vec = vec;
        const int fi = (int)G.fa.size();
        G.fa.push_back(a);
        ReduceArgs rr{};
        rr.L = L;
        rr.part = scr;
        rr.N = p->N;
        rr.Nz = p->Nz;
        rr.nslab = t.nslab;
        rr.nchunk = t.nchunk;
        rr.kmc = p->kmc;
        rr.mode = 1;
        rr.g = it.g;
        rr.s_add = it.s_add;
        rr.q = lay.q;
        const int ri = (int)ra.size();
        ra.push_back(rr);
        BackRotArgs bb{};
        bb.g = p->g;
        bb.L = L;
        bb.y = lay.q;
        bb.y_compact = 1;
        bb.att = lay.table;
        bb.z = scr;
        bb.nslab = t.nslab;
        bb.nchunk = t.nchunk_b;
        bb.cbset = chunk_set(att, T_BOTH);
        bb.vec = vec;
        G.ba.push_back(bb);
        GatherArgs gg{};
        gg.g = p->g;
        gg.L = L;
        gg.z = scr;
        gg.nslab = t.nslab;
        gg.mode = 2;
        gg.out = it.f;
        gg.sens = lay.sens;
        gg.fpad = lay.fpad;
        gg.zs = lay.zs;
        gg.v4 = gather_v4(p, {it.f, lay.sens, lay.fpad});
        const int gi = (int)ga.size();
        ga.push_back(gg);
        for (int al = 0; al < L.n; ++al) {
            for (int c = 0; c < t.nchunk; ++c) {
                const long fc = (long)(chunk_work(p, a.cbset, t.nchunk, L.idx[al], c) * p->N);
                for (int sl = 0; sl < t.nslab; ++sl) G.ft.push_back({fc, Task{fi, sl, c, al}});
            }
            for (int c = 0; c < t.nchunk_b; ++c) {
                const long bc = (long)(chunk_work(p, bb.cbset, t.nchunk_b, L.idx[al], c) * p->N);
                for (int sl = 0; sl < t.nslab; ++sl) G.bt.push_back({bc, Task{fi, sl, c, al}});
            }
        }
        const int blocks = (p->N * p->Nz + 255) / 256;
        for (int al = 0; al < L.n; ++al)
            for (int k = 0; k < blocks; ++k) rt.push_back(Task{ri, k, 0, al});
        for (int sp = 0; sp < (t.nslab + GS - 1) / GS; ++sp)
            for (int k = 0; k < tiles * tiles; ++k) gt.push_back(Task{gi, k, sp, 0});
    }
    auto by_cost = [](const std::pair<long, Task> &x, const std::pair<long, Task> &y) { return x.first > y.first; };
    auto add = [&](int kind, const void *fn, int threads, size_t smem, size_t args, size_t tasks, int ntasks) {
        if (ntasks > 0) T->launches.push_back(TickTables::Launch{kind, fn, threads, smem, args, tasks, ntasks});
    };
    // stage order: sensitivity passes, forward, reduction, rotated-frame, gather
    for (auto &sg : sgroups) {
        const void *fn = sg.first == 0   ? reinterpret_cast<const void *>(sensl_batch<ATT_NONE, false>)
                         : sg.first == 2 ? reinterpret_cast<const void *>(sensl_batch<ATT_WRITE, true>)
                                         : reinterpret_cast<const void *>(sensl_batch<ATT_WRITE, false>);
        const size_t ao = put(T->blob, sg.second.sa), to = put(T->blob, sg.second.st);
        add(0, fn, SL_THREADS, sg.second.smem, ao, to, (int)sg.second.st.size());
    }
    std::vector<size_t> bo(groups.size()), bto(groups.size());
    std::vector<int> bn(groups.size());
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        Group &G = groups[gi].second;
        const int kmc = groups[gi].first.first, vec = groups[gi].first.second;
        std::stable_sort(G.ft.begin(), G.ft.end(), by_cost);
        std::stable_sort(G.bt.begin(), G.bt.end(), by_cost);
        std::vector<Task> ftv, btv;
        for (auto &x : G.ft) ftv.push_back(x.second);
        for (auto &x : G.bt) btv.push_back(x.second);
        const int att = G.fa[0].att ? ATT_READ : ATT_NONE;
        const size_t ao = put(T->blob, G.fa), to = put(T->blob, ftv);
        add(1, reinterpret_cast<const void *>(fwd_batch_kernel(att, kmc, vec, false)), fwd_threads(G.nmax),
            fwd_smem(G.nmax, kmc), ao, to, (int)ftv.size());
        bo[gi] = put(T->blob, G.ba);
        bto[gi] = put(T->blob, btv);
        bn[gi] = (int)btv.size();
    }
    {
        const size_t ao = put(T->blob, ra), to = put(T->blob, rt);
        add(2, reinterpret_cast<const void *>(reduce_batch), 256, 0, ao, to, (int)rt.size());
    }
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        Group &G = groups[gi].second;
        const int kmc = groups[gi].first.first, vec = groups[gi].first.second;
        const int att = G.fa[0].att ? ATT_READ : ATT_NONE;
        add(3, reinterpret_cast<const void *>(back_batch_kernel(att, kmc, vec, false)), block_threads(G.nmax),
            back_smem(G.nmax, kmc), bo[gi], bto[gi], bn[gi]);
    }
    {
        const size_t ao = put(T->blob, ga), to = put(T->blob, gt);
        add(4, reinterpret_cast<const void *>(gather_batch), 256, 0, ao, to, (int)gt.size());
    }
    *status = SPECT_OK;
    return T;
}

size_t tick_bytes(const TickTables *T) { return T->blob.size(); }

int tick_launch(TickTables *T, char *host, char *dev, hipStream_t st, hipStream_t up, hipEvent_t uploaded)
{
    if (!T->blob.empty()) {
        std::memcpy(host, T->blob.data(), T->blob.size());
        hipError_t e = hipMemcpyAsync(dev, host, T->blob.size(), hipMemcpyHostToDevice, up);
        if (e == hipSuccess) e = hipEventRecord(uploaded, up);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, uploaded, 0);
        if (e != hipSuccess) return hip_fail(e, "tick table upload");
    }
    for (const TickTables::Pad &pd : T->pads)
        if (const int st2 = launch_pad(pd.p, pd.src, pd.dst, pd.zs, st)) return st2;
    for (const TickTables::Launch &l : T->launches) {
        static const int prof[5] = {K_SENS, K_FWD_B, K_REDUCE_B, K_BACK_B, K_GATHER_B};
        allow_smem(l.fn, l.smem);
        ProfScope ps(prof[l.kind], st);
        const Task *tasks = reinterpret_cast<const Task *>(dev + l.tasks);
        switch (l.kind) {
        case 0:
        case 3: {
            BatchList<BackRotArgs> b{reinterpret_cast<const BackRotArgs *>(dev + l.args), tasks, l.ntasks};
            hipLaunchKernelGGL(reinterpret_cast<void (*)(BatchList<BackRotArgs>)>(const_cast<void *>(l.fn)),
                               dim3(l.ntasks), dim3(l.threads), l.smem, st, b);
            break;
        }
        case 1: {
            BatchList<FwdArgs> b{reinterpret_cast<const FwdArgs *>(dev + l.args), tasks, l.ntasks};
            hipLaunchKernelGGL(reinterpret_cast<void (*)(BatchList<FwdArgs>)>(const_cast<void *>(l.fn)),
                               dim3(l.ntasks), dim3(l.threads), l.smem, st, b);
            break;
        }
        case 2: {
            BatchList<ReduceArgs> b{reinterpret_cast<const ReduceArgs *>(dev + l.args), tasks, l.ntasks};
            hipLaunchKernelGGL(reduce_batch, dim3(l.ntasks), dim3(256), 0, st, b);
            break;
        }
        default: {
            BatchList<GatherArgs> b{reinterpret_cast<const GatherArgs *>(dev + l.args), tasks, l.ntasks};
            hipLaunchKernelGGL(gather_batch, dim3(l.ntasks), dim3(256), 0, st, b);
            break;
        }
        }
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? SPECT_OK : hip_fail(e, "tick launch");
}

void tick_free(TickTables *T) { delete T; }

}  // namespace spect_internal
