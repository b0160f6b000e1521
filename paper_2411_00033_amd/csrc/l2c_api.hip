// l2c_api.hip -- C ABI (include/leg2cheb.h): argument checking, plan sizes, the exact
// B(0), B(1) of the upward and downward transfers (the other plan tables are built on the
// device), device memory ownership, and dispatch to the kernels.
#include <atomic>
#include <cmath>
#include <mutex>
#include <cstdlib>
#include <cstring>
#include <new>
#include <algorithm>
#include <vector>

#include "../../include/leg2cheb.h"
#include "l2c_alloc.h"
#include "l2c_internal.h"
#include "l2c_batched.h"
#include "l2c_math.h"
#include "l2c_tuning_table.h"

namespace l2c {

int check_geometry_indices(int L, int M, int s);   // l2c_check.hip

// Allocation-failure hook: the k-th allocation from the arming call fails (0: disarmed).
static std::atomic<int64_t> g_fail_at{0};
static std::atomic<int64_t> g_live{0};   // allocations made here and not yet released

static bool injected_failure()
{
    int64_t k = g_fail_at.load();
    while (k > 0)
        if (g_fail_at.compare_exchange_weak(k, k - 1)) return k == 1;
    return false;
}

hipError_t dev_alloc_raw(void **ptr, size_t bytes)
{
    *ptr = nullptr;
    if (injected_failure()) return hipErrorOutOfMemory;
    const hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) *ptr = nullptr;
    else if (*ptr) ++g_live;
    return e;
}

void dev_free(const void *ptr)
{
    if (!ptr) return;
    (void)hipFree(const_cast<void *>(ptr));
    --g_live;
}

hipError_t host_alloc(void **ptr, size_t bytes, unsigned flags)
{
    *ptr = nullptr;
    if (injected_failure()) return hipErrorOutOfMemory;
    const hipError_t e = hipHostMalloc(ptr, bytes, flags);
    if (e != hipSuccess) *ptr = nullptr;
    else if (*ptr) ++g_live;
    return e;
}

void host_free(void *ptr)
{
    if (!ptr) return;
    (void)hipHostFree(ptr);
    --g_live;
}

}  // namespace l2c

namespace {

// Sizes of Eq. (numlevels): s_hat = leaf/2, L = ceil(log2(n/s_hat)) - 2,
// s = ceil(n / 2^(L+2)), N = s 2^(L+2).  L <= 0: the plan applies Alg. 1 directly.
void plan_sizes(int64_t n, int leaf, int *L, int *s, int64_t *n_pad)
{
    const int64_t shat = leaf / 2;
    int p = 0;
    while ((shat << p) < n) ++p;
    *L = p - 2;
    if (*L <= 0) {
        *L = 0;
        *s = 0;
        *n_pad = n;
        return;
    }
    const int64_t span = int64_t(1) << (*L + 2);
    *s = (int)((n + span - 1) / span);
    *n_pad = (int64_t)(*s) * span;
}

// B(0) and B(1) of Eq. (Tky): row n holds the coefficients of T_n((Y + 2l - 1)/2) in
// T_k(Y).  Built by the three-term recurrence T_{n+1}(u) = 2u T_n(u) - T_{n-1}(u)
// with u = (Y + a)/2, a = 2l - 1, and Y T_j = (T_{j+1} + T_{|j-1|})/2.  Every
// coefficient is a dyadic rational with a small denominator (App. A3), so the FP64
// arithmetic here is exact.
void b_matrices(int M, std::vector<double> &B)
{
    B.assign(2 * M * M, 0.0);
    for (int l = 0; l < 2; ++l) {
        const double a = 2.0 * l - 1.0;
        std::vector<std::vector<double>> c(M, std::vector<double>(M + 1, 0.0));
        c[0][0] = 1.0;
        if (M > 1) {
            c[1][0] = 0.5 * a;
            c[1][1] = 0.5;
        }
        for (int n = 1; n + 1 < M; ++n) {
            std::vector<double> nxt(M + 1, 0.0);
            for (int j = 0; j <= n; ++j) {
                const double v = c[n][j];
                if (v == 0.0) continue;
                // 2u T_n = (Y + a) T_n
                nxt[j + 1] += 0.5 * v;
                nxt[j == 0 ? 1 : j - 1] += 0.5 * v;
                nxt[j] += a * v;
            }
            for (int j = 0; j <= n + 1; ++j) nxt[j] -= c[n - 1][j];
            c[n + 1] = nxt;
        }
        for (int n = 0; n < M; ++n)
            for (int k = 0; k < M; ++k) B[(size_t)l * M * M + n * M + k] = c[n][k];
    }
}

// The nodal basis (Eq. (AijLag)): Lagrange polynomials l_k on the Chebyshev-Gauss nodes
// x_k = cos((k + 1/2) pi / M), evaluated through the discrete orthogonality of T_j at those
// nodes, l_k(x) = (1/M) (1 + 2 sum_{j=1}^{M-1} T_j(x_k) T_j(x)), in long double.
long double lagrange(int M, int k, long double x)
{
    const long double xk = cosl(((long double)k + 0.5L) * 3.141592653589793238462643383279502884L / (long double)M);
    long double tk0 = 1.0L, tk1 = xk, t0 = 1.0L, t1 = x, sum = 1.0L;
    if (M > 1) sum += 2.0L * tk1 * t1;
    for (int j = 2; j < M; ++j) {
        const long double tk = 2.0L * xk * tk1 - tk0, t = 2.0L * x * t1 - t0;
        sum += 2.0L * tk * t;
        tk0 = tk1;
        tk1 = tk;
        t0 = t1;
        t1 = t;
    }
    return sum / (long double)M;
}

// Nodal transfers: B(l)[k][j] = l_k((x_j + 2l - 1)/2), the parent's basis function k at
// child l's node j (left child l = 0), so that w(parent) = B(0) w(2b) + B(1) w(2b+1) and
// c(child l) += B(l)^T c(parent), as in the modal case.
void nodal_b_matrices(int M, std::vector<double> &B)
{
    B.assign(2 * M * M, 0.0);
    for (int l = 0; l < 2; ++l)
        for (int j = 0; j < M; ++j) {
            const long double xj =
                cosl(((long double)j + 0.5L) * 3.141592653589793238462643383279502884L / (long double)M);
            const long double u = (xj + 2.0L * l - 1.0L) / 2.0L;
            for (int k = 0; k < M; ++k) B[(size_t)l * M * M + k * M + j] = (double)lagrange(M, k, u);
        }
}

// Nodal leaf matrices: L[sigma][m][k] = l_k(X), X = -1 + (2m + sigma)/s (the points of
// Eq. (Xs)).
void nodal_leaf_matrices(int M, int s, std::vector<double> &Lm)
{
    Lm.assign((size_t)2 * s * M, 0.0);
    for (int sg = 0; sg < 2; ++sg)
        for (int m = 0; m < s; ++m) {
            const long double x = -1.0L + (long double)(2 * m + sg) / (long double)s;
            for (int k = 0; k < M; ++k) Lm[((size_t)sg * s + m) * M + k] = (double)lagrange(M, k, x);
        }
}

bool rank_supported(int M)
{
    switch (M) {
#define L2C_CASE(MM) \
    case MM: return true;
        L2C_FOR_EACH_RANK(L2C_CASE)
#undef L2C_CASE
    default: return false;
    }
}

void free_plan(l2c_plan_s *p)
{
    if (!p) return;
    l2c::dev_free(p->d_top);
    l2c::dev_free(p->d_bot);
    l2c::dev_free(p->d_T);
    l2c::dev_free(p->d_B);
    l2c::dev_free(p->d_P);
    l2c::dev_free(p->d_XG);
    l2c::dev_free(p->d_D);
    l2c::dev_free(p->d_w);
    l2c::dev_free(p->d_pub);
    l2c::dev_free(p->d_topsch);
    l2c::host_free(p->h_status);
    l2c::dev_free(p->d_bA);
    l2c::dev_free(p->d_bT);
    l2c::dev_free(p->d_bB);
    l2c::dev_free(p->d_bP);
    l2c::dev_free(p->d_bQ);
    l2c::dev_free(p->d_bw);
    l2c::dev_free(p->d_bS);
    l2c::dev_free(p->d_dense);
    l2c::dev_free(p->d_dir);
    l2c::dev_free(p->d_lm);
    l2c::dev_free(p->d_cf);
    delete p;
}

bool use_fused(const l2c_plan_s *p) { return p->fused_ok && p->fused_on; }

// Status words of the plan's single-launch executes that have ended, as bits (word k ->
// bit k).  A plain read of pinned host memory: it does not wait for running kernels.
int status_bits(const l2c_plan_s *p)
{
    if (!p->h_status) return 0;
    const volatile int *w = p->h_status;
    int bits = 0;
    for (int k = 0; k < l2c::kStatusWords; ++k)
        if (w[k] != 0) bits |= 1 << k;
    return bits;
}
bool batched_form(int precision)
{
    return precision == L2C_FP32 || precision == L2C_BF16X2 || precision == L2C_FP16X2;
}
bool use_batched(const l2c_plan_s *p) { return p->L > 0 && (batched_form(p->precision) || p->tile64); }
size_t elem_bytes(const l2c_plan_s *p) { return batched_form(p->precision) ? sizeof(float) : sizeof(double); }

}  // namespace

struct l2c_batch_s {
    int device = 0;
    int64_t count = 0;
    std::vector<int64_t> n;                 // caller order
    std::vector<l2c_plan_s *> plans;        // one per group
    std::vector<int64_t> gstart;            // group g holds positions [gstart[g], gstart[g+1])
    std::vector<int64_t> order;             // position -> caller index
    int64_t *d_n = nullptr;                 // [count] lengths, in position order
    const double **d_in = nullptr;          // [count] input pointers, in position order
    double **d_out = nullptr;               // [count] output pointers, in position order
    void *h_stage = nullptr;                // pinned [2][count] pointers for the copies
    void *h_cap = nullptr;                  // pinned [2][count] pointers of the latest captured call
    hipEvent_t staged = nullptr;            // the last pointer copy
    hipEvent_t done = nullptr;              // the end of the last execute on its stream
    bool any = false;                       // done has been recorded
    // groups run concurrently on side streams (default priority), forked from and joined
    // back into the caller's stream; group g runs on side stream lane[g] (balanced by work)
    static constexpr int kSide = 4;
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr, join[kSide] = {};
    std::vector<int> lane;
    // batched forms: one launch per kernel shape for all groups with L >= 1
    l2c::BatGrouped *grouped = nullptr;
    // the kernels of an execute (everything after the pointer copies) captured once into a
    // graph on a private stream and replayed by every later execute
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_failed = false;              // capture or instantiation failed: launch directly
};

namespace {

void free_batch(l2c_batch_s *b)
{
    for (l2c_plan_s *p : b->plans) leg2cheb_destroy(p);
    l2c::dev_free(b->d_n);
    l2c::dev_free((void *)b->d_in);
    l2c::dev_free(b->d_out);
    l2c::host_free(b->h_stage);
    l2c::host_free(b->h_cap);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->staged) (void)hipEventDestroy(b->staged);
    if (b->done) (void)hipEventDestroy(b->done);
    l2c::batched_grouped_free(b->grouped);
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (int k = 0; k < l2c_batch_s::kSide; ++k) {
        if (b->join[k]) (void)hipEventDestroy(b->join[k]);
        if (b->side[k]) (void)hipStreamDestroy(b->side[k]);
    }
    delete b;
}

// Pointer lists of a ragged execute in group (position) order: dst[0:count] inputs,
// dst[count:2 count] outputs.
void stage_pointers(const l2c_batch_s *b, void **dst, const double *const *in, double *const *out)
{
    for (int64_t k = 0; k < b->count; ++k) {
        dst[k] = (void *)in[b->order[k]];
        dst[b->count + k] = (void *)out[b->order[k]];
    }
}

int ensure_workspace(l2c_plan_s *p, int64_t batch);
int ensure_bworkspace(l2c_plan_s *p, int64_t items);

// The kernels of a ragged execute on stream st (the pointer lists are on the device).
// Batched forms: direct groups (L = 0), then every other group in grouped launches.  FP64:
// the groups run concurrently on the side streams, forked from and joined back into st;
// FP64 groups take the three-launch path (single-launch kernels need all their workgroups
// resident and are never run side by side).  Nothing here allocates (the workspaces are
// sized at batch-plan time) or synchronizes, so the sequence can be captured.
int enqueue_batch(l2c_batch_s *b, hipStream_t st)
{
    if (b->grouped) {
        for (size_t g = 0; g < b->plans.size(); ++g) {
            l2c_plan_s *p = b->plans[g];
            if (p->L != 0) continue;
            const int64_t k0 = b->gstart[g], items = b->gstart[g + 1] - k0;
            const l2c::ItemArrays ia = {b->d_n + k0, b->d_in + k0, b->d_out + k0};
            if (l2c::launch_execute(*p, nullptr, nullptr, items, st, &ia) != hipSuccess) return L2C_EHIP;
        }
        return l2c::batched_grouped_launch(b->grouped, st) == hipSuccess ? L2C_OK : L2C_EHIP;
    }
    if (hipEventRecord(b->fork, st) != hipSuccess) return L2C_EHIP;
    for (int k = 0; k < l2c_batch_s::kSide; ++k)
        if (hipStreamWaitEvent(b->side[k], b->fork, 0) != hipSuccess) return L2C_EHIP;
    for (size_t g = 0; g < b->plans.size(); ++g) {
        l2c_plan_s *p = b->plans[g];
        hipStream_t gs = b->side[b->lane[g]];
        const int64_t k0 = b->gstart[g], items = b->gstart[g + 1] - k0;
        const l2c::ItemArrays ia = {b->d_n + k0, b->d_in + k0, b->d_out + k0};
        if (use_batched(p)) {
            if (items > p->bw_tiles * 16) return L2C_EINVAL;
            if (l2c::launch_batched(*p, nullptr, nullptr, items, gs, &ia) != hipSuccess) return L2C_EHIP;
        } else if (p->d_dense) {
            if (l2c::launch_dense(*p, nullptr, nullptr, items, gs, &ia) != hipSuccess) return L2C_EHIP;
        } else {
            if (p->L > 0 && items > p->ws_batch) return L2C_EINVAL;
            if (l2c::launch_execute(*p, nullptr, nullptr, items, gs, &ia) != hipSuccess) return L2C_EHIP;
        }
    }
    for (int k = 0; k < l2c_batch_s::kSide; ++k)
        if (hipEventRecord(b->join[k], b->side[k]) != hipSuccess || hipStreamWaitEvent(st, b->join[k], 0) != hipSuccess)
            return L2C_EHIP;
    return L2C_OK;
}

// Capture the kernels of an execute once, on the batch's private stream, and instantiate
// the graph; on any failure the batch launches directly from then on.
void build_batch_graph(l2c_batch_s *b)
{
    hipGraph_t g = nullptr;
    bool ok = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        const int rc = enqueue_batch(b, b->cap);
        ok = hipStreamEndCapture(b->cap, &g) == hipSuccess && rc == L2C_OK && g;
    }
    if (ok) ok = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {
        b->exec = nullptr;
        b->graph_failed = true;
        (void)hipGetLastError();
    }
}

int ensure_workspace(l2c_plan_s *p, int64_t batch)
{
    if (p->L == 0 || batch <= p->ws_batch) return L2C_OK;
    if (p->ws_batch > 0) {
        if (hipDeviceSynchronize() != hipSuccess) return L2C_EHIP;
    }
    l2c::dev_free(p->d_w);
    l2c::dev_free(p->d_cf);
    p->d_w = nullptr;
    p->d_cf = nullptr;
    p->ws_batch = 0;
    const size_t bytes = (size_t)batch * p->geo.NT * 2 * p->M * sizeof(double);
    if (l2c::dev_alloc(&p->d_w, bytes) != hipSuccess ||
        (p->regen &&
         l2c::dev_alloc(&p->d_cf, std::max<size_t>(256, (size_t)batch * l2c::regen_cf_per_item(p->geo) * sizeof(double))) !=
             hipSuccess)) {
        (void)hipGetLastError();
        l2c::dev_free(p->d_w);
        p->d_w = nullptr;
        return L2C_ENOMEM;
    }
    p->ws_batch = batch;
    return L2C_OK;
}

int plan_impl(l2c_plan_t *plan, int64_t n, int direction, int leaf_size, int rank, int precision, int64_t max_batch,
              void *stream, bool full_leaf, int basis = L2C_MODAL, bool regen = false);

// Workspace of the batched form: tiles of 16 items, NT nodes x 2 parities x 256 values.
int ensure_bworkspace(l2c_plan_s *p, int64_t items)
{
    const int64_t tiles = std::min((items + 15) / 16, l2c::kBatMaxTiles);
    if (tiles <= p->bw_tiles) return L2C_OK;
    if (p->bw_tiles > 0) {
        if (hipDeviceSynchronize() != hipSuccess) return L2C_EHIP;
    }
    l2c::dev_free(p->d_bw);
    p->d_bw = nullptr;
    p->bw_tiles = 0;
    const size_t bytes = (size_t)tiles * p->geo.NT * 2 * 256 * elem_bytes(p);
    if (l2c::dev_alloc(&p->d_bw, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p->d_bw = nullptr;
        return L2C_ENOMEM;
    }
    p->bw_tiles = tiles;
    return L2C_OK;
}

// k_direct's P and Q tables (plans with L = 0 and short FP64 plans).
int build_direct_tables(l2c_plan_s *p, hipStream_t st)
{
    if (l2c::dev_alloc(&p->d_dir, (size_t)l2c::direct_table_len(p->n) * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return L2C_ENOMEM;
    }
    if (l2c::direct_build(*p, p->d_dir, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        return L2C_EHIP;
    }
    p->table_bytes += l2c::direct_table_len(p->n) * (int64_t)sizeof(double);
    return L2C_OK;
}

// Tables of the batched form from the FP64 plan tables (rounded once to FP32 on the
// device), then the FP64 Ahat is released.
int build_batched_tables(l2c_plan_s *p, hipStream_t st)
{
    const int M = p->M, s = p->s;
    const int64_t blocks = l2c::level_block_offset(p->L);
    const int64_t qlen = p->n_pad + 2 * (int64_t)s;
    const int64_t nT = 2 * (int64_t)s * M, nP = 2 * (int64_t)s;
    const int64_t nB = (int64_t)M * M * (p->basis == L2C_NODAL ? 2 : 1);   // nodal: B(1) is a table too
    const size_t eb = elem_bytes(p);
    bool ok = l2c::dev_alloc(&p->d_bA, (size_t)blocks * 3 * 256 * eb) == hipSuccess &&
              l2c::dev_alloc(&p->d_bQ, (size_t)qlen * sizeof(double)) == hipSuccess &&   // near field: FP64
              l2c::dev_alloc(&p->d_bT, nT * eb) == hipSuccess &&
              l2c::dev_alloc(&p->d_bB, nB * eb) == hipSuccess &&
              l2c::dev_alloc(&p->d_bP, nP * sizeof(double)) == hipSuccess &&
              (p->precision != L2C_FP16X2 || l2c::dev_alloc(&p->d_bS, (size_t)blocks * 3 * sizeof(float)) == hipSuccess);
    if (!ok) {
        (void)hipGetLastError();
        return L2C_ENOMEM;
    }
    // P (near field) stays FP64 in every form; the FP64 tile form keeps T and B(0) in FP64
    ok = hipMemcpyAsync(p->d_bP, p->d_P + l2c::kPLead, nP * 8, hipMemcpyDeviceToDevice, st) == hipSuccess;
    if (p->tile64)
        ok = ok && hipMemcpyAsync(p->d_bT, p->d_T, nT * 8, hipMemcpyDeviceToDevice, st) == hipSuccess &&
             hipMemcpyAsync(p->d_bB, p->d_B, nB * 8, hipMemcpyDeviceToDevice, st) == hipSuccess;
    else
        ok = ok && l2c::launch_to_f32(p->d_T, (float *)p->d_bT, nT, st) == hipSuccess &&
             l2c::launch_to_f32(p->d_B, (float *)p->d_bB, nB, st) == hipSuccess;
    ok = ok && l2c::batched_build_tables(*p, p->d_bA, p->d_bQ, qlen, st) == hipSuccess &&
         hipStreamSynchronize(st) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        return L2C_EHIP;
    }
    l2c::dev_free(p->d_top);
    l2c::dev_free(p->d_bot);
    p->d_top = p->d_bot = nullptr;
    p->top_bytes = (int64_t)blocks * 3 * 256 * (int64_t)eb;   // Ahat as stored
    p->bot_bytes = 0;
    p->table_bytes = p->top_bytes + (nT + nB) * (int64_t)eb + (qlen + nP) * 8 +
                     (nT + 3 * (int64_t)M * M + l2c::p_table_len(s) + M) * 8 +   // FP64 T, B(0), B(1), D, P, points
                     (p->d_bS ? blocks * 3 * (int64_t)sizeof(float) : 0);
    return L2C_OK;
}

}  // namespace

extern "C" {

const char *leg2cheb_strerror(int code)
{
    switch (code) {
    case L2C_OK: return "success";
    case L2C_EINVAL: return "invalid argument";
    case L2C_ENOMEM: return "out of memory";
    case L2C_EHIP: return "HIP runtime error";
    case L2C_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
    }
}

int leg2cheb_batch_tuning(int precision, struct l2c_tuning_bucket *buckets, int32_t cap, int32_t *count)
{
    if (!count || cap < 0 || (cap > 0 && !buckets)) return L2C_EINVAL;
    if (precision != L2C_FP64 && !batched_form(precision)) return L2C_EINVAL;
    const l2c::TuneRow *rows = nullptr;
    const int nr = l2c::builtin_tuning(precision, &rows);
    *count = nr;
    for (int k = 0; k < nr && k < cap; ++k) buckets[k] = {rows[k].n_max, rows[k].leaf_size, rows[k].rank};
    return L2C_OK;
}

int leg2cheb_batch_plan(l2c_batch_t *batch, int64_t count, const int64_t *n, const int *direction, int precision,
                        const struct l2c_tuning *tuning, void *stream)
{
    if (!batch) return L2C_EINVAL;
    *batch = nullptr;
    if (count < 1 || !n || !direction) return L2C_EINVAL;
    for (int64_t i = 0; i < count; ++i)
        if (n[i] < 1 || (direction[i] != L2C_LEG2CHEB && direction[i] != L2C_CHEB2LEG)) return L2C_EINVAL;
    if (precision != L2C_FP64 && !batched_form(precision)) return L2C_EINVAL;
    // size buckets: the caller's, or the library's table for the precision
    std::vector<l2c_tuning_bucket> bk;
    if (tuning) {
        if (tuning->count < 1 || tuning->count > 32 || !tuning->buckets) return L2C_EINVAL;
        bk.assign(tuning->buckets, tuning->buckets + tuning->count);
    } else {
        const l2c::TuneRow *rows = nullptr;
        const int nr = l2c::builtin_tuning(precision, &rows);
        for (int k = 0; k < nr; ++k) bk.push_back({rows[k].n_max, rows[k].leaf_size, rows[k].rank});
    }
    for (size_t k = 0; k < bk.size(); ++k) {
        if (k > 0 && bk[k].n_max <= bk[k - 1].n_max) return L2C_EINVAL;
        if (bk[k].leaf_size < 4 || bk[k].leaf_size > 128 || (bk[k].leaf_size & 1)) return L2C_EINVAL;
        if (bk[k].rank < 1 || bk[k].rank > 32) return L2C_EINVAL;
    }
    for (const auto &b : bk) {
        if (!leg2cheb_rank_supported(b.rank)) return L2C_EUNSUPPORTED;
        if (batched_form(precision) && (b.rank > 16 || b.leaf_size > 64)) return L2C_EUNSUPPORTED;
    }
    if (batched_form(precision))
        for (int64_t i = 0; i < count; ++i)
            if (n[i] > (int64_t(1) << 28)) return L2C_EUNSUPPORTED;
    l2c_batch_s *b = new (std::nothrow) l2c_batch_s;
    if (!b) return L2C_ENOMEM;
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return L2C_EHIP;
    }
    b->count = count;
    // Groups: one per (bucket, L, direction); L = 0 transforms form one group per bucket and
    // direction.  Every group is planned with its bucket's full half-leaf s = leaf/2 (the same
    // L as Eq. (numlevels) gives, with more padding), so that few groups cover the batch and
    // the batched forms fill their 16-transform tiles.
    struct Key {
        int bucket, L, s, dir;
    };
    std::vector<int> Ls(count), Ss(count), Bs(count);
    for (int64_t i = 0; i < count; ++i) {
        int k = 0;
        while (k + 1 < (int)bk.size() && n[i] > bk[k].n_max) ++k;
        Bs[i] = k;
        int64_t np;
        plan_sizes(n[i], bk[k].leaf_size, &Ls[i], &Ss[i], &np);
        Ss[i] = Ls[i] > 0 ? bk[k].leaf_size / 2 : 0;   // full half-leaf
    }
    std::vector<Key> keys;
    std::vector<int64_t> ord(count);
    {
        std::vector<int> gof(count);
        for (int64_t i = 0; i < count; ++i) {
            int g = -1;
            for (size_t k = 0; k < keys.size(); ++k)
                if (keys[k].bucket == Bs[i] && keys[k].L == Ls[i] && keys[k].s == Ss[i] && keys[k].dir == direction[i]) {
                    g = (int)k;
                    break;
                }
            if (g < 0) {
                keys.push_back({Bs[i], Ls[i], Ss[i], direction[i]});
                g = (int)keys.size() - 1;
            }
            gof[i] = g;
        }
        b->gstart.assign(keys.size() + 1, 0);
        for (int64_t i = 0; i < count; ++i) ++b->gstart[gof[i] + 1];
        for (size_t g = 0; g < keys.size(); ++g) b->gstart[g + 1] += b->gstart[g];
        std::vector<int64_t> fill(b->gstart.begin(), b->gstart.end() - 1);
        for (int64_t i = 0; i < count; ++i) ord[fill[gof[i]]++] = i;
        // longest first inside each group: tiles of 16 transforms of the batched forms then
        // hold similar lengths, and workgroups past a tile's longest transform end at once
        for (size_t g = 0; g < keys.size(); ++g)
            std::stable_sort(ord.begin() + b->gstart[g], ord.begin() + b->gstart[g + 1],
                             [&](int64_t x, int64_t y) { return n[x] > n[y]; });
    }
    const int G = (int)keys.size();
    b->order = ord;
    std::vector<int64_t> nord(count);
    for (int64_t k = 0; k < count; ++k) nord[k] = n[ord[k]];
    int rc = L2C_OK;
    for (int g = 0; g < G && rc == L2C_OK; ++g) {
        int64_t nmax = 0;
        for (int64_t k = b->gstart[g]; k < b->gstart[g + 1]; ++k) nmax = std::max(nmax, nord[k]);
        l2c_plan_t pl = nullptr;
        const int64_t items = b->gstart[g + 1] - b->gstart[g];
        const l2c_tuning_bucket &tb = bk[keys[g].bucket];
        rc = plan_impl(&pl, nmax, keys[g].dir, tb.leaf_size, tb.rank, precision, items, stream, true);
        if (rc == L2C_OK) {
            b->plans.push_back(pl);
            // groups run side by side: FP64 groups use the three-launch path
            pl->fused_on = false;
            if (!use_batched(pl) && !pl->d_dense) rc = ensure_workspace(pl, items);
        }
    }
    const size_t cb = (size_t)count * sizeof(void *);
    if (rc == L2C_OK &&
        (l2c::dev_alloc(&b->d_n, (size_t)count * sizeof(int64_t)) != hipSuccess ||
         l2c::dev_alloc(&b->d_in, cb) != hipSuccess || l2c::dev_alloc(&b->d_out, cb) != hipSuccess ||
         l2c::host_alloc(&b->h_stage, 2 * cb) != hipSuccess || l2c::host_alloc(&b->h_cap, 2 * cb) != hipSuccess ||
         hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess))
        rc = L2C_ENOMEM;
    if (rc == L2C_OK && hipMemcpy(b->d_n, nord.data(), (size_t)count * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess)
        rc = L2C_EHIP;
    if (rc == L2C_OK && (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
                         hipEventCreateWithFlags(&b->done, hipEventDisableTiming) != hipSuccess ||
                         hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess))
        rc = L2C_EHIP;
    for (int k = 0; k < l2c_batch_s::kSide && rc == L2C_OK; ++k)
        if (hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming) != hipSuccess)
            rc = L2C_EHIP;
    if (rc == L2C_OK && batched_form(precision)) {
        std::vector<l2c::ItemArrays> ia(G);
        std::vector<int64_t> items(G);
        for (int g = 0; g < G; ++g) {
            const int64_t k0 = b->gstart[g];
            ia[g] = {b->d_n + k0, b->d_in + k0, b->d_out + k0};
            items[g] = b->gstart[g + 1] - k0;
        }
        const hipError_t e = l2c::batched_grouped_make(b->plans.data(), ia.data(), items.data(), G, &b->grouped);
        if (e == hipErrorOutOfMemory) rc = L2C_ENOMEM;
        else if (e != hipSuccess) b->grouped = nullptr;   // per-group launches instead
        (void)hipGetLastError();
    }
    if (rc == L2C_OK) {
        // longest work first onto the least-loaded side stream (work ~ items x padded length)
        std::vector<int> gi(G);
        std::vector<double> work(G), load(l2c_batch_s::kSide, 0.0);
        for (int g = 0; g < G; ++g) {
            gi[g] = g;
            work[g] = (double)(b->gstart[g + 1] - b->gstart[g]) * (double)std::max<int64_t>(b->plans[g]->n_pad, 1);
        }
        std::sort(gi.begin(), gi.end(), [&](int x, int y) { return work[x] > work[y]; });
        b->lane.assign(G, 0);
        for (int g : gi) {
            const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            b->lane[g] = k;
            load[k] += work[g];
        }
    }
    if (rc != L2C_OK) {
        (void)hipGetLastError();
        free_batch(b);
        return rc;
    }
    b->n.assign(n, n + count);
    *batch = b;
    return L2C_OK;
}

int leg2cheb_batch_execute(l2c_batch_t b, const double *const *in, double *const *out, void *stream)
{
    if (!b || !in || !out) return L2C_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return L2C_EHIP;
    if (dev != b->device) return L2C_EINVAL;
    // every output disjoint from every input and every other output
    std::vector<std::pair<const char *, const char *>> outs(b->count);
    for (int64_t i = 0; i < b->count; ++i) {
        if (!in[i] || !out[i]) return L2C_EINVAL;
        outs[i] = {(const char *)out[i], (const char *)(out[i] + b->n[i])};
    }
    std::sort(outs.begin(), outs.end());
    for (int64_t i = 1; i < b->count; ++i)
        if (outs[i].first < outs[i - 1].second) return L2C_EINVAL;
    for (int64_t i = 0; i < b->count; ++i) {
        const char *lo = (const char *)in[i], *hi = (const char *)(in[i] + b->n[i]);
        auto it = std::lower_bound(outs.begin(), outs.end(), std::make_pair(hi, hi));
        if (it != outs.begin() && std::prev(it)->second > lo) return L2C_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return L2C_EHIP;
    const size_t cb = (size_t)b->count * sizeof(void *);
    if (cs == hipStreamCaptureStatusActive) {
        // the caller captures this call into a graph of its own: the pointer copies read the
        // batch's capture staging (the pointers of the latest captured call) when the graph
        // runs; nothing here waits or synchronizes
        stage_pointers(b, (void **)b->h_cap, in, out);
        if (hipMemcpyAsync(b->d_in, b->h_cap, cb, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(b->d_out, (void **)b->h_cap + b->count, cb, hipMemcpyHostToDevice, st) != hipSuccess)
            return L2C_EHIP;
        return enqueue_batch(b, st);
    }
    if (cs != hipStreamCaptureStatusNone) return L2C_EINVAL;   // a capture that was invalidated
    if (hipEventSynchronize(b->staged) != hipSuccess) return L2C_EHIP;   // previous pointer copy done
    // the previous execute (possibly on another stream) still reads the device pointer
    // lists and the group workspaces until it ends: this one starts after it
    if (b->any && hipStreamWaitEvent(st, b->done, 0) != hipSuccess) return L2C_EHIP;
    stage_pointers(b, (void **)b->h_stage, in, out);
    if (hipMemcpyAsync(b->d_in, b->h_stage, cb, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(b->d_out, (void **)b->h_stage + b->count, cb, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventRecord(b->staged, st) != hipSuccess)
        return L2C_EHIP;
    if (!b->exec && !b->graph_failed) build_batch_graph(b);
    if (b->exec) {
        if (hipGraphLaunch(b->exec, st) != hipSuccess) return L2C_EHIP;
    } else {
        const int rc = enqueue_batch(b, st);
        if (rc != L2C_OK) return rc;
    }
    if (hipEventRecord(b->done, st) != hipSuccess) return L2C_EHIP;
    b->any = true;
    return L2C_OK;
}

int leg2cheb_batch_info(l2c_batch_t b, int64_t *groups, int64_t *table_bytes)
{
    if (!b) return L2C_EINVAL;
    if (groups) *groups = (int64_t)b->plans.size();
    if (table_bytes) {
        int64_t t = 0;
        for (l2c_plan_s *p : b->plans) t += p->table_bytes;
        *table_bytes = t;
    }
    return L2C_OK;
}

int leg2cheb_batch_destroy(l2c_batch_t b)
{
    if (!b) return L2C_OK;
    const bool ok = hipDeviceSynchronize() == hipSuccess;
    free_batch(b);
    return ok ? L2C_OK : L2C_EHIP;
}

int leg2cheb_rank_supported(int rank) { return rank_supported(rank) ? 1 : 0; }

int leg2cheb_debug_alloc_hook(int64_t fail_at, int64_t *pending, int64_t *live)
{
    if (fail_at < -1) return L2C_EINVAL;
    const int64_t before = fail_at >= 0 ? l2c::g_fail_at.exchange(fail_at) : l2c::g_fail_at.load();
    if (pending) *pending = before;
    if (live) *live = l2c::g_live.load();
    return L2C_OK;
}

int leg2cheb_debug_check_geometry(int64_t n, int leaf_size, int rank)
{
    if (n < 1 || n > (int64_t(1) << 31) || leaf_size < 4 || leaf_size > 128 || (leaf_size & 1) ||
        !rank_supported(rank))
        return L2C_EINVAL;
    int L = 0, s = 0;
    int64_t n_pad = 0;
    plan_sizes(n, leaf_size, &L, &s, &n_pad);
    if (L == 0) return L2C_OK;   // the direct product: no multipole index maps
    if (L >= L2C_MAX_LEVELS - 1) return L2C_EINVAL;
    return l2c::check_geometry_indices(L, rank, s);
}

}  // extern "C"

namespace {
// full_leaf: s = leaf_size / 2 instead of the smallest s of Eq. (numlevels) that covers n
// (same L; more padding), so that transforms of one L share every table.
int plan_impl(l2c_plan_t *plan, int64_t n, int direction, int leaf_size, int rank, int precision, int64_t max_batch,
              void *stream, bool full_leaf, int basis, bool regen);
}  // namespace

extern "C" {

int leg2cheb_plan_ex(l2c_plan_t *plan, int64_t n, int direction, int leaf_size, int rank, int precision,
                     int64_t max_batch, void *stream)
{
    return plan_impl(plan, n, direction, leaf_size, rank, precision, max_batch, stream, false);
}

int leg2cheb_plan_basis(l2c_plan_t *plan, int64_t n, int direction, int leaf_size, int rank, int precision,
                        int64_t max_batch, int basis, void *stream)
{
    return plan_impl(plan, n, direction, leaf_size, rank, precision, max_batch, stream, false, basis);
}

int leg2cheb_plan_tables(l2c_plan_t *plan, int64_t n, int direction, int leaf_size, int rank, int64_t max_batch,
                         int tables, void *stream)
{
    if (tables != L2C_TABLES_STORED && tables != L2C_TABLES_REGEN) {
        if (plan) *plan = nullptr;
        return L2C_EINVAL;
    }
    return plan_impl(plan, n, direction, leaf_size, rank, L2C_FP64, max_batch, stream, false, L2C_MODAL,
                     tables == L2C_TABLES_REGEN);
}

}  // extern "C"

namespace {
int plan_impl(l2c_plan_t *plan, int64_t n, int direction, int leaf_size, int rank, int precision, int64_t max_batch,
              void *stream, bool full_leaf, int basis, bool regen)
{
    if (!plan) return L2C_EINVAL;
    *plan = nullptr;
    if (n < 1 || n > (int64_t(1) << 31)) return L2C_EINVAL;
    if (direction != L2C_LEG2CHEB && direction != L2C_CHEB2LEG) return L2C_EINVAL;
    if (leaf_size < 4 || leaf_size > 128 || (leaf_size & 1)) return L2C_EINVAL;
    if (rank < 1 || rank > 32) return L2C_EINVAL;
    if (max_batch < 1) return L2C_EINVAL;
    if (precision != L2C_FP64 && !batched_form(precision)) return L2C_EINVAL;
    if (!rank_supported(rank)) return L2C_EUNSUPPORTED;
    // the batched forms: one 16 x 16 tile per node (M <= 16), s <= 32, rows of at most
    // 2^28 values (32-bit buffer ranges)
    if (batched_form(precision) && (rank > 16 || leaf_size > 64 || n > (int64_t(1) << 28))) return L2C_EUNSUPPORTED;
    if (basis != L2C_MODAL && basis != L2C_NODAL) return L2C_EINVAL;
    // regenerated far-field blocks: FP64, modal basis, the three-launch path
    if (regen && (precision != L2C_FP64 || basis != L2C_MODAL)) return L2C_EUNSUPPORTED;
    // the FP64 tile form: batches of FP64 transforms at rank <= 16, unless the dense or
    // direct products serve them better
    const bool tile64 = !regen && !batched_form(precision) && rank <= 16 && leaf_size <= 64 && n <= (int64_t(1) << 28) &&
                        max_batch >= l2c::kTile64MinBatch && !(n <= l2c::kDenseMaxN && max_batch >= l2c::kDenseMinBatch) &&
                        !(n <= l2c::kDirectMaxN && max_batch <= l2c::direct_max_work(n) / (n * n));
    // the nodal basis runs on the batched kernels only (dense tile products)
    if (basis == L2C_NODAL && !batched_form(precision) && !tile64) return L2C_EUNSUPPORTED;

    l2c_plan_s *p = new (std::nothrow) l2c_plan_s();
    if (!p) return L2C_ENOMEM;
    p->n = n;
    p->direction = direction;
    p->precision = precision;
    p->leaf = leaf_size;
    p->M = rank;
    p->basis = basis;
    p->max_batch = max_batch;
    p->regen = regen;
    if (hipGetDevice(&p->device) != hipSuccess) {
        delete p;
        return L2C_EHIP;
    }
    plan_sizes(n, leaf_size, &p->L, &p->s, &p->n_pad);
    if (full_leaf && p->L > 0) {
        p->s = leaf_size / 2;
        p->n_pad = (int64_t)p->s << (p->L + 2);
    }
    if (p->L >= L2C_MAX_LEVELS - 1) {
        delete p;
        return L2C_EINVAL;
    }
    if (!batched_form(precision) && l2c::prepare_launches(*p) != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        return L2C_EHIP;
    }
    hipStream_t st = (hipStream_t)stream;
    if (p->L > 0) {
        const int L = p->L, M = p->M, s = p->s;
        p->nb = (p->n_pad / (2 * s)) - L - 2;   // Eq. (total_blocks_and_mats)
        p->nc = 3 * p->nb;
        p->geo = l2c::make_geometry(L, M, s);
        const int64_t top_blocks = l2c::level_block_offset(p->geo.groot + 1);
        p->top_bytes = top_blocks * 3 * M * M * (int64_t)sizeof(double);
        p->bot_bytes = regen ? 0 : (int64_t(1) << (p->geo.groot + 2)) * p->geo.sub_groups * 64 * 3 * M * (int64_t)sizeof(double);
        // Lambda((y-x)/2) per level and offset (the plan's samples; regenerating executes)
        const int64_t nlm = (int64_t)L * 2 * M * M;

        // B(0), B(1) on the host (exact dyadic rationals); T, P, the Chebyshev-Gauss points,
        // the DCT matrix and Ahat on the device
        std::vector<double> B, Lnod;
        if (basis == L2C_NODAL) {
            nodal_b_matrices(M, B);
            nodal_leaf_matrices(M, s, Lnod);
        } else {
            b_matrices(M, B);
        }
        const int64_t nT = 2 * (int64_t)s * M, nP = l2c::p_table_len(s);

        bool ok = l2c::dev_alloc(&p->d_top, p->top_bytes) == hipSuccess &&
                  (p->bot_bytes == 0 || l2c::dev_alloc(&p->d_bot, p->bot_bytes) == hipSuccess) &&
                  l2c::dev_alloc(&p->d_T, nT * sizeof(double)) == hipSuccess &&
                  l2c::dev_alloc(&p->d_B, B.size() * sizeof(double)) == hipSuccess &&
                  l2c::dev_alloc(&p->d_P, nP * sizeof(double)) == hipSuccess &&
                  l2c::dev_alloc(&p->d_XG, M * sizeof(double)) == hipSuccess &&
                  l2c::dev_alloc(&p->d_D, (size_t)M * M * sizeof(double)) == hipSuccess &&
                  l2c::dev_alloc(&p->d_lm, nlm * sizeof(double)) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            free_plan(p);
            return L2C_ENOMEM;
        }
        p->table_bytes = p->top_bytes + p->bot_bytes + (nT + (int64_t)B.size() + nP + M + (int64_t)M * M + nlm) * 8;
        ok = hipMemcpyAsync(p->d_B, B.data(), B.size() * 8, hipMemcpyHostToDevice, st) == hipSuccess &&
             l2c::launch_build_small(*p, st) == hipSuccess &&
             (Lnod.empty() || hipMemcpyAsync(p->d_T, Lnod.data(), Lnod.size() * 8, hipMemcpyHostToDevice, st) == hipSuccess) &&
             (p->bot_bytes == 0 || hipMemsetAsync(p->d_bot, 0, p->bot_bytes, st) == hipSuccess) &&
             l2c::launch_build_lminus(*p, st) == hipSuccess && l2c::launch_build_ahat(*p, st) == hipSuccess &&
             hipStreamSynchronize(st) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            free_plan(p);
            return L2C_EHIP;
        }
        p->tile64 = tile64;
        if (batched_form(precision) || p->tile64) {
            int rc = build_batched_tables(p, st);
            if (rc == L2C_OK) rc = ensure_bworkspace(p, max_batch);
            if (rc != L2C_OK) {
                free_plan(p);
                return rc;
            }
            *plan = p;
            return L2C_OK;
        }
        // short transforms: Alg. 1 row by row (the multipole tables stay available)
        p->direct_ok = !regen && n <= l2c::kDirectMaxN && max_batch <= l2c::direct_max_work(n) / (n * n);
        if (p->direct_ok) {
            const int rc = build_direct_tables(p, st);
            if (rc != L2C_OK) {
                free_plan(p);
                return rc;
            }
        }
        // batches of short transforms: the direct product on the matrix cores
        if (!regen && n <= l2c::kDenseMaxN && max_batch >= l2c::kDenseMinBatch) {
            const int64_t HP = l2c::dense_hp(n);
            ok = l2c::dev_alloc(&p->d_dense, (size_t)2 * HP * HP * sizeof(double)) == hipSuccess &&
                 l2c::dense_build(*p, p->d_dense, st) == hipSuccess && hipStreamSynchronize(st) == hipSuccess;
            if (!ok) {
                (void)hipGetLastError();
                free_plan(p);
                return L2C_ENOMEM;
            }
            p->table_bytes += 2 * HP * HP * (int64_t)sizeof(double);
        }
        // single-launch path: items per launch with every workgroup resident
        int64_t items = 0;
        if (!regen && l2c::fused_max_items(*p, &items) != hipSuccess) {
            (void)hipGetLastError();
            items = 0;
        }
        if (items > 0) {
            // both halves of the exchange buffer start out "not written"
            const size_t pwords = (size_t)2 * items * p->geo.NX * 2 * p->M * 2;
            ok = l2c::dev_alloc(&p->d_pub, pwords * 4) == hipSuccess &&
                 l2c::fused_top_table(*p, &p->d_topsch) == hipSuccess &&
                 l2c::host_alloc((void **)&p->h_status, l2c::kStatusWords * sizeof(int),
                                 hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess;
            if (!ok) {
                (void)hipGetLastError();
                free_plan(p);
                return L2C_ENOMEM;
            }
            std::memset(p->h_status, 0, l2c::kStatusWords * sizeof(int));
            ok = hipHostGetDevicePointer((void **)&p->d_status, p->h_status, 0) == hipSuccess &&
                 hipDeviceGetAttribute(&p->clock_khz, hipDeviceAttributeWallClockRate, p->device) == hipSuccess &&
                 p->clock_khz > 0 &&
                 hipMemsetD32Async((hipDeviceptr_t)p->d_pub, (int)l2c::kPubEmptyHalf, pwords, st) == hipSuccess &&
                 hipStreamSynchronize(st) == hipSuccess;
            if (!ok) {
                (void)hipGetLastError();
                free_plan(p);
                return L2C_EHIP;
            }
            p->fused_ok = true;
            p->fused_items = items;
        }
        const int rc = ensure_workspace(p, use_fused(p) ? std::min(max_batch, p->fused_items) : max_batch);
        if (rc != L2C_OK) {
            free_plan(p);
            return rc;
        }
    } else {
        const int rc = build_direct_tables(p, st);   // L = 0: Alg. 1 only
        if (rc != L2C_OK) {
            free_plan(p);
            return rc;
        }
    }
    *plan = p;
    return L2C_OK;
}
}  // namespace

extern "C" {

int leg2cheb_plan(l2c_plan_t *plan, int64_t n, int direction, int leaf_size, int rank)
{
    return leg2cheb_plan_ex(plan, n, direction, leaf_size, rank, L2C_FP64, 1, nullptr);
}

}  // extern "C"

namespace {
// Argument checks shared by leg2cheb_execute and leg2cheb_execute_noalloc (batch >= 1).
int check_execute(l2c_plan_t plan, const double *in, double *out, int64_t batch)
{
    if (!in || !out) return L2C_EINVAL;
    const int64_t len = batch * plan->n;
    if (batch > (int64_t(1) << 40) / plan->n) return L2C_EINVAL;
    const char *ib = (const char *)in, *ie = (const char *)(in + len);
    const char *ob = (const char *)out, *oe = (const char *)(out + len);
    if (ib < oe && ob < ie) return L2C_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return L2C_EHIP;
    if (dev != plan->device) return L2C_EINVAL;
    if (status_bits(plan) != 0) return L2C_EHIP;   // an earlier single-launch execute gave up a wait
    return L2C_OK;
}

bool direct_now(const l2c_plan_s *plan, int64_t batch)
{
    return plan->L > 0 && plan->direct_ok && plan->direct_on &&
           batch <= l2c::direct_max_work(plan->n) / (plan->n * plan->n);
}
}  // namespace

extern "C" {

int leg2cheb_execute_noalloc(l2c_plan_t plan, const double *in, double *out, int64_t batch, void *stream)
{
    if (!plan || batch < 0) return L2C_EINVAL;
    if (batch == 0) return L2C_OK;
    if (plan->precision != L2C_FP64 || plan->tile64 || (plan->regen && plan->L > 0)) return L2C_EUNSUPPORTED;
    const int rc = check_execute(plan, in, out, batch);
    if (rc != L2C_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    // the dense and direct paths use no workspace and allocate nothing
    if (plan->d_dense) return l2c::launch_dense(*plan, in, out, batch, st) == hipSuccess ? L2C_OK : L2C_EHIP;
    if (plan->L == 0 || direct_now(plan, batch))
        return l2c::launch_direct(*plan, in, out, batch, st) == hipSuccess ? L2C_OK : L2C_EHIP;
    const int64_t per_item = plan->geo.NT * 2 * plan->M * (int64_t)sizeof(double);
    if (batch > (int64_t)l2c::kNoallocScratchBytes / per_item) return L2C_EINVAL;
    double *w = nullptr;
    if (l2c::noalloc_scratch(plan->device, &w) != hipSuccess) {
        (void)hipGetLastError();
        return L2C_EHIP;
    }
    return l2c::launch_execute_scratch(*plan, in, out, batch, st, w) == hipSuccess ? L2C_OK : L2C_EHIP;
}

int leg2cheb_execute(l2c_plan_t plan, const double *in, double *out, int64_t batch, void *stream)
{
    if (!plan || batch < 0) return L2C_EINVAL;
    if (batch == 0) return L2C_OK;
    const int crc = check_execute(plan, in, out, batch);
    if (crc != L2C_OK) return crc;
    if (plan->d_dense) {
        if (l2c::launch_dense(*plan, in, out, batch, (hipStream_t)stream) != hipSuccess) return L2C_EHIP;
        return L2C_OK;
    }
    if (direct_now(plan, batch)) {
        if (l2c::launch_direct(*plan, in, out, batch, (hipStream_t)stream) != hipSuccess) return L2C_EHIP;
        return L2C_OK;
    }
    if (use_batched(plan)) {
        const int rc = ensure_bworkspace(plan, batch);
        if (rc != L2C_OK) return rc;
        if (l2c::launch_batched(*plan, in, out, batch, (hipStream_t)stream) != hipSuccess) return L2C_EHIP;
        return L2C_OK;
    }
    if (plan->L > 0 && use_fused(plan)) {
        const int rc = ensure_workspace(plan, std::min(batch, plan->fused_items));
        if (rc != L2C_OK) return rc;
        if (l2c::launch_fused(*plan, in, out, batch, (hipStream_t)stream) != hipSuccess) return L2C_EHIP;
        return L2C_OK;
    }
    const int rc = ensure_workspace(plan, batch);
    if (rc != L2C_OK) return rc;
    if (l2c::launch_execute(*plan, in, out, batch, (hipStream_t)stream) != hipSuccess) return L2C_EHIP;
    return L2C_OK;
}

}  // extern "C"

namespace {
// The plan cache: shared plans keyed by every plan argument and the device, each with a
// reference count; leg2cheb_destroy releases one reference.
std::mutex g_cache_mu;
std::vector<l2c_plan_s *> g_cache;
}  // namespace

extern "C" {

int leg2cheb_plan_cached(l2c_plan_t *plan, int64_t n, int direction, int leaf_size, int rank, int precision,
                         int64_t max_batch, int basis, void *stream)
{
    if (!plan) return L2C_EINVAL;
    *plan = nullptr;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return L2C_EHIP;
    std::lock_guard<std::mutex> lock(g_cache_mu);
    for (l2c_plan_s *p : g_cache) {
        if (p->device == dev && p->n == n && p->direction == direction && p->leaf == leaf_size && p->M == rank &&
            p->precision == precision && p->max_batch == max_batch && p->basis == basis) {
            ++p->cache_refs;
            *plan = p;
            return L2C_OK;
        }
    }
    l2c_plan_t p = nullptr;
    const int rc = plan_impl(&p, n, direction, leaf_size, rank, precision, max_batch, stream, false, basis);
    if (rc != L2C_OK) return rc;
    p->cache_refs = 1;
    g_cache.push_back(p);
    *plan = p;
    return L2C_OK;
}

int leg2cheb_plan_cache_size(int64_t *plans, int64_t *references)
{
    std::lock_guard<std::mutex> lock(g_cache_mu);
    int64_t r = 0;
    for (l2c_plan_s *p : g_cache) r += p->cache_refs;
    if (plans) *plans = (int64_t)g_cache.size();
    if (references) *references = r;
    return L2C_OK;
}

int leg2cheb_destroy(l2c_plan_t plan)
{
    if (!plan) return L2C_OK;
    {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        if (plan->cache_refs > 0) {
            if (--plan->cache_refs > 0) return L2C_OK;
            g_cache.erase(std::find(g_cache.begin(), g_cache.end(), plan));
        }
    }
    const bool ok = hipDeviceSynchronize() == hipSuccess;
    free_plan(plan);
    return ok ? L2C_OK : L2C_EHIP;
}

int leg2cheb_plan_info(l2c_plan_t plan, struct l2c_plan_info *info)
{
    if (!plan || !info) return L2C_EINVAL;
    std::memset(info, 0, sizeof(*info));
    info->n = plan->n;
    info->n_pad = plan->n_pad;
    info->levels = plan->L;
    info->s = plan->s;
    info->rank = plan->M;
    info->direction = plan->direction;
    info->precision = plan->precision;
    info->n_blocks = plan->nb;
    info->n_submatrices = plan->nc;
    info->table_bytes = plan->table_bytes;
    info->workspace_bytes = plan->ws_batch * plan->geo.NT * 2 * plan->M * (int64_t)sizeof(double) +
                            plan->bw_tiles * plan->geo.NT * 2 * 256 * (int64_t)elem_bytes(plan);
    info->ahat_bytes = plan->top_bytes + plan->bot_bytes;
    info->basis = plan->basis;
    info->path = plan->L == 0                           ? L2C_PATH_DIRECT
                 : plan->d_dense                        ? L2C_PATH_DENSE
                 : use_batched(plan)                    ? L2C_PATH_BATCHED
                 : plan->direct_ok && plan->direct_on   ? L2C_PATH_DIRECT
                 : use_fused(plan)                      ? L2C_PATH_SINGLE
                 : plan->regen                          ? L2C_PATH_REGEN
                                                        : L2C_PATH_THREE;
    return L2C_OK;
}

int leg2cheb_plan_export(l2c_plan_t plan, int table, void *dst, int64_t bytes, int64_t *needed)
{
    if (!plan || plan->L == 0) return L2C_EINVAL;
    const int M = plan->M;
    int64_t need;
    switch (table) {
    case 0: need = plan->nc * M * M * 8; break;
    case 1: need = (int64_t)2 * plan->s * M * 8; break;
    case 2: need = (int64_t)2 * M * M * 8; break;
    case 3: need = plan->geo.NT * 2 * M * 8; break;
    default: return L2C_EINVAL;
    }
    if (needed) *needed = need;
    if (!dst) return L2C_OK;
    if (bytes != need) return L2C_EINVAL;
    if (table == 3) {
        if (!plan->d_w) return L2C_EUNSUPPORTED;   // no FP64 workspace on this plan's paths
        return hipMemcpy(dst, plan->d_w, need, hipMemcpyDeviceToHost) == hipSuccess ? L2C_OK : L2C_EHIP;
    }
    if (table == 1) return hipMemcpy(dst, plan->d_T, need, hipMemcpyDeviceToHost) == hipSuccess ? L2C_OK : L2C_EHIP;
    if (table == 2) return hipMemcpy(dst, plan->d_B, need, hipMemcpyDeviceToHost) == hipSuccess ? L2C_OK : L2C_EHIP;
    if (!plan->d_top || plan->regen) return L2C_EUNSUPPORTED;   // FP32 plans keep Ahat only in the batched layout;
                                                                 // regenerating plans keep its top levels only
    double *tmp = nullptr;
    if (l2c::dev_alloc(&tmp, need) != hipSuccess) {
        (void)hipGetLastError();
        return L2C_ENOMEM;
    }
    bool ok = l2c::launch_export_ahat(*plan, tmp, nullptr) == hipSuccess &&
              hipMemcpy(dst, tmp, need, hipMemcpyDeviceToHost) == hipSuccess;
    l2c::dev_free(tmp);
    return ok ? L2C_OK : L2C_EHIP;
}

int leg2cheb_plan_set_option(l2c_plan_t plan, int option, int64_t value)
{
    if (!plan) return L2C_EINVAL;
    switch (option) {
    case L2C_OPT_SINGLE_LAUNCH:
        if (value != 0 && value != 1) return L2C_EINVAL;
        if (value == 1 && !plan->fused_ok) return L2C_EUNSUPPORTED;
        plan->fused_on = value == 1;
        return L2C_OK;
    case L2C_OPT_DIRECT:
        if (value != 0 && value != 1) return L2C_EINVAL;
        if (value == 1 && !plan->direct_ok) return L2C_EUNSUPPORTED;
        plan->direct_on = value == 1;
        return L2C_OK;
    case L2C_OPT_EXCHANGE_TIMEOUT_US:
        if (value < 0 || value > 60000000) return L2C_EINVAL;
        plan->poll_us = value;
        return L2C_OK;
    default: return L2C_EINVAL;
    }
}

int leg2cheb_plan_status(l2c_plan_t plan, int *status)
{
    if (!plan || !status) return L2C_EINVAL;
    *status = 0;
    if (!plan->h_status) return L2C_OK;
    if (hipDeviceSynchronize() != hipSuccess) return L2C_EHIP;
    *status = status_bits(plan);
    volatile int *w = plan->h_status;
    for (int k = 0; k < l2c::kStatusWords; ++k) w[k] = 0;
    return L2C_OK;
}

int leg2cheb_set_timing_events(l2c_plan_t plan, void *before, void *after)
{
    if (!plan) return L2C_EINVAL;
    plan->ev_before = (hipEvent_t)before;
    plan->ev_after = (hipEvent_t)after;
    return L2C_OK;
}

}  // extern "C"
