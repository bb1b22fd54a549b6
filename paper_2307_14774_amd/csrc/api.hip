// C ABI of libspc5: argument checks, CSR validation, device memory ownership
// and kernel dispatch.  See include/spc5.h for the contract of every call.
#include "spc5_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <vector>

namespace spc5 {

static thread_local std::string g_err;

int fail(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return status;
}

int hip_fail(hipError_t e, const char *what) {
    const int st = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? SPC5_ENOMEM
                                                                             : SPC5_EDEVICE;
    return fail(st, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

int default_ppt(double blockrows_per_panel) {
    // aim at about four sweeps of 64 block rows per wavefront
    if (!(blockrows_per_panel > 0.0)) return 64;
    const double p = std::floor(256.0 / blockrows_per_panel + 0.5);
    return (int)std::max(1.0, std::min(64.0, p));
}

// The staged and row kernels gather x through a raw buffer descriptor,
// whose byte offsets must stay below 2^31.
bool x_fits_buffer(const spc5_matrix *A) {
    return A->ncols * (A->dtype == SPC5_F64 ? 8 : 4) <= 0x7FFFFFF0LL;
}

int auto_kernel(const spc5_matrix *A) {
    // The staged kernel (value mode for beta(1,c)) whenever its 2 GiB buffer
    // range covers x; the sweep kernel otherwise.
    if (!A->staged_ok || !x_fits_buffer(A)) return SPC5_KERNEL_SWEEP;
    return SPC5_KERNEL_STAGED;
}

int finish_matrix(spc5_matrix *A) {
    A->ppt = default_ppt(A->npanels ? (double)A->nblocks * A->r / (double)A->npanels : 0.0);
    const int st = build_staged_schedule(A, 0);
    if (st != SPC5_OK) return st;
    A->kernel = auto_kernel(A);
    return SPC5_OK;
}

// Lanes per row of the CSR-vector comparison kernel: the power of two
// nearest the mean row length, within 1..64.
static int csr_group(double mean_row) {
    int g = 1;
    while (g < 64 && g * 2 <= mean_row * 1.5) g *= 2;
    return g;
}

// Test hook: SPC5_TEST_FAIL_ALLOC=1 makes every device allocation of the
// creation calls fail, to exercise the SPC5_ENOMEM path.
static bool alloc_fail_hook() {
    const char *e = getenv("SPC5_TEST_FAIL_ALLOC");
    return e && e[0] == '1';
}

// Host-side CSR validation, parallel over row ranges.
int validate_csr(int64_t nrows, int64_t ncols, const int64_t *rowptr,
                        const int32_t *colidx, const void *values, int64_t *nnz_out) {
    if (!rowptr) return fail(SPC5_EINVAL, "rowptr is NULL");
    if (rowptr[0] != 0) return fail(SPC5_EBADCSR, "rowptr[0] = %lld, expected 0",
                                    (long long)rowptr[0]);
    for (int64_t i = 0; i < nrows; ++i)
        if (rowptr[i + 1] < rowptr[i])
            return fail(SPC5_EBADCSR, "rowptr decreases at row %lld", (long long)i);
    const int64_t nnz = rowptr[nrows];
    if (nnz >= ((int64_t)1 << 31))
        return fail(SPC5_EUNSUPPORTED, "nnz = %lld does not fit int32 device indices",
                    (long long)nnz);
    if (nnz > 0 && (!colidx || !values)) return fail(SPC5_EINVAL, "colidx or values is NULL");
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (nnz < (1 << 20)) nth = 1;
    std::vector<int64_t> bad(nth, -1);
    std::vector<int> kind(nth, 0);
    auto work = [&](unsigned t) {
        const int64_t lo = nrows * t / nth, hi = nrows * (t + 1) / nth;
        for (int64_t i = lo; i < hi; ++i) {
            int64_t prev = -1;
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                const int64_t cc = colidx[k];
                if (cc < 0 || cc >= ncols) { bad[t] = i; kind[t] = 1; return; }
                if (cc <= prev) { bad[t] = i; kind[t] = 2; return; }
                prev = cc;
            }
        }
    };
    if (nth == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nth; ++t) th.emplace_back(work, t);
        for (auto &t : th) t.join();
    }
    for (unsigned t = 0; t < nth; ++t)
        if (bad[t] >= 0)
            return fail(SPC5_EBADCSR, kind[t] == 1 ? "column out of range in row %lld"
                                                   : "unsorted or duplicate column in row %lld",
                        (long long)bad[t]);
    *nnz_out = nnz;
    return SPC5_OK;
}

static int check_create_args(int64_t nrows, int64_t ncols, spc5_dtype dtype) {
    if (nrows < 0 || ncols < 0) return fail(SPC5_EINVAL, "negative matrix size");
    if (dtype != SPC5_F64 && dtype != SPC5_F32) return fail(SPC5_EINVAL, "bad dtype %d", (int)dtype);
    if (ncols > INT32_MAX) return fail(SPC5_EUNSUPPORTED, "ncols >= 2^31");
    if (nrows >= ((int64_t)1 << 40)) return fail(SPC5_EUNSUPPORTED, "nrows too large");
    return SPC5_OK;
}

// Device allocation wrapper honouring the test hook.
static hipError_t dmalloc(void **p, size_t bytes) {
    if (alloc_fail_hook()) return hipErrorOutOfMemory;
    return hipMalloc(p, bytes < 256 ? 256 : bytes);
}

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard() {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// One scratch set per stream that has called a product of the handle.  A
// stream's set only grows (a part is allocated when a call first needs it),
// and the handle frees them all.
struct ScratchPool {
    std::mutex mu;
    struct Slot {
        hipStream_t stream;
        Scratch sc;
    };
    std::vector<Slot> slots;
};

void free_pool(spc5_matrix *A) {
    if (!A->pool) return;
    for (auto &sl : A->pool->slots)
        for (void *p : {sl.sc.partial, sl.sc.tr_partial, sl.sc.stage, sl.sc.edges})
            if (p) (void)hipFree(p);
    delete A->pool;
    A->pool = nullptr;
}

// hipMalloc that also works while the calling thread captures a graph (the
// allocation itself is not a stream operation).
static hipError_t scratch_alloc(void **p, size_t bytes) {
    hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
    hipError_t e = hipThreadExchangeStreamCaptureMode(&mode);
    if (e != hipSuccess) return e;
    e = hipMalloc(p, bytes + kPad);
    hipStreamCaptureMode back = mode;
    const hipError_t e2 = hipThreadExchangeStreamCaptureMode(&back);
    return e != hipSuccess ? e : e2;
}

int pool_scratch(const spc5_matrix *A, hipStream_t s, int need, Scratch *out) {
    *out = Scratch();
    const size_t vb = A->dtype == SPC5_F64 ? 8 : 4;
    const spc5_matrix *T = A->tr;
    size_t want[4] = {0, 0, 0, 0};    // partial, tr_partial, stage, edges
    if ((need & kNeedPartial) && A->npieces > 0) want[0] = (size_t)A->npieces * A->r * vb;
    if ((need & kNeedTrPartial) && T && T->npieces > 0)
        want[1] = (size_t)T->npieces * T->r * vb;
    if ((need & kNeedTheta) && A->nnz > 0) {
        want[2] = (size_t)(A->nnz + 16) * vb;    // read 16 at a time by the bucket pass
        want[3] = (size_t)2 * A->tr_nbuckets * vb;
    }
    if (!want[0] && !want[1] && !want[2]) return SPC5_OK;
    if (!A->pool) return fail(SPC5_EINVAL, "handle has no scratch pool");
    std::lock_guard<std::mutex> lock(A->pool->mu);
    ScratchPool::Slot *slot = nullptr;
    for (auto &sl : A->pool->slots)
        if (sl.stream == s) slot = &sl;
    if (!slot) {
        A->pool->slots.push_back({s, Scratch()});
        slot = &A->pool->slots.back();
    }
    void **part[4] = {&slot->sc.partial, &slot->sc.tr_partial, &slot->sc.stage,
                      &slot->sc.edges};
    for (int q = 0; q < 4; ++q) {
        if (!want[q] || *part[q]) continue;
        const hipError_t e = scratch_alloc(part[q], want[q]);
        if (e != hipSuccess) {
            *part[q] = nullptr;
            return hip_fail(e, "allocating per-stream scratch");
        }
    }
    *out = slot->sc;
    return SPC5_OK;
}

void free_matrix(spc5_matrix *A) {
    if (!A) return;
    DeviceGuard g(A->device);
    free_matrix(A->tr);
    free_pool(A);
    for (void *p : {(void *)A->tr_lidx, (void *)A->tr_rslot, (void *)A->tr_rbase,
                    (void *)A->tr_rstart, (void *)A->tr_src, A->tr_arow, (void *)A->tr_cbase,
                    (void *)A->tr_hoff, (void *)A->tr_hbits, (void *)A->tr_hrow,
                    (void *)A->tr_rlo, (void *)A->tr_edge_rows})
        if (p) (void)hipFree(p);
    if (A->blk_ptr) (void)hipFree(A->blk_ptr);
    if (A->blk_col) (void)hipFree(A->blk_col);
    if (A->masks) (void)hipFree(A->masks);
    if (A->val) (void)hipFree(A->val);
    if (A->panel_val) (void)hipFree(A->panel_val);
    free_staged_schedule(A);
    delete A;
}

// Scratch of the allocation-free forward product: a fixed device array (one
// copy per GPU, held until the process ends).  In host code `scratch` names
// a host-side stand-in, never the device memory: kernels get the address
// that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[SPC5_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::once_flag g_scratch_once[kMaxDevices];
static void *g_scratch_ptr[kMaxDevices];
static hipError_t g_scratch_err[kMaxDevices];

// Device address of `scratch` on `dev`, looked up once per device with that
// device current (the caller has made it current).
static int static_scratch(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices)
        return fail(SPC5_EUNSUPPORTED, "device %d: the fixed scratch covers devices 0..%d", dev,
                    kMaxDevices - 1);
    std::call_once(g_scratch_once[dev], [dev]() {
        void *ptr = nullptr;
        g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? ptr : nullptr;
    });
    if (g_scratch_err[dev] != hipSuccess) return hip_fail(g_scratch_err[dev], "hipGetSymbolAddress");
    *out = g_scratch_ptr[dev];
    return SPC5_OK;
}

}  // namespace spc5

using namespace spc5;

extern "C" {

const char *spc5_last_error(void) { return g_err.c_str(); }

const char *spc5_version(void) { return "spc5-mi355x 0.1 (gfx950)"; }

int csr_to_spc5(int64_t nrows, int64_t ncols, const int64_t *rowptr, const int32_t *colidx,
                const void *values, spc5_dtype dtype, int r, int c, spc5_matrix **out) {
    if (!out) return fail(SPC5_EINVAL, "out is NULL");
    *out = nullptr;
    int st;
    if ((st = check_create_args(nrows, ncols, dtype)) != SPC5_OK) return st;
    if (r < 1 || r > 8 || c < 1 || c > 16)
        return fail(SPC5_EUNSUPPORTED, "beta(%d,%d): need 1 <= r <= 8 and 1 <= c <= 16", r, c);
    int64_t nnz = 0;
    if ((st = validate_csr(nrows, ncols, rowptr, colidx, values, &nnz)) != SPC5_OK) return st;
    const int64_t npanels = (nrows + r - 1) / r;
    if (npanels >= ((int64_t)1 << 31) - 1)
        return fail(SPC5_EUNSUPPORTED, "too many panels for int32 indices");

    spc5_matrix *A = new (std::nothrow) spc5_matrix();
    if (!A) return fail(SPC5_ENOMEM, "host allocation failed");
    A->nrows = nrows; A->ncols = ncols; A->nnz = nnz; A->npanels = npanels;
    A->r = r; A->c = c; A->dtype = dtype; A->mask_bytes = c <= 8 ? 1 : 2;
    A->pool = new (std::nothrow) ScratchPool();
    if (!A->pool) { delete A; return fail(SPC5_ENOMEM, "host allocation failed"); }
    hipError_t e = hipGetDevice(&A->device);
    if (e != hipSuccess) { free_matrix(A); return hip_fail(e, "hipGetDevice"); }
    const int vb = dtype == SPC5_F64 ? 8 : 4;
    int64_t *d_rowptr = nullptr;
    int32_t *d_colidx = nullptr;
    void *d_val = nullptr;
    auto drop = [&]() {
        if (d_rowptr) (void)hipFree(d_rowptr);
        if (d_colidx) (void)hipFree(d_colidx);
        if (d_val) (void)hipFree(d_val);
    };
    if ((e = dmalloc((void **)&d_rowptr, (size_t)(nrows + 1) * 8)) != hipSuccess ||
        (e = dmalloc((void **)&d_colidx, (size_t)nnz * 4)) != hipSuccess ||
        (e = dmalloc(&d_val, (size_t)nnz * vb)) != hipSuccess) {
        drop();
        free_matrix(A);
        return hip_fail(e, "allocating device CSR");
    }
    if ((e = hipMemcpy(d_rowptr, rowptr, (size_t)(nrows + 1) * 8, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (nnz > 0 &&
         ((e = hipMemcpy(d_colidx, colidx, (size_t)nnz * 4, hipMemcpyHostToDevice)) !=
              hipSuccess ||
          (e = hipMemcpy(d_val, values, (size_t)nnz * vb, hipMemcpyHostToDevice)) !=
              hipSuccess))) {
        drop();
        free_matrix(A);
        return hip_fail(e, "uploading CSR");
    }
    st = convert_on_device(A, d_rowptr, d_colidx, d_val);
    drop();
    if (st != SPC5_OK) { free_matrix(A); return st; }
    if ((st = finish_matrix(A)) != SPC5_OK) { free_matrix(A); return st; }
    *out = A;
    return SPC5_OK;
}

void spc5_free(spc5_matrix *A) { free_matrix(A); }

int spc5_get_info(const spc5_matrix *A, spc5_info *out) {
    if (!A || !out) return fail(SPC5_EINVAL, "NULL argument");
    memset(out, 0, sizeof *out);
    out->nrows = A->nrows; out->ncols = A->ncols; out->nnz = A->nnz;
    out->nblocks = A->nblocks; out->npanels = A->npanels;
    out->r = A->r; out->c = A->c; out->dtype = A->dtype; out->mask_bytes = A->mask_bytes;
    out->panels_per_tile = A->kernel == SPC5_KERNEL_STAGED ? A->sppt : A->ppt;
    out->kernel = A->kernel;
    out->max_panel_blocks = A->max_panel_blocks;
    out->ntiles = A->kernel == SPC5_KERNEL_ROWS ? (A->npanels + 64 / A->r - 1) / (64 / A->r)
                  : A->kernel == SPC5_KERNEL_STAGED ? A->ntiles_staged
                                                    : (A->npanels + A->ppt - 1) / A->ppt;
    out->fill = A->nblocks ? (double)A->nnz / ((double)A->nblocks * A->r * A->c) : 0.0;
    const int64_t vb = A->dtype == SPC5_F64 ? 8 : 4;
    out->spmv_bytes = vb * A->nnz + 4 * A->nblocks + (int64_t)A->r * A->mask_bytes * A->nblocks +
                      4 * (A->npanels + 1) + vb * A->ncols + vb * A->nrows;
    out->device_bytes = vb * A->nnz + 4 * A->nblocks + (int64_t)A->r * A->mask_bytes * A->nblocks +
                        8 * (A->npanels + 1);
    out->split_panels = A->kernel == SPC5_KERNEL_STAGED ? A->nsplit : 0;
    out->variant = A->variant;
    if (const spc5_matrix *T = A->tr) {
        out->transpose_r = T->r;
        out->transpose_c = T->c;
        out->transpose_kernel = T->kernel;
        out->transpose_bytes = vb * T->nnz + 4 * T->nblocks +
                               (int64_t)T->r * T->mask_bytes * T->nblocks + 4 * (T->npanels + 1) +
                               vb * T->ncols + vb * T->nrows;
    }
    return SPC5_OK;
}

int spc5_export(const spc5_matrix *A, int64_t *blk_ptr, int32_t *blk_col, void *masks,
                void *values) {
    if (!A) return fail(SPC5_EINVAL, "A is NULL");
    DeviceGuard g(A->device);
    if (!g.ok) return fail(SPC5_EDEVICE, "cannot select the matrix's device");
    hipError_t e;
    if (blk_ptr) {
        std::vector<int32_t> tmp((size_t)A->npanels + 1);
        if ((e = hipMemcpy(tmp.data(), A->blk_ptr, tmp.size() * 4, hipMemcpyDeviceToHost)) !=
            hipSuccess)
            return hip_fail(e, "exporting blk_ptr");
        for (size_t i = 0; i < tmp.size(); ++i) blk_ptr[i] = tmp[i];
    }
    if (blk_col && A->nblocks &&
        (e = hipMemcpy(blk_col, A->blk_col, (size_t)A->nblocks * 4, hipMemcpyDeviceToHost)) !=
            hipSuccess)
        return hip_fail(e, "exporting blk_col");
    if (masks && A->nblocks &&
        (e = hipMemcpy(masks, A->masks, (size_t)A->nblocks * A->r * A->mask_bytes,
                       hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "exporting masks");
    if (values && A->nnz &&
        (e = hipMemcpy(values, A->val, (size_t)A->nnz * (A->dtype == SPC5_F64 ? 8 : 4),
                       hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "exporting values");
    return SPC5_OK;
}

int spc5_to_csr(const spc5_matrix *A, int64_t *rowptr, int32_t *colidx, void *values) {
    if (!A) return fail(SPC5_EINVAL, "A is NULL");
    if (!rowptr) return fail(SPC5_EINVAL, "rowptr is NULL");
    const int r = A->r, vb = A->dtype == SPC5_F64 ? 8 : 4;
    std::vector<int64_t> bp;
    std::vector<int32_t> bc;
    std::vector<uint16_t> mk;
    std::vector<unsigned char> va;
    try {
        bp.resize((size_t)A->npanels + 1);
        bc.resize((size_t)A->nblocks);
        mk.resize((size_t)A->nblocks * r);
        va.resize((size_t)A->nnz * vb);
    } catch (...) {
        return fail(SPC5_ENOMEM, "host allocation failed");
    }
    std::vector<uint8_t> mk8;
    if (A->mask_bytes == 1) {
        try {
            mk8.resize(mk.size());
        } catch (...) {
            return fail(SPC5_ENOMEM, "host allocation failed");
        }
    }
    int st = spc5_export(A, bp.data(), bc.data(),
                         A->mask_bytes == 1 ? (void *)mk8.data() : (void *)mk.data(), va.data());
    if (st != SPC5_OK) return st;
    if (A->mask_bytes == 1)
        for (size_t i = 0; i < mk.size(); ++i) mk[i] = mk8[i];
    // per-row counts, then the entries row by row
    std::fill(rowptr, rowptr + A->nrows + 1, (int64_t)0);
    for (int64_t p = 0; p < A->npanels; ++p)
        for (int64_t b = bp[p]; b < bp[p + 1]; ++b)
            for (int i = 0; i < r; ++i)
                if (p * r + i < A->nrows) rowptr[p * r + i + 1] += __builtin_popcount(mk[b * r + i]);
    for (int64_t i = 0; i < A->nrows; ++i) rowptr[i + 1] += rowptr[i];
    int64_t v = 0;    // next packed value
    for (int64_t p = 0; p < A->npanels; ++p) {
        int64_t at[8];
        for (int i = 0; i < r; ++i) at[i] = p * r + i < A->nrows ? rowptr[p * r + i] : 0;
        for (int64_t b = bp[p]; b < bp[p + 1]; ++b)
            for (int i = 0; i < r; ++i)
                for (unsigned m = mk[b * r + i]; m; m &= m - 1u) {
                    const int k = __builtin_ctz(m);
                    if (colidx) colidx[at[i]] = bc[b] + k;
                    if (values) memcpy((unsigned char *)values + at[i] * vb, va.data() + v * vb, vb);
                    ++at[i];
                    ++v;
                }
    }
    return SPC5_OK;
}

int spc5_set_schedule(spc5_matrix *A, int kernel, int ppt) {
    if (!A) return fail(SPC5_EINVAL, "A is NULL");
    if (kernel < SPC5_KERNEL_AUTO || kernel > SPC5_KERNEL_STAGED)
        return fail(SPC5_EINVAL, "unknown kernel %d", kernel);
    if (ppt < 0 || ppt > 64) return fail(SPC5_EINVAL, "panels_per_tile must be in 0..64");
    if (kernel == SPC5_KERNEL_STAGED && !A->staged_ok)
        return fail(SPC5_EUNSUPPORTED, "a panel is longer than the staged kernel's window");
    if ((kernel == SPC5_KERNEL_STAGED || kernel == SPC5_KERNEL_ROWS) && !x_fits_buffer(A))
        return fail(SPC5_EUNSUPPORTED, "x exceeds 2 GiB: only the sweep kernel applies");
    A->kernel = kernel == SPC5_KERNEL_AUTO ? auto_kernel(A) : kernel;
    if (A->kernel != SPC5_KERNEL_STAGED) A->variant = 0;
    if (A->kernel == SPC5_KERNEL_STAGED) {
        DeviceGuard g(A->device);
        int st = build_staged_schedule(A, ppt);
        if (st == SPC5_OK && A->variant != 0) st = fit_schedule_to_variants(A, true);
        return st;
    }
    A->ppt = ppt ? ppt
                 : default_ppt(A->npanels ? (double)A->nblocks * A->r / (double)A->npanels : 0.0);
    return SPC5_OK;
}

// A vector pointer may be NULL only when its length is zero.
static int compute_guard(const spc5_matrix *A,
                         std::initializer_list<std::pair<const void *, int64_t>> vecs) {
    if (!A) return fail(SPC5_EINVAL, "A is NULL");
    for (const auto &v : vecs)
        if (!v.first && v.second > 0) return fail(SPC5_EINVAL, "NULL vector");
    return SPC5_OK;
}

// Partial-sum scratch of a forward product of A on stream s (none when A
// has no piece tiles or another kernel than the staged one runs).
static int forward_scratch(const spc5_matrix *A, hipStream_t s, Scratch *sc) {
    *sc = Scratch();
    if (A->kernel != SPC5_KERNEL_STAGED || A->npieces == 0) return SPC5_OK;
    return pool_scratch(A, s, kNeedPartial, sc);
}

int spc5_spmv(const spc5_matrix *A, const void *x, void *y, void *stream) {
    int st = compute_guard(A, {{x, A ? A->ncols : 0}, {y, A ? A->nrows : 0}});
    if (st) return st;
    DeviceGuard g(A->device);
    Scratch sc;
    if ((st = forward_scratch(A, (hipStream_t)stream, &sc)) != SPC5_OK) return st;
    hipError_t e = launch_spmv(A, nullptr, x, y, (hipStream_t)stream, sc.partial);
    return e == hipSuccess ? SPC5_OK : hip_fail(e, "spc5_spmv launch");
}

int spc5_spmv_values(const spc5_matrix *A, const void *values, const void *x, void *y,
                     void *stream) {
    int st = compute_guard(A, {{x, A ? A->ncols : 0}, {y, A ? A->nrows : 0}});
    if (st) return st;
    if (!values && A->nnz) return fail(SPC5_EINVAL, "values is NULL");
    DeviceGuard g(A->device);
    Scratch sc;
    if ((st = forward_scratch(A, (hipStream_t)stream, &sc)) != SPC5_OK) return st;
    hipError_t e = launch_spmv(A, values ? values : A->val, x, y, (hipStream_t)stream,
                               sc.partial);
    return e == hipSuccess ? SPC5_OK : hip_fail(e, "spc5_spmv_values launch");
}

int spc5_spmv_noalloc(const spc5_matrix *A, const void *x, void *y, void *stream) {
    int st = compute_guard(A, {{x, A ? A->ncols : 0}, {y, A ? A->nrows : 0}});
    if (st) return st;
    DeviceGuard g(A->device);
    if (!g.ok) return fail(SPC5_EDEVICE, "cannot select the matrix's device");
    void *partial = nullptr;
    if (A->kernel == SPC5_KERNEL_STAGED && A->npieces > 0) {
        const int64_t need = A->npieces * A->r * (A->dtype == SPC5_F64 ? 8 : 4);
        if (need > SPC5_NOALLOC_SCRATCH_BYTES)
            return fail(SPC5_EUNSUPPORTED,
                        "the piece tiles' partial sums need %lld bytes, above the fixed "
                        "scratch of %d bytes",
                        (long long)need, SPC5_NOALLOC_SCRATCH_BYTES);
        if ((st = static_scratch(A->device, &partial)) != SPC5_OK) return st;
    }
    hipError_t e = launch_spmv(A, nullptr, x, y, (hipStream_t)stream, partial);
    return e == hipSuccess ? SPC5_OK : hip_fail(e, "spc5_spmv_noalloc launch");
}

int spc5_spmv_transpose(const spc5_matrix *A, const void *ybar, void *xbar, void *stream) {
    return spc5_spmv_transpose_values(A, nullptr, ybar, xbar, stream);
}

int spc5_spmv_transpose_values(const spc5_matrix *A, const void *values, const void *ybar,
                               void *xbar, void *stream) {
    int st = compute_guard(A, {{ybar, A ? A->nrows : 0}, {xbar, A ? A->ncols : 0}});
    if (st) return st;
    DeviceGuard g(A->device);
    Scratch sc;
    if (A->tr && (st = pool_scratch(A, (hipStream_t)stream, values ? kNeedTheta : kNeedTrPartial,
                                    &sc)) != SPC5_OK)
        return st;
    hipError_t e = A->tr ? launch_transpose_plan(A, values, ybar, xbar, (hipStream_t)stream, sc)
                         : launch_transpose(A, values ? values : A->val, ybar, xbar,
                                            (hipStream_t)stream);
    return e == hipSuccess ? SPC5_OK : hip_fail(e, "spc5_spmv_transpose launch");
}

int spc5_set_variant(spc5_matrix *A, int flags) {
    if (!A) return fail(SPC5_EINVAL, "A is NULL");
    const bool known = flags >= 0 && flags <= (SPC5_VARIANT_PARTIAL_X | SPC5_VARIANT_ROW_REDUCE);
    if (!known && flags != SPC5_VARIANT_UNION_X)
        return fail(SPC5_EINVAL, "unknown variant flags %d (union-x load combines with none)",
                    flags);
    if (flags != 0) {
        if (A->kernel != SPC5_KERNEL_STAGED)
            return fail(SPC5_EUNSUPPORTED, "variants apply to the staged kernel only");
        if (!(A->r == 2 || A->r == 4 || A->r == 8) || A->c > 8)
            return fail(SPC5_EUNSUPPORTED, "variants exist for r in {2,4,8}, c <= 8");
    }
    if (A->kernel == SPC5_KERNEL_STAGED && (flags != 0) != (A->variant != 0)) {
        DeviceGuard g(A->device);
        const int st = fit_schedule_to_variants(A, flags != 0);
        if (st != SPC5_OK) return st;
    }
    A->variant = flags;
    return SPC5_OK;
}

int spc5_prepare_transpose(spc5_matrix *A, int r, int c) {
    if (!A) return fail(SPC5_EINVAL, "A is NULL");
    if (r == 0) r = A->r;
    if (c == 0) c = A->c;
    if (r < 1 || r > 8 || c < 1 || c > 16)
        return fail(SPC5_EUNSUPPORTED, "beta(%d,%d) is out of range", r, c);
    if (A->tr) {
        if (A->tr->r == r && A->tr->c == c) return SPC5_OK;
        return fail(SPC5_EINVAL, "a transpose plan with another shape exists");
    }
    DeviceGuard g(A->device);
    if (!g.ok) return fail(SPC5_EDEVICE, "cannot select the matrix's device");
    return build_transpose_plan(A, r, c);
}

int spc5_values_grad(const spc5_matrix *A, const void *ybar, const void *x, void *vbar,
                     void *stream) {
    int st = compute_guard(A, {{ybar, A ? A->nrows : 0}, {x, A ? A->ncols : 0}});
    if (st) return st;
    if (!vbar && A->nnz) return fail(SPC5_EINVAL, "vbar is NULL");
    DeviceGuard g(A->device);
    hipError_t e = launch_values_grad(A, ybar, x, vbar, (hipStream_t)stream);
    return e == hipSuccess ? SPC5_OK : hip_fail(e, "spc5_values_grad launch");
}

int spc5_spmm(const spc5_matrix *A, int nrhs, const void *X, void *Y, void *stream) {
    int st = compute_guard(A, {{X, A ? A->ncols : 0}, {Y, A ? A->nrows : 0}});
    if (st) return st;
    if (nrhs < 1 || nrhs > 64) return fail(SPC5_EINVAL, "nrhs must be in 1..64");
    DeviceGuard g(A->device);
    hipError_t e = launch_spmm(A, nrhs, X, Y, (hipStream_t)stream);
    return e == hipSuccess ? SPC5_OK : hip_fail(e, "spc5_spmm launch");
}

// ---------------------------------------------------------------- CSR

int spc5_csr_create(int64_t nrows, int64_t ncols, const int64_t *rowptr,
                    const int32_t *colidx, const void *values, spc5_dtype dtype,
                    spc5_csr **out) {
    if (!out) return fail(SPC5_EINVAL, "out is NULL");
    *out = nullptr;
    int st;
    if ((st = check_create_args(nrows, ncols, dtype)) != SPC5_OK) return st;
    int64_t nnz = 0;
    if ((st = validate_csr(nrows, ncols, rowptr, colidx, values, &nnz)) != SPC5_OK) return st;
    if (nrows >= ((int64_t)1 << 31) - 1) return fail(SPC5_EUNSUPPORTED, "nrows >= 2^31-1");
    spc5_csr *A = new (std::nothrow) spc5_csr();
    if (!A) return fail(SPC5_ENOMEM, "host allocation failed");
    A->nrows = nrows; A->ncols = ncols; A->nnz = nnz; A->dtype = dtype;
    hipError_t e = hipGetDevice(&A->device);
    if (e != hipSuccess) { delete A; return hip_fail(e, "hipGetDevice"); }
    const int vb = dtype == SPC5_F64 ? 8 : 4;
    std::vector<int32_t> rp32((size_t)nrows + 1);
    for (int64_t i = 0; i <= nrows; ++i) rp32[i] = (int32_t)rowptr[i];
    auto drop = [&]() {
        if (A->rowptr) (void)hipFree(A->rowptr);
        if (A->colidx) (void)hipFree(A->colidx);
        if (A->val) (void)hipFree(A->val);
        delete A;
    };
    if ((e = dmalloc((void **)&A->rowptr, rp32.size() * 4)) != hipSuccess ||
        (e = dmalloc((void **)&A->colidx, (size_t)nnz * 4)) != hipSuccess ||
        (e = dmalloc(&A->val, (size_t)nnz * vb)) != hipSuccess) {
        drop();
        return hip_fail(e, "allocating device CSR");
    }
    if ((e = hipMemcpy(A->rowptr, rp32.data(), rp32.size() * 4, hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (nnz > 0 &&
         ((e = hipMemcpy(A->colidx, colidx, (size_t)nnz * 4, hipMemcpyHostToDevice)) !=
              hipSuccess ||
          (e = hipMemcpy(A->val, values, (size_t)nnz * vb, hipMemcpyHostToDevice)) !=
              hipSuccess))) {
        drop();
        return hip_fail(e, "uploading CSR");
    }
    A->rpt = default_ppt(nrows ? (double)nnz / (double)nrows : 0.0);
    A->group = csr_group(nrows ? (double)nnz / (double)nrows : 1.0);
    *out = A;
    return SPC5_OK;
}

void spc5_csr_free(spc5_csr *A) {
    if (!A) return;
    DeviceGuard g(A->device);
    if (A->rowptr) (void)hipFree(A->rowptr);
    if (A->colidx) (void)hipFree(A->colidx);
    if (A->val) (void)hipFree(A->val);
    delete A;
}

int spc5_csr_spmv(const spc5_csr *A, const void *x, void *y, void *stream) {
    if (!A) return fail(SPC5_EINVAL, "A is NULL");
    if ((!x && A->ncols > 0) || (!y && A->nrows > 0)) return fail(SPC5_EINVAL, "NULL vector");
    DeviceGuard g(A->device);
    hipError_t e = launch_csr_spmv(A, x, y, (hipStream_t)stream);
    return e == hipSuccess ? SPC5_OK : hip_fail(e, "spc5_csr_spmv launch");
}

int64_t spc5_csr_bytes(const spc5_csr *A) {
    if (!A) return -1;
    const int64_t vb = A->dtype == SPC5_F64 ? 8 : 4;
    return vb * A->nnz + 4 * A->nnz + 4 * (A->nrows + 1) + vb * A->ncols + vb * A->nrows;
}

}  // extern "C"
