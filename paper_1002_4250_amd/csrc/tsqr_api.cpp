// tsqr_api.cpp -- the C ABI of libtsqr.so (declared and documented in
// include/tsqr.h): handle, argument checks, launch geometry, workspace layout
// and dispatch to the compiled kernel instantiations.
#include "tsqr.h"

#include <hip/hip_runtime.h>

#include <new>
#include <string.h>

#include "tsqr_internal.h"

struct tsqr_handle_s {
    int device;
    int cu_count;
    int64_t leaf_rows;     // 0 = automatic
    int64_t rpl;           // rows per lane of the leaf kernel; 0 = default
    int64_t waves_per_cu;  // leaves per compute unit targeted by the automatic policy
    int last_hip_error;
    bool planning_only;    // no device: checks and planning only
};

namespace {

constexpr int kRowsPerLaneUnit = 16;   // a chunk is 16 * rows-per-lane rows (16 lanes share a column)
constexpr int64_t kAlign = 256;

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

int padded_columns(int64_t n)
{
    for (int nc : {TSQR_NC_VALUES})
        if (n <= nc) return nc;
    return -1;
}

bool leaf_instance_exists(int dtype, int nc, int rpl)
{
#define TSQR_HAS(tag, NC, RPL) \
    if ((dtype == TSQR_F64) == (sizeof(tsqr::tag) == 8) && nc == NC && rpl == RPL) return true;
    TSQR_LEAF_INSTANCES(TSQR_HAS)
#undef TSQR_HAS
    return false;
}

int elem_bytes(int dtype) { return dtype == TSQR_F64 ? 8 : 4; }

struct Geometry {
    int nc = 0;
    int rpl = 0;
    int64_t leaf_rows = 0;
    int64_t leaves = 0;
    int64_t ticket_bytes = 0;
    int64_t tri_elems = 0;     // per leaf
    int64_t ws_bytes = 0;
};

// Leaf policy: a chunk is 16*RPL rows; the automatic leaf size gives about
// waves_per_cu leaves per compute unit (each leaf is one wavefront), never
// less than one chunk.  The tree then has ceil(log2 P) levels.
int plan(const tsqr_handle_s* h, int64_t m, int64_t n, int dtype, Geometry* g)
{
    g->nc = padded_columns(n);
    if (g->nc < 0) return TSQR_ERR_UNSUPPORTED;
    g->rpl = (int)(h->rpl > 0 ? h->rpl : (dtype == TSQR_F64 ? TSQR_DEFAULT_RPL_F64 : TSQR_DEFAULT_RPL_F32));
    if (!leaf_instance_exists(dtype, g->nc, g->rpl)) {
        // fall back to the default rows-per-lane, else any compiled one, for this column count
        g->rpl = dtype == TSQR_F64 ? TSQR_DEFAULT_RPL_F64 : TSQR_DEFAULT_RPL_F32;
        if (!leaf_instance_exists(dtype, g->nc, g->rpl)) {
            g->rpl = 0;
#define TSQR_ANY(tag, NC, RPL) \
    if (g->rpl == 0 && (dtype == TSQR_F64) == (sizeof(tsqr::tag) == 8) && g->nc == NC) g->rpl = RPL;
            TSQR_LEAF_INSTANCES(TSQR_ANY)
#undef TSQR_ANY
            if (g->rpl == 0) return TSQR_ERR_UNSUPPORTED;
        }
    }
    const int64_t chunk = (int64_t)kRowsPerLaneUnit * g->rpl;
    int64_t L;
    if (h->leaf_rows > 0) {
        L = align_up(h->leaf_rows, chunk);
    } else {
        const int64_t target = (int64_t)h->cu_count * (h->waves_per_cu > 0 ? h->waves_per_cu : 4);
        L = (m + target - 1) / (target > 0 ? target : 1);
        L = align_up(L > chunk ? L : chunk, chunk);
    }
    g->leaf_rows = L;
    g->leaves = m > 0 ? (m + L - 1) / L : 1;
    if (g->leaves > (int64_t)1 << 30) return TSQR_ERR_UNSUPPORTED;
    g->ticket_bytes = align_up(g->leaves * 4, kAlign);
    g->tri_elems = (int64_t)g->nc * (g->nc + 1) / 2;
    g->ws_bytes = g->ticket_bytes + align_up(g->leaves * g->tri_elems * elem_bytes(dtype), kAlign);
    return 0;
}

int hip_status(tsqr_handle_s* h, hipError_t e)
{
    if (e == hipSuccess) return 0;
    h->last_hip_error = (int)e;
    return TSQR_ERR_HIP;
}

template <typename T>
hipError_t dispatch_leaf(const tsqr::LeafTreeArgs<T>& a, int nc, int rpl, hipStream_t s)
{
#define TSQR_CALL(tag, NC, RPL)                                                         \
    if constexpr (sizeof(T) == sizeof(tsqr::tag)) {                                     \
        if (nc == NC && rpl == RPL)                                                     \
            return tsqr::launch_leaf_tree_##tag##_##NC##_##RPL(                         \
                reinterpret_cast<const tsqr::LeafTreeArgs<tsqr::tag>&>(a), s);          \
    }
    TSQR_LEAF_INSTANCES(TSQR_CALL)
#undef TSQR_CALL
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch_op(int n, int nc, T* R1, T* R2, T* tau, hipStream_t s)
{
#define TSQR_CALL(tag, NC)                                                                         \
    if constexpr (sizeof(T) == sizeof(tsqr::tag)) {                                                \
        if (nc == NC)                                                                              \
            return tsqr::launch_qr_uppers_##tag##_##NC(n, reinterpret_cast<tsqr::tag*>(R1),        \
                                                      reinterpret_cast<tsqr::tag*>(R2),            \
                                                      reinterpret_cast<tsqr::tag*>(tau), s);       \
    }
    TSQR_OP_INSTANCES(TSQR_CALL)
#undef TSQR_CALL
    return hipErrorInvalidValue;
}

template <typename T>
int geqr_r(tsqr_handle_t h, int64_t m, int64_t n, const T* A, int64_t lda, T* R, int64_t ldr, void* ws,
           int64_t ws_bytes, void* stream, int dtype)
{
    if (!h) return -1;
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (m > 0 && n > 0 && !A) return -4;
    if (lda < (m > 1 ? m : 1)) return -5;
    if (n > 0 && !R) return -6;
    if (ldr < (n > 1 ? n : 1)) return -7;
    if (n == 0) return 0;
    Geometry g;
    int rc = plan(h, m, n, dtype, &g);
    if (rc) return rc;
    if (!ws) return -8;
    if (ws_bytes < g.ws_bytes) return -9;
    if ((reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) != 0) return -8;
    if (h->planning_only) return TSQR_ERR_NO_DEVICE;

    tsqr::LeafTreeArgs<T> a;
    a.A = A;
    a.m = m;
    a.lda = lda;
    a.n = (int)n;
    a.leaf_rows = g.leaf_rows;
    a.leaves = (int)g.leaves;
    a.tickets = static_cast<unsigned*>(ws);
    a.tri = reinterpret_cast<T*>(static_cast<char*>(ws) + g.ticket_bytes);
    a.R = R;
    a.ldr = ldr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the tree counters are zeroed by a kernel on every call: their position
    // depends on the leaf count, so a previous call with another leaf count may
    // have left triangle data there
    hipError_t e = tsqr::launch_zero_u32(a.tickets, a.leaves, s);
    if (e == hipSuccess) e = dispatch_leaf<T>(a, g.nc, g.rpl, s);
    return hip_status(h, e);
}

template <typename T>
int qr_uppers(tsqr_handle_t h, int64_t n, T* R1, T* R2, T* tau, void* stream)
{
    if (!h) return -1;
    if (n < 0) return -2;
    if (n > 0 && !R1) return -3;
    if (n > 0 && !R2) return -4;
    if (n > 0 && !tau) return -5;
    if (n == 0) return 0;
    const int nc = padded_columns(n);
    if (nc < 0) return TSQR_ERR_UNSUPPORTED;
    if (h->planning_only) return TSQR_ERR_NO_DEVICE;
    return hip_status(h, dispatch_op<T>((int)n, nc, R1, R2, tau, static_cast<hipStream_t>(stream)));
}

}  // namespace

extern "C" {

int tsqr_create(tsqr_handle_t* handle, int device)
{
    if (!handle) return -1;
    *handle = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return TSQR_ERR_NO_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return TSQR_ERR_NO_DEVICE;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TSQR_ERR_NO_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return TSQR_ERR_NO_DEVICE;
    tsqr_handle_s* h = new (std::nothrow) tsqr_handle_s;
    if (!h) return TSQR_ERR_ALLOC;
    h->device = device;
    h->cu_count = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    h->leaf_rows = 0;
    h->rpl = 0;
    h->waves_per_cu = 4;
    h->last_hip_error = 0;
    h->planning_only = false;
    *handle = h;
    return 0;
}

int tsqr_create_planning(tsqr_handle_t* handle, int cu_count)
{
    if (!handle) return -1;
    *handle = nullptr;
    if (cu_count < 1) return -2;
    tsqr_handle_s* h = new (std::nothrow) tsqr_handle_s;
    if (!h) return TSQR_ERR_ALLOC;
    h->device = -1;
    h->cu_count = cu_count;
    h->leaf_rows = 0;
    h->rpl = 0;
    h->waves_per_cu = 4;
    h->last_hip_error = 0;
    h->planning_only = true;
    *handle = h;
    return 0;
}

int tsqr_destroy(tsqr_handle_t handle)
{
    delete handle;
    return 0;
}

int tsqr_last_hip_error(tsqr_handle_t handle) { return handle ? handle->last_hip_error : 0; }

const char* tsqr_status_string(int status)
{
    if (status == 0) return "success";
    if (status < 0) return "invalid argument";
    switch (status) {
    case TSQR_ERR_HIP: return "HIP runtime error";
    case TSQR_ERR_UNSUPPORTED: return "unsupported size (n > TSQR_MAX_N or index range)";
    case TSQR_ERR_NO_DEVICE: return "no usable gfx950 device";
    case TSQR_ERR_ALLOC: return "allocation failed";
    default: return "unknown status";
    }
}

int tsqr_set_option(tsqr_handle_t handle, int option, int64_t value)
{
    if (!handle) return -1;
    if (value < 0) return -3;
    switch (option) {
    case TSQR_OPT_LEAF_ROWS: handle->leaf_rows = value; return 0;
    case TSQR_OPT_ROWS_PER_LANE: handle->rpl = value; return 0;
    case TSQR_OPT_WAVES_PER_CU: handle->waves_per_cu = value; return 0;
    default: return -2;
    }
}

int tsqr_plan_info(tsqr_handle_t handle, int64_t m, int64_t n, int dtype, int64_t* leaf_rows, int64_t* leaves)
{
    if (!handle) return -1;
    if (m < 0) return -2;
    if (n < 1) return -3;
    if (dtype != TSQR_F64 && dtype != TSQR_F32) return -4;
    Geometry g;
    int rc = plan(handle, m, n, dtype, &g);
    if (rc) return rc;
    if (leaf_rows) *leaf_rows = g.leaf_rows;
    if (leaves) *leaves = g.leaves;
    return 0;
}

int64_t tsqr_workspace_bytes(tsqr_handle_t handle, int64_t m, int64_t n, int dtype)
{
    if (!handle) return -1;
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (dtype != TSQR_F64 && dtype != TSQR_F32) return -4;
    if (n == 0) return 0;
    Geometry g;
    int rc = plan(handle, m, n, dtype, &g);
    if (rc) return -(int64_t)1000 - rc;
    return g.ws_bytes;
}

int tsqr_geqr_r_f64(tsqr_handle_t handle, int64_t m, int64_t n, const double* A, int64_t lda, double* R,
                    int64_t ldr, void* ws, int64_t ws_bytes, void* stream)
{
    return geqr_r<double>(handle, m, n, A, lda, R, ldr, ws, ws_bytes, stream, TSQR_F64);
}

int tsqr_geqr_r_f32(tsqr_handle_t handle, int64_t m, int64_t n, const float* A, int64_t lda, float* R,
                    int64_t ldr, void* ws, int64_t ws_bytes, void* stream)
{
    return geqr_r<float>(handle, m, n, A, lda, R, ldr, ws, ws_bytes, stream, TSQR_F32);
}

int tsqr_qr_uppers_f64(tsqr_handle_t handle, int64_t n, double* R1, double* R2, double* tau, void* stream)
{
    return qr_uppers<double>(handle, n, R1, R2, tau, stream);
}

int tsqr_qr_uppers_f32(tsqr_handle_t handle, int64_t n, float* R1, float* R2, float* tau, void* stream)
{
    return qr_uppers<float>(handle, n, R1, R2, tau, stream);
}

}  // extern "C"
