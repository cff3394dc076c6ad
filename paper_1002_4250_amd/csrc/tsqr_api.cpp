// tsqr_api.cpp -- the C ABI of libtsqr.so (declared and documented in
// include/tsqr.h): handle, argument checks, launch geometry, workspace layout
// and dispatch to the compiled kernel instantiations.
#include "tsqr.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <string.h>
#include <vector>

#include "tsqr_internal.h"

// One row of the tuning table: the launch configuration the automatic policy
// uses for one element type, one compiled column width and a range of m.
struct TuneEntry {
    int dtype;
    int nc;                // compiled column width the entry applies to
    int64_t m_max;         // applies to m <= m_max (the smallest such entry wins); batched entries ignore it
    int rpl;               // rows per lane
    int64_t waves_per_cu;  // leaves per compute unit (0 = as many as are resident)
    int64_t leaf_rows;     // explicit leaf size (0 = from waves_per_cu)
    bool batch;            // an entry for batched plans
};

struct tsqr_handle_s {
    int device;
    void* scratch;         // this device's address of the fixed scratch array (tsqr_geqr_r_f64_noalloc)
    int cu_count;
    int64_t leaf_rows;     // 0 = automatic
    int64_t rpl;           // rows per lane of the leaf kernel; 0 = default
    int64_t waves_per_cu;  // leaves per compute unit targeted by the automatic policy
    int last_hip_error;
    bool planning_only;    // no device: checks and planning only
    std::vector<TuneEntry> tuning;
};

// Fixed scratch for tsqr_geqr_r_f64_noalloc: the tree counters and leaf
// triangles that tsqr_geqr_r_f64 takes from the caller's workspace.  Every
// device the library runs on holds its own copy until the process ends.  In
// host code `scratch` is only a stand-in for the symbol: its device address
// comes from hipGetSymbolAddress, once per device (device_scratch).
static __device__ __align__(256) unsigned char scratch[TSQR_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of `scratch` on `device` (which must be current), looked up
// once per device; nullptr if the lookup fails.
void* device_scratch(int device)
{
    static std::mutex mu;
    static std::vector<void*> addr;
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0) return nullptr;
    if ((int)addr.size() <= device) addr.resize(device + 1, nullptr);
    if (!addr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) addr[device] = p;
    }
    return addr[device];
}

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

// Workgroups of the leaf kernel that fit on one compute unit at once (one
// wavefront each): 4 for a kernel that needs more than half of a SIMD's
// registers, 8 when two wavefronts fit per SIMD.  4 on a planning handle.
int leaf_occupancy(const tsqr_handle_s* h, int dtype, int nc, int rpl)
{
    if (h->planning_only) return 4;
    int occ = 0;
#define TSQR_OCC(tag, NC, RPL) \
    if ((dtype == TSQR_F64) == (sizeof(tsqr::tag) == 8) && nc == NC && rpl == RPL) occ = tsqr::occupancy_leaf_##tag##_##NC##_##RPL();
    TSQR_LEAF_INSTANCES(TSQR_OCC)
#undef TSQR_OCC
    return occ > 0 ? occ : 4;
}

// The tuning-table entry for a call: the smallest m_max >= m among the
// single-matrix entries, or the batched entry; NULL if none applies.
const TuneEntry* find_tuning(const tsqr_handle_s* h, int dtype, int nc, int64_t m, bool batch)
{
    const TuneEntry* best = nullptr;
    for (const TuneEntry& e : h->tuning) {
        if (e.dtype != dtype || e.nc != nc || e.batch != batch) continue;
        if (batch) return &e;
        if (m <= e.m_max && (!best || e.m_max < best->m_max)) best = &e;
    }
    return best;
}

// Leaf policy: a chunk is 16*RPL rows; the automatic leaf size gives
// waves_per_cu leaves per compute unit (each leaf is one wavefront; by default
// as many as are resident at once), never less than one chunk.  The tree then
// has ceil(log2 P) levels.  Options set on the handle take precedence over
// the tuning table, which takes precedence over the built-in defaults.
// `force_rpl` (if positive) fixes the rows per lane, as the Q-factor mode does.
int plan(const tsqr_handle_s* h, int64_t m, int64_t n, int dtype, Geometry* g, bool batch = false,
         int force_rpl = 0)
{
    g->nc = padded_columns(n);
    if (g->nc < 0) return TSQR_ERR_UNSUPPORTED;
    const TuneEntry* te = find_tuning(h, dtype, g->nc, m, batch);
    g->rpl = force_rpl > 0 ? force_rpl
             : (int)(h->rpl > 0 ? h->rpl
                                : (te ? te->rpl : (dtype == TSQR_F64 ? TSQR_DEFAULT_RPL_F64 : TSQR_DEFAULT_RPL_F32)));
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
    } else if (te && te->leaf_rows > 0) {
        L = align_up(te->leaf_rows, chunk);
    } else if (batch) {
        // batched leaves: 64 chunks (8192 rows at 8 rows per lane).  Leaves
        // that long keep most instances of a ragged batch in a single leaf,
        // with no tree at all, and give the large ones shallow trees; the
        // many instances supply the parallelism.
        L = 64 * chunk;
    } else {
        const int64_t wpc = h->waves_per_cu > 0 ? h->waves_per_cu
                            : (te && te->waves_per_cu > 0) ? te->waves_per_cu
                                                           : leaf_occupancy(h, dtype, g->nc, g->rpl);
        const int64_t target = (int64_t)h->cu_count * wpc;
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
hipError_t dispatch_batch(const tsqr::BatchArgs<T>& a, int tiles, int nc, int rpl, hipStream_t s)
{
#define TSQR_CALL(tag, NC, RPL)                                                         \
    if constexpr (sizeof(T) == sizeof(tsqr::tag)) {                                     \
        if (nc == NC && rpl == RPL)                                                     \
            return tsqr::launch_batch_##tag##_##NC##_##RPL(                             \
                reinterpret_cast<const tsqr::BatchArgs<tsqr::tag>&>(a), tiles, s);      \
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
           int64_t ws_bytes, void* stream, int dtype, bool stamped = false, uint64_t* stamps = nullptr)
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
    if (stamped && !stamps) return -10;
    if (h->planning_only) return TSQR_ERR_NO_DEVICE;

    tsqr::LeafTreeArgs<T> a;
    a.stamps = stamps;
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
    h->scratch = device_scratch(device);
    h->cu_count = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    h->leaf_rows = 0;
    h->rpl = 0;
    h->waves_per_cu = 0;
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
    h->scratch = nullptr;
    h->cu_count = cu_count;
    h->leaf_rows = 0;
    h->rpl = 0;
    h->waves_per_cu = 0;
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
    case TSQR_ERR_SCRATCH: return "problem needs more than the fixed scratch of the allocation-free entry point";
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

int tsqr_tuning_add(tsqr_handle_t handle, int dtype, int64_t n, int64_t m_max, int64_t rows_per_lane,
                    int64_t waves_per_cu, int64_t leaf_rows, int batch)
{
    if (!handle) return -1;
    if (dtype != TSQR_F64 && dtype != TSQR_F32) return -2;
    const int nc = n >= 1 ? padded_columns(n) : -1;
    if (nc < 0) return -3;
    if (m_max < 0) return -4;
    if (rows_per_lane < 1 || rows_per_lane > 64 || !leaf_instance_exists(dtype, nc, (int)rows_per_lane)) return -5;
    if (waves_per_cu < 0) return -6;
    if (leaf_rows < 0) return -7;
    if (handle->tuning.size() >= 4096) return TSQR_ERR_UNSUPPORTED;
    TuneEntry e;
    e.dtype = dtype;
    e.nc = nc;
    e.m_max = m_max;
    e.rpl = (int)rows_per_lane;
    e.waves_per_cu = waves_per_cu;
    e.leaf_rows = leaf_rows;
    e.batch = batch != 0;
    // a later entry for the same key replaces the earlier one
    for (TuneEntry& old : handle->tuning) {
        if (old.dtype == e.dtype && old.nc == e.nc && old.batch == e.batch && (e.batch || old.m_max == e.m_max)) {
            old = e;
            return 0;
        }
    }
    try {
        handle->tuning.push_back(e);
    } catch (...) {
        return TSQR_ERR_ALLOC;
    }
    return 0;
}

int tsqr_tuning_clear(tsqr_handle_t handle)
{
    if (!handle) return -1;
    handle->tuning.clear();
    return 0;
}

int64_t tsqr_rows_per_lane_compiled(int dtype, int64_t n, int64_t* values, int64_t capacity)
{
    if (dtype != TSQR_F64 && dtype != TSQR_F32) return -1;
    const int nc = n >= 1 ? padded_columns(n) : -1;
    if (nc < 0) return -2;
    if (capacity < 0 || (capacity > 0 && !values)) return -3;
    int64_t count = 0;
#define TSQR_LIST(tag, NC, RPL)                                                 \
    if ((dtype == TSQR_F64) == (sizeof(tsqr::tag) == 8) && nc == NC) {          \
        if (count < capacity) values[count] = RPL;                              \
        ++count;                                                                \
    }
    TSQR_LEAF_INSTANCES(TSQR_LIST)
#undef TSQR_LIST
    return count;
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

int tsqr_geqr_r_f64_stamped(tsqr_handle_t handle, int64_t m, int64_t n, const double* A, int64_t lda, double* R,
                            int64_t ldr, void* ws, int64_t ws_bytes, uint64_t* stamps, void* stream)
{
    return geqr_r<double>(handle, m, n, A, lda, R, ldr, ws, ws_bytes, stream, TSQR_F64, true, stamps);
}

int tsqr_geqr_r_f64_noalloc(tsqr_handle_t handle, int64_t m, int64_t n, const double* A, int64_t lda, double* R,
                            int64_t ldr, void* stream)
{
    if (!handle) return -1;
    if (m < 0) return -2;
    if (n < 0) return -3;
    if (m > 0 && n > 0 && !A) return -4;
    if (lda < (m > 1 ? m : 1)) return -5;
    if (n > 0 && !R) return -6;
    if (ldr < (n > 1 ? n : 1)) return -7;
    if (n == 0) return 0;
    Geometry g;
    int rc = plan(handle, m, n, TSQR_F64, &g);
    if (rc) return rc;
    if (g.ws_bytes > TSQR_NOALLOC_SCRATCH_BYTES) return TSQR_ERR_SCRATCH;
    if (handle->planning_only) return TSQR_ERR_NO_DEVICE;
    if (!handle->scratch) {
        handle->last_hip_error = (int)hipErrorInvalidSymbol;
        return TSQR_ERR_HIP;
    }
    return geqr_r<double>(handle, m, n, A, lda, R, ldr, handle->scratch, TSQR_NOALLOC_SCRATCH_BYTES, stream,
                          TSQR_F64);
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

// ---- batched --------------------------------------------------------------

struct tsqr_batch_plan_s {
    tsqr_handle_s* h;
    int dtype;
    int64_t batch;
    int64_t n;
    int nc;
    int rpl;
    int64_t leaf_rows;
    int64_t leaves;          // all instances
    int64_t tiles;
    int64_t ticket_bytes;
    int64_t ws_bytes;
    tsqr::BatchInstance* d_inst;
    tsqr::BatchTile* d_tiles;
    std::vector<tsqr::BatchInstance> h_inst;   // host copies of the two tables
    std::vector<tsqr::BatchTile> h_tiles;
};

namespace {
int batch_plan_make(tsqr_handle_t h, int64_t batch, int64_t n, const int64_t* m, const int64_t* a_offset,
                    const int64_t* lda, int dtype, int force_rpl, tsqr_batch_plan_t* out,
                    int64_t leaf_rows = 0);
}

int tsqr_batch_plan_create(tsqr_handle_t h, int64_t batch, int64_t n, const int64_t* m, const int64_t* a_offset,
                           const int64_t* lda, int dtype, tsqr_batch_plan_t* out)
{
    return batch_plan_make(h, batch, n, m, a_offset, lda, dtype, 0, out);
}

namespace {
// The batched plan; force_rpl (if positive) fixes the rows per lane, as the
// mixed-precision fallback (compiled at 8 rows per lane only) needs, and
// leaf_rows (if positive) the leaf size, rounded up to whole chunks.
int batch_plan_make(tsqr_handle_t h, int64_t batch, int64_t n, const int64_t* m, const int64_t* a_offset,
                    const int64_t* lda, int dtype, int force_rpl, tsqr_batch_plan_t* out, int64_t leaf_rows)
{
    if (!h) return -1;
    if (batch < 0) return -2;
    if (n < 0) return -3;
    if (batch > 0 && !m) return -4;
    if (batch > 0 && !a_offset) return -5;
    if (dtype != TSQR_F64 && dtype != TSQR_F32) return -7;
    if (!out) return -8;
    *out = nullptr;
    for (int64_t b = 0; b < batch; ++b) {
        if (m[b] < 0) return -4;
        if (a_offset[b] < 0) return -5;
        const int64_t ld = lda ? lda[b] : (m[b] > 1 ? m[b] : 1);
        if (ld < (m[b] > 1 ? m[b] : 1)) return -6;
    }
    if (n > TSQR_MAX_N) return TSQR_ERR_UNSUPPORTED;
    Geometry g;
    int rc = n > 0 ? plan(h, 1, n, dtype, &g, true, force_rpl) : 0;
    if (rc) return rc;
    // the leaf size: the handle's option, else the tuning table's batched
    // entry, else 64 chunks (see plan)
    int64_t L = n > 0 ? g.leaf_rows
                      : (h->leaf_rows > 0 ? align_up(h->leaf_rows, kRowsPerLaneUnit) : 64 * kRowsPerLaneUnit);
    if (n > 0 && leaf_rows > 0) L = align_up(leaf_rows, (int64_t)kRowsPerLaneUnit * g.rpl);
    std::vector<tsqr::BatchInstance> inst((size_t)batch);
    std::vector<tsqr::BatchTile> tiles;
    std::vector<int64_t> tile_rows;
    int64_t leaves = 0;
    for (int64_t b = 0; b < batch; ++b) {
        tsqr::BatchInstance& in = inst[(size_t)b];
        in.a_off = a_offset[b];
        in.m = m[b];
        in.lda = lda ? lda[b] : (m[b] > 1 ? m[b] : 1);
        in.leaf_rows = L;
        const int64_t P = m[b] > 0 ? (m[b] + L - 1) / L : 1;
        if (P > ((int64_t)1 << 30)) return TSQR_ERR_UNSUPPORTED;
        in.leaves = (int32_t)P;
        in.pad = 0;
        in.ticket_off = leaves;
        in.tri_off = leaves * (n > 0 ? g.tri_elems : 0);
        for (int64_t i = 0; i < P; ++i) {
            tiles.push_back(tsqr::BatchTile{(int32_t)b, (int32_t)i});
            const int64_t r = std::min(L, m[b] - i * L);
            tile_rows.push_back(r > 0 ? r : 0);
        }
        leaves += P;
    }
    if (batch > ((int64_t)1 << 31) - 1 || (int64_t)tiles.size() > ((int64_t)1 << 31) - 1) return TSQR_ERR_UNSUPPORTED;
    // longest tiles first (stable: equal lengths keep instance order)
    std::vector<int64_t> order(tiles.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int64_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return tile_rows[(size_t)x] > tile_rows[(size_t)y]; });
    std::vector<tsqr::BatchTile> sorted(tiles.size());
    for (size_t i = 0; i < order.size(); ++i) sorted[i] = tiles[(size_t)order[i]];

    tsqr_batch_plan_s* p = new (std::nothrow) tsqr_batch_plan_s;
    if (!p) return TSQR_ERR_ALLOC;
    p->h = h;
    p->dtype = dtype;
    p->batch = batch;
    p->n = n;
    p->nc = n > 0 ? g.nc : 0;
    p->rpl = n > 0 ? g.rpl : 0;
    p->leaf_rows = L;
    p->leaves = leaves;
    p->tiles = (int64_t)sorted.size();
    p->ticket_bytes = align_up(leaves * 4, kAlign);
    p->ws_bytes = p->ticket_bytes + align_up(leaves * (n > 0 ? g.tri_elems : 0) * elem_bytes(dtype), kAlign);
    p->d_inst = nullptr;
    p->d_tiles = nullptr;
    if (!h->planning_only && batch > 0 && n > 0) {
        hipError_t e = hipMalloc(&p->d_inst, sizeof(tsqr::BatchInstance) * inst.size());
        if (e == hipSuccess) e = hipMalloc(&p->d_tiles, sizeof(tsqr::BatchTile) * sorted.size());
        if (e == hipSuccess)
            e = hipMemcpy(p->d_inst, inst.data(), sizeof(tsqr::BatchInstance) * inst.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(p->d_tiles, sorted.data(), sizeof(tsqr::BatchTile) * sorted.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (p->d_inst) (void)hipFree(p->d_inst);
            if (p->d_tiles) (void)hipFree(p->d_tiles);
            delete p;
            h->last_hip_error = (int)e;
            return TSQR_ERR_ALLOC;
        }
    }
    p->h_inst = std::move(inst);
    p->h_tiles = std::move(sorted);
    *out = p;
    return 0;
}
}  // namespace

int tsqr_batch_plan_schedule(tsqr_batch_plan_t plan, int64_t* inst, int64_t* tiles)
{
    if (!plan) return -1;
    if (inst) {
        for (size_t b = 0; b < plan->h_inst.size(); ++b) {
            const tsqr::BatchInstance& in = plan->h_inst[b];
            int64_t* o = inst + 7 * b;
            o[0] = in.a_off;
            o[1] = in.m;
            o[2] = in.lda;
            o[3] = in.leaf_rows;
            o[4] = in.leaves;
            o[5] = in.ticket_off;
            o[6] = in.tri_off;
        }
    }
    if (tiles) {
        for (size_t t = 0; t < plan->h_tiles.size(); ++t) {
            tiles[2 * t] = plan->h_tiles[t].inst;
            tiles[2 * t + 1] = plan->h_tiles[t].leaf;
        }
    }
    return 0;
}

int tsqr_batch_plan_destroy(tsqr_batch_plan_t plan)
{
    if (!plan) return 0;
    if (plan->d_inst) (void)hipFree(plan->d_inst);
    if (plan->d_tiles) (void)hipFree(plan->d_tiles);
    delete plan;
    return 0;
}

int64_t tsqr_batch_workspace_bytes(tsqr_batch_plan_t plan)
{
    if (!plan) return -1;
    return plan->ws_bytes;
}

int tsqr_batch_plan_info(tsqr_batch_plan_t plan, int64_t* tiles, int64_t* leaves, int64_t* leaf_rows)
{
    if (!plan) return -1;
    if (tiles) *tiles = plan->tiles;
    if (leaves) *leaves = plan->leaves;
    if (leaf_rows) *leaf_rows = plan->leaf_rows;
    return 0;
}

namespace {
// Argument checks of tsqr_batch_exec, in argument order: 0, a negative code,
// or 1 for a plan with nothing to do
int batch_check(tsqr_batch_plan_t plan, const void* A, void* R, int64_t ldr, void* ws, int64_t ws_bytes)
{
    if (!plan) return -1;
    if (plan->batch > 0 && plan->n > 0 && !A) return -2;
    if (plan->batch > 0 && plan->n > 0 && !R) return -3;
    if (ldr < (plan->n > 1 ? plan->n : 1)) return -4;
    if (plan->batch == 0 || plan->n == 0) return 1;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) != 0) return -5;
    if (ws_bytes < plan->ws_bytes) return -6;
    return 0;
}

int batch_exec(tsqr_batch_plan_t plan, const void* A, void* R, int64_t ldr, void* ws, int64_t ws_bytes,
               uint64_t* stamps, void* stream)
{
    const int rc = batch_check(plan, A, R, ldr, ws, ws_bytes);
    if (rc) return rc > 0 ? 0 : rc;
    if (plan->h->planning_only) return TSQR_ERR_NO_DEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned* tickets = static_cast<unsigned*>(ws);
    hipError_t e = tsqr::launch_zero_u32(tickets, plan->leaves, s);
    if (e != hipSuccess) return hip_status(plan->h, e);
    if (plan->dtype == TSQR_F64) {
        tsqr::BatchArgs<double> a;
        a.A = static_cast<const double*>(A);
        a.run_if = nullptr;
        a.n = (int)plan->n;
        a.inst = plan->d_inst;
        a.tiles = plan->d_tiles;
        a.tri = reinterpret_cast<double*>(static_cast<char*>(ws) + plan->ticket_bytes);
        a.tickets = tickets;
        a.R = static_cast<double*>(R);
        a.ldr = ldr;
        a.stamps = stamps;
        e = dispatch_batch<double>(a, (int)plan->tiles, plan->nc, plan->rpl, s);
    } else {
        tsqr::BatchArgs<float> a;
        a.A = static_cast<const float*>(A);
        a.run_if = nullptr;
        a.n = (int)plan->n;
        a.inst = plan->d_inst;
        a.tiles = plan->d_tiles;
        a.tri = reinterpret_cast<float*>(static_cast<char*>(ws) + plan->ticket_bytes);
        a.tickets = tickets;
        a.R = static_cast<float*>(R);
        a.ldr = ldr;
        a.stamps = stamps;
        e = dispatch_batch<float>(a, (int)plan->tiles, plan->nc, plan->rpl, s);
    }
    return hip_status(plan->h, e);
}
}  // namespace

int tsqr_batch_exec(tsqr_batch_plan_t plan, const void* A, void* R, int64_t ldr, void* ws, int64_t ws_bytes,
                    void* stream)
{
    return batch_exec(plan, A, R, ldr, ws, ws_bytes, nullptr, stream);
}

int tsqr_batch_exec_stamped(tsqr_batch_plan_t plan, const void* A, void* R, int64_t ldr, void* ws, int64_t ws_bytes,
                            uint64_t* stamps, void* stream)
{
    const int rc = batch_check(plan, A, R, ldr, ws, ws_bytes);
    if (rc) return rc > 0 ? 0 : rc;
    if (!stamps) return -7;
    return batch_exec(plan, A, R, ldr, ws, ws_bytes, stamps, stream);
}

int64_t tsqr_device_clock_khz(tsqr_handle_t h)
{
    if (!h) return -1;
    if (h->planning_only) return -1000 - TSQR_ERR_NO_DEVICE;
    int khz = 0;
    const hipError_t e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device);
    if (e != hipSuccess) return -1000 - hip_status(h, e);
    return khz > 0 ? khz : -1000 - TSQR_ERR_HIP;
}

// ---- mixed precision: FP32 TSQR, then one FP64 correction --------------------

struct tsqr_mixed_plan_s {
    tsqr_handle_s* h;
    int64_t batch, m, n, lda, stride_a;
    int nc;
    tsqr_batch_plan_t inner;     // the FP32 batched factorization
    tsqr_batch_plan_t fb;        // the FP64 fallback over the FP32 storage (8 rows per lane), fixed at creation
    int64_t sample_rows;         // rows of the sample R~ is computed from (0: all of A)
    uint64_t seed;
    int64_t rows_per_block;
    int blocks;
    int64_t off_sample, off_inner, inner_bytes, off_rt, off_part, off_flags, off_fb, fb_bytes, ws_bytes;
};

namespace {
// Rows per correction workgroup: about 1024 workgroups over the whole batch
// (four two-wavefront workgroups fit a CU at n = 50, by LDS), at least 1024
// rows, always a multiple of the 16-row tile.
int64_t mixed_rows_per_block(int64_t batch, int64_t m)
{
    constexpr int64_t kTargetBlocks = 1024;
    const int64_t per_inst = batch > 0 ? (kTargetBlocks + batch - 1) / batch : 1;
    int64_t rows = (m + per_inst - 1) / per_inst;
    if (rows < 1024) rows = 1024;
    return (rows + 15) / 16 * 16;
}

hipError_t dispatch_fallback(const tsqr::BatchArgs<double, float>& a, int tiles, int nc, hipStream_t s)
{
    switch (nc) {
    case 16: return tsqr::launch_batch_f64in32_16(a, tiles, s);
    case 32: return tsqr::launch_batch_f64in32_32(a, tiles, s);
    case 50: return tsqr::launch_batch_f64in32_50(a, tiles, s);
    case 64: return tsqr::launch_batch_f64in32_64(a, tiles, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t dispatch_mixed(const tsqr::MixedArgs& a, int nc, int batch, hipStream_t s)
{
    switch (nc) {
    case 16: return tsqr::launch_mixed_16(a, batch, s);
    case 32: return tsqr::launch_mixed_32(a, batch, s);
    case 50: return tsqr::launch_mixed_50(a, batch, s);
    case 64: return tsqr::launch_mixed_64(a, batch, s);
    default: return hipErrorInvalidValue;
    }
}

int gram_width(int nc)
{
    switch (nc) {
    case 16: return tsqr::MfmaGram<16>::W;
    case 32: return tsqr::MfmaGram<32>::W;
    case 50: return tsqr::MfmaGram<50>::W;
    default: return tsqr::MfmaGram<64>::W;
    }
}
}  // namespace

namespace {
// Both creators: sample_rows = 0 factors all of A in FP32, otherwise a sample
// of that many rows (rounded up to a multiple of the 64-row sample block; all
// of A when that reaches m).
int mixed_plan_make(tsqr_handle_t h, int64_t batch, int64_t m, int64_t n, int64_t lda, int64_t stride_a,
                    int64_t sample_rows, uint64_t seed, tsqr_mixed_plan_t* out)
{
    if (n > TSQR_MAX_N) return TSQR_ERR_UNSUPPORTED;
    const int nc = n > 0 ? padded_columns(n) : 16;
    if (nc < 0) return TSQR_ERR_UNSUPPORTED;
    int64_t srows = (sample_rows + tsqr::kSampleBlock - 1) / tsqr::kSampleBlock * tsqr::kSampleBlock;
    if (srows >= m) srows = 0;
    // the FP32 factorization runs over A itself, or over the sample buffer
    // (instance b's s x n sample at b*s*n in it, ld s)
    const int64_t im = srows ? srows : m, ilda = srows ? srows : lda;
    std::vector<int64_t> ms((size_t)batch, im), offs((size_t)batch), ldas((size_t)batch, ilda);
    for (int64_t b = 0; b < batch; ++b) offs[(size_t)b] = srows ? b * srows * n : b * stride_a;
    std::vector<int64_t> fms((size_t)batch, m), foffs((size_t)batch), fldas((size_t)batch, lda);
    for (int64_t b = 0; b < batch; ++b) foffs[(size_t)b] = b * stride_a;
    tsqr_batch_plan_t inner = nullptr, fb = nullptr;
    // a sample is short: its leaves are sized so the batch has about 2048 of
    // them (every SIMD busy) instead of the batched default
    const int64_t sample_leaf = srows ? (batch * srows + 2047) / 2048 : 0;
    int rc = batch_plan_make(h, batch, n, ms.data(), offs.data(), ldas.data(), TSQR_F32, 0, &inner, sample_leaf);
    if (rc) return rc;
    rc = batch_plan_make(h, batch, n, fms.data(), foffs.data(), fldas.data(), TSQR_F64, 8, &fb);
    if (rc) {
        tsqr_batch_plan_destroy(inner);
        return rc;
    }
    if (n > 0 && fb->rpl != 8) {
        tsqr_batch_plan_destroy(inner);
        tsqr_batch_plan_destroy(fb);
        return TSQR_ERR_UNSUPPORTED;
    }
    tsqr_mixed_plan_s* p = new (std::nothrow) tsqr_mixed_plan_s;
    if (!p) {
        tsqr_batch_plan_destroy(inner);
        tsqr_batch_plan_destroy(fb);
        return TSQR_ERR_ALLOC;
    }
    p->h = h;
    p->batch = batch;
    p->m = m;
    p->n = n;
    p->lda = lda;
    p->stride_a = stride_a;
    p->nc = nc;
    p->inner = inner;
    p->fb = fb;
    p->sample_rows = srows;
    p->seed = seed;
    p->rows_per_block = mixed_rows_per_block(batch, m);
    p->blocks = (int)(m > 0 ? (m + p->rows_per_block - 1) / p->rows_per_block : 1);
    const int64_t W = gram_width(nc);
    p->inner_bytes = tsqr_batch_workspace_bytes(inner);
    p->fb_bytes = tsqr_batch_workspace_bytes(fb);
    int64_t off = 0;
    p->off_sample = off;
    off += align_up(batch * srows * n * 4, kAlign);
    p->off_inner = off;
    off += align_up(p->inner_bytes > 0 ? p->inner_bytes : 0, kAlign);
    p->off_rt = off;
    off += align_up(batch * n * n * 4, kAlign);
    p->off_part = off;
    off += align_up(batch * p->blocks * W * W * 8, kAlign);
    p->off_flags = off;
    off += align_up(batch * 4, kAlign);
    p->off_fb = off;
    off += align_up(p->fb_bytes > 0 ? p->fb_bytes : 0, kAlign);
    p->ws_bytes = off;
    *out = p;
    return 0;
}
}  // namespace

int tsqr_mixed_plan_create(tsqr_handle_t h, int64_t batch, int64_t m, int64_t n, int64_t lda, int64_t stride_a,
                           tsqr_mixed_plan_t* out)
{
    if (!h) return -1;
    if (batch < 0) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (lda < (m > 1 ? m : 1)) return -5;
    if (batch > 1 && stride_a < lda * n) return -6;
    if (stride_a < 0) return -6;
    if (!out) return -7;
    *out = nullptr;
    return mixed_plan_make(h, batch, m, n, lda, stride_a, 0, 0, out);
}

int tsqr_mixed_plan_create_sampled(tsqr_handle_t h, int64_t batch, int64_t m, int64_t n, int64_t lda,
                                   int64_t stride_a, int64_t sample_rows, uint64_t seed, tsqr_mixed_plan_t* out)
{
    if (!h) return -1;
    if (batch < 0) return -2;
    if (m < 0) return -3;
    if (n < 0) return -4;
    if (lda < (m > 1 ? m : 1)) return -5;
    if (batch > 1 && stride_a < lda * n) return -6;
    if (stride_a < 0) return -6;
    if (sample_rows < 0) return -7;
    if (!out) return -9;
    *out = nullptr;
    return mixed_plan_make(h, batch, m, n, lda, stride_a, sample_rows, seed, out);
}

int64_t tsqr_mixed_rtilde_offset(tsqr_mixed_plan_t plan)
{
    if (!plan) return -1;
    return plan->off_rt;
}

int tsqr_mixed_plan_destroy(tsqr_mixed_plan_t plan)
{
    if (!plan) return 0;
    tsqr_batch_plan_destroy(plan->inner);
    tsqr_batch_plan_destroy(plan->fb);
    delete plan;
    return 0;
}

int64_t tsqr_mixed_workspace_bytes(tsqr_mixed_plan_t plan)
{
    if (!plan) return -1;
    return plan->ws_bytes;
}

namespace {
int mixed_exec(tsqr_mixed_plan_t plan, const float* A, const float* Rt_in, double* R, int64_t ldr, int* fallback,
               void* ws, int64_t ws_bytes, void* stream);
int rtilde_stage(tsqr_mixed_plan_t plan, const float* A, char* base, void* stream);
}

int tsqr_mixed_exec(tsqr_mixed_plan_t plan, const float* A, double* R, int64_t ldr, int* fallback, void* ws,
                    int64_t ws_bytes, void* stream)
{
    return mixed_exec(plan, A, nullptr, R, ldr, fallback, ws, ws_bytes, stream);
}

int tsqr_mixed_exec_rtilde(tsqr_mixed_plan_t plan, const float* A, const float* Rt, double* R, int64_t ldr,
                           int* fallback, void* ws, int64_t ws_bytes, void* stream)
{
    if (plan && plan->batch > 0 && plan->n > 0 && plan->m > 0 && !Rt) return -3;
    const int rc = mixed_exec(plan, A, Rt, R, ldr, fallback, ws, ws_bytes, stream);
    // argument codes shift by one past A (the R~ argument is -3)
    return rc <= -3 ? rc - 1 : rc;
}

int tsqr_mixed_rtilde_exec(tsqr_mixed_plan_t plan, const float* A, void* ws, int64_t ws_bytes, void* stream)
{
    if (!plan) return -1;
    const bool work = plan->batch > 0 && plan->n > 0 && plan->m > 0;
    if (work && !A) return -2;
    if (!work) return 0;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) != 0) return -3;
    if (ws_bytes < plan->ws_bytes) return -4;
    if (plan->h->planning_only) return TSQR_ERR_NO_DEVICE;
    return rtilde_stage(plan, A, static_cast<char*>(ws), stream);
}

namespace {
// The first stage: R~ of A (or of its row sample) by the FP32 batched TSQR,
// into the plan's R~ area of the workspace at base
int rtilde_stage(tsqr_mixed_plan_t plan, const float* A, char* base, void* stream)
{
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* Rt = reinterpret_cast<float*>(base + plan->off_rt);
    const float* src = A;
    if (plan->sample_rows) {
        tsqr::SampleArgs sa;
        sa.A = A;
        sa.m = plan->m;
        sa.lda = plan->lda;
        sa.stride_a = plan->stride_a;
        sa.n = (int)plan->n;
        sa.S = reinterpret_cast<float*>(base + plan->off_sample);
        sa.s = plan->sample_rows;
        sa.seed = plan->seed;
        hipError_t e = tsqr::launch_mixed_sample(sa, (int)plan->batch, s);
        if (e != hipSuccess) return hip_status(plan->h, e);
        src = sa.S;
    }
    return tsqr_batch_exec(plan->inner, src, Rt, plan->n, base + plan->off_inner, plan->inner_bytes, stream);
}

int mixed_exec(tsqr_mixed_plan_t plan, const float* A, const float* Rt_in, double* R, int64_t ldr, int* fallback,
               void* ws, int64_t ws_bytes, void* stream)
{
    if (!plan) return -1;
    const bool work = plan->batch > 0 && plan->n > 0;
    if (work && plan->m > 0 && !A) return -2;
    if (work && !R) return -3;
    if (ldr < (plan->n > 1 ? plan->n : 1)) return -4;
    if (!work) return 0;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) != 0) return -6;
    if (ws_bytes < plan->ws_bytes) return -7;
    if (plan->h->planning_only) return TSQR_ERR_NO_DEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    float* Rt = reinterpret_cast<float*>(base + plan->off_rt);
    if (plan->m > 0 && !Rt_in) {
        const int rc = rtilde_stage(plan, A, base, stream);
        if (rc) return rc;
    }
    tsqr::MixedArgs a;
    a.A = A;
    a.m = plan->m;
    a.lda = plan->lda;
    a.stride_a = plan->stride_a;
    a.n = (int)plan->n;
    a.Rt = Rt_in ? Rt_in : Rt;     // the caller's R~ (tsqr_mixed_exec_rtilde), else the one just computed
    a.part = reinterpret_cast<double*>(base + plan->off_part);
    a.rows_per_block = plan->rows_per_block;
    a.blocks = plan->blocks;
    a.R = R;
    a.ldr = ldr;
    a.flags = reinterpret_cast<int*>(base + plan->off_flags);
    a.flags_out = fallback;
    hipError_t e = hipSuccess;
    if (plan->m > 0) e = dispatch_mixed(a, plan->nc, (int)plan->batch, s);
    if (e != hipSuccess) return hip_status(plan->h, e);
    // the plain FP64 path over the FP32 storage for the instances whose
    // Cholesky factorization failed (every instance when m = 0, where it gives
    // R = 0); the other instances' workgroups exit at once
    tsqr::BatchArgs<double, float> f;
    char* fws = base + plan->off_fb;
    f.A = A;
    f.run_if = plan->m > 0 ? a.flags : nullptr;
    f.n = (int)plan->n;
    f.inst = plan->fb->d_inst;
    f.tiles = plan->fb->d_tiles;
    f.tickets = reinterpret_cast<unsigned*>(fws);
    f.tri = reinterpret_cast<double*>(fws + plan->fb->ticket_bytes);
    f.R = R;
    f.ldr = ldr;
    e = tsqr::launch_zero_u32(f.tickets, plan->fb->leaves, s);
    if (e == hipSuccess) e = dispatch_fallback(f, (int)plan->fb->tiles, plan->nc, s);
    if (e == hipSuccess && plan->m == 0 && fallback)
        e = tsqr::launch_fill_u32(reinterpret_cast<unsigned*>(fallback), plan->batch, 1u, s);
    return hip_status(plan->h, e);
}
}  // namespace

// ---- the Q factor ------------------------------------------------------------

extern "C++" {
namespace {
constexpr int kQrRpl = 8;    // rows per lane of the compiled Q-factor kernels

struct QrLayout {
    Geometry g;
    int64_t nchunks;         // chunks over all of A (leaf sizes are whole chunks)
    int64_t ldv;             // rows of V: every row of every chunk
    int64_t off_v, off_tau_leaf, off_vn, off_tau_node, off_qblk, off_tq, ws_bytes;
    int levels;
};

int qr_plan(const tsqr_handle_s* h, int64_t m, int64_t n, int dtype, QrLayout* L)
{
    int rc = plan(h, m, n, dtype, &L->g, false, kQrRpl);
    if (rc) return rc;
    if (L->g.rpl != kQrRpl) return TSQR_ERR_UNSUPPORTED;
    const int64_t w = elem_bytes(dtype);
    const int64_t nc = L->g.nc, P = L->g.leaves, CH = (int64_t)kRowsPerLaneUnit * kQrRpl;
    L->nchunks = m > 0 ? (m + CH - 1) / CH : 1;
    int64_t off = L->g.ws_bytes;
    L->ldv = L->nchunks * CH;
    L->off_v = off;
    off += align_up(L->ldv * n * w, kAlign);
    L->off_tau_leaf = off;
    off += align_up(L->nchunks * nc * w, kAlign);
    L->off_vn = off;
    off += align_up(P * L->g.tri_elems * w, kAlign);
    L->off_tau_node = off;
    off += align_up(P * nc * w, kAlign);
    L->off_qblk = off;
    off += align_up(P * nc * nc * w, kAlign);
    L->off_tq = off;     // the per-leaf n x 64 blocks of tsqr_apply_qt_*
    off += align_up(P * nc * tsqr::kQtCols * w, kAlign);
    L->ws_bytes = off;
    int levels = 0;
    while (((int64_t)1 << levels) < P) ++levels;
    L->levels = levels;
    return 0;
}

// The factorization with reflector storage alone (Q == nullptr: tsqr_geqrf_*),
// or followed by the passes that form Q.
template <typename T>
hipError_t dispatch_qr(const tsqr::LeafTreeArgs<T>& a, int nc, T* Q, int64_t ldq, int levels, hipStream_t s)
{
    hipError_t e = hipErrorInvalidValue;
#define TSQR_CALL(tag, NC, RPL)                                                                          \
    if constexpr (sizeof(T) == sizeof(tsqr::tag)) {                                                      \
        if (nc == NC) {                                                                                  \
            const auto& at = reinterpret_cast<const tsqr::LeafTreeArgs<tsqr::tag>&>(a);                  \
            tsqr::tag* Qt = reinterpret_cast<tsqr::tag*>(Q);                                             \
            e = tsqr::launch_qr_leaf_tree_##tag##_##NC##_##RPL(at, s);                                   \
            if (!Qt) return e;                                                                           \
            for (int lv = levels - 1; lv >= 0 && e == hipSuccess; --lv) {                                \
                const int64_t span = (int64_t)1 << lv;                                                   \
                const int64_t nodes = at.leaves > span ? (at.leaves - 1 - span) / (2 * span) + 1 : 0;    \
                e = tsqr::launch_q_tree_##tag##_##NC##_##RPL(at, lv, (int)nodes, s);                      \
            }                                                                                            \
            if (e == hipSuccess) e = tsqr::launch_q_leaf_##tag##_##NC##_##RPL(at, Qt, ldq, s);           \
            return e;                                                                                    \
        }                                                                                                \
    }
    TSQR_QR_INSTANCES(TSQR_CALL)
#undef TSQR_CALL
    return e;
}

template <typename T>
hipError_t dispatch_qt(const tsqr::QtArgs<T>& x, int nc, int levels, hipStream_t s)
{
    hipError_t e = hipErrorInvalidValue;
#define TSQR_CALL(tag, NC, RPL)                                                                          \
    if constexpr (sizeof(T) == sizeof(tsqr::tag)) {                                                      \
        if (nc == NC) return tsqr::launch_qt_##tag##_##NC##_##RPL(                                        \
            reinterpret_cast<const tsqr::QtArgs<tsqr::tag>&>(x), levels, s);                             \
    }
    TSQR_QR_INSTANCES(TSQR_CALL)
#undef TSQR_CALL
    return e;
}

// Q may be null (the factorization only: R and the stored reflectors).
template <typename T>
int geqr_qr(tsqr_handle_t handle, int64_t m, int64_t n, const T* A, int64_t lda, T* Q, int64_t ldq, T* R,
            int64_t ldr, void* ws, int64_t ws_bytes, void* stream, bool form_q = true)
{
    constexpr int dtype = sizeof(T) == 8 ? TSQR_F64 : TSQR_F32;
    if (!handle) return -1;
    if (m < 0) return -2;
    if (n < 0 || n > m) return -3;
    if (n > 0 && !A) return -4;
    if (lda < (m > 1 ? m : 1)) return -5;
    if (form_q && n > 0 && !Q) return -6;
    if (form_q && ldq < (m > 1 ? m : 1)) return -7;
    if (n > 0 && !R) return -8;
    if (ldr < (n > 1 ? n : 1)) return -9;
    if (n == 0) return 0;
    if (n > TSQR_MAX_N) return TSQR_ERR_UNSUPPORTED;
    QrLayout L;
    int rc = qr_plan(handle, m, n, dtype, &L);
    if (rc) return rc;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) != 0) return -10;
    if (ws_bytes < L.ws_bytes) return -11;
    if (handle->planning_only) return TSQR_ERR_NO_DEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(ws);
    unsigned* tickets = reinterpret_cast<unsigned*>(base);
    hipError_t e = tsqr::launch_zero_u32(tickets, L.g.leaves, s);
    if (e != hipSuccess) return hip_status(handle, e);
    tsqr::LeafTreeArgs<T> a;
    a.A = A;
    a.m = m;
    a.lda = lda;
    a.n = (int)n;
    a.leaf_rows = L.g.leaf_rows;
    a.leaves = (int)L.g.leaves;
    a.tri = reinterpret_cast<T*>(base + L.g.ticket_bytes);
    a.tickets = tickets;
    a.R = R;
    a.ldr = ldr;
    a.qs.V = reinterpret_cast<T*>(base + L.off_v);
    a.qs.ldv = L.ldv;
    a.qs.tau_leaf = reinterpret_cast<T*>(base + L.off_tau_leaf);
    a.qs.Vn = reinterpret_cast<T*>(base + L.off_vn);
    a.qs.tau_node = reinterpret_cast<T*>(base + L.off_tau_node);
    a.qs.qblk = reinterpret_cast<T*>(base + L.off_qblk);
    e = dispatch_qr<T>(a, L.g.nc, form_q ? Q : nullptr, ldq, L.levels, s);
    return hip_status(handle, e);
}

template <typename T>
int apply_qt(tsqr_handle_t handle, int64_t m, int64_t n, int64_t k, const T* B, int64_t ldb, T* C, int64_t ldc,
             void* ws, int64_t ws_bytes, void* stream)
{
    constexpr int dtype = sizeof(T) == 8 ? TSQR_F64 : TSQR_F32;
    if (!handle) return -1;
    if (m < 0) return -2;
    if (n < 0 || n > m) return -3;
    if (k < 0) return -4;
    if (n > 0 && k > 0 && !B) return -5;
    if (ldb < (m > 1 ? m : 1)) return -6;
    if (n > 0 && k > 0 && !C) return -7;
    if (ldc < (n > 1 ? n : 1)) return -8;
    if (n == 0 || k == 0) return 0;
    if (n > TSQR_MAX_N) return TSQR_ERR_UNSUPPORTED;
    if (k > INT32_MAX) return TSQR_ERR_UNSUPPORTED;
    QrLayout L;
    int rc = qr_plan(handle, m, n, dtype, &L);
    if (rc) return rc;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) != 0) return -9;
    if (ws_bytes < L.ws_bytes) return -10;
    if (handle->planning_only) return TSQR_ERR_NO_DEVICE;
    char* base = static_cast<char*>(ws);
    tsqr::QtArgs<T> x;
    tsqr::LeafTreeArgs<T>& a = x.a;
    a.A = nullptr;
    a.m = m;
    a.lda = m > 1 ? m : 1;
    a.n = (int)n;
    a.leaf_rows = L.g.leaf_rows;
    a.leaves = (int)L.g.leaves;
    a.tri = nullptr;
    a.tickets = nullptr;
    a.R = nullptr;
    a.ldr = 0;
    a.qs.V = reinterpret_cast<T*>(base + L.off_v);
    a.qs.ldv = L.ldv;
    a.qs.tau_leaf = reinterpret_cast<T*>(base + L.off_tau_leaf);
    a.qs.Vn = reinterpret_cast<T*>(base + L.off_vn);
    a.qs.tau_node = reinterpret_cast<T*>(base + L.off_tau_node);
    a.qs.qblk = reinterpret_cast<T*>(base + L.off_qblk);
    x.B = B;
    x.ldb = ldb;
    x.k = (int)k;
    x.tq = reinterpret_cast<T*>(base + L.off_tq);
    x.C = C;
    x.ldc = ldc;
    const hipError_t e = dispatch_qt<T>(x, L.g.nc, L.levels, static_cast<hipStream_t>(stream));
    return hip_status(handle, e);
}
}  // namespace
}  // extern "C++"

int64_t tsqr_qr_workspace_bytes(tsqr_handle_t handle, int64_t m, int64_t n, int dtype)
{
    if (!handle) return -1;
    if (m < 0) return -2;
    if (n < 0 || n > m) return -3;
    if (dtype != TSQR_F64 && dtype != TSQR_F32) return -4;
    if (n == 0) return 0;
    QrLayout L;
    const int rc = qr_plan(handle, m, n, dtype, &L);
    if (rc) return -1000 - rc;
    return L.ws_bytes;
}

int tsqr_geqr_qr_f64(tsqr_handle_t handle, int64_t m, int64_t n, const double* A, int64_t lda, double* Q,
                     int64_t ldq, double* R, int64_t ldr, void* ws, int64_t ws_bytes, void* stream)
{
    return geqr_qr<double>(handle, m, n, A, lda, Q, ldq, R, ldr, ws, ws_bytes, stream);
}

int tsqr_geqr_qr_f32(tsqr_handle_t handle, int64_t m, int64_t n, const float* A, int64_t lda, float* Q,
                     int64_t ldq, float* R, int64_t ldr, void* ws, int64_t ws_bytes, void* stream)
{
    return geqr_qr<float>(handle, m, n, A, lda, Q, ldq, R, ldr, ws, ws_bytes, stream);
}

int tsqr_geqrf_f64(tsqr_handle_t handle, int64_t m, int64_t n, const double* A, int64_t lda, double* R, int64_t ldr,
                   void* ws, int64_t ws_bytes, void* stream)
{
    const int rc = geqr_qr<double>(handle, m, n, A, lda, nullptr, m > 1 ? m : 1, R, ldr, ws, ws_bytes, stream, false);
    return rc <= -8 ? rc + 2 : rc;
}

int tsqr_geqrf_f32(tsqr_handle_t handle, int64_t m, int64_t n, const float* A, int64_t lda, float* R, int64_t ldr,
                   void* ws, int64_t ws_bytes, void* stream)
{
    const int rc = geqr_qr<float>(handle, m, n, A, lda, nullptr, m > 1 ? m : 1, R, ldr, ws, ws_bytes, stream, false);
    return rc <= -8 ? rc + 2 : rc;
}

int tsqr_apply_qt_f64(tsqr_handle_t handle, int64_t m, int64_t n, int64_t k, const double* B, int64_t ldb, double* C,
                      int64_t ldc, void* ws, int64_t ws_bytes, void* stream)
{
    return apply_qt<double>(handle, m, n, k, B, ldb, C, ldc, ws, ws_bytes, stream);
}

int tsqr_apply_qt_f32(tsqr_handle_t handle, int64_t m, int64_t n, int64_t k, const float* B, int64_t ldb, float* C,
                      int64_t ldc, void* ws, int64_t ws_bytes, void* stream)
{
    return apply_qt<float>(handle, m, n, k, B, ldb, C, ldc, ws, ws_bytes, stream);
}

// ---- the learned correction of the sampled preconditioner -----------------------

namespace {
int kernel_status(tsqr_handle_t h, hipError_t e) { return hip_status(h, e); }
bool dims_ok(int64_t v) { return v >= 0 && v <= INT32_MAX; }
}  // namespace

int tsqr_gemm_bf16(tsqr_handle_t h, int ta, int tb, int64_t M, int64_t N, int64_t K, float alpha, const float* A,
                   int64_t lda, const float* B, int64_t ldb, float beta, float* C, int64_t ldc, void* stream)
{
    if (!h) return -1;
    if (!dims_ok(M)) return -4;
    if (!dims_ok(N)) return -5;
    if (!dims_ok(K)) return -6;
    const int64_t arows = ta ? K : M, brows = tb ? N : K;
    if (M > 0 && N > 0 && K > 0 && !A) return -8;
    if (lda < (arows > 1 ? arows : 1)) return -9;
    if (M > 0 && N > 0 && K > 0 && !B) return -10;
    if (ldb < (brows > 1 ? brows : 1)) return -11;
    if (M > 0 && N > 0 && !C) return -13;
    if (ldc < (M > 1 ? M : 1)) return -14;
    if (M == 0 || N == 0) return 0;
    if (h->planning_only) return TSQR_ERR_NO_DEVICE;
    tsqr::GemmArgs g;
    g.ta = ta ? 1 : 0;
    g.tb = tb ? 1 : 0;
    g.M = (int)M;
    g.N = (int)N;
    g.K = (int)K;
    g.alpha = alpha;
    g.beta = beta;
    g.A = A;
    g.lda = lda;
    g.B = B;
    g.ldb = ldb;
    g.C = C;
    g.ldc = ldc;
    return kernel_status(h, tsqr::launch_gemm_bf16(g, static_cast<hipStream_t>(stream)));
}

int tsqr_mlp_bias_act(tsqr_handle_t h, float* Z, int64_t rows, int64_t cols, int64_t ld, const float* bias, int relu,
                      void* stream)
{
    if (!h) return -1;
    if (!dims_ok(rows)) return -3;
    if (!dims_ok(cols)) return -4;
    if (rows > 0 && cols > 0 && (!Z || !bias)) return !Z ? -2 : -6;
    if (ld < (rows > 1 ? rows : 1)) return -5;
    if (rows == 0 || cols == 0) return 0;
    if (h->planning_only) return TSQR_ERR_NO_DEVICE;
    return kernel_status(h, tsqr::launch_bias_act(Z, (int)rows, (int)cols, ld, bias, relu ? 1 : 0,
                                                  static_cast<hipStream_t>(stream)));
}

int tsqr_mlp_relu_grad(tsqr_handle_t h, float* dA, const float* out, int64_t rows, int64_t cols, int64_t ld,
                       void* stream)
{
    if (!h) return -1;
    if (!dims_ok(rows)) return -4;
    if (!dims_ok(cols)) return -5;
    if (rows > 0 && cols > 0 && (!dA || !out)) return !dA ? -2 : -3;
    if (ld < (rows > 1 ? rows : 1)) return -6;
    if (rows == 0 || cols == 0) return 0;
    if (h->planning_only) return TSQR_ERR_NO_DEVICE;
    return kernel_status(h, tsqr::launch_relu_grad(dA, out, (int)rows, (int)cols, ld, static_cast<hipStream_t>(stream)));
}

int tsqr_mlp_colsum(tsqr_handle_t h, const float* Z, int64_t rows, int64_t cols, int64_t ld, float* s, void* stream)
{
    if (!h) return -1;
    if (!dims_ok(rows)) return -3;
    if (!dims_ok(cols)) return -4;
    if (cols > 0 && ((rows > 0 && !Z) || !s)) return !s ? -6 : -2;
    if (ld < (rows > 1 ? rows : 1)) return -5;
    if (cols == 0) return 0;
    if (h->planning_only) return TSQR_ERR_NO_DEVICE;
    return kernel_status(h, tsqr::launch_colsum(Z, (int)rows, (int)cols, ld, s, static_cast<hipStream_t>(stream)));
}

int tsqr_mlp_mse(tsqr_handle_t h, const float* Y, const float* T, float* D, int64_t rows, int64_t cols, int64_t ld,
                 float* loss, void* stream)
{
    if (!h) return -1;
    if (!dims_ok(rows) || rows == 0) return -5;
    if (!dims_ok(cols) || cols == 0) return -6;
    if (!Y) return -2;
    if (!T) return -3;
    if (!D) return -4;
    if (ld < rows) return -7;
    if (!loss) return -8;
    if (h->planning_only) return TSQR_ERR_NO_DEVICE;
    return kernel_status(h, tsqr::launch_mse(Y, T, D, (int)rows, (int)cols, ld, loss, static_cast<hipStream_t>(stream)));
}

int tsqr_mlp_adam(tsqr_handle_t h, float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1,
                  float b2, float eps, int64_t step, void* stream)
{
    if (!h) return -1;
    if (count < 0) return -6;
    if (count > 0 && (!p || !g || !m || !v)) return !p ? -2 : (!g ? -3 : (!m ? -4 : -5));
    if (step < 1) return -11;
    if (count == 0) return 0;
    if (h->planning_only) return TSQR_ERR_NO_DEVICE;
    // the bias corrections in FP64 (1 - b2^t loses most of its bits in FP32)
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
    return kernel_status(h, tsqr::launch_adam(p, g, m, v, count, lr, b1, b2, eps, c1, c2,
                                              static_cast<hipStream_t>(stream)));
}

int tsqr_surrogate_features(tsqr_handle_t h, const float* Rt, int64_t batch, int64_t n, float* X, void* stream)
{
    if (!h) return -1;
    if (!dims_ok(batch)) return -3;
    if (n < 1 || n > TSQR_MAX_N) return -4;
    if (batch > 0 && !Rt) return -2;
    if (batch > 0 && !X) return -5;
    if (batch == 0) return 0;
    if (h->planning_only) return TSQR_ERR_NO_DEVICE;
    return kernel_status(h, tsqr::launch_surrogate_features(Rt, (int)batch, (int)n, X, static_cast<hipStream_t>(stream)));
}

int tsqr_surrogate_targets(tsqr_handle_t h, const double* R, int64_t ldr, const float* Rt, int64_t batch, int64_t n,
                           float* Y, void* stream)
{
    if (!h) return -1;
    if (!dims_ok(batch)) return -5;
    if (n < 1 || n > TSQR_MAX_N) return -6;
    if (batch > 0 && !R) return -2;
    if (ldr < n) return -3;
    if (batch > 0 && !Rt) return -4;
    if (batch > 0 && !Y) return -7;
    if (batch == 0) return 0;
    if (h->planning_only) return TSQR_ERR_NO_DEVICE;
    return kernel_status(h, tsqr::launch_surrogate_targets(R, ldr, Rt, (int)batch, (int)n, Y,
                                                           static_cast<hipStream_t>(stream)));
}

int tsqr_surrogate_apply(tsqr_handle_t h, const float* Rt, const float* Y, int64_t batch, int64_t n, float* Rout,
                         void* stream)
{
    if (!h) return -1;
    if (!dims_ok(batch)) return -4;
    if (n < 1 || n > TSQR_MAX_N) return -5;
    if (batch > 0 && !Rt) return -2;
    if (batch > 0 && !Y) return -3;
    if (batch > 0 && !Rout) return -6;
    if (batch == 0) return 0;
    if (h->planning_only) return TSQR_ERR_NO_DEVICE;
    return kernel_status(h, tsqr::launch_surrogate_apply(Rt, Y, (int)batch, (int)n, Rout,
                                                         static_cast<hipStream_t>(stream)));
}

}  // extern "C"
