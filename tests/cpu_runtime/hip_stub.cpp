// A host-only stand-in for the parts of the HIP runtime (and rocBLAS) that
// libfsv calls, for checking the library's host side on a machine without a
// GPU.  Test infrastructure: it never computes anything.
//
//  - "Device" memory is host memory from malloc, so AddressSanitizer sees every
//    allocation; each copy is checked against the allocation it names (device
//    side) or the pinned buffer it touches (host side) and then performed.
//  - Kernel launches are checked (a registered kernel, a launch shape the
//    hardware accepts, dynamic LDS within the limit set for that kernel) and
//    logged; kernels do not run.
//  - Streams, events, graphs and BLAS handles live in registries: use or
//    destruction of an unknown or already destroyed handle aborts with a
//    message, as does freeing memory that is not allocated.
//  - Stream capture records copies and launches; a graph replay repeats the
//    checks of every recorded node.
//
// Every violation prints "hip_stub: ..." to stderr and aborts.
#include <hip/hip_runtime_api.h>

#include <cxxabi.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

namespace {

std::mutex g_mu;

[[noreturn]] void die(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::fprintf(stderr, "hip_stub: ");
    std::vfprintf(stderr, fmt, ap);
    std::fprintf(stderr, "\n");
    va_end(ap);
    std::fflush(stderr);
    std::abort();
}

struct Kernel {
    std::string name;
    int max_dyn = 65536;  // hipFuncAttributeMaxDynamicSharedMemorySize
};

struct Node {
    int kind = 0;  // 0 launch, 1 copy
    const void *fn = nullptr;
    dim3 grid, block;
    size_t shm = 0;
    void *dst = nullptr;
    const void *src = nullptr;
    size_t bytes = 0;
    hipMemcpyKind ck = hipMemcpyDefault;
};

struct Stream {
    bool capturing = false;
    std::vector<Node> rec;
};

std::map<uintptr_t, size_t> &dev_allocs() { static std::map<uintptr_t, size_t> m; return m; }
std::map<uintptr_t, size_t> &pin_allocs() { static std::map<uintptr_t, size_t> m; return m; }
std::map<const void *, Kernel> &kernels() { static std::map<const void *, Kernel> m; return m; }
std::map<const void *, std::string> &symbols() { static std::map<const void *, std::string> m; return m; }
std::map<hipStream_t, Stream *> &streams() { static std::map<hipStream_t, Stream *> m; return m; }
std::set<hipEvent_t> &events() { static std::set<hipEvent_t> s; return s; }
std::map<hipGraph_t, std::vector<Node> *> &graphs() { static std::map<hipGraph_t, std::vector<Node> *> m; return m; }
std::map<hipGraphExec_t, std::vector<Node> *> &execs() { static std::map<hipGraphExec_t, std::vector<Node> *> m; return m; }
std::set<void *> &blas_handles() { static std::set<void *> s; return s; }

unsigned long g_launches = 0, g_replays = 0;

std::string demangle(const char *s) {
    int st = 0;
    char *d = abi::__cxa_demangle(s, nullptr, nullptr, &st);
    std::string out = (st == 0 && d) ? d : s;
    std::free(d);
    return out;
}

// The allocation of `map` containing [p, p + n), or die.
void in_alloc(const std::map<uintptr_t, size_t> &m, const void *p, size_t n, const char *what) {
    const uintptr_t a = (uintptr_t)p;
    auto it = m.upper_bound(a);
    if (it == m.begin()) die("%s: %p (+%zu bytes) is not inside a live allocation", what, p, n);
    --it;
    if (a + n > it->first + it->second)
        die("%s: [%p, +%zu) runs past the end of the allocation at %p of %zu bytes (by %zu bytes)", what, p, n,
            (void *)it->first, it->second, (size_t)(a + n - (it->first + it->second)));
}

bool is_pinned(const void *p) {
    const uintptr_t a = (uintptr_t)p;
    auto it = pin_allocs().upper_bound(a);
    if (it == pin_allocs().begin()) return false;
    --it;
    return a < it->first + it->second;
}

Stream *stream_of(hipStream_t s, const char *what) {
    if (!s) return nullptr;
    auto it = streams().find(s);
    if (it == streams().end()) die("%s: unknown or destroyed stream %p", what, (void *)s);
    return it->second;
}

void check_event(hipEvent_t e, const char *what) {
    if (!events().count(e)) die("%s: unknown or destroyed event %p", what, (void *)e);
}

void check_copy(void *dst, const void *src, size_t n, hipMemcpyKind k, const char *what) {
    if (n == 0) return;
    switch (k) {
    case hipMemcpyHostToDevice:
        in_alloc(dev_allocs(), dst, n, what);
        if (is_pinned(src)) in_alloc(pin_allocs(), src, n, what);
        break;
    case hipMemcpyDeviceToHost:
        in_alloc(dev_allocs(), src, n, what);
        if (is_pinned(dst)) in_alloc(pin_allocs(), dst, n, what);
        break;
    case hipMemcpyDeviceToDevice:
        in_alloc(dev_allocs(), dst, n, what);
        in_alloc(dev_allocs(), src, n, what);
        break;
    default:
        die("%s: copy kind %d is not used by the library", what, (int)k);
    }
}

void do_copy(void *dst, const void *src, size_t n, hipMemcpyKind k, const char *what) {
    check_copy(dst, src, n, k, what);
    if (n) std::memmove(dst, src, n);
}

void check_launch(const void *fn, dim3 g, dim3 b, size_t shm, const char *what) {
    auto it = kernels().find(fn);
    if (it == kernels().end()) die("%s: launch of an unregistered kernel %p", what, fn);
    const Kernel &K = it->second;
    const char *nm = K.name.c_str();
    if (g.x == 0 || g.y == 0 || g.z == 0) die("%s: %s launched with an empty grid (%u, %u, %u)", what, nm, g.x, g.y, g.z);
    if (g.y > 65535 || g.z > 65535) die("%s: %s grid (%u, %u, %u) exceeds 65535 in y or z", what, nm, g.x, g.y, g.z);
    const unsigned long thr = (unsigned long)b.x * b.y * b.z;
    if (thr == 0 || thr > 1024) die("%s: %s launched with %lu threads per workgroup", what, nm, thr);
    if ((unsigned long)g.x * g.y * g.z * thr > (1ul << 32))
        die("%s: %s launches more than 2^32 work-items", what, nm);
    if (shm > (size_t)K.max_dyn)
        die("%s: %s asks for %zu bytes of dynamic LDS, its limit is %d", what, nm, shm, K.max_dyn);
}

void launch_or_record(const void *fn, dim3 g, dim3 b, size_t shm, hipStream_t st, const char *what) {
    check_launch(fn, g, b, shm, what);
    Stream *s = stream_of(st, what);
    if (s && s->capturing) {
        Node n;
        n.kind = 0;
        n.fn = fn;
        n.grid = g;
        n.block = b;
        n.shm = shm;
        s->rec.push_back(n);
        return;
    }
    ++g_launches;
}

struct CallCfg {
    dim3 g, b;
    size_t shm;
    hipStream_t st;
};
thread_local std::vector<CallCfg> g_cfg;

}  // namespace

extern "C" {

// ---- registration emitted by the HIP compiler ----
void **__hipRegisterFatBinary(const void *) {
    static void *mod = nullptr;
    return &mod;
}
void __hipUnregisterFatBinary(void **) {}
void __hipRegisterFunction(void **, const void *hostFunction, char *, const char *deviceName, unsigned int, void *,
                           void *, void *, void *, int *) {
    std::lock_guard<std::mutex> lk(g_mu);
    kernels()[hostFunction].name = demangle(deviceName);
}
void __hipRegisterVar(void **, void *var, char *, const char *deviceName, int, size_t size, int, int) {
    std::lock_guard<std::mutex> lk(g_mu);
    // a __device__ variable lives in host memory here: register it as device memory
    symbols()[var] = deviceName;
    dev_allocs()[(uintptr_t)var] = size;
}
void __hipRegisterManagedVar(void *, void **, void *, const char *, size_t, unsigned) {}
void __hipRegisterSurface(void **, void *, char *, const char *, int, int) {}
void __hipRegisterTexture(void **, void *, char *, const char *, int, int, int) {}

hipError_t __hipPushCallConfiguration(dim3 g, dim3 b, size_t shm, hipStream_t st) {
    g_cfg.push_back({g, b, shm, st});
    return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3 *g, dim3 *b, size_t *shm, hipStream_t *st) {
    if (g_cfg.empty()) die("__hipPopCallConfiguration without a pushed configuration");
    const CallCfg c = g_cfg.back();
    g_cfg.pop_back();
    *g = c.g;
    *b = c.b;
    *shm = c.shm;
    *st = c.st;
    return hipSuccess;
}

hipError_t hipLaunchKernel(const void *fn, dim3 g, dim3 b, void **, size_t shm, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_mu);
    launch_or_record(fn, g, b, shm, st, "hipLaunchKernel");
    return hipSuccess;
}
hipError_t hipExtLaunchKernel(const void *fn, dim3 g, dim3 b, void **, size_t shm, hipStream_t st, hipEvent_t e0,
                              hipEvent_t e1, int) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (e0) check_event(e0, "hipExtLaunchKernel start event");
    if (e1) check_event(e1, "hipExtLaunchKernel stop event");
    launch_or_record(fn, g, b, shm, st, "hipExtLaunchKernel");
    return hipSuccess;
}

hipError_t hipFuncSetAttribute(const void *fn, hipFuncAttribute attr, int value) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = kernels().find(fn);
    if (it == kernels().end()) die("hipFuncSetAttribute on an unregistered kernel");
    if (attr == hipFuncAttributeMaxDynamicSharedMemorySize) {
        if (value < 0 || value > 163840) return hipErrorInvalidValue;
        it->second.max_dyn = value;
    }
    return hipSuccess;
}
hipError_t hipFuncGetAttributes(hipFuncAttributes *a, const void *fn) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = kernels().find(fn);
    if (it == kernels().end()) die("hipFuncGetAttributes on an unregistered kernel");
    std::memset(a, 0, sizeof *a);
    a->maxDynamicSharedSizeBytes = it->second.max_dyn;
    a->maxThreadsPerBlock = 1024;
    a->sharedSizeBytes = 128;  // the block-sum scratch of the reducing kernels
    return hipSuccess;
}

// ---- device, errors ----
hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t attr, int) {
    *v = attr == hipDeviceAttributeMultiprocessorCount ? 256 : 0;
    return hipSuccess;
}
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600 *p, int) {
    std::memset(p, 0, sizeof *p);
    std::strcpy(p->name, "host stand-in");
    p->multiProcessorCount = 256;
    p->sharedMemPerBlock = 65536;
    p->maxThreadsPerBlock = 1024;
    p->warpSize = 64;
    return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
const char *hipGetErrorString(hipError_t) { return "hip_stub error"; }

// ---- memory ----
hipError_t hipMalloc(void **p, size_t n) {
    std::lock_guard<std::mutex> lk(g_mu);
    void *q = std::malloc(n ? n : 1);
    if (!q) return hipErrorOutOfMemory;
    dev_allocs()[(uintptr_t)q] = n ? n : 1;
    *p = q;
    return hipSuccess;
}
hipError_t hipFree(void *p) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!p) return hipSuccess;
    auto it = dev_allocs().find((uintptr_t)p);
    if (it == dev_allocs().end() || symbols().count(p)) die("hipFree of %p, which is not a live device allocation", p);
    dev_allocs().erase(it);
    std::free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned int) {
    std::lock_guard<std::mutex> lk(g_mu);
    void *q = std::malloc(n ? n : 1);
    if (!q) return hipErrorOutOfMemory;
    pin_allocs()[(uintptr_t)q] = n ? n : 1;
    *p = q;
    return hipSuccess;
}
hipError_t hipHostFree(void *p) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!p) return hipSuccess;
    auto it = pin_allocs().find((uintptr_t)p);
    if (it == pin_allocs().end()) die("hipHostFree of %p, which is not a live pinned allocation", p);
    pin_allocs().erase(it);
    std::free(p);
    return hipSuccess;
}
hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind k) {
    std::lock_guard<std::mutex> lk(g_mu);
    do_copy(dst, src, n, k, "hipMemcpy");
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind k, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_mu);
    Stream *s = stream_of(st, "hipMemcpyAsync");
    if (s && s->capturing) {
        check_copy(dst, src, n, k, "hipMemcpyAsync (captured)");
        Node nd;
        nd.kind = 1;
        nd.dst = dst;
        nd.src = src;
        nd.bytes = n;
        nd.ck = k;
        s->rec.push_back(nd);
        return hipSuccess;
    }
    do_copy(dst, src, n, k, "hipMemcpyAsync");
    return hipSuccess;
}
hipError_t hipMemsetAsync(void *dst, int v, size_t n, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_mu);
    stream_of(st, "hipMemsetAsync");
    in_alloc(dev_allocs(), dst, n, "hipMemsetAsync");
    std::memset(dst, v, n);
    return hipSuccess;
}
hipError_t hipGetSymbolAddress(void **out, const void *sym) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!symbols().count(sym)) die("hipGetSymbolAddress of an unregistered symbol");
    *out = const_cast<void *>(sym);
    return hipSuccess;
}

// ---- streams and events ----
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) {
    std::lock_guard<std::mutex> lk(g_mu);
    Stream *x = new Stream();
    *s = (hipStream_t)x;
    streams()[*s] = x;
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    Stream *x = stream_of(s, "hipStreamDestroy");
    if (!x) die("hipStreamDestroy of the null stream");
    if (x->capturing) die("hipStreamDestroy of a stream that is capturing");
    streams().erase(s);
    delete x;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    Stream *x = stream_of(s, "hipStreamSynchronize");
    if (x && x->capturing) die("hipStreamSynchronize on a capturing stream");
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
    std::lock_guard<std::mutex> lk(g_mu);
    stream_of(s, "hipStreamWaitEvent");
    check_event(e, "hipStreamWaitEvent");
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) {
    std::lock_guard<std::mutex> lk(g_mu);
    *e = (hipEvent_t)std::malloc(16);
    events().insert(*e);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned int) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    std::lock_guard<std::mutex> lk(g_mu);
    check_event(e, "hipEventDestroy");
    events().erase(e);
    std::free((void *)e);
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    check_event(e, "hipEventRecord");
    Stream *x = stream_of(s, "hipEventRecord");
    if (x && x->capturing) die("hipEventRecord on a capturing stream");
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    std::lock_guard<std::mutex> lk(g_mu);
    check_event(e, "hipEventSynchronize");
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::mutex> lk(g_mu);
    check_event(a, "hipEventElapsedTime");
    check_event(b, "hipEventElapsedTime");
    *ms = 0.001f;
    return hipSuccess;
}

// ---- capture and graphs ----
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    std::lock_guard<std::mutex> lk(g_mu);
    Stream *x = stream_of(s, "hipStreamBeginCapture");
    if (!x) die("capture on the null stream");
    if (x->capturing) die("hipStreamBeginCapture on a stream that is already capturing");
    x->capturing = true;
    x->rec.clear();
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g) {
    std::lock_guard<std::mutex> lk(g_mu);
    Stream *x = stream_of(s, "hipStreamEndCapture");
    if (!x || !x->capturing) die("hipStreamEndCapture on a stream that is not capturing");
    x->capturing = false;
    auto *nodes = new std::vector<Node>(x->rec);
    x->rec.clear();
    *g = (hipGraph_t)nodes;
    graphs()[*g] = nodes;
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = graphs().find(g);
    if (it == graphs().end()) die("hipGraphDestroy of an unknown or destroyed graph");
    delete it->second;
    graphs().erase(it);
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *ex, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = graphs().find(g);
    if (it == graphs().end()) die("hipGraphInstantiate of an unknown graph");
    auto *nodes = new std::vector<Node>(*it->second);
    *ex = (hipGraphExec_t)nodes;
    execs()[*ex] = nodes;
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t ex) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = execs().find(ex);
    if (it == execs().end()) die("hipGraphExecDestroy of an unknown or destroyed graph");
    delete it->second;
    execs().erase(it);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = execs().find(ex);
    if (it == execs().end()) die("hipGraphLaunch of an unknown or destroyed graph");
    Stream *x = stream_of(s, "hipGraphLaunch");
    if (x && x->capturing) die("hipGraphLaunch on a capturing stream");
    for (const Node &n : *it->second) {
        if (n.kind == 0) {
            check_launch(n.fn, n.grid, n.block, n.shm, "graph replay");
            ++g_launches;
        } else {
            do_copy(n.dst, n.src, n.bytes, n.ck, "graph replay copy");
        }
    }
    ++g_replays;
    return hipSuccess;
}

// ---- test hooks ----
unsigned long hip_stub_launches(void) { return g_launches; }
unsigned long hip_stub_replays(void) { return g_replays; }
size_t hip_stub_live_device_bytes(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    size_t t = 0;
    for (auto &kv : dev_allocs())
        if (!symbols().count((const void *)kv.first)) t += kv.second;
    return t;
}
size_t hip_stub_live_handles(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    return streams().size() + events().size() + graphs().size() + execs().size() + pin_allocs().size() +
           blas_handles().size();
}

// ---- rocBLAS (the FP64 GEMM the library calls) ----
typedef void *rocblas_handle_t;
int rocblas_create_handle(rocblas_handle_t *h) {
    std::lock_guard<std::mutex> lk(g_mu);
    *h = std::malloc(8);
    blas_handles().insert(*h);
    return 0;
}
int rocblas_destroy_handle(rocblas_handle_t h) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!blas_handles().erase(h)) die("rocblas_destroy_handle of an unknown handle");
    std::free(h);
    return 0;
}
int rocblas_set_stream(rocblas_handle_t h, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!blas_handles().count(h)) die("rocblas_set_stream on an unknown handle");
    stream_of(s, "rocblas_set_stream");
    return 0;
}
int rocblas_set_atomics_mode(rocblas_handle_t h, int) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!blas_handles().count(h)) die("rocblas_set_atomics_mode on an unknown handle");
    return 0;
}
// Column-major C (m x n, ldc) = alpha op(A) op(B) + beta C; only untransposed
// operands are used by the library.
int rocblas_dgemm(rocblas_handle_t h, int ta, int tb, int m, int n, int k, const double *, const double *A, int lda,
                  const double *B, int ldb, const double *, double *C, int ldc) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!blas_handles().count(h)) die("rocblas_dgemm on an unknown handle");
    if (ta != 111 || tb != 111) die("rocblas_dgemm: transposed operands are not used by the library");
    if (m < 0 || n < 0 || k < 0 || lda < (m > 1 ? m : 1) || ldb < (k > 1 ? k : 1) || ldc < (m > 1 ? m : 1))
        die("rocblas_dgemm: bad sizes m %d n %d k %d lda %d ldb %d ldc %d", m, n, k, lda, ldb, ldc);
    if (m && n && k) {
        in_alloc(dev_allocs(), A, 8 * ((size_t)lda * (k - 1) + m), "rocblas_dgemm A");
        in_alloc(dev_allocs(), B, 8 * ((size_t)ldb * (n - 1) + k), "rocblas_dgemm B");
    }
    if (m && n) in_alloc(dev_allocs(), C, 8 * ((size_t)ldc * (n - 1) + m), "rocblas_dgemm C");
    return 0;
}

}  // extern "C"
