// A host-only stand-in for the parts of the HIP runtime (and rocBLAS) that
// libfsv calls, for checking the library on a machine without a GPU.  Test
// infrastructure.  Two builds use it:
//
//  - the host-check build (library compiled by hipcc): kernels do not run;
//  - the kernel-executing build (library compiled as plain C++ against
//    kexec/hip/hip_runtime.h): each launch runs the kernel on the host, one
//    fiber per work-item, one workgroup after another, with workgroup
//    barriers, wavefront exchanges and a dynamic LDS block of exactly the
//    launch's size (so AddressSanitizer checks LDS accesses too); the GEMM is
//    computed.
//
//  - "Device" memory is host memory from malloc, so AddressSanitizer sees every
//    allocation; each copy is checked against the allocation it names (device
//    side) or the pinned buffer it touches (host side) and then performed.
//  - Kernel launches are checked (a registered kernel, a launch shape the
//    hardware accepts, dynamic LDS within the limit set for that kernel) and
//    logged.
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

#include <sanitizer/common_interface_defs.h>
#include <sys/mman.h>
#include <ucontext.h>

#include <array>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

// work-item coordinates of the kernel-executing build (kexec/hip/hip_runtime.h)
struct fsv_cpu_idx {
    uint32_t x, y, z;
};
thread_local fsv_cpu_idx threadIdx, blockIdx;
thread_local dim3 blockDim, gridDim;

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
    int kind = 0;  // 0 launch, 1 copy, 2 GEMM (kernel-executing build)
    const void *fn = nullptr;
    dim3 grid, block;
    size_t shm = 0;
    void *dst = nullptr;
    const void *src = nullptr;
    size_t bytes = 0;
    hipMemcpyKind ck = hipMemcpyDefault;
    std::shared_ptr<void> ctx;  // kernel-executing build: the launch's bound arguments
    void (*run)(void *) = nullptr;
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
bool g_exec = false;  // kernel-executing build loaded

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

// The kernel-executing build has no registration: kernels are known by
// their host address.
std::map<const void *, Kernel>::iterator find_kernel(const void *fn, const char *what) {
    auto it = kernels().find(fn);
    if (it == kernels().end()) {
        if (!g_exec) die("%s: unregistered kernel %p", what, fn);
        it = kernels().emplace(fn, Kernel{}).first;
        char buf[32];
        std::snprintf(buf, sizeof buf, "kernel@%p", fn);
        it->second.name = buf;
    }
    return it;
}

void check_launch(const void *fn, dim3 g, dim3 b, size_t shm, const char *what) {
    auto it = find_kernel(fn, what);
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

// ---- kernel execution (kernel-executing build) ----
// One workgroup at a time, each work-item a fiber (ucontext) on the calling
// thread, run in lane order until it returns or waits.  A workgroup barrier
// releases when every work-item that has not returned waits at it (the
// hardware counts the waves still running); a wavefront exchange releases
// when every live lane of the wavefront waits at it.  Any other standstill
// is reported as a hang.  Deterministic: the same launch always runs the
// work-items in the same order.
enum FiberState { F_RUN, F_BARRIER, F_WAVE, F_DONE };

struct Fiber {
    ucontext_t ctx;
    void *stack = nullptr;
    void *fake = nullptr;  // AddressSanitizer's fake-stack handle while suspended
    int state = F_DONE;
};

constexpr size_t kFiberStack = 256 << 10;

struct Exec {
    std::vector<Fiber> fibers;
    ucontext_t sched;
    void *sched_fake = nullptr;
    const void *sched_bottom = nullptr;
    size_t sched_size = 0;
    int cur = -1, n = 0;
    void (*fn)(void *) = nullptr;
    void *arg = nullptr;
    dim3 bdim, gdim;
    fsv_cpu_idx bidx{0, 0, 0};
    void *dyn = nullptr;
    const char *name = "";
    std::vector<std::array<unsigned char, 64>> slot;  // one exchange slot per work-item
};

Exec g_x;
bool g_in_kernel = false;

void set_coords(int i) {
    blockDim = g_x.bdim;
    gridDim = g_x.gdim;
    blockIdx = g_x.bidx;
    threadIdx = fsv_cpu_idx{i % g_x.bdim.x, (i / g_x.bdim.x) % g_x.bdim.y, i / (g_x.bdim.x * g_x.bdim.y)};
}

// From a work-item back to the scheduler (state already set).
void yield_fiber(bool dying) {
    Fiber &f = g_x.fibers[g_x.cur];
    __sanitizer_start_switch_fiber(dying ? nullptr : &f.fake, g_x.sched_bottom, g_x.sched_size);
    swapcontext(&f.ctx, &g_x.sched);
    __sanitizer_finish_switch_fiber(f.fake, &g_x.sched_bottom, &g_x.sched_size);
    set_coords(g_x.cur);
}

void fiber_main() {
    __sanitizer_finish_switch_fiber(nullptr, &g_x.sched_bottom, &g_x.sched_size);
    set_coords(g_x.cur);
    g_x.fn(g_x.arg);
    g_x.fibers[g_x.cur].state = F_DONE;
    yield_fiber(true);
}

void resume(int i) {
    g_x.cur = i;
    Fiber &f = g_x.fibers[i];
    __sanitizer_start_switch_fiber(&g_x.sched_fake, f.stack, kFiberStack);
    swapcontext(&g_x.sched, &f.ctx);
    __sanitizer_finish_switch_fiber(g_x.sched_fake, nullptr, nullptr);
}

void run_block(const char *name) {
    const int n = g_x.n;
    while ((int)g_x.fibers.size() < n) {
        Fiber f;
        f.stack = mmap(nullptr, kFiberStack, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
        if (f.stack == MAP_FAILED) die("mmap of a work-item stack failed");
        g_x.fibers.push_back(f);
    }
    for (int i = 0; i < n; ++i) {
        Fiber &f = g_x.fibers[i];
        getcontext(&f.ctx);
        f.ctx.uc_stack.ss_sp = f.stack;
        f.ctx.uc_stack.ss_size = kFiberStack;
        f.ctx.uc_link = nullptr;
        makecontext(&f.ctx, fiber_main, 0);
        f.state = F_RUN;
        f.fake = nullptr;
    }
    g_x.slot.assign((size_t)((n + 63) / 64) * 64, std::array<unsigned char, 64>{});
    for (;;) {
        for (int i = 0; i < n; ++i)
            if (g_x.fibers[i].state == F_RUN) resume(i);
        bool all_done = true, released = false;
        for (int w = 0; w * 64 < n; ++w) {
            const int lo = w * 64, hi = std::min(n, lo + 64);
            bool any_wave = false, all_wave = true;
            for (int i = lo; i < hi; ++i) {
                const int st = g_x.fibers[i].state;
                if (st == F_DONE) continue;
                all_done = false;
                if (st == F_WAVE) any_wave = true;
                else all_wave = false;
            }
            if (any_wave && all_wave) {
                for (int i = lo; i < hi; ++i)
                    if (g_x.fibers[i].state == F_WAVE) g_x.fibers[i].state = F_RUN;
                released = true;
            }
        }
        if (all_done) break;
        if (released) continue;
        bool all_barrier = true;
        for (int i = 0; i < n; ++i) {
            const int st = g_x.fibers[i].state;
            if (st != F_DONE && st != F_BARRIER) all_barrier = false;
        }
        if (!all_barrier) {
            int nb = 0, nw = 0;
            for (int i = 0; i < n; ++i) {
                nb += g_x.fibers[i].state == F_BARRIER;
                nw += g_x.fibers[i].state == F_WAVE;
            }
            die("kernel %s hangs: block (%u, %u, %u), %d work-items at a workgroup barrier, %d at a wavefront "
                "exchange whose wavefront has lanes elsewhere", name, g_x.bidx.x, g_x.bidx.y, g_x.bidx.z, nb, nw);
        }
        for (int i = 0; i < n; ++i)
            if (g_x.fibers[i].state == F_BARRIER) g_x.fibers[i].state = F_RUN;
    }
}

struct ExecProfile {
    std::map<std::string, std::pair<double, long>> t;
    ~ExecProfile() {
        if (!std::getenv("FSV_STUB_PROFILE")) return;
        for (auto &kv : t)
            std::fprintf(stderr, "hip_stub: %9.3f s %6ld launches  %s\n", kv.second.first, kv.second.second,
                         kv.first.c_str());
    }
};
ExecProfile g_prof;

void exec_grid(void (*f)(void *), void *c, dim3 g, dim3 b, size_t shm, const char *name) {
    if (g_in_kernel) die("kernel launch from inside kernel %s", g_x.name);
    const auto t0 = std::chrono::steady_clock::now();
    g_in_kernel = true;
    g_x.fn = f;
    g_x.arg = c;
    g_x.gdim = g;
    g_x.bdim = b;
    g_x.n = (int)(b.x * b.y * b.z);
    g_x.name = name;
    for (uint32_t z = 0; z < g.z; ++z)
        for (uint32_t y = 0; y < g.y; ++y)
            for (uint32_t x = 0; x < g.x; ++x) {
                g_x.bidx = fsv_cpu_idx{x, y, z};
                g_x.dyn = std::malloc(shm ? shm : 1);
                std::memset(g_x.dyn, 0xFF, shm ? shm : 1);  // LDS starts undefined: NaN pattern
                run_block(name);
                std::free(g_x.dyn);
                g_x.dyn = nullptr;
            }
    g_in_kernel = false;
    auto &e = g_prof.t[name];
    e.first += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    e.second += 1;
}

std::map<void *, hipStream_t> &blas_stream() { static std::map<void *, hipStream_t> m; return m; }

struct Gemm {
    int m, n, k;
    double alpha;
    const double *A;
    int lda;
    const double *B;
    int ldb;
    double beta;
    double *C;
    int ldc;
};

void run_gemm(void *p) {
    const Gemm &g = *(const Gemm *)p;
    std::vector<double> col((size_t)g.m);
    for (int j = 0; j < g.n; ++j) {
        for (int i = 0; i < g.m; ++i) col[i] = 0.0;
        for (int q = 0; q < g.k; ++q) {
            const double bv = g.B[(size_t)j * g.ldb + q];
            for (int i = 0; i < g.m; ++i) col[i] += g.A[(size_t)q * g.lda + i] * bv;
        }
        for (int i = 0; i < g.m; ++i) {
            double &cv = g.C[(size_t)j * g.ldc + i];
            cv = g.alpha * col[i] + (g.beta == 0.0 ? 0.0 : g.beta * cv);
        }
    }
}

struct CallCfg {
    dim3 g, b;
    size_t shm;
    hipStream_t st;
};
thread_local std::vector<CallCfg> g_cfg;

}  // namespace

// ---- entry points of the kernel-executing build (C++ linkage) ----
void fsv_cpu_enable() {
    std::lock_guard<std::mutex> lk(g_mu);
    g_exec = true;
}

void *fsv_cpu_dyn_lds() { return g_x.dyn; }

void fsv_cpu_syncthreads() {
    g_x.fibers[g_x.cur].state = F_BARRIER;
    yield_fiber(false);
}

static void wave_wait() {
    g_x.fibers[g_x.cur].state = F_WAVE;
    yield_fiber(false);
}

void fsv_cpu_wave_exchange(const void *mine, void *out, size_t n, int src) {
    const int me = g_x.cur, base = me & ~63;
    if (n > 64 || src < 0 || src > 63) die("wavefront exchange of %zu bytes from lane %d", n, src);
    std::memcpy(g_x.slot[me].data(), mine, n);
    wave_wait();
    std::memcpy(out, g_x.slot[base + src].data(), n);
    wave_wait();
}

void fsv_cpu_mfma_f64_16x16x4(double a, double b, const double *c, double *d) {
    const int me = g_x.cur, base = me & ~63, l = me & 63;
    const double mine[2] = {a, b};
    std::memcpy(g_x.slot[me].data(), mine, sizeof mine);
    wave_wait();
    auto op = [&](int lane, int which) {
        double v[2];
        std::memcpy(v, g_x.slot[base + lane].data(), sizeof v);
        return v[which];
    };
    for (int r = 0; r < 4; ++r) {
        const int row = 4 * r + l / 16, col = l % 16;
        double acc = c[r];
        for (int k = 0; k < 4; ++k) acc += op(row + 16 * k, 0) * op(col + 16 * k, 1);
        d[r] = acc;
    }
    wave_wait();
}

const void *fsv_cpu_symbol(const void *p, size_t n) {
    std::lock_guard<std::mutex> lk(g_mu);
    symbols()[p] = "symbol";
    dev_allocs()[(uintptr_t)p] = n;
    return p;
}

hipError_t fsv_cpu_launch(const void *fn, const char *name, dim3 g, dim3 b, size_t shm, hipStream_t st,
                          hipEvent_t e0, hipEvent_t e1, void (*run)(void *), void *ctx, void (*del)(void *),
                          void *(*)(void *)) {
    std::shared_ptr<void> c(ctx, del);
    std::string nm;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_exec = true;
        if (e0) check_event(e0, "kernel launch start event");
        if (e1) check_event(e1, "kernel launch stop event");
        auto it = find_kernel(fn, name);
        if (it->second.name.rfind("kernel@", 0) == 0) it->second.name = name;
        nm = it->second.name;
        check_launch(fn, g, b, shm, name);
        Stream *s = stream_of(st, name);
        if (s && s->capturing) {
            Node n;
            n.kind = 0;
            n.fn = fn;
            n.grid = g;
            n.block = b;
            n.shm = shm;
            n.ctx = c;
            n.run = run;
            s->rec.push_back(n);
            return hipSuccess;
        }
        ++g_launches;
    }
    exec_grid(run, c.get(), g, b, shm, nm.c_str());
    return hipSuccess;
}

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
    auto it = find_kernel(fn, "hipFuncSetAttribute");
    if (attr == hipFuncAttributeMaxDynamicSharedMemorySize) {
        if (value < 0 || value > 163840) return hipErrorInvalidValue;
        it->second.max_dyn = value;
    }
    return hipSuccess;
}
hipError_t hipFuncGetAttributes(hipFuncAttributes *a, const void *fn) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = find_kernel(fn, "hipFuncGetAttributes");
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
    void *q = nullptr;  // device allocations are at least 256-byte aligned
    if (posix_memalign(&q, 256, n ? n : 1) != 0) return hipErrorOutOfMemory;
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
// Work runs at launch here, so a stream is idle, unless FSV_STUB_BUSY_STREAMS
// is set: then every query reports pending work and the callers' fences run.
hipError_t hipStreamQuery(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    Stream *x = stream_of(s, "hipStreamQuery");
    if (x && x->capturing) return hipErrorStreamCaptureUnsupported;
    static const bool busy = std::getenv("FSV_STUB_BUSY_STREAMS") != nullptr;
    return busy ? hipErrorNotReady : hipSuccess;
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
            if (n.run) exec_grid(n.run, n.ctx.get(), n.grid, n.block, n.shm, kernels()[n.fn].name.c_str());
        } else if (n.kind == 2) {
            run_gemm(n.ctx.get());
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
    blas_stream()[*h] = nullptr;
    return 0;
}
int rocblas_destroy_handle(rocblas_handle_t h) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!blas_handles().erase(h)) die("rocblas_destroy_handle of an unknown handle");
    blas_stream().erase(h);
    std::free(h);
    return 0;
}
int rocblas_set_stream(rocblas_handle_t h, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!blas_handles().count(h)) die("rocblas_set_stream on an unknown handle");
    stream_of(s, "rocblas_set_stream");
    blas_stream()[h] = s;
    return 0;
}
int rocblas_set_atomics_mode(rocblas_handle_t h, int) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!blas_handles().count(h)) die("rocblas_set_atomics_mode on an unknown handle");
    return 0;
}
// Column-major C (m x n, ldc) = alpha op(A) op(B) + beta C; only untransposed
// operands are used by the library.  The kernel-executing build computes it
// (recorded into a graph when the handle's stream is capturing).
int rocblas_dgemm(rocblas_handle_t h, int ta, int tb, int m, int n, int k, const double *alpha, const double *A,
                  int lda, const double *B, int ldb, const double *beta, double *C, int ldc) {
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
    if (!g_exec || !m || !n) return 0;
    auto *g = new Gemm{m, n, k, *alpha, A, lda, B, ldb, *beta, C, ldc};
    std::shared_ptr<void> ctx(g, [](void *p) { delete (Gemm *)p; });
    Stream *s = stream_of(blas_stream()[h], "rocblas_dgemm");
    if (s && s->capturing) {
        Node nd;
        nd.kind = 2;
        nd.ctx = ctx;
        nd.run = &run_gemm;
        s->rec.push_back(nd);
        return 0;
    }
    run_gemm(g);
    return 0;
}

}  // extern "C"
