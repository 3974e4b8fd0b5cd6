// Host build of the HIP subset the library's kernels and host code use, for CPU
// tests of the kernels' index arithmetic: every kernel runs on the CPU, each block as
// cooperative fibers (one per work-item, switched at __syncthreads), blocks spread
// over OS threads.  Device memory is host memory of the exact requested size and
// each block's dynamic LDS is a heap buffer of exactly the launch's size, so an
// AddressSanitizer build reports any out-of-bounds access of a kernel.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>
#include <atomic>
#include <functional>
#include <mutex>
#include <algorithm>
#include <sanitizer/common_interface_defs.h>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __align__(n) __attribute__((aligned(n)))
#define __launch_bounds__(...)
#define __shared__ static thread_local

struct dim3 {
    unsigned x = 1, y = 1, z = 1;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct uint4 { unsigned x, y, z, w; };
struct uint2 { unsigned x, y; };
struct int2 { int x, y; };
struct double2 { double x, y; };
struct double4 { double x, y, z, w; };
struct float2 { float x, y; };
inline float2 make_float2(float a, float b) { return {a, b}; }
struct float4 { float x, y, z, w; };
inline float4 make_float4(float a, float b, float c, float d) { return {a, b, c, d}; }
inline unsigned __brev(unsigned v) {
    unsigned r = 0;
    for (int i = 0; i < 32; ++i) r |= ((v >> i) & 1u) << (31 - i);
    return r;
}
inline uint4 make_uint4(unsigned a, unsigned b, unsigned c, unsigned d) { return {a, b, c, d}; }
inline uint2 make_uint2(unsigned a, unsigned b) { return {a, b}; }
inline int2 make_int2(int a, int b) { return {a, b}; }
inline double2 make_double2(double a, double b) { return {a, b}; }
inline double4 make_double4(double a, double b, double c, double d) { return {a, b, c, d}; }

inline thread_local dim3 threadIdx, blockIdx, blockDim, gridDim;


template <class A, class B> inline auto min(A a, B b) { return a < b ? a : b; }
template <class A, class B> inline auto max(A a, B b) { return a < b ? b : a; }
inline float __fmul_rn(float a, float b) { return a * b; }
inline int __mul24(int a, int b) { return a * b; }
inline float __uint_as_float(unsigned u) { float f; std::memcpy(&f, &u, 4); return f; }
inline unsigned __float_as_uint(float f) { unsigned u; std::memcpy(&u, &f, 4); return u; }
inline double emu_fract(double x) { return x - std::floor(x); }
inline float emu_med3(float a, float b, float c) { return std::fmax(std::fmin(a, b), std::fmin(std::fmax(a, b), c)); }
#define __builtin_amdgcn_fract(x) emu_fract(x)
inline float emu_fractf(float x) { return x - std::floor(x); }
#define __builtin_amdgcn_fractf(x) emu_fractf(x)
#define __builtin_amdgcn_fmed3f(a, b, c) emu_med3(a, b, c)
#define __builtin_amdgcn_readfirstlane(x) (x)
// memory-counter waits: every emulated access has completed already, but after a wait
// the lanes of a wave read what the other lanes of that wave copied asynchronously (the
// device issues one copy instruction for all 64 lanes), so the wait synchronises the
// lanes: here all the block's work-items, a stronger order than the device's (every use
// is reached by the whole block)
#define __builtin_amdgcn_s_waitcnt(x) __syncthreads()
// v_rcp_f32 (1 ulp on the device; the correctly rounded quotient here)
inline float emu_rcpf(float x) { return 1.0f / x; }
#define __builtin_amdgcn_rcpf(x) emu_rcpf(x)
// v_dot2c_f32_f16 / v_dot2c_f32_bf16: the two 16-bit products are exact, their sum with
// the FP32 accumulator is rounded once
template <class V> inline float emu_fdot2(V a, V b, float c) {
    return (float)((double)(float)a[0] * (double)(float)b[0] + (double)(float)a[1] * (double)(float)b[1] +
                   (double)c);
}
#define __builtin_amdgcn_fdot2(a, b, c, clamp) emu_fdot2(a, b, c)
#define __builtin_amdgcn_fdot2_f32_bf16(a, b, c, clamp) emu_fdot2(a, b, c)
template <class T> inline T atomicAdd(T *p, T v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2, hipErrorLaunchFailure = 3,
       hipErrorInvalidSymbol = 4 };
typedef void *hipStream_t;
typedef void *hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
enum hipStreamCaptureStatus { hipStreamCaptureStatusNone = 0, hipStreamCaptureStatusActive = 1 };
struct hipDeviceProp_t { int multiProcessorCount = 4; };

namespace emu {
inline hipError_t &last_error() { static hipError_t e = hipSuccess; return e; }
inline size_t &lds_limit() { static size_t l = 160 * 1024; return l; }
inline std::atomic<long> &launches() { static std::atomic<long> n{0}; return n; }

// One block runs as cooperative fibers (one per work-item) on one OS thread; blocks are
// spread over OS threads.  __syncthreads() switches back to the block's scheduler,
// which resumes every live fiber once per barrier round.
extern "C" void emu_ctx_switch(void **from_sp, void *to_sp);
asm(R"(
.text
.weak emu_ctx_switch
.type emu_ctx_switch,@function
emu_ctx_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
)");
struct Fiber { void *sp; char *stack; bool done; };
struct Sched {
    void *sp = nullptr;
    std::vector<Fiber> fibers;
    int cur = -1;
    char *lds = nullptr;
    std::function<void()> body;
    const void *sched_bottom = nullptr;
    size_t sched_size = 0;
};
inline thread_local Sched *tl_sched = nullptr;
inline void *dyn_lds() { return tl_sched->lds; }
constexpr size_t kStack = 64 * 1024;

inline void fiber_yield(bool dying) {
    Sched *s = tl_sched;
    Fiber &f = s->fibers[s->cur];
    void *fake = nullptr;
    __sanitizer_start_switch_fiber(dying ? nullptr : &fake, s->sched_bottom, s->sched_size);
    emu_ctx_switch(&f.sp, s->sp);
    __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
}
inline void fiber_entry() {
    Sched *s = tl_sched;
    __sanitizer_finish_switch_fiber(nullptr, &s->sched_bottom, &s->sched_size);
    s->body();
    s->fibers[s->cur].done = true;
    fiber_yield(true);
}

// Stream capture: launches on a capturing stream are recorded (with the bytes of
// their arguments) instead of run, and replay_graph() runs a recorded sequence later,
// as a graph replay would.  An allocation while any stream captures is counted.
struct Recorded {
    hipStream_t stream;
    std::vector<unsigned char> args;
    std::function<void()> run;
};
struct Capture {
    std::mutex mu;
    std::vector<hipStream_t> streams;
    std::vector<Recorded> launches;
    long allocs_while_capturing = 0;
};
inline Capture &capture() { static Capture c; return c; }
inline bool capturing(hipStream_t s) {
    std::lock_guard<std::mutex> lk(capture().mu);
    for (hipStream_t c : capture().streams)
        if (c == s) return true;
    return false;
}
inline void begin_capture(hipStream_t s) {
    std::lock_guard<std::mutex> lk(capture().mu);
    capture().streams.push_back(s);
}
// Ends the capture of s and returns its recorded launches (the "graph").
inline std::vector<Recorded> end_capture(hipStream_t s) {
    std::lock_guard<std::mutex> lk(capture().mu);
    auto &v = capture().streams;
    v.erase(std::remove(v.begin(), v.end(), s), v.end());
    std::vector<Recorded> out, keep;
    for (auto &r : capture().launches) (r.stream == s ? out : keep).push_back(std::move(r));
    capture().launches.swap(keep);
    return out;
}
inline void replay_graph(const std::vector<Recorded> &g) {
    for (const Recorded &r : g) r.run();
}
template <class T> inline void append_bytes(std::vector<unsigned char> &v, const T &x) {
    const unsigned char *p = reinterpret_cast<const unsigned char *>(&x);
    v.insert(v.end(), p, p + sizeof(T));
}

template <class K, class... A>
void launch_now(K kernel, dim3 grid, dim3 block, size_t lds, A... args);

template <class K, class... A>
void launch(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t stream, A... args) {
    if (capturing(stream)) {
        Recorded r;
        r.stream = stream;
        (append_bytes(r.args, args), ...);
        r.run = [=] { launch_now(kernel, grid, block, lds, args...); };
        std::lock_guard<std::mutex> lk(capture().mu);
        capture().launches.push_back(std::move(r));
        return;
    }
    launch_now(kernel, grid, block, lds, args...);
}

template <class K, class... A>
void launch_now(K kernel, dim3 grid, dim3 block, size_t lds, A... args) {
    ++launches();
    const int nt = (int)(block.x * block.y * block.z);
    const long nb = (long)grid.x * grid.y * grid.z;
    if (nt <= 0 || nt > 1024 || lds > lds_limit()) {
        std::fprintf(stderr, "[emu] bad launch: %d threads, %zu bytes LDS\n", nt, lds);
        last_error() = hipErrorInvalidValue;
        return;
    }
    if (nb == 0) return;
    std::atomic<long> next{0};
    const int workers = std::max(1, std::min<int>((int)std::thread::hardware_concurrency(), (int)std::min<long>(nb, 64)));
    auto worker = [&] {
        Sched s;
        tl_sched = &s;
        s.fibers.resize(nt);
        // fiber stack sets are recycled across launches
        static std::mutex mu;
        static std::vector<std::vector<char *>> free_sets;
        std::vector<char *> stacks;
        {
            std::lock_guard<std::mutex> lk(mu);
            if (!free_sets.empty()) { stacks = std::move(free_sets.back()); free_sets.pop_back(); }
        }
        while ((int)stacks.size() < nt) stacks.push_back(new char[kStack]);
        for (int t = 0; t < nt; ++t) s.fibers[t].stack = stacks[t];
        s.lds = lds ? new char[lds] : nullptr;     // exact size, reused by this worker's blocks
        blockDim = block;
        gridDim = grid;
        for (;;) {
            const long b = next.fetch_add(1);
            if (b >= nb) break;
            blockIdx = dim3(b % grid.x, (b / grid.x) % grid.y, b / ((long)grid.x * grid.y));
            if (lds) std::memset(s.lds, 0xA5, lds);   // garbage, like real LDS
            s.body = [&] { kernel(args...); };
            for (int t = 0; t < nt; ++t) {
                Fiber &f = s.fibers[t];
                f.done = false;
                uintptr_t top = ((uintptr_t)(f.stack + kStack)) & ~(uintptr_t)15;
                void **sp = (void **)(top - 8);
                *--sp = (void *)&fiber_entry;             // returned to by the first switch
                for (int r = 0; r < 6; ++r) *--sp = nullptr; // rbp rbx r12-r15
                f.sp = sp;
            }
            for (;;) {          // barrier rounds
                bool any = false;
                for (int t = 0; t < nt; ++t) {
                    Fiber &f = s.fibers[t];
                    if (f.done) continue;
                    any = true;
                    s.cur = t;
                    threadIdx = dim3(t % block.x, (t / block.x) % block.y, t / (block.x * block.y));
                    void *fake = nullptr;
                    __sanitizer_start_switch_fiber(&fake, f.stack, kStack);
                    emu_ctx_switch(&s.sp, f.sp);
                    __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
                }
                if (!any) break;
            }
        }
        delete[] s.lds;
        {
            std::lock_guard<std::mutex> lk(mu);
            free_sets.push_back(std::move(stacks));
        }
        tl_sched = nullptr;
    };
    std::vector<std::thread> pool;
    for (int w = 0; w < workers; ++w) pool.emplace_back(worker);
    for (auto &th : pool) th.join();
}
}  // namespace emu

inline void __syncthreads() { emu::fiber_yield(false); }

#define hipLaunchKernelGGL(kernel, grid, block, lds, stream, ...) \
    emu::launch(kernel, dim3(grid), dim3(block), (size_t)(lds), (hipStream_t)(stream), __VA_ARGS__)

inline hipError_t hipGetLastError() { hipError_t e = emu::last_error(); emu::last_error() = hipSuccess; return e; }
inline hipError_t hipMalloc(void **p, size_t n) {
    {
        std::lock_guard<std::mutex> lk(emu::capture().mu);
        if (!emu::capture().streams.empty()) ++emu::capture().allocs_while_capturing;
    }
    *p = nullptr;
    if (posix_memalign(p, 256, n ? n : 1) != 0) return hipErrorOutOfMemory;
    return hipSuccess;
}
template <class T> inline hipError_t hipMalloc(T **p, size_t n) { return hipMalloc((void **)p, n); }
inline hipError_t hipFree(void *p) { std::free(p); return hipSuccess; }
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipMemset(void *d, int v, size_t n) { std::memset(d, v, n); return hipSuccess; }
inline hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
// a __device__ variable is an ordinary host object here; its address is the symbol's
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void **p, const void *sym) {
    *p = const_cast<void *>(sym);
    return hipSuccess;
}
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int) { *p = hipDeviceProp_t{}; return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipStreamIsCapturing(hipStream_t st, hipStreamCaptureStatus *s) {
    *s = emu::capturing(st) ? hipStreamCaptureStatusActive : hipStreamCaptureStatusNone;
    return hipSuccess;
}
inline hipError_t hipEventCreate(hipEvent_t *e) { *e = new int(0); return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete (int *)e; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t = nullptr) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) { *ms = 1.0f; return hipSuccess; }
template <class K>
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, K, int, size_t) { *n = 1; return hipSuccess; }
