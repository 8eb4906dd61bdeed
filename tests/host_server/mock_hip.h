// Test infrastructure, never linked into the library: a host-only stand-in
// for the HIP runtime calls the library's host code makes (streams that run
// their work asynchronously on worker threads, events, kernel launches,
// explicitly built graphs, device allocations), so that the real solve
// driver, the C ABI and the server run on the CPU under AddressSanitizer,
// UndefinedBehaviorSanitizer and ThreadSanitizer.
//
// "Device" memory is reserved address space (mmap, never fully touched);
// every allocation is recorded, and each emulated kernel checks that every
// range it would read or write lies inside one live allocation (else the
// process aborts with a message naming the kernel and the range).
#pragma once

#include <cstddef>
#include <cstdint>
#include <functional>
#include <vector>

#include <hip/hip_runtime_api.h>

namespace mock {

// Checks that [p, p + n) lies inside one live device allocation; `what`
// names the access in the abort message.  Touches the first and the last
// byte of the range (write = true: writes them).
void check_range(const void* p, size_t n, const char* what, bool write);

// Enqueues host work on a stream (the emulation of a kernel).
void submit(hipStream_t st, std::function<void()> fn);

// Registers an emulated kernel: `fn` is the address the library passes to
// hipLaunchKernel / hipGraphAddKernelNode, `sizes` the byte size of each
// argument, `emu` runs on the stream with pointers to copies of the values.
void register_kernel(const void* fn, std::vector<size_t> sizes, std::function<void(void**)> emu);

// Emulated GPU time per algorithmic flop (seconds), for the contraction.
extern double seconds_per_flop;

// Counters of the emulation (for the drivers' reports).
struct Counters {
    uint64_t launches, graph_launches, graph_nodes, allocs, frees;
};
Counters counters();

}  // namespace mock
