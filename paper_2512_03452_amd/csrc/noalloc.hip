// Device-resident scratch of the allocation-free deposit entry point
// (sipf_deposit_noalloc in api.cpp): a file-scope device array, looked up
// once per device, and the kernel that writes the call's descriptors and
// tables into it.  Nothing here allocates.
#include <mutex>

#include "internal.h"

namespace sipf {

// Room for two particle buffer sets of NOALLOC_MAX_P FP64 particles
// (2 x (3 x 8 + 4) bytes each) plus the sort's counts, cursors, item lists
// and descriptors.  Each GPU the library runs on holds its own copy until the
// process ends.
constexpr size_t NOALLOC_BYTES = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

// Device address of the current device's scratch array.  The array's name is
// a host-side stand-in in host code; its address on each device comes from
// hipGetSymbolAddress, called once per device with that device current.
hipError_t noalloc_scratch(void** out, size_t* bytes) {
    *out = nullptr;
    *bytes = 0;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    *bytes = NOALLOC_BYTES;
    return hipSuccess;
}

// One call's set-up in scratch: the two particle descriptors, the sort chunk
// table and item segment offset of a single instance, and zeroed tile counts,
// item header, error flag and step counter (a kernel, so that nothing is
// recorded as a memset).
template <typename T>
__global__ void k_noalloc_setup(PartDesc<T> d0, PartDesc<T> d1, PartDesc<T>* pd, SortChunk* chunks, int nchunks,
                                int sort_chunk_size, int* seg_off, uint32_t* counts, int nkeys, int* nitems,
                                int* err, uint32_t* step) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int stride = gridDim.x * blockDim.x;
    if (t == 0) {
        pd[0] = d0;
        pd[1] = d1;
        seg_off[0] = 0;
        nitems[0] = 0;
        nitems[1] = 0;
        *err = 0;
        *step = 0u;
    }
    for (int i = t; i < nchunks; i += stride) chunks[i] = SortChunk{(int64_t)i * sort_chunk_size, 0, 0};
    for (int i = t; i < nkeys; i += stride) counts[i] = 0u;
}

template <typename T>
hipError_t launch_noalloc_setup(const PartDesc<T>& d0, const PartDesc<T>& d1, PartDesc<T>* pd, SortChunk* chunks,
                                int nchunks, int sort_chunk_size, int* seg_off, uint32_t* counts, int nkeys,
                                int* nitems, int* err, uint32_t* step, hipStream_t s) {
    hipLaunchKernelGGL((k_noalloc_setup<T>), dim3(16), dim3(256), 0, s, d0, d1, pd, chunks, nchunks, sort_chunk_size,
                       seg_off, counts, nkeys, nitems, err, step);
    return hipGetLastError();
}

template hipError_t launch_noalloc_setup<float>(const PartDesc<float>&, const PartDesc<float>&, PartDesc<float>*,
                                                SortChunk*, int, int, int*, uint32_t*, int, int*, int*, uint32_t*,
                                                hipStream_t);
template hipError_t launch_noalloc_setup<double>(const PartDesc<double>&, const PartDesc<double>&,
                                                 PartDesc<double>*, SortChunk*, int, int, int*, uint32_t*, int, int*,
                                                 int*, uint32_t*, hipStream_t);

}  // namespace sipf
