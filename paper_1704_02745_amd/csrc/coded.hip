// Coded operator coefficients for the 40-byte pass (FP32).
//
// With the two-point dielectric model of Eq. 3 the coupling arrays hold a
// handful of distinct values (eps_in, eps_out and their harmonic mean, over
// h^2, and zero across the box faces), and the diagonal a few dozen (sums of
// six such couplings plus one of two salt terms). When the four FP32 operator
// arrays together hold at most 256 distinct values, each node's four
// coefficients are stored as one 4-byte word of dictionary codes (byte 0: cx,
// 1: cy, 2: cz, 3: d), and the pass reads 4 bytes of operator per node
// instead of 16. Decoding returns the FP32 values themselves, so coded and
// uncoded passes compute identical iterates.
//
// Codes are the ranks of the values' bit patterns in ascending order, so they
// do not depend on the order in which threads meet the values. The dictionary
// always holds +0.0, which has the smallest pattern and therefore code 0: the
// zero words the pass uses for absent neighbours decode to 0, as in the
// uncoded pass.
#include "pb_internal.hpp"
#include "solver.hpp"

namespace pb {

namespace {

constexpr int kHashSlots = 4096;            // open addressing, linear probing
constexpr uint32_t kEmpty = 0xFFFFFFFFu;    // a NaN pattern; coefficients are finite
constexpr int kMaxCodes = kCodedTableSize;  // 256

__device__ __forceinline__ uint32_t hash_slot(uint32_t v) { return (v * 2654435761u) >> 20; }   // 12 bits

// Every value of cx, cy, cz, d (and +0.0) into the hash set, in two levels:
// each workgroup first collects the distinct values of its range in an LDS
// set, then merges those few into the device set. Slots are read with
// relaxed atomic loads (workgroup scope in LDS, agent scope in the device
// set) and only ever go from empty to a value, so a load that sees a value
// sees its final one; a load that still sees an empty slot is settled by the
// compare-and-swap that follows: when another thread filled the slot first,
// the swap fails and returns that value, which is compared like a load's. A
// workgroup that meets more than kMaxCodes distinct values raises the device
// count past kMaxCodes and stops (the dictionary cannot hold them).
constexpr int kLocalSlots = 1024;

__device__ __forceinline__ bool set_insert(uint32_t* keys, int nslots, uint32_t v, int* count, bool lds) {
    uint32_t s = hash_slot(v) & (uint32_t)(nslots - 1);
    for (int probe = 0; probe < nslots; ++probe) {
        const uint32_t cur = lds ? __hip_atomic_load(keys + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)
                                 : __hip_atomic_load(keys + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cur == v) return true;
        if (cur == kEmpty) {
            const uint32_t old = atomicCAS(keys + s, kEmpty, v);
            if (old == kEmpty) {
                atomicAdd(count, 1);
                return true;
            }
            if (old == v) return true;
        }
        s = (s + 1) & (uint32_t)(nslots - 1);
    }
    return false;   // the set is full
}

__global__ __launch_bounds__(256) void k_dict_insert(const float* __restrict__ cx, const float* __restrict__ cy,
                                                     const float* __restrict__ cz, const float* __restrict__ d,
                                                     int64_t npad, uint32_t* keys, int* count) {
    __shared__ uint32_t lk[kLocalSlots];
    __shared__ int lcount;
    for (int i = threadIdx.x; i < kLocalSlots; i += blockDim.x) lk[i] = kEmpty;
    if (threadIdx.x == 0) lcount = 0;
    __syncthreads();
    bool full = blockIdx.x == 0 && threadIdx.x == 0 && !set_insert(lk, kLocalSlots, 0u, &lcount, true);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npad && !full;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float v[4] = {cx[i], cy[i], cz[i], d[i]};
#pragma unroll
        for (int a = 0; a < 4; ++a) full = full || !set_insert(lk, kLocalSlots, __float_as_uint(v[a]), &lcount, true);
        full = full || __hip_atomic_load(&lcount, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) > kMaxCodes;
    }
    __syncthreads();
    if (lcount > kMaxCodes) {
        if (threadIdx.x == 0) atomicAdd(count, kHashSlots);   // more values than the dictionary holds
        return;
    }
    for (int i = threadIdx.x; i < kLocalSlots; i += blockDim.x) {
        const uint32_t v = lk[i];
        if (v != kEmpty) (void)set_insert(keys, kHashSlots, v, count, false);
    }
}

// One workgroup: rank the distinct values, write the dictionary (code ->
// value) and each occupied slot's code; ok = 1 when the values fit.
__global__ __launch_bounds__(1024) void k_dict_rank(const uint32_t* __restrict__ keys, const int* __restrict__ count,
                                                    int* __restrict__ slot_code, float* __restrict__ table,
                                                    int* __restrict__ ok) {
    __shared__ uint32_t vals[kMaxCodes];
    __shared__ int n;
    const int c = *count;
    if (c > kMaxCodes) {
        if (threadIdx.x == 0) *ok = 0;
        return;
    }
    if (threadIdx.x == 0) n = 0;
    __syncthreads();
    for (int s = threadIdx.x; s < kHashSlots; s += blockDim.x) {
        const uint32_t v = keys[s];
        if (v != kEmpty) vals[atomicAdd(&n, 1)] = v;
    }
    __syncthreads();
    const int nv = n;
    for (int s = threadIdx.x; s < kHashSlots; s += blockDim.x) {
        const uint32_t v = keys[s];
        int rank = -1;
        if (v != kEmpty) {
            rank = 0;
            for (int j = 0; j < nv; ++j) rank += vals[j] < v ? 1 : 0;
            table[rank] = __uint_as_float(v);
        }
        slot_code[s] = rank;
    }
    for (int j = nv + (int)threadIdx.x; j < kMaxCodes; j += blockDim.x) table[j] = 0.0f;
    if (threadIdx.x == 0) *ok = nv <= kMaxCodes && nv == c ? 1 : 0;
}

__device__ __forceinline__ uint32_t code_of(const uint32_t* __restrict__ k, const int* __restrict__ sc, float f) {
    const uint32_t v = __float_as_uint(f);
    uint32_t s = hash_slot(v);
    for (int probe = 0; probe < kHashSlots; ++probe) {
        if (k[s] == v) return (uint32_t)sc[s];
        s = (s + 1) & (kHashSlots - 1);
    }
    return 0u;   // not reached: every value was inserted
}

// One code word per padded position; the hash set is staged in LDS.
__global__ __launch_bounds__(256) void k_dict_encode(const float* __restrict__ cx, const float* __restrict__ cy,
                                                     const float* __restrict__ cz, const float* __restrict__ d,
                                                     int64_t npad, const uint32_t* __restrict__ keys,
                                                     const int* __restrict__ slot_code, uint32_t* __restrict__ codes,
                                                     const int* __restrict__ fit) {
    if (fit && *fit != 1) return;   // the values did not fit: the codes are not used
    __shared__ uint32_t k[kHashSlots];
    __shared__ int sc[kHashSlots];
    for (int s = threadIdx.x; s < kHashSlots; s += blockDim.x) {
        k[s] = keys[s];
        sc[s] = slot_code[s];
    }
    __syncthreads();
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t w = code_of(k, sc, cx[t]) | (code_of(k, sc, cy[t]) << 8) | (code_of(k, sc, cz[t]) << 16) |
                           (code_of(k, sc, d[t]) << 24);
        codes[t] = w;
    }
}

unsigned grid_for_n(int64_t n, int bs, int64_t cap) {
    const int64_t b = (n + bs - 1) / bs;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

}  // namespace

size_t coded_scratch_bytes() {
    return sizeof(uint32_t) * kHashSlots + sizeof(int) * kHashSlots + sizeof(float) * kMaxCodes + 2 * sizeof(int);
}

namespace {
struct DictWs {
    uint32_t* keys;
    int* slot_code;
    float* tab;
    int* count;
    int* ok;
};
DictWs dict_ws(const void* scratch) {
    char* b = (char*)scratch;
    DictWs w;
    w.keys = (uint32_t*)b;
    w.slot_code = (int*)(b + sizeof(uint32_t) * kHashSlots);
    w.tab = (float*)(b + (sizeof(uint32_t) + sizeof(int)) * kHashSlots);
    w.count = (int*)(w.tab + kMaxCodes);
    w.ok = w.count + 1;
    return w;
}
}  // namespace

const float* dictionary_table(const void* scratch) { return dict_ws(scratch).tab; }

pb_status enqueue_dictionary(const Op<float>& op, int64_t npad, void* scratch, int* ok_out, hipStream_t st) {
    const DictWs w = dict_ws(scratch);
    pb_status e = launch_fill<int>((int*)w.keys, kHashSlots, -1, st);
    if (e != PB_OK) return e;
    e = launch_fill<int>(w.count, 2, 0, st);
    if (e != PB_OK) return e;
    hipLaunchKernelGGL(k_dict_insert, dim3(grid_for_n(npad, 256 * 8, 2048)), dim3(256), 0, st, op.cx, op.cy,
                       op.cz, op.d, npad, w.keys, w.count);
    hipLaunchKernelGGL(k_dict_rank, dim3(1), dim3(1024), 0, st, (const uint32_t*)w.keys, (const int*)w.count,
                       w.slot_code, w.tab, ok_out ? ok_out : w.ok);
    PB_HIP(hipGetLastError());
    return PB_OK;
}

pb_status enqueue_encode(const Op<float>& op, int64_t npad, const void* scratch, uint32_t* codes, hipStream_t st,
                         const int* fit) {
    const DictWs w = dict_ws(scratch);
    hipLaunchKernelGGL(k_dict_encode, dim3(grid_for_n(npad, 256, 4096)), dim3(256), 0, st, op.cx, op.cy, op.cz,
                       op.d, npad, (const uint32_t*)w.keys, (const int*)w.slot_code, codes, fit);
    PB_HIP(hipGetLastError());
    return PB_OK;
}

pb_status build_codes(const Op<float>& op, int64_t npad, void* scratch, uint32_t* codes, hipStream_t st,
                      bool& fits, const float** table) {
    fits = false;
    const DictWs w = dict_ws(scratch);
    pb_status e = enqueue_dictionary(op, npad, scratch, nullptr, st);
    if (e != PB_OK) return e;
    int hok = 0;
    PB_HIP(hipMemcpyAsync(&hok, w.ok, sizeof(int), hipMemcpyDeviceToHost, st));
    PB_HIP(hipStreamSynchronize(st));
    if (!hok) return PB_OK;
    e = enqueue_encode(op, npad, scratch, codes, st);
    if (e != PB_OK) return e;
    fits = true;
    *table = w.tab;
    return PB_OK;
}

}  // namespace pb
