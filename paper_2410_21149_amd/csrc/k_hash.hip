// Hash-table stress insertion (the hash-table stress test of Sec. IV): n
// distinct keys go into an open-addressing table with linear probing that
// the caller owns -- the table kind, home slot (SplitMix64 finaliser of the
// key, masked to the capacity), probe order and compare-and-swap that map
// block coordinates to block indices in every submap (Sec. III-B).
//
//   k_hash_stress  one lane per key: the bounded insertion, then the
//                  workgroup's longest probe, probe sum and failures are
//                  reduced in LDS and added to the three counters with one
//                  atomic each.
//
// Memory traffic per key: the key (8 B) in, one 8-byte compare-and-swap per
// probed slot, the value (4 B) out.  The slots are random, so every probe
// touches its own 64-byte line of the key array (and of the value array for
// the store): the kernel is bound by the rate of random atomics to HBM, not
// by streamed bytes.
#include "covox_impl.h"

namespace covox {
namespace {

constexpr int kHashThreads = 256;

__global__ __launch_bounds__(kHashThreads) void k_hash_stress(uint64_t *tkeys, uint32_t *tvals, uint64_t mask,
                                                              const uint64_t *keys, int64_t n, uint32_t val_base,
                                                              unsigned long long *stats)
{
    __shared__ unsigned long long s_max[kHashThreads / 64], s_sum[kHashThreads / 64], s_fail[kHashThreads / 64];
    const int64_t i = (int64_t)blockIdx.x * kHashThreads + threadIdx.x;
    unsigned long long probe = 0, failed = 0;
    if (i < n) {
        const int64_t p = hash_insert_bounded(tkeys, tvals, mask, keys[i], val_base + (uint32_t)i, mask + 1);
        if (p < 0)
            failed = 1;
        else
            probe = (unsigned long long)p;
    }
    unsigned long long mx = probe, sm = probe, fl = failed;
    for (int o = 32; o > 0; o >>= 1) {
        mx = max(mx, (unsigned long long)__shfl_xor((long long)mx, o, 64));
        sm += (unsigned long long)__shfl_xor((long long)sm, o, 64);
        fl += (unsigned long long)__shfl_xor((long long)fl, o, 64);
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_max[wave] = mx;
        s_sum[wave] = sm;
        s_fail[wave] = fl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kHashThreads / 64; ++w) {
            mx = max(mx, s_max[w]);
            sm += s_sum[w];
            fl += s_fail[w];
        }
        atomicMax(&stats[0], mx);
        atomicAdd(&stats[1], sm);
        if (fl) atomicAdd(&stats[2], fl);
    }
}

}  // namespace

int hash_insert_keys(covox_ctx *ctx, uint64_t *tkeys, uint32_t *tvals, int64_t capacity, int64_t n_present,
                     const uint64_t *keys, int64_t n, uint32_t val_base, int64_t *stats)
{
    if (!tkeys || !tvals || !stats || (n > 0 && !keys))
        return fail(ctx, COVOX_EINVAL, "hash_insert: null argument");
    if (capacity < 2 || capacity > ((int64_t)1 << 32) || (capacity & (capacity - 1)))
        return fail(ctx, COVOX_EINVAL, "hash_insert: capacity must be a power of two in [2, 2^32]");
    if (n < 0 || n_present < 0 || n > ((int64_t)1 << 32))
        return fail(ctx, COVOX_EINVAL, "hash_insert: negative or oversized key count");
    // at most 15/16 of the slots occupied after the call
    if (n_present + n > capacity - capacity / 16)
        return fail(ctx, COVOX_ETABLE_FULL, "hash_insert: load would exceed 15/16");
    if (n == 0) return COVOX_OK;
    const int64_t blocks = (n + kHashThreads - 1) / kHashThreads;
    {
        TimedLaunch tl(ctx, COVOX_K_HASH);
        hipLaunchKernelGGL(k_hash_stress, dim3((unsigned)blocks), dim3(kHashThreads), 0, ctx->stream, tkeys, tvals,
                           (uint64_t)(capacity - 1), keys, n, val_base, (unsigned long long *)stats);
    }
    return hip_check(ctx, hipGetLastError(), "hash_insert launch");
}

}  // namespace covox
