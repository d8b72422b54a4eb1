/*
 * hg_membench.h -- C ABI of libhg_membench.so: microbenchmarks that measure,
 * on the GPU they run on, the ceilings the renderer's kernels are judged
 * against (measurement infrastructure; no renderer arithmetic).
 *
 *   - random gathers of 4-, 8- or 16-byte items from a table of 2^k items,
 *     the access pattern of the hash-grid encoder's corner lookups (a
 *     multi-resolution hash encoding reads its tables at effectively random
 *     addresses; paper Sec. 3.2 builds its renderer on such tables);
 *   - random FP32 atomic adds into a table, alone, with groups of lanes on
 *     one address, or with groups of lanes on adjacent words of one line,
 *     the pattern of the backward's scatter into the table gradients
 *     (Sec. 3.3 distillation);
 *   - matrix-core throughput loops (FP32 32x32x2 and BF16 16x16x32) with
 *     independent accumulator chains, the steps the MLP layers run on.
 *
 * Conventions as in hg.h: device pointers, asynchronous on `stream`, host
 * validation first (HG_E_INVALID-style codes: 0 ok, 1 invalid argument,
 * 4 launch failure), nothing allocated.  Item addresses come from a 32-bit
 * integer hash (a bijection) of a per-access counter, masked to the table,
 * so every run touches the same addresses for the same seed.
 */
#ifndef HG_MEMBENCH_H
#define HG_MEMBENCH_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Gather `rounds` x 8 items per thread over `blocks` x 256 threads from
 * `table` (2^log2_items items of item_bytes = 4, 8 or 16 bytes; 16-byte
 * aligned), eight independent loads in flight per lane; each thread writes
 * one 32-bit fold of what it read to sink[thread] (sink: blocks * 256
 * uint32).  log2_items in [4, 31 - log2(item_bytes)], blocks in
 * [1, 2^20], rounds in [1, 2^16]. */
int hgmb_gather(const void *table, int32_t log2_items, int32_t item_bytes, int32_t blocks, int32_t rounds,
                uint32_t seed, uint32_t *sink, hipStream_t stream);

/* Replay of a recorded address stream: a persistent grid of blocks x 256
 * threads walks the eight-item groups of idx (thread t takes groups t,
 * t + threads, ...; consecutive lanes on consecutive groups), gathers
 * table[idx[8g .. 8g+7]] with all eight loads in flight and prefetches the
 * next group's indices behind them; n mod 8 tail items go one per thread.
 * With idx = the hash-grid encoder's corner indices in its order (one group
 * per point and level) this is that encoder's address stream without its
 * arithmetic: the time is the memory system's for those addresses, plus
 * 4 bytes of streamed index per item.  item_bytes = 4, 8 or 16; idx: n
 * uint32 item indices (16-byte aligned, each inside the table); each thread
 * writes one fold to sink[thread] (blocks * 256 uint32).  n in [0, 2^40],
 * blocks in [1, 2^20]. */
int hgmb_gather_indexed(const void *table, int32_t item_bytes, const uint32_t *idx, int64_t n, int32_t blocks,
                        uint32_t *sink, hipStream_t stream);

/* FP32 atomic add of 1.0 (no return value) into `table` (2^log2_items
 * floats, 16-byte aligned): `rounds` x 4 atomics per thread over blocks x 256
 * threads; lanes_per_address (1, 2, 4, ..., 64) consecutive lanes of a wave
 * share one address per atomic, the rest are random.  Same ranges as
 * hgmb_gather. */
int hgmb_atomic(float *table, int32_t log2_items, int32_t blocks, int32_t rounds, int32_t lanes_per_address,
                uint32_t seed, hipStream_t stream);

/* FP32 atomic add of 1.0 (no return value) into `table` (2^log2_items
 * floats, 16-byte aligned): `rounds` x 4 atomics per thread over blocks x 256
 * threads; lanes_per_line (1, 2, 4, 8 or 16) consecutive lanes of a wave add
 * to that many adjacent words of one aligned block (inside one 64-byte
 * line), the blocks random.  The rate per group against the rate per lane
 * tells whether the atomic unit's cost is per lane or per request (the
 * lanes of one instruction that fall in one line).  Same ranges as
 * hgmb_atomic. */
int hgmb_atomic_lines(float *table, int32_t log2_items, int32_t blocks, int32_t rounds, int32_t lanes_per_line,
                      uint32_t seed, hipStream_t stream);

/* Matrix-core loop: every wave of blocks x 256 threads issues `iters`
 * rounds of `chains` (1, 2, 4, 8 or 16) independent accumulating steps of
 * kind 0 = v_mfma_f32_32x32x2f32 (4096 FLOP each) or 1 =
 * v_mfma_f32_16x16x32_bf16 (16384 FLOP each), then writes one float per
 * thread to sink (blocks * 256 floats).  iters in [1, 2^20]. */
int hgmb_mfma(int32_t kind, int32_t blocks, int32_t iters, int32_t chains, float *sink, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* HG_MEMBENCH_H */
