/*
 * mirng measurement kernels: the denominators against which the generation
 * kernels are measured on one MI355X.  Same conventions as mirng.h (device
 * pointers, `void *` hipStream_t, status codes, asynchronous on the stream).
 *
 * The paper profiles per-kernel durations of its seeding, generation and
 * range-transform kernels (arXiv:2109.01329, Sec. 7, kernel-time figure);
 * these probes give the ceilings those durations are compared with here:
 * the HBM write bandwidth a store-only kernel reaches, the VALU rate of the
 * Philox rounds without stores, and the issue rates of the instructions
 * the generators are built from.
 */
#ifndef MIRNG_BENCH_H
#define MIRNG_BENCH_H

#include <stddef.h>
#include <stdint.h>

#include "mirng.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Write `bytes` (a multiple of 16) of a constant pattern to `out` (16-byte
 * aligned device buffer) with one 16-byte store per lane per step, in the
 * walk and launch shape the Philox configuration selects.  nontemporal != 0 uses
 * streaming stores.  Errors: NULL out, bytes % 16 != 0 or misaligned out
 * -> INVALID_ARG; launch -> LAUNCH. */
mirng_status mirng_bench_store(void *out, uint64_t bytes, int32_t nontemporal,
                               void *stream);

/* Evaluate `nblocks` Philox4x32-10 blocks (counter = block index, key =
 * (k0, k1)) on a persistent grid-stride grid and XOR-fold them into one
 * word per wave written to `sink` (device, at least CUs * 64 words): the
 * generation work without its stores. */
mirng_status mirng_bench_philox_nostore(uint64_t nblocks, uint32_t k0, uint32_t k1,
                                        uint32_t *sink, void *stream);

/* Instruction-rate probes: `threads` lanes each run `iters` iterations of
 * 8 independent chains of one operation; the folded result goes to
 * sink[thread].  op: 0 = 32x32->64 integer multiply-add (v_mad_u64_u32),
 * 1 = 32-bit xor, 2 = FP64 fused multiply-add,
 * 3 = FP64 floor, 4 = FP32 fused multiply-add.
 * Operations per call = threads * iters * 8. */
mirng_status mirng_bench_valu(int32_t op, uint32_t threads, uint32_t iters,
                              uint32_t *sink, void *stream);

/* Test-only: the pieces of the FP32 Gaussian transforms on single 24-bit
 * inputs, so that a test can check every input (all 2^24 of each) against
 * the oracle.  For i < n, k = first + i, the engine word is w = k << 8:
 *   which 0: out (double)[i] = the Box-Muller radius sqrt(-2 ln u1),
 *            u1 = (k + 1) 2^-24, as the FP32 Gaussian computes it before
 *            its one rounding;
 *   which 1: out (double)[2i], [2i+1] = (cos, sin)(2 pi u2), u2 = k 2^-24,
 *            likewise; a Gaussian FP32 pair (z0, z1) is exactly
 *            (RN32(r cos), RN32(r sin)) of these two factors;
 *   which 2: out (float)[i] = the inverse-CDF Gaussian FP32 of w (mean 0,
 *            sd 1), u = (k + 1/2) 2^-24.
 * first + n must not exceed 2^24; out is device memory of n doubles, 2n
 * doubles or n floats.  Otherwise INVALID_ARG; unknown `which` ->
 * UNSUPPORTED.  Asynchronous on `stream`. */
mirng_status mirng_bench_transform_f32(int32_t which, uint32_t first, uint32_t n, void *out,
                                       void *stream);

/* Open-loop load generator for the serving loop: submits reqs[i] to `s` at
 * arrival_s[i] seconds after the call starts (non-decreasing times; the
 * caller's thread sleeps until each one, spinning for the last 50 us),
 * storing each submission's status and ticket.  With `engines` not NULL,
 * request i goes to resident engine engines[i] (mirng_server_submit_engine
 * with reqs[i]'s distribution, n and out; its engine type, seed and offset
 * are ignored); otherwise it is submitted as it is.  Latencies of these
 * requests count from their scheduled arrival, not from the (possibly
 * later) submission, so a generator that falls behind does not hide
 * queueing delay.  Returns once the last request has been submitted;
 * completion is left to mirng_server_wait / mirng_server_drain.  NULL
 * arguments -> INVALID_ARG. */
mirng_status mirng_bench_server_replay(mirng_server s, const mirng_request *reqs,
                                       const uint32_t *engines, const double *arrival_s,
                                       size_t count, uint64_t *tickets,
                                       int32_t *submit_status);

#ifdef __cplusplus
}
#endif

#endif /* MIRNG_BENCH_H */
