/* Measurement aid of libks.so: the device's achievable HBM read bandwidth.
 *
 * Not part of the method. The scan and the feature pass are bound by how fast
 * they read the samples; their roofline fraction is quoted against the
 * published HBM peak, and this probe gives the ceiling a plain read actually
 * reaches on the same device, with the same 16-byte nontemporal loads. */
#ifndef KS_PROBE_H
#define KS_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Reads words[0 .. num_words) once: a grid-stride loop of `grid` workgroups of
 * 256 threads, each thread issuing `unroll` (1 or 8) 16-byte nontemporal loads
 * per step, folded into a value that is stored to *sink only in a case that
 * does not occur for real data, so no load can be removed. Asynchronous on
 * `stream` (a hipStream_t, NULL for the default stream); the caller brackets
 * it with events. words: device, 16-byte aligned, num_words a multiple of 4;
 * sink: device, one uint32. KS_E_INVALID (-1) on a NULL pointer, a misaligned
 * buffer, num_words % 4 != 0, grid == 0 or unroll not 1 or 8; KS_E_HIP (-4)
 * if the launch fails. */
int ks_probe_read(const uint32_t *words, uint64_t num_words, uint32_t grid, uint32_t unroll, uint32_t *sink,
                  void *stream);

#ifdef __cplusplus
}
#endif

#endif /* KS_PROBE_H */
