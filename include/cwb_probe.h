/* cwb_probe.h -- measurement utility of the binned componentwise-boosting
 * library (libcwb.so), not part of the method: the LDS atomic rate that
 * bounds its histogram pass, measured on the GPU without HBM traffic.
 * Conventions (status codes, cwb_last_error, device pointers) as in cwb.h.
 */
#ifndef CWB_PROBE_H_
#define CWB_PROBE_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The LDS histogram ceiling: `blocks` blocks of 1,024 threads each add
 * `steps` x `learners` x 8 rows per thread into `learners` LDS histograms of
 * `nb` words of `word_bytes` bytes (4 or 8: the histogram pass's 32-bit and
 * int64 accumulators), as the histogram pass does, but read their bin
 * indices from the device table `idx` (`idx_len` uint16 bins, 8 times a
 * power of two, 16-byte aligned, small enough to stay in L2; row r of the
 * probe reads entry r mod idx_len) instead of streaming them from HBM.  Bins
 * at or above nb are clamped to nb - 1.  Each block adds its histogram
 * total to out[block] (device, `blocks` int64, zeroed by the caller).
 * Asynchronous on `stream`; the caller times it.  Returns CWB_E_INVALID_ARG
 * for sizes outside learners 1..4, nb 1..8192, word_bytes other than 4 or 8,
 * learners x nb x word_bytes above 152 KiB, or a table of another length or
 * alignment. */
int cwb_probe_lds_hist(const uint16_t* idx, int64_t idx_len, int32_t nb, int32_t learners,
                       int32_t word_bytes, int32_t steps, int32_t blocks, long long* out,
                       void* stream);

#ifdef __cplusplus
}
#endif
#endif /* CWB_PROBE_H_ */
