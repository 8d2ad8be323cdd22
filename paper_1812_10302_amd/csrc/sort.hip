// Ascending radix sort of 64-bit keys on the device (rocPRIM through hipCUB), for the LB-sorted
// visiting order of the plain search.
#include <hipcub/hipcub.hpp>

#include "dtws_internal.h"

namespace dtws {

// With temp == nullptr only sets temp_bytes; otherwise sorts in[count] into out[count] on stream s.
hipError_t sort_keys_u64(void *temp, size_t &temp_bytes, const uint64_t *in, uint64_t *out, int64_t count,
                         hipStream_t s) {
    return hipcub::DeviceRadixSort::SortKeys(temp, temp_bytes, in, out, count, 0, 64, s);
}

}  // namespace dtws
