// Radix sort of (key, index) pairs on the device (hipCUB), for the Morton order of the compact-support
// culling of Eq. (6).  Kept in a file of its own: hipCUB's headers are heavy to compile.
#include <hipcub/hipcub.hpp>

#include "gcb_internal.h"

namespace gcb {

// Sorts n (key, value) pairs by the low `bits` bits of the key, stably; with temp == nullptr only sets
// *temp_bytes to the scratch the sort needs.
hipError_t sort_pairs_u32(void* temp, size_t* temp_bytes, const uint32_t* keys_in, uint32_t* keys_out,
                          const int32_t* vals_in, int32_t* vals_out, int64_t n, int bits, hipStream_t s) {
    return hipcub::DeviceRadixSort::SortPairs(temp, *temp_bytes, keys_in, keys_out, vals_in, vals_out, (int)n, 0, bits,
                                              s);
}

}  // namespace gcb
