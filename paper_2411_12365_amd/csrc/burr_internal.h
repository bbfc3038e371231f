// burr_internal.h - entry points shared between the library's C ABI files
// (not part of the public interface in include/burr.h).
#pragma once

#include <stdint.h>

#include "../../include/burr.h"

// Records `code` as the calling thread's last error (burr_last_error); returns it.
int burr_set_error(int code);

// Device bytes a batch holds for its members' tables (all layers).
uint64_t burr_batch_device_bytes(const burr_batch* b);

// Table bits of all members of a batch: codes and solution words of every
// layer, without allocation padding.
uint64_t burr_batch_table_bits(const burr_batch* b);

// Workspace bytes of one build of `count` structures with n keys in total
// and largest value width rmax, including (staged != 0) a contiguous copy of
// the inputs of structures that arrive in separate arrays.
uint64_t burr_workspace_bytes(uint64_t n, uint32_t rmax, uint32_t count, const burr_params* p,
                              int staged);
