// Internal accessors of a context for the test-only hook library
// (tests/native): not part of the C ABI.
#pragma once

#include "gsys.h"
#include "gsys_abi.h"

namespace gsys_host {
class Pool;
class Doorbell;
}  // namespace gsys_host

namespace gsys_internal {

bool no_device(gsys_ctx* ctx);
gsys_host::Pool* pool(gsys_ctx* ctx);
// the doorbell the pollers block on, or null
gsys_host::Doorbell* doorbell(gsys_ctx* ctx);
// host view of the slot ring and its number of slots
gsys_slot* ring_host(gsys_ctx* ctx, uint64_t* slots);

}  // namespace gsys_internal
