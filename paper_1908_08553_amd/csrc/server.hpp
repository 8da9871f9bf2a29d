// Served request loop (server.cpp).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

#include "tn.h"

namespace tn {

struct ServerImpl;

tn_status server_create(void* arena, size_t arena_bytes, int32_t max_slots, int32_t queue_depth,
                        ServerImpl** out, std::string& err);
tn_status server_submit(ServerImpl* s, const tn_grid& grid, int32_t order, int32_t prec,
                        const double* const* host_sites, uint64_t* ticket, std::string& err);
tn_status server_poll(ServerImpl* s, uint64_t ticket, tn_result* out, int64_t* times_ns,
                      std::string& err);
void server_info(ServerImpl* s, tn_server_info* out);
void server_destroy(ServerImpl* s);

}  // namespace tn
