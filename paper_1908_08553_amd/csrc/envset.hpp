// Networks that differ from one base network in a few sites, contracted with
// cached column environments (envset.cpp).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "tn.h"

namespace tn {

struct EnvSetImpl;

// Network k replaces the sites subst_site[o_k .. o_k + n_subst[k]) (row-major
// site indices, o_k = n_subst[0] + ... + n_subst[k-1]) of the base network.
tn_status envset_workspace(const tn_grid& grid, int32_t prec, int32_t n, const int32_t* n_subst,
                           const int32_t* subst_site, size_t* bytes, std::string& err);
tn_status envset_create(const tn_grid& grid, int32_t prec, int32_t n, const int32_t* n_subst,
                        const int32_t* subst_site, void* ws, size_t ws_bytes, EnvSetImpl** out,
                        std::string& err);
// outs[0]: the base network, outs[1 + k]: network k.
tn_status envset_run(EnvSetImpl* es, const double* const* base, const double* const* subst,
                     hipStream_t stream, tn_result* outs, std::string& err);
void envset_destroy(EnvSetImpl* es);

// Streams an environment set spreads its networks over (1..4), read by
// envset_workspace and envset_create.
void set_env_streams(int32_t n);
extern int32_t g_env_streams;
// Most GiB the environments inside columns may add to a set's workspace
// (0: none, only column environments).
void set_env_rows(int32_t gib);
extern int32_t g_env_rows;
// 1: single-site networks through site environments (with rows inside columns).
void set_env_sites(int32_t on);
extern int32_t g_env_sites;

}  // namespace tn
