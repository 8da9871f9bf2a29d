// Imaginary-time evolution of a PEPS (ite.cpp, ite.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "tn.h"

namespace tn {

struct IteImpl;

tn_status ite_workspace(const tn_ite_config& cfg, size_t* bytes, std::string& err);
tn_status ite_create(const tn_ite_config& cfg, void* ws, size_t ws_bytes, hipStream_t stream,
                     IteImpl** out, std::string& err);
tn_status ite_step(IteImpl* t, double dtau, int32_t n_steps, std::string& err);
tn_status ite_energy(IteImpl* t, double* energy, double* mx, double* mz, double* czz,
                     std::string& err);
void ite_sites(const IteImpl* t, double** sites);
int32_t ite_bonds(const IteImpl* t);
void ite_destroy(IteImpl* t);

}  // namespace tn
