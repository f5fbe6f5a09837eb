// Accelerated subiteration steps (paper Sect. 3.1 Eq. 3 applied inside the subtree of a
// subiteration, Sect. 3.2 and App. B): launchers of the two per-leaf kernels in thermal.hip.
#pragma once

#include "internal.h"

// For every leaf of the model: inside the subtree (sub_lev < 0: the whole model) the absorbed
// power the diagonal operator balances with the new emission, (a_tot - e_self) / (1 - lambda*)
// with lambda* = e_self / e_emit (clamped below 1 - 1e-9; 0 where the step emitted nothing from
// the leaf); outside it a_tot itself.  a_tot, e_self, e_emit, a_solve: canonical [n_nodes] of
// the model, device.  Values of refined nodes are copied from a_tot.
hipError_t launch_subiter_ali(const ModelDev* models, int model, int64_t n_nodes, int64_t n_leaves,
                              const int32_t* leaf_node, const uint8_t* leaf_level, const int32_t* leaf_coord,
                              int sub_lev, const int32_t sub_I[3], const double* a_tot, const double* e_self,
                              const double* e_emit, double* a_solve, hipStream_t s);

// Restores the temperatures of the leaves outside the subtree from t_old (canonical [n_nodes],
// device), so that a step changes only its subtree whatever its absorbed power there.
hipError_t launch_subiter_keep(const ModelDev* models, int model, int64_t n_leaves, const int32_t* leaf_node,
                               const uint8_t* leaf_level, const int32_t* leaf_coord, int sub_lev,
                               const int32_t sub_I[3], const double* t_old, double* t_node, hipStream_t s);
