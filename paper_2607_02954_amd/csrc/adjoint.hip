// Reverse-mode (adjoint) kernels of the filament-fluid step.
#include "engine.h"
#include "microcosm.h"

extern "C" {

sim_status sim_backward_workspace_size(const sim_world* w, int32_t ckpt_every, size_t* bytes) {
  (void)w;
  (void)ckpt_every;
  if (bytes) *bytes = 0;
  return SIM_E_STATE;
}

sim_status sim_backward(sim_world* w, int64_t t0, int32_t n_steps, int32_t ckpt_every, const void* ckpt,
                        const float* g_pos, float* g_rest_angle, float* g_pos0, void* adj_ws, size_t adj_ws_bytes) {
  (void)w; (void)t0; (void)n_steps; (void)ckpt_every; (void)ckpt; (void)g_pos; (void)g_rest_angle;
  (void)g_pos0; (void)adj_ws; (void)adj_ws_bytes;
  return SIM_E_STATE;
}

}
