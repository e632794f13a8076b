"""Error measures shared by the GPU-versus-oracle tests.

  e_x = max_i |x_gpu - x_ref|_inf / max_i |x_ref|_inf      (positions, relative)
  e_a = max_i |x_gpu - x_ref|_inf                          (positions, in cells)
  e_u = max_c |u_gpu - u_ref|_inf / max_c |u_ref|_inf      (grid velocity)
  e_d = max_i |dx_gpu - dx_ref|_inf / max(max_i |dx_ref|_inf, DISP_FLOOR)
        with dx the displacement of a step (or of a run of steps) taken by
        both sides from the same state: the motion itself is compared, not
        the absolute coordinate.  The floor keeps the measure defined when
        nothing moves: below it the bar becomes an absolute 1e-4 * DISP_FLOOR
        cells, about the resolution of the FP32 cell fraction.
"""
import numpy as np
import torch

import oracle as O

TOL_X = 1e-5
TOL_U = 1e-4
TOL_D = 1e-4
DISP_FLOOR = 1e-3


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b)) if b.size else 0.0
    num = np.max(np.abs(a - b)) if b.size else 0.0
    return num / den if den > 0 else num


def abs_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b))) if b.size else 0.0


def disp_err(d_gpu, d_ref):
    d_gpu = np.asarray(d_gpu, dtype=np.float64)
    d_ref = np.asarray(d_ref, dtype=np.float64)
    if not d_ref.size:
        return 0.0
    return float(np.max(np.abs(d_gpu - d_ref))) / max(float(np.max(np.abs(d_ref))), DISP_FLOOR)


def oracle_params(p):
    return O.Params(nx=p.nx, ny=p.ny, tau=p.tau, trt_magic=p.trt_magic, k_bend=p.k_bend,
                    k_stretch=p.k_stretch, k_shear=p.k_shear, pbd_iters=p.pbd_iters,
                    k_elastic=p.k_elastic, k_repulse=p.k_repulse, sigma=p.sigma_repulse,
                    radius=p.repulse_radius, u_max=p.u_max,
                    mdf_iters=getattr(p, "mdf_iters", 1), marker_offset=getattr(p, "marker_offset", 0.0))


def state64(st):
    """(x, f) of a device state as float64 CPU tensors (exact widening)."""
    return torch.from_numpy(st.positions64()), torch.from_numpy(st.populations64())


def oracle_from(x, f, t0, n, inp, op):
    """n oracle steps from (x, f); returns (x_n, f_n, u of the last step)."""
    u = None
    with torch.no_grad():
        for k in range(n):
            x, f, u = O.step(x, f, t0 + k, inp, op)
    return x, f, u


def final_state_errors(world, st, op, t0, steps):
    """A world's state after `steps` steps on the GPU (DeviceState st) against
    the oracle run from the same initial world: (e_x, e_a, e_u, e_d) with the
    displacement measured over the whole run."""
    inp = O.inputs_from_world(world)
    x0 = O.positions_from_world(world)
    xr, _, ur = oracle_from(x0, O.rest_populations(op), t0, steps, inp, op)
    xg = st.positions64()
    return (rel(xg, xr.numpy()), abs_err(xg, xr.numpy()), rel(st.velocity64(), ur.numpy()),
            disp_err(xg - x0.numpy(), (xr - x0).numpy()))
