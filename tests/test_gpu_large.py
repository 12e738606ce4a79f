"""The largest lattices: direction planes of more than 2^31 elements.

A 46,400 x 46,400 FP32 cavity (2.15e9 nodes, 155 GB of populations) runs 41
steps from the cold start with its default launches (ten four-step launches
and a one-step launch).  Information moves one node per step, so near the two
top corners, where the lid sets the flow going, the field must equal the same
corners of a 160 x 160 cavity run by the oracle with the same tau (both are at
least 42 nodes from every wall the two lattices do not share), and every node
more than 41 rows below the lid must still be exactly at rest.  The top rows
sit at the far end of each direction plane, so this checks the 64-bit plane
and row addressing of the kernels beyond 2^31 elements.
"""
import gc

import numpy as np
import pytest

import oracle as O
from gpu_util import require_gpu, torch

pytestmark = pytest.mark.gpu

N, M, STEPS, U, TAU = 46_400, 160, 41, 0.1, 0.6


def test_cavity_with_planes_beyond_2_31_elements():
    smrt = require_gpu()
    need = smrt.workspace_bytes(nx=N, ny=N, storage="f32", tau=TAU) + 3 * 4 * N * N
    free, _ = torch.cuda.mem_get_info()
    if free < need + (4 << 30):
        pytest.skip("needs %.0f GB of device memory, %.0f GB free" % (need / 1e9, free / 1e9))
    W = M - STEPS - 1  # corner window: more than STEPS nodes from the walls not shared
    try:
        s = smrt.Solver(N, N, scheme="smrt", boundary="cavity", storage="f32", tau=TAU, u_lid=U)
        print("cavity %d^2 f32, %d steps" % (N, STEPS), flush=True)
        s.step(STEPS)
        mass = s.mass()
        rho, ux, uy = s.moments(torch.float32)
        s.close()
        del s
        left = [t[N - W:, :W].double().cpu().numpy() for t in (rho, ux, uy)]
        right = [t[N - W:, N - W:].double().cpu().numpy() for t in (rho, ux, uy)]
        below = slice(0, N - STEPS)  # rows the lid cannot have reached
        at_rest = bool((rho[below] == 1).all() and (ux[below] == 0).all() and (uy[below] == 0).all())
        moved = float(ux[N - 1, N // 2])
    finally:
        rho = ux = uy = None
        gc.collect()
        torch.cuda.empty_cache()
    L = O.Lattice(M, M, "smrt", tau=TAU, u_lid=U)
    o = L.fields(L.run(L.init_equilibrium(), STEPS))
    o_left = [a[M - W:, :W] for a in o]
    o_right = [a[M - W:, M - W:] for a in o]
    err = max(np.max(np.abs(g - w)) for g, w in zip(left[1:] + right[1:], o_left[1:] + o_right[1:])) / U
    derr = max(np.max(np.abs(left[0] - o_left[0])), np.max(np.abs(right[0] - o_right[0])))
    print("corners max|du|/U = %.3e, max|drho| = %.3e, top-row ux %.4f, mass drift %.3e"
          % (err, derr, moved, mass / N / N - 1))
    assert at_rest
    # mid-lid, as far from the side walls as the centre of the small cavity's lid
    assert abs(moved - o[1][M - 1, M // 2]) <= 1e-5 * U
    assert err <= 1e-5 and derr <= 1e-6
    assert abs(mass / N / N - 1) < 1e-9
