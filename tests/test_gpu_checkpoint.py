"""GPU: N fused steps in one call equal K steps, a checkpoint file, a fresh
context and N - K steps, bit for bit (2D and 3D, cubic L-J and Morse on the
hexagonal lattice)."""
import numpy as np
import pytest
import torch

from paper_1502_07722_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("ndim,variant", [(2, "lj"), (3, "lj"), (2, "morse_hcp")])
def test_resume_from_checkpoint_is_bit_identical(tmp_path, ndim, variant):
    from paper_1502_07722_amd import binding as B
    from paper_1502_07722_amd import checkpoint as CK
    if ndim == 2:
        grid, parts = W.make_slab(2, (64, 48), 24, 16, W.H_CELL, 61, fluence_Jcm2=3.0, R_cells=16)
    else:
        grid, parts = W.make_slab(3, (16, 16, 16), 8, 8, W.H_CELL, 62, fluence_Jcm2=3.0, R_cells=8)
    pot = W.Potential(c_att=0.27) if variant == "lj" else W.hcp(W.morse_cu(c_att=0.2))
    print(f"[checkpoint] {ndim}D {variant} N={parts.n}", flush=True)
    ctx = B.Context(grid, pot, W.DT, parts.n)
    a = B.DeviceParticles.from_host(parts)
    ctx.start_leapfrog(a)
    b = a.clone()
    ctx.pic_step(a, 60)
    ctx.pic_step(b, 25)
    f = tmp_path / "mid.npz"
    CK.save_state(f, b, grid, pot, W.DT, 25)
    del ctx, b
    p2, g2, pot2, dt, step, _ = CK.load_state(f)
    ctx2 = B.Context(g2, pot2, dt, p2.n)
    c = B.DeviceParticles.from_host(p2)
    ctx2.pic_step(c, 60 - step)
    torch.cuda.synchronize()
    for x, y in zip(a.to_host(), c.to_host()):
        assert np.array_equal(x, y)
