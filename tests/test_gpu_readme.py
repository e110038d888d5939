"""The README's Python example, run as written (two walkers of 22 atoms,
phi/psi, well-tempered metadynamics, an eager step then a 50-step graph):
step 0 sees no bias and deposits one hill per walker at its own CV values
(stored in float32); the graph's steps then see that hill's height, 1.2
kJ/mol, and a force that is zero up to the centre's float32 rounding."""
import numpy as np
import pytest
import torch

from paper_2301_04835_amd import Sampler

pytestmark = pytest.mark.gpu


def test_readme_example(gpu):
    s = Sampler(0)
    s.add_dihedral([4, 5, 6, 7])
    s.add_dihedral([5, 6, 7, 8])
    s.set_walkers(np.array([0, 22, 44]))
    s.metad([0.35, 0.35], height=1.2, temperature=300.0, bias_factor=6.0, stride=500, capacity=4096)
    s.bind()
    g = torch.Generator(device="cuda").manual_seed(5)
    pos = torch.randn(44, 3, device="cuda", generator=g)
    forces = torch.zeros_like(pos)
    V = torch.empty(2, dtype=torch.float64, device="cuda")
    s.step(pos, forces=forces, V_out=V)
    s.check()
    assert torch.all(V == 0)                       # no hills before the first deposit
    assert list(s.hill_counts()) == [1, 1]         # step 0 deposits one hill per walker
    s.graph_capture(50, pos, forces=forces, V_out=V)
    s.graph_launch()
    torch.cuda.synchronize()
    s.check()
    assert s.get_step() == 51
    assert torch.all((V - 1.2).abs() <= 1e-6)
    assert torch.isfinite(forces).all() and forces.abs().max() < 1e-3
