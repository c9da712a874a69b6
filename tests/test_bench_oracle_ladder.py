"""The CPU side of bench.py's oracle ladder (CPU only): its sampled mode hands each point's
periodic neighbourhood cube to the oracle instead of the whole field, which must give the
same bits, and its full-field worker must time the oracle's own full path."""
import math
import os
import sys

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from oracle import fields as F  # noqa: E402
from paper_2605_19796_amd import synth  # noqa: E402

KEYS = ("rho_bar", "ut", "tau", "G", "tau_gm", "tau_smag", "k_sgs", "nu_t", "omega_t")


@pytest.mark.parametrize("name,n,kind,nd", [("c32_box4", 20, F.BOX, 4),
                                            ("c256_gauss8", 30, F.GAUSS, 8)])
def test_neighbourhood_cubes_match_the_whole_field(name, n, kind, nd):
    rho, u = synth.workload_fields(name, device="cpu", n=n)
    R = F.filter_weights(kind, nd)[1]
    npts, seed = 6, 11
    cr, cu = bench._neighbourhoods(rho, u, R, npts, seed)
    assert cr.shape == (npts,) + (2 * R + 3,) * 3 and cu.shape == (npts, 3) + (2 * R + 3,) * 3
    # the same points the helper drew
    g = torch.Generator(device="cpu").manual_seed(seed)
    pts = torch.randint(0, n, (npts, 3), generator=g).numpy()
    h = 2 * math.pi / n
    whole = F.sampled_points(rho.numpy(), u.numpy(), kind, nd, h, pts)
    c = R + 1
    for p in range(npts):
        one = F.sampled_points(cr[p], cu[p], kind, nd, h, [(c, c, c)])
        for k in KEYS:
            assert np.array_equal(np.asarray(whole[k])[p], np.asarray(one[k])[0]), (k, p)


def test_full_worker_times_the_full_path():
    dt = bench._ladder_full_worker(("c32_box4", 12, F.BOX, 4))
    assert dt > 0.0
