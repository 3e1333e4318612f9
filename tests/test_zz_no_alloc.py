"""The allocation-free device assembly (mmsd_assemble_device_noalloc) against
the allocating one (mmsd_assemble_device), through the C ABI: the same
kernels on the same inputs, so every output array must be equal bit for bit.
Two calls in a row, the second on a smaller mesh (the fixed region keeps the
first call's contents), and a mesh too large for the region is refused."""
import sys

import numpy as np
import pytest

from paper_1309_5796_amd import meshgen

pytestmark = pytest.mark.gpu

KEYS = ["mrp", "mci", "K", "D1", "D2", "Q", "V", "pot_global", "lrp", "lci", "L"]


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def _grain(edge_nm, seed):
    rng = np.random.default_rng(seed)
    n = meshgen.config4_cells(edge_nm * 1e-9)
    mesh = meshgen.kuhn_box((edge_nm * 0.5e-9,) * 3, (n, n, n), air=True)
    mesh.materials = [meshgen.Material(1, meshgen.JS_T, meshgen.K1_JM3, meshgen.A_JM, meshgen.cap_axis(rng))]
    return mesh


def test_noalloc_assembly_equals_allocating_assembly():
    import torch
    from paper_1309_5796_amd import binding
    ctx = binding.Context(0)
    try:
        for name, mesh in (("config 1 (20 nm cube, jittered)", meshgen.config1()["mesh"]),
                           ("10 nm grain cube", _grain(10, 7))):
            say(f"no-alloc assembly: {name}, {mesh.tets.shape[0]} tets")
            ref = binding.assemble_device(ctx, mesh)
            got = binding.assemble_device(ctx, mesh, no_alloc=True)
            torch.cuda.synchronize()
            assert (got["N"], got["Nt"]) == (ref["N"], ref["Nt"])
            for k in KEYS:
                assert got[k].shape == ref[k].shape, k
                assert torch.equal(got[k], ref[k]), k
        say("no-alloc assembly: oversized mesh")
        with pytest.raises(binding.MMSDError) as e:
            binding.assemble_device(ctx, meshgen.config2()["mesh"], no_alloc=True)
        assert e.value.code == binding.E_INVALID and "bytes of device temporaries" in str(e.value)
    finally:
        ctx.close()
