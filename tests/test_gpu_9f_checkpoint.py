"""Chain checkpoint and resume through the C ABI (rd_chains_save /
rd_chains_load): a chain saved after some steps and loaded into a fresh
state continues exactly as the original, and malformed files are refused."""
import os

import numpy as np
import pytest

from gpu_common import need_gpu
from test_gpu_2_sampler import _pde_chain_setup, chains_at

pytestmark = pytest.mark.gpu

FIELDS = ("phi", "loglik", "n_accept", "n_accept1", "n_solves", "cg_iters", "imex_steps",
          "fail_bits")


def test_resume_from_a_file_continues_the_chain_bit_for_bit(tmp_path):
    import torch
    need_gpu()
    p, phi0, ll_fn, _ = _pde_chain_setup()
    ll0 = ll_fn(phi0)
    a = chains_at(phi0, ll0, seed=17)
    p.mcmc_step(a, 3)
    path = str(tmp_path / "chains.bin")
    a.save(path)
    p.mcmc_step(a, 3)
    torch.cuda.synchronize()
    # a state with other values everywhere, then the file
    b = chains_at(phi0[::-1].copy(), np.zeros(len(phi0)), seed=99)
    b.step = 12345
    for f in FIELDS[2:]:
        getattr(b, f).fill_(7)
    b.load(path)
    assert b.seed == 17 and b.step == 3
    p.mcmc_step(b, 3)
    torch.cuda.synchronize()
    assert b.step == a.step
    for f in FIELDS:
        assert torch.equal(getattr(a, f), getattr(b, f)), f
    assert int(a.n_solves.sum()) > 0
    # header: 48 bytes, then n rows of each array the state has
    n = len(phi0)
    per_row = 8 * 4 + 8 + 8 + 8 + 8 + 8 * 2 + 8 + 8 * 8   # no loglik_sur, no grid_id
    assert os.path.getsize(path) == 48 + n * per_row
    p.close()


def test_malformed_files_and_shapes_are_refused(tmp_path):
    import torch
    from paper_1605_04718_amd._lib import RD_EINVAL, RD_EIO, RDError
    need_gpu()
    p, phi0, ll_fn, _ = _pde_chain_setup()
    a = chains_at(phi0, np.zeros(len(phi0)), seed=3)
    path = str(tmp_path / "c.bin")
    a.save(path)
    torch.cuda.synchronize()
    raw = open(path, "rb").read()

    def refused(chains, data, code):
        q = str(tmp_path / "x.bin")
        with open(q, "wb") as f:
            f.write(data)
        with pytest.raises(RDError) as e:
            chains.load(q)
        assert e.value.code == code

    refused(a, raw[:40], RD_EIO)                         # shorter than the header
    refused(a, raw[:-8], RD_EIO)                         # ends inside an array
    refused(a, raw + b"\0", RD_EINVAL)                   # trailing bytes
    refused(a, b"NOTCHAIN" + raw[8:], RD_EINVAL)         # magic
    fewer = chains_at(phi0[:-1], np.zeros(len(phi0) - 1))
    refused(fewer, raw, RD_EINVAL)                       # other n_chains
    da = chains_at(phi0, np.zeros(len(phi0)))
    da.loglik_sur = torch.zeros(len(phi0), dtype=torch.float64, device="cuda")
    refused(da, raw, RD_EINVAL)                          # the file has no loglik_sur
    with pytest.raises(RDError) as e:
        a.load(str(tmp_path / "missing.bin"))
    assert e.value.code == RD_EIO
    # grid classes are compared, not written
    g = torch.zeros(len(phi0), dtype=torch.int32, device="cuda")
    a.grid_id = g
    a.save(path)
    b = chains_at(phi0, np.zeros(len(phi0)))
    b.grid_id = torch.ones(len(phi0), dtype=torch.int32, device="cuda")
    with pytest.raises(RDError) as e:
        b.load(path)
    assert e.value.code == RD_EINVAL
    assert int(b.grid_id.sum()) == len(phi0)
    b.grid_id = g.clone()
    b.load(path)
    p.close()
