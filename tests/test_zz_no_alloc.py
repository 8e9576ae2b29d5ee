"""The allocation-free hydro step (hpac_hydro_step_noalloc) against
hpac_hydro_step: the same kernels with the time-step partials in the
library's scratch array instead of the caller's buffer, so every field must
be bitwise equal.  Two meshes in a row, the second smaller, so the second
run reads partials the first left behind only if the kernels do not write
every entry they read."""
import numpy as np
import pytest
import torch

from paper_2308_16877_amd import hpac
from paper_2308_16877_amd.hydro import Hydro, Tech

pytestmark = pytest.mark.gpu

FIELDS = ("x", "u", "e", "p", "q", "c", "vol", "force", "weos", "rho_eos", "z_eos", "whg", "rho_hg", "z_hg", "clock")


def techs():
    return [Tech(eos=(4, 4, 0.01), perfo=("small", 5, 4)),      # EOS TAF at wave level, herded hourglass perforation
            Tech(hg=(2, 2, 0.01, "thread"))]                     # hourglass TAF at thread level


@pytest.mark.parametrize("which", [0, 1])
def test_noalloc_step_matches_step_on_two_meshes(which):
    for n, steps in ((24, 12), (10, 15)):
        print("noalloc hydro: tech %d, n %d, %d steps" % (which, n, steps), flush=True)
        ref = Hydro(n, tech=techs()[which])
        got = Hydro(n, tech=techs()[which])
        got.dt_partials = None                                   # the entry point ignores the caller's partials
        got._bind()
        rec = ref.tech.c.eos_history or ref.tech.c.hg_history
        for _ in range(steps):
            ref.step(record=bool(rec))
            got.step(record=bool(rec), noalloc=True)
            torch.cuda.synchronize()
            if rec:
                assert torch.equal(ref.dec_eos, got.dec_eos) and torch.equal(ref.dec_hg, got.dec_hg)
        a, b = ref.numpy_state(), got.numpy_state()
        for f in FIELDS:
            if a.get(f) is None:
                continue
            assert np.array_equal(a[f], b[f]), "n %d: field %s differs" % (n, f)
        assert ref.time() > 0 and ref.time() == got.time()
        ref.check()
        got.check()


def test_noalloc_step_rejects_meshes_past_its_scratch():
    h = Hydro(8, tech=Tech())
    p = hpac.hpac_hydro_params(n=hpac.HYDRO_NOALLOC_MAX_N + 1, **{k: getattr(h.params, k) for k in
                                                                 ("side", "gamma", "cq", "cl", "khg", "cfl",
                                                                  "growth", "dvmax", "dt0")})
    with pytest.raises(hpac.HpacError) as e:
        hpac.hpac_hydro_step_noalloc(p, h.tech.c, 0, h.state)
    assert e.value.status == hpac.HPAC_EINVAL and "scratch" in str(e.value)
