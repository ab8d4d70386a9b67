"""One EA generation step (zg_ea_step) on the GPU against the oracle through
the C ABI.

Covered:
- winners equal the oracle's exactly;
- children follow tests/parity.py: copied genes bit for bit, mutated genes
  through the rules of the ziggurat's outcome (fast path bit-exact, slow
  path within 2 ulp before the clamp);
- tournaments of 1 to 70 draws, NaN and tied fitness, ragged gene counts;
- the benchmark's population (16384 x 1024, tournament 2, rate 0.05) in full;
- argument errors.
"""
import numpy as np
import pytest
import torch

from oracle import coracle as orc
from parity import compare_mutated

pytestmark = pytest.mark.gpu


def _run(ctx, zg, P, F, k, seed, stream, gen, rate, sigma, lo, hi):
    Pt = torch.from_numpy(P).cuda()
    Ft = torch.from_numpy(F).cuda()
    Ct = torch.empty_like(Pt)
    Wt = torch.empty(P.shape[0], dtype=torch.int32, device="cuda")
    ctx.zg_ea_step(Pt, Ft, Ct, Wt, tournament=k, rate=rate, sigma=sigma, lo=lo, hi=hi, seed=seed,
                   stream=stream, generation=gen)
    torch.cuda.synchronize()
    return Ct.cpu().numpy(), Wt.cpu().numpy().view(np.uint32)


def _check(ctx, zg, P, F, k, seed, stream, gen, rate, sigma, lo, hi):
    C, W = _run(ctx, zg, P, F, k, seed, stream, gen, rate, sigma, lo, hi)
    Co, Wo, cls, errs = orc.ea_step(P, F, k, seed, stream, gen, rate, sigma, lo, hi, nthreads=16)
    assert errs == 0
    assert np.array_equal(W, Wo)
    # copied genes (cls 255) compare as fast-path values: bit for bit
    c = np.where(cls == 255, 0, cls).astype(np.uint8)
    pop, genes = P.shape

    def z_of(idx):
        # the oracle's variate of each gene: index (gen pop + c) genes + g of stream + 2
        w = (gen * pop + idx // genes) * genes + idx % genes
        return np.array([orc.fill_f64(orc.SM64, seed, stream + 2, int(v), 1)[0][0] for v in w])

    compare_mutated(C.ravel(), Co.ravel(), c.ravel(), z_of, sigma, ("ea", P.shape, k, gen))
    assert ctx.zg_error_flags() == 0


@pytest.mark.parametrize("pop,genes,k,gen,rate,sigma,lo,hi,nanfit", [
    (37, 70, 2, 3, 0.1, 0.5, -2.0, 2.0, False), (5, 1, 1, 0, 1.0, 3.0, -1.0, 1.0, False),
    (300, 129, 4, 7, 0.05, 0.1, -5.0, 5.0, True), (64, 64, 70, 1, 0.5, 1.0, -1.5, 1.5, True),
    (4099, 33, 3, 100, 0.2, 0.7, -2.5, 2.5, False), (1, 1000, 5, 9, 0.3, 0.1, -5.0, 5.0, False),
    (20000, 300, 2, 5, 0.05, 0.1, -5.0, 5.0, False), (50, 2048, 256, 2, 1.0, 0.2, -3.0, 3.0, True),
    (9000, 513, 8, 1, 0.9, 0.3, -4.0, 4.0, False)])
def test_ea_step_matches_oracle(ctx, zg, pop, genes, k, gen, rate, sigma, lo, hi, nanfit):
    rng = np.random.Generator(np.random.PCG64(pop + genes))
    P = rng.uniform(-2, 2, (pop, genes))
    F = np.floor(rng.uniform(0, 10, pop))
    if nanfit:
        F[::3] = np.nan
    _check(ctx, zg, P, F, k, 123, 10, gen, rate, sigma, lo, hi)


def test_ea_benchmark_population_in_full(ctx, zg):
    """The benchmark's EA step: 16384 x 1024 genes, sphere fitness, binary
    tournament, rate 0.05, sigma 0.1, bounds [-5, 5], generation 3."""
    rng = np.random.Generator(np.random.PCG64(7))
    P = rng.uniform(-5, 5, (16384, 1024))
    F = (P * P).sum(axis=1)
    _check(ctx, zg, P, F, 2, 2024, 100, 3, 0.05, 0.1, -5.0, 5.0)


def test_ea_argument_errors(ctx, zg):
    P = torch.zeros((8, 4), dtype=torch.float64, device="cuda")
    F = torch.zeros(8, dtype=torch.float64, device="cuda")
    C = torch.empty_like(P)
    for kw in ({"tournament": 0}, {"tournament": 257}, {"rate": 1.5}, {"rate": -0.1},
               {"lo": 1.0, "hi": -1.0}, {"stream": 65534}):
        with pytest.raises(zg.ZgError) as e:
            ctx.zg_ea_step(P, F, C, **kw)
        assert e.value.status == zg.ZG_EINVAL, kw
    with pytest.raises(zg.ZgError) as e:
        ctx.zg_ea_step(P, F, P)   # children over the parents
    assert e.value.status == zg.ZG_EINVAL
    with pytest.raises(zg.ZgError) as e:
        ctx.zg_ea_step(P, F, C, generation=2**40)
    assert e.value.status == zg.ZG_ERANGE
