"""Element-by-element parity at the full benchmark sizes.

tests/golden/fullsize_digests.json holds, for every full-size case, the
SHA-256 of each output array of the oracle (written on a CPU host by
tests/golden/make_fullsize_digests.py, which calls only the oracle).  Here
the GPU computes the same cases in the configurations the benchmark runs --
the 512^3 and 256^3 fields one per ms_complex call with the path schedule
and gradient tile the autotuner picks there (entry ranking, 16x16x8) and with
the defaults, the 64-field batch as one ms_complex_batch call, the served
stream's timesteps and requests as batches -- and the digest of every output
array must equal the oracle's: gradient words, the critical list, the six
arc matrices (rowptr, col, val) and both manifold label arrays."""
import hashlib
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "fullsize_digests.json")
MATS = ("m10", "m10t", "m21", "m21t", "m32", "m32t")


def _golden():
    if not os.path.exists(GOLDEN):
        pytest.skip("tests/golden/fullsize_digests.json not generated")
    with open(GOLDEN) as fh:
        return json.load(fh)["cases"]


def _case(cases, name):
    if name not in cases:
        pytest.skip(f"{name} not in tests/golden/fullsize_digests.json")
    return cases[name]


def _h(t: torch.Tensor) -> str:
    return hashlib.sha256(np.ascontiguousarray(t.cpu().numpy()).tobytes()).hexdigest()


def digests(c) -> dict:
    """Digests of a msc.Complex in the layout the oracle digests use."""
    d = {"grad": _h(c.grad), "counts": list(c.count),
         "crit": {"id": _h(c.crit_id), "index": _h(c.crit_index), "value": _h(c.crit_value.view(torch.int32)),
                  "vmax": _h(c.crit_vmax)},
         "min_label": _h(c.min_label), "max_label": _h(c.max_label), "n_saturated": c.n_saturated}
    for nm in MATS:
        m = getattr(c, nm)
        d[nm] = {"rowptr": _h(m.rowptr), "col": _h(m.col), "val": _h(m.val), "nnz": int(m.col.numel())}
    return d


def check(name, got: dict, want: dict):
    assert got["counts"] == want["counts"], (name, "counts")
    assert got["grad"] == want["grad"], (name, "gradient words")
    for k in ("id", "index", "value", "vmax"):
        assert got["crit"][k] == want["crit"][k], (name, "critical " + k)
    for nm in MATS:
        assert got[nm]["nnz"] == want[nm]["nnz"], (name, nm, "nnz", got[nm]["nnz"], want[nm]["nnz"])
        for k in ("rowptr", "col", "val"):
            assert got[nm][k] == want[nm][k], (name, nm, k)
    assert got["min_label"] == want["min_label"], (name, "min_label")
    assert got["max_label"] == want["max_label"], (name, "max_label")
    assert got["n_saturated"] == want["n_saturated"], (name, "n_saturated")


def _field(name, want):
    from golden.make_fullsize_digests import make_field
    print(f"[fullsize] generating {name}", flush=True)
    f = make_field(name)
    assert hashlib.sha256(np.ascontiguousarray(f).tobytes()).hexdigest() == want["input"], \
        f"{name}: the generated input differs from the one the oracle ran on"
    return f


BENCH_CONFIG = {"schedule": 2, "tile": 5}   # what the autotuner picks at 512^3
DEFAULT_CONFIG = {"schedule": 0, "tile": 0}


def _ctx(cfg):
    from paper_2009_03707_amd import msc
    c = msc.Context()
    c.set_path_schedule(cfg["schedule"])
    c.set_option(msc.MS_OPT_GRADIENT_TILE, cfg["tile"])
    return c


@pytest.mark.parametrize("name", ["blobs512", "grf256"])
@pytest.mark.parametrize("cfg", ["bench", "default"])
def test_single_field_at_size(name, cfg):
    from paper_2009_03707_amd import msc
    want = _case(_golden(), name)
    f = _field(name, want)
    fd = torch.from_numpy(f).cuda()
    del f
    ctx = _ctx(BENCH_CONFIG if cfg == "bench" else DEFAULT_CONFIG)
    print(f"[fullsize] ms_complex {name} {cfg}", flush=True)
    got = digests(msc.complex_(fd, ctx))
    ctx.close()
    check(name, got, want)


def _batch_check(names, cases, cfg=BENCH_CONFIG):
    from paper_2009_03707_amd import msc
    wants = [_case(cases, n) for n in names]
    fs = [torch.from_numpy(_field(n, w)).cuda() for n, w in zip(names, wants)]
    ctx = _ctx(cfg)
    print(f"[fullsize] ms_complex_batch of {len(fs)} fields", flush=True)
    outs = msc.complex_batch(fs, ctx)
    for n, w, c in zip(names, wants, outs):
        check(n, digests(c), w)
    ctx.close()


def test_batch64_at_size():
    """All 64 uneven fields (sides 64..320) in one ms_complex_batch call."""
    cases = _golden()
    _batch_check([f"batch64/{i}" for i in range(64)], cases)


def test_served_stream_at_size():
    """Timesteps 0, 1, 199 of the advected 384x384x256 GRF and the stream's
    first 20 requests (sides 64..256), batched as the server batches them."""
    cases = _golden()
    _batch_check([f"serve/timestep{t}" for t in (0, 1, 199)], cases)
    _batch_check([f"serve/request{i}" for i in range(20)], cases)
