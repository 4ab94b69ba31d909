"""GPU test of the entry point that allocates nothing
(ndrho_density_matrix_noalloc), through the C ABI: its rho equals that of
ndrho_density_matrix on the same structure, on two calls in a row (the second
on a smaller structure, after the first left its contents in the fixed
scratch), in the FP64 form and in the split-BF16 form; a structure whose one
pole does not fit the scratch is refused with ENOMEM."""
import numpy as np
import pytest

from synth import lattice

pytestmark = pytest.mark.gpu

BETA = 10.0


def _rho_both(c, sysd, n_poles, mu):
    print("case: noalloc dims=%s n=%d poles=%d" % (sysd["dims"], sysd["n"], n_poles), flush=True)
    sid = c.set_structure(sysd["n"], sysd["row_ptr"], sysd["col"], sysd["h"], sysd["s"], sysd["coords"])
    c.set_poles(sid, mu, BETA, n_poles)
    nnz = int(sysd["row_ptr"][-1])
    a, b = c.device_buffer(nnz), c.device_buffer(nnz)
    c.density_matrix(sid, a)
    c.density_matrix_noalloc(sid, b)
    ref, got = a.numpy(), b.numpy()
    a.free()
    b.free()
    return ref, got


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed_bf16x3", 1e-10)])
def test_noalloc_matches_density_matrix_on_two_calls(precision, tol):
    import paper_1005_0088_amd as nd
    big = lattice((12, 10, 6), "nn", 90)     # 2880 rows: its 80 poles take several passes of the scratch
    small = lattice((40,), "nn", 91)         # 160 rows
    with nd.Context(0, precision=precision) as c:
        ref1, got1 = _rho_both(c, big, 80, 0.1)
        ref2, got2 = _rho_both(c, small, 60, -0.2)
    for ref, got in ((ref1, got1), (ref2, got2)):
        err = float(np.max(np.abs(got - ref)))
        print("%s: max |noalloc - density_matrix| = %.3e" % (precision, err))
        assert np.all(np.isfinite(got))
        assert err <= tol
    if precision == "fp64":
        # same kernels, poles summed in the same order: identical values
        assert np.array_equal(got1, ref1) and np.array_equal(got2, ref2)


def test_noalloc_refuses_structure_beyond_scratch():
    import paper_1005_0088_amd as nd
    sysd = lattice((12, 12, 12), "nn", 92)  # about 93 MiB of workspace per pole
    with nd.Context(0) as c:
        sid = c.set_structure(sysd["n"], sysd["row_ptr"], sysd["col"], sysd["h"], sysd["s"], sysd["coords"])
        c.set_poles(sid, 0.0, BETA, 4)
        out = c.device_buffer(int(sysd["row_ptr"][-1]))
        with pytest.raises(nd.NdrhoError) as e:
            c.density_matrix_noalloc(sid, out)
        out.free()
    assert e.value.name == "ENOMEM" and "67108864" in str(e.value)
