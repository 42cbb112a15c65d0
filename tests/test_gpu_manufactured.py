"""End-to-end check on the GPU: the CG1 manufactured problem solved by the library's
PCG (FP64 cycle and FP32 cycle) converges at the P1 rates on meshes of 16,641 and
66,049 DOFs (L2 rate 2, H1 rate 1, within 0.1)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1])
def test_cg1_rates_with_the_gpu_solver(precision):
    import paper_2607_07485_amd as P
    from test_manufactured import _p1_errors, _rates
    dev = torch.device("cuda:0")

    def solve(prob, b):
        with P.Hierarchy.setup_problem(prob, P.Params.default(tau_const=1.0, precision=precision,
                                                              rtol=1e-10)) as h:
            h.set_cycle_precision(precision)
            x, infos = h.solve(torch.from_numpy(b).to(dev))
            assert infos[0].converged == 1
            return x.cpu().numpy()

    Ns = [64, 128, 256]
    errs = [_p1_errors(N, solve) for N in Ns]
    r0 = _rates([e[0] for e in errs], [1.0 / N for N in Ns])
    r1 = _rates([e[1] for e in errs], [1.0 / N for N in Ns])
    assert abs(r0[-1] - 2.0) <= 0.1, (errs, r0)
    assert abs(r1[-1] - 1.0) <= 0.1, (errs, r1)
