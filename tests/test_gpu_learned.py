"""What the trained network gains: the learned correction of red-black SOR,
trained on the GPU by the network's own kernels from solver snapshots, against
the same SOR started from the previous step's correction, both to the same
1e-8 residual; also with FP32 sweeps and FP64 refinement.  A half-resolution
(512x384) version of the plunging workload keeps the test to seconds."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_trained_correction_cuts_sor_iterations():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_17337_amd import ibm
    from paper_2402_17337_amd import warmstart as WS
    from paper_2402_17337_amd import workloads as W
    wl = W.plunging_stretched(512, 384, 0.02)
    F, every = 8, 2000
    params, scale, info = WS.train_default(wl, factor=F, every=every, cases=8, iters=1500,
                                           snap_iters=(200, 1000, 4000), policy_iters=(4000, 8000, 16000))
    assert np.all(np.isfinite(params)) and scale > 0
    res = WS.evaluate(wl, params, scale, warm_steps=2, method=ibm.RBSOR,
                      modes=(ibm.INIT_PREVIOUS, ibm.INIT_LEARNED), factor=F, every=every, guess=False,
                      options=WS.RECIPE_OPTIONS)
    prev, lrn = res[ibm.INIT_PREVIOUS][0], res[ibm.INIT_LEARNED][0]
    tol = wl["params"]["p_tol"]
    assert prev["rc"] == ibm.OK and lrn["rc"] == ibm.OK
    assert prev["p_rel"] <= tol and lrn["p_rel"] <= tol
    assert lrn["n_net"] >= 1
    print(f"previous guess {prev['p_iters']} iterations, learned {lrn['p_iters']} "
          f"({lrn['n_net']} network steps, mean step {lrn['net_step']:.3f})")
    assert lrn["p_iters"] < 0.67 * prev["p_iters"], (prev["p_iters"], lrn["p_iters"])
    # the same network correcting the FP32-sweep solve (FP64 refinement and
    # stop test every 100 iterations, a divisor of the correction interval)
    wl_mp = dict(wl, params=dict(wl["params"], p_check=100))
    mp = WS.evaluate(wl_mp, params, scale, warm_steps=2, method=ibm.RBSOR_MP, modes=(ibm.INIT_LEARNED,),
                     factor=F, every=every, guess=False, options=WS.RECIPE_OPTIONS)[ibm.INIT_LEARNED][0]
    print(f"learned with FP32 sweeps: {mp['p_iters']} iterations ({mp['n_net']} network steps)")
    assert mp["rc"] == ibm.OK and mp["p_rel"] <= tol and mp["n_net"] >= 1
    assert mp["p_iters"] < 0.67 * prev["p_iters"], (prev["p_iters"], mp["p_iters"])
