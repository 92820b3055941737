"""Host-side checks: the benchmark refuses more than one GPU, and the packaged
eigenbound model, evaluated by the FP64 oracle network on oracle features, predicts
lambda_max of a problem from its training distribution."""
import os
import subprocess
import sys

import numpy as np

import synth
from oracle import mlp as ML
from oracle import solve as OS
from oracle import sparse as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_packaged_model_on_oracle_features():
    sys.path.insert(0, ROOT)
    from paper_2606_24748_amd import train_eigmlp
    model = train_eigmlp.load_model().astype(np.float64)
    assert model.shape == (ML.N_PARAMS + 28,)
    theta = model[:ML.N_PARAMS]
    fm, fs = model[ML.N_PARAMS:ML.N_PARAMS + 12], model[ML.N_PARAMS + 12:ML.N_PARAMS + 24]
    tm, ts = model[ML.N_PARAMS + 24:ML.N_PARAMS + 26], model[ML.N_PARAMS + 26:ML.N_PARAMS + 28]
    assert np.all(fs > 0) and np.all(ts > 0)
    m = synth.make_mesh(16)
    i, j = synth.coo_indices(m)
    A = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, synth.coo_values(m, *synth.lame(*synth.materials(m.n_elem, 4321))))
    Dinv = S.block_diag_inverse(A)
    f = ML.features(A, Dinv, 0)
    _, _, y = ML.forward(theta, ((f - fm) / fs)[None, :])
    lam_pred = float(np.exp(y[0, 0] * ts[0] + tm[0]))
    lam_true = ML.judge_lambda(A, Dinv, 50, OS.Options().lanczos_seed)
    assert abs(lam_pred / lam_true - 1.0) <= 0.15, (lam_pred, lam_true)
