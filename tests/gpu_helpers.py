"""Shared set-up for GPU tests: one workload -> (GPU problem, oracle, inputs)."""
import sys

import numpy as np
import torch

import paper_2506_00746_amd as feod
from oracle import Discretisation
from workloads import Workload, make_inputs

DEV = "cuda:0"


def announce(*what):
    print("[gpu case]", *what, file=sys.stderr, flush=True)


def relerr(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def setup(w: Workload, oracle=True, compute_load=True):
    inp = make_inputs(w)
    prob = feod.Problem(w.nx, w.ny, w.nz, w.k, w.nq, w.p, w.eps, vertices=inp["vertices"],
                        rho=inp["rho"], device=DEV)
    ora = None
    if oracle:
        ora = Discretisation(w.nx, w.ny, w.nz, w.k, w.nq, w.p, w.eps, vertices=inp["vertices"],
                             rho=inp["rho"], compute_load=compute_load)
    return prob, ora, inp


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()
