"""Train the window-predicting MLP on the GPU and save it.

Training set: 2^20 (nu, x) pairs, nu ~ U[0.01, 10], x log-uniform on [1e-4, 1e3]
(seed 4); targets are the plain solver's windows at L = 15 and node counts for
exp(-14.5) (bk_window). Training runs in the library's own kernels (forward /
backward / Adam, bk_model_train); this script only marshals arguments.

Usage: python -m paper_2502_00356_amd.train_window_mlp [--out PATH] [--n N] [--epochs E]
"""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "models", "window_mlp.bin")


def train(out=DEFAULT_OUT, n=1 << 20, epochs=40, batch=4096, lr=2e-3, seed=1234, verbose=True):
    import torch
    from . import api, workloads
    nu_h, x_h = workloads.training_pairs(n, seed=4)
    dev = torch.device("cuda:0")
    nu = torch.from_numpy(nu_h).to(dev)
    x = torch.from_numpy(x_h).to(dev)
    m = api.Model()
    t0 = time.perf_counter()
    loss = m.train(nu, x, epochs=epochs, batch=batch, lr=lr, seed=seed)
    dt = time.perf_counter() - t0
    if verbose:
        print("trained window MLP on %d pairs, %d epochs, final loss %.4g, %.1f s; margins from "
              "inference-path residuals" % (n, epochs, loss, dt), flush=True)
    if out:
        os.makedirs(os.path.dirname(out), exist_ok=True)
        m.save(out)
    return m, loss


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    a = ap.parse_args()
    train(a.out, a.n, a.epochs, a.batch, a.lr)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    main()
