"""Write the FP64 oracle's first iteration on a full-size large workload.

Workloads (seeded generator in datagen/, K = 1,000,000 subjects, J = 5000,
Zipf(1.1) columns):
  2: R = 10, I_k uniform in [10, 100], 1 + Poisson(0.145) nonzeros per row
     (about 63M nonzeros);
  3: R = 40, I_k uniform in [40, 100], 1 + Poisson(6) nonzeros per row
     (about 490M nonzeros);
default initial state H0 = I, W0 = 1, V0 ~ U[0, 1) from seed
[170304219, cfg, 1].

Calls only datagen/ and oracle/ (the process-pool driver of the FP64 oracle).
Writes tests/golden/full_c<cfg>_iter1.npz with
  M1, M2, H1, V1          full (R x R, J x R; V1 in the caller's column order)
  loss, fit, nx2          scalars
  idx                     sampled subjects (1000 at random, plus the first and last)
  M3s, W1s                M3 and W_{t+1} rows of the sampled subjects
  kappa_s                 condition number of B_k = X_k V0 S_k H0^T of each
                          sampled subject (numerically zero singular values,
                          below 1e-8 sigma_max, left out)
  K, J, R, nnz            sizes of the input, to check it was regenerated alike

Run from the repository root: python tests/golden/make_full_golden.py <cfg>
(about 2 minutes for cfg 2 and 25 minutes for cfg 3 on 8 cores).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)



def main(cfg):
    from datagen import gen_config, gen_init
    from oracle.parallel import Pool
    out = os.path.join(ROOT, "tests", "golden", f"full_c{cfg}_iter1.npz")
    X, R = gen_config(cfg)
    H0, V0, W0 = gen_init(X.J, X.K, R, [170304219, cfg, 1])
    rng = np.random.default_rng(20240)
    idx = np.unique(np.concatenate([[0, X.K - 1], rng.choice(X.K, 1000, replace=False)]))
    t0 = time.time()
    with Pool(X.subj_ptr, X.row_ptr, X.col, X.val, X.J) as pool:
        print(f"K={X.K} nnz={X.nnz}: {pool.workers} workers", flush=True)
        H1, V1, W1, info = pool.iterate(H0, V0, W0)
        print(f"iteration {time.time() - t0:.0f} s, fit {info['fit']:.12f}", flush=True)
    from datagen import take_subjects
    sub = [take_subjects(X, int(k), int(k) + 1) for k in idx]
    from datagen import concat_slices
    Xs = concat_slices(sub)
    with Pool(Xs.subj_ptr, Xs.row_ptr, Xs.col, Xs.val, Xs.J, workers=2) as pool:
        kap = pool.kappa(H0, V0, W0[idx], cut=1e-8)
    np.savez(out, M1=info["M1"], M2=info["M2"], H1=H1, V1=V1, loss=info["loss"],
             fit=info["fit"], nx2=info["nx2"], idx=idx,
             M3s=info["M3"][idx], W1s=W1[idx], kappa_s=kap, K=X.K, J=X.J, R=R, nnz=X.nnz)
    print(f"wrote {out} after {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]))
