"""FP64 CPU oracle for the DPMM sub-cluster split/merge sampler.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU product
path (``paper_2204_08988_amd``) never imports, calls or links anything here,
and nothing here imports the product package.

The oracle is a plain, slow, step-by-step restatement of the sampler of
Chang & Fisher III as described in Dinari et al. (arXiv 2204.08988), Sec. 2.3
and Sec. 4.1 steps (a)-(f) plus the split and merge moves, in float64.  Every
random draw comes from the counter-based Philox4x32-10 stream defined in
``oracle.rng``; the GPU path implements the same published generator on its
own, so both sides see the same random numbers.

Modules
-------
philox    Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).
rng       uniform / Gumbel / logistic / normal / gamma transforms and the
          (seed, iteration, entity, tag, block) stream layout.
niw       Normal-Inverse-Wishart posterior, log marginal likelihood, Bartlett
          draw and Gaussian log-density.
dirmult   Dirichlet-multinomial posterior, log marginal likelihood, draws.
sampler   one sampler iteration and its parts (weights, params, labels,
          sub-labels, sufficient statistics, splits, merges, compaction).
partitions  exact posterior over set partitions and Neal's Algorithm 3, used
          to check the whole chain on tiny inputs.
mlp       float64 MLP forward/backward for the learned split proposal.
poisson   Poisson components with a Gamma prior (marginal, draws, log-likelihood).
nmi       normalised mutual information.
"""
