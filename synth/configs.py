"""Workload definitions: graph shapes follow Table I of the paper (vertices /
edges / number of clusters), the block-structure knobs are the synthetic
stand-ins for the challenge datasets."""

CONFIGS = {
    # 1K vertices, 8 equal blocks, mean degree 20, 80% intra-block edges;
    # FP64, 20 fixed iterations, k-means with 10 restarts.
    "sbm1k": dict(n=1000, blocks=8, mean_degree=20.0, intra=0.8, sizes="equal",
                  alpha=1.0, k=8, maxit=20, tol=0.0, precision="fp64", restarts=10),
    # 50K / 1M / 44 (Table I column 3), Dirichlet(5) block sizes.
    "sbm50k": dict(n=50_000, blocks=44, mean_degree=40.0, intra=0.75, sizes="dirichlet",
                   alpha=5.0, k=44, maxit=30, tol=1e-2, precision="fp64", restarts=10),
    # .5M / 10M / 98 (Table I column 4), high overlap, Dirichlet(1) sizes;
    # mixed precision: FP32 SpMM, BF16 Gram on MFMA, FP64 Cholesky / RR.
    "sbm500k": dict(n=500_000, blocks=98, mean_degree=40.0, intra=0.6, sizes="dirichlet",
                    alpha=1.0, k=98, maxit=30, tol=1e-2, precision="fp32_bf16gram",
                    restarts=10),
    # 2M / 40M / 160 (Table I column 5): FP32 SpMM / Gram, FP64 RR.
    "sbm2m": dict(n=2_000_000, blocks=160, mean_degree=40.0, intra=0.7, sizes="dirichlet",
                  alpha=2.0, k=160, maxit=30, tol=1e-2, precision="fp32", restarts=10),
    # 5K / .1M / 19 (Table I column 1): smallest member of the serving mix.
    "sbm5k": dict(n=5_000, blocks=19, mean_degree=40.0, intra=0.75, sizes="dirichlet",
                  alpha=5.0, k=19, maxit=30, tol=1e-2, precision="fp64", restarts=10),
}


def config(name: str) -> dict:
    return dict(CONFIGS[name])


def graph_for(name: str, seed: int = 1):
    from .sbm import dcsbm
    c = CONFIGS[name]
    return dcsbm(c["n"], c["blocks"], c["mean_degree"], c["intra"], c["sizes"],
                 c["alpha"], seed)
