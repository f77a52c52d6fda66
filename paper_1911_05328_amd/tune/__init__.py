"""Schedule selection: exhaustive autotuner (timing DB) and the learned MLP
cost model that proposes a schedule per (shape, dtype, workspace budget)."""
