"""MI355X exchange-matrix library: hextree traversal with the Schwarz x |P|
metric query and Head-Gordon-Pople shell-quartet kernels (libfx.so), with a
thin ctypes binding (fx.py)."""
from .fx import (FX_PREC_FP64, FX_PREC_MIXED, FX_SCHED_BOUND, FX_SCHED_MLP, FX_SCHED_NONE, FX_SYM_AUTO,
                 FX_SYM_OFF, FX_LEAF_SHELL, FX_LEAF_BLOCK, FxError, Tree, fx_exchange_opts, opts_init,
                 build_quadtree_from, fx_build_quadtree, fx_exchange, fx_exchange_batched, fx_exchange_ex, fx_exchange_multi,
                 fx_exchange_noalloc,
                 fx_plan_tree, lib, make_opts, fx_set_class_variant, fx_get_class_variant,
                 fx_class_variants_available, CostModel, TaskTimings, fx_record_task_timings,
                 fx_costmodel_train, fx_set_class_launch, fx_get_class_launch, set_progress_stderr,
                 set_group_screen, get_group_screen, plan_row_cuts)
