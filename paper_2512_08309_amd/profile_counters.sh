#!/bin/bash
# Profiler runs behind the committed summaries in profiles/: the kernel trace
# of one cold C2 query per precision, and hardware counters (HBM bytes, MFMA
# busy cycles, LDS bank conflicts) of the convolution kernels through the
# kbench driver.  Run from the repository root on a GPU machine, after build();
# writes under gpurun_out/.
set -e
cd /tmp && export TMPDIR=/tmp
cd "${GRAFT_REPO_ROOT:-$(dirname "$0")/..}"
OUT=gpurun_out/counters
mkdir -p $OUT
KB=./paper_2512_08309_amd/kbench
for P in 0 1; do
  timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/trace_p$P -o run -- \
    python3 bench.py --query-only $P > $OUT/trace_p$P.log 2>&1
  echo "trace precision $P done"
done
run() {   # name, counters..., -- kbench args
  local name=$1; shift
  local ctr=()
  while [ "$1" != "--" ]; do ctr+=("$1"); shift; done
  shift
  timeout -s KILL 90 rocprofv3 --pmc "${ctr[@]}" --output-format csv -d $OUT/$name -o run -- $KB "$@" > $OUT/$name.log 2>&1
  echo "$name done"
}
for spec in "f32_l0res f32 6 128 128 1024 1" "f32_l1 f32 5 256 256 1024 0" "bf16_l0 bf16 6 128 128 1024 9 0" \
            "bf16_l0fused bf16 6 128 128 1024 9 1" "bf16_l0res bf16 6 128 128 1024 9 2" \
            "bf16_l1 bf16 5 256 256 1024 9 0"; do
  set -- $spec
  name=$1; shift
  run ${name}_fetch FETCH_SIZE -- "$@"
  run ${name}_write WRITE_SIZE -- "$@"
  run ${name}_sq SQ_BUSY_CYCLES SQ_VALU_MFMA_BUSY_CYCLES SQ_LDS_BANK_CONFLICT SQ_INSTS_LDS GRBM_GUI_ACTIVE -- "$@"
done
