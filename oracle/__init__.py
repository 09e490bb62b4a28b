"""CPU FP64 oracle -- test infrastructure only (tests, smoke check, CPU baseline).

The product path never imports this package."""
