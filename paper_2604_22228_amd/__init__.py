"""pcoll: partitioned reduction of P rank contributions on one MI355X."""
