// A ring of per-launch scratch slots (a large fill's tile-counter pair,
// the moments kernel's partial sums).  Each launch takes the next slot;
// the stream it runs on first waits for the event recorded after the
// slot's previous launch, so no two launches ever hold a slot at the same
// time, whatever streams or host threads they come from.  The ring's lock
// is held from taking a slot until its event is recorded, so a later user
// of the slot always waits for the record of the earlier one.
//
// The runtime calls come from Ops, which supplies the Event and Stream
// types and
//   static int wait(Stream s, Event e);    later work on s waits for e
//   static int record(Event e, Stream s);  e completes with s's work so far
// each returning 0 or an error value.  The library uses HIP's streams and
// events; the host test program uses a simulated device.
#pragma once

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <vector>

namespace zig {

template <class Ops>
struct SlotRing {
  std::mutex mu;
  char* base = nullptr;  // slots * slot_bytes of device memory
  size_t slot_bytes = 0;
  uint32_t slots = 0, next = 0;
  std::vector<typename Ops::Event> ev;  // recorded after each slot's last launch
  std::vector<char> recorded;           // whether ev[k] has been recorded
};

// Runs launch(slot) on `stream` with the next slot of r.  launch returns 0
// or an error value, which is passed on (the slot then keeps its previous
// event).
template <class Ops, class F>
int ring_launch(SlotRing<Ops>* r, typename Ops::Stream stream, F launch) {
  std::lock_guard<std::mutex> lk(r->mu);
  const uint32_t k = r->next;
  r->next = (r->next + 1) % r->slots;
  if (r->recorded[k]) {
    const int e = Ops::wait(stream, r->ev[k]);
    if (e != 0) return e;
  }
  const int e = launch(static_cast<void*>(r->base + k * r->slot_bytes));
  if (e != 0) return e;
  const int er = Ops::record(r->ev[k], stream);
  if (er != 0) return er;
  r->recorded[k] = 1;
  return 0;
}

}  // namespace zig
